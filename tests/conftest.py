import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (HIP device) to run")
    config.addinivalue_line("markers", "slow: CPU test that takes more than a few seconds")


@pytest.fixture(scope="session")
def orc():
    """The oracle package, built on first use."""
    import oracle
    if not os.path.exists(oracle.LIB_PATH):
        from oracle import build
        build.build()
    oracle._load()
    return oracle


@pytest.fixture(scope="session")
def inputs():
    from paper_2309_14085_amd import inputs as _inputs
    return _inputs
