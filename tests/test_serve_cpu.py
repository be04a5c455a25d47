"""Host-side logic of the serving loop: the request generator and the memory estimate."""
import math

import numpy as np


def test_requests_are_seeded_and_in_range():
    from paper_2309_14085_amd import serve
    a = serve.make_requests(200, rate=4.0, seed=9, n_range=(16384, 131072), n_range_3d=(16384, 32768), nrhs_max=4)
    b = serve.make_requests(200, rate=4.0, seed=9, n_range=(16384, 131072), n_range_3d=(16384, 32768), nrhs_max=4)
    assert [(r.arrival, r.d, r.n, r.nrhs, r.seed) for r in a] == [(r.arrival, r.d, r.n, r.nrhs, r.seed) for r in b]
    arr = np.array([r.arrival for r in a])
    assert np.all(np.diff(arr) > 0)
    # Poisson arrivals at 4/s: the mean gap is 0.25 s (within 4 standard errors)
    gaps = np.diff(np.concatenate([[0.0], arr]))
    assert abs(gaps.mean() - 0.25) < 4 * 0.25 / math.sqrt(len(gaps))
    assert {r.d for r in a} == {2, 3}
    for r in a:
        lo, hi = (16384, 131072) if r.d == 2 else (16384, 32768)
        assert lo <= r.n <= hi and 1 <= r.nrhs <= 4
        assert r.shift == r.n / 2 ** r.d
        assert r.kind == (0 if r.d == 2 else 1)


def test_memory_estimate_grows_with_size_and_dimension():
    from paper_2309_14085_amd import serve
    small = serve.Request(0, 0.0, 2, 16384, 1, 1)
    big = serve.Request(1, 0.0, 2, 131072, 1, 1)
    three = serve.Request(2, 0.0, 3, 16384, 1, 1)
    assert serve.estimate_bytes(big) > serve.estimate_bytes(small) > 0
    assert serve.estimate_bytes(three) > serve.estimate_bytes(small)
