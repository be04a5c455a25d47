"""The register-resident evaluation-rate loop behind the roofline's R_eval (h2s_eval_rate)."""
import math

import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.mark.parametrize("kind,d,param", [(0, 2, 0.0), (1, 3, 0.0), (2, 2, 0.1), (6, 3, 0.0)])
def test_eval_rate_is_a_plausible_rate(kind, d, param):
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2309_14085_amd import h2s
    r64 = h2s.eval_rate(kind, d, h2s.FP64, param=param)
    r32 = h2s.eval_rate(kind, d, h2s.FP32, param=param)
    print(f"kind {kind} d {d}: fp64 {r64:.3e} fp32 {r32:.3e} evaluations/s", flush=True)
    # 256 CUs x 64 FP64 lanes x 2.4 GHz bounds any formula of at least one instruction
    for r in (r64, r32):
        assert math.isfinite(r) and 1e10 < r < 256 * 64 * 2.4e9


def test_eval_rate_rejects_bad_arguments():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2309_14085_amd import h2s
    for args in ((0, 4, h2s.FP64), (6, 2, h2s.FP64), (0, 2, 7), (9, 2, h2s.FP64)):
        with pytest.raises(h2s.H2SError):
            h2s.eval_rate(*args)
    with pytest.raises(h2s.H2SError):
        h2s.eval_rate(h2s.GAUSSIAN, 2, h2s.FP64, param=0.0)
