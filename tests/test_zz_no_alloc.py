"""h2s_apply_noalloc (batch buffers in the library's file-scope device array) against
h2s_apply on the same handle and columns: equal bit for bit, on two calls in a row, the second
on a smaller tree and fewer columns, and a size beyond the array is rejected."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _block(T, lib, Q, noalloc):
    n, m = Q.shape
    dev = torch.device("cuda:0")
    x = torch.from_numpy(np.asfortranarray(Q).ravel(order="F").copy()).to(dev)
    y = torch.full((n * m,), 5.0, dtype=torch.float64, device=dev)
    if noalloc:
        st = T.apply_noalloc_ptr(x.data_ptr(), y.data_ptr(), m)
    else:
        st = T.apply_ptr(x.data_ptr(), y.data_ptr(), nrhs=m)
    assert st == lib.OK, lib.last_error()
    torch.cuda.synchronize()
    return y.cpu().numpy().reshape((n, m), order="F")


def test_noalloc_equals_apply_on_two_calls(inputs):
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2309_14085_amd import h2s
    h2s.load()
    for n, d, kind, m, seed in ((20000, 2, 0, 32, 81), (6000, 3, 1, 11, 82)):
        print(f"noalloc n={n} d={d} m={m}", flush=True)
        pts = inputs.uniform_points(n, d, seed)
        Q = inputs.normal_rhs(n, m, seed + 1)
        T = h2s.build(pts, kind=kind, leaf_size=64, eps=1e-8 if d == 2 else 1e-6)
        a = _block(T, h2s, Q, True)
        b = _block(T, h2s, Q, False)
        assert np.all(np.isfinite(a))
        assert np.array_equal(a, b)
        T.free()


def test_noalloc_rejects_what_it_cannot_hold(inputs):
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2309_14085_amd import h2s
    h2s.load()
    n = 600000  # 32 columns of 600000 points need about 340 MB of batch buffers, above 256 MiB
    pts = inputs.uniform_points(n, 2, 83)
    T = h2s.build(pts, kind=0, leaf_size=64, eps=1e-6)
    dev = torch.device("cuda:0")
    x = torch.zeros(n * 32, dtype=torch.float64, device=dev)
    y = torch.zeros(n * 32, dtype=torch.float64, device=dev)
    assert T.apply_noalloc_ptr(x.data_ptr(), y.data_ptr(), 32) == h2s.ERR_UNSUPPORTED
    assert "scratch" in h2s.last_error()
    assert T.apply_noalloc_ptr(x.data_ptr(), y.data_ptr(), 33) == h2s.ERR_INVALID_ARG
    # one block of 8 columns fits and matches h2s_apply
    Q = inputs.normal_rhs(n, 8, 84)
    a = _block(T, h2s, Q, True)
    b = _block(T, h2s, Q, False)
    assert np.array_equal(a, b)
    T.free()
