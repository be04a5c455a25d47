"""Device layout of the interpolative operators and the build's size limits.

The row of a leaf basis U_X = K(X, s) K(t, s)^-1 at the point of row pivot a
is the unit vector e_a, and so is the row of a stacked transfer at a child
pivot that is also the box's row pivot (Sec. 3.4.3, nested pivots).  The
upload stores only the other rows; the products stay equal to the oracle's to
the FP64 bar (the parity tests check every kernel and variant), and the
operator bytes must show that the unit rows are gone.
"""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def lib():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2309_14085_amd import h2s
    h2s.load()
    return h2s


@pytest.mark.parametrize("d,kind,eps", [(2, 0, 1e-8), (3, 1, 1e-6)])
def test_unit_rows_are_not_stored(lib, orc, inputs, d, kind, eps):
    n = 20000
    print(f"layout d={d} kind={kind}", flush=True)
    pts = inputs.uniform_points(n, d, 31 + d)
    T = lib.build(pts, kind=kind, leaf_size=64, eps=eps)
    st = T.stats()
    full = 16 * (st["leaf_basis_entries"] + st["transfer_entries"])  # two FP64 copies of every entry
    ratio = st["operator_bytes"] / full
    print(f"operator bytes {st['operator_bytes']} of {full} with the unit rows: {ratio:.3f}", flush=True)
    # every row pivot of a leaf gives one unit row in each copy: at least r_X of n_X rows go
    assert 0.3 < ratio < 0.9
    # and the product is still the oracle's
    q = inputs.normal_rhs(n, 1, 41 + d)[:, 0]
    x = torch.from_numpy(q).to("cuda:0")
    y = T.apply(x)
    torch.cuda.synchronize()
    want = orc.Tree(pts, kind, 64, eps).apply(q)
    err = np.linalg.norm(y.cpu().numpy() - want) / np.linalg.norm(want)
    print(f"relative error against the oracle {err:.2e}", flush=True)
    assert err <= 1e-12


def test_oversized_leaf_is_rejected(lib, orc, inputs):
    # one leaf (kappa = 0) of 4200 points: the kernels stage at most 4096 points of a leaf
    pts = inputs.uniform_points(4200, 2, 51)
    with pytest.raises(lib.H2SError) as e:
        lib.build(pts, kind=0, leaf_size=5000, eps=1e-8)
    assert e.value.status == lib.ERR_UNSUPPORTED
    assert "4096" in str(e.value)
    # a leaf of 4096 points is accepted and multiplies correctly
    pts = inputs.uniform_points(4096, 2, 52)
    T = lib.build(pts, kind=0, leaf_size=5000, eps=1e-8)
    assert T.stats()["kappa"] == 0
    q = inputs.normal_rhs(4096, 1, 53)[:, 0]
    y = T.apply(torch.from_numpy(q).to("cuda:0"))
    torch.cuda.synchronize()
    want = orc.Tree(pts, 0, 5000, 1e-8).apply(q)
    assert np.linalg.norm(y.cpu().numpy() - want) / np.linalg.norm(want) <= 1e-12
