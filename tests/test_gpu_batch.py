"""Batched multi-RHS product (blocks of 8 right-hand sides, h2s_apply with nrhs > 1)
against the FP64 oracle column by column, and against the single-column path.

Bars: FP64 <= 1e-12 relative 2-norm per column (a phase's error relative to the
column's whole product); FP32 <= 1e-5; batched and single-column FP64 products
agree to 1e-12 (the single-column M2L takes accurate dot products over each
unordered pair, the batched one plain sums on the matrix cores, and the
interpolation operators amplify that rounding difference; in 3D they agree to
about 1e-14).
Columns beyond the block's active count, and the padding rows of ld > n, are
never written.
"""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch.device("cuda:0")


@pytest.fixture(scope="module")
def lib():
    from paper_2309_14085_amd import h2s
    h2s.load()
    return h2s


def rel(a, b):
    return np.linalg.norm(a - b) / np.linalg.norm(b)


def apply_block(T, lib, Q, ld, mask=7):
    """Q (n, m) host; returns the (n, m) result of one h2s_apply_phases call with leading dimension ld."""
    n, m = Q.shape
    dev = _dev()
    xb = torch.zeros(m * ld, dtype=torch.float64, device=dev)
    yb = torch.full((m * ld,), 3.0, dtype=torch.float64, device=dev)
    for c in range(m):
        xb[c * ld:c * ld + n] = torch.from_numpy(Q[:, c].copy()).to(dev)
    assert T.apply_ptr(xb.data_ptr(), yb.data_ptr(), nrhs=m, ldx=ld, ldy=ld, mask=mask) == lib.OK
    torch.cuda.synchronize()
    y = yb.cpu().numpy()
    for c in range(m):
        assert np.all(y[c * ld + n:(c + 1) * ld] == 3.0)  # padding untouched
    return np.stack([y[c * ld:c * ld + n] for c in range(m)], axis=1)


CASES = [
    # name, d, n, kind, nmax, eps, param, shift, seed
    ("2d_log_5000", 2, 5000, 0, 48, 1e-10, 0.0, 0.0, 61),
    ("3d_invr_6000", 3, 6000, 1, 64, 1e-6, 0.0, 0.0, 62),
    ("2d_gauss_4000", 2, 4000, 2, 32, 1e-10, 0.2, 1e-2, 63),
    ("3d_expr_3000", 3, 3000, 3, 32, 1e-10, 0.0, 0.0, 64),
    ("3d_rbf_log_3000", 3, 3000, 5, 32, 1e-8, 0.1, 54.77, 65),
    ("3d_nti_mq_3000", 3, 3000, 6, 32, 1e-8, 0.0, 54.77, 66),
]


@pytest.mark.parametrize("case", CASES, ids=[c[0] for c in CASES])
@pytest.mark.parametrize("m", [3, 8, 11, 20, 32, 40])
def test_batched_fp64_matches_oracle_per_column(lib, orc, inputs, case, m):
    name, d, n, kind, nmax, eps, param, shift, seed = case
    print(f"batched {name} m={m}", flush=True)
    pts = inputs.uniform_points(n, d, seed)
    Q = inputs.normal_rhs(n, m, seed + 100)
    O = orc.Tree(pts, kind, nmax, eps, param=param, shift=shift)
    T = lib.build(pts, kind=kind, leaf_size=nmax, eps=eps, param=param, shift=shift)
    Y = apply_block(T, lib, Q, n + 5)
    for c in range(m):
        assert rel(Y[:, c], O.apply(Q[:, c])) <= 1e-12, c


def test_batched_phases_match_oracle_parts(lib, orc, inputs):
    n, m = 5000, 8
    print("batched phases", flush=True)
    pts = inputs.uniform_points(n, 2, 65)
    Q = inputs.normal_rhs(n, m, 66)
    O = orc.Tree(pts, 0, 48, 1e-10)
    T = lib.build(pts, kind=0, leaf_size=48, eps=1e-10)
    parts = [O.apply_parts(Q[:, c]) for c in range(m)]
    for mask, idx in ((lib.PHASE_NEAR, 0), (lib.PHASE_FAR, 1), (lib.PHASE_VER, 2)):
        Y = apply_block(T, lib, Q, n, mask=mask)
        for c in range(m):
            total = sum(parts[c])
            assert np.linalg.norm(Y[:, c] - parts[c][idx]) <= 1e-12 * np.linalg.norm(total), (mask, c)


@pytest.mark.parametrize("m", [8, 32])
def test_batched_agrees_with_single_column_path(lib, inputs, m):
    """8 columns: one block (M2L on the vector units); 32: four blocks sharing every M2L kernel
    value on the matrix cores."""
    n = 20000
    print(f"batched vs single m={m}", flush=True)
    pts = inputs.uniform_points(n, 2, 67)
    Q = inputs.normal_rhs(n, m, 68)
    T = lib.build(pts, kind=0, leaf_size=64, eps=1e-8)
    Y = apply_block(T, lib, Q, n)
    dev = _dev()
    for c in range(m):
        y1 = T.apply(torch.from_numpy(Q[:, c].copy()).to(dev))
        torch.cuda.synchronize()
        assert rel(Y[:, c], y1.cpu().numpy()) <= 1e-12, c


@pytest.mark.parametrize("d,kind,eps", [(2, 0, 1e-8), (3, 1, 1e-6)])
def test_batched_fp32_within_1e5(lib, orc, inputs, d, kind, eps):
    n, m = (8192, 5) if d == 2 else (6000, 5)
    print(f"batched fp32 d={d}", flush=True)
    pts = inputs.uniform_points(n, d, 69 + d)
    Q = inputs.normal_rhs(n, m, 71 + d)
    O = orc.Tree(pts, kind, 64, eps)
    T = lib.build(pts, kind=kind, leaf_size=64, eps=eps, prec=lib.FP32)
    Y = apply_block(T, lib, Q, n)
    for c in range(m):
        assert rel(Y[:, c], O.apply(Q[:, c])) <= 1e-5, c


def test_multi_rhs_fallbacks_match_oracle(lib, orc, inputs):
    """(H2+H)* takes the column loop; its multi-RHS results still match."""
    n, m = 4000, 4
    print("multi-rhs fallbacks", flush=True)
    pts = inputs.uniform_points(n, 2, 73)
    Q = inputs.normal_rhs(n, m, 74)
    O = orc.Tree(pts, 0, 48, 1e-10, variant=1)
    T = lib.build(pts, kind=0, leaf_size=48, eps=1e-10, variant=1)
    Y = apply_block(T, lib, Q, n)
    for c in range(m):
        assert rel(Y[:, c], O.apply(Q[:, c])) <= 1e-12


LOWP_CASES = [
    # name, d, n, kind, nmax, eps, param, shift, seed
    ("2d_log_8192", 2, 8192, 0, 64, 1e-8, 0.0, 0.0, 75),
    ("3d_invr_12000", 3, 12000, 1, 64, 1e-6, 0.0, 0.0, 76),
    ("2d_gauss_6000", 2, 6000, 2, 64, 1e-8, 0.2, 1e-2, 77),
]


@pytest.mark.parametrize("case", LOWP_CASES, ids=[c[0] for c in LOWP_CASES])
@pytest.mark.parametrize("m", [5, 8, 20, 32])
def test_batched_low_precision_m2l_against_oracle(lib, orc, inputs, case, m):
    """FP32_M2L and FP32_BF16M2L with several right-hand sides: the far-field M2L on the matrix
    cores in float / with bfloat16 inputs (one block of 8 columns when m <= 8, else up to four
    sharing each kernel value).  Against the FP64 oracle per column: FP32_M2L within 1e-4 (the
    cap of its single-column form), and within 1e-4 of its single-column product (float
    accumulation on the matrix cores against double accumulation there; a column taken from the
    wrong block would be off by O(1)).  BF16 is reported, with a sanity cap of 0.25: bfloat16
    keeps 8 significant bits of the kernel values and multipoles, and the interpolation
    operators amplify that rounding (about 1e-3 for the Gaussian, 1e-2 for 1/r in 3D and up to
    1e-1 for log r in 2D on these inputs)."""
    name, d, n, kind, nmax, eps, param, shift, seed = case
    pts = inputs.uniform_points(n, d, seed)
    Q = inputs.normal_rhs(n, m, seed + 100)
    O = orc.Tree(pts, kind, nmax, eps, param=param, shift=shift)
    want = np.stack([O.apply(Q[:, c]) for c in range(m)], axis=1)
    dev = _dev()
    errs, agree = {}, []
    for prec in (lib.FP32_M2L, lib.FP32_BF16M2L):
        T = lib.build(pts, kind=kind, leaf_size=nmax, eps=eps, param=param, shift=shift, prec=prec)
        Y = apply_block(T, lib, Q, n + 3)
        errs[prec] = [rel(Y[:, c], want[:, c]) for c in range(m)]
        if prec == lib.FP32_M2L:
            for c in (0, m // 2, m - 1):
                y1 = T.apply(torch.from_numpy(Q[:, c].copy()).to(dev))
                torch.cuda.synchronize()
                agree.append(rel(Y[:, c], y1.cpu().numpy()))
    print(f"low-precision M2L {name} m={m}: fp32 {max(errs[lib.FP32_M2L]):.2e} (vs single column "
          f"{max(agree):.2e}) bf16 {max(errs[lib.FP32_BF16M2L]):.2e}", flush=True)
    assert max(errs[lib.FP32_M2L]) <= 1e-4 and max(agree) <= 1e-4
    assert max(errs[lib.FP32_BF16M2L]) <= 0.25
