"""Pins for the oracle's direct product phi = (K + shift I) q (Sec. 6, t_direct / RE_MVP).

Each expected value is a closed form of classical geometry, not a retyping of
the oracle's loop.
"""
import math

import numpy as np
import pytest


def test_log_r_on_unit_circle(orc):
    # N equally spaced points on the unit circle: prod_{j != i} |x_i - x_j| = N,
    # so with q = 1 and K_ii = 0 every potential equals log N.
    for n in (3, 7, 64, 257):
        th = 2 * np.pi * np.arange(n) / n
        pts = np.stack([np.cos(th), np.sin(th)], 1)
        phi = orc.direct(pts, np.ones(n), orc.LOG_R)
        assert np.allclose(phi, math.log(n), rtol=0, atol=1e-12 * max(1.0, math.log(n)))


def test_log_r_scaled_circle(orc):
    # radius rho: prod |x_i - x_j| = N rho^(N-1)
    n, rho = 16, 0.37
    th = 2 * np.pi * np.arange(n) / n
    pts = rho * np.stack([np.cos(th), np.sin(th)], 1) + np.array([0.25, -0.5])
    phi = orc.direct(pts, np.ones(n), orc.LOG_R)
    assert np.allclose(phi, math.log(n) + (n - 1) * math.log(rho), rtol=1e-13)


def test_inv_r_cube_vertices(orc):
    # unit cube: every vertex has 3 neighbours at 1, 3 at sqrt 2, 1 at sqrt 3
    pts = np.array([[i, j, k] for i in (0, 1) for j in (0, 1) for k in (0, 1)], float) * 0.5
    phi = orc.direct(pts, np.ones(8), orc.INV_R)
    want = (3 + 3 / math.sqrt(2) + 1 / math.sqrt(3)) / 0.5
    assert np.allclose(phi, want, rtol=1e-14)


def test_gaussian_and_exp_two_points_with_diag_and_shift(orc):
    pts = np.array([[0.0, 0.0], [0.3, 0.4]])  # distance 0.5
    q = np.array([2.0, -3.0])
    h = 0.7
    phi = orc.direct(pts, q, orc.GAUSS, param=h, diag=1.0, shift=0.01)
    g = math.exp(-0.25 / h**2)
    assert np.allclose(phi, [2 * 1.0 + g * -3 + 0.02, g * 2 + -3 * 1.0 - 0.03], rtol=1e-14)
    phi = orc.direct(pts, q, orc.EXP_R, diag=1.0)
    e = math.exp(-0.5)
    assert np.allclose(phi, [2 + e * -3, e * 2 - 3], rtol=1e-14)


def test_diagonal_convention_and_rows_subset(orc):
    # K_ii = 0 for log r (Sec. 6.1.1): a single point has zero potential
    assert orc.direct(np.array([[0.1, 0.2]]), np.array([5.0]), orc.LOG_R)[0] == 0.0
    rng = np.random.default_rng(0)
    pts = rng.uniform(-1, 1, (50, 2))
    q = rng.standard_normal(50)
    full = orc.direct(pts, q, orc.LOG_R)
    rows = np.array([3, 17, 49, 0])
    assert np.array_equal(orc.direct(pts, q, orc.LOG_R, rows=rows), full[rows])


def test_symmetric_matrix(orc):
    # x^T K y = y^T K x for a symmetric kernel
    rng = np.random.default_rng(1)
    pts = rng.uniform(-1, 1, (200, 3))
    x, y = rng.standard_normal(200), rng.standard_normal(200)
    a = x @ orc.direct(pts, y, orc.INV_R)
    b = y @ orc.direct(pts, x, orc.INV_R)
    assert abs(a - b) <= 1e-12 * abs(a)


def test_piecewise_rbfs_values_and_continuity(orc):
    """The two RBFs of the paper's 2D / 3D interpolation solves (Sec. 6), at points worked by hand.

    a/r | r/a with a = 0.5: G(1) = 0.5, G(0.25) = 0.5, G(0.5) = 1.
    log r / log a | (r log r - 1)/(a log a - 1) with a = 1/e (log a = -1):
    G(e) = -1, G(1/e^2) = (1 + 2/e^2) / (1 + 1/e), and G -> 1 from both sides of r = a."""
    def pair(r, kind, a, d):
        pts = np.zeros((2, d))
        pts[1, 0] = r
        return orc.direct(pts, np.array([0.0, 1.0]), kind, param=a)[0]

    assert pair(1.0, orc.RBF_AR, 0.5, 2) == pytest.approx(0.5, rel=1e-15)
    assert pair(0.25, orc.RBF_AR, 0.5, 2) == pytest.approx(0.5, rel=1e-15)
    assert pair(0.5, orc.RBF_AR, 0.5, 2) == pytest.approx(1.0, rel=1e-15)
    a = math.exp(-1.0)
    assert pair(math.e, orc.RBF_LOG, a, 3) == pytest.approx(-1.0, rel=1e-14)
    assert pair(math.exp(-2.0), orc.RBF_LOG, a, 3) == pytest.approx((1 + 2 / math.e**2) / (1 + 1 / math.e), rel=1e-14)
    for kind, d in ((orc.RBF_AR, 2), (orc.RBF_LOG, 3)):
        lo, hi = pair(a * (1 - 1e-9), kind, a, d), pair(a * (1 + 1e-9), kind, a, d)
        assert abs(lo - 1.0) < 1e-7 and abs(hi - 1.0) < 1e-7
    # their systems leave out j = i: K_ii = 0
    assert orc.default_diag(orc.RBF_AR) == 0.0 and orc.default_diag(orc.RBF_LOG) == 0.0


def test_nti_multiquadric_values_and_invariances(orc):
    """The NTI scaled multiquadric of Sec. 6, F(x, y) = (|x - y|^2 + (c(x) - c(y))^2 + 1)^(3/2),
    c(x) = exp(-(x_1 + x_3)), at points worked by hand, and the invariances its definition gives.

    x = 0 and y = (0, sqrt 3, 0): c(x) = c(y) = 1, |x - y|^2 = 3, so F = 4^(3/2) = 8.
    x = 0 and y = (-ln 2, sqrt(2 - ln^2 2), 0): c(y) = 2, |x - y|^2 = 2, (c(x) - c(y))^2 = 1, so F = 8.
    x = y: F = 1, the default diagonal.  F is symmetric; moving both points along (1, 0, -1)
    or along (0, 1, 0) keeps |x - y| and every c, so F is unchanged; along (1, 0, 0) it is not."""
    def F(x, y):
        pts = np.array([x, y], dtype=np.float64)
        return orc.direct(pts, np.array([0.0, 1.0]), orc.NTI_MQ)[0]

    o = [0.0, 0.0, 0.0]
    assert F(o, [0.0, math.sqrt(3.0), 0.0]) == pytest.approx(8.0, rel=1e-15)
    l2 = math.log(2.0)
    assert F(o, [-l2, math.sqrt(2.0 - l2 * l2), 0.0]) == pytest.approx(8.0, rel=1e-14)
    assert orc.default_diag(orc.NTI_MQ) == 1.0
    x, y = [0.3, -0.2, 0.1], [-0.4, 0.5, 0.7]
    f0 = F(x, y)
    assert F(y, x) == f0
    for sh in ([0.25, 0.0, -0.25], [0.0, 0.6, 0.0]):
        assert F(np.add(x, sh), np.add(y, sh)) == pytest.approx(f0, rel=1e-14)
    moved = F(np.add(x, [0.5, 0, 0]), np.add(y, [0.5, 0, 0]))
    assert abs(moved - f0) > 1e-3 * f0  # not translation invariant
    with pytest.raises(ValueError):
        orc.direct(np.zeros((2, 2)), np.ones(2), orc.NTI_MQ)
