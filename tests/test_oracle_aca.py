"""Pins for the oracle's partially pivoted ACA (Sec. 3.4) and NCA operators (Sec. 3.4.3).

The ACA is checked against properties every cross approximation must have:
  * the cross (skeleton) identity U V^T = M[:, sigma] M[tau, sigma]^{-1} M[tau, :]
    (the paper's equation for K^(p));
  * exactness on the pivot rows and columns;
  * the stopping rule, with ||S||_F recomputed from the factors;
  * exact recovery of low-rank matrices, rank 0 for a zero block;
  * error near the SVD truncation error on smooth kernel blocks (a textbook special case).
"""
import numpy as np
import pytest


def kblock(a, b, kind):
    r = np.sqrt(((a[:, None, :] - b[None, :, :]) ** 2).sum(-1))
    return np.log(r) if kind == 0 else 1.0 / r


@pytest.fixture(scope="module")
def blocks():
    rng = np.random.default_rng(4)
    a = rng.uniform(0, 1, (150, 2))
    out = {
        "far": kblock(a, rng.uniform(0, 1, (180, 2)) + [2.0, 0.5], 0),
        "vertex": kblock(a, rng.uniform(0, 1, (170, 2)) - 1.0, 0),
        "far3d": kblock(rng.uniform(0, 1, (120, 3)), rng.uniform(0, 1, (130, 3)) + [2.0, 0, 0], 1),
    }
    return out


@pytest.mark.parametrize("name", ["far", "vertex", "far3d"])
@pytest.mark.parametrize("eps", [1e-4, 1e-8])
def test_cross_identity_and_pivot_exactness(orc, blocks, name, eps):
    M = blocks[name]
    tau, sigma, U, V = orc.aca_dense(M, eps)
    r = len(tau)
    assert r >= 1 and len(set(tau)) == r and len(set(sigma)) == r
    S = U @ V.T
    skel = M[:, sigma] @ np.linalg.solve(M[np.ix_(tau, sigma)], M[tau, :])
    assert np.linalg.norm(S - skel) <= 1e-9 * np.linalg.norm(M)
    # the residual vanishes on the pivot rows and columns
    scale = np.abs(M).max()
    assert np.abs(S[tau, :] - M[tau, :]).max() <= 1e-11 * scale
    assert np.abs(S[:, sigma] - M[:, sigma]).max() <= 1e-11 * scale


ACA_RUN = 6  # successive terms that must meet the stopping condition (reading of Sec. 3.4)


@pytest.mark.parametrize("eps", [1e-3, 1e-6, 1e-9])
def test_stopping_rule(orc, blocks, eps):
    """The iteration ends at the first term that completes a run of ACA_RUN successive terms
    with ||u_p|| ||v_p|| <= eps ||S_p||_F (S_p recomputed from the factors), and not earlier."""
    M = blocks["vertex"]
    tau, sigma, U, V = orc.aca_dense(M, eps)
    r = len(tau)
    assert r < min(M.shape)
    run = 0
    for p in range(r):
        Sp = U[:, : p + 1] @ V[:, : p + 1].T
        term = np.linalg.norm(U[:, p]) * np.linalg.norm(V[:, p])
        bound = eps * np.linalg.norm(Sp)
        # no term sits so close to the bound that the recomputed norm could decide otherwise
        assert abs(term - bound) > 1e-10 * bound
        run = run + 1 if term <= bound else 0
        if p < r - 1:
            assert run < ACA_RUN
    assert run == ACA_RUN


def test_single_small_term_does_not_end_the_iteration(orc, blocks):
    """A vertex-sharing block whose residual sits on a few close pairs: the run rule keeps going
    past terms that are small by chance, and the final error is at the tolerance
    (the SVD truncation at the same rank is the floor)."""
    M = blocks["vertex"]
    eps = 1e-8
    tau, sigma, U, V = orc.aca_dense(M, eps)
    err = np.linalg.norm(M - U @ V.T) / np.linalg.norm(M)
    assert err <= 2 * eps

def test_first_pivots_follow_reading(orc, blocks):
    M = blocks["far"]
    tau, sigma, U, V = orc.aca_dense(M, 1e-6)
    assert tau[0] == 0 and sigma[0] == np.argmax(np.abs(M[0]))
    # the second row pivot maximises |u_1| over the remaining rows
    u1 = np.abs(U[:, 0]).copy()
    u1[0] = -1
    assert tau[1] == np.argmax(u1)


def test_low_rank_recovery_and_zero_block(orc):
    rng = np.random.default_rng(9)
    for k in (1, 3, 7):
        A, B = rng.standard_normal((60, k)), rng.standard_normal((80, k))
        M = A @ B.T
        tau, sigma, U, V = orc.aca_dense(M, 1e-12)
        assert k <= len(tau) <= k + ACA_RUN
        assert np.linalg.norm(M - U @ V.T) <= 1e-12 * np.linalg.norm(M)
    tau, sigma, U, V = orc.aca_dense(np.zeros((20, 30)), 1e-8)
    assert len(tau) == 0
    # full rank at eps = 0 on a small well-conditioned matrix
    M = rng.standard_normal((6, 9))
    tau, sigma, U, V = orc.aca_dense(M, 0.0)
    assert len(tau) == 6 and np.allclose(U @ V.T, M, atol=1e-12)


@pytest.mark.parametrize("name", ["far", "vertex", "far3d"])
@pytest.mark.parametrize("eps", [1e-6, 1e-10])
def test_error_near_svd_truncation(orc, blocks, name, eps):
    M = blocks[name]
    tau, sigma, U, V = orc.aca_dense(M, eps)
    err = np.linalg.norm(M - U @ V.T) / np.linalg.norm(M)
    s = np.linalg.svd(M, compute_uv=False)
    tail = np.sqrt(np.cumsum((s ** 2)[::-1]))[::-1] / np.linalg.norm(s)
    r_svd = int(np.argmax(tail <= eps))
    assert err <= 10 * eps
    assert len(tau) <= 2 * r_svd + 4


def test_operators_interpolate_at_pivots(orc, inputs):
    """L2P operator U_X = K(t^X, s^{X,i}) K(t^{X,i}, s^{X,i})^{-1} is the identity on the
    row pivots (Sec. 3.4.3), and B2T parents pick their row pivots among the children's,
    so the stacked L2L operator has identity rows there."""
    pts = inputs.uniform_points(4096, 2, 21)
    T = orc.Tree(pts, orc.LOG_R, 64, 1e-8)
    K = T.kappa
    leaves = T.boxes(K)
    for fam in (orc.FAR, orc.VER):
        for x in range(0, len(leaves["begin"]), 7):
            rows, cols = T.pivots(fam, K, x)
            U = T.operator(fam, K, x)
            local = rows - leaves["begin"][x]
            assert np.abs(U[local] - np.eye(len(rows))).max() <= 1e-9
            # U A = K(t^X, s^{X,i}) by definition
            tp = T.tree_points()
            Kx = kblock(tp[leaves["begin"][x]:leaves["end"][x]], tp[cols], 0)
            A = kblock(tp[rows], tp[cols], 0)
            assert np.linalg.norm(U @ A - Kx) <= 1e-11 * np.linalg.norm(Kx)
    lvl = K - 1
    b = T.boxes(lvl)
    ch = T.boxes(K)
    for x in range(len(b["begin"])):
        rows, _ = T.pivots(orc.FAR, lvl, x)
        kids = np.nonzero(ch["parent"] == x)[0]
        child_rows = np.concatenate([T.pivots(orc.FAR, K, c)[0] for c in kids])
        assert set(rows) <= set(child_rows)
        Ut = T.operator(orc.FAR, lvl, x)
        pos = [int(np.nonzero(child_rows == r)[0][0]) for r in rows]
        assert np.abs(Ut[pos] - np.eye(len(rows))).max() <= 1e-9
