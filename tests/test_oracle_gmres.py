"""Pins of the GMRES solve oracle (oracle/gmres.py) against what linear algebra fixes.

* A dense system: the GMRES solution equals numpy's LU solve.
* Finite termination: A = Q diag(lambda) Q^T with k distinct eigenvalues is
  solved in k Arnoldi steps (the minimal polynomial of A has degree k).
* The minimal-residual property: within a cycle the least-squares residual
  estimate never increases, and at the end of the solve it equals the true
  residual.
* Restarts: GMRES(5) still converges on a well-conditioned system.
* With the oracle's H2* product (Gaussian kernel plus shift, tolerance near
  zero) the solution equals a dense solve of the exact kernel matrix written
  out from its definition.
"""
import numpy as np
import pytest

from oracle.gmres import gmres


def _dense(A):
    return lambda v: A @ v


def test_dense_system_matches_lu_solve():
    rng = np.random.default_rng(11)
    n = 80
    A = rng.standard_normal((n, n)) / np.sqrt(n) + 3.0 * np.eye(n)
    b = rng.standard_normal(n)
    x, info = gmres(_dense(A), b, restart=n, rtol=1e-13)
    want = np.linalg.solve(A, b)
    assert info["converged"]
    assert info["iterations"] <= n
    assert np.linalg.norm(x - want) / np.linalg.norm(want) <= 1e-11


@pytest.mark.parametrize("eigs", [(1.0, 2.0, 3.0, 5.0, 8.0), (0.5, 4.0, 9.0)])
def test_distinct_eigenvalues_finite_termination(eigs):
    rng = np.random.default_rng(12)
    n = 120
    lam = np.array([eigs[i % len(eigs)] for i in range(n)])
    Q, _ = np.linalg.qr(rng.standard_normal((n, n)))
    A = (Q * lam) @ Q.T
    b = rng.standard_normal(n)
    x, info = gmres(_dense(A), b, restart=50, rtol=1e-10)
    assert info["converged"]
    assert info["iterations"] == len(eigs)
    assert np.linalg.norm(A @ x - b) / np.linalg.norm(b) <= 1e-10


def test_residual_estimate_monotone_and_exact():
    rng = np.random.default_rng(13)
    n = 60
    A = rng.standard_normal((n, n)) / np.sqrt(n) + 1.5 * np.eye(n)
    b = rng.standard_normal(n)
    x, info = gmres(_dense(A), b, restart=n, rtol=1e-7)
    h = info["history"]
    assert all(h[i + 1] <= h[i] * (1 + 1e-12) for i in range(len(h) - 1))
    true = np.linalg.norm(b - A @ x) / np.linalg.norm(b)
    assert abs(true - h[-1]) <= 1e-6 * h[-1]
    assert info["residual"] == pytest.approx(true, rel=1e-12)


def test_restarted_gmres_converges():
    rng = np.random.default_rng(14)
    n = 100
    A = rng.standard_normal((n, n)) / np.sqrt(n) + 4.0 * np.eye(n)
    b = rng.standard_normal(n)
    x, info = gmres(_dense(A), b, restart=5, rtol=1e-10, max_iter=5000)
    assert info["converged"]
    assert info["iterations"] > 5  # at least one restart happened
    assert np.linalg.norm(x - np.linalg.solve(A, b)) / np.linalg.norm(x) <= 1e-8


def test_zero_rhs_gives_zero():
    x, info = gmres(lambda v: 2.0 * v, np.zeros(7))
    assert np.all(x == 0.0) and info["iterations"] == 0


def test_oracle_h2_product_solve_matches_dense_kernel_solve(orc, inputs):
    n, h, shift = 1000, 0.2, 1.0
    pts = inputs.uniform_points(n, 2, 31)
    b = inputs.normal_rhs(n, 1, 32)[:, 0]
    T = orc.Tree(pts, orc.GAUSS, 32, 1e-14, param=h, shift=shift)
    x, info = gmres(T.apply, b, restart=50, rtol=1e-12)
    assert info["converged"]
    # the kernel matrix from its definition: exp(-|x_i - x_j|^2 / h^2), K_ii = 1, plus shift I
    d2 = ((pts[:, None, :] - pts[None, :, :]) ** 2).sum(-1)
    K = np.exp(-d2 / (h * h)) + shift * np.eye(n)
    want = np.linalg.solve(K, b)
    assert np.linalg.norm(x - want) / np.linalg.norm(want) <= 1e-9
