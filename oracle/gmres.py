"""Plain restarted GMRES in FP64 (NumPy), the solve oracle.

TEST INFRASTRUCTURE: only tests/, __graft_entry__.smoke() and bench.py's
cpu_baseline leg may import this module.  It shares no code with the
library in paper_2309_14085_amd/.

The paper solves K sigma = f with GMRES to a relative residual tolerance
(Sec. 6, the integral-equation and RBF-interpolation experiments), with the
matrix-vector product supplied by the fast representation.  This is the
textbook restarted GMRES(m) (Saad, Iterative Methods for Sparse Linear
Systems, 2nd ed., Alg. 6.9 with restarts): Arnoldi with modified
Gram-Schmidt, Givens rotations on the Hessenberg matrix, the least-squares
residual |g_{j+1}| as the stopping estimate, and a restart from the true
residual b - A x after every m steps.
"""
import numpy as np


def gmres(apply, b, restart=50, rtol=1e-10, max_iter=10000, x0=None):
    """Solve A x = b for a linear operator `apply(v) -> A v` (FP64 vectors).

    Returns (x, info) with info = {"iterations": Arnoldi steps taken,
    "residual": ||b - A x|| / ||b|| computed with `apply` at the end,
    "history": least-squares residual estimates / ||b||, one per step,
    "converged": bool}.
    """
    b = np.asarray(b, dtype=np.float64)
    n = b.shape[0]
    x = np.zeros(n) if x0 is None else np.array(x0, dtype=np.float64)
    bnorm = np.linalg.norm(b)
    if bnorm == 0.0:
        return np.zeros(n), {"iterations": 0, "residual": 0.0, "history": [], "converged": True}
    history = []
    its = 0
    m = max(1, int(restart))
    while True:
        r = b - apply(x)
        beta = np.linalg.norm(r)
        if beta / bnorm <= rtol or its >= max_iter:
            break
        V = np.zeros((n, m + 1))
        H = np.zeros((m + 1, m))
        cs = np.zeros(m)
        sn = np.zeros(m)
        g = np.zeros(m + 1)
        g[0] = beta
        V[:, 0] = r / beta
        k = 0
        for j in range(m):
            w = apply(V[:, j])
            # modified Gram-Schmidt against v_0 .. v_j
            for i in range(j + 1):
                H[i, j] = np.dot(V[:, i], w)
                w = w - H[i, j] * V[:, i]
            H[j + 1, j] = np.linalg.norm(w)
            if H[j + 1, j] != 0.0:
                V[:, j + 1] = w / H[j + 1, j]
            # earlier rotations on the new column, then the one that zeroes H[j+1, j]
            for i in range(j):
                t = cs[i] * H[i, j] + sn[i] * H[i + 1, j]
                H[i + 1, j] = -sn[i] * H[i, j] + cs[i] * H[i + 1, j]
                H[i, j] = t
            den = np.hypot(H[j, j], H[j + 1, j])
            cs[j] = H[j, j] / den if den != 0.0 else 1.0
            sn[j] = H[j + 1, j] / den if den != 0.0 else 0.0
            H[j, j] = cs[j] * H[j, j] + sn[j] * H[j + 1, j]
            H[j + 1, j] = 0.0
            g[j + 1] = -sn[j] * g[j]
            g[j] = cs[j] * g[j]
            its += 1
            k = j + 1
            history.append(abs(g[j + 1]) / bnorm)
            if abs(g[j + 1]) / bnorm <= rtol or its >= max_iter or den == 0.0:
                break
        # x += V_k y with H_k y = g_k (upper triangular)
        y = np.zeros(k)
        for i in range(k - 1, -1, -1):
            y[i] = (g[i] - np.dot(H[i, i + 1:k], y[i + 1:k])) / H[i, i]
        x = x + V[:, :k] @ y
    res = np.linalg.norm(b - apply(x)) / bnorm
    return x, {"iterations": its, "residual": float(res), "history": history, "converged": bool(res <= rtol)}
