"""Seeded synthetic inputs shared by the library's tests, the oracle's tests and the benchmark.

This module holds input generation only: no part of the method's
arithmetic.  Random point sets are uniform in [-1, 1]^d and every right-hand
side is N(0, 1), the distributions of the paper's MVP experiments (Sec. 6.1.1,
Sec. 6.2.1: uniformly distributed particles in [-1,1]^d, random vectors q);
the RBF interpolation experiments of Sec. 6 place the particles on a tensor
Chebyshev grid instead (`chebyshev_grid`).  Generators are NumPy PCG64
(`numpy.random.default_rng(seed)`), so any seed reproduces the same arrays on
every machine.
"""
from dataclasses import dataclass, field

import numpy as np

LOG_R, INV_R, GAUSS, EXP_R, RBF_AR, RBF_LOG, NTI_MQ = 0, 1, 2, 3, 4, 5, 6


def uniform_points(n: int, d: int, seed: int) -> np.ndarray:
    """n points i.i.d. uniform in [-1, 1]^d, row-major (n, d) float64."""
    return np.random.default_rng(seed).uniform(-1.0, 1.0, size=(n, d))


def chebyshev_grid(m: int, d: int) -> np.ndarray:
    """The m^d tensor grid of first-kind Chebyshev nodes cos((2k + 1) pi / (2m)),
    k = 0 .. m-1, in [-1, 1]^d: row-major (m^d, d) float64, last coordinate fastest."""
    nodes = np.cos((2.0 * np.arange(m) + 1.0) * np.pi / (2.0 * m))
    axes = np.meshgrid(*([nodes] * d), indexing="ij")
    return np.ascontiguousarray(np.stack([a.ravel() for a in axes], axis=1))


def normal_rhs(n: int, m: int, seed: int) -> np.ndarray:
    """m right-hand sides of length n with N(0, 1) entries, column-major (n, m) float64."""
    return np.asfortranarray(np.random.default_rng(seed).standard_normal(size=(n, m)))


@dataclass(frozen=True)
class Workload:
    name: str
    d: int
    n: int
    kind: int
    param: float
    diag: float
    shift: float
    nmax: int
    eps: float
    nrhs: int
    seed_points: int
    seed_rhs: int
    extra: dict = field(default_factory=dict)

    def points(self) -> np.ndarray:
        return uniform_points(self.n, self.d, self.seed_points)

    def rhs(self) -> np.ndarray:
        return normal_rhs(self.n, self.nrhs, self.seed_rhs)


def _w(c, name, d, n, kind, eps, nrhs, param=0.0, diag=None, shift=0.0, nmax=64, **extra):
    if diag is None:
        diag = 0.0 if kind in (LOG_R, INV_R, RBF_AR, RBF_LOG) else 1.0
    return Workload(name, d, n, kind, param, diag, shift, nmax, eps, nrhs, 1000 + c, 2000 + c, extra)


# The five workloads the project measures and tests (index = config number - 1).
WORKLOADS = [
    _w(0, "2d_log_n4096", 2, 4096, LOG_R, 1e-8, 1),
    _w(1, "2d_log_n1048576", 2, 1 << 20, LOG_R, 1e-8, 1),
    _w(2, "3d_invr_n262144_m32", 3, 1 << 18, INV_R, 1e-6, 32),
    _w(3, "2d_gauss_rbf_n262144", 2, 1 << 18, GAUSS, 1e-8, 1, param=0.1, shift=1e-2),
    _w(4, "serving_mixed", 0, 0, LOG_R, 1e-8, 1, requests=512),
]


def workload(name_or_index) -> Workload:
    if isinstance(name_or_index, int):
        return WORKLOADS[name_or_index]
    for w in WORKLOADS:
        if w.name == name_or_index:
            return w
    raise KeyError(name_or_index)


def scaled(w: Workload, n: int, seed_offset: int = 0) -> Workload:
    """The same workload recipe at another size (and optionally other seeds)."""
    return Workload(w.name + f"_n{n}", w.d, n, w.kind, w.param, w.diag, w.shift, w.nmax, w.eps, w.nrhs,
                    w.seed_points + seed_offset, w.seed_rhs + seed_offset, dict(w.extra))


def clustered_points(n: int, d: int, seed: int, clusters: int = 6, frac: float = 0.7,
                     width: float = 0.01) -> np.ndarray:
    """Points whose leaves are very uneven: a fraction `frac` of them in `clusters` tight Gaussian
    clusters of standard deviation `width` (clipped to [-1, 1]^d), the rest uniform.  With the
    paper's depth rule (the average leaf holds n_max) this leaves many boxes empty and puts far
    more than n_max points into the clusters' leaves.  Two points are pinned at opposite corners
    so the bounding cube is [-1, 1]^d."""
    rng = np.random.default_rng(seed)
    nc = int(frac * n)
    centres = rng.uniform(-0.9, 0.9, size=(clusters, d))
    which = rng.integers(0, clusters, size=nc)
    pc = np.clip(centres[which] + width * rng.standard_normal(size=(nc, d)), -1.0, 1.0)
    pu = rng.uniform(-1.0, 1.0, size=(n - nc, d))
    out = np.concatenate([pc, pu])[rng.permutation(n)]
    out[0], out[1] = -1.0, 1.0
    return np.ascontiguousarray(out)


def with_coincident_points(points: np.ndarray, copies: int, seed: int) -> np.ndarray:
    """The same set with `copies` of its points repeated exactly (coincident pairs, which the
    kernels give the diagonal value), appended in a seeded order."""
    rng = np.random.default_rng(seed)
    src = rng.choice(len(points), size=copies, replace=False)
    return np.ascontiguousarray(np.concatenate([points, points[src]]))


def face_grid_points(m: int, d: int) -> np.ndarray:
    """The m^d tensor grid of equally spaced points -1 + 2k/(m-1), k = 0 .. m-1: with m - 1 a
    power of two every coordinate is a dyadic fraction, so many points lie exactly on the faces
    of the tree's boxes (the root cube is [-1, 1]^d).  Row-major (m^d, d), last coordinate fastest."""
    nodes = -1.0 + 2.0 * np.arange(m) / (m - 1)
    axes = np.meshgrid(*([nodes] * d), indexing="ij")
    return np.ascontiguousarray(np.stack([a.ravel() for a in axes], axis=1))
