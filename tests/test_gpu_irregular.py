"""GPU parity on irregular point sets: very uneven leaves with many empty boxes (tight
clusters, leaves of more than 1024 points), exactly coincident points, and points lying on
the faces of the tree's boxes.  Per phase, both variants, FP64 against the oracle.

Bars as in the uniform parity tests: each phase's error <= 1e-12 of the whole product's
2-norm and <= 5e-11 of its largest element.
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
    nb = np.linalg.norm(b)
    return np.linalg.norm(a - b) / (nb if nb > 0 else 1.0)


def relmax(a, b):
    mb = np.abs(b).max()
    return np.abs(a - b).max() / (mb if mb > 0 else 1.0)


def gpu_apply(T, q, mask=7):
    y = T.apply(torch.from_numpy(np.ascontiguousarray(q)).to(_dev()), mask=mask)
    torch.cuda.synchronize()
    return y.cpu().numpy()


def _sets(inputs):
    return {
        # 97% of the points in 8 clusters of width 0.005: about half the leaves are empty and
        # the clusters' leaves hold up to about 2500 points
        "clustered_2d": (inputs.clustered_points(20000, 2, 11, clusters=8, frac=0.97, width=0.005), 0, 64, 1e-8),
        "clustered_3d": (inputs.clustered_points(12000, 3, 12, clusters=8, frac=0.9, width=0.01), 1, 32, 1e-6),
        # 60 exact duplicates: K takes the diagonal value on every coincident pair
        "coincident_2d": (inputs.with_coincident_points(inputs.uniform_points(6000, 2, 13), 60, 14), 0, 48, 1e-10),
        "coincident_3d": (inputs.with_coincident_points(inputs.uniform_points(5000, 3, 15), 40, 16), 1, 32, 1e-6),
        # dyadic grids: many points on box faces down to the leaves
        "faces_2d": (inputs.face_grid_points(65, 2), 0, 32, 1e-10),
        "faces_3d": (inputs.face_grid_points(17, 3), 1, 32, 1e-6),
    }


NAMES = ["clustered_2d", "clustered_3d", "coincident_2d", "coincident_3d", "faces_2d", "faces_3d"]


@pytest.mark.parametrize("name", NAMES)
@pytest.mark.parametrize("variant", [0, 1])
def test_irregular_sets_match_oracle_per_phase(lib, orc, inputs, name, variant):
    pts, kind, nmax, eps = _sets(inputs)[name]
    n = len(pts)
    print(f"irregular {name} n={n} variant={variant}", flush=True)
    q = inputs.normal_rhs(n, 1, 4242)[:, 0]
    O = orc.Tree(pts, kind, nmax, eps, variant=variant)
    near, far, ver = O.apply_parts(q)
    T = lib.build(pts, kind=kind, leaf_size=nmax, eps=eps, variant=variant)
    total = near + far + ver
    for mask, want, what in ((lib.PHASE_NEAR, near, "near"), (lib.PHASE_FAR, far, "far"),
                             (lib.PHASE_VER, ver, "ver"), (lib.PHASE_ALL, total, "total")):
        if not np.any(want):
            continue
        got = gpu_apply(T, q, mask)
        assert np.all(np.isfinite(got)), what
        e2 = np.linalg.norm(got - want) / np.linalg.norm(total)
        em = np.abs(got - want).max() / np.abs(total).max()
        print(f"  {what}: {e2:.2e} (max {em:.2e})", flush=True)
        assert e2 <= 1e-12 and em <= 5e-11, (what, e2, em)


def test_coincident_points_take_the_diagonal(lib, orc, inputs):
    """A point and its exact copy: the product over the pair is diag * (q_i + q_j), here 0 for
    log r, so moving charge between the two copies changes no other potential."""
    pts = inputs.with_coincident_points(inputs.uniform_points(3000, 2, 17), 30, 18)
    n = len(pts)
    T = lib.build(pts, kind=0, leaf_size=32, eps=1e-10)
    q = inputs.normal_rhs(n, 1, 19)[:, 0]
    q2 = q.copy()
    q2[3000:] += 1.0  # add charge on the copies ...
    src = np.array([np.flatnonzero((pts[:3000] == p).all(1))[0] for p in pts[3000:]])
    q2[src] -= 1.0    # ... and take it off their originals
    y1, y2 = gpu_apply(T, q), gpu_apply(T, q2)
    others = np.setdiff1d(np.arange(n), np.concatenate([src, np.arange(3000, n)]))
    assert np.abs(y1[others] - y2[others]).max() <= 1e-11 * np.abs(y1).max()
