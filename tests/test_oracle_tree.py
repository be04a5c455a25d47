"""Pins for the oracle's tree and lists (Sec. 3.1, Sec. 3.3, Table HOD_notation, Sec. 5.1).

Expected values are the paper's printed closed forms (tests/golden/), counting
identities of a full 2^d grid, and brute-force geometric checks.
"""
import json
import os

import numpy as np
import pytest

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def full_grid_points(d, per_dim_leaves, per_leaf_side, seed=0):
    """A jittered grid with exactly per_leaf_side^d points in every leaf box."""
    rng = np.random.default_rng(seed)
    m = per_dim_leaves * per_leaf_side
    g = (np.arange(m) + 0.5) / m * 2 - 1
    mesh = np.stack(np.meshgrid(*([g] * d), indexing="ij"), -1).reshape(-1, d)
    mesh += rng.uniform(-0.2, 0.2, mesh.shape) / m
    # pin the bounding cube to exactly [-1, 1]^d
    corners = np.array([[-1.0] * d, [1.0] * d])
    return np.vstack([mesh, corners])


@pytest.mark.parametrize("case", json.load(open(os.path.join(GOLDEN, "paper_tree_depth.json")))["cases"])
def test_depth_matches_paper(orc, case):
    assert orc.depth(case["n"], case["d"], case["nmax"]) == case["kappa"]


def test_depth_formula_edges(orc):
    for d in (2, 3):
        for k in range(0, 6):
            n = 64 * 2 ** (d * k)
            assert orc.depth(n, d, 64) == k
            assert orc.depth(n + 1, d, 64) == k + 1
    assert orc.depth(1, 2, 64) == 0


@pytest.mark.parametrize("d", [2, 3])
def test_points_lie_in_their_boxes(orc, inputs, d):
    n = 3000
    pts = inputs.uniform_points(n, d, 11)
    T = orc.Tree(pts, orc.LOG_R if d == 2 else orc.INV_R, 16, 1e-2)
    ctr, h = T.cube()
    lo, hi = pts.min(0), pts.max(0)
    assert np.allclose(ctr, (lo + hi) / 2) and np.isclose(h, ((hi - lo) / 2).max())
    perm = T.perm()
    assert np.array_equal(np.sort(perm), np.arange(n))
    tp = T.tree_points()
    assert np.array_equal(tp, pts[perm])
    origin = ctr - h
    for l in range(T.kappa + 1):
        b = T.boxes(l)
        w = 2 * h / 2**l
        assert np.all(np.diff(b["morton"]) > 0)
        assert b["begin"][0] == 0 and b["end"][-1] == n and np.array_equal(b["begin"][1:], b["end"][:-1])
        for x in range(len(b["begin"])):
            p = tp[b["begin"][x]:b["end"][x]]
            lo_box = origin + b["coord"][x] * w
            assert np.all(p >= lo_box - 1e-12) and np.all(p <= lo_box + w + 1e-12)
        if l > 0:
            pb = T.boxes(l - 1)
            assert np.array_equal(pb["coord"][b["parent"]], b["coord"] // 2)


def _cover_counts(T, d):
    """For every ordered pair of leaves, how many times the lists cover it."""
    K = T.kappa
    leaves = T.boxes(K)
    L = len(leaves["begin"])
    # leaf -> ancestor index per level
    anc = [None] * (K + 1)
    anc[K] = np.arange(L)
    for l in range(K, 0, -1):
        anc[l - 1] = T.boxes(l)["parent"][anc[l]]
    cover = np.zeros((L, L), np.int64)
    off, idx = T.lists(orc_list_near(), K)
    for x in range(L):
        cover[x, idx[off[x]:off[x + 1]]] += 1
    for l in range(1, K + 1):
        for which in (1, 2):
            off, idx = T.lists(which, l)
            for X in range(len(off) - 1):
                rows = np.nonzero(anc[l] == X)[0]
                cols = np.nonzero(np.isin(anc[l], idx[off[X]:off[X + 1]]))[0]
                cover[np.ix_(rows, cols)] += 1
    return cover


def orc_list_near():
    return 0


@pytest.mark.parametrize("d,leaves_per_dim", [(2, 16), (3, 8)])
def test_exact_cover_and_paper_maxima(orc, d, leaves_per_dim):
    """Every ordered leaf pair is either near or in exactly one IL block (one level),
    and the list sizes reach the paper's closed-form maxima."""
    gold = json.load(open(os.path.join(GOLDEN, "paper_list_maxima.json")))[str(d)]
    pts = full_grid_points(d, leaves_per_dim, 2)
    nmax = 2**d
    T = orc.Tree(pts, orc.LOG_R if d == 2 else orc.INV_R, nmax + 1, 0.5)
    assert 2 ** (d * T.kappa) == leaves_per_dim**d
    cover = _cover_counts(T, d)
    assert cover.min() == 1 and cover.max() == 1
    K = T.kappa
    off, _ = T.lists(0, K)
    assert np.diff(off).max() == gold["near_max"]
    mx_far = mx_ver = mx_il = 0
    for l in range(1, K + 1):
        of, _ = T.lists(1, l)
        ov, _ = T.lists(2, l)
        mx_far = max(mx_far, np.diff(of).max())
        mx_ver = max(mx_ver, np.diff(ov).max())
        mx_il = max(mx_il, (np.diff(of) + np.diff(ov)).max())
        if l == 1:
            assert np.diff(of).max() == 0  # no far field at level 1 (Sec. 5.1.2 level ranges)
            assert np.all(np.diff(ov) == 1)  # the diagonally opposite child of the root
    assert (mx_far, mx_ver, mx_il) == (gold["far_max"], gold["ver_max"], gold["il_max"])


@pytest.mark.parametrize("d", [2, 3])
def test_vertex_and_near_pair_counts_full_grid(orc, d):
    """Counting identities on a full 2^l grid: ordered vertex pairs at level l are the
    all-diagonal neighbours, minus the one pair per parent-level vertex pair that
    the parent level already covers; near pairs are self + (d-1)-face/edge sharing."""
    per = 8 if d == 2 else 4
    pts = full_grid_points(d, per, 2, seed=3)
    T = orc.Tree(pts, orc.LOG_R if d == 2 else orc.INV_R, 2**d + 1, 0.5)
    K = T.kappa
    for l in range(1, K + 1):
        _, idx = T.lists(2, l)
        m, mp = 2**l - 1, 2 ** (l - 1) - 1
        assert len(idx) == 2**d * (m**d - mp**d)
    s = 2**K
    _, near = T.lists(0, K)
    if d == 2:
        want = s * s + 4 * s * (s - 1)
    else:
        want = s**3 + 3 * 2 * (s - 1) * s * s + 3 * 4 * (s - 1) ** 2 * s
    assert len(near) == want


def test_lists_sorted_and_symmetric(orc, inputs):
    pts = inputs.uniform_points(4096, 2, 5)
    T = orc.Tree(pts, orc.LOG_R, 64, 1e-2)
    for l in range(1, T.kappa + 1):
        for which in (1, 2):
            off, idx = T.lists(which, l)
            pairs = set()
            for x in range(len(off) - 1):
                ys = idx[off[x]:off[x + 1]]
                assert np.all(np.diff(ys) > 0)
                pairs.update((x, int(y)) for y in ys)
            assert all((y, x) in pairs for (x, y) in pairs)
