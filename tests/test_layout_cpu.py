"""The interpolative structure the device layout relies on, checked on the host build.

The leaf basis U_X = K(X, s) K(t, s)^-1 (Sec. 3.4.3) has the unit vector e_a
as its row at the point of row pivot a, and with nested pivots the stacked
transfer of a box has e_a as its row at a child pivot that is also the box's
row pivot a.  The upload drops rows that are exactly e_a, so this test pins
that the host build's LU solves reproduce them exactly, for most pivots.
"""
import numpy as np
import pytest


@pytest.fixture(scope="module")
def lib():
    from paper_2309_14085_amd import h2s
    return h2s


def unit_rows(e, fam, nbox, leaf0):
    rk, co = e[f"fam_{fam}_rank"], e[f"fam_{fam}_coef_off"]
    pr, oo, op, rows = e[f"fam_{fam}_piv_row"], e[f"fam_{fam}_op_off"], e[f"fam_{fam}_op"], e[f"fam_{fam}_op_rows"]
    bb, par = e["box_begin"], e["box_parent"]
    children = [[] for _ in range(nbox)]
    for c in range(nbox):
        if par[c] >= 0:
            children[par[c]].append(c)
    leaf = [0, 0, 0]      # pivots checked, exact unit rows, leaf rows
    trans = [0, 0, 0]     # child pivots that are box pivots, exact unit rows, transfer rows
    for x in range(nbox):
        r = rk[x]
        if r == 0:
            continue
        n = rows[x]
        block = op[oo[x]:oo[x] + n * r]
        piv = pr[co[x]:co[x + 1]]
        if x >= leaf0:
            U = block.reshape(r, n).T  # column-major n x r
            for a, p in enumerate(piv):
                leaf[0] += 1
                leaf[1] += np.array_equal(U[p - bb[x]], np.eye(r)[a])
            leaf[2] += n
        else:
            Tr = block.reshape(n, r)  # row-major (sum r_c) x r
            stack = np.concatenate([pr[co[c]:co[c + 1]] for c in sorted(children[x])])
            assert len(stack) == n
            where = {int(p): a for a, p in enumerate(piv)}
            for k, p in enumerate(stack):
                a = where.get(int(p))
                if a is not None:
                    trans[0] += 1
                    trans[1] += np.array_equal(Tr[k], np.eye(r)[a])
            trans[2] += n
    return leaf, trans


@pytest.mark.parametrize("d,kind,eps", [(2, 0, 1e-8), (3, 1, 1e-6)])
def test_pivot_rows_are_exact_unit_rows(lib, inputs, tmp_path, d, kind, eps):
    pts = inputs.uniform_points(8192 if d == 2 else 6000, d, 91 + d)
    T = lib.build(pts, kind=kind, leaf_size=64, eps=eps, host_only=True)
    e = T.export(tmp_path / "rep.h2sx")
    nbox = len(e["fam_far_rank"])
    st = T.stats()
    # leaves are the boxes of the deepest level: the last 2^(d kappa) boxes
    leaf0 = nbox - (1 << (d * st["kappa"]))
    for fam in ("far", "ver"):
        leaf, trans = unit_rows(e, fam, nbox, leaf0)
        # every row pivot of a leaf gives an exact unit row
        assert leaf[0] > 0 and leaf[1] == leaf[0], (fam, leaf)
        # nested pivots: every child pivot that is also the box's pivot gives an exact unit row
        assert trans[1] == trans[0], (fam, trans)
        if st["kappa"] >= 2:
            assert trans[0] > 0.15 * trans[2], (fam, trans)
        assert leaf[1] > 0.25 * leaf[2], (fam, leaf)
