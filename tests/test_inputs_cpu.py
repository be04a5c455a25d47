"""The seeded input generators: shapes, ranges and the Chebyshev grid's nodes."""
import numpy as np
from numpy.polynomial import chebyshev


def test_chebyshev_grid_nodes_are_roots_of_t_m():
    from paper_2309_14085_amd import inputs
    for m, d in ((1, 2), (7, 2), (96, 2), (5, 3), (20, 3)):
        g = inputs.chebyshev_grid(m, d)
        assert g.shape == (m ** d, d) and g.flags.c_contiguous
        assert np.all(np.abs(g) < 1.0)
        nodes = np.unique(g[:, 0])
        assert len(nodes) == m
        tm = np.zeros(m + 1)
        tm[m] = 1.0
        assert np.max(np.abs(chebyshev.chebval(nodes, tm))) < 1e-12
        # tensor grid, last coordinate fastest, all points distinct
        assert np.array_equal(g[:m, -1], g[:m, -1][np.argsort(-g[:m, -1])])
        assert len(np.unique(g, axis=0)) == m ** d


def test_uniform_points_and_rhs_are_seeded():
    from paper_2309_14085_amd import inputs
    a, b = inputs.uniform_points(1000, 3, 5), inputs.uniform_points(1000, 3, 5)
    assert np.array_equal(a, b) and a.shape == (1000, 3) and np.all(np.abs(a) <= 1.0)
    q = inputs.normal_rhs(1000, 4, 6)
    assert q.shape == (1000, 4) and q.flags.f_contiguous
    assert not np.array_equal(q[:, 0], q[:, 1])


def test_irregular_point_sets():
    from paper_2309_14085_amd import inputs
    a = inputs.clustered_points(20000, 2, 11)
    assert a.shape == (20000, 2) and np.all(np.abs(a) <= 1.0)
    assert np.array_equal(a, inputs.clustered_points(20000, 2, 11))
    assert a.min() == -1.0 and a.max() == 1.0
    b = inputs.with_coincident_points(a, 50, 12)
    assert b.shape == (20050, 2) and len(np.unique(b, axis=0)) == len(np.unique(a, axis=0))
    g = inputs.face_grid_points(33, 2)
    assert g.shape == (33 * 33, 2) and g.min() == -1.0 and g.max() == 1.0
    assert np.all((g * 16) == np.round(g * 16))  # dyadic: on the faces of boxes down to level 4
