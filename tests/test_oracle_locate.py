"""Pins of the point-location oracle (the general restriction of Section 2.3).

Facts outside the oracle: a P1 interpolant reproduces linear fields exactly; at a mesh
node it returns the nodal value; the coordinates sum to one and rebuild the point;
points outside the domain are reported outside; for the nested hierarchy the located
value at a coarse node is the injection (Eq. 19); a hand-made two-triangle square.
"""
import numpy as np

import cgp_inputs as ci
from oracle import locate as loc
from oracle import mesh


def test_two_triangles_by_hand():
    xy = np.array([[0.0, 0.0], [1.0, 0.0], [1.0, 1.0], [0.0, 1.0]])
    tri = np.array([[0, 1, 2], [0, 2, 3]])
    f = np.array([1.0, 2.0, 4.0, 8.0])
    v, t = loc.interpolate(xy, tri, f, np.array([[0.75, 0.25], [0.25, 0.75], [0.5, 0.5], [1.5, 0.5]]))
    # (0.75, 0.25) in triangle 0 with coordinates (0.25, 0.5, 0.25); (0.25, 0.75) in 1 with (0.25, 0.25, 0.5)
    assert list(t) == [0, 1, 0, -1]      # the diagonal point: both give min 0, the lowest id wins
    # (0.5, 0.5) on the diagonal: coordinates (0.5, 0, 0.5) of vertices 0 and 2
    np.testing.assert_allclose(v[:3], [0.25 + 1.0 + 1.0, 0.25 + 1.0 + 4.0, 0.5 + 2.0], rtol=1e-15)
    assert np.isnan(v[3])


def test_linear_fields_nodes_and_coordinates():
    m = ci.rect_with_hole(17, 11, (5, 9, 3, 7), seed=2)
    rng = np.random.default_rng(4)
    pts = np.column_stack([rng.uniform(0, 2, 400), rng.uniform(0, 1, 400)])
    f = 0.7 * m.xy[:, 0] - 1.3 * m.xy[:, 1] + 0.2
    v, t = loc.interpolate(m.xy, m.tri, f, pts)
    inside = t >= 0
    # the hole (cells 5..9 x 3..7 of the 16 x 10 grid) is outside the domain
    hole = (pts[:, 0] > 5 * 2 / 16) & (pts[:, 0] < 9 * 2 / 16) & (pts[:, 1] > 3 / 10) & (pts[:, 1] < 7 / 10)
    np.testing.assert_array_equal(inside, ~hole)
    np.testing.assert_allclose(v[inside], 0.7 * pts[inside, 0] - 1.3 * pts[inside, 1] + 0.2, rtol=0, atol=1e-13)
    _, lam = loc.locate(m.xy, m.tri, pts)
    np.testing.assert_allclose(lam[inside].sum(axis=1), 1.0, rtol=0, atol=1e-14)
    rebuilt = np.einsum("ij,ijk->ik", lam[inside], m.xy[m.tri[t[inside]]])
    np.testing.assert_allclose(rebuilt, pts[inside], rtol=0, atol=1e-14)
    # at the nodes: the nodal values
    g = rng.standard_normal(m.n_nodes)
    vn, tn = loc.interpolate(m.xy, m.tri, g, m.xy)
    assert np.all(tn >= 0)
    np.testing.assert_allclose(vn, g, rtol=0, atol=1e-14 * np.abs(g).max())


def test_located_coarse_nodes_give_the_injection():
    m = ci.jittered_rect(9, 5, 3)
    h = mesh.Hierarchy(m.xy, m.tri, m.dirichlet, 2)
    q = np.random.default_rng(5).standard_normal(h.n_nodes(2))
    v, t = loc.interpolate(h.xy[2], h.tri[2], q, m.xy)
    assert np.all(t >= 0)
    np.testing.assert_allclose(v, mesh.restrict_inject(q, m.n_nodes), rtol=0, atol=1e-14 * np.abs(q).max())
