"""Pins of the cylinder-in-channel workload (Section 3): the mesh generator's structure,
the surface force against closed forms, the per-component Dirichlet rows of the momentum
step against a manufactured solution with natural boundaries, and the CGP step's fixed
point (uniform flow in an empty channel)."""
import numpy as np
import pytest

import cgp_inputs as ci
from oracle import channel as och
from oracle import fem, mesh
from oracle import momentum as mom


@pytest.fixture(scope="module")
def small():
    return ci.cylinder_channel(seed=3, n_circle=16, growth=0.5, h_max=4.0)


def _angles(xy, tri):
    a = xy[tri]
    out = []
    for i in range(3):
        u = a[:, (i + 1) % 3] - a[:, i]
        w = a[:, (i + 2) % 3] - a[:, i]
        c = (u * w).sum(1) / np.linalg.norm(u, axis=1) / np.linalg.norm(w, axis=1)
        out.append(np.degrees(np.arccos(np.clip(c, -1.0, 1.0))))
    return np.stack(out, 1)


def test_generator_structure(small):
    for m in (small, ci.cylinder_channel()):
        g = m.geometry
        e1 = m.xy[m.tri[:, 1]] - m.xy[m.tri[:, 0]]
        e2 = m.xy[m.tri[:, 2]] - m.xy[m.tri[:, 0]]
        assert np.all(e1[:, 0] * e2[:, 1] - e1[:, 1] * e2[:, 0] > 0.0)              # CCW
        assert np.unique(m.tri).size == m.n_nodes                                  # every node used
        ends, _, _ = mesh.edges(m.n_nodes, m.tri)
        assert m.n_nodes - ends.shape[0] + m.n_tris == 0                           # one hole
        nb = int((m.inflow | m.outflow | m.walls | m.cylinder).sum())
        assert m.n_tris == 2 * m.n_nodes - nb
        r = np.hypot(m.xy[:, 0] - g["xc"], m.xy[:, 1] - g["yc"])
        cyl = m.cylinder.astype(bool)
        assert cyl.sum() == g["n_circle"] and np.allclose(r[cyl], 0.5 * g["d"], rtol=0, atol=1e-14)
        assert r.min() >= 0.5 * g["d"] - 1e-14
        b = ci.channel_boundary(m.xy, m.tri, g)
        ce = b["cyl_edges"]
        assert ce.shape[0] == g["n_circle"]
        assert np.all(np.bincount(ce[:, :2].ravel(), minlength=m.n_nodes)[cyl] == 2)   # a closed polygon
        assert _angles(m.xy, m.tri).min() > 15.0
        for cx, cy in ((0, 0), (g["L"], 0), (g["L"], g["H"]), (0, g["H"])):
            assert np.any(np.all(m.xy == (cx, cy), axis=1))
    big = ci.cylinder_channel()
    assert abs(big.n_nodes - 1749) < 0.05 * 1749 and abs(big.n_tris - 3370) < 0.05 * 3370
    again = ci.cylinder_channel(seed=3, n_circle=16, growth=0.5, h_max=4.0)
    np.testing.assert_array_equal(again.xy, small.xy)
    np.testing.assert_array_equal(again.tri, small.tri)


def _upper_half(m, edges):
    yc = m.geometry["yc"]
    up = (m.xy[edges[:, 0], 1] >= yc) & (m.xy[edges[:, 1], 1] >= yc)
    return edges[up]


def test_surface_force_closed_forms(small):
    m = small
    g = m.geometry
    edges = ci.channel_boundary(m.xy, m.tri, g)["cyl_edges"]
    zero = np.zeros(m.n_nodes)
    # constant pressure on a closed body: no force
    fp, fv = och.surface_force(m.xy, m.tri, edges, np.full(m.n_nodes, 3.0), zero, zero, 0.01)
    assert np.abs(fp).max() < 1e-13 and np.abs(fv).max() == 0.0
    # linear pressure: -(body polygon's area) grad p (divergence theorem, exact for a polygon)
    th = np.sort(np.arctan2(*(m.xy[m.cylinder.astype(bool)] - [g["xc"], g["yc"]]).T[::-1]))
    poly = np.stack([np.cos(th), np.sin(th)], 1) * 0.5
    area = 0.5 * np.sum(poly[:, 0] * np.roll(poly[:, 1], -1) - np.roll(poly[:, 0], -1) * poly[:, 1])
    p = 0.7 * m.xy[:, 0] - 1.9 * m.xy[:, 1] + 4.0
    fp, _ = och.surface_force(m.xy, m.tri, edges, p, zero, zero, 0.01)
    np.testing.assert_allclose(fp, -area * np.array([0.7, -1.9]), rtol=1e-12, atol=1e-13)
    # a linear velocity: constant stress; over the upper half (from angle 0 to pi) the sum of
    # n ds is (0, 2 r) = (0, d)
    gu, gv = np.array([0.3, -1.1]), np.array([2.0, 0.4])
    u, v = m.xy @ gu, m.xy @ gv
    mu = 0.05
    s = mu * np.array([[2 * gu[0], gu[1] + gv[0]], [gu[1] + gv[0], 2 * gv[1]]])
    fp, fv = och.surface_force(m.xy, m.tri, edges, zero, u, v, mu)
    assert np.abs(fv).max() < 1e-13
    half = _upper_half(m, edges)
    assert half.shape[0] == g["n_circle"] // 2
    fp, fv = och.surface_force(m.xy, m.tri, half, np.full(m.n_nodes, 2.0), u, v, mu)
    nds = np.array([0.0, g["d"]])
    np.testing.assert_allclose(fp, -2.0 * nds, rtol=0, atol=1e-13)
    np.testing.assert_allclose(fv, s @ nds, rtol=0, atol=1e-13)
    np.testing.assert_allclose(och.coefficients(fv, 1.0, 2.0, 0.5), fv, rtol=1e-15)


def test_momentum_per_component_dirichlet_rows():
    # u* = c + gamma y is fixed on the walls (y = 0, 1) and natural at x = 0, 2 (du/dx = 0);
    # v* = c2 + gamma2 x the other way round.  The boundary values handed in elsewhere are
    # wrong on purpose: a row that is Dirichlet by mistake takes them.
    m = ci.jittered_rect(11, 6, 21)
    x, y = m.xy[:, 0], m.xy[:, 1]
    lr = (np.abs(x) < 1e-12) | (np.abs(x - 2.0) < 1e-12)
    tb = (np.abs(y) < 1e-12) | (np.abs(y - 1.0) < 1e-12)
    mask = (tb * 1 | lr * 2).astype(np.uint8)
    rho, mu, dt = 1.0, 0.3, 0.1
    a = np.array([0.4, -0.2])
    un, vn = np.full(m.n_nodes, a[0]), np.full(m.n_nodes, a[1])
    us, vs = 0.5 + 1.5 * y, -0.2 + 0.8 * x
    fx = (rho / dt) * (us - un) + rho * (a[1] * 1.5)
    fy = (rho / dt) * (vs - vn) + rho * (a[0] * 0.8)
    gu = np.where(tb, us, us + 1.0)
    gv = np.where(lr, vs, vs - 1.0)
    ut, vt = mom.step(m.xy, m.tri, None, un, vn, fx, fy, rho, mu, dt, gu=gu, gv=gv, mask=mask)
    np.testing.assert_allclose(ut, us, rtol=0, atol=1e-12)
    np.testing.assert_allclose(vt, vs, rtol=0, atol=1e-12)
    # the same mask for both components reduces to the single Dirichlet set
    d = (tb | lr).astype(np.uint8)
    a1 = mom.step(m.xy, m.tri, d, un, vn, fx, fy, rho, mu, dt, gu=us, gv=vs)
    a2 = mom.step(m.xy, m.tri, None, un, vn, fx, fy, rho, mu, dt, gu=us, gv=vs, mask=d * 3)
    np.testing.assert_array_equal(a1[0], a2[0])
    np.testing.assert_array_equal(a1[1], a2[1])


def test_velocity_correction_mask():
    m = ci.jittered_rect(9, 5, 22)
    p = 0.3 * m.xy[:, 0] + 1.2 * m.xy[:, 1]
    ut, vt = np.cos(m.xy[:, 0]), np.sin(m.xy[:, 1])
    mask = np.random.default_rng(4).integers(0, 4, m.n_nodes).astype(np.uint8)
    u, v = fem.velocity_correction(m.xy, m.tri, p, ut, vt, 0.5, mask=mask)
    np.testing.assert_allclose(u, np.where(mask & 1, ut, ut - 0.15), rtol=0, atol=1e-14)
    np.testing.assert_allclose(v, np.where(mask & 2, vt, vt - 0.6), rtol=0, atol=1e-14)


def test_cgp_step_keeps_uniform_flow_in_an_empty_channel():
    m = ci.jittered_rect(13, 7, 23)
    geo = {"L": 2.0, "H": 1.0}
    b = ci.channel_boundary(m.xy, m.tri, geo)
    assert b["cylinder"].sum() == 0
    phi_dir = b["inflow"] | b["outflow"] | b["walls"]
    hphi = mesh.Hierarchy(m.xy, m.tri, phi_dir, 1)
    hp = mesh.Hierarchy(m.xy, m.tri, b["outflow"], 1)
    bf = ci.channel_boundary(hp.xy[1], hp.tri[1], geo)
    vmask = (bf["inflow"] * 3 | bf["walls"] * 2).astype(np.uint8)
    n = hp.n_nodes(1)
    u, v = np.ones(n), np.zeros(n)
    for _ in range(2):
        u, v, phi, p, fx, fy, _, _ = och.cgp_step(hphi, hp, u, v, vmask, np.ones(n), np.zeros(n), 1.0, 0.01, 0.05,
                                                 0.0, 1.0)
    np.testing.assert_allclose(u, 1.0, rtol=0, atol=1e-12)
    np.testing.assert_allclose(v, 0.0, rtol=0, atol=1e-12)
    assert np.abs(p).max() < 1e-10 and np.abs(phi).max() < 1e-10


def test_channel_hierarchy_follows_the_papers_counts_law():
    # Section 3's four meshes satisfy N' = 2 N + T, T' = 4 T (one hole); so does the
    # stand-in channel mesh under the oracle's refinement, and its boundary classes carry over
    m = ci.cylinder_channel()
    h = mesh.Hierarchy(m.xy, m.tri, m.dirichlet, 3)
    for lvl in range(3):
        n, t = h.n_nodes(lvl), h.tri[lvl].shape[0]
        assert h.tri[lvl + 1].shape[0] == 4 * t and h.n_nodes(lvl + 1) == 2 * n + t
    assert (h.n_nodes(3), h.tri[3].shape[0]) == (107244, 213440)
    b = ci.channel_boundary(h.xy[3], h.tri[3], m.geometry)
    assert b["cyl_edges"].shape[0] == 8 * m.geometry["n_circle"]
    assert int(b["cylinder"].sum()) == 8 * m.geometry["n_circle"]
    nb_f = int((b["inflow"] | b["outflow"] | b["walls"] | b["cylinder"]).sum())
    nb_c = int((m.inflow | m.outflow | m.walls | m.cylinder).sum())
    assert nb_f == 8 * nb_c                               # every boundary edge split in 2, three times
