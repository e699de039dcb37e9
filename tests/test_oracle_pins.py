"""Pins of the CPU oracle against facts that do not come from the oracle itself.

Every check here is fixed by the paper's own numbers, a closed form, an
invariant of the mathematics, a textbook special case or a brute-force
computation, so that a plausible slip in the oracle (a dropped term, a flipped
sign, a swapped index or operand) fails at least one of them.
"""
import os

import numpy as np
import pytest
import scipy.sparse as sp

import cgp_inputs as ci
from oracle import fem, mesh, solve

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _grid(nx, ny, seed=None):
    return ci.jittered_rect(nx, ny, seed)


# ---------------------------------------------------------------- refinement (Eq. 18)

def test_paper_hierarchy_is_nested_four_way_refinement_of_a_one_hole_domain():
    """Section 3 mesh sizes: T_{k-1} = 4 T_k (Eq. 18) and N_{k-1} = 2 N_k + T_k.

    For a triangulated domain with one hole (Euler characteristic 0) the edge
    count is E = N + T and a 4-way split adds one node per edge."""
    rows = np.loadtxt(os.path.join(GOLDEN, "paper_mesh_hierarchy.txt"), dtype=np.int64)
    rows = rows[np.argsort(-rows[:, 0])]          # coarsest first
    for (k, n, t), (k2, n2, t2) in zip(rows[:-1], rows[1:]):
        assert k2 == k - 1
        assert t2 == 4 * t
        assert n2 == 2 * n + t


def test_oracle_refinement_counts_on_a_one_hole_mesh():
    m = ci.rect_with_hole(17, 11, (5, 9, 3, 7), seed=3)
    h = mesh.Hierarchy(m.xy, m.tri, m.dirichlet, 3)
    for lvl in range(3):
        n, t = h.n_nodes(lvl), h.tri[lvl].shape[0]
        assert h.tri[lvl + 1].shape[0] == 4 * t
        assert h.n_nodes(lvl + 1) == 2 * n + t


def test_oracle_refinement_counts_on_a_rectangle():
    nx, ny = 9, 6
    m = _grid(nx, ny, 5)
    n, t = m.n_nodes, m.n_tris
    ends, tri_edge, n_adj = mesh.edges(n, m.tri)
    assert ends.shape[0] == n + t - 1                      # Euler: V - E + F = 1
    assert int((n_adj == 1).sum()) == 2 * (nx - 1) + 2 * (ny - 1)
    assert set(np.unique(n_adj)) == {1, 2}
    xf, tf, df, _ = mesh.refine(m.xy, m.tri, m.dirichlet)
    assert xf.shape[0] == 2 * n + t - 1 == (2 * nx - 1) * (2 * ny - 1)
    assert tf.shape[0] == 4 * t
    # boundary of the fine rectangle: all nodes on the outer frame, nothing else
    on_frame = ((xf[:, 0] == 0) | (xf[:, 0] == 2) | (xf[:, 1] == 0) | (xf[:, 1] == 1))
    np.testing.assert_array_equal(df.astype(bool), on_frame)


def test_refined_unjittered_grid_is_the_twice_finer_grid():
    """The midpoints of a uniform grid with power-of-two spacing are exactly the finer grid."""
    coarse = _grid(33, 17)
    fine = _grid(65, 33)
    xf, _, df, _ = mesh.refine(coarse.xy, coarse.tri, coarse.dirichlet)
    a = np.lexsort((xf[:, 0], xf[:, 1]))
    b = np.lexsort((fine.xy[:, 0], fine.xy[:, 1]))
    np.testing.assert_array_equal(xf[a], fine.xy[b])
    np.testing.assert_array_equal(df[a], fine.dirichlet[b])


def test_children_are_ccw_quarters_of_their_parent():
    m = _grid(12, 7, 11)
    xf, tf, _, _ = mesh.refine(m.xy, m.tri, m.dirichlet)
    a_par, _, _ = fem.element_geometry(m.xy, m.tri)
    a_ch, _, _ = fem.element_geometry(xf, tf)
    assert np.all(a_ch > 0)
    np.testing.assert_allclose(a_ch.reshape(-1, 4), np.repeat(a_par[:, None] / 4, 4, axis=1), rtol=1e-12)
    # child 4t+s keeps parent vertex s (s < 3) and the middle child has only midpoints
    n = m.n_nodes
    for s in range(3):
        assert np.all(tf[s::4, s] == m.tri[:, s])
    assert np.all(tf[3::4] >= n)


def test_injection_after_prolongation_is_identity():
    m = _grid(10, 6, 2)
    h = mesh.Hierarchy(m.xy, m.tri, m.dirichlet, 2)
    q = np.random.default_rng(0).standard_normal(m.n_nodes)
    np.testing.assert_array_equal(mesh.restrict_inject(mesh.prolong(q, h), m.n_nodes), q)


def test_prolongation_is_exact_for_linear_fields():
    m = _grid(14, 8, 4)
    h = mesh.Hierarchy(m.xy, m.tri, m.dirichlet, 2)
    lin = lambda xy: 0.3 - 1.7 * xy[:, 0] + 2.9 * xy[:, 1]
    qf = mesh.prolong(lin(h.xy[0]), h)
    np.testing.assert_allclose(qf, lin(h.xy[2]), rtol=0, atol=1e-14)


def test_levelwise_prolongation_equals_one_shot_barycentric_interpolation():
    """Eq. 20 applied once per level equals P1 interpolation inside the level-0 ancestor."""
    m = _grid(9, 5, 8)
    h = mesh.Hierarchy(m.xy, m.tri, m.dirichlet, 2)
    q = np.random.default_rng(1).standard_normal(m.n_nodes)
    qf = mesh.prolong(q, h)
    parent = mesh.parent_triangle(h, 2)
    for corner in range(3):
        nodes = h.tri[2][:, corner]
        pt = h.xy[2][nodes]
        tri = m.tri[parent]
        p0, p1, p2 = m.xy[tri[:, 0]], m.xy[tri[:, 1]], m.xy[tri[:, 2]]
        det = (p1[:, 0] - p0[:, 0]) * (p2[:, 1] - p0[:, 1]) - (p2[:, 0] - p0[:, 0]) * (p1[:, 1] - p0[:, 1])
        l1 = ((pt[:, 0] - p0[:, 0]) * (p2[:, 1] - p0[:, 1]) - (p2[:, 0] - p0[:, 0]) * (pt[:, 1] - p0[:, 1])) / det
        l2 = ((p1[:, 0] - p0[:, 0]) * (pt[:, 1] - p0[:, 1]) - (pt[:, 0] - p0[:, 0]) * (p1[:, 1] - p0[:, 1])) / det
        l0 = 1.0 - l1 - l2
        bary = l0 * q[tri[:, 0]] + l1 * q[tri[:, 1]] + l2 * q[tri[:, 2]]
        np.testing.assert_allclose(qf[nodes], bary, rtol=0, atol=1e-14 * np.abs(q).max() * 8)


# ---------------------------------------------------------------- P1 stiffness

def test_unconstrained_stiffness_has_zero_row_sums_and_reproduces_linear_fields():
    m = _grid(15, 9, 21)
    k = fem.stiffness(m.xy, m.tri)
    scale = np.abs(k.data).max()
    np.testing.assert_allclose(k @ np.ones(m.n_nodes), 0, atol=1e-14 * scale)
    interior = ~m.dirichlet.astype(bool)
    for f in (m.xy[:, 0], m.xy[:, 1]):
        np.testing.assert_allclose((k @ f)[interior], 0, atol=1e-14 * scale)
    assert (k - k.T).count_nonzero() == 0 or abs(k - k.T).max() <= 1e-15 * scale


def test_unjittered_stiffness_is_the_five_point_stencil():
    """Right triangles of equal legs: P1 gives 4, -1 x 4 and exact zeros on the diagonals."""
    nx, ny = 33, 17
    m = _grid(nx, ny)
    k = fem.stiffness(m.xy, m.tri).tolil()
    for j in range(1, ny - 1):
        for i in range(1, nx - 1):
            r = j * nx + i
            row = dict(zip(k.rows[r], k.data[r]))
            assert row.pop(r) == 4.0
            for nb in (r - 1, r + 1, r - nx, r + nx):
                assert row.pop(nb) == -1.0
            assert all(v == 0.0 for v in row.values())


def test_element_areas_sum_to_the_domain_area():
    m = _grid(21, 11, 9)
    area, _, _ = fem.element_geometry(m.xy, m.tri)
    assert abs(area.sum() - 2.0) <= 1e-14


def test_system_matrix_structure():
    nx, ny = 33, 17
    m = _grid(nx, ny, 1001)
    a = fem.system_matrix(m.xy, m.tri, m.dirichlet)
    a_, b_ = nx - 2, ny - 2
    assert a.nnz == 7 * a_ * b_ - 4 * a_ - 4 * b_ + 2 + (m.n_nodes - a_ * b_)
    assert abs(a - a.T).max() == 0.0
    d = m.dirichlet.astype(bool)
    dense = a.toarray()
    np.testing.assert_array_equal(dense[d][:, d], np.eye(d.sum()))
    assert np.all(dense[d][:, ~d] == 0) and np.all(dense[~d][:, d] == 0)
    assert np.all(np.linalg.eigvalsh(dense) > 0)


# ---------------------------------------------------------------- sources (Eqs. 12, 15)

@pytest.mark.parametrize("kind", [fem.CURL, fem.DIV])
def test_source_of_a_linear_velocity(kind):
    """u = (al x + be y, ga x + de y): curl = ga - be and div = al + de on every element."""
    m = _grid(11, 7, 13)
    al, be, ga, de = 0.7, -1.3, 2.1, 0.4
    u = al * m.xy[:, 0] + be * m.xy[:, 1]
    v = ga * m.xy[:, 0] + de * m.xy[:, 1]
    area, curl, div = fem.element_curl_div(m.xy, m.tri, u, v)
    np.testing.assert_allclose(curl, ga - be, rtol=1e-12)
    np.testing.assert_allclose(div, al + de, rtol=1e-12)
    s = 1.7
    b = fem.source(m.xy, m.tri, m.dirichlet, u, v, kind, s)
    patch = np.zeros(m.n_nodes)
    for c in range(3):
        np.add.at(patch, m.tri[:, c], area)
    q = (ga - be) if kind == fem.CURL else (al + de)
    expect = np.where(m.dirichlet.astype(bool), 0.0, -s * q * patch / 3.0)
    np.testing.assert_allclose(b, expect, rtol=1e-12, atol=1e-15)


def test_source_of_a_rigid_rotation():
    m = _grid(9, 5, 17)
    u, v = -m.xy[:, 1], m.xy[:, 0]
    b = fem.source(m.xy, m.tri, m.dirichlet, u, v, fem.CURL, 1.0)
    bdiv = fem.source(m.xy, m.tri, m.dirichlet, u, v, fem.DIV, 1.0)
    area, _, _ = fem.element_geometry(m.xy, m.tri)
    patch = np.zeros(m.n_nodes)
    for c in range(3):
        np.add.at(patch, m.tri[:, c], area)
    interior = ~m.dirichlet.astype(bool)
    np.testing.assert_allclose(b[interior], -2.0 * patch[interior] / 3.0, rtol=1e-12)
    np.testing.assert_allclose(bdiv, 0.0, atol=1e-14)


def test_source_equals_the_integrated_by_parts_weak_form():
    """On interior rows: -B0 int curl(u) psi_i = B0 int (v d_x psi_i - u d_y psi_i) for P1 u, v."""
    m = _grid(13, 8, 23)
    rng = np.random.default_rng(2)
    u, v = rng.standard_normal(m.n_nodes), rng.standard_normal(m.n_nodes)
    b0 = 0.9
    b = fem.source(m.xy, m.tri, m.dirichlet, u, v, fem.CURL, b0)
    area, gx, gy = fem.element_geometry(m.xy, m.tri)
    ubar, vbar = u[m.tri].mean(axis=1), v[m.tri].mean(axis=1)
    weak = np.zeros(m.n_nodes)
    for c in range(3):
        np.add.at(weak, m.tri[:, c], b0 * area * (gx[:, c] * vbar - gy[:, c] * ubar))
    interior = ~m.dirichlet.astype(bool)
    np.testing.assert_allclose(b[interior], weak[interior], rtol=1e-11, atol=1e-14)
    # and the divergence form: -s int div(u) psi_i = s int (u d_x psi_i + v d_y psi_i)
    bd = fem.source(m.xy, m.tri, m.dirichlet, u, v, fem.DIV, b0)
    weak_d = np.zeros(m.n_nodes)
    for c in range(3):
        np.add.at(weak_d, m.tri[:, c], b0 * area * (gx[:, c] * ubar + gy[:, c] * vbar))
    np.testing.assert_allclose(bd[interior], weak_d[interior], rtol=1e-11, atol=1e-14)


# ---------------------------------------------------------------- solves

def _c1_system(seed=1001):
    m = _grid(33, 17, seed)
    return m, fem.system_matrix(m.xy, m.tri, m.dirichlet)


def test_pcg_matches_a_dense_factorisation_on_the_small_mesh():
    m, a = _c1_system()
    rng = np.random.default_rng(5)
    b = rng.standard_normal(m.n_nodes) * (~m.dirichlet.astype(bool))
    x_direct = np.linalg.solve(a.toarray(), b)          # brute force on 561 unknowns
    x, info = solve.pcg(a, b, tol=1e-13)
    assert info["status"] == "ok" and info["rel_res"] <= 1e-13
    assert np.linalg.norm(x - x_direct) / np.linalg.norm(x_direct) <= 1e-10
    xm, infom = solve.pcg_mixed(a, b, tol=1e-10)
    assert infom["status"] == "ok" and infom["rel_res"] <= 1e-10
    assert np.linalg.norm(xm - x_direct) / np.linalg.norm(x_direct) <= 1e-7


def _start_at_relative_residual(a, b, free, rel, seed):
    """x* plus a random free-node perturbation scaled so that ||b - K x0|| = rel ||b||."""
    xs = np.linalg.solve(a.toarray(), b)
    y = np.random.default_rng(seed).standard_normal(b.shape[0]) * free
    return xs + y * (rel * np.linalg.norm(b) / np.linalg.norm(a @ y)), xs


@pytest.mark.parametrize("rel, phases", [(1.66e-2, 3), (2.0e-3, 3), (6.0e-2, 4)])
def test_mixed_refinement_runs_a_short_last_phase_into_the_previous_one(rel, phases):
    """fp32 PCG refined every two decades (delta = 0.01) to 1e-8 from a start at relative residual
    rel.  From 1.66e-2 the phases end near 1.66e-4 and 1.66e-6; the third one's refinement point
    1.66e-8 is within half a decade of the tolerance, so that phase runs to it: three true
    residuals after the start (where refining at every point would take four).  From 2e-3 the third
    phase reaches the tolerance before its point 2e-9 anyway (three); from 6e-2 the third point
    6e-8 is more than half a decade above it, so a fourth, short phase follows (four).  Each start
    solves to the tolerance."""
    m, a = _c1_system()
    free = ~m.dirichlet.astype(bool)
    b = np.random.default_rng(11).standard_normal(m.n_nodes) * free
    x0, xs = _start_at_relative_residual(a, b, free, rel, seed=12)
    x, info = solve.pcg_mixed(a, b, x0=x0, tol=1e-8, delta=0.01)
    assert info["status"] == "ok" and info["rel_res"] <= 1e-8
    assert info["updates"] == phases, info
    assert np.linalg.norm(x - xs) / np.linalg.norm(xs) <= 1e-6


def test_pcg_recovers_discrete_sine_modes_in_as_many_steps_as_modes():
    """Unjittered grid: K v_pq = lambda_pq v_pq with lambda = 4 - 2cos(p pi/(nx-1)) - 2cos(q pi/(ny-1))."""
    nx, ny = 33, 17
    m = _grid(nx, ny)
    a = fem.system_matrix(m.xy, m.tri, m.dirichlet)
    i = np.arange(m.n_nodes) % nx
    j = np.arange(m.n_nodes) // nx
    modes = [(1, 1, 1.0), (3, 2, -0.5), (7, 5, 0.25), (20, 9, 2.0)]
    b = np.zeros(m.n_nodes)
    expect = np.zeros(m.n_nodes)
    for p, q, c in modes:
        vpq = np.sin(p * np.pi * i / (nx - 1)) * np.sin(q * np.pi * j / (ny - 1))
        lam = 4 - 2 * np.cos(p * np.pi / (nx - 1)) - 2 * np.cos(q * np.pi / (ny - 1))
        b += c * vpq
        expect += c * vpq / lam
    b[m.dirichlet.astype(bool)] = 0.0
    expect[m.dirichlet.astype(bool)] = 0.0
    x, info = solve.pcg(a, b, tol=1e-12)
    # m distinct eigenvalues: exact arithmetic ends after m steps; one more absorbs rounding
    assert info["iters"] <= len(modes) + 1
    np.testing.assert_allclose(x, expect, rtol=0, atol=1e-12 * np.abs(expect).max())


def _load_by_midpoint_rule(xy, tri, f):
    """int f psi_i by the edge-midpoint rule (exact for quadratics): A_e/6 (f(m_ij) + f(m_ik))."""
    area, _, _ = fem.element_geometry(xy, tri)
    out = np.zeros(xy.shape[0])
    for c in range(3):
        a, b, d = tri[:, c], tri[:, (c + 1) % 3], tri[:, (c + 2) % 3]
        fab = f(0.5 * (xy[a] + xy[b]))
        fad = f(0.5 * (xy[a] + xy[d]))
        np.add.at(out, a, area / 6.0 * (fab + fad))
    return out


def _rms(e):
    """Discrete L2 error over the nodes (the max norm carries an extra log factor on jittered meshes)."""
    return float(np.sqrt(np.mean(np.asarray(e) ** 2)))


def _orders(errors):
    e = np.asarray(errors)
    return np.log2(e[:-1] / e[1:])


def test_manufactured_solution_converges_at_second_order():
    """phi = sin(pi x) sin(pi y) on [0,2]x[0,1]: Delta phi = -2 pi^2 phi, nodal error O(h^2)."""
    base = _grid(17, 9, 77)
    h = mesh.Hierarchy(base.xy, base.tri, base.dirichlet, 3)
    exact = lambda xy: np.sin(np.pi * xy[:, 0]) * np.sin(np.pi * xy[:, 1])
    errs = []
    for lvl in range(4):
        xy, tri, d = h.xy[lvl], h.tri[lvl], h.dirichlet[lvl]
        a = fem.system_matrix(xy, tri, d)
        b = 2 * np.pi ** 2 * _load_by_midpoint_rule(xy, tri, exact)   # -int f psi_i
        b[d.astype(bool)] = 0.0
        phi = solve.direct(a, b)
        errs.append(_rms(phi - exact(xy)))
    order = _orders(errs)
    assert np.all(order > 1.85) and np.all(order < 2.15), (errs, order)


# ---------------------------------------------------------------- gradient and Lorentz force (Eqs. 13-14)

def test_gradient_of_a_linear_field_is_constant():
    m = _grid(12, 7, 31)
    phi = 0.5 + 1.25 * m.xy[:, 0] - 3.0 * m.xy[:, 1]
    g = fem.nodal_gradient(m.xy, m.tri, phi)
    np.testing.assert_allclose(g[:, 0], 1.25, rtol=1e-13)
    np.testing.assert_allclose(g[:, 1], -3.0, rtol=1e-13)


def test_lorentz_force_closed_forms():
    m = _grid(12, 7, 37)
    rng = np.random.default_rng(3)
    u, v = rng.standard_normal(m.n_nodes), rng.standard_normal(m.n_nodes)
    sigma, b0 = 0.37, 1.6
    fx, fy, _ = fem.lorentz_force(m.xy, m.tri, np.zeros(m.n_nodes), u, v, sigma, b0)
    np.testing.assert_allclose(fx, -sigma * b0 * b0 * u, rtol=4e-16, atol=0)
    np.testing.assert_allclose(fy, -sigma * b0 * b0 * v, rtol=4e-16, atol=0)
    # linear phi: F = sigma B0 (-phi_y - B0 u, phi_x - B0 v) with constant gradient
    phi = 2.0 * m.xy[:, 0] + 0.5 * m.xy[:, 1]
    fx, fy, _ = fem.lorentz_force(m.xy, m.tri, phi, u, v, sigma, b0)
    np.testing.assert_allclose(fx, sigma * b0 * (-0.5 - b0 * u), rtol=1e-12)
    np.testing.assert_allclose(fy, sigma * b0 * (2.0 - b0 * v), rtol=1e-12)
    # linear in sigma
    phi = rng.standard_normal(m.n_nodes)
    f1 = fem.lorentz_force(m.xy, m.tri, phi, u, v, 1.0, b0)
    f3 = fem.lorentz_force(m.xy, m.tri, phi, u, v, 3.0, b0)
    np.testing.assert_allclose(f3[0], 3.0 * f1[0], rtol=1e-14)
    np.testing.assert_allclose(f3[1], 3.0 * f1[1], rtol=1e-14)


def test_velocity_correction_of_a_linear_pressure():
    m = _grid(12, 7, 43)
    rng = np.random.default_rng(5)
    ut, vt = rng.standard_normal(m.n_nodes), rng.standard_normal(m.n_nodes)
    p = -0.75 + 2.5 * m.xy[:, 0] + 0.25 * m.xy[:, 1]
    u, v = fem.velocity_correction(m.xy, m.tri, p, ut, vt, 0.2)
    np.testing.assert_allclose(u, ut - 0.2 * 2.5, rtol=0, atol=1e-13)
    np.testing.assert_allclose(v, vt - 0.2 * 0.25, rtol=0, atol=1e-13)


def test_gradient_of_a_quadratic_is_exact_on_point_symmetric_patches():
    # unjittered grid: the six equal triangles around an interior node are point-symmetric
    # about it, so the averaged gradient of the interpolated quadratic is the exact gradient
    m = _grid(9, 6, None)
    x, y = m.xy[:, 0], m.xy[:, 1]
    p = x * x + 3.0 * x * y - 2.0 * y * y
    g = fem.nodal_gradient(m.xy, m.tri, p)
    inner = m.dirichlet == 0
    np.testing.assert_allclose(g[inner, 0], (2 * x + 3 * y)[inner], rtol=0, atol=1e-12)
    np.testing.assert_allclose(g[inner, 1], (3 * x - 4 * y)[inner], rtol=0, atol=1e-12)


def _projection_residual(coarse, rho_dt=4.0):
    """One CGP pressure projection (steps 5-8) of ut = grad(chi) + curl(psi) on the fine mesh.

    chi and psi vanish on the boundary, so Eq. 15 gives p = (rho/dt) chi and Eqs. 16-17
    return the divergence-free part curl(psi) = (psi_y, -psi_x)."""
    h = mesh.Hierarchy(coarse.xy, coarse.tri, coarse.dirichlet, 1)
    x, y = h.xy[1][:, 0], h.xy[1][:, 1]
    sx, cx = np.sin(np.pi * x / 2), np.cos(np.pi * x / 2)
    sy, cy = np.sin(np.pi * y), np.cos(np.pi * y)
    chi_x, chi_y = np.pi / 2 * cx * sy, np.pi * sx * cy           # chi = sin(pi x/2) sin(pi y)
    s2x, c2x = np.sin(np.pi * x), np.cos(np.pi * x)
    psi_x, psi_y = np.pi * c2x * sy * sy, 2 * np.pi * s2x * sy * cy   # psi = sin(pi x) sin(pi y)^2
    ut, vt = chi_x + psi_y, chi_y - psi_x
    n = coarse.n_nodes
    a = fem.system_matrix(coarse.xy, coarse.tri, coarse.dirichlet)
    b = fem.source(coarse.xy, coarse.tri, coarse.dirichlet, mesh.restrict_inject(ut, n),
                   mesh.restrict_inject(vt, n), fem.DIV, rho_dt)
    p_f = mesh.prolong(solve.direct(a, b), h)
    u, v = fem.velocity_correction(h.xy[1], h.tri[1], p_f, ut, vt, 1.0 / rho_dt)
    return _rms(np.hypot(u - psi_y, v + psi_x)), _rms(np.hypot(chi_x, chi_y))


def test_projection_removes_the_gradient_part():
    base = _grid(17, 9, 5)
    h = mesh.Hierarchy(base.xy, base.tri, base.dirichlet, 2)
    res = [_projection_residual(ci.Mesh(h.xy[l], h.tri[l], h.dirichlet[l])) for l in range(3)]
    err = [r for r, _ in res]
    assert err[-1] < 0.05 * res[-1][1], res
    order = _orders(err)
    assert np.all(order > 0.9), (err, order)


def test_prolonged_field_has_the_parent_gradient_on_every_child():
    m = _grid(10, 6, 41)
    h = mesh.Hierarchy(m.xy, m.tri, m.dirichlet, 2)
    q = np.random.default_rng(4).standard_normal(m.n_nodes)
    g0 = fem.element_gradient(m.xy, m.tri, q)
    g2 = fem.element_gradient(h.xy[2], h.tri[2], mesh.prolong(q, h))
    np.testing.assert_allclose(g2, g0[mesh.parent_triangle(h, 2)], rtol=1e-10, atol=1e-12 * np.abs(g0).max())


def _cgp_phi_error(coarse, b0=1.0):
    """Restrict -> solve Eq. 12 -> prolong for the stream function psi = sin(pi x/2) sin(pi y).

    psi vanishes on the boundary, so Delta phi = B0 curl(u) = -B0 Delta psi gives phi = -B0 psi
    and j = sigma(-grad phi + u x B) = 0."""
    h = mesh.Hierarchy(coarse.xy, coarse.tri, coarse.dirichlet, 1)
    xy = h.xy[1]
    psi = lambda p: np.sin(np.pi * p[:, 0] / 2) * np.sin(np.pi * p[:, 1])
    u = np.pi * np.sin(np.pi * xy[:, 0] / 2) * np.cos(np.pi * xy[:, 1])
    v = -np.pi / 2 * np.cos(np.pi * xy[:, 0] / 2) * np.sin(np.pi * xy[:, 1])
    n = coarse.n_nodes
    a = fem.system_matrix(coarse.xy, coarse.tri, coarse.dirichlet)
    b = fem.source(coarse.xy, coarse.tri, coarse.dirichlet, mesh.restrict_inject(u, n),
                   mesh.restrict_inject(v, n), fem.CURL, b0)
    phi_f = mesh.prolong(solve.direct(a, b), h)
    fx, fy, _ = fem.lorentz_force(xy, h.tri[1], phi_f, u, v, 1.0, b0)
    return _rms(phi_f + b0 * psi(xy)), _rms(np.sqrt(fx ** 2 + fy ** 2))


def test_cgp_step_reproduces_the_manufactured_potential():
    base = _grid(17, 9, 5)
    h = mesh.Hierarchy(base.xy, base.tri, base.dirichlet, 2)
    phi_err, force = zip(*[_cgp_phi_error(ci.Mesh(h.xy[l], h.tri[l], h.dirichlet[l])) for l in range(3)])
    order = _orders(phi_err)
    assert np.all(order > 1.8) and np.all(order < 2.3), (phi_err, order)
    force_order = _orders(force)
    assert np.all(force_order > 0.7), (force, force_order)


def test_pressure_step_reproduces_a_gradient_velocity():
    """u~ = grad chi with chi = 0 on the boundary: Delta p = (rho/dt) div u~ gives p = (rho/dt) chi."""
    base = _grid(17, 9, 6)
    h = mesh.Hierarchy(base.xy, base.tri, base.dirichlet, 3)
    rho_dt = 1.0 / ci.DT
    errs = []
    for lvl in range(3):
        xy_c, tri_c, d_c = h.xy[lvl], h.tri[lvl], h.dirichlet[lvl]
        xy_f = h.xy[lvl + 1]
        u = np.pi / 2 * np.cos(np.pi * xy_f[:, 0] / 2) * np.sin(np.pi * xy_f[:, 1])
        v = np.pi * np.sin(np.pi * xy_f[:, 0] / 2) * np.cos(np.pi * xy_f[:, 1])
        n = xy_c.shape[0]
        a = fem.system_matrix(xy_c, tri_c, d_c)
        b = fem.source(xy_c, tri_c, d_c, u[:n], v[:n], fem.DIV, rho_dt)
        p = solve.direct(a, b)
        chi = np.sin(np.pi * xy_c[:, 0] / 2) * np.sin(np.pi * xy_c[:, 1])
        errs.append(_rms(p - rho_dt * chi) / rho_dt)
    order = _orders(errs)
    assert np.all(order > 1.8) and np.all(order < 2.3), (errs, order)


# ---------------------------------------------------------------- solver edge cases

def test_zero_rhs_gives_zero_in_zero_iterations():
    m, a = _c1_system()
    for fn in (solve.pcg, solve.pcg_mixed):
        x, info = fn(a, np.zeros(m.n_nodes), np.ones(m.n_nodes))
        assert info["status"] == "ok" and info["iters"] == 0 and not x.any()


def test_exact_guess_needs_no_iteration():
    m, a = _c1_system()
    b = np.random.default_rng(7).standard_normal(m.n_nodes) * (~m.dirichlet.astype(bool))
    xs = solve.direct(a, b)
    for fn in (solve.pcg, solve.pcg_mixed):
        _, info = fn(a, b, xs, tol=1e-8)
        assert info["status"] == "ok" and info["iters"] == 0


def test_failure_statuses():
    m, a = _c1_system()
    b = np.random.default_rng(8).standard_normal(m.n_nodes) * (~m.dirichlet.astype(bool))
    _, info = solve.pcg(a, b, tol=1e-10, max_iter=1)
    assert info["status"] == "noconv" and info["iters"] == 1
    _, info = solve.pcg_mixed(a, b, tol=1e-10, max_iter=1)
    assert info["status"] == "noconv"
    bad = b.copy()
    bad[100] = np.nan
    for fn in (solve.pcg, solve.pcg_mixed):
        _, info = fn(a, bad)
        assert info["status"] == "breakdown"
    # indefinite matrix: p.Kp <= 0 is detected
    neg = sp.csr_matrix(-a.toarray())
    _, info = solve.pcg(neg, b)
    assert info["status"] == "breakdown"


def test_guess_independence_of_the_result():
    m, a = _c1_system()
    b = np.random.default_rng(9).standard_normal(m.n_nodes) * (~m.dirichlet.astype(bool))
    xs = solve.direct(a, b)
    kappa = np.linalg.cond(a.toarray())
    for x0 in (None, np.ones(m.n_nodes), xs + 1e-3):
        x, info = solve.pcg(a, b, x0, tol=1e-10)
        assert np.linalg.norm(x - xs) / np.linalg.norm(xs) <= kappa * 1e-10
