"""Pins of the momentum-step oracle (Eqs. 13-14, Galerkin P1).

Independent of the oracle's closed forms: the mass and convection entries against
a quadrature of the shape functions evaluated at points (the edge-midpoint rule,
exact for the quadratic integrands), the area of the domain, the null spaces and
the exact action on linear fields, and a manufactured intermediate velocity that
the step must reproduce.
"""
import numpy as np
import pytest

import cgp_inputs as ci
from oracle import fem
from oracle import momentum as mom


def _shape(xy, t, p):
    """Barycentric coordinates (the three P1 shape functions) of point p in triangle t."""
    a, b, c = xy[t]
    m = np.array([[b[0] - a[0], c[0] - a[0]], [b[1] - a[1], c[1] - a[1]]])
    l1, l2 = np.linalg.solve(m, p - a)
    return np.array([1.0 - l1 - l2, l1, l2])


def _quadrature(xy, tri, ax, ay):
    """M and C by the edge-midpoint rule (exact for polynomials of degree two); the
    gradients of the shape functions from finite differences of the barycentric map."""
    n = xy.shape[0]
    mq = np.zeros((n, n))
    cq = np.zeros((n, n))
    for t in tri:
        v = xy[t]
        e1, e2 = v[1] - v[0], v[2] - v[0]
        area = 0.5 * abs(e1[0] * e2[1] - e1[1] * e2[0])
        h = 1e-6
        c0 = v.mean(axis=0)
        grad = np.stack([(_shape(xy, t, c0 + [h, 0]) - _shape(xy, t, c0 - [h, 0])) / (2 * h),
                         (_shape(xy, t, c0 + [0, h]) - _shape(xy, t, c0 - [0, h])) / (2 * h)], axis=1)
        for p in (0.5 * (v[0] + v[1]), 0.5 * (v[1] + v[2]), 0.5 * (v[2] + v[0])):
            s = _shape(xy, t, p)
            a = np.array([s @ ax[t], s @ ay[t]])
            for i in range(3):
                for j in range(3):
                    mq[t[i], t[j]] += area / 3.0 * s[i] * s[j]
                    cq[t[i], t[j]] += area / 3.0 * s[i] * (a @ grad[j])
    return mq, cq


def test_mass_and_convection_against_quadrature():
    m = ci.jittered_rect(5, 4, 3)
    rng = np.random.default_rng(0)
    ax, ay = rng.standard_normal(m.n_nodes), rng.standard_normal(m.n_nodes)
    mq, cq = _quadrature(m.xy, m.tri, ax, ay)
    np.testing.assert_allclose(mom.mass(m.xy, m.tri).toarray(), mq, rtol=0, atol=1e-14)
    np.testing.assert_allclose(mom.convection(m.xy, m.tri, ax, ay).toarray(), cq, rtol=0, atol=1e-8)


def test_mass_integrates_the_domain_and_convection_kills_constants():
    m = ci.rect_with_hole(13, 9, (4, 7, 3, 5), seed=4)
    ms = mom.mass(m.xy, m.tri)
    area, _, _ = fem.element_geometry(m.xy, m.tri)
    one = np.ones(m.n_nodes)
    assert one @ (ms @ one) == pytest.approx(area.sum(), rel=1e-14)
    assert one @ (ms @ one) == pytest.approx(2.0 - (3 * 2) * (2.0 / 12) * (1.0 / 8), rel=1e-12)   # box minus hole
    rng = np.random.default_rng(1)
    c = mom.convection(m.xy, m.tri, rng.standard_normal(m.n_nodes), rng.standard_normal(m.n_nodes))
    np.testing.assert_allclose(c @ one, 0.0, atol=1e-13)


def test_convection_of_a_linear_field_by_a_constant_velocity():
    # int psi_i (a . grad w) = (a . g) int psi_i for w = g . x + c: C w = (a . g) M 1, at every row
    m = ci.jittered_rect(11, 7, 5)
    a, g = np.array([0.7, -1.3]), np.array([2.0, 0.5])
    w = m.xy @ g + 0.25
    c = mom.convection(m.xy, m.tri, np.full(m.n_nodes, a[0]), np.full(m.n_nodes, a[1]))
    np.testing.assert_allclose(c @ w, (a @ g) * (mom.mass(m.xy, m.tri) @ np.ones(m.n_nodes)), rtol=0, atol=1e-13)


def test_step_reproduces_a_manufactured_intermediate_velocity():
    # w* linear, u^n constant: K w* vanishes on interior rows and C w* = (a . g) M 1, so the
    # force f = (rho/dt)(w* - w^n) + rho (a . g) makes w* the exact solution
    m = ci.jittered_rect(17, 9, 6)
    rho, mu, dt = 1.3, 0.02, 0.05
    a = np.array([0.4, -0.2])
    un, vn = np.full(m.n_nodes, a[0]), np.full(m.n_nodes, a[1])
    gu, gv = np.array([1.5, -0.5]), np.array([-0.3, 0.8])
    us, vs = m.xy @ gu + 0.1, m.xy @ gv - 0.2
    fx = (rho / dt) * (us - un) + rho * (a @ gu)
    fy = (rho / dt) * (vs - vn) + rho * (a @ gv)
    ut, vt = mom.step(m.xy, m.tri, m.dirichlet, un, vn, fx, fy, rho, mu, dt, gu=us, gv=vs)
    np.testing.assert_allclose(ut, us, rtol=0, atol=1e-12)
    np.testing.assert_allclose(vt, vs, rtol=0, atol=1e-12)


def test_operator_rows():
    m = ci.jittered_rect(9, 6, 7)
    rng = np.random.default_rng(2)
    un, vn = rng.standard_normal(m.n_nodes), rng.standard_normal(m.n_nodes)
    a = mom.operator(m.xy, m.tri, m.dirichlet, un, vn, 1.0, 0.01, 0.05)
    d = m.dirichlet.astype(bool)
    ad = a.toarray()
    np.testing.assert_array_equal(ad[d], np.eye(m.n_nodes)[d])          # identity rows
    free = np.flatnonzero(~d)
    # free rows: (rho/dt) M + rho C + mu K, their Dirichlet columns kept
    full = (20.0 * mom.mass(m.xy, m.tri) + mom.convection(m.xy, m.tri, un, vn)
            + 0.01 * fem.stiffness(m.xy, m.tri)).toarray()
    np.testing.assert_allclose(ad[free], full[free], rtol=0, atol=1e-15 * np.abs(full).max())
