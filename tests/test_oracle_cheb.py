"""Pins of the oracle's Chebyshev polynomial preconditioner (CPU only).

The preconditioner is the iterate after d steps of Chebyshev iteration for K z = r
preconditioned by D = diag(K), from z = 0, with the spectrum of D^-1 K taken in
[lo, hi].  On an eigenvector it acts as a scalar fixed by the Chebyshev
polynomial T_d (numpy's Chebyshev-series routine gives T_d independently).
"""
import numpy as np
import pytest
from numpy.polynomial import chebyshev as C

import cgp_inputs as ci
from oracle import fem, solve


def _scalar(mu, d, lo, hi):
    """s(mu) with mu s(mu) = 1 - T_d((c - mu)/e) / T_d(c/e)."""
    c, e = 0.5 * (hi + lo), 0.5 * (hi - lo)
    td = np.zeros(d + 1)
    td[d] = 1.0
    return (1.0 - C.chebval((c - mu) / e, td) / C.chebval(c / e, td)) / mu


@pytest.mark.parametrize("d", [2, 3, 5, 8])
def test_acts_on_sine_modes_through_the_chebyshev_polynomial(d):
    nx, ny = 33, 17
    m = ci.jittered_rect(nx, ny, None)
    a = fem.system_matrix(m.xy, m.tri, m.dirichlet)   # 5-point stencil, diag 4 on free rows
    i = np.arange(m.n_nodes) % nx
    j = np.arange(m.n_nodes) // nx
    lo, hi = 2.2e-3, 2.2
    r = np.zeros(m.n_nodes)
    expect = np.zeros(m.n_nodes)
    for p, q, c in ((1, 1, 1.0), (4, 3, -0.7), (9, 2, 0.3), (30, 15, 1.5)):
        v = np.sin(p * np.pi * i / (nx - 1)) * np.sin(q * np.pi * j / (ny - 1))
        v[m.dirichlet.astype(bool)] = 0.0
        mu = (4 - 2 * np.cos(p * np.pi / (nx - 1)) - 2 * np.cos(q * np.pi / (ny - 1))) / 4.0
        r += c * 4.0 * v
        expect += c * _scalar(mu, d, lo, hi) * v
    z = solve.cheb_apply(a, r, d, lo, hi)
    np.testing.assert_allclose(z, expect, rtol=0, atol=1e-12 * np.abs(expect).max())


def test_degree_one_is_jacobi():
    m = ci.jittered_rect(15, 9, 4)
    a = fem.system_matrix(m.xy, m.tri, m.dirichlet)
    r = np.random.default_rng(0).standard_normal(m.n_nodes)
    np.testing.assert_array_equal(solve.cheb_apply(a, r, 1), (1.0 / a.diagonal()) * r)


def test_is_symmetric_positive_definite_on_a_jittered_mesh():
    m = ci.jittered_rect(25, 13, 7)
    a = fem.system_matrix(m.xy, m.tri, m.dirichlet)
    rng = np.random.default_rng(1)
    for d in (2, 4, 7):
        v, w = rng.standard_normal(m.n_nodes), rng.standard_normal(m.n_nodes)
        cv, cw = solve.cheb_apply(a, v, d), solve.cheb_apply(a, w, d)
        assert w @ cv == pytest.approx(v @ cw, rel=1e-12)
        assert v @ cv > 0 and w @ cw > 0


def test_gershgorin_bound_bounds_the_spectrum():
    m = ci.jittered_rect(17, 9, 3)
    a = fem.system_matrix(m.xy, m.tri, m.dirichlet)
    d = a.diagonal()
    s = np.diag(d ** -0.5) @ a.toarray() @ np.diag(d ** -0.5)
    lam = np.linalg.eigvalsh(s)
    hi = solve.gershgorin_bound(a)
    assert lam.max() <= hi * (1 + 1e-14)
    assert hi < 3.0


@pytest.mark.parametrize("degree", [3, 6])
def test_polynomial_pcg_solves_with_fewer_iterations(degree):
    m = ci.jittered_rect(65, 33, 12)
    a = fem.system_matrix(m.xy, m.tri, m.dirichlet)
    u, v = ci.stream_velocity(m.xy, ci.fourier_modes(5), 0.0)
    b = fem.source(m.xy, m.tri, m.dirichlet, u, v, fem.CURL, 1.0)
    xs = solve.direct(a, b)
    _, jac = solve.pcg(a, b, tol=1e-10)
    x, info = solve.pcg(a, b, tol=1e-10, degree=degree)
    assert info["status"] == "ok" and info["rel_res"] <= 1e-10
    assert np.linalg.norm(x - xs) / np.linalg.norm(xs) <= 1e-8
    assert info["iters"] <= 2.2 * jac["iters"] / degree, (info, jac)
    xm, mixed = solve.pcg_mixed(a, b, tol=1e-8, degree=degree)
    assert mixed["status"] == "ok" and mixed["rel_res"] <= 1e-8
    assert np.linalg.norm(xm - xs) / np.linalg.norm(xs) <= 1e-6
    assert mixed["iters"] <= 2.2 * jac["iters"] / degree, (mixed, jac)
