"""Pins of the learned-guess network oracle (CPU only).

The network is an extension of the paper's method (a learned initial guess for
the coarse Poisson solves of Section 2.2), so nothing in the paper fixes its
values; the pins below fix what mathematics does: bfloat16 rounding against
hand-worked cases and torch's own conversion, the analytic backward pass
against central differences, the loss against the energy norm of the guess
error written in the solution's units, the zero-decoder case that reduces to
the extrapolation 2 phi^{n-1} - phi^{n-2}, homogeneity of degree one in the
inputs, and equivariance under a renumbering of the nodes.
"""
import numpy as np
import pytest

import cgp_inputs as ci
from oracle import fem, gnn


def _problem(nx=9, ny=6, seed=11):
    m = ci.jittered_rect(nx, ny, seed)
    k = fem.system_matrix(m.xy, m.tri, m.dirichlet)
    rng = np.random.default_rng(seed)
    free = m.dirichlet == 0
    b, p1, p2, tgt = (rng.standard_normal(m.n_nodes) * free for _ in range(4))
    mean_op = gnn.neighbour_mean_operator(gnn.triangle_adjacency(m.n_nodes, m.tri))
    return m, k, b, p1, p2, tgt, mean_op


def _theta(seed=3, scale=0.3):
    rng = np.random.default_rng(seed)
    return rng.standard_normal(gnn.param_count()) * scale


def test_param_layout():
    assert gnn.param_count() == 16 * 64 + 64 + 3 * (128 * 64 + 64) + 64 + 1
    th = _theta()
    np.testing.assert_array_equal(gnn.pack(gnn.unpack(th)), th)


def test_bf16_rounding_hand_cases():
    u = 2.0 ** -7                       # bfloat16 spacing just above 1
    cases = [(1.0, 1.0), (1 + u / 2, 1.0), (1 + 3 * u / 2, 1 + 2 * u), (1 + u / 2 + 2 ** -20, 1 + u),
             (-(1 + 3 * u / 2), -(1 + 2 * u)), (3.0, 3.0), (0.0, 0.0), (2.0 ** -130, 2.0 ** -130)]
    for x, want in cases:
        assert gnn.bf16(np.array([x]))[0] == want, x


def test_bf16_matches_torch_conversion():
    torch = pytest.importorskip("torch")
    x = np.random.default_rng(0).standard_normal(20000) * np.exp(np.random.default_rng(1).uniform(-20, 20, 20000))
    want = torch.tensor(x.astype(np.float32)).to(torch.bfloat16).to(torch.float64).numpy()
    np.testing.assert_array_equal(gnn.bf16(x), want)


def test_mean_operator_rows():
    m = ci.jittered_rect(6, 5, 2)
    mo = gnn.neighbour_mean_operator(gnn.triangle_adjacency(m.n_nodes, m.tri))
    np.testing.assert_allclose(np.asarray(mo.sum(axis=1)).ravel(), 1.0, rtol=1e-15)
    assert np.all(mo.diagonal() == 0)
    # interior node of the "/" split grid: six neighbours
    i = 2 * 6 + 2
    assert mo[i].nnz == 6


def test_backward_matches_central_differences():
    m, k, b, p1, p2, tgt, mo = _problem()
    th = _theta()
    loss, g = gnn.loss_and_grad(th, k, m.dirichlet, b, p1, p2, tgt, mo, emulate=False)
    rng = np.random.default_rng(5)
    names = [n for n, _ in gnn.param_shapes()]
    offs = np.cumsum([0] + [int(np.prod(s)) for _, s in gnn.param_shapes()])
    picks = []
    for q, name in enumerate(names):
        lo, hi = offs[q], offs[q + 1]
        if name == "W0":
            hi = lo + 8 * 64                 # rows 9..16 multiply zero padding
        picks += list(rng.integers(lo, hi, size=min(6, hi - lo)))
    h = 1e-6
    for p in picks:
        tp, tm = th.copy(), th.copy()
        tp[p] += h
        tm[p] -= h
        lp, _ = gnn.loss_and_grad(tp, k, m.dirichlet, b, p1, p2, tgt, mo, emulate=False)
        lm, _ = gnn.loss_and_grad(tm, k, m.dirichlet, b, p1, p2, tgt, mo, emulate=False)
        fd = (lp - lm) / (2 * h)
        assert abs(fd - g[p]) <= 1e-6 * max(1.0, abs(fd)) + 1e-7 * loss, (p, fd, g[p])
    np.testing.assert_array_equal(g[8 * 64:16 * 64], 0.0)


def test_loss_is_energy_norm_of_guess_error():
    m, k, b, p1, p2, tgt, mo = _problem()
    th = _theta()
    for emulate in (False, True):
        loss, _ = gnn.loss_and_grad(th, k, m.dirichlet, b, p1, p2, tgt, mo, emulate=emulate)
        g = gnn.guess(th, k, m.dirichlet, b, p1, p2, mo, emulate=emulate, sweeps=0)
        d = p1 - p2
        sd = np.sqrt(np.mean(d * d))
        err = g - tgt
        nfree = np.count_nonzero(m.dirichlet == 0)
        assert loss == pytest.approx(float(err @ (k @ err)) / (sd * sd * nfree), rel=1e-12)


def test_zero_decoder_gives_extrapolation():
    m, k, b, p1, p2, tgt, mo = _problem()
    p = gnn.unpack(_theta())
    p["wd"][:] = 0.0
    p["cd"][:] = 0.0
    g = gnn.guess(gnn.pack(p), k, m.dirichlet, b, p1, p2, mo, emulate=True, sweeps=0)
    free = m.dirichlet == 0
    np.testing.assert_array_equal(g[free], (2 * p1 - p2)[free])
    np.testing.assert_array_equal(g[~free], 0.0)
    # with the smoothing sweeps: the extrapolation, smoothed
    g4 = gnn.guess(gnn.pack(p), k, m.dirichlet, b, p1, p2, mo, emulate=True)
    np.testing.assert_array_equal(g4, gnn.smooth(k, b, (2 * p1 - p2) * free))


def test_smoothing_damps_sine_modes_by_the_jacobi_factor():
    # unjittered grid: K = 5-point stencil (D = 4 on free rows); with b = K x* the error
    # of a sine mode is multiplied by (1 - omega lam / 4) per sweep
    nx, ny = 33, 17
    m = ci.jittered_rect(nx, ny, None)
    k = fem.system_matrix(m.xy, m.tri, m.dirichlet)
    i = np.arange(m.n_nodes) % nx
    j = np.arange(m.n_nodes) // nx
    xs = np.sin(np.pi * i / (nx - 1)) * np.sin(2 * np.pi * j / (ny - 1))
    b = k @ xs
    err = np.zeros(m.n_nodes)
    expect = np.zeros(m.n_nodes)
    for p, q, c in ((1, 1, 1.0), (20, 10, 0.5), (31, 15, -0.25)):
        v = np.sin(p * np.pi * i / (nx - 1)) * np.sin(q * np.pi * j / (ny - 1))
        lam = 4 - 2 * np.cos(p * np.pi / (nx - 1)) - 2 * np.cos(q * np.pi / (ny - 1))
        err += c * v
        expect += c * v * (1 - gnn.SMOOTH_OMEGA * lam / 4) ** 3
    x = gnn.smooth(k, b, xs + err, sweeps=3)
    np.testing.assert_allclose(x - xs, expect, rtol=0, atol=1e-13)


def test_guess_is_homogeneous_of_degree_one():
    m, k, b, p1, p2, tgt, mo = _problem()
    th = _theta()
    g1 = gnn.guess(th, k, m.dirichlet, b, p1, p2, mo, emulate=False)
    g2 = gnn.guess(th, k, m.dirichlet, 4.0 * b, 4.0 * p1, 4.0 * p2, mo, emulate=False)   # smoothing is linear
    np.testing.assert_allclose(g2, 4.0 * g1, rtol=1e-12, atol=1e-14 * np.abs(g1).max())


def test_guess_is_equivariant_under_renumbering():
    m0 = ci.jittered_rect(9, 6, 11)
    m1 = ci.permuted(m0, seed=7)
    # recover the permutation from the coordinates
    key0 = {tuple(c): i for i, c in enumerate(m0.xy)}
    perm = np.array([key0[tuple(c)] for c in m1.xy])      # node i of m1 is node perm[i] of m0
    rng = np.random.default_rng(2)
    free = m0.dirichlet == 0
    b, p1, p2 = (rng.standard_normal(m0.n_nodes) * free for _ in range(3))
    th = _theta()
    out = []
    for m, bb, q1, q2 in ((m0, b, p1, p2), (m1, b[perm], p1[perm], p2[perm])):
        k = fem.system_matrix(m.xy, m.tri, m.dirichlet)
        mo = gnn.neighbour_mean_operator(gnn.triangle_adjacency(m.n_nodes, m.tri))
        out.append(gnn.guess(th, k, m.dirichlet, bb, q1, q2, mo, emulate=False))
    np.testing.assert_allclose(out[1], out[0][perm], rtol=1e-10, atol=1e-12 * np.abs(out[0]).max())
