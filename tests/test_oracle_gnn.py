"""Pins of the learned-guess network oracle (CPU only).

The network is an extension of the paper's method (a learned initial guess for
the coarse Poisson solves of Section 2.2), so nothing in the paper fixes its
values; the pins below fix what mathematics does: bfloat16 rounding against
hand-worked cases and torch's own conversion, the analytic backward pass
against central differences, the loss against the energy norm of the guess
error written in the solution's units, the zero-decoder case that reduces to
the extrapolation 2 phi^{n-1} - phi^{n-2}, homogeneity of degree one in the
inputs, and equivariance under a renumbering of the nodes.  A hand-worked
forward pass on a two-triangle mesh (encoder, neighbour means without the node
itself, the [h, m] order, relu(a) + h, biases, decoder) and hand-worked
features (r_e = b - K e, K d, the RMS scales, the Dirichlet zero) fix the
values themselves; copies of the oracle with a planted mistake miss them.
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


# ---------------------------------------------------------------- hand-worked forward pass
#
# A unit square cut into the triangles (0, 1, 2) and (0, 2, 3): node 0 ~ {1, 2, 3},
# node 1 ~ {0, 2}, node 2 ~ {0, 1, 3}, node 3 ~ {0, 2}.  Only hidden units 0 and 1 carry
# weights; every weight is a small power-of-two multiple (exact in bfloat16), so the
# emulated and the plain fp64 network give the same values, worked out by hand below.

_SQ_TRI = np.array([[0, 1, 2], [0, 2, 3]])
# features [b, p1, p2, r_e, K d, d, dirichlet, 1] of the four nodes (only b and p1 are weighted)
_SQ_X = np.array([[1.0, 0.5, 0, 0, 0, 0, 0, 1],
                  [-1.0, -1.0, 0, 0, 0, 0, 0, 1],
                  [0.5, 1.0, 0, 0, 0, 0, 0, 1],
                  [2.0, 0.0, 0, 0, 0, 0, 1, 1]])


def _hand_params():
    p = {name: np.zeros(shape) for name, shape in gnn.param_shapes()}
    H = gnn.HIDDEN
    # encoder: u0 = relu(b + 1/2), u1 = relu(-p1 + 1/4)
    p["W0"][0, 0], p["c0"][0] = 1.0, 0.5
    p["W0"][1, 1], p["c0"][1] = -1.0, 0.25
    # layer 1 (rows 0..63 multiply h, rows 64..127 the neighbour mean m):
    #   a0 = 2 h0 - m1 - 1,  a1 = m0 - 2 h1
    p["W1"][0, 0], p["W1"][H + 1, 0], p["c1"][0] = 2.0, -1.0, -1.0
    p["W1"][H + 0, 1], p["W1"][1, 1] = 1.0, -2.0
    # layer 2: a0 = m0 - 2,  a1 = h1 - h0 + 1/2
    p["W2"][H + 0, 0], p["c2"][0] = 1.0, -2.0
    p["W2"][1, 1], p["W2"][0, 1], p["c2"][1] = 1.0, -1.0, 0.5
    # layer 3: a0 = m1 - h0 + 1,  a1 = -1 (unit 1 passes through the residual)
    p["W3"][H + 1, 0], p["W3"][0, 0], p["c3"][0] = 1.0, -1.0, 1.0
    p["c3"][1] = -1.0
    # decoder: y = h0 - 2 h1 + 1/8
    p["wd"][0], p["wd"][1], p["cd"][0] = 1.0, -2.0, 0.125
    return gnn.pack(p)


# By hand (node order 0, 1, 2, 3):
#   encoder   h0 = relu(b + 1/2)   = [3/2, 0, 1, 5/2]
#             h1 = relu(1/4 - p1)  = [0, 5/4, 0, 1/4]
#   layer 1   m0 = [(0+1+5/2)/3, (3/2+1)/2, (3/2+0+5/2)/3, (3/2+1)/2] = [7/6, 5/4, 4/3, 5/4]
#             m1 = [(5/4+0+1/4)/3, 0, (0+5/4+1/4)/3, 0]               = [1/2, 0, 1/2, 0]
#             a0 = 2 h0 - m1 - 1 = [3/2, -1, 1/2, 4]   -> h0 = relu(a0) + h0 = [3, 0, 3/2, 13/2]
#             a1 = m0 - 2 h1     = [7/6, -5/4, 4/3, 3/4] -> h1 = [7/6, 5/4, 4/3, 1]
#             (node 1, unit 1: relu(a) + h = 5/4, while relu(a + h) would be 0)
#   layer 2   m0 = [(0+3/2+13/2)/3, (3+3/2)/2, (3+0+13/2)/3, (3+3/2)/2] = [8/3, 9/4, 19/6, 9/4]
#             a0 = m0 - 2 = [2/3, 1/4, 7/6, 1/4]   -> h0 = [11/3, 1/4, 8/3, 27/4]
#             a1 = h1 - h0 + 1/2 = [-4/3, 7/4, 1/3, -5] -> h1 = [7/6, 3, 5/3, 1]
#   layer 3   m1 = [(3+5/3+1)/3, (7/6+5/3)/2, (7/6+3+1)/3, (7/6+5/3)/2] = [17/9, 17/12, 31/18, 17/12]
#             a0 = m1 - h0 + 1 = [-7/9, 13/6, 1/18, -13/3] -> h0 = [11/3, 29/12, 49/18, 27/4]
#             h1 unchanged = [7/6, 3, 5/3, 1]
#   decoder   y = h0 - 2 h1 + 1/8 = [35/24, -83/24, -35/72, 39/8]
_SQ_Y = np.array([35 / 24, -83 / 24, -35 / 72, 39 / 8])
_SQ_H3 = np.array([[11 / 3, 7 / 6], [29 / 12, 3.0], [49 / 18, 5 / 3], [27 / 4, 1.0]])


def _square_mean_op():
    return gnn.neighbour_mean_operator(gnn.triangle_adjacency(4, _SQ_TRI))


def test_forward_hand_worked_square():
    mo = _square_mean_op()
    th = _hand_params()
    for emulate in (False, True):
        y, cache = gnn.forward(th, _SQ_X, mo, emulate=emulate)
        np.testing.assert_allclose(y, _SQ_Y, rtol=0, atol=1e-14)
        np.testing.assert_allclose(cache["h"][-1][:, :2], _SQ_H3, rtol=0, atol=1e-14)
        np.testing.assert_array_equal(cache["h"][-1][:, 2:], 0.0)


# features of the same square with a hand-written stiffness (right isosceles triangles:
# K = [[1, -1/2, 0, -1/2], [-1/2, 1, -1/2, 0], [0, -1/2, 1, -1/2], [-1/2, 0, -1/2, 1]]),
# node 3 Dirichlet, b = [1, 0, -1, 0], p1 = [1, 2, 0, 1], p2 = [0, 1, 1, 1]:
#   e = 2 p1 - p2 = [2, 3, -1, 1],  d = p1 - p2 = [1, 1, -1, 0]
#   K e = [0, 5/2, -3, 1/2]  -> r_e = b - K e = [1, -5/2, 2, -1/2]
#   K d = [1/2, 1, -3/2, 0]
#   s_b = sqrt(2/4), s_p = rms(p1) = sqrt(6/4), s_r = rms(r_e) = sqrt(23/8), s_d = sqrt(3/4)
def test_features_hand_worked_square():
    import scipy.sparse as sp
    k = sp.csr_matrix(np.array([[1, -0.5, 0, -0.5], [-0.5, 1, -0.5, 0], [0, -0.5, 1, -0.5],
                                [-0.5, 0, -0.5, 1]]))
    dirichlet = np.array([0, 0, 0, 1], dtype=np.uint8)
    b, p1, p2 = np.array([1.0, 0, -1, 0]), np.array([1.0, 2, 0, 1]), np.array([0.0, 1, 1, 1])
    x, e, sd = gnn.features(k, dirichlet, b, p1, p2)
    sb, sp_, sr = np.sqrt(0.5), np.sqrt(1.5), np.sqrt(23 / 8)
    want = np.array([
        [1 / sb, 1 / sp_, 0 / sp_, 1 / sr, 0.5 / sr, 1 / np.sqrt(0.75), 0, 1],
        [0 / sb, 2 / sp_, 1 / sp_, -2.5 / sr, 1 / sr, 1 / np.sqrt(0.75), 0, 1],
        [-1 / sb, 0 / sp_, 1 / sp_, 2 / sr, -1.5 / sr, -1 / np.sqrt(0.75), 0, 1],
        [0 / sb, 1 / sp_, 1 / sp_, -0.5 / sr, 0 / sr, 0 / np.sqrt(0.75), 1, 1]])
    np.testing.assert_allclose(x, want, rtol=1e-15, atol=1e-15)
    np.testing.assert_array_equal(e, [2, 3, -1, 1])
    assert sd == pytest.approx(np.sqrt(0.75), rel=1e-15)
    # the guess before smoothing: e + s_d y on free nodes, 0 on the Dirichlet node; with only
    # the decoder bias set, y = c_d at every node
    p = {name: np.zeros(shape) for name, shape in gnn.param_shapes()}
    p["cd"][0] = 2.0
    mo = _square_mean_op()
    g = gnn.guess(gnn.pack(p), k, dirichlet, b, p1, p2, mo, sweeps=0)
    np.testing.assert_allclose(g, [2 + 2 * np.sqrt(0.75), 3 + 2 * np.sqrt(0.75), -1 + 2 * np.sqrt(0.75), 0.0],
                               rtol=1e-15, atol=1e-15)


def _mutant_forward(kind):
    """The oracle's forward pass with one planted mistake (for the pins above to catch)."""
    def fwd(theta, x, mean_op, emulate=True):
        p = gnn.unpack(theta)
        h = np.maximum(x @ p["W0"][:gnn.F_IN] + (0.0 if kind == "nobias" else p["c0"]), 0.0)
        for l in range(1, gnn.LAYERS + 1):
            m = mean_op @ h
            z = np.concatenate([m, h] if kind == "swap" else [h, m], axis=1)
            a = z @ p[f"W{l}"] + (0.0 if kind == "nobias" else p[f"c{l}"])
            h = np.maximum(a + h, 0.0) if kind == "relu_sum" else np.maximum(a, 0.0) + h
        return h @ p["wd"] + p["cd"][0], None
    return fwd


@pytest.mark.parametrize("kind", ["relu_sum", "swap", "nobias"])
def test_planted_forward_mistakes_fail_the_hand_pin(kind):
    y, _ = _mutant_forward(kind)(_hand_params(), _SQ_X, _square_mean_op())
    assert np.abs(y - _SQ_Y).max() > 1e-3
    # and the unmutated copy reproduces the oracle (so the mutant differs by its mistake only)
    y0, _ = _mutant_forward("none")(_hand_params(), _SQ_X, _square_mean_op())
    np.testing.assert_allclose(y0, gnn.forward(_hand_params(), _SQ_X, _square_mean_op(), emulate=False)[0],
                               rtol=0, atol=1e-14)


def test_planted_feature_mistake_fails_the_hand_pin():
    """The oracle's feature map with r_e = b + K e planted in place of b - K e misses the
    hand-worked features above."""
    import scipy.sparse as sp
    k = sp.csr_matrix(np.array([[1, -0.5, 0, -0.5], [-0.5, 1, -0.5, 0], [0, -0.5, 1, -0.5],
                                [-0.5, 0, -0.5, 1]]))
    dirichlet = np.array([0, 0, 0, 1], dtype=np.uint8)
    b, p1, p2 = np.array([1.0, 0, -1, 0]), np.array([1.0, 2, 0, 1]), np.array([0.0, 1, 1, 1])

    class Planted:
        def __matmul__(self, v):      # b - (K @ e) becomes b - (-K e) = b + K e for the first product
            Planted.calls += 1
            return -(k @ v) if Planted.calls == 1 else k @ v
    Planted.calls = 0
    x_bad, _, _ = gnn.features(Planted(), dirichlet, b, p1, p2)
    x_ok, _, _ = gnn.features(k, dirichlet, b, p1, p2)
    want_re = np.array([1, -2.5, 2, -0.5]) / np.sqrt(23 / 8)
    np.testing.assert_allclose(x_ok[:, 3], want_re, rtol=1e-15)
    assert np.abs(x_bad[:, 3] - want_re).max() > 0.1
