"""Parity at the benchmark's sizes.

* 513 x 257 coarse mesh (131841 nodes, the single-sequence size): the learned guess of the
  device (its smoothing runs 256 tiles of two own rows on some threads, with XCD-contiguous
  row groups, a path the small meshes do not reach) against the network oracle, and a
  learned fp32-refined, Chebyshev, deflated solve against phi* = K^-1 b (SuperLU).
* 1025 x 513 coarse mesh refined twice (525825 coarse, 8394753 fine nodes; the two-level
  batch workload): the restricted source against the oracle's, plain fp64 Jacobi-PCG and the
  learned fp32-refined Chebyshev deflated solve of one instance against phi* (1e-8 and 1e-6),
  and a batch of eight such instances by the true fp64 residual of each, formed on the host
  with the oracle's matrix.
"""
import numpy as np
import pytest
import scipy.sparse.linalg as spla

import cgp_inputs as ci
from oracle import fem, gnn

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
DEV = "cuda:0"


@pytest.fixture(scope="module")
def cgp():
    import paper_2003_00082_amd as lib
    lib.load()
    return lib


@pytest.fixture(scope="module")
def ctx(cgp):
    c = cgp.Context(0)
    yield c
    c.close()


def dt(a):
    return torch.tensor(np.ascontiguousarray(a), dtype=torch.float64, device=DEV)


def rel(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def random_theta(seed):
    rng = np.random.default_rng(seed)
    p = {}
    for name, shape in gnn.param_shapes():
        fan = shape[0] if len(shape) == 2 else 64
        p[name] = rng.standard_normal(shape) * (np.sqrt(2.0 / fan) if len(shape) == 2 else 0.1)
    p["W0"][8:] = 0.0
    p["wd"] = rng.standard_normal(64) * 0.2
    return gnn.pack(p).astype(np.float32)


def test_learned_guess_and_solve_at_513x257(ctx, cgp):
    m = ci.jittered_rect(513, 257, 2000)
    a = fem.system_matrix(m.xy, m.tri, m.dirichlet)
    lu = spla.splu(a.tocsc())
    sq = ci.FourierSequence(m.xy, ci.fourier_modes(2500), ci.fourier_modes(2700))
    b = [fem.source(m.xy, m.tri, m.dirichlet, *sq.at(n)[:2], fem.CURL, 1.0) for n in range(3)]
    x = [lu.solve(bb) for bb in b]
    h = ctx.mesh_upload(m.xy, m.tri, m.dirichlet, 0)
    md = ctx.model_create()
    try:
        th = random_theta(7)
        ctx.model_set_params(md, th)
        g = torch.full((m.n_nodes,), np.nan, dtype=torch.float64, device=DEV)
        ctx.model_predict(md, h, dt(b[2]), dt(x[1]), dt(x[0]), g)
        ctx.sync()
        got = g.cpu().numpy()
        mo = gnn.neighbour_mean_operator(gnn.triangle_adjacency(m.n_nodes, m.tri))
        feats, e, sd = gnn.features(a, m.dirichlet, b[2], x[1], x[0])
        y_ref, _ = gnn.forward(th.astype(np.float64), feats, mo, emulate=True)
        free = m.dirichlet == 0
        np.testing.assert_array_equal(got[~free], 0.0)
        # the network's part of the (affine) smoothed guess, as in the small-mesh test
        part_ref = gnn.smooth(a, np.zeros_like(b[2]), sd * y_ref * free)
        part_got = got - gnn.smooth(a, b[2], e * free)
        assert rel(part_got, part_ref) <= 1e-4
        # the learned solve (fp32 with fp64 refinement, Chebyshev degree 6, deflated)
        phi = torch.zeros(m.n_nodes, dtype=torch.float64, device=DEV)
        st = cgp.stats_buffer(1)
        ctx.poisson_solve([h], [dt(b[2])], [phi], st, prev1=[dt(x[1])], prev2=[dt(x[0])],
                          precision=cgp.CGP_FP32_IR, guess=cgp.CGP_GUESS_LEARNED, model=md, tol=1e-8,
                          precond_degree=6, deflation=1, refine_delta=1e-3)
        s = ctx.solve_check(1, st)[0]
        print("513x257 learned solve", s, flush=True)
        assert s["status"] == "ok" and s["rel_res"] <= 1e-8
        assert rel(phi.cpu().numpy(), x[2]) <= 1e-6
    finally:
        ctx.model_free(md)
        ctx.mesh_free(h)


def test_two_level_batch_at_1025x513(ctx, cgp):
    M = 8
    meshes = [ci.jittered_rect(1025, 513, 5000 + i) for i in range(M)]
    H = [ctx.mesh_upload(m.xy, m.tri, m.dirichlet, 2) for m in meshes]
    md = ctx.model_create(seed=11)
    try:
        nc = meshes[0].n_nodes
        assert ctx.mesh_info(H[0], 2)["n_nodes"] == 8394753
        seqs = [ci.DeviceFourierSequence(torch.from_numpy(ctx.mesh_download(h, 2)[0]).to(DEV),
                                         ci.fourier_modes(5500 + i), ci.fourier_modes(5700 + i))
                for i, h in enumerate(H)]
        b = [[torch.empty(nc, dtype=torch.float64, device=DEV) for _ in range(M)] for _ in range(3)]
        uv0 = []                     # instance 0's velocity at the coarse nodes (the oracle's input)
        for n in range(3):
            for i in range(M):
                u, v, _, _ = seqs[i].at(n - 2)
                ctx.restrict(H[i], u, v, cgp.CGP_SRC_CURL, 1.0, b[n][i])
                if i == 0:
                    uv0.append((u[:nc].cpu().numpy(), v[:nc].cpu().numpy()))
        ctx.sync()
        m0 = meshes[0]
        a0 = fem.system_matrix(m0.xy, m0.tri, m0.dirichlet)
        b_ref = [fem.source(m0.xy, m0.tri, m0.dirichlet, u, v, fem.CURL, 1.0) for u, v in uv0]
        got_b = b[2][0].cpu().numpy()
        assert np.abs(got_b - b_ref[2]).max() <= 1e-12 * np.abs(b_ref[2]).max()
        lu = spla.splu(a0.tocsc())
        xs = [lu.solve(bb) for bb in b_ref]
        st = cgp.stats_buffer(1)
        # plain fp64 Jacobi-PCG of instance 0 (form A's arithmetic) against phi*
        phi = torch.zeros(nc, dtype=torch.float64, device=DEV)
        ctx.poisson_solve([H[0]], [b[2][0]], [phi], st, precision=cgp.CGP_FP64, guess=cgp.CGP_GUESS_ZERO,
                          tol=1e-10)
        s = ctx.solve_check(1, st)[0]
        print("1025x513 fp64 Jacobi", s, flush=True)
        assert s["status"] == "ok" and s["rel_res"] <= 1e-10
        assert rel(phi.cpu().numpy(), xs[2]) <= 1e-8
        # the learned fp32-refined Chebyshev deflated solve of instance 0 (form B) against phi*
        ctx.model_set_params(md, random_theta(3))
        phi = torch.zeros(nc, dtype=torch.float64, device=DEV)
        ctx.poisson_solve([H[0]], [b[2][0]], [phi], st, prev1=[dt(xs[1])], prev2=[dt(xs[0])],
                          precision=cgp.CGP_FP32_IR, guess=cgp.CGP_GUESS_LEARNED, model=md, tol=1e-8,
                          precond_degree=6, deflation=1, refine_delta=1e-3)
        s = ctx.solve_check(1, st)[0]
        print("1025x513 learned", s, flush=True)
        assert s["status"] == "ok" and s["rel_res"] <= 1e-8
        assert rel(phi.cpu().numpy(), xs[2]) <= 1e-6
        # the batch of eight from the extrapolation of the two previous sources' solutions
        # (previous solutions from the batched solve itself)
        phis = [[torch.zeros(nc, dtype=torch.float64, device=DEV) for _ in range(M)] for _ in range(3)]
        stb = cgp.stats_buffer(M)
        for n in range(3):
            kw = dict(precision=cgp.CGP_FP32_IR, tol=1e-8, precond_degree=6, deflation=1, refine_delta=1e-3)
            if n < 2:
                ctx.poisson_solve(H, b[n], phis[n], stb, guess=cgp.CGP_GUESS_ZERO, **kw)
            else:
                ctx.poisson_solve(H, b[n], phis[n], stb, prev1=phis[1], prev2=phis[0], guess=cgp.CGP_GUESS_LEARNED,
                                  model=md, **kw)
            res = ctx.solve_check(M, stb)
            assert all(r["status"] == "ok" and r["rel_res"] <= 1e-8 for r in res), res
        for i in range(M):
            mi = meshes[i]
            ai = a0 if i == 0 else fem.system_matrix(mi.xy, mi.tri, mi.dirichlet)
            bi, xi = b[2][i].cpu().numpy(), phis[2][i].cpu().numpy()
            r = np.linalg.norm(bi - ai @ xi) / np.linalg.norm(bi)
            assert r <= 1e-8, (i, r)
        assert rel(phis[2][0].cpu().numpy(), xs[2]) <= 1e-6
    finally:
        ctx.model_free(md)
        for h in H:
            ctx.mesh_free(h)
