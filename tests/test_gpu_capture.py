"""Staged solves recorded in HIP graphs (a fixed stage budget per recorded solve), and a whole
CGP step (restrict, solve, prolong, Lorentz force, restrict, solve, prolong, velocity
correction) replayed as one graph.

A recorded solve runs the same stage kernels in the same order as the uncaptured solve of the
same launch records, so every replay must equal the uncaptured result bit for bit; the launches
past the end find the solve finished and change nothing.  Each graph is replayed several times
with the program's own eager work (fills, copies, uncaptured solves on the same buffers) and
synchronisations between the replays.
"""
import numpy as np
import pytest

import cgp_inputs as ci
from oracle import fem, mesh, solve

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

DEV = "cuda:0"
F64 = dict(dtype=torch.float64, device=DEV)


@pytest.fixture(scope="module")
def cgp():
    import paper_2003_00082_amd as lib
    lib.load()
    return lib


@pytest.fixture(scope="module")
def gctx(cgp):
    # capture needs a stream of its own (not the null stream)
    c = cgp.Context(0, stream=torch.cuda.Stream())
    yield c
    c.close()


def dt(a):
    return torch.tensor(np.ascontiguousarray(a), **F64)


class Inst:
    """One instance: a jittered rectangle, its hierarchy (k = 1) and the inputs of a CGP step."""

    def __init__(self, nx, ny, seed):
        self.m = ci.jittered_rect(nx, ny, seed)
        self.h = mesh.Hierarchy(self.m.xy, self.m.tri, self.m.dirichlet, 1)
        self.a = fem.system_matrix(self.m.xy, self.m.tri, self.m.dirichlet)
        nc = self.m.n_nodes
        xf = self.h.xy[1]
        u, v = ci.stream_velocity(xf, ci.fourier_modes(seed + 500), 0.0)
        du, dv = ci.potential_velocity(xf, ci.fourier_modes(seed + 700), 0.0)
        self.u, self.v, self.ut, self.vt = u, v, u + du, v + dv
        self.b0 = fem.source(self.m.xy, self.m.tri, self.m.dirichlet, u[:nc], v[:nc], fem.CURL, 1.0)
        u1, v1 = ci.stream_velocity(self.m.xy, ci.fourier_modes(seed + 600), 0.3)
        self.b1 = fem.source(self.m.xy, self.m.tri, self.m.dirichlet, u1, v1, fem.CURL, 1.0)
        self.x0 = solve.direct(self.a, self.b0)


SIZES = [(65, 33, 4101), (129, 65, 4102), (33, 17, 4103)]

FORMS = {
    # fp32 inner CG with fp64 refinement, Chebyshev degree 4, deflation, extrapolated guess
    "fp32ir_cheb4_defl": dict(precision=1, precond_degree=4, deflation=1, guess=2),
    # plain fp64 Jacobi PCG on the tiled iteration
    "fp64_jacobi_tiled": dict(precision=0, precond_degree=1, deflation=0, guess=0),
    # the learned initial guess ahead of the deflated fp32 solve
    "learned_fp32ir_cheb4_defl": dict(precision=1, precond_degree=4, deflation=1, guess=3),
}


@pytest.fixture(scope="module")
def insts():
    return [Inst(*s) for s in SIZES]


def _upload(gctx, insts):
    hs = [gctx.mesh_upload(i.m.xy, i.m.tri, i.m.dirichlet, 1) for i in insts]
    torch.cuda.synchronize()
    return hs


@pytest.mark.parametrize("form", list(FORMS))
def test_recorded_solve_replays_match_uncaptured(gctx, cgp, insts, form):
    f = FORMS[form]
    hs = _upload(gctx, insts)
    model = gctx.model_create(seed=11) if f["guess"] == cgp.CGP_GUESS_LEARNED else -1
    try:
        b = [dt(i.b0) for i in insts]
        x = [torch.zeros(i.m.n_nodes, **F64) for i in insts]
        p1 = [dt(0.9 * i.x0) for i in insts]
        p2 = [dt(0.7 * i.x0) for i in insts]
        stats = cgp.stats_buffer(len(insts))
        kw = dict(prev1=p1, prev2=p2, precision=f["precision"], guess=f["guess"], tol=1e-8, model=model,
                  engine=cgp.CGP_ENGINE_STAGED, precond_degree=f["precond_degree"], deflation=f["deflation"])

        def uncaptured(bs):
            for t, a in zip(b, bs):
                t.copy_(dt(a))
            torch.cuda.synchronize()
            gctx.poisson_solve(hs, b, x, stats, **kw)
            st = gctx.solve_check(len(insts), stats)
            assert all(s["status"] == "ok" for s in st)
            return [t.cpu().numpy().copy() for t in x], st

        ref0, st0 = uncaptured([i.b0 for i in insts])
        for i, r in zip(insts, ref0):
            assert np.linalg.norm(r - i.x0) / np.linalg.norm(i.x0) <= 1e-5
        gctx.graph_begin()
        gctx.poisson_solve(hs, b, x, stats, **kw)
        g = gctx.graph_end()
        try:
            ref1, st1 = uncaptured([i.b1 for i in insts])   # eager work on the same buffers
            for rep, (bs, ref, st_ref) in enumerate([(0, ref0, st0), (1, ref1, st1), (0, ref0, st0)]):
                for t, i in zip(b, insts):
                    t.copy_(dt(i.b0 if bs == 0 else i.b1))
                for t in x:
                    t.fill_(123.0)
                stats.fill_(0)
                torch.cuda.synchronize()
                gctx.graph_launch(g)
                gctx.sync()
                st = gctx.solve_check(len(insts), stats)
                for k in range(len(insts)):
                    np.testing.assert_array_equal(x[k].cpu().numpy(), ref[k], err_msg=f"replay {rep} instance {k}")
                    assert st[k] == st_ref[k], (rep, k)
        finally:
            gctx.graph_free(g)
    finally:
        if model >= 0:
            gctx.model_free(model)
        for h in hs:
            gctx.mesh_free(h)


def test_stage_budget_cuts_off_and_reports(gctx, cgp, insts):
    hs = _upload(gctx, insts[:2])
    try:
        b = [dt(i.b0) for i in insts[:2]]
        x = [torch.zeros(i.m.n_nodes, **F64) for i in insts[:2]]
        stats = cgp.stats_buffer(2)
        kw = dict(precision=cgp.CGP_FP32_IR, guess=cgp.CGP_GUESS_ZERO, tol=1e-8, engine=cgp.CGP_ENGINE_STAGED,
                  precond_degree=4, deflation=1)
        gctx.poisson_solve(hs, b, x, stats, **kw)
        ok = gctx.solve_check(2, stats)
        ref = [t.cpu().numpy().copy() for t in x]
        gctx.graph_begin()
        gctx.poisson_solve(hs, b, x, stats, stage_budget=3, **kw)
        g = gctx.graph_end()
        try:
            for _ in range(2):
                stats.fill_(0)
                torch.cuda.synchronize()
                gctx.graph_launch(g)
                gctx.sync()
                st = gctx.solve_check(2, stats)
                assert [s["status"] for s in st] == ["aborted", "aborted"]
                assert all(s["iters"] < ok[k]["iters"] for k, s in enumerate(st))
            # an uncaptured solve on the same launch records afterwards is unaffected
            gctx.poisson_solve(hs, b, x, stats, **kw)
            assert gctx.solve_check(2, stats) == ok
            for t, r in zip(x, ref):
                np.testing.assert_array_equal(t.cpu().numpy(), r)
        finally:
            gctx.graph_free(g)
        # no uncaptured solve of these vectors yet: nothing to size the recorded launches by
        fresh = [torch.zeros_like(t) for t in x]
        gctx.graph_begin()
        with pytest.raises(cgp.CGPError):
            gctx.poisson_solve(hs, b, fresh, stats, **kw)
        gctx.graph_free(gctx.graph_end())
        with pytest.raises(cgp.CGPError):
            gctx.poisson_solve(hs, b, x, stats, stage_budget=-1, **kw)
    finally:
        for h in hs:
            gctx.mesh_free(h)


def test_whole_cgp_step_is_one_graph(gctx, cgp, insts):
    """Steps 1-7 for a batch of instances (both solves deflated fp32 on the staged engine)."""
    hs = _upload(gctx, insts)
    M = len(insts)
    try:
        nc = [i.m.n_nodes for i in insts]
        nf = [i.h.n_nodes(1) for i in insts]
        u, v, ut, vt = ([dt(getattr(i, a)) for i in insts] for a in ("u", "v", "ut", "vt"))
        bphi, phi, bp, p = ([torch.zeros(n, **F64) for n in nc] for _ in range(4))
        phif, fx, fy, pf, un, vn = ([torch.zeros(n, **F64) for n in nf] for _ in range(6))
        st_phi, st_p = cgp.stats_buffer(M), cgp.stats_buffer(M)
        outs = phi + p + phif + fx + fy + pf + un + vn
        kw = dict(precision=cgp.CGP_FP32_IR, guess=cgp.CGP_GUESS_ZERO, tol=1e-8, engine=cgp.CGP_ENGINE_STAGED,
                  precond_degree=4, deflation=1)
        rho_dt = 1.0 / ci.DT

        def step():
            for k in range(M):
                gctx.restrict(hs[k], u[k], v[k], cgp.CGP_SRC_CURL, 1.0, bphi[k])
            gctx.poisson_solve(hs, bphi, phi, st_phi, **kw)
            for k in range(M):
                gctx.prolong(hs[k], phi[k], phif[k])
                gctx.lorentz_force(hs[k], phif[k], u[k], v[k], 0.5 + k, 1.0, fx[k], fy[k])
                gctx.restrict(hs[k], ut[k], vt[k], cgp.CGP_SRC_DIV, rho_dt, bp[k])
            gctx.poisson_solve(hs, bp, p, st_p, **kw)
            for k in range(M):
                gctx.prolong(hs[k], p[k], pf[k])
                gctx.velocity_correct(hs[k], pf[k], ut[k], vt[k], 1.0 / rho_dt, un[k], vn[k])

        step()
        gctx.sync()
        eager = [t.cpu().numpy().copy() for t in outs]
        s_phi, s_p = gctx.solve_check(M, st_phi), gctx.solve_check(M, st_p)
        assert all(s["status"] == "ok" for s in s_phi + s_p)
        for k, i in enumerate(insts):
            assert np.linalg.norm(eager[k] - i.x0) / np.linalg.norm(i.x0) <= 1e-5
        gctx.graph_begin()
        step()
        g = gctx.graph_end()
        try:
            for rep in range(3):
                for t in outs + bphi + bp:
                    t.fill_(-7.0)
                st_phi.fill_(0)
                st_p.fill_(0)
                torch.cuda.synchronize()
                gctx.graph_launch(g)
                gctx.sync()
                for t, e in zip(outs, eager):
                    np.testing.assert_array_equal(t.cpu().numpy(), e, err_msg=f"replay {rep}")
                assert gctx.solve_check(M, st_phi) == s_phi and gctx.solve_check(M, st_p) == s_p
                step()   # the same step uncaptured between replays
                gctx.sync()
        finally:
            gctx.graph_free(g)
    finally:
        for h in hs:
            gctx.mesh_free(h)
