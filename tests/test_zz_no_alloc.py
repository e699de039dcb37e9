"""The no-allocation solve (cgp_poisson_solve_noalloc) against cgp_poisson_solve.

Both run the same stage kernels; the no-allocation call takes its buffers from the
library's fixed device array instead of allocating.  Each case solves a larger mesh,
then a smaller one (two calls in a row on the shared array), and checks the result
against the existing entry point (same iterations, relative difference <= 1e-12) and
against the exact solution phi* = K^-1 b (fp64 <= 1e-8, fp32 with fp64 refinement
<= 1e-6, the solve parity bars).  Requests the call cannot serve are refused before
anything is enqueued.
"""
import numpy as np
import pytest

import cgp_inputs as ci
from oracle import fem, solve

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


def _problem(nx, ny, seed):
    m = ci.jittered_rect(nx, ny, seed)
    a = fem.system_matrix(m.xy, m.tri, m.dirichlet)
    rng = np.random.default_rng(seed)
    free = m.dirichlet == 0
    # a smooth source (the Fourier flow's curl) plus a little noise, zero on Dirichlet rows
    u, v = ci.stream_velocity(m.xy, ci.fourier_modes(seed + 1), 0.0)
    b = fem.source(m.xy, m.tri, m.dirichlet, u, v, fem.CURL, 1.0) + 1e-3 * rng.standard_normal(m.n_nodes) * free
    return m, a, b, solve.direct(a, b)


CASES = {
    # precision, guess, degree, deflation, engine, tol, bar
    "fp64_jacobi_rows": (0, 0, 0, 0, 3, 1e-10, 1e-8),
    "fp64_chebyshev4_tiled": (0, 1, 4, 0, 1, 1e-10, 1e-8),
    "fp32ir_chebyshev6_deflated": (1, 2, 6, 1, 1, 1e-8, 1e-6),
}


@pytest.mark.parametrize("case", list(CASES))
def test_noalloc_matches_poisson_solve(ctx, cgp, case):
    prec, guess, deg, defl, engine, tol, bar = CASES[case]
    kw = dict(precision=prec, guess=guess, precond_degree=deg, deflation=defl, engine=engine, tol=tol)
    for nx, ny, seed in ((129, 65, 41), (65, 33, 42)):     # the second call is the smaller one
        m, a, b, exact = _problem(nx, ny, seed)
        h = ctx.mesh_upload(m.xy, m.tri, m.dirichlet, 0)
        try:
            bd = dt(b)
            start = 0.9 * exact
            p1, p2 = dt(0.8 * exact), dt(0.7 * exact)
            extra = dict(prev1=[p1], prev2=[p2]) if guess == cgp.CGP_GUESS_EXTRAP else {}
            x_ref = dt(start)
            st_ref = cgp.stats_buffer(1)
            ctx.poisson_solve([h], [bd], [x_ref], st_ref, **kw, **extra)      # also builds the tiled plan
            ref = ctx.solve_check(1, st_ref)[0]
            x_na = dt(start)
            st_na = cgp.stats_buffer(1)
            na_extra = dict(prev1=p1, prev2=p2) if guess == cgp.CGP_GUESS_EXTRAP else {}
            ctx.poisson_solve_noalloc(h, bd, x_na, st_na, **kw, **na_extra)
            got = ctx.solve_check(1, st_na)[0]
            print(case, nx, ny, ref, got, flush=True)
            assert ref["status"] == "ok" and got["status"] == "ok"
            assert got["iters"] == ref["iters"] and got["refinements"] == ref["refinements"]
            assert got["rel_res"] <= tol
            xr, xn = x_ref.cpu().numpy(), x_na.cpu().numpy()
            assert np.linalg.norm(xn - xr) <= 1e-12 * np.linalg.norm(xr)
            assert np.linalg.norm(xn - exact) <= bar * np.linalg.norm(exact)
        finally:
            ctx.mesh_free(h)


def test_noalloc_refuses_what_it_cannot_serve(ctx, cgp):
    m, a, b, exact = _problem(33, 17, 7)
    h = ctx.mesh_upload(m.xy, m.tri, m.dirichlet, 0)
    try:
        bd = dt(b)
        x = torch.full((m.n_nodes,), 7.0, dtype=torch.float64, device=DEV)
        st = cgp.stats_buffer(1)
        # a tiled plan of a degree no solve on this mesh has built
        with pytest.raises(cgp.CGPError) as e:
            ctx.poisson_solve_noalloc(h, bd, x, st, precond_degree=3)
        assert e.value.code == cgp.CGP_E_INVALID
        # the learned guess and the persistent engine are not served
        with pytest.raises(cgp.CGPError) as e:
            ctx.poisson_solve_noalloc(h, bd, x, st, guess=cgp.CGP_GUESS_LEARNED, prev1=x, prev2=x)
        assert e.value.code == cgp.CGP_E_UNSUPPORTED
        with pytest.raises(cgp.CGPError) as e:
            ctx.poisson_solve_noalloc(h, bd, x, st, engine=cgp.CGP_ENGINE_PERSISTENT)
        assert e.value.code == cgp.CGP_E_UNSUPPORTED
        ctx.sync()
        assert bool(torch.all(x == 7.0))          # nothing was enqueued
    finally:
        ctx.mesh_free(h)
    # a mesh beyond the array's size
    big = ci.jittered_rect(1201, 601, 9)
    hb = ctx.mesh_upload(big.xy, big.tri, big.dirichlet, 0)
    try:
        bb = torch.zeros(big.n_nodes, dtype=torch.float64, device=DEV)
        xb = torch.full((big.n_nodes,), 7.0, dtype=torch.float64, device=DEV)
        with pytest.raises(cgp.CGPError) as e:
            ctx.poisson_solve_noalloc(hb, bb, xb, cgp.stats_buffer(1), engine=cgp.CGP_ENGINE_STAGED_ROWS)
        assert e.value.code == cgp.CGP_E_INVALID and "scratch" in str(e.value)
        ctx.sync()
        assert bool(torch.all(xb == 7.0))
    finally:
        ctx.mesh_free(hb)
