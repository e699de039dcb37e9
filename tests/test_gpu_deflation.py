"""Subdomain-deflated solves on the GPU (through the C ABI) against the deflation oracle.

fp64: the device's single-reduction deflated CG is the oracle's deflated PCG in
exact arithmetic, so the iteration counts agree to within two (rounding order)
and the solution meets the direct solve at the tolerance's level.  Mixed
precision: the refined solution meets the direct solve to 1e-6.
"""
import numpy as np
import pytest

import cgp_inputs as ci
from oracle import deflation as dfl
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


class Case:
    def __init__(self, ctx, nx, ny, seed):
        self.m = ci.jittered_rect(nx, ny, seed)
        self.a = fem.system_matrix(self.m.xy, self.m.tri, self.m.dirichlet)
        self.h = ctx.mesh_upload(self.m.xy, self.m.tri, self.m.dirichlet, 0)
        u, v = ci.stream_velocity(self.m.xy, ci.fourier_modes(seed))
        self.b = fem.source(self.m.xy, self.m.tri, self.m.dirichlet, u, v, fem.CURL, 1.0)
        self.xs = solve.direct(self.a, self.b)


@pytest.fixture(scope="module")
def cases(ctx):
    cs = {"65x33": Case(ctx, 65, 33, 21), "129x65": Case(ctx, 129, 65, 22), "257x129": Case(ctx, 257, 129, 23)}
    yield cs
    for c in cs.values():
        ctx.mesh_free(c.h)


def _solve(ctx, cgp, c, precision=0, degree=8, tol=1e-10, guess=None, x0=None, **kw):
    n = c.m.n_nodes
    phi = dt(x0) if x0 is not None else torch.zeros(n, dtype=torch.float64, device=DEV)
    if guess is None:
        guess = cgp.CGP_GUESS_GIVEN if x0 is not None else cgp.CGP_GUESS_ZERO
    stats = cgp.stats_buffer(1)
    ctx.poisson_solve([c.h], [dt(c.b)], [phi], stats, precision=precision, guess=guess, tol=tol,
                      precond_degree=degree, deflation=1, **kw)
    return phi.cpu().numpy(), ctx.solve_check(1, stats)[0]


def rel(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


@pytest.mark.parametrize("name", ["65x33", "129x65", "257x129"])
@pytest.mark.parametrize("degree", [1, 4, 8])
def test_fp64_deflated_solve_matches_oracle(ctx, cgp, cases, name, degree):
    c = cases[name]
    x, st = _solve(ctx, cgp, c, degree=degree, tol=1e-10)
    assert st["status"] == "ok" and st["rel_res"] <= 1e-10
    assert rel(x, c.xs) <= 1e-8
    parts = dfl.aggregates(c.a, c.m.xy, degree)
    z, e = dfl.deflation_space(c.a, c.m.dirichlet, parts)
    xo, info = dfl.dpcg(c.a, c.b, z, e, tol=1e-10, degree=degree)
    assert info["status"] == "ok"
    assert abs(st["iters"] - info["iters"]) <= 2, (st, info)
    assert rel(x, xo) <= 1e-8


@pytest.mark.parametrize("name", ["129x65", "257x129"])
@pytest.mark.parametrize("degree", [4, 8])
def test_mixed_deflated_solve_meets_the_direct_solve(ctx, cgp, cases, name, degree):
    c = cases[name]
    for delta in (0.0, 1e-3):
        x, st = _solve(ctx, cgp, c, precision=cgp.CGP_FP32_IR, degree=degree, tol=1e-8, refine_delta=delta)
        assert st["status"] == "ok" and st["rel_res"] <= 1e-8
        assert rel(x, c.xs) <= 1e-6
    x64, st64 = _solve(ctx, cgp, c, degree=degree, tol=1e-8)
    assert st["iters"] <= 1.5 * st64["iters"] + 10, (st, st64)


def test_deflation_cuts_iterations(ctx, cgp, cases):
    c = cases["257x129"]
    _, sd = _solve(ctx, cgp, c, degree=8, tol=1e-8)
    phi = torch.zeros(c.m.n_nodes, dtype=torch.float64, device=DEV)
    stats = cgp.stats_buffer(1)
    ctx.poisson_solve([c.h], [dt(c.b)], [phi], stats, tol=1e-8, precond_degree=8)
    sp = ctx.solve_check(1, stats)[0]
    assert sd["iters"] <= 0.8 * sp["iters"], (sd, sp)


def test_guess_modes_and_repeatability(ctx, cgp, cases):
    c = cases["129x65"]
    rng = np.random.default_rng(5)
    p1 = c.xs * (1 + 1e-3 * rng.standard_normal(c.m.n_nodes)) * (c.m.dirichlet == 0)
    p2 = c.xs * (1 + 2e-3 * rng.standard_normal(c.m.n_nodes)) * (c.m.dirichlet == 0)
    for guess in (cgp.CGP_GUESS_ZERO, cgp.CGP_GUESS_GIVEN, cgp.CGP_GUESS_EXTRAP):
        outs = []
        for _ in range(2):
            phi = dt(p1) if guess == cgp.CGP_GUESS_GIVEN else torch.zeros(c.m.n_nodes, dtype=torch.float64,
                                                                            device=DEV)
            stats = cgp.stats_buffer(1)
            ctx.poisson_solve([c.h], [dt(c.b)], [phi], stats, prev1=[dt(p1)], prev2=[dt(p2)], guess=guess,
                              precision=cgp.CGP_FP32_IR, tol=1e-8, precond_degree=8, deflation=1)
            st = ctx.solve_check(1, stats)[0]
            assert st["status"] == "ok" and st["rel_res"] <= 1e-8
            outs.append(phi.cpu().numpy())
        np.testing.assert_array_equal(outs[0], outs[1])        # deterministic
        assert rel(outs[0], c.xs) <= 1e-6
        start = {cgp.CGP_GUESS_ZERO: np.zeros_like(p1), cgp.CGP_GUESS_GIVEN: p1,
                 cgp.CGP_GUESS_EXTRAP: (2 * p1 - p2) * (c.m.dirichlet == 0)}[guess]
        assert st["rel_res_guess"] == pytest.approx(solve.relative_residual(c.a, c.b, start), rel=1e-6)


def test_batch_of_uneven_meshes_equals_single_solves(ctx, cgp, cases):
    cs = [cases["65x33"], cases["257x129"], cases["129x65"]]
    single = [_solve(ctx, cgp, c, precision=cgp.CGP_FP32_IR, tol=1e-8)[0] for c in cs]
    phis = [torch.zeros(c.m.n_nodes, dtype=torch.float64, device=DEV) for c in cs]
    stats = cgp.stats_buffer(len(cs))
    ctx.poisson_solve([c.h for c in cs], [dt(c.b) for c in cs], phis, stats, precision=cgp.CGP_FP32_IR,
                      guess=cgp.CGP_GUESS_ZERO, tol=1e-8, precond_degree=8, deflation=1)
    sts = ctx.solve_check(len(cs), stats)
    for c, phi, st, x1 in zip(cs, phis, sts, single):
        assert st["status"] == "ok" and st["rel_res"] <= 1e-8
        np.testing.assert_array_equal(phi.cpu().numpy(), x1)   # instances are independent


def test_zero_rhs_and_plain_solve_after_deflation(ctx, cgp, cases):
    c = cases["65x33"]
    phi = dt(np.ones(c.m.n_nodes))
    stats = cgp.stats_buffer(1)
    ctx.poisson_solve([c.h], [torch.zeros(c.m.n_nodes, dtype=torch.float64, device=DEV)], [phi], stats,
                      tol=1e-8, precond_degree=8, deflation=1)
    st = ctx.solve_check(1, stats)[0]
    assert st["status"] == "ok"
    assert not phi.cpu().numpy().any()
    # the tile records were extended in place: a solve without deflation on the same mesh still works
    for engine in (cgp.CGP_ENGINE_AUTO, cgp.CGP_ENGINE_STAGED):
        phi = torch.zeros(c.m.n_nodes, dtype=torch.float64, device=DEV)
        ctx.poisson_solve([c.h], [dt(c.b)], [phi], stats, tol=1e-10, precond_degree=8, engine=engine)
        st = ctx.solve_check(1, stats)[0]
        assert st["status"] == "ok" and rel(phi.cpu().numpy(), c.xs) <= 1e-8


def test_deflation_needs_the_tiled_engine(ctx, cgp, cases):
    c = cases["65x33"]
    phi = torch.zeros(c.m.n_nodes, dtype=torch.float64, device=DEV)
    stats = cgp.stats_buffer(1)
    for engine in (cgp.CGP_ENGINE_PERSISTENT, cgp.CGP_ENGINE_STAGED_ROWS):
        with pytest.raises(cgp.CGPError) as ei:
            ctx.poisson_solve([c.h], [dt(c.b)], [phi], stats, tol=1e-8, precond_degree=1, deflation=1,
                              engine=engine)
        assert ei.value.code == cgp.CGP_E_UNSUPPORTED
    with pytest.raises(cgp.CGPError) as ei:
        ctx.poisson_solve([c.h], [dt(c.b)], [phi], stats, tol=1e-8, deflation=2)
    assert ei.value.code == cgp.CGP_E_INVALID


def test_more_aggregates_than_the_coarse_step_holds(ctx, cgp):
    """A 1449x725 mesh (1050525 rows) takes more than 1024 tiles at degree 6, so more than the
    2048 aggregates the coarse step holds: a deflated solve is refused with CGP_E_UNSUPPORTED and
    leaves the mesh usable; the undeflated fp32-refined solve meets the tolerance on the true
    residual, checked on the host with the oracle's matrix."""
    m = ci.jittered_rect(1449, 725, 31)
    a = fem.system_matrix(m.xy, m.tri, m.dirichlet)
    u, v = ci.stream_velocity(m.xy, ci.fourier_modes(31))
    b = fem.source(m.xy, m.tri, m.dirichlet, u, v, fem.CURL, 1.0)
    h = ctx.mesh_upload(m.xy, m.tri, m.dirichlet, 0)
    try:
        phi = torch.zeros(m.n_nodes, dtype=torch.float64, device=DEV)
        stats = cgp.stats_buffer(1)
        kw = dict(precision=cgp.CGP_FP32_IR, guess=cgp.CGP_GUESS_ZERO, tol=1e-8, precond_degree=6)
        with pytest.raises(cgp.CGPError) as ei:
            ctx.poisson_solve([h], [dt(b)], [phi], stats, deflation=1, **kw)
        assert ei.value.code == cgp.CGP_E_UNSUPPORTED
        ctx.poisson_solve([h], [dt(b)], [phi], stats, deflation=0, **kw)
        st = ctx.solve_check(1, stats)[0]
        assert st["status"] == "ok" and st["rel_res"] <= 1e-8
        x = phi.cpu().numpy()
        assert np.linalg.norm(b - a @ x) <= 1.01e-8 * np.linalg.norm(b)
    finally:
        ctx.mesh_free(h)
