"""Parity of the HIP library (through the C ABI) with the CPU oracle.

Index and mesh-map work is compared bit for bit; floating-point results within
the tolerances stated next to each assertion.
"""
import numpy as np
import pytest

import cgp_inputs as ci
from oracle import fem, mesh, solve

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


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


DEV = "cuda:0"


def dt(a):
    return torch.tensor(np.ascontiguousarray(a), dtype=torch.float64, device=DEV)


def meshes_for_bitexact():
    return {
        "rect_33x17": ci.jittered_rect(33, 17, 1001),
        "rect_ragged_7x4": ci.jittered_rect(7, 4, 5),
        "hole_17x11": ci.rect_with_hole(17, 11, (5, 9, 3, 7), seed=3),
        "permuted_12x9": ci.permuted(ci.jittered_rect(12, 9, 8), seed=4),
    }


@pytest.mark.parametrize("name", list(meshes_for_bitexact()))
@pytest.mark.parametrize("k", [0, 1, 2, 3])
def test_hierarchy_is_bit_exact(ctx, name, k):
    m = meshes_for_bitexact()[name]
    h = ctx.mesh_upload(m.xy, m.tri, m.dirichlet, k)
    ref = mesh.Hierarchy(m.xy, m.tri, m.dirichlet, k)
    try:
        assert ctx.mesh_levels(h) == k
        for lvl in range(k + 1):
            xy, tri, d, ends = ctx.mesh_download(h, lvl)
            np.testing.assert_array_equal(xy, ref.xy[lvl])
            np.testing.assert_array_equal(tri, ref.tri[lvl])
            np.testing.assert_array_equal(d, ref.dirichlet[lvl])
            if lvl < k:
                np.testing.assert_array_equal(ends, ref.ends[lvl])
        a = fem.system_matrix(m.xy, m.tri, m.dirichlet)
        rowptr, col, val, dinv = ctx.mesh_matrix(h)
        np.testing.assert_array_equal(rowptr, a.indptr)
        np.testing.assert_array_equal(col, a.indices)
        scale = np.abs(a.data).max()
        np.testing.assert_allclose(val, a.data, rtol=0, atol=1e-14 * scale)
        np.testing.assert_allclose(dinv, 1.0 / a.diagonal(), rtol=1e-13)
    finally:
        ctx.mesh_free(h)


def test_mesh_rejections(ctx, cgp):
    m = ci.jittered_rect(5, 4, 1)
    bad = m.tri.copy()
    bad[3] = bad[3][::-1]                      # clockwise triangle
    with pytest.raises(cgp.CGPError) as e:
        ctx.mesh_upload(m.xy, bad, m.dirichlet, 1)
    assert e.value.code == cgp.CGP_E_MESH
    bad = m.tri.copy()
    bad[0, 0] = m.n_nodes                      # out of range
    with pytest.raises(cgp.CGPError) as e:
        ctx.mesh_upload(m.xy, bad, m.dirichlet, 0)
    assert e.value.code == cgp.CGP_E_MESH
    with pytest.raises(cgp.CGPError) as e:
        ctx.mesh_upload(m.xy, m.tri, m.dirichlet, -1)
    assert e.value.code == cgp.CGP_E_INVALID


class Step:
    """One CGP step's inputs and oracle results on a jittered rectangle."""

    def __init__(self, nx, ny, seed, k=1, t=0.0):
        self.m = ci.jittered_rect(nx, ny, seed)
        self.h = mesh.Hierarchy(self.m.xy, self.m.tri, self.m.dirichlet, k)
        self.k = k
        modes = ci.fourier_modes(seed + 500)
        chi = ci.fourier_modes(seed + 700)
        xf = self.h.xy[k]
        self.u, self.v = ci.stream_velocity(xf, modes, t)
        du, dv = ci.potential_velocity(xf, chi, t)
        self.ut, self.vt = self.u + du, self.v + dv
        self.a = fem.system_matrix(self.m.xy, self.m.tri, self.m.dirichlet)
        nc = self.m.n_nodes
        self.b_phi = fem.source(self.m.xy, self.m.tri, self.m.dirichlet, self.u[:nc], self.v[:nc], fem.CURL, 1.0)
        self.b_p = fem.source(self.m.xy, self.m.tri, self.m.dirichlet, self.ut[:nc], self.vt[:nc], fem.DIV,
                              1.0 / ci.DT)


@pytest.fixture(scope="module")
def c1(ctx):
    s = Step(33, 17, 1001)
    s.handle = ctx.mesh_upload(s.m.xy, s.m.tri, s.m.dirichlet, 1)
    yield s
    ctx.mesh_free(s.handle)


def test_restrict_matches_oracle(ctx, cgp, c1):
    nc = c1.m.n_nodes
    uf, vf = dt(c1.u), dt(c1.v)
    b = torch.empty(nc, dtype=torch.float64, device=DEV)
    uc = torch.empty_like(b)
    vc = torch.empty_like(b)
    ctx.restrict(c1.handle, uf, vf, cgp.CGP_SRC_CURL, 1.0, b, uc, vc)
    bp = torch.empty_like(b)
    ctx.restrict(c1.handle, dt(c1.ut), dt(c1.vt), cgp.CGP_SRC_DIV, 1.0 / ci.DT, bp)
    ctx.sync()
    np.testing.assert_array_equal(uc.cpu().numpy(), c1.u[:nc])      # injection is a copy
    np.testing.assert_array_equal(vc.cpu().numpy(), c1.v[:nc])
    for got, ref in ((b, c1.b_phi), (bp, c1.b_p)):
        np.testing.assert_allclose(got.cpu().numpy(), ref, rtol=0, atol=1e-12 * np.abs(ref).max())


def test_restrict_from_the_fourth_level(ctx, cgp):
    # k = 3 (four nested levels, the paper's deepest coarsening): injection from level 3
    m = ci.jittered_rect(17, 9, 91)
    h = ctx.mesh_upload(m.xy, m.tri, m.dirichlet, 3)
    ref = mesh.Hierarchy(m.xy, m.tri, m.dirichlet, 3)
    try:
        nc, nf = m.n_nodes, ref.n_nodes(3)
        rng = np.random.default_rng(9)
        u, v = rng.standard_normal(nf), rng.standard_normal(nf)
        b, uc, vc = (torch.empty(nc, dtype=torch.float64, device=DEV) for _ in range(3))
        ctx.restrict(h, dt(u), dt(v), cgp.CGP_SRC_CURL, 1.0, b, uc, vc)
        ctx.sync()
        np.testing.assert_array_equal(uc.cpu().numpy(), mesh.restrict_inject(u, nc))
        np.testing.assert_array_equal(vc.cpu().numpy(), mesh.restrict_inject(v, nc))
        b_ref = fem.source(m.xy, m.tri, m.dirichlet, u[:nc], v[:nc], fem.CURL, 1.0)
        np.testing.assert_allclose(b.cpu().numpy(), b_ref, rtol=0, atol=1e-12 * np.abs(b_ref).max())
    finally:
        ctx.mesh_free(h)


@pytest.mark.parametrize("k", [1, 2, 3])
def test_prolong_is_bit_exact(ctx, k):
    m = ci.jittered_rect(21, 11, 77)
    h = ctx.mesh_upload(m.xy, m.tri, m.dirichlet, k)
    ref = mesh.Hierarchy(m.xy, m.tri, m.dirichlet, k)
    try:
        q = np.random.default_rng(3).standard_normal(m.n_nodes)
        qf = torch.empty(ref.n_nodes(k), dtype=torch.float64, device=DEV)
        ctx.prolong(h, dt(q), qf)
        ctx.sync()
        np.testing.assert_array_equal(qf.cpu().numpy(), mesh.prolong(q, ref))
    finally:
        ctx.mesh_free(h)


@pytest.mark.parametrize("k", [1, 2, 3])
def test_lorentz_force_matches_oracle(ctx, k):
    m = ci.jittered_rect(21, 11, 78)
    h = ctx.mesh_upload(m.xy, m.tri, m.dirichlet, k)
    ref = mesh.Hierarchy(m.xy, m.tri, m.dirichlet, k)
    try:
        rng = np.random.default_rng(4)
        nf = ref.n_nodes(k)
        phi, u, v = rng.standard_normal(nf), rng.standard_normal(nf), rng.standard_normal(nf)
        fx, fy = (torch.empty(nf, dtype=torch.float64, device=DEV) for _ in range(2))
        g = torch.empty(2 * ref.tri[k].shape[0], dtype=torch.float64, device=DEV)
        ctx.lorentz_force(h, dt(phi), dt(u), dt(v), 0.37, 1.3, fx, fy, g)
        ctx.sync()
        fxr, fyr, gr = fem.lorentz_force(ref.xy[k], ref.tri[k], phi, u, v, 0.37, 1.3)
        scale = np.abs(gr).max()
        np.testing.assert_allclose(fx.cpu().numpy(), fxr, rtol=0, atol=1e-12 * scale)
        np.testing.assert_allclose(fy.cpu().numpy(), fyr, rtol=0, atol=1e-12 * scale)
        np.testing.assert_allclose(g.cpu().numpy().reshape(-1, 2), gr, rtol=0, atol=1e-12 * scale)
    finally:
        ctx.mesh_free(h)


@pytest.mark.parametrize("k", [0, 1, 2])
def test_velocity_correction_matches_oracle(ctx, cgp, k):
    m = ci.jittered_rect(21, 11, 79)
    h = ctx.mesh_upload(m.xy, m.tri, m.dirichlet, k)
    ref = mesh.Hierarchy(m.xy, m.tri, m.dirichlet, k)
    try:
        rng = np.random.default_rng(5)
        nf = ref.n_nodes(k)
        p, ut, vt = rng.standard_normal(nf), rng.standard_normal(nf), rng.standard_normal(nf)
        ur, vr = fem.velocity_correction(ref.xy[k], ref.tri[k], p, ut, vt, 0.05)
        gscale = np.abs(fem.nodal_gradient(ref.xy[k], ref.tri[k], p)).max() * 0.05
        u, v = (torch.empty(nf, dtype=torch.float64, device=DEV) for _ in range(2))
        ctx.velocity_correct(h, dt(p), dt(ut), dt(vt), 0.05, u, v)
        # in place: the outputs overwrite the intermediate velocity
        ui, vi = dt(ut), dt(vt)
        ctx.velocity_correct(h, dt(p), ui, vi, 0.05, ui, vi)
        ctx.sync()
        for a, r in ((u, ur), (v, vr), (ui, ur), (vi, vr)):
            np.testing.assert_allclose(a.cpu().numpy(), r, rtol=0, atol=1e-12 * (gscale + 1.0))
        pf = dt(p)
        with pytest.raises(cgp.CGPError):
            ctx.velocity_correct(h, pf, dt(ut), dt(vt), 0.05, pf, v)
        with pytest.raises(cgp.CGPError):
            ctx.velocity_correct(h, pf, dt(ut), dt(vt), 0.05, u, u)
        with pytest.raises(cgp.CGPError):
            ctx.velocity_correct(h, pf, dt(ut), dt(vt), float("nan"), u, v)
    finally:
        ctx.mesh_free(h)


def _solve(ctx, cgp, handle, b, x0=None, guess=None, precision=0, tol=1e-10, **kw):
    n = b.shape[0]
    phi = dt(x0) if x0 is not None else torch.zeros(n, dtype=torch.float64, device=DEV)
    stats = cgp.stats_buffer(1)
    if guess is None:
        guess = cgp.CGP_GUESS_GIVEN if x0 is not None else cgp.CGP_GUESS_ZERO
    ctx.poisson_solve([handle], [dt(b)], [phi], stats, precision=precision, guess=guess, tol=tol, **kw)
    st = ctx.solve_check(1, stats)[0]
    return phi.cpu().numpy(), st


ENGINES = [1, 2, 3]   # CGP_ENGINE_STAGED (tiled), CGP_ENGINE_PERSISTENT, CGP_ENGINE_STAGED_ROWS


@pytest.mark.parametrize("engine", ENGINES)
@pytest.mark.parametrize("lanes", [1, 2, 4, 8])
def test_fp64_solve_matches_direct_and_oracle_pcg(ctx, cgp, c1, lanes, engine):
    for b in (c1.b_phi, c1.b_p):
        xs = solve.direct(c1.a, b)
        x, st = _solve(ctx, cgp, c1.handle, b, tol=1e-10, spmv_lanes=lanes, engine=engine)
        assert st["status"] == "ok" and st["rel_res"] <= 1e-10
        assert np.linalg.norm(x - xs) / np.linalg.norm(xs) <= 1e-8
        xo, info = solve.pcg(c1.a, b, tol=1e-10)
        assert abs(st["iters"] - info["iters"]) <= 2, (st, info)
        assert np.linalg.norm(x - xo) / np.linalg.norm(xo) <= 1e-9


@pytest.mark.parametrize("engine", ENGINES)
@pytest.mark.parametrize("lanes", [1, 4])
def test_mixed_solve_matches_direct(ctx, cgp, c1, lanes, engine):
    for b in (c1.b_phi, c1.b_p):
        xs = solve.direct(c1.a, b)
        x, st = _solve(ctx, cgp, c1.handle, b, precision=cgp.CGP_FP32_IR, tol=1e-8, spmv_lanes=lanes,
                       engine=engine, refine_delta=0.1)
        assert st["status"] == "ok" and st["rel_res"] <= 1e-8 and st["refinements"] >= 1
        assert np.linalg.norm(x - xs) / np.linalg.norm(xs) <= 1e-6
        _, info = solve.pcg_mixed(c1.a, b, tol=1e-8)
        assert abs(st["iters"] - info["iters"]) <= max(3, info["iters"] // 20), (st, info)


@pytest.mark.parametrize("engine", ENGINES)
def test_guess_modes(ctx, cgp, c1, engine):
    b = c1.b_phi
    xs = solve.direct(c1.a, b)
    for prec in (cgp.CGP_FP64, cgp.CGP_FP32_IR):
        _, st = _solve(ctx, cgp, c1.handle, b, x0=xs, precision=prec, tol=1e-8, engine=engine)
        assert st["iters"] == 0 and st["status"] == "ok"          # exact guess: nothing to do
        # extrapolation 2 p1 - p2 with p1 = p2 = x* is x*
        n = b.shape[0]
        phi = torch.zeros(n, dtype=torch.float64, device=DEV)
        stats = cgp.stats_buffer(1)
        ctx.poisson_solve([c1.handle], [dt(b)], [phi], stats, prev1=[dt(xs)], prev2=[dt(xs)],
                          precision=prec, guess=cgp.CGP_GUESS_EXTRAP, tol=1e-8, engine=engine)
        st = ctx.solve_check(1, stats)[0]
        assert st["iters"] == 0 and st["rel_res_guess"] <= 1e-8


@pytest.mark.parametrize("engine", ENGINES)
def test_edge_cases(ctx, cgp, c1, engine):
    n = c1.m.n_nodes
    # zero right-hand side: phi = 0 whatever the guess
    x, st = _solve(ctx, cgp, c1.handle, np.zeros(n), x0=np.ones(n), engine=engine)
    assert st["status"] == "ok" and st["iters"] == 0 and not x.any()
    # iteration cap
    _, st = _solve(ctx, cgp, c1.handle, c1.b_phi, max_iter=1, engine=engine)
    assert st["status"] == "noconv" and st["iters"] == 1
    _, st = _solve(ctx, cgp, c1.handle, c1.b_phi, precision=cgp.CGP_FP32_IR, tol=1e-8, max_iter=3, engine=engine)
    assert st["status"] == "noconv"
    # non-finite input
    bad = c1.b_phi.copy()
    bad[100] = np.nan
    for prec in (cgp.CGP_FP64, cgp.CGP_FP32_IR):
        _, st = _solve(ctx, cgp, c1.handle, bad, precision=prec, engine=engine)
        assert st["status"] == "breakdown"
    # argument validation: nothing enqueued, error code returned
    with pytest.raises(cgp.CGPError) as e:
        _solve(ctx, cgp, c1.handle, c1.b_phi, tol=-1.0)
    assert e.value.code == cgp.CGP_E_INVALID
    with pytest.raises(cgp.CGPError):
        _solve(ctx, cgp, c1.handle, c1.b_phi, spmv_lanes=3)
    with pytest.raises(cgp.CGPError):
        _solve(ctx, cgp, c1.handle, c1.b_phi, launches_per_graph=3)


@pytest.mark.parametrize("engine", ENGINES)
@pytest.mark.parametrize("nx,ny", [(3, 3), (2, 2), (4, 3)])
def test_degenerate_meshes(ctx, cgp, nx, ny, engine):
    m = ci.jittered_rect(nx, ny, 9)
    h = ctx.mesh_upload(m.xy, m.tri, m.dirichlet, 1)
    try:
        a = fem.system_matrix(m.xy, m.tri, m.dirichlet)
        b = np.where(m.dirichlet.astype(bool), 0.0, 1.0)
        x, st = _solve(ctx, cgp, h, b, tol=1e-12, engine=engine)
        assert st["status"] == "ok"
        if b.any():
            np.testing.assert_allclose(x, solve.direct(a, b), rtol=1e-10)
        else:
            assert not x.any()
    finally:
        ctx.mesh_free(h)


@pytest.mark.parametrize("engine", ENGINES)
def test_solves_are_bitwise_reproducible(ctx, cgp, c1, engine):
    x1, s1 = _solve(ctx, cgp, c1.handle, c1.b_phi, engine=engine)
    x2, s2 = _solve(ctx, cgp, c1.handle, c1.b_phi, engine=engine)
    np.testing.assert_array_equal(x1, x2)
    assert s1 == s2


@pytest.mark.parametrize("engine", ENGINES)
def test_batched_instances_match_single_solves(ctx, cgp, engine):
    sizes = [(17, 9), (33, 17), (9, 5), (65, 33), (25, 13)]
    steps = [Step(nx, ny, 3000 + i) for i, (nx, ny) in enumerate(sizes)]
    hs = [ctx.mesh_upload(s.m.xy, s.m.tri, s.m.dirichlet, 1) for s in steps]
    try:
        for prec, tol, bound in ((cgp.CGP_FP64, 1e-10, 1e-8), (cgp.CGP_FP32_IR, 1e-8, 1e-6)):
            bs = [dt(s.b_phi) for s in steps]
            xs = [torch.zeros_like(b) for b in bs]
            stats = cgp.stats_buffer(len(steps))
            ctx.poisson_solve(hs, bs, xs, stats, precision=prec, guess=cgp.CGP_GUESS_ZERO, tol=tol, engine=engine)
            sts = ctx.solve_check(len(steps), stats)
            for s, h, x, st in zip(steps, hs, xs, sts):
                assert st["status"] == "ok" and st["rel_res"] <= tol
                ref = solve.direct(s.a, s.b_phi)
                assert np.linalg.norm(x.cpu().numpy() - ref) / np.linalg.norm(ref) <= bound
                alone, st1 = _solve(ctx, cgp, h, s.b_phi, precision=prec, tol=tol, engine=engine)
                assert abs(st1["iters"] - st["iters"]) <= 2
                assert np.linalg.norm(x.cpu().numpy() - alone) / np.linalg.norm(ref) <= bound
    finally:
        for h in hs:
            ctx.mesh_free(h)


def test_graph_replay_matches_eager(ctx, cgp, c1):
    """A whole CGP step captured once and replayed: every replay equals the eager result bitwise."""
    nc, nf = c1.m.n_nodes, c1.h.n_nodes(1)
    uf, vf = dt(c1.u), dt(c1.v)
    b = torch.empty(nc, dtype=torch.float64, device=DEV)
    phi = torch.zeros(nc, dtype=torch.float64, device=DEV)
    phif, fx, fy = (torch.empty(nf, dtype=torch.float64, device=DEV) for _ in range(3))
    stats = cgp.stats_buffer(1)
    stream = torch.cuda.Stream()
    gctx = cgp.Context(0, stream=stream)
    h = gctx.mesh_upload(c1.m.xy, c1.m.tri, c1.m.dirichlet, 1)
    torch.cuda.synchronize()

    def step():
        gctx.restrict(h, uf, vf, cgp.CGP_SRC_CURL, 1.0, b)
        gctx.poisson_solve([h], [b], [phi], stats, precision=cgp.CGP_FP32_IR, guess=cgp.CGP_GUESS_ZERO, tol=1e-8,
                           engine=cgp.CGP_ENGINE_PERSISTENT)
        gctx.prolong(h, phi, phif)
        gctx.lorentz_force(h, phif, uf, vf, 0.5, 1.0, fx, fy)

    step()
    gctx.sync()
    eager = [t.cpu().numpy().copy() for t in (b, phi, phif, fx, fy)]
    xs = solve.direct(c1.a, c1.b_phi)
    assert np.linalg.norm(eager[1] - xs) / np.linalg.norm(xs) <= 1e-6
    gctx.graph_begin()
    step()
    g = gctx.graph_end()
    for rep in range(3):
        for t in (b, phi, phif, fx, fy):
            t.fill_(123.0)
        torch.cuda.synchronize()
        gctx.graph_launch(g)
        gctx.sync()
        for t, e in zip((b, phi, phif, fx, fy), eager):
            np.testing.assert_array_equal(t.cpu().numpy(), e)
        assert gctx.solve_check(1, stats)[0]["status"] == "ok"
    gctx.graph_free(g)
    # the staged engine records a solve only after an uncaptured one of the same launch records
    gctx.graph_begin()
    with pytest.raises(cgp.CGPError):
        gctx.poisson_solve([h], [b], [phi], stats, precision=cgp.CGP_FP32_IR, guess=cgp.CGP_GUESS_ZERO, tol=1e-8,
                           engine=cgp.CGP_ENGINE_STAGED)
    gctx.graph_free(gctx.graph_end())
    gctx.mesh_free(h)
    gctx.close()


# ---------------------------------------------------------------- Chebyshev polynomial preconditioner

def cheb_meshes():
    return {
        "rect_33x17": ci.jittered_rect(33, 17, 1001),
        "rect_129x65": ci.jittered_rect(129, 65, 1002),      # 17 tiles, regions several rows deep
        "hole_41x21": ci.rect_with_hole(41, 21, (12, 28, 6, 14), seed=5),
        "permuted_40x21": ci.permuted(ci.jittered_rect(40, 21, 6), seed=7),
        "ragged_7x4": ci.jittered_rect(7, 4, 5),
        # rows of 7 and 11 off-diagonal entries at the centre: the tiled iteration's width-8 and
        # width-12 records (the meshes above have at most 6 and take the split records)
        "wheel_7": ci.wheel(30, 7, 21),
        "wheel_11": ci.wheel(30, 11, 22),
    }


@pytest.fixture(scope="module")
def cheb_cases(ctx):
    out = {}
    for name, m in cheb_meshes().items():
        a = fem.system_matrix(m.xy, m.tri, m.dirichlet)
        u, v = ci.stream_velocity(m.xy, ci.fourier_modes(77), 0.0)
        b = fem.source(m.xy, m.tri, m.dirichlet, u, v, fem.CURL, 1.0)
        out[name] = (m, a, b, ctx.mesh_upload(m.xy, m.tri, m.dirichlet, 1))
    yield out
    for m, a, b, h in out.values():
        ctx.mesh_free(h)


@pytest.mark.parametrize("name", list(cheb_meshes()))
@pytest.mark.parametrize("degree", [1, 2, 3, 5, 8])
def test_chebyshev_fp64_matches_direct_and_oracle(ctx, cgp, cheb_cases, name, degree):
    m, a, b, h = cheb_cases[name]
    xs = solve.direct(a, b)
    x, st = _solve(ctx, cgp, h, b, tol=1e-10, precond_degree=degree)
    assert st["status"] == "ok" and st["rel_res"] <= 1e-10
    assert np.linalg.norm(x - xs) / np.linalg.norm(xs) <= 1e-8
    _, info = solve.pcg(a, b, tol=1e-10, degree=degree)
    assert abs(st["iters"] - info["iters"]) <= 2, (st, info)


@pytest.mark.parametrize("name", ["rect_129x65", "hole_41x21", "permuted_40x21", "wheel_7", "wheel_11"])
@pytest.mark.parametrize("degree", [2, 4, 8])
def test_chebyshev_mixed_matches_direct_and_oracle(ctx, cgp, cheb_cases, name, degree):
    m, a, b, h = cheb_cases[name]
    xs = solve.direct(a, b)
    x, st = _solve(ctx, cgp, h, b, precision=cgp.CGP_FP32_IR, tol=1e-8, precond_degree=degree, refine_delta=0.1)
    assert st["status"] == "ok" and st["rel_res"] <= 1e-8
    assert np.linalg.norm(x - xs) / np.linalg.norm(xs) <= 1e-6
    _, info = solve.pcg_mixed(a, b, tol=1e-8, degree=degree)
    assert abs(st["iters"] - info["iters"]) <= max(3, info["iters"] // 10), (st, info)


@pytest.mark.parametrize("names", [["rect_33x17", "rect_129x65", "hole_41x21"],
                                   ["rect_33x17", "wheel_7", "rect_129x65"]])   # split records with width 8
def test_chebyshev_guess_modes_and_batches(ctx, cgp, cheb_cases, names):
    hs = [cheb_cases[k][3] for k in names]
    bs = [dt(cheb_cases[k][2]) for k in names]
    refs = [solve.direct(cheb_cases[k][1], cheb_cases[k][2]) for k in names]
    for prec, tol, bound in ((cgp.CGP_FP64, 1e-10, 1e-8), (cgp.CGP_FP32_IR, 1e-8, 1e-6)):
        xs = [torch.zeros_like(b) for b in bs]
        stats = cgp.stats_buffer(len(hs))
        ctx.poisson_solve(hs, bs, xs, stats, precision=prec, guess=cgp.CGP_GUESS_ZERO, tol=tol, precond_degree=4)
        for x, ref, st in zip(xs, refs, ctx.solve_check(len(hs), stats)):
            assert st["status"] == "ok"
            assert np.linalg.norm(x.cpu().numpy() - ref) / np.linalg.norm(ref) <= bound
        # exact previous solutions: the extrapolation is exact, nothing to iterate
        xs = [torch.zeros_like(b) for b in bs]
        ctx.poisson_solve(hs, bs, xs, stats, prev1=[dt(r) for r in refs], prev2=[dt(r) for r in refs],
                          precision=prec, guess=cgp.CGP_GUESS_EXTRAP, tol=1e-8, precond_degree=4)
        assert all(st["iters"] == 0 for st in ctx.solve_check(len(hs), stats))


EARLY_END_CONFIGS = ["fp64_jacobi_rows", "fp64_jacobi_persistent", "fp64_cheb6", "fp32ir_cheb6",
                     "fp32ir_cheb6_deflated"]


def _early_end_kw(cgp, cfg):
    return {"fp64_jacobi_rows": dict(precision=cgp.CGP_FP64, tol=1e-10, engine=cgp.CGP_ENGINE_STAGED_ROWS),
            "fp64_jacobi_persistent": dict(precision=cgp.CGP_FP64, tol=1e-10, engine=cgp.CGP_ENGINE_PERSISTENT),
            "fp64_cheb6": dict(precision=cgp.CGP_FP64, tol=1e-10, precond_degree=6),
            "fp32ir_cheb6": dict(precision=cgp.CGP_FP32_IR, tol=1e-8, precond_degree=6),
            "fp32ir_cheb6_deflated": dict(precision=cgp.CGP_FP32_IR, tol=1e-8, precond_degree=6,
                                          deflation=1)}[cfg]


@pytest.mark.parametrize("cfg", EARLY_END_CONFIGS)
def test_batch_members_that_end_at_their_first_residual(ctx, cgp, cheb_cases, cfg):
    """A batch with a member whose b = 0 (started from ones, x must come back zero) and one
    started from its exact solution (nothing to iterate), beside a member that iterates: the first
    two end at their first residual stage and the launches after it find them finished, while the
    third solves to the tolerance in the iterations it takes alone."""
    kw = _early_end_kw(cgp, cfg)
    bound = 1e-8 if kw["precision"] == cgp.CGP_FP64 else 1e-6
    names = ["rect_33x17", "rect_129x65", "hole_41x21"]
    hs = [cheb_cases[k][3] for k in names]
    _, a1, b1, _ = cheb_cases[names[1]]
    _, a2, b2, _ = cheb_cases[names[2]]
    ref1, ref2 = solve.direct(a1, b1), solve.direct(a2, b2)
    n0 = cheb_cases[names[0]][0].n_nodes
    bs = [dt(np.zeros(n0)), dt(b1), dt(b2)]
    xs = [dt(np.ones(n0)), torch.zeros_like(bs[1]), dt(ref2)]
    stats = cgp.stats_buffer(3)
    ctx.poisson_solve(hs, bs, xs, stats, guess=cgp.CGP_GUESS_GIVEN, **kw)
    s0, s1, s2 = ctx.solve_check(3, stats)
    assert s0["status"] == "ok" and s0["iters"] == 0 and not xs[0].cpu().numpy().any(), s0
    assert s2["status"] == "ok" and s2["iters"] == 0, s2
    np.testing.assert_array_equal(xs[2].cpu().numpy(), ref2)
    x1 = xs[1].cpu().numpy()
    assert s1["status"] == "ok" and s1["iters"] > 0, s1
    assert np.linalg.norm(x1 - ref1) / np.linalg.norm(ref1) <= bound
    _, solo = _solve(ctx, cgp, hs[1], b1, x0=np.zeros_like(b1), **kw)
    assert abs(s1["iters"] - solo["iters"]) <= 1, (s1, solo)


@pytest.mark.parametrize("cfg", EARLY_END_CONFIGS)
def test_initial_iterate_ignores_what_x_holds(ctx, cgp, cheb_cases, cfg):
    """With a zero or extrapolated start the solve takes its initial iterate from the guess's
    source, not from x: the same batch started with x full of ones or of zeros gives the same bits
    and the same statistics."""
    kw = _early_end_kw(cgp, cfg)
    names = ["rect_33x17", "rect_129x65", "hole_41x21"]
    hs = [cheb_cases[k][3] for k in names]
    bs = [dt(cheb_cases[k][2]) for k in names]
    prev = [dt(0.5 * solve.direct(cheb_cases[k][1], cheb_cases[k][2])) for k in names]
    for guess, extra in ((cgp.CGP_GUESS_ZERO, {}), (cgp.CGP_GUESS_EXTRAP, dict(prev1=prev, prev2=prev))):
        runs = []
        for fill in (1.0, 0.0):
            xs = [torch.full_like(b, fill) for b in bs]
            stats = cgp.stats_buffer(3)
            ctx.poisson_solve(hs, bs, xs, stats, guess=guess, **extra, **kw)
            runs.append(([x.cpu().numpy() for x in xs], ctx.solve_check(3, stats)))
        (xa, sa), (xb, sb) = runs
        assert all(s["status"] == "ok" for s in sa), sa
        assert sa == sb
        for p, q in zip(xa, xb):
            np.testing.assert_array_equal(p, q)


def test_chebyshev_edge_cases(ctx, cgp, c1):
    n = c1.m.n_nodes
    x, st = _solve(ctx, cgp, c1.handle, np.zeros(n), x0=np.ones(n), precond_degree=5)
    assert st["status"] == "ok" and st["iters"] == 0 and not x.any()
    _, st = _solve(ctx, cgp, c1.handle, c1.b_phi, max_iter=2, precond_degree=5)
    assert st["status"] == "noconv" and st["iters"] == 2
    bad = c1.b_phi.copy()
    bad[7] = np.inf
    _, st = _solve(ctx, cgp, c1.handle, bad, precond_degree=3)
    assert st["status"] == "breakdown"
    x1, s1 = _solve(ctx, cgp, c1.handle, c1.b_phi, precision=cgp.CGP_FP32_IR, tol=1e-8, precond_degree=6)
    x2, s2 = _solve(ctx, cgp, c1.handle, c1.b_phi, precision=cgp.CGP_FP32_IR, tol=1e-8, precond_degree=6)
    np.testing.assert_array_equal(x1, x2)
    assert s1 == s2
    for kw in (dict(engine=cgp.CGP_ENGINE_PERSISTENT), dict(engine=cgp.CGP_ENGINE_STAGED_ROWS)):
        with pytest.raises(cgp.CGPError) as e:
            _solve(ctx, cgp, c1.handle, c1.b_phi, precond_degree=4, **kw)
        assert e.value.code == cgp.CGP_E_UNSUPPORTED
    with pytest.raises(cgp.CGPError) as e:
        _solve(ctx, cgp, c1.handle, c1.b_phi, precond_degree=9)
    assert e.value.code == cgp.CGP_E_INVALID
