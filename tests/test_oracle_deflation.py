"""Pins of the deflation oracle (subdomain deflation of the coarse solves).

The checks rest on facts outside the oracle: a hand-worked bisection, the
partition's defining properties, finite termination of CG on a deflated
spectrum, exactness when the coarse space holds the solution, the invariants
Z^T r = 0 and Z^T K p = 0 that define the method, and the direct solve.
"""
import numpy as np
import pytest
import scipy.sparse as sp

import cgp_inputs as ci
from oracle import deflation as dfl
from oracle import fem, solve


def _system(nx, ny, seed):
    m = ci.jittered_rect(nx, ny, seed)
    return m, fem.system_matrix(m.xy, m.tri, m.dirichlet)


def test_bisection_of_a_small_grid_by_hand():
    # 4 x 2 points, ids row by row: (0..3) at y = 0, (4..7) at y = 1
    xy = np.array([[x, y] for y in (0.0, 1.0) for x in (0.0, 1.0, 2.0, 3.0)])
    two = dfl.rcb_parts(xy, np.arange(8), 2)
    assert [p.tolist() for p in two] == [[0, 1, 4, 5], [2, 3, 6, 7]]
    # three parts: 8 * 1 // 3 = 2 smallest by (x, id) = ids 0 and 4; the rest is 3 | 3, cut across x
    # (extent 2 > 1), the three smallest by (x, id) being 1, 5 (x = 1) and 2 (x = 2, smaller id than 6)
    three = dfl.rcb_parts(xy, np.arange(8), 3)
    assert [p.tolist() for p in three] == [[0, 4], [1, 2, 5], [3, 6, 7]]
    # a tall box is cut across y first
    tall = dfl.rcb_parts(xy[:, ::-1].copy(), np.arange(8), 2)
    assert [p.tolist() for p in tall] == [[0, 1, 4, 5], [2, 3, 6, 7]]


@pytest.mark.parametrize("degree", [1, 4, 8])
def test_tile_parts_partition_the_rows_within_capacity(degree):
    m, k = _system(97, 49, 11)
    parts = dfl.tile_parts(k, m.xy, degree)
    assert parts is not None
    allrows = np.sort(np.concatenate(parts))
    np.testing.assert_array_equal(allrows, np.arange(m.n_nodes))
    assert len(parts) == -(-m.n_nodes // 512)          # the first count fits this mesh
    assert max(len(p) for p in parts) <= 512
    # bisection halves: sizes differ by at most one level of integer division
    sizes = np.array([len(p) for p in parts])
    assert sizes.max() - sizes.min() <= 2


def test_a_mesh_past_the_tile_grid_takes_256_larger_tiles():
    # 513 x 257 = 131841 rows need 258 tiles of 512: the rule takes 256 tiles (one per compute
    # unit) of up to 1024 rows instead; 509 x 257 = 130813 rows fit 256 tiles of 512
    for nx, size in ((513, (515, 516)), (509, (510, 511))):
        m, k = _system(nx, 257, 11)
        parts = dfl.tile_parts(k, m.xy, 6)
        assert len(parts) == 256
        np.testing.assert_array_equal(np.sort(np.concatenate(parts)), np.arange(m.n_nodes))
        assert {len(p) for p in parts} <= set(size)
    # a mesh needing more than 256 x 1024 rows starts from ceil(n / 1024) parts
    m, k = _system(641, 513, 11)
    parts = dfl.tile_parts(k, m.xy, 2)
    assert len(parts) == -(-m.n_nodes // 1024) and max(len(p) for p in parts) <= 1024


def test_aggregates_halve_every_tile():
    m, k = _system(97, 49, 11)
    tiles = dfl.tile_parts(k, m.xy, 8)
    aggs = dfl.aggregates(k, m.xy, 8)
    assert len(aggs) == 2 * len(tiles)
    for t, tile in enumerate(tiles):
        a, b = aggs[2 * t], aggs[2 * t + 1]
        np.testing.assert_array_equal(np.sort(np.concatenate([a, b])), tile)
        assert len(a) == len(tile) // 2
        # a cut across the longer side of the tile's bounding box
        ext = m.xy[tile].max(axis=0) - m.xy[tile].min(axis=0)
        ax = 0 if ext[0] >= ext[1] else 1
        assert m.xy[a, ax].max() <= m.xy[b, ax].min()


def test_empty_aggregate_gets_a_unit_diagonal():
    m, k = _system(9, 5, 3)
    dirich = np.flatnonzero(m.dirichlet)
    free = np.flatnonzero(m.dirichlet == 0)
    z, e = dfl.deflation_space(k, m.dirichlet, [free, dirich])
    assert e[1, 1] == 1.0 and e[0, 1] == 0.0 and e[1, 0] == 0.0
    ones = np.zeros(m.n_nodes)
    ones[free] = 1.0
    assert e[0, 0] == pytest.approx(ones @ (k @ ones), rel=1e-14)
    assert z[:, 1].nnz == 0


def test_coarse_space_holding_the_solution_needs_no_iteration():
    m, k = _system(21, 11, 5)
    rng = np.random.default_rng(1)
    b = rng.standard_normal(m.n_nodes) * (m.dirichlet == 0)
    xs = solve.direct(k, b)
    z = sp.csr_matrix(xs.reshape(-1, 1))
    e = np.array([[xs @ (k @ xs)]])
    x, info = dfl.dpcg(k, b, z, e, tol=1e-12, max_iter=2000, degree=1)
    assert info["iters"] == 0 and info["status"] == "ok"
    np.testing.assert_allclose(x, xs, rtol=0, atol=1e-12 * np.abs(xs).max())


def test_deflating_all_but_three_eigenvectors_terminates_in_three_iterations():
    m, k = _system(9, 6, None)
    kd = k.toarray()
    lam, v = np.linalg.eigh(kd)
    keep = [0, 1, len(lam) - 1]                   # three distinct eigenvalues (the Dirichlet rows give 1s)
    assert lam[1] - lam[0] > 1e-8 and lam[-1] - lam[1] > 1e-8 and abs(lam[1] - 1.0) > 1e-8
    z = sp.csr_matrix(np.delete(v, keep, axis=1))
    e = z.T.toarray() @ kd @ z.toarray()
    b = np.random.default_rng(2).standard_normal(m.n_nodes) * (m.dirichlet == 0)
    x, info = dfl.dpcg(k, b, z, e, tol=1e-10, max_iter=2000, degree=0)
    assert info["status"] == "ok" and info["iters"] <= 3
    np.testing.assert_allclose(x, np.linalg.solve(kd, b), rtol=0, atol=1e-9 * np.abs(x).max())


@pytest.mark.parametrize("degree", [1, 4])
def test_deflated_iteration_keeps_its_invariants_and_solves(degree):
    m, k = _system(65, 33, 7)
    parts = dfl.aggregates(k, m.xy, degree)
    z, e = dfl.deflation_space(k, m.dirichlet, parts)
    b = np.random.default_rng(3).standard_normal(m.n_nodes) * (m.dirichlet == 0)
    hist = []
    x, info = dfl.dpcg(k, b, z, e, tol=1e-10, max_iter=2000, degree=degree, history=hist)
    assert info["status"] == "ok" and info["rel_res"] <= 1e-10
    xs = solve.direct(k, b)
    np.testing.assert_allclose(x, xs, rtol=0, atol=1e-8 * np.abs(xs).max())
    zb = np.linalg.norm(z.T @ b)
    width = np.sqrt(max(len(p) for p in parts))      # an aggregate sum of unit vectors has norm <= this
    for ztr, ztkp, kpn in hist:
        assert np.linalg.norm(ztr) <= 1e-9 * zb                    # Z^T r = 0
        assert np.linalg.norm(ztkp) <= 1e-12 * width * kpn * len(parts)   # Z^T K p = 0
    # the coarse space removes the slow components: fewer iterations than without it
    _, plain = solve.pcg(k, b, tol=1e-10, degree=degree)
    assert info["iters"] < plain["iters"]


def test_deflation_with_chebyshev_cuts_iterations_on_a_smooth_source():
    m, k = _system(257, 129, 9)
    parts = dfl.aggregates(k, m.xy, 8)
    z, e = dfl.deflation_space(k, m.dirichlet, parts)
    u, v = ci.stream_velocity(m.xy, ci.fourier_modes(3))
    b = fem.source(m.xy, m.tri, m.dirichlet, u, v, fem.CURL, 1.0)
    x, info = dfl.dpcg(k, b, z, e, tol=1e-8, max_iter=2000, degree=8)
    _, plain = solve.pcg(k, b, tol=1e-8, degree=8)
    assert info["status"] == "ok" and info["rel_res"] <= 1e-8
    assert info["iters"] <= 0.8 * plain["iters"], (info, plain)
