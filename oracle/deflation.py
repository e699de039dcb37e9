"""Oracle: subdomain deflation of the coarse Poisson solves (test infrastructure).

An extension of the method, not part of the paper: the preconditioned CG of the
coarse solves (Eqs. 12 and 15) is run on the complement of a coarse space of
aggregates, "deflated CG" (Nicolaides, SIAM J. Numer. Anal. 24, 1987; Saad,
Yeung, Erhel and Guyomarc'h, SIAM J. Sci. Comput. 21, 2000).  With Z the n x m
matrix whose column a is the indicator of the free rows of aggregate a and
E = Z^T K Z, the iteration keeps Z^T r = 0 and K-orthogonalises every search
direction against range(Z):

    x0 <- x0 + Z E^-1 Z^T (b - K x0),  r0 = b - K x0,  u0 = M^-1 r0
    p0 = u0 - Z E^-1 Z^T K u0
    alpha = (r, u) / (p, K p);  x += alpha p;  r -= alpha K p;  u = M^-1 r
    beta = (r', u') / (r, u);   p <- u' + beta p - Z E^-1 Z^T K u'

so that the smooth error components that range(Z) captures, which a local
preconditioner removes only slowly, cost no iterations.

* ``rcb_parts``        recursive coordinate bisection of the nodes;
* ``tile_parts``       the tiles of the tiled solver: RCB into ceil(n / 512)
                       parts (or, when that exceeds 256, into 256 parts of up
                       to 1024 rows), more while a part or its matrix-graph
                       neighbourhood outgrows a workgroup's capacity;
* ``aggregates``       the coarse space's aggregates: every tile bisected once
                       more by the same rule (two per tile);
* ``deflation_space``  Z and E (an aggregate without free rows gets E_aa = 1,
                       which keeps E positive definite and its coefficient 0);
* ``dpcg``             the deflated PCG above in fp64, with the Jacobi, no, or
                       Chebyshev preconditioner.

Nothing here is shared with the device library; only the partition rule is
the same by definition.
"""
from __future__ import annotations

import numpy as np
import scipy.linalg
import scipy.sparse as sp

from . import solve

TILE_ROWS = 512        # rows of a part (one per thread of a workgroup)
TILE_ROWS_MAX = 1024   # rows a part may have (two per thread)
TILE_GRID = 256        # parts aimed for when more than this many parts of TILE_ROWS are needed
TILE_REGION = 2048     # rows within distance d of a part
TILE_SPMV = 1536       # rows within distance d - 1 of a part
MIN_ROWS = 64          # parts are never cut below this size
# lower end of the Chebyshev interval as a fraction of its upper end, with deflation
DEFL_CHEB_RATIO = 30.0
AGGREGATES_PER_TILE = 2


def rcb_parts(xy: np.ndarray, ids: np.ndarray, parts: int) -> list[np.ndarray]:
    """Split ``ids`` into ``parts`` pieces by recursive coordinate bisection.

    A piece of c nodes that must yield q parts is cut across the longer side of
    its bounding box (x on a tie): its c q' / q nodes (q' = q // 2, integer
    division) with the smallest (coordinate, id) form the first piece, cut again
    into q' parts, the rest into q - q'.  Returned in that depth-first order,
    each piece sorted by id.
    """
    ids = np.asarray(ids, dtype=np.int64)
    if parts <= 1:
        return [np.sort(ids)]
    p = xy[ids]
    ext = p.max(axis=0) - p.min(axis=0)
    ax = 0 if ext[0] >= ext[1] else 1
    pl = parts // 2
    nl = len(ids) * pl // parts
    order = np.lexsort((ids, p[:, ax]))      # by coordinate, then by id
    return rcb_parts(xy, ids[order[:nl]], pl) + rcb_parts(xy, ids[order[nl:]], parts - pl)


def _rings(k: sp.csr_matrix, own: np.ndarray, degree: int) -> list[int]:
    """Row counts of the part's neighbourhood at distance <= t in the matrix graph, t = 0..degree."""
    seen = set(int(i) for i in own)
    front = list(seen)
    counts = [len(seen)]
    for _ in range(degree):
        nxt = set()
        for i in front:
            for j in k.indices[k.indptr[i]:k.indptr[i + 1]]:
                j = int(j)
                if j not in seen:
                    nxt.add(j)
        seen |= nxt
        front = list(nxt)
        counts.append(len(seen))
    return counts


def tile_parts(k: sp.csr_matrix, xy: np.ndarray, degree: int) -> list[np.ndarray] | None:
    """Tiles: RCB parts of at most TILE_ROWS_MAX rows whose distance-<=d neighbourhood
    holds at most TILE_REGION rows and distance-<=(d-1) neighbourhood TILE_SPMV rows.

    Starts from ceil(n / TILE_ROWS) parts, or, when that exceeds TILE_GRID, from
    max(TILE_GRID, ceil(n / TILE_ROWS_MAX)) parts, and adds max(1, parts // 8) until
    every part fits, giving up (None) past ceil(n / MIN_ROWS) parts.
    """
    k = sp.csr_matrix(k)
    n = k.shape[0]
    parts = -(-n // TILE_ROWS)
    if parts > TILE_GRID:
        parts = max(TILE_GRID, -(-n // TILE_ROWS_MAX))
    max_parts = -(-n // MIN_ROWS)
    while parts <= max_parts:
        pieces = rcb_parts(xy, np.arange(n), parts)
        ok = True
        for own in pieces:
            if len(own) > TILE_ROWS_MAX:
                ok = False
                break
            c = _rings(k, own, degree)
            if c[degree] > TILE_REGION or c[max(degree - 1, 0)] > TILE_SPMV:
                ok = False
                break
        if ok:
            return pieces
        parts += max(1, parts // 8)
    return None


def aggregates(k: sp.csr_matrix, xy: np.ndarray, degree: int) -> list[np.ndarray] | None:
    """The tiles of ``tile_parts``, each cut in two by ``rcb_parts``: aggregates 2t and 2t + 1."""
    tiles = tile_parts(k, xy, degree)
    if tiles is None:
        return None
    return [half for t in tiles for half in rcb_parts(xy, t, AGGREGATES_PER_TILE)]


def deflation_space(k: sp.csr_matrix, dirichlet, pieces: list[np.ndarray]):
    """Returns ``(Z, E)``: Z (n x m, CSR) indicators of the free rows of each piece, E = Z^T K Z
    (dense), with E_aa = 1 for a piece without free rows."""
    n = k.shape[0]
    free = np.asarray(dirichlet) == 0
    rows, cols = [], []
    for a, own in enumerate(pieces):
        own = own[free[own]]
        rows.append(own)
        cols.append(np.full(len(own), a))
    rows = np.concatenate(rows) if rows else np.zeros(0, dtype=np.int64)
    cols = np.concatenate(cols) if cols else np.zeros(0, dtype=np.int64)
    z = sp.csr_matrix((np.ones(len(rows)), (rows, cols)), shape=(n, len(pieces)))
    e = (z.T @ (k @ z)).toarray()
    empty = np.asarray(z.sum(axis=0)).ravel() == 0
    e[empty, :] = 0.0
    e[:, empty] = 0.0
    e[empty, empty] = 1.0
    return z, e


def dpcg(k: sp.csr_matrix, b: np.ndarray, z: sp.csr_matrix, e: np.ndarray, x0: np.ndarray | None = None,
         tol: float = 1e-8, max_iter: int = 100000, degree: int = 1, ratio: float = DEFL_CHEB_RATIO,
         history: list | None = None):
    """fp64 deflated PCG, stopping on ||r|| <= tol ||b|| of the recursive residual and then
    verifying the true residual.  ``degree``: 0 none, 1 Jacobi, d >= 2 Chebyshev of degree d on
    [hi / ratio, hi].  ``history`` (optional) receives (Z^T r, Z^T K p, ||K p||) of every iteration.
    Returns ``(x, info)`` with info = {status, iters, rel_res}."""
    k = sp.csr_matrix(k)
    n = k.shape[0]
    if degree <= 0:
        prec = lambda r: r.copy()
    elif degree == 1:
        dinv = 1.0 / k.diagonal()
        prec = lambda r: dinv * r
    else:
        hi = solve.gershgorin_bound(k)
        prec = lambda r: solve.cheb_apply(k, r, degree, hi / ratio, hi)
    cf = scipy.linalg.cho_factor(e)
    coarse = lambda v: z @ scipy.linalg.cho_solve(cf, z.T @ v)
    b = np.asarray(b, dtype=np.float64)
    bn = float(np.linalg.norm(b))
    x = np.zeros(n) if x0 is None else np.array(x0, dtype=np.float64, copy=True)
    if bn == 0.0:
        return np.zeros(n), {"status": "ok", "iters": 0, "rel_res": 0.0}
    x = x + coarse(b - k @ x)
    r = b - k @ x
    if np.linalg.norm(r) <= tol * bn:
        return x, {"status": "ok", "iters": 0, "rel_res": float(np.linalg.norm(r)) / bn}
    u = prec(r)
    p = u - coarse(k @ u)
    g = float(r @ u)
    it = 0
    while it < max_iter:
        kp = k @ p
        a = g / float(p @ kp)
        x += a * p
        r -= a * kp
        it += 1
        if history is not None:
            history.append((z.T @ r, z.T @ kp, float(np.linalg.norm(kp))))
        if np.linalg.norm(r) <= tol * bn:
            rt = float(np.linalg.norm(b - k @ x)) / bn
            if rt <= tol:
                return x, {"status": "ok", "iters": it, "rel_res": rt}
            r = b - k @ x                      # a failed verification restarts from the true residual
            x = x + coarse(r)
            r = b - k @ x
            u = prec(r)
            p = u - coarse(k @ u)
            g = float(r @ u)
            continue
        u = prec(r)
        g2 = float(r @ u)
        p = u + (g2 / g) * p - coarse(k @ u)
        g = g2
    return x, {"status": "noconv", "iters": it, "rel_res": float(np.linalg.norm(b - k @ x)) / bn}
