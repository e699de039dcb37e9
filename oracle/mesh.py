"""Oracle: nested mesh hierarchy and the two-grid transfer operators.

Section 2.3 of the paper builds every fine mesh by uniformly subdividing each
triangle of the coarser one into four (Eq. 18: P = 4^-k M), restricts by
injection at coincident nodes (Eq. 19) and prolongs with the linear shape
functions of the containing coarse triangle, one level at a time (Eq. 20).

Numbering convention of the hierarchy (shared contract with the library, the
reading listed with the other readings of the paper):

* the nodes of level l keep their ids on level l+1;
* edges of level l are the sorted unique pairs (min id, max id), ordered
  lexicographically; the midpoint of edge e gets id N_l + e;
* triangle t = (a, b, c) with midpoints mab, mbc, mca has children
  4t+0 = (a, mab, mca), 4t+1 = (mab, b, mbc), 4t+2 = (mca, mbc, c),
  4t+3 = (mab, mbc, mca);
* a midpoint is a Dirichlet node iff its edge lies on the boundary (exactly one
  adjacent triangle) and both end points are Dirichlet nodes.
"""
from __future__ import annotations

import numpy as np


def triangle_edges(tri: np.ndarray) -> np.ndarray:
    """The three edges (a,b), (b,c), (c,a) of every triangle, shape (T, 3, 2)."""
    return np.stack([tri[:, [0, 1]], tri[:, [1, 2]], tri[:, [2, 0]]], axis=1)


def edges(n_nodes: int, tri: np.ndarray):
    """Unique undirected edges sorted by (min, max).

    Returns ``(ends, tri_edge, n_adjacent)``: ``ends`` (E,2) int64 end points
    (min, max); ``tri_edge`` (T,3) the edge id of each triangle side in the order
    (a,b), (b,c), (c,a); ``n_adjacent`` (E,) the number of triangles sharing it.
    """
    te = triangle_edges(np.asarray(tri, dtype=np.int64))
    lo = te.min(axis=2)
    hi = te.max(axis=2)
    key = lo * np.int64(n_nodes) + hi
    uniq, inverse, counts = np.unique(key.ravel(), return_inverse=True, return_counts=True)
    ends = np.stack([uniq // n_nodes, uniq % n_nodes], axis=1)
    return ends, inverse.reshape(-1, 3), counts


def refine(xy: np.ndarray, tri: np.ndarray, dirichlet: np.ndarray):
    """One uniform 4-way subdivision (Eq. 18 with k = 1).

    Returns ``(xy_f, tri_f, dirichlet_f, ends)`` where ``ends`` (E,2) gives the two
    parent nodes of midpoint node ``N + e``.
    """
    n = xy.shape[0]
    ends, tri_edge, n_adj = edges(n, tri)
    mid_xy = (xy[ends[:, 0]] + xy[ends[:, 1]]) * 0.5
    xy_f = np.concatenate([xy, mid_xy], axis=0)
    on_boundary = n_adj == 1
    mid_dir = on_boundary & (dirichlet[ends[:, 0]] != 0) & (dirichlet[ends[:, 1]] != 0)
    dir_f = np.concatenate([dirichlet.astype(np.uint8), mid_dir.astype(np.uint8)])
    a, b, c = tri[:, 0].astype(np.int64), tri[:, 1].astype(np.int64), tri[:, 2].astype(np.int64)
    mab = n + tri_edge[:, 0]
    mbc = n + tri_edge[:, 1]
    mca = n + tri_edge[:, 2]
    children = np.stack([
        np.stack([a, mab, mca], axis=1),
        np.stack([mab, b, mbc], axis=1),
        np.stack([mca, mbc, c], axis=1),
        np.stack([mab, mbc, mca], axis=1),
    ], axis=1)                                   # (T, 4, 3): child 4t+s
    tri_f = children.reshape(-1, 3).astype(np.int32)
    return xy_f, tri_f, dir_f, ends


class Hierarchy:
    """Levels 0 (coarse, the input mesh) .. k (finest)."""

    def __init__(self, xy, tri, dirichlet, k: int):
        if k < 0:
            raise ValueError("k must be >= 0")
        self.xy = [np.asarray(xy, dtype=np.float64)]
        self.tri = [np.asarray(tri, dtype=np.int32)]
        self.dirichlet = [np.asarray(dirichlet, dtype=np.uint8)]
        self.ends = []
        for _ in range(k):
            xf, tf, df, ends = refine(self.xy[-1], self.tri[-1], self.dirichlet[-1])
            self.xy.append(xf)
            self.tri.append(tf)
            self.dirichlet.append(df)
            self.ends.append(ends)
        self.k = k

    def n_nodes(self, level: int) -> int:
        return int(self.xy[level].shape[0])


def restrict_inject(q_f: np.ndarray, n_coarse: int) -> np.ndarray:
    """Eq. 19: q_c(beta) = q_f(alpha) where the nodes coincide.

    Under the hierarchical numbering coarse node beta *is* fine node beta, so the
    coincidence map is the identity on the first ``n_coarse`` ids.
    """
    return np.array(q_f[:n_coarse], dtype=np.float64, copy=True)


def prolong_one_level(q: np.ndarray, ends: np.ndarray) -> np.ndarray:
    """Eq. 20 from level l to level l+1: coinciding nodes copy, a midpoint takes
    the mean of its edge's end points (the P1 shape functions there are 1/2, 1/2, 0)."""
    mid = (q[ends[:, 0]] + q[ends[:, 1]]) * 0.5
    return np.concatenate([q, mid])


def prolong(q_c: np.ndarray, hier: Hierarchy) -> np.ndarray:
    """Prolong from level 0 to level k, one level at a time (the paper runs the
    prolongation once per coarsening level)."""
    q = np.asarray(q_c, dtype=np.float64)
    for ends in hier.ends:
        q = prolong_one_level(q, ends)
    return q


def parent_triangle(hier: Hierarchy, level: int) -> np.ndarray:
    """Level-0 ancestor of every triangle of ``level`` (child 4t+s has parent t)."""
    t = np.arange(hier.tri[level].shape[0], dtype=np.int64)
    return t >> (2 * level)
