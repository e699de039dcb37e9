"""Oracle: P1 interpolation at arbitrary points by point location (test infrastructure).

The general restriction of Section 2.3 maps a fine field onto the nodes of a coarse
mesh that need not be nested in it: each coarse node is located in a fine triangle
and the fine P1 field is evaluated there.  ``locate`` is brute force over all
triangles: a point is in triangle t when its three barycentric coordinates are
>= -EPS; among several (a point on an edge or at a vertex), the triangle with the
largest smallest coordinate is taken, the lowest id on a tie.  Outside every
triangle: -1 and NaN.  On a shared edge any of the triangles gives the same value
of a continuous P1 field (up to rounding), so tests compare values and check the
chosen triangle for validity.
"""
from __future__ import annotations

import numpy as np

EPS = 1e-12


def barycentric(xy: np.ndarray, tri: np.ndarray, p: np.ndarray) -> np.ndarray:
    """(T, 3) barycentric coordinates of the point p in every triangle (Cramer's rule on
    p - a = l1 (b - a) + l2 (c - a))."""
    a, b, c = xy[tri[:, 0]], xy[tri[:, 1]], xy[tri[:, 2]]
    e1, e2, d = b - a, c - a, p[None, :] - a
    det = e1[:, 0] * e2[:, 1] - e1[:, 1] * e2[:, 0]
    l1 = (d[:, 0] * e2[:, 1] - d[:, 1] * e2[:, 0]) / det
    l2 = (e1[:, 0] * d[:, 1] - e1[:, 1] * d[:, 0]) / det
    return np.stack([1.0 - l1 - l2, l1, l2], axis=1)


def locate(xy, tri, pts):
    """Returns (triangle per point or -1, barycentric coordinates (n, 3))."""
    xy = np.asarray(xy, dtype=np.float64)
    tri = np.asarray(tri, dtype=np.int64)
    pts = np.asarray(pts, dtype=np.float64).reshape(-1, 2)
    out_t = np.full(pts.shape[0], -1, dtype=np.int64)
    out_l = np.full((pts.shape[0], 3), np.nan)
    for i, p in enumerate(pts):
        lam = barycentric(xy, tri, p)
        m = lam.min(axis=1)
        best = int(np.argmax(m))          # first maximum: the lowest id on a tie
        if m[best] >= -EPS:
            out_t[i] = best
            out_l[i] = lam[best]
    return out_t, out_l


def interpolate(xy, tri, field, pts):
    """The P1 field at the points (NaN outside the mesh) and the containing triangles."""
    t, lam = locate(xy, tri, pts)
    tri = np.asarray(tri, dtype=np.int64)
    val = np.full(t.shape[0], np.nan)
    inside = t >= 0
    val[inside] = (lam[inside] * np.asarray(field, dtype=np.float64)[tri[t[inside]]]).sum(axis=1)
    return val, t
