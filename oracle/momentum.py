"""Oracle: the semi-implicit momentum step on the fine mesh (Eqs. 8, 13-14; test infrastructure).

Galerkin P1 (Section 2.3) form of Eqs. 13-14 for one velocity component w (u or v):

    (rho/dt) M w~ + rho C(u^n) w~ + mu K w~ = (rho/dt) M w^n + M f

* ``mass``        M_ij = sum_e int_e psi_i psi_j = sum_e A_e (1 + delta_ij) / 12;
* ``convection``  C_ij = sum_e int_e psi_i (a . grad psi_j) with the advecting velocity
                  a = u^n interpolated in P1: int_e psi_i psi_k = A_e (1 + delta_ik) / 12,
                  so C^e_ij = (A_e / 12) (sum_k a_k + a_i) . grad psi_j;
* ``K``           the P1 stiffness of ``fem.stiffness`` (the viscous term, -Delta);
* ``operator``    A = (rho/dt) M + rho C + mu K with every Dirichlet row replaced by the
                  identity row (the Dirichlet columns of the other rows stay: A is not
                  symmetric anyway);
* ``rhs``         (rho/dt) M w^n + M f on free rows (f: the nodal Lorentz force, in P1),
                  the boundary value g on Dirichlet rows;
* ``step``        both components, by the sparse direct solver (the exact result).

Readings: the time derivative uses the projected velocity u^n (the general scheme,
Eq. 8; Eq. 13 writes the intermediate velocity there); both components are advected by
u^n (the linearisation Eqs. 13-14 state); the boundary values of the intermediate
velocity are the caller's (inflow and walls are not specified by the method).
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from .fem import element_geometry, stiffness


def _assemble(tri: np.ndarray, n: int, ke: np.ndarray) -> sp.csr_matrix:
    rows = np.repeat(tri[:, :, None], 3, axis=2)
    cols = np.repeat(tri[:, None, :], 3, axis=1)
    m = sp.coo_matrix((ke.ravel(), (rows.ravel(), cols.ravel())), shape=(n, n)).tocsr()
    m.sum_duplicates()
    m.sort_indices()
    return m


def mass(xy: np.ndarray, tri: np.ndarray) -> sp.csr_matrix:
    """Consistent P1 mass matrix."""
    area, _, _ = element_geometry(xy, tri)
    local = (np.ones((3, 3)) + np.eye(3)) / 12.0
    return _assemble(tri, xy.shape[0], area[:, None, None] * local[None, :, :])


def convection(xy: np.ndarray, tri: np.ndarray, ax: np.ndarray, ay: np.ndarray) -> sp.csr_matrix:
    """C_ij = int psi_i (a . grad psi_j), a the P1 interpolant of the nodal field (ax, ay)."""
    area, gx, gy = element_geometry(xy, tri)
    sx = ax[tri].sum(axis=1)
    sy = ay[tri].sum(axis=1)
    # weight of row i: (A_e / 12) (sum_k a_k + a_i)
    wx = area[:, None] / 12.0 * (sx[:, None] + ax[tri])
    wy = area[:, None] / 12.0 * (sy[:, None] + ay[tri])
    ke = wx[:, :, None] * gx[:, None, :] + wy[:, :, None] * gy[:, None, :]
    return _assemble(tri, xy.shape[0], ke)


def operator(xy, tri, dirichlet, un, vn, rho: float, mu: float, dt: float) -> sp.csr_matrix:
    """A = (rho/dt) M + rho C(u^n) + mu K, Dirichlet rows replaced by identity rows."""
    a = (rho / dt) * mass(xy, tri) + rho * convection(xy, tri, un, vn) + mu * stiffness(xy, tri)
    a = sp.csr_matrix(a)
    d = np.asarray(dirichlet, dtype=bool)
    coo = a.tocoo()
    keep = ~d[coo.row]
    nd = np.flatnonzero(d)
    out = sp.coo_matrix((np.concatenate([coo.data[keep], np.ones(nd.size)]),
                         (np.concatenate([coo.row[keep], nd]), np.concatenate([coo.col[keep], nd]))),
                        shape=a.shape).tocsr()
    out.sum_duplicates()
    out.sort_indices()
    return out


def rhs(xy, tri, dirichlet, wn, f, g, rho: float, dt: float) -> np.ndarray:
    """(rho/dt) M w^n + M f on free rows, g on Dirichlet rows."""
    m = mass(xy, tri)
    b = m @ ((rho / dt) * np.asarray(wn, dtype=np.float64) + np.asarray(f, dtype=np.float64))
    d = np.asarray(dirichlet, dtype=bool)
    b[d] = np.asarray(g, dtype=np.float64)[d]
    return b


def step(xy, tri, dirichlet, un, vn, fx, fy, rho: float, mu: float, dt: float, gu=None, gv=None, mask=None):
    """The intermediate velocity (u~, v~) of Eqs. 13-14 by a direct solve; boundary values
    gu, gv (default: those of u^n, v^n).  ``mask`` (per node, optional) sets the Dirichlet
    rows of each component apart: bit 0 for u, bit 1 for v (a slip wall fixes v only, a
    natural outflow neither); without it both components use ``dirichlet``."""
    gu = un if gu is None else gu
    gv = vn if gv is None else gv
    if mask is None:
        du = dv = np.asarray(dirichlet, dtype=bool)
    else:
        m = np.asarray(mask, dtype=np.uint8)
        du, dv = (m & 1) != 0, (m & 2) != 0
    lu_u = spla.splu(sp.csc_matrix(operator(xy, tri, du, un, vn, rho, mu, dt)))
    lu_v = lu_u if np.array_equal(du, dv) else spla.splu(sp.csc_matrix(operator(xy, tri, dv, un, vn, rho, mu, dt)))
    ut = lu_u.solve(rhs(xy, tri, du, un, fx, gu, rho, dt))
    vt = lu_v.solve(rhs(xy, tri, dv, vn, fy, gv, rho, dt))
    return ut, vt
