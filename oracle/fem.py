"""Oracle: Galerkin P1 operators on a triangular mesh (Section 2.3).

* ``stiffness``          K_ij = sum_e A_e grad(psi_i) . grad(psi_j) (linear P1 shape functions);
* ``eliminate_dirichlet`` homogeneous Dirichlet rows/columns removed symmetrically,
                          Dirichlet rows replaced by identity rows;
* ``source``             the weak right-hand side of the coarse Poisson problems:
                          Eq. 12 (electric potential, curl of the restricted velocity
                          times B0) and Eq. 15 (pressure, divergence times rho/dt);
* ``gradient_lorentz``   grad(phi_f) and the Lorentz force of Eqs. 13-14;
* ``velocity_correction`` the projection of Eqs. 16-17 with grad(p_f).

Sign convention (Eq. 12 / Eq. 15 are Delta(phi) = f): multiplying by a test
function and integrating by parts gives K phi = b with b_i = -int f psi_i, so K is
the symmetric positive definite stiffness matrix and phi is the paper's phi.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp

CURL = 0   # Eq. 12 source: f = B0 (dv/dx - du/dy)
DIV = 1    # Eq. 15 source: f = (rho/dt) (du/dx + dv/dy)


def element_geometry(xy: np.ndarray, tri: np.ndarray):
    """Per triangle: area A_e and the constant shape-function gradients.

    Returns ``(area, gx, gy)`` with ``gx[e, a] = d psi_a / dx`` for local vertex a.
    """
    x = xy[tri, 0]
    y = xy[tri, 1]
    xa, xb, xc = x[:, 0], x[:, 1], x[:, 2]
    ya, yb, yc = y[:, 0], y[:, 1], y[:, 2]
    twice_area = (xb - xa) * (yc - ya) - (xc - xa) * (yb - ya)
    gx = np.stack([yb - yc, yc - ya, ya - yb], axis=1) / twice_area[:, None]
    gy = np.stack([xc - xb, xa - xc, xb - xa], axis=1) / twice_area[:, None]
    return 0.5 * twice_area, gx, gy


def stiffness(xy: np.ndarray, tri: np.ndarray) -> sp.csr_matrix:
    """Unconstrained P1 stiffness matrix (no boundary conditions), CSR with sorted columns."""
    n = xy.shape[0]
    area, gx, gy = element_geometry(xy, tri)
    if np.any(area <= 0):
        raise ValueError("non-positive triangle area (triangles must be CCW)")
    ke = area[:, None, None] * (gx[:, :, None] * gx[:, None, :] + gy[:, :, None] * gy[:, None, :])
    rows = np.repeat(tri[:, :, None], 3, axis=2)
    cols = np.repeat(tri[:, None, :], 3, axis=1)
    k = sp.coo_matrix((ke.ravel(), (rows.ravel(), cols.ravel())), shape=(n, n)).tocsr()
    k.sum_duplicates()
    k.sort_indices()
    return k


def eliminate_dirichlet(k: sp.csr_matrix, dirichlet: np.ndarray) -> sp.csr_matrix:
    """Drop every entry in a Dirichlet row or column and put 1 on the Dirichlet diagonal."""
    coo = k.tocoo()
    d = np.asarray(dirichlet, dtype=bool)
    keep = ~d[coo.row] & ~d[coo.col]
    nd = np.flatnonzero(d)
    rows = np.concatenate([coo.row[keep], nd])
    cols = np.concatenate([coo.col[keep], nd])
    vals = np.concatenate([coo.data[keep], np.ones(nd.size)])
    out = sp.coo_matrix((vals, (rows, cols)), shape=k.shape).tocsr()
    out.sort_indices()
    return out


def system_matrix(xy, tri, dirichlet) -> sp.csr_matrix:
    """The SPD matrix of the coarse Poisson solves."""
    return eliminate_dirichlet(stiffness(xy, tri), dirichlet)


def jacobi_inverse(a: sp.csr_matrix) -> np.ndarray:
    return 1.0 / a.diagonal()


def element_curl_div(xy, tri, u, v):
    """Element-constant curl (dv/dx - du/dy) and divergence (du/dx + dv/dy) of the P1 interpolant."""
    area, gx, gy = element_geometry(xy, tri)
    ue = u[tri]
    ve = v[tri]
    curl = (ve * gx - ue * gy).sum(axis=1)
    div = (ue * gx + ve * gy).sum(axis=1)
    return area, curl, div


def source(xy, tri, dirichlet, u_c, v_c, kind: int, scale: float) -> np.ndarray:
    """Right-hand side b of K phi = b for Eq. 12 (kind=CURL, scale=B0) or Eq. 15 (kind=DIV, scale=rho/dt).

    f = scale * q_e is constant on each element, and int_e q_e psi_i = q_e A_e / 3,
    so b_i = -scale * sum_{e containing i} q_e A_e / 3; b_i = 0 on Dirichlet rows.
    """
    area, curl, div = element_curl_div(xy, tri, u_c, v_c)
    q = curl if kind == CURL else div
    contrib = -scale * q * area / 3.0
    b = np.zeros(xy.shape[0])
    for a in range(3):
        np.add.at(b, tri[:, a], contrib)
    b[np.asarray(dirichlet, dtype=bool)] = 0.0
    return b


def element_gradient(xy, tri, phi):
    """grad(phi) on each element of a P1 field: sum_a phi_a grad(psi_a). Returns (T, 2)."""
    area, gx, gy = element_geometry(xy, tri)
    pe = phi[tri]
    return np.stack([(pe * gx).sum(axis=1), (pe * gy).sum(axis=1)], axis=1)


def nodal_gradient(xy, tri, phi):
    """Area-weighted average of the element gradients around each node."""
    area, _, _ = element_geometry(xy, tri)
    g = element_gradient(xy, tri, phi)
    n = xy.shape[0]
    num = np.zeros((n, 2))
    den = np.zeros(n)
    for a in range(3):
        np.add.at(num, tri[:, a], area[:, None] * g)
        np.add.at(den, tri[:, a], area)
    return num / den[:, None]


def lorentz_force(xy, tri, phi_f, u_f, v_f, sigma: float, b0: float):
    """Source of Eqs. 13-14: j x B with j = sigma (-grad phi + u x B) and B = B0 z (Eqs. 4, 11).

    F_x = sigma B0 (-dphi/dy - B0 u),  F_y = sigma B0 (dphi/dx - B0 v).
    Returns ``(fx, fy, grad_elem)``.
    """
    g = nodal_gradient(xy, tri, phi_f)
    fx = sigma * b0 * (-g[:, 1] - b0 * u_f)
    fy = sigma * b0 * (g[:, 0] - b0 * v_f)
    return fx, fy, element_gradient(xy, tri, phi_f)


def velocity_correction(xy, tri, p_f, ut, vt, scale: float, mask=None):
    """Eqs. 16-17: u = ut - scale dp/dx, v = vt - scale dp/dy with scale = dt/rho.

    The derivatives of the prolonged pressure are its nodal gradient (the same
    area-weighted mean of element gradients as the Lorentz source uses).  ``mask``
    (per node, optional): a component whose bit is set (0: u, 1: v) keeps its
    intermediate value there (its Dirichlet value from the momentum step).
    """
    g = nodal_gradient(xy, tri, p_f)
    u, v = ut - scale * g[:, 0], vt - scale * g[:, 1]
    if mask is not None:
        m = np.asarray(mask, dtype=np.uint8)
        u = np.where((m & 1) != 0, ut, u)
        v = np.where((m & 2) != 0, vt, v)
    return u, v
