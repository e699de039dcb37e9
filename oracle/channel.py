"""Oracle: the flow past a cylinder of Section 3 — surface force and one CGP time step
(test infrastructure).

* ``surface_force``  the force of the fluid on a body over a list of its boundary edges
  (a, b, t): t the fluid triangle that owns edge ab.  Per edge, the unit normal n points
  out of the body, into t; the pressure part is -int p n ds with p linear along the
  edge (exact: the mean of its end values times the length), the viscous part
  int mu (grad w + grad w^T) n ds with the constant P1 gradient of t.  Returns the
  pressure and the viscous force, 2-vectors each.  The paper names drag and lift and
  their viscous parts without writing a formula: this is the standard traction
  integral of the Newtonian stress -p I + mu (grad w + grad w^T).
* ``coefficients``   C = 2 F / (rho u_inf^2 d) for each force.
* ``cgp_step``       one time step of the algorithm of Section 2.3 with the
  electric-potential and pressure solves on the coarse level: (1) inject u_f; (2) solve
  Eq. 12 with the electric potential's Dirichlet set; (3) prolong phi; the Lorentz
  source (Eqs. 13-14); (4) the momentum step with per-component Dirichlet rows;
  (5) inject u~; (6) solve Eq. 15 with the pressure's Dirichlet set; (7) prolong p;
  (8) correct (Eqs. 16-17), components with a Dirichlet bit keeping their value.
"""
from __future__ import annotations

import numpy as np

from . import fem, mesh, solve
from . import momentum as mom


def surface_force(xy, tri, edges, p, u, v, mu: float):
    xy = np.asarray(xy, dtype=np.float64)
    tri = np.asarray(tri, dtype=np.int64)
    e = np.asarray(edges, dtype=np.int64).reshape(-1, 3)
    fp = np.zeros(2)
    fv = np.zeros(2)
    if e.shape[0] == 0:
        return fp, fv
    a, b, t = e[:, 0], e[:, 1], e[:, 2]
    d = xy[b] - xy[a]
    length = np.hypot(d[:, 0], d[:, 1])
    n = np.stack([d[:, 1], -d[:, 0]], axis=1) / length[:, None]
    third = tri[t].sum(axis=1) - a - b                 # the triangle's vertex off the edge
    flip = ((xy[third] - xy[a]) * n).sum(axis=1) < 0.0
    n[flip] = -n[flip]                                 # into the fluid triangle
    pm = 0.5 * (np.asarray(p)[a] + np.asarray(p)[b])
    fp = -(pm[:, None] * n * length[:, None]).sum(axis=0)
    gu = fem.element_gradient(xy, tri[t], np.asarray(u, dtype=np.float64))
    gv = fem.element_gradient(xy, tri[t], np.asarray(v, dtype=np.float64))
    sxx, syy, sxy = 2.0 * gu[:, 0], 2.0 * gv[:, 1], gu[:, 1] + gv[:, 0]
    tx = mu * (sxx * n[:, 0] + sxy * n[:, 1])
    ty = mu * (sxy * n[:, 0] + syy * n[:, 1])
    fv = np.array([(tx * length).sum(), (ty * length).sum()])
    return fp, fv


def coefficients(force, rho: float = 1.0, u_inf: float = 1.0, d: float = 1.0):
    return 2.0 * np.asarray(force, dtype=np.float64) / (rho * u_inf * u_inf * d)


def cgp_step(hier_phi: mesh.Hierarchy, hier_p: mesh.Hierarchy, u, v, vel_mask, gu, gv, rho: float, mu: float,
             dt: float, sigma: float, b0: float):
    """One CGP step on the finest level of two hierarchies of the same mesh (one per Dirichlet
    set); returns (u, v, phi_f, p_f, fx, fy, ut, vt)."""
    k = hier_p.k
    nc = hier_p.n_nodes(0)
    xy, tri = hier_p.xy[k], hier_p.tri[k]
    c0 = (hier_phi.xy[0], hier_phi.tri[0], hier_phi.dirichlet[0])
    b = fem.source(*c0, mesh.restrict_inject(u, nc), mesh.restrict_inject(v, nc), fem.CURL, b0)
    phi_c = solve.direct(fem.system_matrix(*c0), b)
    phi_f = mesh.prolong(phi_c, hier_phi)
    fx, fy, _ = fem.lorentz_force(xy, tri, phi_f, u, v, sigma, b0)
    m = np.asarray(vel_mask, dtype=np.uint8)
    ut0 = np.where((m & 1) != 0, gu, u)
    vt0 = np.where((m & 2) != 0, gv, v)
    ut, vt = mom.step(xy, tri, None, u, v, fx, fy, rho, mu, dt, gu=ut0, gv=vt0, mask=m)
    c1 = (hier_p.xy[0], hier_p.tri[0], hier_p.dirichlet[0])
    b = fem.source(*c1, mesh.restrict_inject(ut, nc), mesh.restrict_inject(vt, nc), fem.DIV, rho / dt)
    p_c = solve.direct(fem.system_matrix(*c1), b)
    p_f = mesh.prolong(p_c, hier_p)
    un, vn = fem.velocity_correction(xy, tri, p_f, ut, vt, dt / rho, mask=m)
    return un, vn, phi_f, p_f, fx, fy, ut, vt
