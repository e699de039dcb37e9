"""Whole CGP time steps of the flow past a cylinder (Section 3), as a sequence of library calls.

Marshalling only: every step runs in the library's kernels (restriction and sources,
coarse solves, prolongation, Lorentz force, momentum step, velocity correction, surface
force).  Used by the channel benchmark workload and its parity tests.
"""
from __future__ import annotations


class ChannelRun:
    """The flow past a cylinder of Section 3 on the device: two hierarchies of one channel
    mesh (the electric potential's Dirichlet set: the box sides; the pressure's: the
    outflow), the fine level's per-component velocity mask (inflow and cylinder: both
    components, slip walls: v, outflow: none), the cylinder's boundary edges, and the
    buffers of one CGP time step (Section 2.3's steps 1-8, every one a library call).

    ``xy``, ``tri``: the channel mesh (level 0); ``phi_dirichlet``, ``p_dirichlet``: its
    Dirichlet nodes for the potential and the pressure; ``boundary(fine_xy, fine_tri)``
    classifies the finest level's boundary nodes (a dict of boolean ``inflow``, ``walls``,
    ``cylinder`` and the cylinder's edges ``cyl_edges`` as (a, b, triangle) rows)."""

    def __init__(self, ctx, xy, tri, phi_dirichlet, p_dirichlet, k: int, boundary, *, rho=1.0, mu=0.01,
                 dt=0.05, sigma=0.01, b0=1.0, solve_kw=None, mom_tol=1e-8, mom_max_iter=5000):
        import numpy as np
        import torch

        from . import CGP_GUESS_GIVEN, stats_buffer

        self.ctx = ctx
        self.rho, self.mu, self.dt, self.sigma, self.b0 = rho, mu, dt, sigma, b0
        self.mom_tol, self.mom_max_iter = mom_tol, mom_max_iter
        self.solve_kw = dict(solve_kw or {})
        dev = torch.device("cuda:0")
        f64 = dict(dtype=torch.float64, device=dev)
        self.h_phi = ctx.mesh_upload(xy, tri, phi_dirichlet, k)
        self.h_p = ctx.mesh_upload(xy, tri, p_dirichlet, k)
        self.k = k
        xy, tri, _, _ = ctx.mesh_download(self.h_p, k)
        self.fine_xy, self.fine_tri = xy, tri
        bnd = boundary(xy, tri)
        self.vmask_np = ((bnd["inflow"] | bnd["cylinder"]) * 3 | bnd["walls"] * 2).astype(np.uint8)
        self.cyl_np = bnd["cylinder"].astype(bool)
        self.edges_np = bnd["cyl_edges"]
        nc, nf = np.asarray(phi_dirichlet).shape[0], xy.shape[0]
        self.nc, self.nf = nc, nf
        self.vmask = torch.from_numpy(self.vmask_np).to(dev)
        self.edges = torch.from_numpy(np.ascontiguousarray(self.edges_np)).to(dev)
        # impulsive start: the free stream everywhere but on the cylinder
        u0 = np.where(self.cyl_np, 0.0, 1.0)
        self.u = torch.from_numpy(u0).to(dev)
        self.v = torch.zeros(nf, **f64)
        self.ut, self.vt = torch.empty(nf, **f64), torch.empty(nf, **f64)
        self.fx, self.fy = torch.empty(nf, **f64), torch.empty(nf, **f64)
        self.phi_c, self.p_c = torch.zeros(nc, **f64), torch.zeros(nc, **f64)
        self.phi_f, self.p_f = torch.empty(nf, **f64), torch.empty(nf, **f64)
        self.b_phi, self.b_p = torch.empty(nc, **f64), torch.empty(nc, **f64)
        self.force = torch.zeros(5, **f64)
        self.stats = stats_buffer(2)
        self._given = CGP_GUESS_GIVEN
        self.mom_iters = []

    def step(self):
        from . import CGP_SRC_CURL, CGP_SRC_DIV, STATS_BYTES
        ctx = self.ctx
        S = STATS_BYTES
        ctx.restrict(self.h_phi, self.u, self.v, CGP_SRC_CURL, self.b0, self.b_phi)          # steps 1-2
        ctx.poisson_solve([self.h_phi], [self.b_phi], [self.phi_c], self.stats[:S], guess=self._given,
                          **self.solve_kw)
        ctx.prolong(self.h_phi, self.phi_c, self.phi_f)                                            # step 3
        ctx.lorentz_force(self.h_phi, self.phi_f, self.u, self.v, self.sigma, self.b0, self.fx, self.fy)
        self.ut.copy_(self.u)                                                                    # step 4
        self.vt.copy_(self.v)
        st = ctx.momentum_step(self.h_p, self.u, self.v, self.fx, self.fy, self.rho, self.mu, self.dt, self.ut,
                               self.vt, tol=self.mom_tol, max_iter=self.mom_max_iter, mask=self.vmask)
        self.mom_iters.append(max(st["iters"]))
        ctx.restrict(self.h_p, self.ut, self.vt, CGP_SRC_DIV, self.rho / self.dt, self.b_p)   # steps 5-6
        ctx.poisson_solve([self.h_p], [self.b_p], [self.p_c], self.stats[S:], guess=self._given,
                          **self.solve_kw)
        ctx.prolong(self.h_p, self.p_c, self.p_f)                                                  # step 7
        ctx.velocity_correct(self.h_p, self.p_f, self.ut, self.vt, self.dt / self.rho, self.u, self.v,
                             mask=self.vmask)                                                    # step 8
        ctx.surface_force(self.h_p, self.k, self.edges, self.p_f, self.u, self.v, self.mu, self.force)
        return st

    def check(self):
        return self.ctx.solve_check(2, self.stats)

    def close(self):
        self.ctx.mesh_free(self.h_phi)
        self.ctx.mesh_free(self.h_p)
