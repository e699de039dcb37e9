"""Seeded synthetic inputs shared by the HIP path, the oracle and the benchmark.

This module only produces input data: meshes (node coordinates, CCW triangles,
Dirichlet flags), analytic velocity fields and sweep parameters.  It performs
none of the coarse-grid-projection arithmetic (no refinement, no assembly, no
transfer operators, no solves), so both sides of every parity test can consume
the same arrays without sharing method code.

The workloads stand in for the paper's cylinder-wake runs (Section 3): the
paper's Gmsh meshes and flow fields are not available, so nested P1 meshes of a
jittered rectangle and divergence-free Fourier stream-function flows are used.

Recipes (all RNG = numpy PCG64 via ``numpy.random.default_rng(seed)``):

* ``jittered_rect(nx, ny, seed)``: node (i, j) has id ``j*nx + i`` and sits at
  ``(lx*i/(nx-1), ly*j/(ny-1))``; every interior coordinate is displaced by an
  independent ``U(-0.2 h, 0.2 h)`` draw (h = the grid spacing along that axis).
  Cell (i, j) is split along its SW-NE diagonal into the CCW triangles
  ``(n00, n10, n11)`` and ``(n00, n11, n01)`` with ids ``2*(j*(nx-1)+i) + {0,1}``.
  Boundary nodes are Dirichlet nodes.
* ``fourier_modes(seed)``: 8 modes with wavevector ``pi*(p, q)``,
  ``p, q ~ U{1..4}``, amplitude ``N(0,1)/|k|^2``, phase ``U[0, 2 pi)`` and angular
  frequency ``U(0.5, 2)``.
* ``stream_velocity``: ``psi = sum_m c_m cos(k_m . x + theta_m + omega_m t)``,
  ``u = d psi / dy``, ``v = -d psi / dx`` evaluated analytically at given points.
* ``potential_velocity``: ``grad chi`` for a second mode set (adds a divergent
  part, used for the pressure-equation source).
* ``cylinder_channel``: the geometry of Section 3 (box [0, 38] x [0, 32], a cylinder of
  diameter 1 centred at (8, 16)) meshed by a Delaunay triangulation of graded points:
  ``n_circle`` nodes on the cylinder, rings around it (radial step 0.866 of the local
  size, alternate rings rotated by half a step), nodes along the box sides at the local
  size, and seeded dart throwing (PCG64, 3000 consecutive rejections end it) in the
  rest, a candidate kept when it is at least 0.8 of the local size from every node.
  Local size h = min(h0 + g r', h_max), h0 = pi d / n_circle, r' = the distance from the
  cylinder's surface with the downstream distance scaled by ``wake`` (finer in the wake).
  Triangles with their centroid inside the cylinder are removed.  The defaults give
  1733 nodes and 3335 triangles, close to the paper's coarsest (k = 3) mesh.
"""
from __future__ import annotations

import numpy as np

__all__ = [
    "Mesh",
    "jittered_rect",
    "rect_with_hole",
    "permuted",
    "wheel",
    "fourier_modes",
    "stream_velocity",
    "potential_velocity",
    "FourierSequence",
    "DeviceFourierSequence",
    "stuart_numbers",
    "batch_sizes",
    "Channel",
    "cylinder_channel",
    "channel_boundary",
    "DT",
]

#: time step of the paper's runs (Section 3), used to advance the synthetic phases
DT = 0.05


class Mesh:
    """Plain container: ``xy`` float64 (N,2), ``tri`` int32 (T,3) CCW, ``dirichlet`` uint8 (N,)."""

    def __init__(self, xy, tri, dirichlet, nx=None, ny=None):
        self.xy = np.ascontiguousarray(xy, dtype=np.float64)
        self.tri = np.ascontiguousarray(tri, dtype=np.int32)
        self.dirichlet = np.ascontiguousarray(dirichlet, dtype=np.uint8)
        self.nx, self.ny = nx, ny

    @property
    def n_nodes(self) -> int:
        return int(self.xy.shape[0])

    @property
    def n_tris(self) -> int:
        return int(self.tri.shape[0])


def _grid_triangles(nx: int, ny: int) -> np.ndarray:
    i, j = np.meshgrid(np.arange(nx - 1), np.arange(ny - 1), indexing="xy")
    i = i.ravel()
    j = j.ravel()
    n00 = j * nx + i
    n10 = n00 + 1
    n01 = n00 + nx
    n11 = n01 + 1
    tri = np.empty((2 * i.size, 3), dtype=np.int32)
    tri[0::2] = np.stack([n00, n10, n11], axis=1)
    tri[1::2] = np.stack([n00, n11, n01], axis=1)
    return tri


def jittered_rect(nx: int, ny: int, seed: int | None, jitter: float = 0.2,
                  lx: float = 2.0, ly: float = 1.0) -> Mesh:
    """Jittered structured P1 mesh of ``[0,lx] x [0,ly]`` (``seed=None`` or ``jitter=0`` = no jitter)."""
    if nx < 2 or ny < 2:
        raise ValueError("need at least 2x2 nodes")
    i, j = np.meshgrid(np.arange(nx), np.arange(ny), indexing="xy")
    i = i.ravel()
    j = j.ravel()
    x = lx * i / (nx - 1)
    y = ly * j / (ny - 1)
    boundary = (i == 0) | (i == nx - 1) | (j == 0) | (j == ny - 1)
    if seed is not None and jitter != 0.0:
        rng = np.random.default_rng(seed)
        d = rng.uniform(-1.0, 1.0, size=(nx * ny, 2))
        hx = lx / (nx - 1)
        hy = ly / (ny - 1)
        x = x + np.where(boundary, 0.0, jitter * hx * d[:, 0])
        y = y + np.where(boundary, 0.0, jitter * hy * d[:, 1])
    xy = np.stack([x, y], axis=1)
    return Mesh(xy, _grid_triangles(nx, ny), boundary.astype(np.uint8), nx, ny)


def rect_with_hole(nx: int, ny: int, hole: tuple[int, int, int, int], seed: int | None = None,
                   jitter: float = 0.2) -> Mesh:
    """Jittered rectangle with the cells ``i0 <= i < i1, j0 <= j < j1`` removed (a one-hole domain).

    Nodes strictly inside the hole are dropped and the rest renumbered in
    ascending order; nodes on the hole's rim are Dirichlet nodes, like the
    outer boundary.  A stand-in for the paper's domain with a cylinder cut out.
    """
    i0, i1, j0, j1 = hole
    if not (0 < i0 < i1 < nx - 1 and 0 < j0 < j1 < ny - 1):
        raise ValueError("hole must be strictly inside the grid")
    base = jittered_rect(nx, ny, seed, jitter)
    ci, cj = np.meshgrid(np.arange(nx - 1), np.arange(ny - 1), indexing="xy")
    cell_in_hole = ((ci >= i0) & (ci < i1) & (cj >= j0) & (cj < j1)).ravel()
    keep_tri = ~np.repeat(cell_in_hole, 2)
    tri = base.tri[keep_tri]
    ni, nj = np.meshgrid(np.arange(nx), np.arange(ny), indexing="xy")
    ni = ni.ravel()
    nj = nj.ravel()
    inside = (ni > i0) & (ni < i1) & (nj > j0) & (nj < j1)
    rim = (ni >= i0) & (ni <= i1) & (nj >= j0) & (nj <= j1) & ~inside
    # the rim may have been jittered as an interior node: put it back on the rim
    xy = base.xy.copy()
    gx = 2.0 * ni / (nx - 1)
    gy = 1.0 * nj / (ny - 1)
    xy[rim, 0] = gx[rim]
    xy[rim, 1] = gy[rim]
    dirichlet = (base.dirichlet.astype(bool) | rim)
    new_id = np.cumsum(~inside) - 1
    tri = new_id[tri].astype(np.int32)
    return Mesh(xy[~inside], tri, dirichlet[~inside].astype(np.uint8))


def wheel(rings: int, spokes: int, seed: int | None = None, jitter: float = 0.1) -> Mesh:
    """Polar P1 mesh of the unit disk: a centre node and ``rings`` rings of ``spokes`` nodes.

    The centre is a vertex of ``spokes`` triangles (the other nodes of at most six), so
    node degrees up to ``spokes`` appear; the outer ring is Dirichlet.  Interior ring
    nodes move radially by up to ``jitter`` of the ring spacing (the triangles stay CCW).
    """
    if rings < 1 or spokes < 3:
        raise ValueError("need a ring and three spokes")
    r = np.repeat(np.arange(1, rings + 1), spokes) / rings
    t = np.tile(np.arange(spokes), rings) * (2.0 * np.pi / spokes)
    if seed is not None and jitter != 0.0:
        rng = np.random.default_rng(seed)
        r = r + np.where(r < 1.0, jitter * rng.uniform(-1.0, 1.0, r.size) / rings, 0.0)
    xy = np.concatenate([[[0.0, 0.0]], np.stack([r * np.cos(t), r * np.sin(t)], axis=1)])
    node = lambda ring, j: 1 + ring * spokes + (j % spokes)
    tri = [(0, node(0, j), node(0, j + 1)) for j in range(spokes)]
    for ring in range(rings - 1):
        for j in range(spokes):
            a, b = node(ring, j), node(ring, j + 1)
            c, d = node(ring + 1, j + 1), node(ring + 1, j)
            tri += [(a, c, b), (a, d, c)]
    tri = np.array(tri, dtype=np.int32)
    e1 = xy[tri[:, 1]] - xy[tri[:, 0]]
    e2 = xy[tri[:, 2]] - xy[tri[:, 0]]
    assert np.all(e1[:, 0] * e2[:, 1] - e1[:, 1] * e2[:, 0] > 0.0), "wheel triangles must be CCW"
    dirichlet = np.zeros(xy.shape[0], dtype=np.uint8)
    dirichlet[1 + (rings - 1) * spokes:] = 1
    return Mesh(xy, tri, dirichlet)


def permuted(mesh: Mesh, seed: int) -> Mesh:
    """Same mesh with node ids, triangle order and each triangle's starting vertex shuffled (still CCW)."""
    rng = np.random.default_rng(seed)
    n = mesh.n_nodes
    perm = rng.permutation(n)          # new id of old node
    inv = np.empty(n, dtype=np.int64)
    inv[perm] = np.arange(n)
    xy = mesh.xy[inv]
    dirichlet = mesh.dirichlet[inv]
    tri = perm[mesh.tri][rng.permutation(mesh.n_tris)]
    rot = rng.integers(0, 3, size=tri.shape[0])
    rows = np.arange(tri.shape[0])[:, None]
    cols = (np.arange(3)[None, :] + rot[:, None]) % 3
    tri = tri[rows, cols]
    return Mesh(xy, tri.astype(np.int32), dirichlet)


def fourier_modes(seed: int, n_modes: int = 8, kmax: int = 4) -> dict:
    """Random Fourier mode set (wavevectors, amplitudes, phases, angular frequencies)."""
    rng = np.random.default_rng(seed)
    p = rng.integers(1, kmax + 1, size=n_modes)
    q = rng.integers(1, kmax + 1, size=n_modes)
    kx = np.pi * p
    ky = np.pi * q
    k2 = kx * kx + ky * ky
    c = rng.standard_normal(n_modes) / k2
    theta = rng.uniform(0.0, 2.0 * np.pi, size=n_modes)
    omega = rng.uniform(0.5, 2.0, size=n_modes)
    return {"kx": kx, "ky": ky, "c": c, "theta": theta, "omega": omega}


def _phase(xy: np.ndarray, modes: dict, t: float) -> np.ndarray:
    return (xy[:, 0:1] * modes["kx"][None, :] + xy[:, 1:2] * modes["ky"][None, :]
            + modes["theta"][None, :] + modes["omega"][None, :] * t)


def stream_velocity(xy: np.ndarray, modes: dict, t: float = 0.0) -> tuple[np.ndarray, np.ndarray]:
    """Divergence-free velocity ``(d psi/dy, -d psi/dx)`` of the Fourier stream function at points ``xy``."""
    s = np.sin(_phase(xy, modes, t))
    u = -(s * (modes["c"] * modes["ky"])[None, :]).sum(axis=1)
    v = (s * (modes["c"] * modes["kx"])[None, :]).sum(axis=1)
    return np.ascontiguousarray(u), np.ascontiguousarray(v)


def potential_velocity(xy: np.ndarray, modes: dict, t: float = 0.0) -> tuple[np.ndarray, np.ndarray]:
    """Curl-free velocity ``grad chi`` of a Fourier potential ``chi`` at points ``xy``."""
    s = np.sin(_phase(xy, modes, t))
    u = -(s * (modes["c"] * modes["kx"])[None, :]).sum(axis=1)
    v = -(s * (modes["c"] * modes["ky"])[None, :]).sum(axis=1)
    return np.ascontiguousarray(u), np.ascontiguousarray(v)


class FourierSequence:
    """Velocity fields of a drifting Fourier flow at fixed points, step after step.

    ``at(n)`` returns the stream-function velocity ``(u, v)`` and the velocity
    with an added gradient part ``(u + chi_x, v + chi_y)`` at time ``n * DT``
    (phases advance by ``omega_m * DT`` per step).  The sines of the mode phases
    are expanded once (sin(a + w t) = sin a cos w t + cos a sin w t), so a step
    costs two small matrix-vector products per field.
    """

    def __init__(self, xy: np.ndarray, modes: dict, chi_modes: dict):
        self.modes, self.chi = modes, chi_modes
        self._tabs = []
        for md in (modes, chi_modes):
            ph = _phase(xy, md, 0.0)
            self._tabs.append((np.sin(ph), np.cos(ph)))

    def _sin(self, which: int, t: float) -> np.ndarray:
        s, c = self._tabs[which]
        md = (self.modes, self.chi)[which]
        return s * np.cos(md["omega"] * t)[None, :] + c * np.sin(md["omega"] * t)[None, :]

    def at(self, n: int):
        t = n * DT
        s = self._sin(0, t)
        m = self.modes
        u = -(s @ (m["c"] * m["ky"]))
        v = s @ (m["c"] * m["kx"])
        s2 = self._sin(1, t)
        c2 = self.chi
        ut = u - s2 @ (c2["c"] * c2["kx"])
        vt = v - s2 @ (c2["c"] * c2["ky"])
        return u, v, ut, vt


class DeviceFourierSequence:
    """The flow of ``FourierSequence`` evaluated with torch on a device, for point sets too
    large to tabulate on the host (the 8.39M nodes of a twice-refined 1025 x 513 mesh).

    ``xy`` is an ``[n, 2]`` float64 tensor on the device; ``at(n)`` returns four device
    tensors ``(u, v, u + chi_x, v + chi_y)`` at time ``n * DT``, computed directly from the
    mode sums (sin of the full phase, not the host class's expansion, so values agree with
    ``FourierSequence`` to rounding, not bitwise).
    """

    def __init__(self, xy, modes: dict, chi_modes: dict):
        import torch
        self.xy = xy
        self.sets = []
        for md in (modes, chi_modes):
            t = {k: torch.tensor(np.asarray(v, dtype=np.float64), device=xy.device) for k, v in md.items()}
            self.sets.append(t)

    def _sin(self, which: int, t: float):
        md = self.sets[which]
        ph = (self.xy[:, 0:1] * md["kx"][None, :] + self.xy[:, 1:2] * md["ky"][None, :]
              + md["theta"][None, :] + md["omega"][None, :] * t)
        return ph.sin_()

    def at(self, n: int):
        t = n * DT
        s = self._sin(0, t)
        m = self.sets[0]
        # mode sums as row sums of broadcast products (a matrix-vector product with 8 columns
        # runs as a slow library reduction on the device)
        u = -(s * (m["c"] * m["ky"])[None, :]).sum(dim=1)
        v = (s * (m["c"] * m["kx"])[None, :]).sum(dim=1)
        del s
        s2 = self._sin(1, t)
        c2 = self.sets[1]
        ut = u - (s2 * (c2["c"] * c2["kx"])[None, :]).sum(dim=1)
        vt = v - (s2 * (c2["c"] * c2["ky"])[None, :]).sum(dim=1)
        return u.contiguous(), v.contiguous(), ut.contiguous(), vt.contiguous()


def stuart_numbers(count: int) -> np.ndarray:
    """Stuart numbers log-spaced over [0.1, 10]."""
    if count == 1:
        return np.array([1.0])
    return 10.0 ** (-1.0 + 2.0 * np.arange(count) / (count - 1))


def batch_sizes(count: int, seed: int, mmin: int = 32, mmax: int = 256) -> list[tuple[int, int]]:
    """Uneven coarse grids for a batched sweep: ``nx = 2m+1``, ``ny = m+1``, ``m ~ U{mmin..mmax}``."""
    rng = np.random.default_rng(seed)
    m = rng.integers(mmin, mmax + 1, size=count)
    return [(int(2 * mi + 1), int(mi + 1)) for mi in m]


class Channel(Mesh):
    """A cylinder-in-channel mesh: ``Mesh`` (``dirichlet`` = the box sides, the far field of
    the electric potential) plus the geometry and per-node boundary classes (``inflow``,
    ``outflow``, ``walls``, ``cylinder``, uint8)."""

    def __init__(self, xy, tri, geometry: dict):
        b = channel_boundary(xy, tri, geometry)
        super().__init__(xy, tri, (b["inflow"] | b["outflow"] | b["walls"]).astype(np.uint8))
        self.geometry = dict(geometry)
        self.inflow, self.outflow, self.walls, self.cylinder = b["inflow"], b["outflow"], b["walls"], b["cylinder"]


def channel_boundary(xy: np.ndarray, tri: np.ndarray, geometry: dict) -> dict:
    """Boundary classes of the nodes of a channel mesh (any level): a node is on the boundary
    when one of its edges belongs to one triangle; it is inflow (x = 0), outflow (x = L),
    wall (y = 0 or H) by position, and cylinder otherwise.  Also ``cyl_edges`` [m, 3]:
    (a, b, triangle) for every boundary edge with both ends on the cylinder."""
    xy = np.asarray(xy, dtype=np.float64)
    tri = np.asarray(tri, dtype=np.int64)
    n = xy.shape[0]
    e = np.concatenate([tri[:, [0, 1]], tri[:, [1, 2]], tri[:, [2, 0]]])
    owner = np.tile(np.arange(tri.shape[0]), 3)
    key = np.minimum(e[:, 0], e[:, 1]) * n + np.maximum(e[:, 0], e[:, 1])
    uniq, inv, cnt = np.unique(key, return_inverse=True, return_counts=True)
    bnd = cnt[inv] == 1
    on = np.zeros(n, dtype=bool)
    on[e[bnd].ravel()] = True
    L, H = geometry["L"], geometry["H"]
    tol = 1e-9 * max(L, H)
    x, y = xy[:, 0], xy[:, 1]
    inflow = on & (np.abs(x) <= tol)
    outflow = on & (np.abs(x - L) <= tol)
    walls = on & ((np.abs(y) <= tol) | (np.abs(y - H) <= tol))
    cyl = on & ~inflow & ~outflow & ~walls
    be = e[bnd]
    both = cyl[be[:, 0]] & cyl[be[:, 1]]
    cyl_edges = np.concatenate([be[both], owner[bnd][both][:, None]], axis=1).astype(np.int32)
    return {"inflow": inflow.astype(np.uint8), "outflow": outflow.astype(np.uint8),
            "walls": walls.astype(np.uint8), "cylinder": cyl.astype(np.uint8), "cyl_edges": cyl_edges}


def cylinder_channel(seed: int = 0, n_circle: int = 40, growth: float = 0.16, h_max: float = 1.6,
                     wake: float = 0.3, L: float = 38.0, H: float = 32.0, xc: float = 8.0, yc: float = 16.0,
                     d: float = 1.0) -> Channel:
    """Graded Delaunay mesh of the box [0, L] x [0, H] minus the disk of diameter d at (xc, yc)."""
    from scipy.spatial import Delaunay

    r0 = 0.5 * d
    h0 = 2.0 * np.pi * r0 / n_circle

    def size(x, y):
        dx = np.where(x > xc, (x - xc) * wake, x - xc)
        r = np.sqrt(dx * dx + (y - yc) ** 2)
        return np.minimum(h0 + growth * np.maximum(r - r0, 0.0), h_max)

    th = 2.0 * np.pi * np.arange(n_circle) / n_circle
    pts = [np.stack([xc + r0 * np.cos(th), yc + r0 * np.sin(th)], axis=1)]
    r, r_last = r0, r0
    r_stop = 0.5 * min(xc, L - xc, yc, H - yc)
    while True:
        r = r + 0.866 * min(h0 + growth * (r - r0), h_max)
        if r > r_stop:
            break
        n = max(int(round(2.0 * np.pi * r / min(h0 + growth * (r - r0), h_max))), 6)
        t = 2.0 * np.pi * (np.arange(n) + (0.5 if len(pts) % 2 else 0.0)) / n
        pts.append(np.stack([xc + r * np.cos(t), yc + r * np.sin(t)], axis=1))
        r_last = r

    def side(p0, p1):
        p0, p1 = np.asarray(p0, dtype=np.float64), np.asarray(p1, dtype=np.float64)
        ln = float(np.hypot(*(p1 - p0)))
        s = [0.0]
        while s[-1] < ln:
            q = p0 + (p1 - p0) * (s[-1] / ln)
            s.append(s[-1] + float(size(q[0:1], q[1:2])[0]))
        s = np.array(s[:-1]) * (ln / s[-1])
        return p0[None, :] + (p1 - p0)[None, :] * (s[:, None] / ln)

    pts.append(np.concatenate([side((0.0, 0.0), (L, 0.0)), side((L, 0.0), (L, H)),
                               side((L, H), (0.0, H)), side((0.0, H), (0.0, 0.0))]))
    fixed = np.concatenate(pts)
    allp = [tuple(p) for p in fixed]
    allh = list(size(fixed[:, 0], fixed[:, 1]))
    gc = 0.5
    grid: dict = {}
    for i, (px, py) in enumerate(allp):
        grid.setdefault((int(px / gc), int(py / gc)), []).append(i)
    rng = np.random.default_rng(seed)
    fails = 0
    while fails < 3000:
        qx, qy = rng.uniform(0.0, L), rng.uniform(0.0, H)
        hq = float(size(np.array([qx]), np.array([qy]))[0])
        if (np.hypot(qx - xc, qy - yc) < r_last + 0.6 * hq or qx < 0.6 * hq or qx > L - 0.6 * hq
                or qy < 0.6 * hq or qy > H - 0.6 * hq):
            fails += 1
            continue
        cx, cy = int(qx / gc), int(qy / gc)
        reach = int(np.ceil(hq / gc)) + 1
        ok = True
        for ix in range(cx - reach, cx + reach + 1):
            for iy in range(cy - reach, cy + reach + 1):
                for j in grid.get((ix, iy), ()):
                    lim = 0.8 * min(hq, allh[j])
                    if (allp[j][0] - qx) ** 2 + (allp[j][1] - qy) ** 2 < lim * lim:
                        ok = False
                        break
                if not ok:
                    break
            if not ok:
                break
        if not ok:
            fails += 1
            continue
        fails = 0
        grid.setdefault((cx, cy), []).append(len(allp))
        allp.append((qx, qy))
        allh.append(hq)
    xy = np.array(allp, dtype=np.float64)
    # node order along a Z curve of 2^10 x 2^10 cells (locality of the gathers)
    ix = np.minimum((xy[:, 0] / L * 1024).astype(np.int64), 1023)
    iy = np.minimum((xy[:, 1] / H * 1024).astype(np.int64), 1023)
    code = np.zeros(xy.shape[0], dtype=np.int64)
    for b in range(10):
        code |= ((ix >> b) & 1) << (2 * b) | ((iy >> b) & 1) << (2 * b + 1)
    order = np.argsort(code, kind="stable")
    xy = xy[order]
    tri = Delaunay(xy).simplices.astype(np.int64)
    c = xy[tri].mean(axis=1)
    tri = tri[np.hypot(c[:, 0] - xc, c[:, 1] - yc) > r0]
    e1 = xy[tri[:, 1]] - xy[tri[:, 0]]
    e2 = xy[tri[:, 2]] - xy[tri[:, 0]]
    cw = e1[:, 0] * e2[:, 1] - e1[:, 1] * e2[:, 0] < 0.0
    tri[cw] = tri[cw][:, [0, 2, 1]]
    geometry = {"L": L, "H": H, "xc": xc, "yc": yc, "d": d, "n_circle": n_circle}
    return Channel(xy, tri.astype(np.int32), geometry)
