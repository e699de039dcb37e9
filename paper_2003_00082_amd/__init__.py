"""Python binding of ``libcgp.so`` (the C ABI of ``include/cgp.h``).

Argument marshalling only: every step of the CGP hot path runs in the HIP
kernels of the library.  PyTorch provides device memory (tensors) and the
stream (``torch.cuda.current_stream()``).  If the library is not built the
import of any entry point raises -- there is no fallback path.

Function names follow the C ABI (``cgp_restrict``, ``cgp_poisson_solve`` ...);
``Context`` bundles a context handle with its stream for convenience.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libcgp.so")

# status codes (include/cgp.h)
CGP_OK = 0
CGP_E_INVALID = -1
CGP_E_NOMEM = -2
CGP_E_HIP = -3
CGP_E_MESH = -4
CGP_E_NOCONV = -5
CGP_E_BREAKDOWN = -6
CGP_E_UNSUPPORTED = -7
CGP_E_ABORTED = -8
CGP_SRC_CURL = 0
CGP_SRC_DIV = 1
CGP_FP64 = 0
CGP_FP32_IR = 1
CGP_GUESS_ZERO = 0
CGP_GUESS_GIVEN = 1
CGP_GUESS_EXTRAP = 2
CGP_GUESS_LEARNED = 3
CGP_ENGINE_AUTO = 0
CGP_ENGINE_STAGED = 1
CGP_ENGINE_PERSISTENT = 2
CGP_ENGINE_STAGED_ROWS = 3
CGP_DEGREE_TUNED = -1
AUTOTUNE_CANDIDATES = 8
SOLVE_STATUS = {0: "ok", 1: "noconv", 2: "breakdown", 3: "aborted"}


class CGPError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"cgp error {code}: {msg}")
        self.code = code


class SolveOpts(ctypes.Structure):
    _fields_ = [("precision", ctypes.c_int32), ("guess", ctypes.c_int32), ("tol", ctypes.c_double),
                ("refine_delta", ctypes.c_double), ("max_iter", ctypes.c_int32), ("model", ctypes.c_int32),
                ("spmv_lanes", ctypes.c_int32), ("blocks", ctypes.c_int32), ("engine", ctypes.c_int32),
                ("launches_per_graph", ctypes.c_int32), ("precond_degree", ctypes.c_int32),
                ("deflation", ctypes.c_int32), ("stage_budget", ctypes.c_int32)]


class SolveStats(ctypes.Structure):
    _fields_ = [("iters", ctypes.c_int32), ("refinements", ctypes.c_int32), ("status", ctypes.c_int32),
                ("guess_used", ctypes.c_int32), ("rel_res", ctypes.c_double), ("rel_res_guess", ctypes.c_double)]


class MomentumStats(ctypes.Structure):
    _fields_ = [("iters", ctypes.c_int32 * 2), ("status", ctypes.c_int32 * 2), ("rel_res", ctypes.c_double * 2)]


STATS_BYTES = ctypes.sizeof(SolveStats)   # 32
_lib = None

_vp = ctypes.c_void_p
_i32 = ctypes.c_int32
_i64 = ctypes.c_int64
_f64 = ctypes.c_double

_SIGS = {
    "cgp_create": ([ctypes.POINTER(_vp), _i32, _vp], _i32),
    "cgp_destroy": ([_vp], _i32),
    "cgp_set_stream": ([_vp, _vp], _i32),
    "cgp_sync": ([_vp], _i32),
    "cgp_last_error": ([_vp], ctypes.c_char_p),
    "cgp_device_cus": ([_vp], _i32),
    "cgp_stage_launches": ([_vp], _i64),
    "cgp_stage_timing": ([_vp, _i32], _i32),
    "cgp_stage_timing_read": ([_vp, ctypes.POINTER(_i64), ctypes.POINTER(_f64), ctypes.POINTER(_i64),
                               ctypes.POINTER(_f64)], _i32),
    "cgp_mesh_upload": ([_vp, _vp, _i64, _vp, _i64, _vp, _i32, ctypes.POINTER(_i32)], _i32),
    "cgp_mesh_info": ([_vp, _i32, _i32, ctypes.POINTER(_i64), ctypes.POINTER(_i64), ctypes.POINTER(_i64),
                       ctypes.POINTER(_i64)], _i32),
    "cgp_mesh_levels": ([_vp, _i32, ctypes.POINTER(_i32)], _i32),
    "cgp_mesh_download": ([_vp, _i32, _i32, _vp, _vp, _vp, _vp], _i32),
    "cgp_mesh_matrix": ([_vp, _i32, _vp, _vp, _vp, _vp], _i32),
    "cgp_mesh_free": ([_vp, _i32], _i32),
    "cgp_restrict": ([_vp, _i32, _vp, _vp, _i32, _f64, _vp, _vp, _vp], _i32),
    "cgp_poisson_solve": ([_vp, _i32, _vp, _vp, _vp, _vp, _vp, ctypes.POINTER(SolveOpts), _vp], _i32),
    "cgp_solve_check": ([_vp, _i32, _vp, _vp], _i32),
    "cgp_poisson_solve_noalloc": ([_vp, _i32, _vp, _vp, _vp, _vp, ctypes.POINTER(SolveOpts), _vp], _i32),
    "cgp_autotune": ([_vp, _i32, _vp, _i32, _i32, _vp, _vp, _vp], _i32),
    "cgp_prolong": ([_vp, _i32, _vp, _vp], _i32),
    "cgp_lorentz_force": ([_vp, _i32, _vp, _vp, _vp, _f64, _f64, _vp, _vp, _vp], _i32),
    "cgp_velocity_correct": ([_vp, _i32, _vp, _vp, _vp, _vp, _f64, _vp, _vp], _i32),
    "cgp_surface_force": ([_vp, _i32, _i32, _i64, _vp, _vp, _vp, _vp, _f64, _vp], _i32),
    "cgp_momentum_step": ([_vp, _i32, _vp, _vp, _vp, _vp, _vp, _f64, _f64, _f64, _f64, _i32, _vp, _vp, _vp],
                          _i32),
    "cgp_interpolate": ([_vp, _i32, _i32, _i64, _vp, _vp, _vp, _vp], _i32),
    "cgp_model_param_count": ([], _i64),
    "cgp_model_create": ([_vp, _i32, _i32, ctypes.c_uint64, ctypes.POINTER(_i32)], _i32),
    "cgp_model_free": ([_vp, _i32], _i32),
    "cgp_model_get_params": ([_vp, _i32, _vp], _i32),
    "cgp_model_set_params": ([_vp, _i32, _vp], _i32),
    "cgp_model_predict": ([_vp, _i32, _i32, _vp, _vp, _vp, _vp], _i32),
    "cgp_model_grad": ([_vp, _i32, _i32, _vp, _vp, _vp, _vp, _vp, _vp], _i32),
    "cgp_model_train": ([_vp, _i32, _i32, _i32, _vp, _vp, _vp, _vp, _i32, _f64, ctypes.c_uint64, _vp], _i32),
    "cgp_model_save": ([_vp, _i32, ctypes.c_char_p], _i32),
    "cgp_model_load": ([_vp, ctypes.c_char_p, ctypes.POINTER(_i32)], _i32),
    "cgp_graph_begin": ([_vp], _i32),
    "cgp_graph_end": ([_vp, ctypes.POINTER(_i32)], _i32),
    "cgp_graph_launch": ([_vp, _i32], _i32),
    "cgp_graph_free": ([_vp, _i32], _i32),
}


def exported_symbols() -> list[str]:
    return sorted(_SIGS)


def load(path: str | None = None):
    """Load the built library (raises if it is missing: there is no fallback)."""
    global _lib
    if _lib is None:
        p = path or LIB_PATH
        if not os.path.exists(p):
            raise ImportError(f"{p} is not built; run __graft_entry__.build() "
                              "(python -c 'import __graft_entry__ as g; g.build()')")
        lib = ctypes.CDLL(p)
        for name, (args, res) in _SIGS.items():
            fn = getattr(lib, name)
            fn.argtypes = args
            fn.restype = res
        _lib = lib
    return _lib


def _check(rc: int):
    if rc != CGP_OK:
        raise CGPError(rc, load().cgp_last_error(None).decode())


def _ptr(t) -> int | None:
    """Device pointer of a torch tensor (None passes through)."""
    if t is None:
        return None
    if not t.is_cuda or not t.is_contiguous():
        raise ValueError("expected a contiguous device tensor")
    return t.data_ptr()


def _np(a, dtype):
    return np.ascontiguousarray(a, dtype=dtype)


class Context:
    """A library context bound to one device and (by default) torch's current stream."""

    def __init__(self, device: int = 0, stream=None):
        import torch
        lib = load()
        self.device = device
        if stream is None:
            stream = torch.cuda.current_stream(device)
        self.stream = stream
        h = _vp()
        _check(lib.cgp_create(ctypes.byref(h), device, _vp(stream.cuda_stream)))
        self.handle = h

    def close(self):
        if getattr(self, "handle", None):
            _check(load().cgp_destroy(self.handle))
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def sync(self):
        _check(load().cgp_sync(self.handle))

    @property
    def cus(self) -> int:
        return int(load().cgp_device_cus(self.handle))

    @property
    def stage_launches(self) -> int:
        return int(load().cgp_stage_launches(self.handle))

    def stage_timing(self, enable: bool):
        """Enable (resetting the totals) or disable the per-kernel timing of the staged solver."""
        _check(load().cgp_stage_timing(self.handle, 1 if enable else 0))

    def stage_timing_read(self) -> dict:
        nl, us, ncl, cus = _i64(), _f64(), _i64(), _f64()
        _check(load().cgp_stage_timing_read(self.handle, ctypes.byref(nl), ctypes.byref(us), ctypes.byref(ncl),
                                            ctypes.byref(cus)))
        return {"stage_launches": nl.value, "stage_us": us.value, "coarse_launches": ncl.value,
                "coarse_us": cus.value}

    # ---------------------------------------------------------------- meshes
    def mesh_upload(self, xy, tri, dirichlet, k_levels: int) -> int:
        xy = _np(xy, np.float64)
        tri = _np(tri, np.int32)
        d = _np(dirichlet, np.uint8)
        out = _i32()
        _check(load().cgp_mesh_upload(self.handle, xy.ctypes.data, xy.shape[0], tri.ctypes.data, tri.shape[0],
                                      d.ctypes.data, k_levels, ctypes.byref(out)))
        return int(out.value)

    def mesh_info(self, mesh: int, level: int) -> dict:
        n, t, e, nnz = _i64(), _i64(), _i64(), _i64()
        _check(load().cgp_mesh_info(self.handle, mesh, level, ctypes.byref(n), ctypes.byref(t), ctypes.byref(e),
                                    ctypes.byref(nnz)))
        return {"n_nodes": n.value, "n_tris": t.value, "n_edges": e.value, "nnz": nnz.value}

    def mesh_levels(self, mesh: int) -> int:
        k = _i32()
        _check(load().cgp_mesh_levels(self.handle, mesh, ctypes.byref(k)))
        return int(k.value)

    def mesh_download(self, mesh: int, level: int):
        info = self.mesh_info(mesh, level)
        xy = np.empty((info["n_nodes"], 2))
        tri = np.empty((info["n_tris"], 3), dtype=np.int32)
        d = np.empty(info["n_nodes"], dtype=np.uint8)
        ends = np.empty((max(info["n_edges"], 0), 2), dtype=np.int32)
        _check(load().cgp_mesh_download(self.handle, mesh, level, xy.ctypes.data, tri.ctypes.data, d.ctypes.data,
                                        ends.ctypes.data if info["n_edges"] > 0 else None))
        return xy, tri, d, ends

    def mesh_matrix(self, mesh: int):
        info = self.mesh_info(mesh, 0)
        n, nnz = info["n_nodes"], info["nnz"]
        rowptr = np.empty(n + 1, dtype=np.int32)
        col = np.empty(nnz, dtype=np.int32)
        val = np.empty(nnz)
        dinv = np.empty(n)
        _check(load().cgp_mesh_matrix(self.handle, mesh, rowptr.ctypes.data, col.ctypes.data, val.ctypes.data,
                                      dinv.ctypes.data))
        return rowptr, col, val, dinv

    def mesh_free(self, mesh: int):
        _check(load().cgp_mesh_free(self.handle, mesh))

    # ---------------------------------------------------------------- CGP steps
    def restrict(self, mesh: int, uf, vf, kind: int, scale: float, b, uc=None, vc=None):
        _check(load().cgp_restrict(self.handle, mesh, _ptr(uf), _ptr(vf), kind, float(scale), _ptr(b), _ptr(uc),
                                   _ptr(vc)))

    def prolong(self, mesh: int, qc, qf):
        _check(load().cgp_prolong(self.handle, mesh, _ptr(qc), _ptr(qf)))

    def lorentz_force(self, mesh: int, phif, uf, vf, sigma: float, b0: float, fx, fy, grad_elem=None):
        _check(load().cgp_lorentz_force(self.handle, mesh, _ptr(phif), _ptr(uf), _ptr(vf), float(sigma), float(b0),
                                        _ptr(fx), _ptr(fy), _ptr(grad_elem)))

    def velocity_correct(self, mesh: int, pf, ut, vt, scale: float, u, v, mask=None):
        _check(load().cgp_velocity_correct(self.handle, mesh, _ptr(pf), _ptr(ut), _ptr(vt), _ptr(mask), float(scale),
                                           _ptr(u), _ptr(v)))

    def surface_force(self, mesh: int, level: int, edges, p, u, v, mu: float, out):
        """Pressure and viscous force on a body over its boundary edges (``edges``: [m, 3] int32
        device tensor of a, b, t); ``out`` (5 fp64 on the device) receives F_p, F_v and the
        number of edges skipped."""
        _check(load().cgp_surface_force(self.handle, mesh, int(level), int(edges.shape[0]), _ptr(edges), _ptr(p),
                                        _ptr(u), _ptr(v), float(mu), _ptr(out)))

    def interpolate(self, mesh: int, level: int, pts, field, out, tri=None):
        """``field`` of ``level`` at the points ``pts`` ([n, 2] fp64 device tensor) into ``out``
        (NaN outside the mesh); ``tri`` (optional int32 tensor) receives the containing triangles."""
        _check(load().cgp_interpolate(self.handle, mesh, int(level), int(out.numel()), _ptr(pts), _ptr(field),
                                      _ptr(out), _ptr(tri) if tri is not None else None))

    def momentum_step(self, mesh: int, un, vn, fx, fy, rho: float, mu: float, dt: float, ut, vt, *,
                      tol: float = 1e-10, max_iter: int = 500, mask=None):
        """The momentum step of Eqs. 13-14 on the finest level; ``ut``/``vt`` carry the initial
        guess and the boundary values in, the intermediate velocity out.  Returns the per-component
        statistics (iterations, status, relative residual); synchronises the stream."""
        st = MomentumStats()
        _check(load().cgp_momentum_step(self.handle, mesh, _ptr(un), _ptr(vn), _ptr(fx), _ptr(fy), _ptr(mask), float(rho),
                                        float(mu), float(dt), float(tol), int(max_iter), _ptr(ut), _ptr(vt),
                                        ctypes.byref(st)))
        return {"iters": list(st.iters), "status": list(st.status), "rel_res": list(st.rel_res)}

    def poisson_solve(self, meshes, b, phi, stats, *, prev1=None, prev2=None, precision=CGP_FP64,
                      guess=CGP_GUESS_GIVEN, tol=1e-8, refine_delta=0.0, max_iter=0, model=-1, spmv_lanes=0,
                      blocks=0, engine=CGP_ENGINE_AUTO, launches_per_graph=0, precond_degree=0, deflation=0,
                      stage_budget=0):
        """Enqueue one (batched) solve.  ``meshes``/``b``/``phi``/``prev*`` are sequences (one per
        instance); ``stats`` is a device uint8 tensor of n_inst * 32 bytes."""
        k = len(meshes)
        arr_m = (_i32 * k)(*meshes)
        arr_b = (_vp * k)(*[_ptr(t) for t in b])
        arr_x = (_vp * k)(*[_ptr(t) for t in phi])
        arr_p1 = (_vp * k)(*[_ptr(t) for t in prev1]) if prev1 is not None else None
        arr_p2 = (_vp * k)(*[_ptr(t) for t in prev2]) if prev2 is not None else None
        opts = SolveOpts(precision, guess, tol, refine_delta, max_iter, model, spmv_lanes, blocks, engine,
                         launches_per_graph, precond_degree, deflation, stage_budget)
        _check(load().cgp_poisson_solve(self.handle, k, arr_m, arr_b, arr_x, arr_p1, arr_p2, ctypes.byref(opts),
                                        _ptr(stats)))

    def poisson_solve_noalloc(self, mesh: int, b, phi, stats, *, prev1=None, prev2=None, precision=CGP_FP64,
                              guess=CGP_GUESS_GIVEN, tol=1e-8, refine_delta=0.0, max_iter=0, spmv_lanes=0,
                              engine=CGP_ENGINE_AUTO, launches_per_graph=0, precond_degree=0, deflation=0):
        """One solve that allocates no device memory (the library's fixed scratch array);
        ``stats`` is a device uint8 tensor of 32 bytes."""
        opts = SolveOpts(precision, guess, tol, refine_delta, max_iter, -1, spmv_lanes, 0, engine,
                         launches_per_graph, precond_degree, deflation, 0)
        _check(load().cgp_poisson_solve_noalloc(self.handle, mesh, _ptr(b), _ptr(phi), _ptr(prev1), _ptr(prev2),
                                                ctypes.byref(opts), _ptr(stats)))

    def solve_check(self, n_inst: int, stats, raise_on_failure: bool = False) -> list[dict]:
        host = (SolveStats * n_inst)()
        rc = load().cgp_solve_check(self.handle, n_inst, _ptr(stats), ctypes.byref(host))
        if rc not in (CGP_OK, CGP_E_NOCONV, CGP_E_BREAKDOWN, CGP_E_ABORTED) or (rc != CGP_OK and raise_on_failure):
            _check(rc)
        return [{"iters": s.iters, "refinements": s.refinements, "status": SOLVE_STATUS.get(s.status, "?"),
                 "guess_used": s.guess_used, "rel_res": s.rel_res, "rel_res_guess": s.rel_res_guess}
                for s in host]

    def autotune(self, meshes, precision: int, deflation: int = 1):
        """Preconditioner degrees for a batch chosen by timing: (degree per mesh, the batch's
        time at each candidate degree 1..8 in ms [8], iterations per mesh and candidate [k, 8];
        -1 where a candidate could not solve)."""
        k = len(meshes)
        arr_m = (_i32 * k)(*meshes)
        out = (_i32 * k)()
        ms = np.empty(AUTOTUNE_CANDIDATES, dtype=np.float64)
        its = np.empty((k, AUTOTUNE_CANDIDATES), dtype=np.int32)
        _check(load().cgp_autotune(self.handle, k, arr_m, precision, deflation, out, ms.ctypes.data, its.ctypes.data))
        return list(out), ms, its

    # ---------------------------------------------------------------- learned guess
    @staticmethod
    def model_param_count() -> int:
        return int(load().cgp_model_param_count())

    def model_create(self, seed: int = 0, hidden: int = 64, layers: int = 3) -> int:
        out = _i32()
        _check(load().cgp_model_create(self.handle, int(hidden), int(layers), int(seed), ctypes.byref(out)))
        return int(out.value)

    def model_free(self, model: int):
        _check(load().cgp_model_free(self.handle, model))

    def model_get_params(self, model: int) -> np.ndarray:
        h = np.empty(self.model_param_count(), dtype=np.float32)
        _check(load().cgp_model_get_params(self.handle, model, h.ctypes.data))
        return h

    def model_set_params(self, model: int, params):
        h = _np(params, np.float32)
        if h.size != self.model_param_count():
            raise ValueError(f"expected {self.model_param_count()} parameters, got {h.size}")
        _check(load().cgp_model_set_params(self.handle, model, h.ctypes.data))

    def model_predict(self, model: int, mesh: int, b, prev1, prev2, guess):
        _check(load().cgp_model_predict(self.handle, model, mesh, _ptr(b), _ptr(prev1), _ptr(prev2), _ptr(guess)))

    def model_grad(self, model: int, mesh: int, b, prev1, prev2, target):
        """(loss, gradient as float32 numpy array) for one sample."""
        loss = _f64()
        g = np.empty(self.model_param_count(), dtype=np.float32)
        _check(load().cgp_model_grad(self.handle, model, mesh, _ptr(b), _ptr(prev1), _ptr(prev2), _ptr(target),
                                     ctypes.byref(loss), g.ctypes.data))
        return float(loss.value), g

    def model_train(self, model: int, mesh: int, b, prev1, prev2, target, *, epochs: int, lr: float,
                    seed: int = 0) -> np.ndarray:
        """Train on the samples (sequences of device tensors); returns the mean loss per epoch."""
        k = len(b)
        if not (len(prev1) == len(prev2) == len(target) == k):
            raise ValueError("sample sequences differ in length")
        arrs = [(_vp * k)(*[_ptr(t) for t in seq]) for seq in (b, prev1, prev2, target)]
        hist = np.empty(int(epochs), dtype=np.float64)
        _check(load().cgp_model_train(self.handle, model, mesh, k, *arrs, int(epochs), float(lr), int(seed),
                                      hist.ctypes.data))
        return hist

    def model_save(self, model: int, path: str):
        _check(load().cgp_model_save(self.handle, model, os.fsencode(path)))

    def model_load(self, path: str) -> int:
        out = _i32()
        _check(load().cgp_model_load(self.handle, os.fsencode(path), ctypes.byref(out)))
        return int(out.value)

    # ---------------------------------------------------------------- graphs
    def graph_begin(self):
        _check(load().cgp_graph_begin(self.handle))

    def graph_end(self) -> int:
        g = _i32()
        _check(load().cgp_graph_end(self.handle, ctypes.byref(g)))
        return int(g.value)

    def graph_launch(self, g: int):
        _check(load().cgp_graph_launch(self.handle, g))

    def graph_free(self, g: int):
        _check(load().cgp_graph_free(self.handle, g))


def stats_buffer(n_inst: int, device: int = 0):
    """Device buffer for n_inst cgp_solve_stats records."""
    import torch
    return torch.zeros(n_inst * STATS_BYTES, dtype=torch.uint8, device=f"cuda:{device}")
