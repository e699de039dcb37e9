"""Oracle: the coarse Poisson solution and the Krylov solvers that reach it.

* ``direct``     phi* = K^-1 b by a library factorisation (dense LAPACK Cholesky
                 for small systems, SuperLU otherwise): the plain definition of
                 the solve's result;
* ``pcg``        fp64 Jacobi-PCG (C, ``pcg_oracle.c``), stopping on the true
                 relative residual ||b - K phi|| / ||b||;
* ``pcg_mixed``  fp32 Jacobi-PCG with fp64 iterative refinement of the
                 residual ("reliable updates", C).
"""
from __future__ import annotations

import ctypes
import os

import numpy as np
import scipy.linalg
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from . import build as _build

STATUS = {0: "ok", 1: "noconv", 2: "breakdown"}

_lib = None


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_build.LIB) or os.path.getmtime(_build.LIB) < os.path.getmtime(_build.SRC):
            _build.build()
        lib = ctypes.CDLL(_build.LIB)
        dp = ctypes.POINTER(ctypes.c_double)
        ip = ctypes.POINTER(ctypes.c_int)
        lib.oracle_pcg_f64.argtypes = [ctypes.c_int, ip, ip, dp, dp, dp, dp, ctypes.c_double,
                                       ctypes.c_int, ip, dp]
        lib.oracle_pcg_f64.restype = ctypes.c_int
        lib.oracle_pcg_mixed.argtypes = [ctypes.c_int, ip, ip, dp, dp, dp, dp, ctypes.c_double,
                                         ctypes.c_double, ctypes.c_int, ip, ip, dp]
        lib.oracle_pcg_mixed.restype = ctypes.c_int
        lib.oracle_spmv_f64.argtypes = [ctypes.c_int, ip, ip, dp, dp, dp]
        lib.oracle_spmv_f64.restype = None
        lib.oracle_threads.argtypes = []
        lib.oracle_threads.restype = ctypes.c_int
        _lib = lib
    return _lib


def _csr_arrays(a: sp.csr_matrix):
    rowptr = np.ascontiguousarray(a.indptr, dtype=np.int32)
    col = np.ascontiguousarray(a.indices, dtype=np.int32)
    val = np.ascontiguousarray(a.data, dtype=np.float64)
    return rowptr, col, val


def _p(arr, ctype):
    return arr.ctypes.data_as(ctypes.POINTER(ctype))


def direct(a: sp.csr_matrix, b: np.ndarray) -> np.ndarray:
    """phi* = K^-1 b (dense Cholesky up to 2000 unknowns, SuperLU above)."""
    n = a.shape[0]
    if n <= 2000:
        c = scipy.linalg.cho_factor(a.toarray())
        return scipy.linalg.cho_solve(c, b)
    return spla.splu(a.tocsc()).solve(np.asarray(b, dtype=np.float64))


def relative_residual(a: sp.csr_matrix, b: np.ndarray, x: np.ndarray) -> float:
    bn = np.linalg.norm(b)
    return float(np.linalg.norm(b - a @ x) / bn) if bn > 0 else 0.0


def pcg(a: sp.csr_matrix, b: np.ndarray, x0: np.ndarray | None = None, tol: float = 1e-8,
        max_iter: int = 100000):
    """fp64 Jacobi-PCG. Returns ``(x, info)`` with info = {status, iters, rel_res}."""
    lib = _load()
    rowptr, col, val = _csr_arrays(a)
    n = a.shape[0]
    dinv = np.ascontiguousarray(1.0 / a.diagonal())
    b = np.ascontiguousarray(b, dtype=np.float64)
    x = np.zeros(n) if x0 is None else np.array(x0, dtype=np.float64, copy=True)
    it = ctypes.c_int(0)
    rel = ctypes.c_double(0.0)
    st = lib.oracle_pcg_f64(n, _p(rowptr, ctypes.c_int), _p(col, ctypes.c_int), _p(val, ctypes.c_double),
                            _p(dinv, ctypes.c_double), _p(b, ctypes.c_double), _p(x, ctypes.c_double),
                            tol, max_iter, ctypes.byref(it), ctypes.byref(rel))
    return x, {"status": STATUS[st], "iters": it.value, "rel_res": rel.value}


def pcg_mixed(a: sp.csr_matrix, b: np.ndarray, x0: np.ndarray | None = None, tol: float = 1e-8,
              delta: float = 0.1, max_iter: int = 100000):
    """fp32 Jacobi-PCG refined by fp64 true residuals. Returns ``(x, info)``."""
    lib = _load()
    rowptr, col, val = _csr_arrays(a)
    n = a.shape[0]
    dinv = np.ascontiguousarray(1.0 / a.diagonal())
    b = np.ascontiguousarray(b, dtype=np.float64)
    x = np.zeros(n) if x0 is None else np.array(x0, dtype=np.float64, copy=True)
    it = ctypes.c_int(0)
    upd = ctypes.c_int(0)
    rel = ctypes.c_double(0.0)
    st = lib.oracle_pcg_mixed(n, _p(rowptr, ctypes.c_int), _p(col, ctypes.c_int), _p(val, ctypes.c_double),
                              _p(dinv, ctypes.c_double), _p(b, ctypes.c_double), _p(x, ctypes.c_double),
                              tol, delta, max_iter, ctypes.byref(it), ctypes.byref(upd), ctypes.byref(rel))
    return x, {"status": STATUS[st], "iters": it.value, "updates": upd.value, "rel_res": rel.value}


def threads() -> int:
    """OpenMP threads the C solvers run with."""
    return int(_load().oracle_threads())


def spmv(a: sp.csr_matrix, x: np.ndarray) -> np.ndarray:
    """y = K x through the C kernel (used to time the oracle's building block)."""
    lib = _load()
    rowptr, col, val = _csr_arrays(a)
    x = np.ascontiguousarray(x, dtype=np.float64)
    y = np.empty(a.shape[0])
    lib.oracle_spmv_f64(a.shape[0], _p(rowptr, ctypes.c_int), _p(col, ctypes.c_int),
                        _p(val, ctypes.c_double), _p(x, ctypes.c_double), _p(y, ctypes.c_double))
    return y
