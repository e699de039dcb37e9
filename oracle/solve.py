"""Oracle: the coarse Poisson solution and the Krylov solvers that reach it.

* ``direct``     phi* = K^-1 b by a library factorisation (dense LAPACK Cholesky
                 for small systems, SuperLU otherwise): the plain definition of
                 the solve's result;
* ``pcg``        fp64 PCG (C, ``pcg_oracle.c``), stopping on the true
                 relative residual ||b - K phi|| / ||b||;
* ``pcg_mixed``  fp32 PCG with fp64 iterative refinement of the residual
                 ("reliable updates", C).

Both take ``degree``: 0 or 1 for the Jacobi preconditioner D^-1, d >= 2 for the
Chebyshev polynomial preconditioner of degree d in D^-1 K on the interval
[hi / CHEB_RATIO, hi] with hi = ``gershgorin_bound(K)`` (``cheb_apply``).
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

# lower end of the Chebyshev interval as a fraction of its upper end
CHEB_RATIO = 1000.0

_lib = None


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_build.LIB) or os.path.getmtime(_build.LIB) < os.path.getmtime(_build.SRC):
            _build.build()
        lib = ctypes.CDLL(_build.LIB)
        dp = ctypes.POINTER(ctypes.c_double)
        ip = ctypes.POINTER(ctypes.c_int)
        ci, cd = ctypes.c_int, ctypes.c_double
        lib.oracle_pcg_f64.argtypes = [ci, ip, ip, dp, dp, ci, cd, cd, dp, dp, cd, ci, ip, dp]
        lib.oracle_pcg_f64.restype = ctypes.c_int
        lib.oracle_pcg_mixed.argtypes = [ci, ip, ip, dp, dp, ci, cd, cd, dp, dp, cd, cd, ci, ip, ip, dp]
        lib.oracle_pcg_mixed.restype = ctypes.c_int
        lib.oracle_cheb_apply_f64.argtypes = [ci, ip, ip, dp, dp, ci, cd, cd, dp, dp]
        lib.oracle_cheb_apply_f64.restype = None
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


def gershgorin_bound(a: sp.csr_matrix) -> float:
    """max_i sum_j |K_ij| / K_ii: an upper bound of the spectrum of D^-1 K (Gershgorin's theorem)."""
    a = sp.csr_matrix(a)
    rows = np.asarray(abs(a).sum(axis=1)).ravel()
    return float(np.max(rows / a.diagonal()))


def _interval(a, degree):
    if degree <= 1:
        return 0.0, 0.0
    hi = gershgorin_bound(a)
    return hi / CHEB_RATIO, hi


def cheb_apply(a: sp.csr_matrix, r: np.ndarray, degree: int, lo: float | None = None,
               hi: float | None = None) -> np.ndarray:
    """z = M^-1 r for the preconditioner of ``degree`` (Jacobi for degree <= 1)."""
    lib = _load()
    rowptr, col, val = _csr_arrays(a)
    n = a.shape[0]
    dinv = np.ascontiguousarray(1.0 / a.diagonal())
    if lo is None or hi is None:
        lo, hi = _interval(a, degree)
    r = np.ascontiguousarray(r, dtype=np.float64)
    z = np.empty(n)
    lib.oracle_cheb_apply_f64(n, _p(rowptr, ctypes.c_int), _p(col, ctypes.c_int), _p(val, ctypes.c_double),
                              _p(dinv, ctypes.c_double), int(degree), lo, hi, _p(r, ctypes.c_double),
                              _p(z, ctypes.c_double))
    return z


def pcg(a: sp.csr_matrix, b: np.ndarray, x0: np.ndarray | None = None, tol: float = 1e-8,
        max_iter: int = 100000, degree: int = 0):
    """fp64 PCG. Returns ``(x, info)`` with info = {status, iters, rel_res}."""
    lib = _load()
    rowptr, col, val = _csr_arrays(a)
    n = a.shape[0]
    dinv = np.ascontiguousarray(1.0 / a.diagonal())
    lo, hi = _interval(a, degree)
    b = np.ascontiguousarray(b, dtype=np.float64)
    x = np.zeros(n) if x0 is None else np.array(x0, dtype=np.float64, copy=True)
    it = ctypes.c_int(0)
    rel = ctypes.c_double(0.0)
    st = lib.oracle_pcg_f64(n, _p(rowptr, ctypes.c_int), _p(col, ctypes.c_int), _p(val, ctypes.c_double),
                            _p(dinv, ctypes.c_double), int(degree), lo, hi, _p(b, ctypes.c_double),
                            _p(x, ctypes.c_double), tol, max_iter, ctypes.byref(it), ctypes.byref(rel))
    return x, {"status": STATUS[st], "iters": it.value, "rel_res": rel.value}


def pcg_mixed(a: sp.csr_matrix, b: np.ndarray, x0: np.ndarray | None = None, tol: float = 1e-8,
              delta: float = 0.1, max_iter: int = 100000, degree: int = 0):
    """fp32 PCG refined by fp64 true residuals. Returns ``(x, info)``."""
    lib = _load()
    rowptr, col, val = _csr_arrays(a)
    n = a.shape[0]
    dinv = np.ascontiguousarray(1.0 / a.diagonal())
    lo, hi = _interval(a, degree)
    b = np.ascontiguousarray(b, dtype=np.float64)
    x = np.zeros(n) if x0 is None else np.array(x0, dtype=np.float64, copy=True)
    it = ctypes.c_int(0)
    upd = ctypes.c_int(0)
    rel = ctypes.c_double(0.0)
    st = lib.oracle_pcg_mixed(n, _p(rowptr, ctypes.c_int), _p(col, ctypes.c_int), _p(val, ctypes.c_double),
                              _p(dinv, ctypes.c_double), int(degree), lo, hi, _p(b, ctypes.c_double),
                              _p(x, ctypes.c_double), tol, delta, max_iter, ctypes.byref(it),
                              ctypes.byref(upd), ctypes.byref(rel))
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
