"""CPU oracle for the predict-and-recompute CG variants (test infrastructure only).

Only the test suite, the smoke check and the CPU-baseline leg of the
benchmark import this package.  The solver library never loads it, and it
imports nothing from the solver package: it takes plain NumPy arrays.

The arithmetic lives in ``prcg_oracle.c`` (plain FP64 C, every operation
rounded separately, deterministic chunked inner products, optional OpenMP
over rows and chunks that does not change any result).  This module only
compiles it with gcc and marshals arguments through ctypes.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
import threading

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "prcg_oracle.c")
_LIB_PATH = os.path.join(_HERE, "_build", "liboracle.so")
_LOCK = threading.Lock()
_LIB = None

VARIANTS = {
    "hs": 0,
    "pr": 1,
    "pipe_pr": 2,
    "m": 3,
    "pipe_m": 4,
    "gv": 5,
    "pr_norecompute": 6,
    "pipe_pr_nowrecompute": 7,
    "cg": 8,
    "pr_unsimplified": 9,
}
STATUS = {0: "ok", 1: "not_converged", 2: "breakdown", -1: "einval", -2: "enomem"}

_DBL = ctypes.POINTER(ctypes.c_double)
_I32 = ctypes.POINTER(ctypes.c_int32)


class _Diag(ctypes.Structure):
    _fields_ = [(name, _DBL) for name in
                ("nu", "nup", "rr", "mu", "alpha", "beta", "true_res", "err_a", "orth", "gap", "xstar")]


def _compile(src: str, out: str) -> str:
    tmp = out + f".tmp{os.getpid()}"
    cmd = ["gcc", "-O2", "-std=c11", "-ffp-contract=off", "-fno-fast-math", "-fopenmp", "-fPIC",
           "-shared", "-Wall", "-o", tmp, src, "-lm"]
    subprocess.run(cmd, check=True)
    os.replace(tmp, out)
    return out


def build(force: bool = False) -> str:
    """Compile the oracle with gcc (-O2, no contraction, no fast math, OpenMP)."""
    os.makedirs(os.path.dirname(_LIB_PATH), exist_ok=True)
    if force or not os.path.exists(_LIB_PATH) or os.path.getmtime(_LIB_PATH) < os.path.getmtime(_SRC):
        _compile(_SRC, _LIB_PATH)
    return _LIB_PATH


def load_library(path: str):
    """Load an oracle build (the default one, or a test's deliberately mutated copy)."""
    lib = ctypes.CDLL(path)
    lib.orc_solve.restype = ctypes.c_int
    lib.orc_solve.argtypes = [ctypes.c_int, ctypes.c_int64, _I32, _I32, _DBL, _DBL, _DBL, _DBL,
                              ctypes.c_double, ctypes.c_int32, _I32, _DBL, ctypes.POINTER(_Diag)]
    lib.orc_spmv_export.restype = None
    lib.orc_spmv_export.argtypes = [ctypes.c_int64, _I32, _I32, _DBL, _DBL, _DBL]
    lib.orc_dot_export.restype = ctypes.c_double
    lib.orc_dot_export.argtypes = [ctypes.c_int64, _DBL, _DBL]
    lib.orc_jacobi.restype = ctypes.c_int
    lib.orc_jacobi.argtypes = [ctypes.c_int64, _I32, _I32, _DBL, _DBL]
    lib.orc_outer_csr.restype = None
    lib.orc_outer_csr.argtypes = [ctypes.c_int64, _I32, _I32, _DBL, _DBL, _DBL]
    lib.orc_max_threads.restype = ctypes.c_int
    lib.orc_max_threads.argtypes = []
    lib.orc_set_threads.restype = None
    lib.orc_set_threads.argtypes = [ctypes.c_int]
    return lib


def _lib():
    global _LIB
    with _LOCK:
        if _LIB is None:
            _LIB = load_library(build())
    return _LIB


def _d(a):
    return a.ctypes.data_as(_DBL) if a is not None else None


def _i(a):
    return a.ctypes.data_as(_I32)


def _csr_arrays(row_ptr, col_idx, values):
    rp = np.ascontiguousarray(row_ptr, dtype=np.int32)
    ci = np.ascontiguousarray(col_idx, dtype=np.int32)
    va = np.ascontiguousarray(values, dtype=np.float64)
    return rp, ci, va


def spmv(row_ptr, col_idx, values, x) -> np.ndarray:
    rp, ci, va = _csr_arrays(row_ptr, col_idx, values)
    x = np.ascontiguousarray(x, dtype=np.float64)
    y = np.empty(rp.shape[0] - 1)
    _lib().orc_spmv_export(rp.shape[0] - 1, _i(rp), _i(ci), _d(va), _d(x), _d(y))
    return y


def dot(a, b) -> float:
    a = np.ascontiguousarray(a, dtype=np.float64)
    b = np.ascontiguousarray(b, dtype=np.float64)
    return float(_lib().orc_dot_export(a.shape[0], _d(a), _d(b)))


def jacobi(row_ptr, col_idx, values) -> np.ndarray:
    """Reciprocal diagonal d_i = 1/a_ii; raises ValueError if a_ii is missing or <= 0."""
    rp, ci, va = _csr_arrays(row_ptr, col_idx, values)
    d = np.empty(rp.shape[0] - 1)
    if _lib().orc_jacobi(rp.shape[0] - 1, _i(rp), _i(ci), _d(va), _d(d)) != 0:
        raise ValueError("Jacobi preconditioner needs a positive diagonal")
    return d


def outer_csr(row_ptr, col_idx, lam, x) -> np.ndarray:
    """g_e = -lam[row(e)] * x[col(e)] for every stored entry e."""
    rp = np.ascontiguousarray(row_ptr, dtype=np.int32)
    ci = np.ascontiguousarray(col_idx, dtype=np.int32)
    lam = np.ascontiguousarray(lam, dtype=np.float64)
    x = np.ascontiguousarray(x, dtype=np.float64)
    g = np.empty(ci.shape[0])
    _lib().orc_outer_csr(rp.shape[0] - 1, _i(rp), _i(ci), _d(lam), _d(x), _d(g))
    return g


def max_threads() -> int:
    return int(_lib().orc_max_threads())


def set_threads(n: int) -> None:
    """OpenMP thread count of later calls (results do not depend on it)."""
    _lib().orc_set_threads(int(n))


_DIAG_KEYS = ("nu", "nup", "rr", "mu", "alpha", "beta", "true_res", "err_a", "orth", "gap")


def solve(row_ptr, col_idx, values, b, variant: str = "pr", precond: str = "none",
          tol: float = 1e-10, maxit: int = 1000, x0=None, diagnostics=None, xstar=None, lib=None):
    """Run one variant of the oracle.

    ``diagnostics`` is an iterable of names from ``nu, nup, rr, mu, alpha,
    beta, true_res, err_a, orth, gap``; each becomes a float64[iters+1] array in
    the result (NaN where the quantity is undefined).  Returns a dict with
    ``x``, ``iters``, ``status`` (string), ``code`` and ``history``
    (||r_k||/||b|| for k = 0..iters).
    """
    rp, ci, va = _csr_arrays(row_ptr, col_idx, values)
    n = rp.shape[0] - 1
    b = np.ascontiguousarray(b, dtype=np.float64)
    x = np.zeros(n) if x0 is None else np.array(x0, dtype=np.float64, copy=True)
    dinv = jacobi(rp, ci, va) if precond == "jacobi" else None
    if precond not in ("none", "jacobi"):
        raise ValueError(f"unknown preconditioner {precond!r}")
    hist = np.full(maxit + 1, np.nan)
    iters = ctypes.c_int32(0)
    dg = None
    arrays = {}
    if diagnostics:
        dg = _Diag()
        for key in diagnostics:
            if key not in _DIAG_KEYS:
                raise ValueError(f"unknown diagnostic {key!r}")
            arrays[key] = np.full(maxit + 1, np.nan)
            setattr(dg, key, _d(arrays[key]))
        xs = None
        if "err_a" in arrays:
            if xstar is None:
                raise ValueError("err_a needs xstar")
            xs = np.ascontiguousarray(xstar, dtype=np.float64)
            dg.xstar = _d(xs)
    lib = _lib() if lib is None else lib
    code = lib.orc_solve(VARIANTS[variant], n, _i(rp), _i(ci), _d(va), _d(dinv), _d(b), _d(x),
                            float(tol), int(maxit), ctypes.byref(iters), _d(hist),
                            ctypes.byref(dg) if dg is not None else None)
    if code < 0:
        raise ValueError(f"oracle returned {STATUS.get(code, code)}")
    k = iters.value
    out = {"x": x, "iters": k, "code": code, "status": STATUS[code], "history": hist[:k + 1].copy()}
    for key, arr in arrays.items():
        out[key] = arr[:k + 1].copy()
    return out
