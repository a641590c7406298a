"""ctypes binding of libprcg (include/prcg.h).

The functions ``prcg_*`` mirror the C ABI one to one (argument marshalling
only).  :class:`Matrix` wraps a handle and takes torch tensors (or NumPy
arrays, which are copied to the GPU) for device memory; the stream is
torch's current stream.  Every step of a solve runs in the HIP library: if
``libprcg.so`` is missing, loading raises instead of falling back to
anything else.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass
from typing import Optional

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libprcg.so")

PRCG_HS, PRCG_PR, PRCG_PIPE_PR, PRCG_M, PRCG_PIPE_M, PRCG_GV = 0, 1, 2, 3, 4, 5
PRCG_PR_NORECOMPUTE, PRCG_PIPE_PR_NOWRECOMPUTE, PRCG_CG, PRCG_PR_UNSIMPLIFIED = 6, 7, 8, 9
VARIANTS = {"hs": PRCG_HS, "pr": PRCG_PR, "pipe_pr": PRCG_PIPE_PR, "m": PRCG_M, "pipe_m": PRCG_PIPE_M,
            "gv": PRCG_GV, "pr_norecompute": PRCG_PR_NORECOMPUTE, "pipe_pr_nowrecompute": PRCG_PIPE_PR_NOWRECOMPUTE,
            "cg": PRCG_CG, "pr_unsimplified": PRCG_PR_UNSIMPLIFIED}
PRECONDS = {"none": 0, "jacobi": 1}
STATUS = {0: "ok", 1: "not_converged", 2: "breakdown", -1: "einval", -2: "enomem", -3: "edevice"}

KERNELS = {"fused": 0, "two_pass": 1, "two_pass_stage2": 2, "textbook": 3, "two_pass_last": 4,
           "two_pass_redundant": 5, "auto": 6}
OPT_KERNELS, OPT_GRID = 0, 1
BATCH_MODES = {"auto": 0, "persistent": 1, "lockstep": 2}
BATCH_FUSION = {"auto": 0, "off": 1, "on": 2}

EXPORTED = ("prcg_create_csr", "prcg_set_values", "prcg_set_option", "prcg_set_stream", "prcg_spmv", "prcg_solve",
            "prcg_time_kernels", "prcg_get_props", "prcg_create_batch", "prcg_solve_batched",
            "prcg_adjoint", "prcg_destroy", "prcg_batch_destroy", "prcg_last_error", "prcg_batch_config",
            "prcg_batch_set_mode", "prcg_batch_mode", "prcg_solve_noalloc", "prcg_batch_set_config",
            "prcg_batch_get_props", "prcg_batch_set_fusion")
NOALLOC_MAX_ITERS = 65536  # PRCG_NOALLOC_MAX_ITERS


class PrcgError(RuntimeError):
    def __init__(self, code: int, message: str):
        super().__init__(f"{STATUS.get(code, code)}: {message}")
        self.code = code


class prcg_info(ctypes.Structure):
    _fields_ = [("iters", ctypes.c_int32), ("status", ctypes.c_int32),
                ("relres_updated", ctypes.c_double), ("relres_true", ctypes.c_double)]


class prcg_matrix_props(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int64), ("nnz", ctypes.c_int64), ("stored_entries", ctypes.c_int64),
                ("format", ctypes.c_int32), ("lanes_per_row", ctypes.c_int32), ("grid", ctypes.c_int32),
                ("block", ctypes.c_int32), ("matrix_bytes", ctypes.c_int64),
                ("aligned_slices_frac", ctypes.c_double), ("kernels", ctypes.c_int32), ("stage2", ctypes.c_int32),
                ("streamed_entries", ctypes.c_int64)]


class prcg_batch_props(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int64), ("stored_entries", ctypes.c_int64), ("matrix_bytes", ctypes.c_int64),
                ("groups", ctypes.c_int64), ("uniform_groups", ctypes.c_int64), ("nsys", ctypes.c_int32),
                ("mode", ctypes.c_int32), ("threads", ctypes.c_int32), ("grid", ctypes.c_int32),
                ("slices_in_flight", ctypes.c_int32), ("group_slices", ctypes.c_int32), ("fused", ctypes.c_int32)]


_VP = ctypes.c_void_p
_LIB = None


def load_library(path: str = LIB_PATH):
    """Load libprcg.so and declare its signatures (raises if it is not built)."""
    global _LIB
    if _LIB is not None:
        return _LIB
    if not os.path.exists(path):
        raise ImportError(f"{path} is missing: build it with `python -m paper_1905_01549_amd.build`")
    # torch ships its own HIP runtime; load it first so that the library binds
    # to the same one (device pointers from torch are then recognised)
    try:
        import torch  # noqa: F401
    except ImportError:
        pass
    lib = ctypes.CDLL(path)
    i32, i64, dbl = ctypes.c_int32, ctypes.c_int64, ctypes.c_double
    sig = {
        "prcg_create_csr": (i32, [i64, i64, _VP, _VP, _VP, i32, _VP, ctypes.POINTER(_VP)]),
        "prcg_set_values": (i32, [_VP, _VP]),
        "prcg_set_stream": (i32, [_VP, _VP]),
        "prcg_set_option": (i32, [_VP, i32, i32]),
        "prcg_spmv": (i32, [_VP, _VP, _VP]),
        "prcg_solve": (i32, [_VP, i32, _VP, _VP, dbl, i32, ctypes.POINTER(prcg_info), _VP]),
        "prcg_solve_noalloc": (i32, [_VP, i32, _VP, _VP, dbl, i32, ctypes.POINTER(prcg_info), _VP]),
        "prcg_time_kernels": (i32, [_VP, i32, i32, _VP, _VP, i32, ctypes.POINTER(i32)]),
        "prcg_get_props": (i32, [_VP, ctypes.POINTER(prcg_matrix_props)]),
        "prcg_create_batch": (i32, [_VP, i32, _VP, ctypes.POINTER(_VP)]),
        "prcg_solve_batched": (i32, [_VP, i32, _VP, _VP, dbl, i32, _VP, _VP]),
        "prcg_adjoint": (i32, [_VP, i32, _VP, _VP, _VP, _VP, dbl, i32, ctypes.POINTER(prcg_info)]),
        "prcg_destroy": (None, [_VP]),
        "prcg_batch_destroy": (None, [_VP]),
        "prcg_last_error": (ctypes.c_char_p, []),
        "prcg_batch_config": (i32, [_VP, i32, ctypes.POINTER(i32), ctypes.POINTER(i32)]),
        "prcg_batch_set_mode": (i32, [_VP, i32]),
        "prcg_batch_mode": (i32, [_VP, i32, ctypes.POINTER(i32)]),
        "prcg_batch_set_config": (i32, [_VP, i32, i32, i32, i32]),
        "prcg_batch_get_props": (i32, [_VP, i32, ctypes.POINTER(prcg_batch_props)]),
        "prcg_batch_set_fusion": (i32, [_VP, i32]),
    }
    for name, (res, args) in sig.items():
        f = getattr(lib, name)
        f.restype = res
        f.argtypes = args
    _LIB = lib
    return lib


def _check(code: int, allow_numeric: bool = False) -> int:
    if code < 0 or (code > 0 and not allow_numeric):
        raise PrcgError(code, load_library().prcg_last_error().decode())
    return code


# ---------------------------------------------------------------- raw C ABI

def prcg_create_csr(n, nnz, row_ptr, col_idx, values, precond, hip_stream) -> int:
    h = _VP()
    _check(load_library().prcg_create_csr(n, nnz, row_ptr, col_idx, values, precond, hip_stream,
                                          ctypes.byref(h)))
    return h.value


def prcg_set_values(A, values):
    _check(load_library().prcg_set_values(A, values))


def prcg_set_option(A, option, value):
    _check(load_library().prcg_set_option(A, option, value))


def prcg_set_stream(A, hip_stream):
    _check(load_library().prcg_set_stream(A, hip_stream))


def prcg_spmv(A, x, y):
    _check(load_library().prcg_spmv(A, x, y))


def prcg_solve(A, variant, b, x, tol, maxit, info=None, history=None) -> int:
    return _check(load_library().prcg_solve(A, variant, b, x, tol, maxit,
                                            ctypes.byref(info) if info is not None else None, history),
                  allow_numeric=True)


def prcg_solve_noalloc(A, variant, b, x, tol, maxit, info=None, history=None) -> int:
    return _check(load_library().prcg_solve_noalloc(A, variant, b, x, tol, maxit,
                                                    ctypes.byref(info) if info is not None else None, history),
                  allow_numeric=True)


def prcg_time_kernels(A, variant, iters, capacity: int = 16):
    ms = (ctypes.c_double * capacity)()
    names = (ctypes.c_char * (capacity * 48))()
    nk = ctypes.c_int32(0)
    _check(load_library().prcg_time_kernels(A, variant, iters, ms, names, capacity, ctypes.byref(nk)))
    raw = bytes(names)
    return [(raw[48 * j:48 * (j + 1)].split(b"\0")[0].decode(), ms[j]) for j in range(nk.value)]


def prcg_get_props(A) -> prcg_matrix_props:
    p = prcg_matrix_props()
    _check(load_library().prcg_get_props(A, ctypes.byref(p)))
    return p


def prcg_create_batch(A, nsys, sys_row_offset_host) -> int:
    h = _VP()
    off = np.ascontiguousarray(sys_row_offset_host, dtype=np.int64)
    _check(load_library().prcg_create_batch(A, nsys, off.ctypes.data, ctypes.byref(h)))
    return h.value


def prcg_solve_batched(B, variant, b, x, tol, maxit, iters=None, status=None) -> int:
    return _check(load_library().prcg_solve_batched(B, variant, b, x, tol, maxit, iters, status),
                  allow_numeric=True)


def prcg_batch_config(B, variant):
    t, g = ctypes.c_int32(0), ctypes.c_int32(0)
    _check(load_library().prcg_batch_config(B, variant, ctypes.byref(t), ctypes.byref(g)))
    return t.value, g.value


def prcg_batch_set_mode(B, mode):
    _check(load_library().prcg_batch_set_mode(B, mode))


def prcg_batch_set_config(B, threads=0, per_cu=0, slices_in_flight=0, group_slices=0):
    _check(load_library().prcg_batch_set_config(B, threads, per_cu, slices_in_flight, group_slices))


def prcg_batch_set_fusion(B, fusion):
    _check(load_library().prcg_batch_set_fusion(B, fusion))


def prcg_batch_get_props(B, variant) -> prcg_batch_props:
    p = prcg_batch_props()
    _check(load_library().prcg_batch_get_props(B, variant, ctypes.byref(p)))
    return p


def prcg_batch_mode(B, variant) -> int:
    m = ctypes.c_int32(0)
    _check(load_library().prcg_batch_mode(B, variant, ctypes.byref(m)))
    return m.value


def prcg_adjoint(A, variant, x, gx, gb, gvals, tol, maxit, info=None) -> int:
    return _check(load_library().prcg_adjoint(A, variant, x, gx, gb, gvals, tol, maxit,
                                              ctypes.byref(info) if info is not None else None),
                  allow_numeric=True)


def prcg_destroy(A):
    if A:
        load_library().prcg_destroy(A)


def prcg_batch_destroy(B):
    if B:
        load_library().prcg_batch_destroy(B)


def prcg_last_error() -> str:
    return load_library().prcg_last_error().decode()


# ---------------------------------------------------------------- convenience layer

def _torch():
    import torch
    return torch


def _dev(a, dtype):
    """A contiguous CUDA tensor of the given torch dtype (copied if needed)."""
    torch = _torch()
    if isinstance(a, torch.Tensor):
        t = a.to(device="cuda", dtype=dtype)
    else:
        t = torch.as_tensor(np.asarray(a), device="cuda").to(dtype)
    return t.contiguous()


def _stream_ptr():
    return _torch().cuda.current_stream().cuda_stream


@dataclass
class SolveInfo:
    iters: int
    status: str
    relres_updated: float
    relres_true: float
    history: Optional[np.ndarray] = None


class Matrix:
    """A sparse SPD matrix resident on the GPU (CSR input, int32 indices)."""

    def __init__(self, row_ptr, col_idx, values, precond: str = "none"):
        torch = _torch()
        self._rp = _dev(row_ptr, torch.int32)
        self._ci = _dev(col_idx, torch.int32)
        self._va = _dev(values, torch.float64)
        self.n = self._rp.numel() - 1
        self.nnz = self._ci.numel()
        self.precond = precond
        self.handle = None
        self.handle = prcg_create_csr(self.n, self.nnz, self._rp.data_ptr(), self._ci.data_ptr(),
                                      self._va.data_ptr(), PRECONDS[precond], _stream_ptr())
        # the library copied the matrix; the tensors are kept only for the autograd layer
        self.row_ptr, self.col_idx = self._rp, self._ci

    def close(self):
        if self.handle:
            prcg_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    @property
    def props(self) -> prcg_matrix_props:
        return prcg_get_props(self.handle)

    def set_kernels(self, mode: str):
        """Kernel structure: "auto" (default: "fused" for HS-CG and PR-CG
        below 2048 workgroups, else "two_pass"), "two_pass" (stage-2 placement by size),
        "two_pass_redundant", "two_pass_stage2", "two_pass_last", "fused" or
        "textbook" (HS-CG one kernel per algorithm line)."""
        prcg_set_option(self.handle, OPT_KERNELS, KERNELS[mode])

    def set_grid(self, g: int):
        prcg_set_option(self.handle, OPT_GRID, int(g))

    def set_values(self, values):
        v = _dev(values, _torch().float64)
        prcg_set_values(self.handle, v.data_ptr())

    def spmv(self, x):
        torch = _torch()
        xd = _dev(x, torch.float64)
        y = torch.empty_like(xd)
        prcg_set_stream(self.handle, _stream_ptr())
        prcg_spmv(self.handle, xd.data_ptr(), y.data_ptr())
        return y

    def solve(self, b, variant: str = "pr", tol: float = 1e-10, maxit: int = 10000, x0=None,
              history: bool = False, noalloc: bool = False):
        """Solve A x = b; returns (x as a CUDA tensor, SolveInfo).  noalloc:
        through prcg_solve_noalloc (the library allocates nothing during the
        call; maxit <= NOALLOC_MAX_ITERS)."""
        torch = _torch()
        bd = _dev(b, torch.float64)
        x = torch.zeros_like(bd) if x0 is None else _dev(x0, torch.float64).clone()
        info = prcg_info()
        hist = np.full(maxit + 1, np.nan) if history else None
        prcg_set_stream(self.handle, _stream_ptr())
        call = prcg_solve_noalloc if noalloc else prcg_solve
        call(self.handle, VARIANTS[variant], bd.data_ptr(), x.data_ptr(), float(tol), int(maxit), info,
             hist.ctypes.data if hist is not None else None)
        return x, SolveInfo(info.iters, STATUS[info.status], info.relres_updated, info.relres_true,
                            hist[:info.iters + 1].copy() if hist is not None else None)

    def adjoint(self, x, gx, variant: str = "pr", tol: float = 1e-10, maxit: int = 10000,
                want_b: bool = True, want_values: bool = True):
        """(dL/db, dL/dvalues, SolveInfo) for x = A^{-1} b and gx = dL/dx."""
        torch = _torch()
        xd = _dev(x, torch.float64)
        gxd = _dev(gx, torch.float64)
        gb = torch.empty_like(gxd) if want_b else None
        gv = torch.empty(self.nnz, dtype=torch.float64, device="cuda") if want_values else None
        info = prcg_info()
        prcg_set_stream(self.handle, _stream_ptr())
        prcg_adjoint(self.handle, VARIANTS[variant], xd.data_ptr(), gxd.data_ptr(),
                     gb.data_ptr() if gb is not None else None, gv.data_ptr() if gv is not None else None,
                     float(tol), int(maxit), info)
        return gb, gv, SolveInfo(info.iters, STATUS[info.status], info.relres_updated, info.relres_true)

    def time_kernels(self, variant: str = "pr", iters: int = 50):
        prcg_set_stream(self.handle, _stream_ptr())
        return prcg_time_kernels(self.handle, VARIANTS[variant], iters)


class Batch:
    """Independent systems stored as one block-diagonal matrix (rows of
    system s: sys_row_offset[s] .. sys_row_offset[s+1])."""

    def __init__(self, matrix: Matrix, sys_row_offset):
        self.matrix = matrix
        self.offsets = np.ascontiguousarray(sys_row_offset, dtype=np.int64)
        self.nsys = self.offsets.size - 1
        self.handle = None
        self.handle = prcg_create_batch(matrix.handle, self.nsys, self.offsets)

    def close(self):
        if self.handle:
            prcg_batch_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def solve(self, b, variant: str = "pr", tol: float = 1e-10, maxit: int = 10000, x0=None):
        """Returns (x, iters[nsys], status[nsys] as strings)."""
        torch = _torch()
        bd = _dev(b, torch.float64)
        x = torch.zeros_like(bd) if x0 is None else _dev(x0, torch.float64).clone()
        iters = np.zeros(self.nsys, dtype=np.int32)
        status = np.zeros(self.nsys, dtype=np.int32)
        prcg_set_stream(self.matrix.handle, _stream_ptr())
        prcg_solve_batched(self.handle, VARIANTS[variant], bd.data_ptr(), x.data_ptr(), float(tol), int(maxit),
                           iters.ctypes.data, status.ctypes.data)
        return x, iters, [STATUS[int(c)] for c in status]

    def config(self, variant: str = "pr"):
        return prcg_batch_config(self.handle, VARIANTS[variant])

    def set_mode(self, mode: str):
        """'auto' (the faster on the first solve), 'persistent' or 'lockstep'."""
        prcg_batch_set_mode(self.handle, BATCH_MODES[mode])

    def mode(self, variant: str = "pr"):
        """The mode in use for a variant, or None before its first solve."""
        m = prcg_batch_mode(self.handle, VARIANTS[variant])
        return {v: k for k, v in BATCH_MODES.items()}.get(m) if m else None

    def set_config(self, threads: int = 0, per_cu: int = 0, slices_in_flight: int = 0, group_slices: int = 0):
        """Fix parts of the configuration (0: left to the autotuner)."""
        prcg_batch_set_config(self.handle, threads, per_cu, slices_in_flight, group_slices)

    def set_fusion(self, fusion: str):
        """'auto' (timed by the autotuner), 'off' (three launches per lockstep
        iteration) or 'on' (the fused iteration only)."""
        prcg_batch_set_fusion(self.handle, BATCH_FUSION[fusion])

    def props(self, variant: str = "pr") -> dict:
        """Storage and the configuration in use for a variant."""
        p = prcg_batch_get_props(self.handle, VARIANTS[variant])
        out = {name: getattr(p, name) for name, _ in p._fields_}
        out["mode"] = {v: k for k, v in BATCH_MODES.items()}.get(out["mode"]) if out["mode"] else None
        return out
