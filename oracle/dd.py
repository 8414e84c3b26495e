"""Double-double reference GEMM C* = op(A) op(B) (Hida, Li and Bailey 2001,
cited in Section 2.2 of the paper for emulating higher precision with FP64).

TEST INFRASTRUCTURE ONLY. The arithmetic lives in dd_gemm.c; this module only
marshals numpy arrays. Results are returned as (hi, lo) with hi + lo within
about L * 2^-104 * (|op(A)| |op(B)|)_ij of the exact product (L = k real terms,
2k per component for complex data).
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

from . import build_dd
from .ozaki import op

_lib = None


def _load():
    global _lib
    if _lib is None:
        path = build_dd.build(force=False)
        lib = ctypes.CDLL(path)
        P = ctypes.c_void_p
        I = ctypes.c_int64
        lib.dd_gemm_real.argtypes = [I, I, I, P, P, P, P]
        lib.dd_gemm_complex.argtypes = [I, I, I, P, P, P]
        lib.dd_entries_real.argtypes = [I, P, P, I, P, P, P, P]
        lib.dd_entries_complex.argtypes = [I, P, P, I, P, P, P]
        _lib = lib
    return _lib


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p)


def _operands(transa, transb, A, B):
    complex_ = np.iscomplexobj(A) or np.iscomplexobj(B)
    dt = np.complex128 if complex_ else np.float64
    opA = np.ascontiguousarray(op(np.asarray(A, dtype=dt), transa))
    opBt = np.ascontiguousarray(op(np.asarray(B, dtype=dt), transb).T)
    return complex_, opA, opBt


def dd_gemm(transa, transb, A, B):
    """Full double-double product. Returns (hi, lo); complex data gives complex
    hi and lo arrays (real and imaginary parts are separate dd numbers)."""
    lib = _load()
    complex_, opA, opBt = _operands(transa, transb, A, B)
    m, L = opA.shape
    n = opBt.shape[0]
    if complex_:
        out = np.empty((m, n, 4), dtype=np.float64)
        lib.dd_gemm_complex(m, n, L, _ptr(opA), _ptr(opBt), _ptr(out))
        hi = out[..., 0] + 0j
        hi.imag = out[..., 2]
        lo = out[..., 1] + 0j
        lo.imag = out[..., 3]
        return hi, lo
    hi = np.empty((m, n))
    lo = np.empty((m, n))
    lib.dd_gemm_real(m, n, L, _ptr(opA), _ptr(opBt), _ptr(hi), _ptr(lo))
    return hi, lo


def dd_entries(transa, transb, A, B, rows, cols):
    """Double-double values of the entries (rows[x], cols[x]). Returns (hi, lo)
    1-D arrays (complex for complex data)."""
    lib = _load()
    complex_, opA, opBt = _operands(transa, transb, A, B)
    ri = np.ascontiguousarray(rows, dtype=np.int64)
    cj = np.ascontiguousarray(cols, dtype=np.int64)
    if ri.shape != cj.shape or ri.ndim != 1:
        raise ValueError("rows and cols must be 1-D of equal length")
    if ri.size and (ri.min() < 0 or ri.max() >= opA.shape[0] or cj.min() < 0 or cj.max() >= opBt.shape[0]):
        raise IndexError("entry index out of range")
    L = opA.shape[1]
    cnt = ri.size
    if complex_:
        out = np.empty((cnt, 4))
        lib.dd_entries_complex(cnt, _ptr(ri), _ptr(cj), L, _ptr(opA), _ptr(opBt), _ptr(out))
        hi = out[:, 0] + 0j
        hi.imag = out[:, 2]
        lo = out[:, 1] + 0j
        lo.imag = out[:, 3]
        return hi, lo
    hi = np.empty(cnt)
    lo = np.empty(cnt)
    lib.dd_entries_real(cnt, _ptr(ri), _ptr(cj), L, _ptr(opA), _ptr(opBt), _ptr(hi), _ptr(lo))
    return hi, lo


def threads_used() -> int:
    """OpenMP threads the helper will use (OMP_NUM_THREADS or all cores)."""
    v = os.environ.get("OMP_NUM_THREADS")
    return int(v) if v and v.isdigit() else (os.cpu_count() or 1)
