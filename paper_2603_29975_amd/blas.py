"""Binding of libozaki_blas.so, the Fortran-BLAS DGEMM/ZGEMM interposer
(include/ozaki_blas.h): host arrays in, host arrays out, the emulated GEMM on
the GPU in between. Argument marshalling only.

``zgemm_`` / ``dgemm_`` take column-major numpy arrays (``np.asfortranarray``
or Fortran-ordered slices) and their leading dimensions exactly as the
Fortran routines do; ``C`` is updated in place. A process can instead preload
the library (``LD_PRELOAD``) under an unmodified application.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

from . import OzakiUnavailable, library as _core_library, ozaki_z

_HERE = os.path.dirname(os.path.abspath(__file__))
library_path = os.path.join(_HERE, "libozaki_blas.so")

_c = ctypes
_ip = _c.POINTER(_c.c_int)
_SIG = {
    "dgemm_": (None, [_c.c_char_p, _c.c_char_p, _ip, _ip, _ip, _c.c_void_p, _c.c_void_p, _ip,
                      _c.c_void_p, _ip, _c.c_void_p, _c.c_void_p, _ip]),
    "zgemm_": (None, [_c.c_char_p, _c.c_char_p, _ip, _ip, _ip, _c.c_void_p, _c.c_void_p, _ip,
                      _c.c_void_p, _ip, _c.c_void_p, _c.c_void_p, _ip]),
    "ozaki_blas_config": (_c.c_int, [_c.c_int, _c.c_int]),
    "ozaki_blas_release": (_c.c_int, []),
}
_lib = None


def library():
    global _lib
    if _lib is None:
        if not os.path.exists(library_path):
            raise OzakiUnavailable(f"{library_path} is missing: build it with "
                                   "`python paper_2603_29975_amd/build.py`")
        _core_library()          # libozaki.so first (the interposer links it)
        lib = ctypes.CDLL(library_path)
        for name, (res, args) in _SIG.items():
            fn = getattr(lib, name)
            fn.restype = res
            fn.argtypes = args
        _lib = lib
    return _lib


def _i(v):
    return _c.byref(_c.c_int(int(v)))


def _addr(X, offset_elems=0):
    return X.ctypes.data + offset_elems * X.itemsize


def _gemm(name, dtype, transa, transb, m, n, k, alpha, A, lda, B, ldb, beta, C, ldc):
    for X in (A, B, C):
        if X.dtype != dtype:
            raise TypeError(f"{name}: arrays must be {dtype}")
    if dtype == np.complex128:
        al = ozaki_z(complex(alpha).real, complex(alpha).imag)
        be = ozaki_z(complex(beta).real, complex(beta).imag)
    else:
        al, be = _c.c_double(float(alpha)), _c.c_double(float(beta))
    getattr(library(), name)(transa.encode(), transb.encode(), _i(m), _i(n), _i(k),
                             _c.cast(_c.pointer(al), _c.c_void_p), _addr(A), _i(lda), _addr(B),
                             _i(ldb), _c.cast(_c.pointer(be), _c.c_void_p), _addr(C), _i(ldc))


def dgemm_(transa, transb, m, n, k, alpha, A, lda, B, ldb, beta, C, ldc):
    """A, B, C: numpy float64 buffers holding the column-major matrices (the
    first element at the buffer's start); C is written in place."""
    _gemm("dgemm_", np.float64, transa, transb, m, n, k, alpha, A, lda, B, ldb, beta, C, ldc)


def zgemm_(transa, transb, m, n, k, alpha, A, lda, B, ldb, beta, C, ldc):
    """As dgemm_ for complex128 buffers."""
    _gemm("zgemm_", np.complex128, transa, transb, m, n, k, alpha, A, lda, B, ldb, beta, C, ldc)


def ozaki_blas_config(slices: int = 0, moduli: int = 0) -> int:
    return library().ozaki_blas_config(int(slices), int(moduli))


def ozaki_blas_release() -> int:
    return library().ozaki_blas_release()
