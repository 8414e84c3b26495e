"""Python binding of libozaki, the MI355X (gfx950) Ozaki-I FP64/complex-FP64
GEMM emulator.

Argument marshalling only: every step of the computation runs in the HIP
kernels of libozaki.so (built in-tree by ``paper_2603_29975_amd/build.py``).
There is no fallback: if the shared library is missing, importing a function
that needs it raises ``OzakiUnavailable``.

The functions named like the C ABI (``ozaki_dgemm`` ...) take column-major
device buffers exactly as the C functions do: matrices are torch CUDA tensors
(their ``data_ptr()`` is passed) or plain integer device addresses, and the
return value is the C status code. They bind the current torch stream first.

``matmul`` is a convenience on torch tensors in their usual row-major layout.
"""
from __future__ import annotations

import ctypes
import os

__all__ = [
    "OzakiError", "OzakiUnavailable", "ozaki_z", "library", "library_path",
    "ozaki_dgemm", "ozaki_zgemm", "ozaki_zgemm_noalloc", "ozaki_native_dgemm", "ozaki_native_zgemm",
    "ozaki_set_stream", "ozaki_set_workspace", "ozaki_workspace_bytes",
    "ozaki_finalize", "ozaki_status_string", "ozaki_timing_enable", "ozaki_timing_read", "ozaki_debug_exponents",
    "ozaki_debug_split", "ozaki_debug_diagonals", "matmul", "S_MAX", "ozaki_zgemm_batched",
    "ozaki_batched_graphs", "ozaki_batched_cache_clear", "ozaki_probe", "ozaki_features",
    "ozaki_mlp_state_bytes", "ozaki_mlp_scratch_bytes", "ozaki_mlp_init", "ozaki_mlp_refresh",
    "ozaki_mlp_forward", "ozaki_mlp_backward", "ozaki_mlp_adam", "MLP_PARAMS",
    "ozaki_load_selector", "ozaki_autotune", "ozaki_tune_set", "ozaki_tune_get",
    "ozaki_tune_configs", "ozaki_tune_save", "ozaki_tune_load", "ozaki_tune_clear",
    "ozaki2_dgemm", "ozaki2_zgemm", "ozaki2_moduli", "ozaki2_beta_bits", "ozaki2_workspace_bytes",
    "MODULI_MIN", "MODULI_MAX", "K2_MAX", "ozaki_set_split", "ozaki_get_split", "SPLIT_TRUNC7",
    "SPLIT_BAL8", "S8_MAX", "ozaki_zgetrf", "ozaki_zgetri", "ozaki_set_grid_limit",
]

_HERE = os.path.dirname(os.path.abspath(__file__))
library_path = os.path.join(_HERE, "libozaki.so")
S_MAX = 12
SPLIT_TRUNC7, SPLIT_BAL8 = 0, 1  # Ozaki-I slice kinds (ozaki_set_split)
S8_MAX = 8                       # slices accepted with 8-bit balanced slices
MODULI_MIN, MODULI_MAX = 2, 20   # Ozaki-II moduli counts
K2_MAX = 131072                  # Ozaki-II contraction length K' (k, or 2k complex)


class OzakiUnavailable(ImportError):
    pass


class OzakiError(RuntimeError):
    def __init__(self, status: int, what: str = ""):
        self.status = status
        super().__init__(f"{what}: status {status} ({ozaki_status_string(status)})")


class ozaki_z(ctypes.Structure):
    _fields_ = [("re", ctypes.c_double), ("im", ctypes.c_double)]


_c = ctypes
_i64 = _c.c_int64
_vp = _c.c_void_p
_SIG = {
    "ozaki_dgemm": (_c.c_int, [_c.c_char, _c.c_char, _i64, _i64, _i64, _c.c_double, _vp, _i64, _vp,
                               _i64, _c.c_double, _vp, _i64, _c.c_int]),
    "ozaki_zgemm": (_c.c_int, [_c.c_char, _c.c_char, _i64, _i64, _i64, ozaki_z, _vp, _i64, _vp,
                               _i64, ozaki_z, _vp, _i64, _c.c_int]),
    "ozaki_zgemm_noalloc": (_c.c_int, [_c.c_char, _c.c_char, _i64, _i64, _i64, ozaki_z, _vp, _i64,
                                       _vp, _i64, ozaki_z, _vp, _i64, _c.c_int]),
    "ozaki2_dgemm": (_c.c_int, [_c.c_char, _c.c_char, _i64, _i64, _i64, _c.c_double, _vp, _i64, _vp,
                                _i64, _c.c_double, _vp, _i64, _c.c_int]),
    "ozaki2_zgemm": (_c.c_int, [_c.c_char, _c.c_char, _i64, _i64, _i64, ozaki_z, _vp, _i64, _vp,
                                _i64, ozaki_z, _vp, _i64, _c.c_int]),
    "ozaki2_moduli": (_c.c_int, [_c.c_int, _vp]),
    "ozaki_set_split": (_c.c_int, [_c.c_int]),
    "ozaki_set_grid_limit": (_c.c_int, [_i64]),
    "ozaki_zgetrf": (_c.c_int, [_i64, _vp, _i64, _vp, _i64, _c.c_int]),
    "ozaki_zgetri": (_c.c_int, [_i64, _vp, _i64, _vp, _vp, _i64, _i64, _c.c_int]),
    "ozaki_get_split": (_c.c_int, []),
    "ozaki2_beta_bits": (_c.c_int, [_c.c_int, _i64]),
    "ozaki2_workspace_bytes": (_c.c_size_t, [_c.c_char, _i64, _i64, _i64, _c.c_int]),
    "ozaki_native_dgemm": (_c.c_int, [_c.c_char, _c.c_char, _i64, _i64, _i64, _c.c_double, _vp,
                                      _i64, _vp, _i64, _c.c_double, _vp, _i64]),
    "ozaki_native_zgemm": (_c.c_int, [_c.c_char, _c.c_char, _i64, _i64, _i64, ozaki_z, _vp, _i64,
                                      _vp, _i64, ozaki_z, _vp, _i64]),
    "ozaki_zgemm_batched": (_c.c_int, [_vp] * 13 + [_i64, _vp, _vp]),
    "ozaki_batched_graphs": (_c.c_int, [_c.c_int]),
    "ozaki_batched_cache_clear": (_c.c_int, []),
    "ozaki_probe": (_c.c_int, [_c.c_char, _c.c_char, _c.c_char, _i64, _i64, _i64, _vp, _i64, _vp,
                               _i64, _vp, _i64, _c.c_int, _c.c_uint64, _vp]),
    "ozaki_features": (_c.c_int, [_c.c_char, _c.c_char, _c.c_char, _i64, _i64, _i64, _vp, _i64,
                                  _vp, _i64, _vp]),
    "ozaki_mlp_state_bytes": (_c.c_size_t, []),
    "ozaki_mlp_scratch_bytes": (_c.c_size_t, [_i64]),
    "ozaki_mlp_init": (_c.c_int, [_vp, _c.c_uint64]),
    "ozaki_mlp_refresh": (_c.c_int, [_vp]),
    "ozaki_mlp_forward": (_c.c_int, [_vp, _i64, _vp, _vp, _vp]),
    "ozaki_mlp_backward": (_c.c_int, [_vp, _i64, _vp, _vp, _c.c_float, _vp, _vp]),
    "ozaki_mlp_adam": (_c.c_int, [_vp, _c.c_float, _c.c_float, _c.c_float, _c.c_float, _i64]),
    "ozaki_load_selector": (_c.c_int, [_vp, _c.c_float, _c.c_double, _c.c_double]),
    "ozaki_autotune": (_c.c_int, [_c.c_char, _i64, _i64, _i64, _c.c_int, _c.c_int, _vp, _vp]),
    "ozaki_tune_set": (_c.c_int, [_c.c_char, _i64, _i64, _i64, _c.c_int, _c.c_int]),
    "ozaki_tune_get": (_c.c_int, [_c.c_char, _i64, _i64, _i64, _c.c_int]),
    "ozaki_tune_configs": (_c.c_int, []),
    "ozaki_tune_save": (_c.c_int, [_c.c_char_p]),
    "ozaki_tune_load": (_c.c_int, [_c.c_char_p]),
    "ozaki_tune_clear": (_c.c_int, []),
    "ozaki_set_stream": (_c.c_int, [_vp]),
    "ozaki_set_workspace": (_c.c_int, [_vp, _c.c_size_t]),
    "ozaki_workspace_bytes": (_c.c_size_t, [_c.c_char, _i64, _i64, _i64, _c.c_int]),
    "ozaki_finalize": (_c.c_int, []),
    "ozaki_timing_enable": (_c.c_int, [_c.c_int]),
    "ozaki_timing_read": (_c.c_int, [_vp, _vp]),
    "ozaki_status_string": (_c.c_char_p, [_c.c_int]),
    "ozaki_debug_exponents": (_c.c_int, [_c.c_char, _c.c_char, _c.c_char, _i64, _i64, _vp, _i64,
                                         _vp, _vp]),
    "ozaki_debug_split": (_c.c_int, [_c.c_char, _c.c_char, _c.c_char, _i64, _i64, _vp, _i64,
                                     _c.c_int, _vp]),
    "ozaki_debug_diagonals": (_c.c_int, [_c.c_char, _c.c_char, _c.c_char, _i64, _i64, _i64, _vp,
                                         _i64, _vp, _i64, _c.c_int, _vp]),
}

_lib = None


def library():
    """The loaded libozaki.so (ctypes.CDLL). Raises OzakiUnavailable if it has
    not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(library_path):
            raise OzakiUnavailable(
                f"{library_path} is missing: build it with `python paper_2603_29975_amd/build.py` "
                "(or __graft_entry__.build()); there is no fallback implementation")
        # PyTorch first: its HIP runtime must be the process's one before the
        # library's dependency on libamdhip64 is resolved (loading the library
        # first pulls in another copy, and device calls made through the two
        # then disagree about the device)
        try:
            import torch  # noqa: F401
        except ImportError:
            pass
        lib = ctypes.CDLL(library_path)
        for name, (res, args) in _SIG.items():
            fn = getattr(lib, name)
            fn.restype = res
            fn.argtypes = args
        _lib = lib
    return _lib


def _ch(c: str) -> bytes:
    return c.encode("ascii") if isinstance(c, str) else bytes(c)


def _ptr(x):
    if x is None:
        return None
    if isinstance(x, int):
        return x
    return x.data_ptr()


def _z(v) -> ozaki_z:
    v = complex(v)
    return ozaki_z(v.real, v.imag)


def _bind_stream():
    import torch
    if torch.cuda.is_available():
        library().ozaki_set_stream(_c.c_void_p(torch.cuda.current_stream().cuda_stream))


def ozaki_dgemm(transa, transb, m, n, k, alpha, A, lda, B, ldb, beta, C, ldc, slices) -> int:
    _bind_stream()
    return library().ozaki_dgemm(_ch(transa), _ch(transb), m, n, k, float(alpha), _ptr(A), lda,
                                 _ptr(B), ldb, float(beta), _ptr(C), ldc, int(slices))


def ozaki_zgemm(transa, transb, m, n, k, alpha, A, lda, B, ldb, beta, C, ldc, slices) -> int:
    _bind_stream()
    return library().ozaki_zgemm(_ch(transa), _ch(transb), m, n, k, _z(alpha), _ptr(A), lda,
                                 _ptr(B), ldb, _z(beta), _ptr(C), ldc, int(slices))


def ozaki_zgemm_noalloc(transa, transb, m, n, k, alpha, A, lda, B, ldb, beta, C, ldc,
                        slices) -> int:
    _bind_stream()
    return library().ozaki_zgemm_noalloc(_ch(transa), _ch(transb), m, n, k, _z(alpha), _ptr(A),
                                         lda, _ptr(B), ldb, _z(beta), _ptr(C), ldc, int(slices))


def ozaki2_dgemm(transa, transb, m, n, k, alpha, A, lda, B, ldb, beta, C, ldc, moduli) -> int:
    _bind_stream()
    return library().ozaki2_dgemm(_ch(transa), _ch(transb), m, n, k, float(alpha), _ptr(A), lda,
                                  _ptr(B), ldb, float(beta), _ptr(C), ldc, int(moduli))


def ozaki2_zgemm(transa, transb, m, n, k, alpha, A, lda, B, ldb, beta, C, ldc, moduli) -> int:
    _bind_stream()
    return library().ozaki2_zgemm(_ch(transa), _ch(transb), m, n, k, _z(alpha), _ptr(A), lda,
                                  _ptr(B), ldb, _z(beta), _ptr(C), ldc, int(moduli))


def ozaki_set_split(mode) -> int:
    """Slice kind of ozaki_dgemm/ozaki_zgemm: SPLIT_TRUNC7 (default) or SPLIT_BAL8
    (8-bit balanced slices, 1..S8_MAX slices); "t7"/"b8" are accepted too."""
    if isinstance(mode, str):
        mode = {"t7": SPLIT_TRUNC7, "b8": SPLIT_BAL8}.get(mode, -1)
    return library().ozaki_set_split(int(mode))


def ozaki_zgetrf(n, A, lda, ipiv, nb, slices) -> int:
    """Blocked LU with partial pivoting in place (A: complex128 device buffer,
    ipiv: int64 device buffer of n, 0-based); slices = 0 uses the native FP64
    ZGEMM for the trailing updates. Synchronises before returning."""
    _bind_stream()
    return library().ozaki_zgetrf(int(n), _ptr(A), int(lda), _ptr(ipiv), int(nb), int(slices))


def ozaki_zgetri(n, LU, lda, ipiv, X, ldx, nb, slices) -> int:
    """X = A^-1 from the factors of ozaki_zgetrf (X must not overlap LU)."""
    _bind_stream()
    return library().ozaki_zgetri(int(n), _ptr(LU), int(lda), _ptr(ipiv), _ptr(X), int(ldx),
                                  int(nb), int(slices))


def ozaki_get_split() -> int:
    return library().ozaki_get_split()


def ozaki_set_grid_limit(max_workgroups) -> int:
    """Cap the persistent slice GEMM's workgroup count (0: no cap)."""
    return library().ozaki_set_grid_limit(int(max_workgroups))


def ozaki2_moduli(moduli):
    """(status, list of the first `moduli` moduli); host-side query."""
    out = (_c.c_int32 * max(int(moduli), 1))()
    rc = library().ozaki2_moduli(int(moduli), _c.cast(out, _c.c_void_p))
    return rc, [out[i] for i in range(int(moduli))] if rc == 0 else []


def ozaki2_beta_bits(moduli, kprime) -> int:
    return library().ozaki2_beta_bits(int(moduli), int(kprime))


def ozaki2_workspace_bytes(kind, m, n, k, moduli) -> int:
    return library().ozaki2_workspace_bytes(_ch(kind), m, n, k, int(moduli))


def ozaki_native_dgemm(transa, transb, m, n, k, alpha, A, lda, B, ldb, beta, C, ldc) -> int:
    _bind_stream()
    return library().ozaki_native_dgemm(_ch(transa), _ch(transb), m, n, k, float(alpha), _ptr(A),
                                        lda, _ptr(B), ldb, float(beta), _ptr(C), ldc)


def ozaki_native_zgemm(transa, transb, m, n, k, alpha, A, lda, B, ldb, beta, C, ldc) -> int:
    _bind_stream()
    return library().ozaki_native_zgemm(_ch(transa), _ch(transb), m, n, k, _z(alpha), _ptr(A), lda,
                                        _ptr(B), ldb, _z(beta), _ptr(C), ldc)


def ozaki_zgemm_batched(transa, transb, m, n, k, alpha, A, lda, B, ldb, beta, C, ldc, batch,
                        slices, slices_used=None) -> int:
    """Batched complex GEMM. Every argument is a sequence of length `batch`
    (A, B, C: tensors or device addresses); `slices` may be None (automatic
    selection). `slices_used`, if given, is a list that receives the slice
    counts used."""
    _bind_stream()
    nb = int(batch)

    def chars(v):
        return (_c.c_char * max(nb, 1))(*[_ch(x) for x in v])

    def i64(v):
        return (_c.c_int64 * max(nb, 1))(*[int(x) for x in v])

    def zs(v):
        return (ozaki_z * max(nb, 1))(*[_z(x) for x in v])

    def ptrs(v):
        return (_c.c_void_p * max(nb, 1))(*[_ptr(x) for x in v])

    args = [chars(transa), chars(transb), i64(m), i64(n), i64(k), zs(alpha), ptrs(A), i64(lda),
            ptrs(B), i64(ldb), zs(beta), ptrs(C), i64(ldc)]
    sl = None if slices is None else (_c.c_int * max(nb, 1))(*[int(x) for x in slices])
    used = (_c.c_int * max(nb, 1))()
    rc = library().ozaki_zgemm_batched(*[_c.cast(a, _c.c_void_p) for a in args], nb,
                                       None if sl is None else _c.cast(sl, _c.c_void_p),
                                       _c.cast(used, _c.c_void_p))
    if slices_used is not None:
        slices_used[:] = [used[i] for i in range(nb)]
    return rc


def ozaki_batched_graphs(on: bool) -> int:
    return library().ozaki_batched_graphs(1 if on else 0)


def ozaki_batched_cache_clear() -> int:
    return library().ozaki_batched_cache_clear()


def ozaki_probe(kind, transa, transb, m, n, k, A, lda, B, ldb, C, ldc, nvec, seed, est) -> int:
    _bind_stream()
    return library().ozaki_probe(_ch(kind), _ch(transa), _ch(transb), m, n, k, _ptr(A), lda, _ptr(B),
                                 ldb, _ptr(C), ldc, int(nvec), int(seed) & (2 ** 64 - 1), _ptr(est))


MLP_PARAMS = 24961


def ozaki_features(kind, transa, transb, m, n, k, A, lda, B, ldb, feat) -> int:
    _bind_stream()
    return library().ozaki_features(_ch(kind), _ch(transa), _ch(transb), m, n, k, _ptr(A), lda,
                                    _ptr(B), ldb, _ptr(feat))


def ozaki_mlp_state_bytes() -> int:
    return library().ozaki_mlp_state_bytes()


def ozaki_mlp_scratch_bytes(batch) -> int:
    return library().ozaki_mlp_scratch_bytes(int(batch))


def ozaki_mlp_init(state, seed) -> int:
    _bind_stream()
    return library().ozaki_mlp_init(_ptr(state), int(seed) & (2 ** 64 - 1))


def ozaki_mlp_refresh(state) -> int:
    _bind_stream()
    return library().ozaki_mlp_refresh(_ptr(state))


def ozaki_mlp_forward(state, batch, X, y, scratch) -> int:
    _bind_stream()
    return library().ozaki_mlp_forward(_ptr(state), int(batch), _ptr(X), _ptr(y), _ptr(scratch))


def ozaki_mlp_backward(state, batch, y, target, under_weight, loss, scratch) -> int:
    _bind_stream()
    return library().ozaki_mlp_backward(_ptr(state), int(batch), _ptr(y), _ptr(target),
                                         float(under_weight), _ptr(loss), _ptr(scratch))


def ozaki_mlp_adam(state, lr, beta1, beta2, eps, step) -> int:
    _bind_stream()
    return library().ozaki_mlp_adam(_ptr(state), float(lr), float(beta1), float(beta2), float(eps),
                                    int(step))


def ozaki_load_selector(params, margin, target, kappa) -> int:
    """params: a host sequence / numpy array of MLP_PARAMS floats."""
    import numpy as np
    p = np.ascontiguousarray(np.asarray(params, dtype=np.float32))
    if p.size != MLP_PARAMS:
        return -1
    return library().ozaki_load_selector(p.ctypes.data_as(_c.c_void_p), float(margin), float(target),
                                         float(kappa))


def ozaki_autotune(kind, m, n, k, slices, reps=10):
    """(status, best tuning id, ms per launch of the best id)."""
    _bind_stream()
    best = _c.c_int(-1)
    ms = _c.c_double(0.0)
    rc = library().ozaki_autotune(_ch(kind), m, n, k, int(slices), int(reps),
                                  _c.cast(_c.pointer(best), _c.c_void_p),
                                  _c.cast(_c.pointer(ms), _c.c_void_p))
    return rc, best.value, ms.value


def ozaki_tune_set(kind, m, n, k, slices, tune_id) -> int:
    return library().ozaki_tune_set(_ch(kind), m, n, k, int(slices), int(tune_id))


def ozaki_tune_get(kind, m, n, k, slices) -> int:
    return library().ozaki_tune_get(_ch(kind), m, n, k, int(slices))


def ozaki_tune_configs() -> int:
    return library().ozaki_tune_configs()


def ozaki_tune_save(path) -> int:
    return library().ozaki_tune_save(None if path is None else os.fsencode(path))


def ozaki_tune_load(path) -> int:
    return library().ozaki_tune_load(None if path is None else os.fsencode(path))


def ozaki_tune_clear() -> int:
    return library().ozaki_tune_clear()


def ozaki_set_stream(stream) -> int:
    return library().ozaki_set_stream(_c.c_void_p(stream if isinstance(stream, int) or stream is None
                                                  else stream.cuda_stream))


def ozaki_set_workspace(ptr, nbytes: int) -> int:
    return library().ozaki_set_workspace(_ptr(ptr), int(nbytes))


def ozaki_workspace_bytes(kind, m, n, k, slices) -> int:
    return library().ozaki_workspace_bytes(_ch(kind), m, n, k, int(slices))


PHASES = ("scan", "split", "gemm", "recon")


def ozaki_timing_enable(on: bool) -> int:
    return library().ozaki_timing_enable(1 if on else 0)


def ozaki_timing_read():
    """(status, {phase: total ms}, calls) since the last read."""
    ms = (_c.c_double * len(PHASES))()
    calls = _c.c_int64(0)
    rc = library().ozaki_timing_read(_c.cast(ms, _c.c_void_p), _c.cast(_c.pointer(calls), _c.c_void_p))
    return rc, {p: ms[i] for i, p in enumerate(PHASES)}, calls.value


def ozaki_finalize() -> int:
    return library().ozaki_finalize()


def ozaki_status_string(status: int) -> str:
    try:
        return library().ozaki_status_string(int(status)).decode()
    except OzakiUnavailable:
        return "library not built"


def ozaki_debug_exponents(kind, side, trans, rows, L, X, ldx, exps, flags) -> int:
    _bind_stream()
    return library().ozaki_debug_exponents(_ch(kind), _ch(side), _ch(trans), rows, L, _ptr(X), ldx,
                                           _ptr(exps), _ptr(flags))


def ozaki_debug_split(kind, side, trans, rows, L, X, ldx, slices, digits) -> int:
    _bind_stream()
    return library().ozaki_debug_split(_ch(kind), _ch(side), _ch(trans), rows, L, _ptr(X), ldx,
                                       int(slices), _ptr(digits))


def ozaki_debug_diagonals(kind, transa, transb, m, n, k, A, lda, B, ldb, slices, S) -> int:
    _bind_stream()
    return library().ozaki_debug_diagonals(_ch(kind), _ch(transa), _ch(transb), m, n, k, _ptr(A),
                                           lda, _ptr(B), ldb, int(slices), _ptr(S))


def matmul(A, B, slices: int = 7, alpha=1.0, beta=0.0, C=None, native: bool = False,
           moduli: int | None = None):
    """C <- alpha A @ B + beta C for row-major torch CUDA tensors (float64 or
    complex128, 2-D, unit stride along rows). `moduli` selects the Ozaki-II
    path with that many moduli instead of Ozaki-I with `slices` slices.

    A row-major m x k tensor is the column-major k x m matrix A^T, so the call
    computes C^T = B^T A^T in BLAS terms; the emulation is symmetric under this
    transposition (exponents and slices are per row of A and per column of B
    either way), so the result is the same as for the column-major problem.
    """
    import torch
    if A.dim() != 2 or B.dim() != 2 or A.shape[1] != B.shape[0]:
        raise ValueError("shapes do not chain")
    if A.dtype != B.dtype or A.dtype not in (torch.float64, torch.complex128):
        raise TypeError("A and B must both be float64 or both complex128")
    if A.stride(1) != 1 or B.stride(1) != 1:
        raise ValueError("rows must be unit stride")
    m, k = A.shape
    n = B.shape[1]
    if C is None:
        C = torch.empty((m, n), dtype=A.dtype, device=A.device)
        beta = 0.0
    elif C.shape != (m, n) or C.dtype != A.dtype or C.stride(1) != 1:
        raise ValueError("bad C")
    lda, ldb, ldc = max(1, A.stride(0)), max(1, B.stride(0)), max(1, C.stride(0))
    cplx = A.dtype == torch.complex128
    if native:
        fn = ozaki_native_zgemm if cplx else ozaki_native_dgemm
        rc = fn("N", "N", n, m, k, alpha, B, ldb, A, lda, beta, C, ldc)
    elif moduli is not None:
        fn = ozaki2_zgemm if cplx else ozaki2_dgemm
        rc = fn("N", "N", n, m, k, alpha, B, ldb, A, lda, beta, C, ldc, moduli)
    else:
        fn = ozaki_zgemm if cplx else ozaki_dgemm
        rc = fn("N", "N", n, m, k, alpha, B, ldb, A, lda, beta, C, ldc, slices)
    if rc != 0:
        raise OzakiError(rc, fn.__name__)
    return C
