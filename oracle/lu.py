"""Blocked LU with partial pivoting and the inverse, with the trailing updates
taken from a GEMM model: the plain CPU model of ozaki_zgetrf / ozaki_zgetri.

TEST INFRASTRUCTURE ONLY (see the package docstring). Never used by the GPU path.

The paper's solver inverts the multiple-scattering matrix by LU, and ZGEMM and
ZTRSM take most of its run time (Section 3.2); the emulated ZGEMM enters as
the trailing update of a blocked factorization. The readings, shared with the
GPU path:

L1 arithmetic: every complex product is (ar br - ai bi, ar bi + ai br) and
   every quotient a / b is ((ar br + ai bi) / d, (ai br - ar bi) / d) with
   d = br br + bi bi, each real operation rounded on its own. The LU
   multipliers are products with the pivot's reciprocal, l = a (1 / p) with
   1 / p = (pr / d, (-pi) / d), as the reference LAPACK's unblocked
   factorization scales a column by the reciprocal of its pivot.
L2 pivoting: in column c the pivot is the first row of rows c..n-1 with the
   largest |Re| + |Im| (the measure of the reference LAPACK's izamax; a NaN
   counts as the largest, as numpy's argmax takes it); rows c and pivot are
   exchanged.
L3 factorization (right-looking, panels of nb columns): per column of the
   panel, pivot and exchange within the panel columns, multipliers
   l_i = a_ic (1 / a_cc) stored in place, a_ik -= l_i a_ck for the later panel
   columns; then the panel's exchanges on all other columns; U12 = L11^-1 A12
   by forward substitution (x_r -= l_rk x_k for k = 0..r-1); then
   A22 <- update(A22, L21, U12), the GEMM model C - A B.
L4 inverse: X = P I (the exchanges applied in order to the identity); block
   rows top down X_i = L_ii^-1 X_i, X_below <- update(X_below, L_below,i, X_i);
   then bottom up X_i = U_ii^-1 X_i (for k = nb-1 down to 0: x_k = x_k / u_kk,
   then x_r -= u_rk x_k for r < k; each x_r subtracts its terms in decreasing
   k), X_above <- update(X_above, U_above,i, X_i).
"""
from __future__ import annotations

import numpy as np

from . import ozaki, ozaki_b8


def _zmul(ar, ai, br, bi):
    return ar * br - ai * bi, ar * bi + ai * br


def _zdiv(ar, ai, br, bi):
    d = br * br + bi * bi
    with np.errstate(divide="ignore", invalid="ignore"):   # a zero pivot gives Inf/NaN, as on the GPU
        return (ar * br + ai * bi) / d, (ai * br - ar * bi) / d


def _zrcp(br, bi):
    d = br * br + bi * bi
    with np.errstate(divide="ignore", invalid="ignore"):   # a zero pivot gives NaN, as on the GPU
        return br / d, -bi / d


def update_model(kind: str, slices: int):
    """The GEMM model of the trailing updates: C - A B under the emulation
    (alpha = -1, beta = 1) of slice kind "t7" or "b8", or the plain FP64
    product (kind "native": numpy, not bit-identical to any GPU kernel)."""
    if kind == "native":
        return lambda C, A, B: C - A @ B
    model = ozaki_b8.ozaki_gemm_b8 if kind == "b8" else ozaki.ozaki_gemm
    return lambda C, A, B: model("N", "N", A, B, slices, -1.0, 1.0, C)


def _swap_rows(R, I, a, b, cols):
    if a == b:
        return
    R[[a, b], cols] = R[[b, a], cols]
    I[[a, b], cols] = I[[b, a], cols]


def _trsm_lower_unit(TR, TI, XR, XI):
    w = TR.shape[0]
    for r in range(1, w):
        for k in range(r):
            pr, pi = _zmul(TR[r, k], TI[r, k], XR[k], XI[k])
            XR[r] = XR[r] - pr
            XI[r] = XI[r] - pi


def _trsm_upper(TR, TI, XR, XI):
    w = TR.shape[0]
    for k in range(w - 1, -1, -1):
        XR[k], XI[k] = _zdiv(XR[k], XI[k], TR[k, k], TI[k, k])
        for r in range(k):
            pr, pi = _zmul(TR[r, k], TI[r, k], XR[k], XI[k])
            XR[r] = XR[r] - pr
            XI[r] = XI[r] - pi


def zgetrf(A, nb: int, update):
    """Reading L3. Returns (LU, ipiv, singular) with LU complex, ipiv 0-based."""
    A = np.array(A, dtype=np.complex128)
    n = A.shape[0]
    R, I = A.real.copy(), A.imag.copy()
    ipiv = np.zeros(n, dtype=np.int64)
    singular = False
    for j0 in range(0, n, nb):
        j1 = min(n, j0 + nb)
        panel = slice(j0, j1)
        for c in range(j0, j1):
            v = np.abs(R[c:, c]) + np.abs(I[c:, c])
            piv = c + int(np.argmax(v))
            singular = singular or not v.max() > 0
            ipiv[c] = piv
            _swap_rows(R, I, c, piv, panel)
            rr, ri = _zrcp(R[c, c], I[c, c])
            lr, li = _zmul(R[c + 1:, c], I[c + 1:, c], rr, ri)
            R[c + 1:, c], I[c + 1:, c] = lr, li
            for k in range(c + 1, j1):
                pr, pi = _zmul(lr, li, R[c, k], I[c, k])
                R[c + 1:, k] = R[c + 1:, k] - pr
                I[c + 1:, k] = I[c + 1:, k] - pi
        for c in range(j0, j1):
            _swap_rows(R, I, c, int(ipiv[c]), slice(0, j0))
            _swap_rows(R, I, c, int(ipiv[c]), slice(j1, n))
        if j1 < n:
            XR, XI = R[j0:j1, j1:], I[j0:j1, j1:]
            _trsm_lower_unit(R[j0:j1, j0:j1], I[j0:j1, j0:j1], XR, XI)
            L21 = ozaki._cplx(R[j1:, j0:j1], I[j1:, j0:j1])
            U12 = ozaki._cplx(XR, XI)
            C = update(ozaki._cplx(R[j1:, j1:], I[j1:, j1:]), L21, U12)
            R[j1:, j1:], I[j1:, j1:] = C.real, C.imag
    return ozaki._cplx(R, I), ipiv, singular


def zgetri(LU, ipiv, nb: int, update):
    """Reading L4: the inverse from the factors."""
    LU = np.asarray(LU, dtype=np.complex128)
    n = LU.shape[0]
    LR, LI = LU.real, LU.imag
    XR, XI = np.eye(n), np.zeros((n, n))
    for c in range(n):
        _swap_rows(XR, XI, c, int(ipiv[c]), slice(0, n))
    for i0 in range(0, n, nb):
        i1 = min(n, i0 + nb)
        _trsm_lower_unit(LR[i0:i1, i0:i1], LI[i0:i1, i0:i1], XR[i0:i1], XI[i0:i1])
        if i1 < n:
            C = update(ozaki._cplx(XR[i1:], XI[i1:]), LU[i1:, i0:i1], ozaki._cplx(XR[i0:i1], XI[i0:i1]))
            XR[i1:], XI[i1:] = C.real, C.imag
    for i0 in range((n - 1) // nb * nb, -1, -nb):
        i1 = min(n, i0 + nb)
        _trsm_upper(LR[i0:i1, i0:i1], LI[i0:i1, i0:i1], XR[i0:i1], XI[i0:i1])
        if i0 > 0:
            C = update(ozaki._cplx(XR[:i0], XI[:i0]), LU[:i0, i0:i1], ozaki._cplx(XR[i0:i1], XI[i0:i1]))
            XR[:i0], XI[:i0] = C.real, C.imag
    return ozaki._cplx(XR, XI)
