"""Ozaki-I with 8-bit balanced slices: the plain CPU model of the "b8" split.

TEST INFRASTRUCTURE ONLY (see the package docstring). Never used by the GPU path.

Section 3.2 of the paper labels the Ozaki-I accuracy modes by mantissa bits
31, 39, 47, 55, 63, i.e. 8s - 1 bits for s = 4..8 INT8 slices: slices that use
all 8 bits of an INT8 rather than 7. The trunc-7 reading R2 (oracle/ozaki.py)
keeps 7 bits per slice. This module is the 8-bit variant, with these readings
(B1..B4 replace R2..R4; exponents R1, alpha/beta R5 and the non-finite rule R6
are those of oracle/ozaki.py):

B1 integer: x = a * 2^-e (exponents as R1), X = trunc(x * 2^(8s - 2)), an
   integer with |X| < 2^(8s - 2). s <= 8 (X fits 62 bits).
B2 digits: the balanced base-256 expansion X = sum_{p=1..s} d_p 256^(s-p)
   with every d_p in [-128, 127], taken from the least significant digit
   upwards: d = ((X + 128) mod 256) - 128, X <- (X - d) / 256. It exists and
   is unique because |X| < 2^(8s-2) lies inside the range of s balanced
   digits. Slice p carries weight 2^(2 - 8p): 6 bits and the sign in the
   first slice, 8 in every other, 8s - 2 bits in all.
B3 slice products: the triangle p + q <= s + 1 as R3; S_t = sum_{p+q=t}
   SA_p SB_q exact. Complex data: the digits of -x are not the negated
   digits of x when some digit is -128, so the real part uses the digit
   planes of -Im b directly: Sr_t = sum (Ar_p Br_q + Ai_p Nb_q) with
   Nb = digits(-Im b), Si_t = sum (Ar_p Bi_q + Ai_p Br_q). (This is the
   construction the GPU path runs: B' rows (Re, -Im) and (Im, Re) are split
   as they stand.)
B4 recombination: acc = 0; acc = RN(acc + S_t * 2^(4 - 8t)) for t = 2..s+1,
   then P = acc * 2^(e_i + f_j).
"""
from __future__ import annotations

import numpy as np

from .ozaki import (_cplx, _imat, apply_alpha_beta, col_exponents, op, pairs, row_exponents,
                    scale_only)

S_MAX_B8 = 8


def integers(X: np.ndarray, e: np.ndarray, s: int, rows_bad=None) -> np.ndarray:
    """Reading B1: trunc(x 2^(8s-2)) per entry of the real matrix X, row i
    scaled by 2^-e[i], as int64 (exact: scaling by powers of two and
    truncation of a float64 below 2^62)."""
    if not 1 <= s <= S_MAX_B8:
        raise ValueError("s out of range for the 8-bit split")
    X = np.asarray(X, dtype=np.float64)
    if rows_bad is not None and rows_bad.any():
        X = X.copy()
        X[rows_bad] = 0.0
    x = np.ldexp(X, (-e).astype(np.int32)[:, None])
    return np.trunc(np.ldexp(x, 8 * s - 2)).astype(np.int64)


def digits(Xi: np.ndarray, s: int) -> np.ndarray:
    """Reading B2: balanced base-256 digits of the int64 array Xi; plane p-1
    holds d_p (int16 to keep -128 visible in checks, values in [-128, 127])."""
    X = np.array(Xi, dtype=np.int64, copy=True)
    D = np.empty((s,) + X.shape, dtype=np.int16)
    for p in range(s, 0, -1):
        d = ((X + 128) & 255) - 128
        D[p - 1] = d
        X = (X - d) >> 8
    if np.any(X != 0):
        raise ValueError("integer outside the range of s balanced digits")
    return D


def split_b8(X: np.ndarray, e: np.ndarray, s: int, rows_bad=None) -> np.ndarray:
    return digits(integers(X, e, s, rows_bad), s)


def diagonals_b8(DA, DB, s: int):
    """Reading B3. DA: (D,) or (Ar, Ai) digit planes of the rows of op(A); DB:
    (D,) or (Br, Bi, Nb) of the columns of op(B) (Nb = digits of -Im)."""
    out = {}
    complex_ = len(DA) == 2
    for t, plist in pairs(s).items():
        if complex_:
            Ar, Ai = DA
            Br, Bi, Nb = DB
            sr = 0.0
            si = 0.0
            for p, q in plist:
                sr = sr + (_imat(Ar[p - 1]) @ _imat(Br[q - 1]).T + _imat(Ai[p - 1]) @ _imat(Nb[q - 1]).T)
                si = si + (_imat(Ar[p - 1]) @ _imat(Bi[q - 1]).T + _imat(Ai[p - 1]) @ _imat(Br[q - 1]).T)
            out[t] = _cplx(sr, si)
        else:
            (A,), (B,) = DA, DB
            acc = 0.0
            for p, q in plist:
                acc = acc + _imat(A[p - 1]) @ _imat(B[q - 1]).T
            out[t] = acc
    return out


def recombine_b8(S: dict, e: np.ndarray, f: np.ndarray) -> np.ndarray:
    """Reading B4 (largest weight first, one rounding per addition)."""
    ts = sorted(S)
    sample = S[ts[0]]
    scale = (e[:, None] + f[None, :]).astype(np.int32)

    def one(parts):
        acc = np.zeros(sample.shape, dtype=np.float64)
        for t in ts:
            acc = acc + np.ldexp(parts[t], 4 - 8 * t)   # exact scaling of an integer < 2^53
        return np.ldexp(acc, scale)

    if np.iscomplexobj(sample):
        return _cplx(one({t: S[t].real for t in ts}), one({t: S[t].imag for t in ts}))
    return one(S)


def ozaki_gemm_b8(transa: str, transb: str, A, B, s: int, alpha=1.0, beta=0.0, C=None):
    """C <- alpha op(A) op(B) + beta C under the 8-bit balanced model."""
    complex_ = np.iscomplexobj(A) or np.iscomplexobj(B) or np.iscomplexobj(alpha) \
        or np.iscomplexobj(beta)
    dt = np.complex128 if complex_ else np.float64
    opA = np.asarray(op(np.asarray(A, dtype=dt), transa))
    opB = np.asarray(op(np.asarray(B, dtype=dt), transb))
    m, k = opA.shape
    if opB.shape[0] != k:
        raise ValueError("inner dimensions differ")
    n = opB.shape[1]
    if m == 0 or n == 0:
        return np.zeros((m, n), dtype=dt)
    if alpha == 0 or k == 0:
        return scale_only(beta, C, (m, n), complex_)
    if not 1 <= s <= S_MAX_B8:
        raise ValueError("s out of range for the 8-bit split")
    e, bad_r = row_exponents(opA)
    f, bad_c = col_exponents(opB)
    BT = opB.T
    if complex_:
        DA = (split_b8(opA.real, e, s, bad_r), split_b8(opA.imag, e, s, bad_r))
        DB = (split_b8(BT.real, f, s, bad_c), split_b8(BT.imag, f, s, bad_c),
              split_b8(-BT.imag, f, s, bad_c))
    else:
        DA = (split_b8(opA, e, s, bad_r),)
        DB = (split_b8(BT, f, s, bad_c),)
    P = recombine_b8(diagonals_b8(DA, DB, s), e, f)
    out = apply_alpha_beta(P, alpha, beta, C)
    bad = bad_r[:, None] | bad_c[None, :]
    if bad.any():
        out = out.copy()
        out[bad] = complex(np.nan, np.nan) if complex_ else np.nan
    return out
