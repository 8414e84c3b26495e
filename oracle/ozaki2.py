"""Ozaki-II emulation of FP64 and complex-FP64 GEMM: the plain CPU model.

TEST INFRASTRUCTURE ONLY (see the package docstring). Never used by the GPU path.

The paper's Section 2.2 describes Ozaki-II in one sentence: the floating-point
matrices are converted into integers, multiplied with several smaller matrix
products modulo pairwise coprime moduli, and the result is reconstructed with
the Chinese Remainder Theorem; its Section 3 sets the accuracy by the number of
moduli (10, 12, 14, 16, 18). The readings below are this build's, kept
identical in the GPU path:

Q1 moduli: the N largest pairwise coprime integers <= 256, taken greedily from
   256 downwards (256, 255, 253, 251, 247, 241, 239, 233, 229, 227, 223, 217,
   211, 199, 197, 193, 191, 181, 179, 173, ...). A residue is the
   representative of x mod m_k in [-floor(m_k/2), ceil(m_k/2) - 1], which fits
   INT8. N ranges over 2..20 (M = prod m_k < 2^160).
Q2 integer conversion: with e_i, f_j the row/column exponents of reading R1
   (frexp exponent of the largest |Re|, |Im| of row i of op(A), column j of
   op(B)), A'_il = trunc(a_il 2^(beta - e_i)) and B'_lj = trunc(b_lj
   2^(beta - f_j)) (Re and Im separately), so |A'|, |B'| < 2^beta, with
   beta = min(63, floor((floor(log2 M) - 1 - ceil(log2 K')) / 2)),
   K' = k (real) or 2k (complex). Then every entry of A'B' is below
   K' 2^(2 beta) <= M/2 in magnitude. beta < 1 (too few moduli for K') is an
   error.
Q3 modular products: C_k = (A' mod m_k)(B' mod m_k) as exact integer
   matrices (residues below 129 in magnitude: sums below 2^31 for K' <= 2^17);
   complex data as one real product (K' = 2k: a'' = (Re, Im) along the
   contraction, column j of B split into (Re, -Im) and (Im, Re)).
Q4 reconstruction: the unique integer c in [-M/2, M/2) with c = C_k mod m_k
   for every k (Garner's mixed-radix form with balanced digits); it equals the
   exact product A'B' by Q2.
Q5 result: P_ij = RN(c_ij) * 2^(e_i + f_j - 2 beta) (one rounding of the exact
   integer, then a power-of-two scaling), then alpha/beta and non-finite
   inputs as readings R5 and R6 of the Ozaki-I model.
"""
from __future__ import annotations

import math

import numpy as np

from .ozaki import _cplx, apply_alpha_beta, col_exponents, op, row_exponents, scale_only

N_MIN, N_MAX = 2, 20
K_MAX = 1 << 17          # contraction length K' with exact INT32 modular sums


def moduli(n: int):
    """Reading Q1: the n largest pairwise coprime integers <= 256."""
    if not N_MIN <= n <= N_MAX:
        raise ValueError("moduli count out of range")
    out = []
    c = 256
    while len(out) < n:
        if all(math.gcd(c, x) == 1 for x in out):
            out.append(c)
        c -= 1
    return out


def beta_bits(n: int, kprime: int) -> int:
    """Reading Q2: bits kept per operand entry below its row/column maximum."""
    M = math.prod(moduli(n))
    lk = max(0, math.ceil(math.log2(max(1, kprime))))
    bet = min(63, (M.bit_length() - 1 - 1 - lk) // 2)
    if bet < 1:
        raise ValueError("too few moduli for this contraction length")
    return bet


def to_integers(X: np.ndarray, e: np.ndarray, beta: int, rows_bad=None) -> np.ndarray:
    """Reading Q2 on the rows of the real matrix X: trunc(x 2^(beta - e_i)) as
    Python ints (object array; exact for beta up to 63)."""
    X = np.asarray(X, dtype=np.float64)
    out = np.empty(X.shape, dtype=object)
    for i in range(X.shape[0]):
        for l in range(X.shape[1]):
            x = float(X[i, l])
            if rows_bad is not None and rows_bad[i]:
                x = 0.0
            q = abs(x)
            # |x| = mant * 2^ex exactly; trunc(|x| 2^(beta - e)) by integer shifts
            mant, ex = math.frexp(q)
            mi = int(mant * (1 << 53))           # exact: 53-bit significand
            sh = ex - 53 + beta - int(e[i])
            v = mi << sh if sh >= 0 else mi >> (-sh)
            out[i, l] = -v if x < 0 else v
    return out


def residue(x: int, m: int) -> int:
    """Balanced representative of x mod m (reading Q1)."""
    r = x % m
    return r - m if r >= (m + 1) // 2 else r


def residues(Xi: np.ndarray, m: int) -> np.ndarray:
    return np.vectorize(lambda v: residue(int(v), m), otypes=[np.int64])(Xi)


def garner(res, mods):
    """Reading Q4: the integer in [-M/2, M/2) with the given residues, by
    Garner's mixed-radix algorithm with balanced digits."""
    digits = []
    for k, mk in enumerate(mods):
        t = res[k]
        for j in range(k):
            t = ((t - digits[j]) * pow(mods[j], -1, mk)) % mk
        digits.append(residue(t, mk))
    x = 0
    for k in range(len(mods) - 1, -1, -1):
        x = x * mods[k] + digits[k]
    return x


def _integer_operands(opA, opB, n):
    """Q2 for op(A) (m x k) and op(B) (k x n), complex as one real product."""
    cplx = np.iscomplexobj(opA)
    e, bad_r = row_exponents(opA)
    f, bad_c = col_exponents(opB)
    k = opA.shape[1]
    kprime = 2 * k if cplx else k
    beta = beta_bits(n, kprime)
    if cplx:
        ar = to_integers(opA.real, e, beta, bad_r)
        ai = to_integers(opA.imag, e, beta, bad_r)
        br = to_integers(opB.real.T, f, beta, bad_c)       # rows = columns j
        bi = to_integers(opB.imag.T, f, beta, bad_c)
        m_, n_ = opA.shape[0], opB.shape[1]
        Ap = np.empty((m_, 2 * k), dtype=object)
        Ap[:, 0::2], Ap[:, 1::2] = ar, ai
        Bp = np.empty((2 * n_, 2 * k), dtype=object)
        Bp[0::2, 0::2], Bp[0::2, 1::2] = br, -bi
        Bp[1::2, 0::2], Bp[1::2, 1::2] = bi, br
    else:
        Ap = to_integers(opA, e, beta, bad_r)
        Bp = to_integers(opB.T, f, beta, bad_c)
    return Ap, Bp, e, f, bad_r, bad_c, beta


def modular_products(Ap, Bp, mods):
    """Reading Q3: exact INT8-residue products (int64 suffices)."""
    out = []
    for m in mods:
        RA = residues(Ap, m)
        RB = residues(Bp, m)
        out.append(RA @ RB.T)
    return out


def ozaki2_gemm(transa: str, transb: str, A, B, n_moduli: int, alpha=1.0, beta=0.0, C=None):
    """C <- alpha op(A) op(B) + beta C under the Ozaki-II model (Q1..Q5)."""
    complex_ = np.iscomplexobj(A) or np.iscomplexobj(B) or np.iscomplexobj(alpha) \
        or np.iscomplexobj(beta)
    dt = np.complex128 if complex_ else np.float64
    opA = np.asarray(op(np.asarray(A, dtype=dt), transa))
    opB = np.asarray(op(np.asarray(B, dtype=dt), transb))
    m, k = opA.shape
    n = opB.shape[1]
    if m == 0 or n == 0:
        return np.zeros((m, n), dtype=dt)
    if alpha == 0 or k == 0:
        return scale_only(beta, C, (m, n), complex_)
    mods = moduli(n_moduli)
    Ap, Bp, e, f, bad_r, bad_c, bet = _integer_operands(opA, opB, n_moduli)
    if Ap.shape[1] > K_MAX:
        raise ValueError("contraction too long for exact INT32 modular sums")
    Cm = modular_products(Ap, Bp, mods)
    rows, cols = Ap.shape[0], Bp.shape[0]
    P = np.empty((rows, cols))
    for i in range(rows):
        for jp in range(cols):
            c = garner([int(Ck[i, jp]) for Ck in Cm], mods)
            P[i, jp] = float(c)                                   # RN of the exact integer
    if complex_:
        fr = np.repeat(f, 2)
        Pn = np.ldexp(P, (e[:, None] + fr[None, :] - 2 * bet).astype(np.int32))
        Pc = _cplx(Pn[:, 0::2], Pn[:, 1::2])
    else:
        Pc = np.ldexp(P, (e[:, None] + f[None, :] - 2 * bet).astype(np.int32))
    out = apply_alpha_beta(Pc, alpha, beta, C)
    bad = bad_r[:, None] | bad_c[None, :]
    if bad.any():
        out = out.copy()
        out[bad] = complex(np.nan, np.nan) if complex_ else np.nan
    return out
