"""Ozaki-I emulation of FP64 and complex-FP64 GEMM: the plain CPU model.

TEST INFRASTRUCTURE ONLY (see the package docstring). Never used by the GPU path.

The paper (Section 2.2, GEMM Emulation on Integer Matrix Multiplication Unit)
describes Ozaki-I in one sentence: the FP64 inputs are split into
lower-precision slices according to their significant bits after aligning
exponents, the slices are multiplied with low-precision matrix products, and the
partial products are accumulated in higher precision. Its Section 3.2 and
Section 4 (Discussion) use the number of mantissa bits (31, 39, 47, 55, 63) as
the accuracy knob and report that the error falls exponentially as it grows.
Nothing more is specified, so every detail below is a reading, stated here and
kept identical in the GPU path:

R1 exponent alignment (step O2). For row i of op(A),
   mu_i = max_l max(|Re a_il|, |Im a_il|)  (just |a_il| for real data), and
   e_i is the frexp exponent of mu_i: mu_i = f * 2^e_i with f in [1/2, 1).
   A zero row takes e_i = 0. A row holding Inf or NaN is flagged. Column j of
   op(B) gets f_j the same way. Real and imaginary parts share the exponent.
R2 slicing (step O3), "trunc-7": x = a * 2^-e_i (exact), then for p = 1..s
   d_p = trunc(r * 2^(7p)), r <- r - d_p * 2^(-7p), starting from r = x.
   Every digit is an integer in [-127, 127]; the s digits hold the top 7s
   bits of |x| with the sign of x. Re and Im are split separately.
R3 slice products (step O4): the triangle of pairs p + q <= s + 1. Diagonal
   t = 2..s+1 is S_t = sum_{p+q=t} SA_p SB_q, an exact integer matrix. Complex
   data uses four real products per pair:
   Sr_t = sum (Ar_p Br_q - Ai_p Bi_q), Si_t = sum (Ar_p Bi_q + Ai_p Br_q).
   ``mode="full"`` keeps every pair p, q <= s (diagonals up to 2s).
R4 recombination (step O5): acc = 0; for t = 2, 3, ... (largest weight first)
   acc = RN(acc + S_t * 2^(-7t)); then P_ij = acc * 2^(e_i + f_j) (ldexp).
R5 alpha/beta follow reference BLAS, every product and sum rounded on its own
   (no fused multiply-add): real C = RN(RN(alpha P) + RN(beta C)); complex
   Re = (ar Pr - ai Pi) + (br Cr - bi Ci), Im = (ar Pi + ai Pr) + (br Ci + bi Cr)
   evaluated left to right in that grouping. beta = 0 means C is not read.
   alpha = 0 or k = 0 gives C = beta C (C untouched when beta = 1).
R6 non-finite input: every C_ij whose row of op(A) or column of op(B) holds
   Inf or NaN is set to NaN (NaN + NaN i for complex).
"""
from __future__ import annotations

import numpy as np

S_MAX = 12          # the slice counts the model is defined for: 1..S_MAX
DIGIT_BITS = 7      # bits per slice (trunc-7 reading R2)


# ----------------------------------------------------------------- step O1
def op(X: np.ndarray, trans: str) -> np.ndarray:
    """op(X) for a BLAS trans character: 'N' as is, 'T' transpose, 'C'
    conjugate transpose ('C' equals 'T' for real data)."""
    t = trans.upper()
    if t == "N":
        return X
    if t == "T":
        return X.T
    if t == "C":
        return np.conj(X.T) if np.iscomplexobj(X) else X.T
    raise ValueError(f"bad trans {trans!r}")


# ----------------------------------------------------------------- step O2
def _magnitude(X: np.ndarray) -> np.ndarray:
    if np.iscomplexobj(X):
        return np.maximum(np.abs(X.real), np.abs(X.imag))
    return np.abs(X)


def _finite(X: np.ndarray) -> np.ndarray:
    if np.iscomplexobj(X):
        return np.isfinite(X.real) & np.isfinite(X.imag)
    return np.isfinite(X)


def row_exponents(X: np.ndarray):
    """Reading R1 on the rows of X (rows x L).

    Returns (e, bad): e[i] is the frexp exponent of the row maximum (0 for a
    zero row or a flagged row), bad[i] is True when the row holds Inf or NaN.
    """
    fin = _finite(X)
    bad = ~np.all(fin, axis=1) if X.shape[1] > 0 else np.zeros(X.shape[0], bool)
    mag = np.where(fin, _magnitude(X), 0.0)
    mu = mag.max(axis=1) if X.shape[1] > 0 else np.zeros(X.shape[0])
    _, e = np.frexp(mu)                     # frexp(0) = (0, 0)
    e = e.astype(np.int64)
    e[bad] = 0
    return e, bad


def col_exponents(Y: np.ndarray):
    """Reading R1 on the columns of Y (L x cols)."""
    return row_exponents(Y.T)


# ----------------------------------------------------------------- step O3
def split(X: np.ndarray, e: np.ndarray, s: int, rows_bad: np.ndarray | None = None) -> np.ndarray:
    """Reading R2: the s trunc-7 digit planes of the real matrix X (rows x L),
    row i scaled by 2^-e[i]. Returns int8 of shape (s, rows, L); plane p-1 holds
    d_p. Rows flagged in ``rows_bad`` are split as zeros.

    ldexp(a, -e) is exact except when the scaled value falls below 2^-1022,
    and such a value has no nonzero digit above 2^(-7 S_MAX).
    """
    if not 1 <= s <= S_MAX:
        raise ValueError("s out of range")
    X = np.asarray(X, dtype=np.float64)
    if rows_bad is not None and rows_bad.any():
        X = X.copy()
        X[rows_bad] = 0.0
    r = np.ldexp(X, (-e).astype(np.int32)[:, None])
    D = np.empty((s,) + X.shape, dtype=np.int8)
    for p in range(1, s + 1):
        d = np.trunc(np.ldexp(r, DIGIT_BITS * p))
        r = r - np.ldexp(d, -DIGIT_BITS * p)       # exact: removes the top bits of r
        D[p - 1] = d.astype(np.int8)
    return D


def split_operand(X: np.ndarray, e: np.ndarray, s: int, rows_bad=None):
    """Split a real or complex operand given per-row exponents.

    Returns a tuple of digit planes: (D,) for real data, (D_re, D_im) for
    complex data, each int8 of shape (s, rows, L).
    """
    if np.iscomplexobj(X):
        return (split(X.real, e, s, rows_bad), split(X.imag, e, s, rows_bad))
    return (split(X, e, s, rows_bad),)


# ----------------------------------------------------------------- step O4
def pairs(s: int, mode: str = "triangle"):
    """Slice pairs (p, q) kept by the model, grouped by diagonal t = p + q."""
    if mode == "triangle":
        tmax = s + 1
    elif mode == "full":
        tmax = 2 * s
    else:
        raise ValueError(mode)
    out = {}
    for t in range(2, tmax + 1):
        out[t] = [(p, t - p) for p in range(max(1, t - s), min(s, t - 1) + 1)]
    return out


def _cplx(re_part, im_part):
    """Complex array from two real arrays without arithmetic (x + 1j*y would
    compute 0*y terms and can flip the sign of a zero or make NaN from Inf)."""
    out = np.empty(np.shape(re_part), dtype=np.complex128)
    out.real = re_part
    out.imag = im_part
    return out


def _imat(D):
    # Integer digit planes as float64: every product is at most 127^2 and every
    # partial sum below is far under 2^53 (k * s * 127^2 < 2^53 for any k below
    # 4e10), so a float64 matrix product on these integer-valued matrices is exact
    # whatever order or fused operations the host BLAS uses.
    return D.astype(np.float64)


def diagonals(DA, DB, s: int, mode: str = "triangle"):
    """Reading R3: exact diagonal sums S_t.

    DA are the digit planes of the rows of op(A) (tuple from split_operand on
    op(A)); DB are the digit planes of the columns of op(B) split as rows of
    op(B)^T, so DB[.][q-1] has shape (n, k). Returns a dict t -> S_t (float64
    holding exact integers, complex128 for complex data).
    """
    out = {}
    complex_ = len(DA) == 2
    for t, plist in pairs(s, mode).items():
        if complex_:
            Ar, Ai = DA
            Br, Bi = DB
            sr = 0.0
            si = 0.0
            for p, q in plist:
                sr = sr + (_imat(Ar[p - 1]) @ _imat(Br[q - 1]).T - _imat(Ai[p - 1]) @ _imat(Bi[q - 1]).T)
                si = si + (_imat(Ar[p - 1]) @ _imat(Bi[q - 1]).T + _imat(Ai[p - 1]) @ _imat(Br[q - 1]).T)
            out[t] = _cplx(sr, si)
        else:
            (A,), (B,) = DA, DB
            acc = 0.0
            for p, q in plist:
                acc = acc + _imat(A[p - 1]) @ _imat(B[q - 1]).T
            out[t] = acc
    return out


# ----------------------------------------------------------------- step O5
def recombine(S: dict, e: np.ndarray, f: np.ndarray) -> np.ndarray:
    """Reading R4: acc = RN(acc + S_t 2^-7t) for increasing t, then scale by
    2^(e_i + f_j). Real and imaginary parts are recombined separately."""
    ts = sorted(S)
    sample = S[ts[0]]
    complex_ = np.iscomplexobj(sample)
    scale = (e[:, None] + f[None, :]).astype(np.int32)

    def one(parts):
        acc = np.zeros(sample.shape, dtype=np.float64)
        for t in ts:
            acc = acc + np.ldexp(parts[t], -DIGIT_BITS * t)   # ldexp exact: S_t < 2^53
        return np.ldexp(acc, scale)

    if complex_:
        re = one({t: S[t].real for t in ts})
        im = one({t: S[t].imag for t in ts})
        return _cplx(re, im)
    return one(S)


def _cmul_parts(ar, ai, xr, xi):
    """(ar + ai i)(xr + xi i) with each product and sum rounded on its own."""
    return ar * xr - ai * xi, ar * xi + ai * xr


def apply_alpha_beta(P, alpha, beta, C):
    """Reading R5 for the product P (the emulated op(A) op(B))."""
    if np.iscomplexobj(P):
        a = complex(alpha)
        pr, pi = _cmul_parts(a.real, a.imag, P.real, P.imag)
        if complex(beta) == 0:
            return _cplx(pr, pi)
        b = complex(beta)
        cr, ci = _cmul_parts(b.real, b.imag, C.real, C.imag)
        return _cplx(pr + cr, pi + ci)
    if beta == 0:
        return alpha * P
    return alpha * P + beta * C


def scale_only(beta, C, shape, complex_: bool):
    """alpha = 0 or k = 0: C <- beta C, with beta = 0 giving zeros (C not
    read) and beta = 1 leaving C untouched."""
    dt = np.complex128 if complex_ else np.float64
    if beta == 0:
        return np.zeros(shape, dtype=dt)
    if beta == 1:
        return np.array(C, dtype=dt, copy=True)
    if complex_:
        b = complex(beta)
        cr, ci = _cmul_parts(b.real, b.imag, C.real, C.imag)
        return _cplx(cr, ci)
    return beta * C


# ----------------------------------------------------------------- whole call
def ozaki_gemm(transa: str, transb: str, A, B, s: int, alpha=1.0, beta=0.0, C=None,
               mode: str = "triangle"):
    """C <- alpha op(A) op(B) + beta C under the Ozaki-I model (steps O1..O5).

    A, B, C are the mathematical matrices (numpy arrays; layout is irrelevant
    here). Complex data (either operand complex) uses the complex model.
    Returns the new C.
    """
    complex_ = np.iscomplexobj(A) or np.iscomplexobj(B) or np.iscomplexobj(alpha) \
        or np.iscomplexobj(beta)
    dt = np.complex128 if complex_ else np.float64
    opA = np.asarray(op(np.asarray(A, dtype=dt), transa))
    opB = np.asarray(op(np.asarray(B, dtype=dt), transb))
    m, k = opA.shape
    k2, n = opB.shape
    if k != k2:
        raise ValueError("inner dimensions differ")
    if m == 0 or n == 0:
        return np.zeros((m, n), dtype=dt)
    if alpha == 0 or k == 0:
        return scale_only(beta, C, (m, n), complex_)
    e, bad_r = row_exponents(opA)
    f, bad_c = col_exponents(opB)
    DA = split_operand(opA, e, s, bad_r)
    DB = split_operand(opB.T, f, s, bad_c)
    S = diagonals(DA, DB, s, mode)
    P = recombine(S, e, f)
    out = apply_alpha_beta(P, alpha, beta, C)
    bad = bad_r[:, None] | bad_c[None, :]
    if bad.any():
        out = out.copy()
        out[bad] = complex(np.nan, np.nan) if complex_ else np.nan
    return out
