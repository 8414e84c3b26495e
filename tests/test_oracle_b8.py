"""Pins of the 8-bit balanced split model (CPU): the digits against an
independent top-down construction and exact reconstruction, the integer
conversion against Fractions, the whole model against an exact-rational
evaluation of its definition, exact integer products and the accuracy gain
over the 7-bit split."""
from fractions import Fraction
import math

import numpy as np
import pytest

from oracle import dd, metrics, ozaki, ozaki_b8
from workloads import uniform_binade


def _topdown_digits(X: int, s: int):
    """Balanced base-256 digits from the most significant end: d_p is the only
    value that leaves a remainder inside the range of the s - p digits still to
    come, [-128 (256^r - 1)/255, 127 (256^r - 1)/255] with r = s - p."""
    out = []
    R = X
    for p in range(1, s + 1):
        r = s - p
        w = 256 ** r
        lo, hi = -128 * (w - 1) // 255, 127 * (w - 1) // 255
        cands = [d for d in range(-128, 128) if lo <= R - d * w <= hi]
        assert len(cands) == 1, (X, s, p, cands)
        out.append(cands[0])
        R -= cands[0] * w
    assert R == 0
    return out


@pytest.mark.parametrize("s", [1, 2, 3, 5, 8])
def test_digits_match_topdown_construction_and_reconstruct(s):
    rng = np.random.default_rng(s)
    lim = 2 ** (8 * s - 2)
    xs = [0, 1, -1, lim - 1, -(lim - 1), 127, -128, 128, -129] + \
         [int(v) for v in rng.integers(-(lim - 1), lim, 300, dtype=np.int64)]
    xs = [x for x in xs if abs(x) < lim]
    D = ozaki_b8.digits(np.array(xs, dtype=np.int64), s)
    assert D.min() >= -128 and D.max() <= 127
    for i, x in enumerate(xs):
        got = [int(D[p, i]) for p in range(s)]
        assert got == _topdown_digits(x, s)
        assert sum(d * 256 ** (s - 1 - p) for p, d in enumerate(got)) == x


def test_negation_is_not_digitwise_when_a_digit_is_minus_128():
    # X = 5 * 256 - 128: digits (5, -128); -X would need (-5, 128), out of
    # range, and is (-4, -128) instead
    s = 2
    X = np.array([5 * 256 - 128], dtype=np.int64)
    d = ozaki_b8.digits(X, s)[:, 0].tolist()
    dn = ozaki_b8.digits(-X, s)[:, 0].tolist()
    assert d == [5, -128]
    assert dn != [-v for v in d] and dn == [-4, -128]


def test_integer_conversion_is_truncation():
    rng = np.random.default_rng(3)
    X = rng.standard_normal((6, 9)) * np.ldexp(1.0, rng.integers(-40, 40, (6, 1)))
    X[1, 2] = 5e-324
    X[2] = 0.0
    e, _ = ozaki.row_exponents(X)
    for s in (1, 4, 8):
        I = ozaki_b8.integers(X, e, s)
        for i in range(6):
            for j in range(9):
                want = int(Fraction(float(X[i, j])) * Fraction(2) ** (8 * s - 2 - int(e[i])))
                assert int(I[i, j]) == want                      # int() truncates toward zero
                assert abs(int(I[i, j])) < 2 ** (8 * s - 2)


def _exact_model(A, B, s):
    """B1..B4 evaluated with Python integers and Fractions: digits from the
    top-down construction, diagonal sums by explicit loops, complex real part
    with the digits of -Im b."""
    cplx = np.iscomplexobj(A) or np.iscomplexobj(B)
    m, k = A.shape
    n = B.shape[1]
    mag = (lambda z: max(abs(z.real), abs(z.imag))) if cplx else abs
    e = [math.frexp(max(mag(A[i, l]) for l in range(k)))[1] for i in range(m)]
    f = [math.frexp(max(mag(B[l, j]) for l in range(k)))[1] for j in range(n)]

    def dig(x, ex):
        X = int(Fraction(float(x)) * Fraction(2) ** (8 * s - 2 - ex))
        return _topdown_digits(X, s)

    out = np.zeros((m, n), dtype=np.complex128 if cplx else np.float64)
    for i in range(m):
        for j in range(n):
            def diag_sum(pa, pb):
                S = {t: 0 for t in range(2, s + 2)}
                for l in range(k):
                    da, db = pa(l), pb(l)
                    for p in range(1, s + 1):
                        for q in range(1, s + 2 - p):
                            S[p + q] += da[p - 1] * db[q - 1]
                return S
            if cplx:
                ar = lambda l: dig(A[i, l].real, e[i])
                ai = lambda l: dig(A[i, l].imag, e[i])
                br = lambda l: dig(B[l, j].real, f[j])
                bi = lambda l: dig(B[l, j].imag, f[j])
                nb = lambda l: dig(-B[l, j].imag, f[j])
                Sr1, Sr2 = diag_sum(ar, br), diag_sum(ai, nb)
                Si1, Si2 = diag_sum(ar, bi), diag_sum(ai, br)
                parts = [{t: Sr1[t] + Sr2[t] for t in Sr1}, {t: Si1[t] + Si2[t] for t in Si1}]
            else:
                parts = [diag_sum(lambda l: dig(A[i, l], e[i]), lambda l: dig(B[l, j], f[j]))]
            vals = []
            for S in parts:
                acc = 0.0
                for t in range(2, s + 2):
                    acc = acc + math.ldexp(float(S[t]), 4 - 8 * t)
                vals.append(math.ldexp(acc, e[i] + f[j]))
            out[i, j] = complex(vals[0], vals[1]) if cplx else vals[0]
    return out


@pytest.mark.parametrize("complex_,s", [(False, 2), (False, 5), (True, 3), (True, 6)])
def test_model_equals_exact_rational_definition(complex_, s):
    A, B = uniform_binade(5, 4, 7, seed=70 + s, complex_=complex_)
    A[1, 3] = 5e-324
    B[2, 1] = -B[2, 1]
    got = ozaki_b8.ozaki_gemm_b8("N", "N", A, B, s)
    want = _exact_model(A, B, s)
    assert np.array_equal(got.view(np.float64), want.view(np.float64))


def test_small_integer_inputs_give_the_exact_product():
    # |a| < 64: the row exponent is at most 6, so X = a 2^(8s - 2 - e) is a
    # multiple of 256^(s-1) and only the pair (1, 1) is nonzero
    rng = np.random.default_rng(8)
    A = rng.integers(-63, 64, (9, 40)).astype(np.float64)
    B = rng.integers(-63, 64, (40, 6)).astype(np.float64)
    exact = (A.astype(np.int64) @ B.astype(np.int64)).astype(np.float64)
    for s in (1, 3, 6):
        assert np.array_equal(ozaki_b8.ozaki_gemm_b8("N", "N", A, B, s), exact)


@pytest.mark.parametrize("complex_", [False, True])
def test_error_falls_with_s_and_beats_the_7_bit_split(complex_):
    A, B = uniform_binade(40, 30, 50, seed=11, complex_=complex_)
    hi, lo = dd.dd_gemm("N", "N", A, B)
    den = metrics.abs_product("N", "N", A, B)
    b8 = {s: metrics.err_comp(ozaki_b8.ozaki_gemm_b8("N", "N", A, B, s), hi, lo, den)
          for s in range(3, 8)}
    t7 = {s: metrics.err_comp(ozaki.ozaki_gemm("N", "N", A, B, s), hi, lo, den) for s in range(3, 8)}
    for s in range(3, 7):
        assert b8[s + 1] < b8[s] / 100          # ~8 bits per slice
        # 8s - 2 against 7s bits: s - 2 more bits, so the gap widens with s
        assert b8[s] < t7[s] * 2.0 ** -(s - 3)
    assert b8[6] < 1e-11 and b8[7] < 1e-13


def test_nonfinite_rows_and_alpha_beta_follow_the_base_model():
    A, B = uniform_binade(6, 5, 4, seed=12, complex_=True)
    A[2, 1] = np.nan
    C0 = np.arange(30).reshape(6, 5) * (1 + 0.5j)
    got = ozaki_b8.ozaki_gemm_b8("N", "N", A, B, 4, 0.5 - 1j, 2.0, C0)
    assert np.all(np.isnan(got[2]))
    P = ozaki_b8.ozaki_gemm_b8("N", "N", A, B, 4)
    want = ozaki.apply_alpha_beta(P, 0.5 - 1j, 2.0, C0)
    keep = np.arange(6) != 2
    assert np.array_equal(got[keep].view(np.float64), want[keep].view(np.float64))
    with pytest.raises(ValueError):
        ozaki_b8.ozaki_gemm_b8("N", "N", A, B, 9)
