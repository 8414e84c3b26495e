"""Pins of the CPU oracle against things other than itself.

Each test checks the oracle's emulation model, double-double reference or
exact-entry code against a hand-derived example, a closed form, brute force on
tiny inputs, a special case that reduces to a textbook routine, or an invariant
the mathematics of the method fixes. None of them calls the GPU library.
"""
from fractions import Fraction
import itertools
import math

import numpy as np
import pytest

from oracle import dd, exact, metrics, ozaki
from workloads import kkr_operands, scaled_gaussian, uniform_binade


def _read_golden(path):
    vals = {}
    with open(path) as fh:
        for line in fh:
            line = line.strip()
            if not line or line.startswith("#"):
                continue
            key, *rest = line.split()
            vals[key] = [int(x) for x in rest]
    return vals


def _bits_equal(x, y):
    """Bitwise equality of float64/complex128 arrays (NaN equal to NaN)."""
    x = np.ascontiguousarray(x)
    y = np.ascontiguousarray(y)
    if x.shape != y.shape or x.dtype != y.dtype:
        return False
    return np.array_equal(x.view(np.uint64), y.view(np.uint64)) or (
        np.array_equal(np.isnan(x), np.isnan(y))
        and np.array_equal(np.where(np.isnan(x), 0, x).view(np.uint64),
                           np.where(np.isnan(y), 0, y).view(np.uint64)))


# ------------------------------------------------------------ worked example
def test_worked_example_digits(golden_dir):
    g = _read_golden(f"{golden_dir}/worked_example.txt")
    a = np.array([[1.0 / 3.0]])
    e, bad = ozaki.row_exponents(a)
    assert e[0] == g["exponent"][0] and not bad[0]
    D = ozaki.split(a, e, 12)
    assert [int(D[p, 0, 0]) for p in range(12)] == g["digits"]
    Dn = ozaki.split(-a, e, 12)
    assert [int(Dn[p, 0, 0]) for p in range(12)] == [-d for d in g["digits"]]


def test_worked_example_gemm(golden_dir):
    g = _read_golden(f"{golden_dir}/worked_example.txt")
    a = np.array([[1.0 / 3.0]])
    for s, key in ((2, "gemm_s2"), (3, "gemm_s3")):
        C = ozaki.ozaki_gemm("N", "N", a, a, s)
        num, ex = g[key]
        assert C[0, 0] == math.ldexp(num, ex)


# ------------------------------------------------------------ exponents (R1)
def _special_values(rng, n):
    v = rng.standard_normal(n) * np.ldexp(1.0, rng.integers(-60, 60, n))
    v[:8] = [0.0, -0.0, 5e-324, -2.2250738585072014e-308, 1.0, -0.5, 2.0 ** 1023, 1.7976931348623157e308]
    return v


def test_row_exponent_definition():
    rng = np.random.default_rng(11)
    X = rng.standard_normal((40, 17)) * np.ldexp(1.0, rng.integers(-1070, 1020, (40, 1)))
    X[3] = 0.0
    X[5, :] = 5e-324 * rng.integers(-3, 4, 17)
    X[7, 2] = 2.0 ** 1023
    e, bad = ozaki.row_exponents(X)
    assert not bad.any()
    for i in range(X.shape[0]):
        mu = max(Fraction(abs(float(v))) for v in X[i])
        if mu == 0:
            assert e[i] == 0
        else:
            assert Fraction(2) ** (int(e[i]) - 1) <= mu < Fraction(2) ** int(e[i])
    # complex rows use max(|Re|, |Im|), not the modulus
    Z = np.array([[0.75 + 0.75j, 0.1 - 0.2j], [0.0 + 0.0j, 0.0 - 3.0j]])
    ez, _ = ozaki.row_exponents(Z)
    assert list(ez) == [0, 2]


def test_row_exponent_nonfinite_flag():
    X = np.ones((4, 3))
    X[1, 2] = np.nan
    X[2, 0] = -np.inf
    e, bad = ozaki.row_exponents(X)
    assert list(bad) == [False, True, True, False]
    assert e[1] == 0 and e[2] == 0 and e[0] == 1


def test_leading_digit_uses_full_range():
    # |x| >= 1/2 for the row maximum, so the first digit of that entry is >= 64
    # in magnitude; an exponent one too large would give <= 63.
    A, _ = uniform_binade(64, 1, 50, seed=5)
    e, _ = ozaki.row_exponents(A)
    D = ozaki.split(A, e, 3)
    assert np.all(np.abs(D[0]).max(axis=1) >= 64)
    assert np.all(np.abs(D[0]).max(axis=1) <= 127)


# ------------------------------------------------------------ slicing (R2)
def _trunc_bits(x: Fraction, bits: int) -> Fraction:
    scale = Fraction(2) ** bits
    t = math.floor(abs(x) * scale)
    return (t if x >= 0 else -t) / scale


@pytest.mark.parametrize("s", [1, 2, 3, 5, 7, 8, 9, 12])
def test_split_is_truncation_to_7s_bits(s):
    rng = np.random.default_rng(100 + s)
    v = _special_values(rng, 64)
    v = v[np.isfinite(v)]
    X = v.reshape(1, -1)
    e, _ = ozaki.row_exponents(X)
    D = ozaki.split(X, e, s)
    assert D.dtype == np.int8
    assert np.abs(D.astype(int)).max() <= 127
    scale = Fraction(2) ** (-int(e[0]))
    for l, a in enumerate(v):
        x = Fraction(float(a)) * scale
        assert abs(x) < 1
        got = sum(Fraction(int(D[p, 0, l])) / Fraction(128) ** (p + 1) for p in range(s))
        assert got == _trunc_bits(x, 7 * s)
        # every digit carries the sign of x (or is zero)
        sg = (x > 0) - (x < 0)
        assert all(int(D[p, 0, l]) * sg >= 0 for p in range(s))


def test_split_prefix_property():
    A, _ = uniform_binade(16, 1, 33, seed=7)
    e, _ = ozaki.row_exponents(A)
    D12 = ozaki.split(A, e, 12)
    for s in range(1, 12):
        assert np.array_equal(ozaki.split(A, e, s), D12[:s])


# ------------------------------------------------------------ products (R3)
def _brute_diagonals(DA, DB, s, mode="triangle"):
    """S_t by scalar Python-int loops over (p, q, i, j, l)."""
    complex_ = len(DA) == 2
    m, k = DA[0].shape[1:]
    n = DB[0].shape[1]
    tmax = s + 1 if mode == "triangle" else 2 * s
    out = {}
    for t in range(2, tmax + 1):
        Sr = [[0] * n for _ in range(m)]
        Si = [[0] * n for _ in range(m)]
        for p in range(1, s + 1):
            q = t - p
            if not 1 <= q <= s:
                continue
            for i in range(m):
                for j in range(n):
                    for l in range(k):
                        if complex_:
                            ar, ai = int(DA[0][p - 1, i, l]), int(DA[1][p - 1, i, l])
                            br, bi = int(DB[0][q - 1, j, l]), int(DB[1][q - 1, j, l])
                            z = complex(ar, ai) * complex(br, bi)   # exact: small ints
                            Sr[i][j] += int(z.real)
                            Si[i][j] += int(z.imag)
                        else:
                            Sr[i][j] += int(DA[0][p - 1, i, l]) * int(DB[0][q - 1, j, l])
        out[t] = (Sr, Si)
    return out


@pytest.mark.parametrize("complex_", [False, True])
@pytest.mark.parametrize("mode", ["triangle", "full"])
def test_diagonals_brute_force(complex_, mode):
    rng = np.random.default_rng(3)
    s = 4
    m, n, k = 3, 4, 5
    A, B = uniform_binade(m, n, k, seed=21, complex_=complex_)
    e, _ = ozaki.row_exponents(A)
    f, _ = ozaki.col_exponents(B)
    DA = ozaki.split_operand(A, e, s)
    DB = ozaki.split_operand(B.T, f, s)
    S = ozaki.diagonals(DA, DB, s, mode)
    ref = _brute_diagonals(DA, DB, s, mode)
    assert sorted(S) == sorted(ref)
    for t in S:
        Sr, Si = ref[t]
        if complex_:
            assert np.array_equal(S[t].real, np.array(Sr, dtype=float))
            assert np.array_equal(S[t].imag, np.array(Si, dtype=float))
        else:
            assert np.array_equal(S[t], np.array(Sr, dtype=float))
    del rng


def test_pair_counts():
    for s in range(1, 13):
        tri = ozaki.pairs(s)
        assert sum(len(v) for v in tri.values()) == s * (s + 1) // 2
        assert all(len(tri[t]) == t - 1 for t in tri)
        full = ozaki.pairs(s, "full")
        assert sum(len(v) for v in full.values()) == s * s


# ------------------------------------------------------------ textbook special cases
@pytest.mark.parametrize("complex_", [False, True])
@pytest.mark.parametrize("ta,tb", [("N", "N"), ("T", "N"), ("N", "T"), ("C", "C")])
def test_small_integer_inputs_give_integer_gemm(complex_, ta, tb):
    # Entries that are integers of magnitude <= 127 fit in the first digit, so
    # the model must return the exact integer product for every s.
    rng = np.random.default_rng(8)
    m, n, k = 7, 6, 9
    def draw(shape):
        x = rng.integers(-127, 128, shape).astype(np.float64)
        if complex_:
            x = x + 1j * rng.integers(-127, 128, shape)
        return x
    A = draw((m, k) if ta == "N" else (k, m))
    B = draw((k, n) if tb == "N" else (n, k))
    opA = ozaki.op(A, ta)
    opB = ozaki.op(B, tb)
    if complex_:
        Ar, Ai = opA.real.astype(np.int64), opA.imag.astype(np.int64)
        Br, Bi = opB.real.astype(np.int64), opB.imag.astype(np.int64)
        ref = (Ar @ Br - Ai @ Bi).astype(float) + 1j * (Ar @ Bi + Ai @ Br).astype(float)
    else:
        ref = (opA.astype(np.int64) @ opB.astype(np.int64)).astype(float)
    for s in range(1, 13):
        C = ozaki.ozaki_gemm(ta, tb, A, B, s)
        assert np.array_equal(C, ref), s


def test_full_mode_exact_for_14_bit_integers():
    # Integers below 2^14 need two digits; with both digits and every pair kept
    # the slice products are the exact integer product (all below 2^53).
    rng = np.random.default_rng(9)
    A = rng.integers(-(2 ** 14) + 1, 2 ** 14, (9, 11)).astype(np.float64)
    B = rng.integers(-(2 ** 14) + 1, 2 ** 14, (11, 8)).astype(np.float64)
    ref = (A.astype(np.int64) @ B.astype(np.int64)).astype(float)
    for s in (2, 3, 5):
        assert np.array_equal(ozaki.ozaki_gemm("N", "N", A, B, s, mode="full"), ref)
    # the triangle drops the (2, 2) pair at s = 2, so it is not exact there
    assert not np.array_equal(ozaki.ozaki_gemm("N", "N", A, B, 2), ref)


# ------------------------------------------------------------ closed-form bound
def _bound(e, f, k_terms, s):
    """Entrywise bound on |C_hat - C*| for alpha = 1, beta = 0.

    With |x| < 1 and |y| < 1 after scaling, truncation to 7s bits costs
    < 2 * 2^-7s per product term, the dropped pairs p + q >= s + 2 cost
    < (s - 1) * (127/128)^2 * 2^-7s * (1 + 1/127) <= (s - 1) * 2^-7s, and the
    s - 1 rounded additions of the recombination each cost at most 2^-53 times
    a partial sum bounded by the number of product terms.
    """
    per_term = (2.0 + (s - 1)) * 2.0 ** (-7 * s) + s * 2.0 ** -53
    return np.ldexp(1.0, (e[:, None] + f[None, :]).astype(np.int32)) * k_terms * per_term


@pytest.mark.parametrize("complex_", [False, True])
def test_error_within_closed_form_bound(complex_):
    m = n = k = 48
    if complex_:
        A, B = scaled_gaussian(m, n, k, seed=31, rmax=12)
    else:
        A, B = uniform_binade(m, n, k, seed=30)
    hi, lo = dd.dd_gemm("N", "N", A, B)
    e, _ = ozaki.row_exponents(A)
    f, _ = ozaki.col_exponents(B)
    for s in range(1, 11):
        C = ozaki.ozaki_gemm("N", "N", A, B, s)
        bnd = _bound(e, f, 2 * k if complex_ else k, s)
        d = (C - hi) - lo
        if complex_:
            assert np.all(np.abs(d.real) <= bnd) and np.all(np.abs(d.imag) <= bnd), s
        else:
            assert np.all(np.abs(d) <= bnd), s


def test_dropping_a_pair_breaks_the_bound():
    # The bound is tight enough to notice one missing pair on the last diagonal.
    A, B = uniform_binade(64, 64, 64, seed=32)
    e, _ = ozaki.row_exponents(A)
    f, _ = ozaki.col_exponents(B)
    s = 5
    DA = ozaki.split_operand(A, e, s)
    DB = ozaki.split_operand(B.T, f, s)
    S = ozaki.diagonals(DA, DB, s)
    t = s + 1
    S_bad = dict(S)
    S_bad[t] = S[t] - DA[0][0].astype(float) @ DB[0][s - 1].astype(float).T
    hi, lo = dd.dd_gemm("N", "N", A, B)
    good = ozaki.recombine(S, e, f)
    bad = ozaki.recombine(S_bad, e, f)
    bnd = _bound(e, f, 64, s)
    assert np.all(np.abs((good - hi) - lo) <= bnd)
    assert np.any(np.abs((bad - hi) - lo) > bnd)


# ------------------------------------------------------------ error vs s
def test_error_falls_by_about_2_to_the_7_per_slice_to_fp64_floor():
    A, B = uniform_binade(128, 128, 128, seed=1001)
    hi, lo = dd.dd_gemm("N", "N", A, B)
    den = metrics.abs_product("N", "N", A, B)
    errs = [metrics.err_comp(ozaki.ozaki_gemm("N", "N", A, B, s), hi, lo, den) for s in range(2, 12)]
    for a, b in zip(errs[:6], errs[1:7]):          # s = 2..8: geometric decrease
        assert 2.0 ** -9 < b / a < 2.0 ** -5
    assert all(b <= a for a, b in zip(errs, errs[1:]))
    assert errs[-1] < 4e-16                          # FP64 rounding level
    native = metrics.err_comp(A @ B, hi, lo, den)
    assert native < 1e-14


# ------------------------------------------------------------ invariants
def test_power_of_two_equivariance():
    A, B = scaled_gaussian(40, 36, 44, seed=1004, rmax=0)
    rng = np.random.default_rng(40)
    r = rng.integers(-30, 31, 40)
    c = rng.integers(-30, 31, 36)
    A2 = A * np.ldexp(1.0, r)[:, None]
    B2 = B * np.ldexp(1.0, c)[None, :]
    for s in (4, 7):
        C = ozaki.ozaki_gemm("N", "N", A, B, s)
        C2 = ozaki.ozaki_gemm("N", "N", A2, B2, s)
        sc = np.ldexp(1.0, (r[:, None] + c[None, :]).astype(np.int32))
        assert _bits_equal(C2, C * sc)


@pytest.mark.parametrize("complex_", [False, True])
def test_transpose_symmetry_and_trans_flags(complex_):
    A, B = uniform_binade(13, 11, 17, seed=41, complex_=complex_)
    for s in (3, 7):
        C = ozaki.ozaki_gemm("N", "N", A, B, s)
        Ct = ozaki.ozaki_gemm("N", "N", B.T.copy(), A.T.copy(), s)
        assert _bits_equal(np.ascontiguousarray(C.T), Ct)
        assert _bits_equal(ozaki.ozaki_gemm("T", "T", A.T.copy(), B.T.copy(), s), C)
        if complex_:
            Ah = np.conj(A.T).copy()
            Bh = np.conj(B.T).copy()
            assert _bits_equal(ozaki.ozaki_gemm("C", "C", Ah, Bh, s), C)


def test_complex_model_on_real_data_equals_real_model():
    A, B = uniform_binade(20, 18, 22, seed=42)
    for s in (2, 5, 8):
        Cd = ozaki.ozaki_gemm("N", "N", A, B, s)
        Cz = ozaki.ozaki_gemm("N", "N", A.astype(np.complex128), B.astype(np.complex128), s)
        assert np.array_equal(Cz.real, Cd) and np.all(Cz.imag == 0)


def test_zero_rows_and_columns_give_zero():
    A, B = uniform_binade(10, 9, 8, seed=43)
    A[3] = 0.0
    B[:, 4] = 0.0
    C = ozaki.ozaki_gemm("N", "N", A, B, 6)
    assert np.all(C[3] == 0) and np.all(C[:, 4] == 0)


def test_incremental_slices_keep_earlier_diagonals():
    A, B = kkr_operands(2, seed=44)
    e, _ = ozaki.row_exponents(A)
    f, _ = ozaki.col_exponents(B)
    prev = None
    for s in range(2, 10):
        S = ozaki.diagonals(ozaki.split_operand(A, e, s), ozaki.split_operand(B.T, f, s), s)
        if prev is not None:
            assert sorted(S) == sorted(prev) + [s + 1]
            for t in prev:
                assert np.array_equal(S[t], prev[t])
        prev = S


# ------------------------------------------------------------ alpha/beta, quick returns
def test_alpha_beta_exact_cases():
    rng = np.random.default_rng(50)
    A = rng.integers(-100, 100, (6, 5)).astype(float)
    B = rng.integers(-100, 100, (5, 4)).astype(float)
    C = rng.integers(-100, 100, (6, 4)).astype(float)
    ref = A @ B
    assert np.array_equal(ozaki.ozaki_gemm("N", "N", A, B, 3, 2.0, 0.5, C), 2 * ref + 0.5 * C)
    Cn = np.full((6, 4), np.nan)
    assert np.array_equal(ozaki.ozaki_gemm("N", "N", A, B, 3, 1.0, 0.0, Cn), ref)
    assert np.array_equal(ozaki.ozaki_gemm("N", "N", A, B, 3, 0.0, 0.0, Cn), np.zeros((6, 4)))
    assert np.array_equal(ozaki.ozaki_gemm("N", "N", A, B, 3, 0.0, 3.0, C), 3 * C)
    assert np.array_equal(ozaki.ozaki_gemm("N", "N", A[:, :0], B[:0], 3, 1.0, 2.0, C), 2 * C)
    Az, Bz = A + 1j * A[::-1], B - 2j * B
    refz = ozaki.ozaki_gemm("N", "N", Az, Bz, 4)
    got = ozaki.ozaki_gemm("N", "N", Az, Bz, 4, 1j, 0.0, None)
    assert np.array_equal(got.real, -refz.imag) and np.array_equal(got.imag, refz.real)


def _gauss_int(rng, shape, lo=-60, hi=60):
    return rng.integers(lo, hi, shape).astype(float) + 1j * rng.integers(lo, hi, shape).astype(float)


def _exact_complex_axpby(alpha, P, beta, C):
    """alpha P + beta C on Gaussian integers with Python ints (no rounding):
    (ar + ai i)(pr + pi i) = (ar pr - ai pi) + (ar pi + ai pr) i."""
    out = np.empty(P.shape, dtype=np.complex128)
    ar, ai = int(alpha.real), int(alpha.imag)
    br, bi = int(beta.real), int(beta.imag)
    for idx in np.ndindex(P.shape):
        pr, pi = int(P[idx].real), int(P[idx].imag)
        cr, ci = (int(C[idx].real), int(C[idx].imag)) if C is not None else (0, 0)
        re = ar * pr - ai * pi + br * cr - bi * ci
        im = ar * pi + ai * pr + br * ci + bi * cr
        out[idx] = complex(re, im)
    return out


def test_complex_alpha_beta_against_gaussian_integers():
    """Reference-BLAS C <- alpha op(A) op(B) + beta C with complex alpha and
    beta (reading R5), on Gaussian-integer data where every rounding is exact:
    the model must equal the exact result computed with Python integers. A
    conjugated or dropped imaginary part of beta or alpha changes the answer."""
    rng = np.random.default_rng(52)
    A, B, C = _gauss_int(rng, (5, 7)), _gauss_int(rng, (7, 4)), _gauss_int(rng, (5, 4))
    P = np.empty((5, 4), dtype=np.complex128)
    for i in range(5):
        for j in range(4):
            re = sum(int(A[i, l].real) * int(B[l, j].real) - int(A[i, l].imag) * int(B[l, j].imag)
                     for l in range(7))
            im = sum(int(A[i, l].real) * int(B[l, j].imag) + int(A[i, l].imag) * int(B[l, j].real)
                     for l in range(7))
            P[i, j] = complex(re, im)
    from oracle import ozaki_b8
    for alpha, beta in ((2 - 3j, -1 + 2j), (-1j, 3 + 1j), (1 + 0j, 2j), (-2 + 0j, -4 - 1j)):
        want = _exact_complex_axpby(alpha, P, beta, C)
        for model in (lambda a, b: ozaki.ozaki_gemm("N", "N", A, B, 3, a, b, C),
                      lambda a, b: ozaki_b8.ozaki_gemm_b8("N", "N", A, B, 3, a, b, C)):
            got = model(alpha, beta)
            assert np.array_equal(got, want), (alpha, beta)
    # beta-only paths (alpha = 0, or k = 0): C <- beta C
    for beta in (-1 + 2j, 2 - 5j, 1j):
        want = _exact_complex_axpby(0j, np.zeros_like(C), beta, C)
        assert np.array_equal(ozaki.ozaki_gemm("N", "N", A, B, 3, 0.0, beta, C), want)
        assert np.array_equal(ozaki.ozaki_gemm("N", "N", A[:, :0], B[:0], 3, 1 + 1j, beta, C),
                              want)
        assert np.array_equal(ozaki.scale_only(beta, C, C.shape, True), want)
    # the epilogue on its own, against the exact result
    assert np.array_equal(ozaki.apply_alpha_beta(P, 2 - 3j, -1 + 2j, C),
                          _exact_complex_axpby(2 - 3j, P, -1 + 2j, C))


def test_nonfinite_rows_and_columns_become_nan():
    A, B = uniform_binade(6, 5, 7, seed=51)
    A2 = A.copy()
    A2[2, 3] = np.inf
    B2 = B.copy()
    B2[1, 4] = np.nan
    C = ozaki.ozaki_gemm("N", "N", A2, B2, 5)
    ref = ozaki.ozaki_gemm("N", "N", A, B, 5)
    mask = np.zeros((6, 5), bool)
    mask[2, :] = True
    mask[:, 4] = True
    assert np.all(np.isnan(C[mask]))
    assert np.array_equal(C[~mask], ref[~mask])


# ------------------------------------------------------------ double-double reference
def test_dd_matches_exact_rational_entries():
    rng = np.random.default_rng(60)
    m, n, k = 5, 4, 300
    A = rng.standard_normal((m, k)) * np.ldexp(1.0, rng.integers(-40, 40, (m, k)))
    B = rng.standard_normal((k, n)) * np.ldexp(1.0, rng.integers(-40, 40, (k, n)))
    # adversarial cancellation in row 0 / column 0
    B[:, 0] = 1.0
    A[0, : k // 2] = rng.standard_normal(k // 2) * 1e10
    A[0, k // 2:] = -A[0, : k // 2]
    A[0, 0] += 1e-9
    rows, cols = zip(*itertools.product(range(m), range(n)))
    hi, lo = dd.dd_entries("N", "N", A, B, rows, cols)
    ex = exact.exact_entries("N", "N", A, B, rows, cols)
    absprod = np.abs(A) @ np.abs(B)
    for x, (i, j) in enumerate(zip(rows, cols)):
        err = abs(Fraction(float(hi[x])) + Fraction(float(lo[x])) - ex[x])
        assert err <= Fraction(float(absprod[i, j])) * Fraction(k, 2 ** 100)
        assert hi[x] == exact.to_float(ex[x]) or abs(Fraction(float(hi[x])) - ex[x]) <= \
            abs(ex[x]) * Fraction(1, 2 ** 52)


def test_dd_complex_and_full_matches_entries():
    A, B = kkr_operands(1, seed=61)
    hi, lo = dd.dd_gemm("N", "N", A, B)
    rows = np.array([0, 5, 31, 17])
    cols = np.array([3, 5, 0, 30])
    h2, l2 = dd.dd_entries("N", "N", A, B, rows, cols)
    assert np.array_equal(hi[rows, cols], h2) and np.array_equal(lo[rows, cols], l2)
    ex = exact.exact_entries("N", "N", A, B, rows, cols)
    for x in range(4):
        re, im = ex[x]
        assert abs(Fraction(float(h2[x].real)) + Fraction(float(l2[x].real)) - re) <= abs(re) * Fraction(1, 2 ** 95) + Fraction(1, 2 ** 200)
        assert abs(Fraction(float(h2[x].imag)) + Fraction(float(l2[x].imag)) - im) <= abs(im) * Fraction(1, 2 ** 95) + Fraction(1, 2 ** 200)


def test_err_comp_zero_denominator_rule():
    A = np.zeros((3, 2))
    B = np.ones((2, 3))
    hi, lo = np.zeros((3, 3)), np.zeros((3, 3))
    den = metrics.abs_product("N", "N", A, B)
    assert metrics.err_comp(np.zeros((3, 3)), hi, lo, den) == 0.0
    bad = np.zeros((3, 3))
    bad[1, 1] = 1e-300
    assert metrics.err_comp(bad, hi, lo, den) == float("inf")


# ------------------------------------------------------------ residual probe
def test_splitmix64_reference_outputs(golden_dir):
    from oracle.probe import splitmix64
    vals = {}
    for line in open(f"{golden_dir}/splitmix64.txt"):
        if line.strip() and not line.startswith("#"):
            k, v = line.split()
            vals[k] = int(v, 16)
    first = splitmix64(0)
    second = splitmix64(0x9E3779B97F4A7C15)     # state after one step
    assert first == vals["state0_output1"] and second == vals["state0_output2"]


def test_probe_closed_form_planted_error():
    # A = B = I (n x n), C = I + delta e_i e_j^T: r_v = delta x_v[j] e_i exactly,
    # u = 1 for every row, so est_i = |delta| sqrt(n) and 0 elsewhere.
    from oracle.probe import probe_est
    n = 9
    A = np.eye(n)
    B = np.eye(n)
    for delta in (2.0 ** -40, 3e-9):
        C = np.eye(n)
        C[4, 7] += delta
        est = probe_est("N", "N", A, B, C, 3, seed=99)
        want = np.zeros(n)
        want[4] = abs(delta) * np.sqrt(n)          # C[4, 7] was 0: the planted entry is delta
        assert np.allclose(est, want, rtol=1e-12, atol=0)


def test_probe_invariant_under_row_scaling_and_tracks_error():
    from oracle.probe import probe_est
    A, B = uniform_binade(30, 24, 20, seed=70)
    rng = np.random.default_rng(71)
    r = rng.integers(-20, 21, 30)
    C4 = ozaki.ozaki_gemm("N", "N", A, B, 4)
    est = probe_est("N", "N", A, B, C4, 2, seed=5)
    A2 = A * np.ldexp(1.0, r)[:, None]
    C42 = ozaki.ozaki_gemm("N", "N", A2, B, 4)
    est2 = probe_est("N", "N", A2, B, C42, 2, seed=5)
    assert np.allclose(est, est2, rtol=1e-14)
    # the estimate sits within a small factor of the true componentwise error
    hi, lo = dd.dd_gemm("N", "N", A, B)
    den = metrics.abs_product("N", "N", A, B)
    true = metrics.err_comp(C4, hi, lo, den)
    assert true / 30 < est.max() < true * 3
    C7 = ozaki.ozaki_gemm("N", "N", A, B, 7)
    assert probe_est("N", "N", A, B, C7, 2, seed=5).max() < est.max() / 1e4


# ------------------------------------------------------------ selector features and MLP
def test_features_hand_counted_histogram():
    from oracle.selector import features
    # rows of A: [1, 0.5, 0] (row exponent 1: deltas 0, 1, zero) and
    # [0.25, 0.25, 2^-40] (row exponent -1: deltas 0, 0, 38 -> clipped to 30)
    A = np.array([[1.0, 0.5, 0.0], [0.25, 0.25, 2.0 ** -40]])
    # columns of B: [3, 1, 0.75] (exp 2: deltas 0, 1, 2) and [0, 0, -2^-3] (exp -2: zero, zero, 0)
    B = np.array([[3.0, 0.0], [1.0, 0.0], [0.75, -0.125]])
    f = features("N", "N", A, B)
    want = np.zeros(64, dtype=np.float32)
    want[0], want[1], want[30], want[31] = 3 / 6, 1 / 6, 1 / 6, 1 / 6
    want[32 + 0], want[32 + 1], want[32 + 2], want[32 + 30] = 2 / 6, 1 / 6, 1 / 6, 2 / 6
    want[63] = np.float32(np.log2(3.0) / 16)
    assert np.allclose(f, want, rtol=0, atol=1e-7)
    # complex entries use the larger of the two exponents
    fz = features("N", "N", A * (1 + 0j) + 1j * np.array([[0, 0, 0], [1.0, 0, 0]]), B + 0j)
    assert fz[0] == np.float32(2 / 6) and fz[1] == np.float32(1 / 6) and fz[2] == np.float32(1 / 6)


def test_mlp_backward_matches_finite_differences():
    from oracle import selector as sel
    rng = np.random.default_rng(80)
    theta = rng.standard_normal(sel.P) * 0.1
    X = rng.uniform(0, 1, (12, 64))
    t = rng.uniform(3, 9, 12)
    g, L = sel.backward(theta, X, t, 4.0, quantize=False)
    idx = list(rng.choice(sel.P, 40, replace=False)) + [sel.P - 1, sel.OFFS["b1"][0] + 3]
    for i in idx:
        h = 1e-6
        tp, tm = theta.copy(), theta.copy()
        tp[i] += h
        tm[i] -= h
        fd = (sel.loss(sel.forward(tp, X, False)[0], t, 4.0) - sel.loss(sel.forward(tm, X, False)[0], t, 4.0)) / (2 * h)
        assert abs(fd - g[i]) <= 1e-6 * max(1.0, abs(fd)), (i, fd, g[i])


def test_bf16_rounding_and_adam_first_step():
    from oracle import selector as sel
    # bf16 keeps 8 significant bits, rounds to nearest even
    assert sel.bf16(1.0 + 2 ** -8) == 1.0                   # tie -> even
    assert sel.bf16(1.0 + 3 * 2 ** -8) == 1.0 + 2 ** -6     # tie -> even (up)
    assert sel.bf16(1.0 + 2 ** -7) == 1.0 + 2 ** -7
    # first Adam step from zero moments: theta - lr * g / (|g| + eps)
    g = np.array([0.5, -2.0, 0.0, 1e-3])
    th, m, v = sel.adam(np.zeros(4), np.zeros(4), np.zeros(4), g, 0.01, 0.9, 0.999, 1e-8, 1)
    assert np.allclose(th, -0.01 * g / (np.abs(g) + 1e-8), rtol=1e-12, atol=0)


def test_sampled_reference_equals_full_dd_on_its_entries():
    """The sampled accuracy check (4096-entry + whole rows/columns form used at
    16384^3) against the full double-double product and the plain definition
    of the denominators, on a product small enough for both."""
    from oracle.sampled import SampledReference, sample_entries
    A, B = scaled_gaussian(40, 36, 50, seed=60, rmax=10)
    ref = SampledReference(A, B, nrand=100, nrows=3, ncols=2, seed=61)
    ri, cj, rows, cols = sample_entries(40, 36, 100, 3, 2, 61)
    assert np.array_equal(ri, ref.ri) and np.array_equal(cj, ref.cj)
    assert 39 in rows and 35 in cols and rows.size == 3 and cols.size == 2
    assert ri.size == 100 + 3 * 36 + 2 * 40
    hi, lo = dd.dd_gemm("N", "N", A, B)
    assert np.array_equal(ref.hi, hi[ri, cj]) and np.array_equal(ref.lo, lo[ri, cj])
    den = metrics.abs_product("N", "N", A, B)[ri, cj]
    assert np.allclose(ref.den, den, rtol=1e-13, atol=0)
    C = ozaki.ozaki_gemm("N", "N", A, B, 4)
    full = metrics.err_comp(C, hi, lo, metrics.abs_product("N", "N", A, B))
    assert ref.err_comp(C[ri, cj]) <= full
    # every row asked for: the whole matrix
    ri2, cj2, rows2, _ = sample_entries(40, 36, 0, 40, 0, 1)
    assert rows2.size == 40 and ri2.size == 40 * 36
    assert ref.err_comp(C[ri, cj]) == metrics.err_comp(C[ri, cj], hi[ri, cj], lo[ri, cj], den)
