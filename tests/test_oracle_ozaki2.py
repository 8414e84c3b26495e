"""Pins of the Ozaki-II oracle (CPU): the moduli and the bit budget, the CRT
reconstruction against brute-force integer arithmetic, the whole model against
an independent exact-rational evaluation of its definition, and its accuracy."""
import math
from fractions import Fraction

import numpy as np
import pytest

from oracle import dd, metrics, ozaki2
from workloads import uniform_binade


def test_moduli_pairwise_coprime_int8_residues_and_bit_budget():
    for n in range(ozaki2.N_MIN, ozaki2.N_MAX + 1):
        mods = ozaki2.moduli(n)
        assert len(mods) == n and max(mods) == 256 and all(2 <= x <= 256 for x in mods)
        for a in range(n):
            for b in range(a):
                assert math.gcd(mods[a], mods[b]) == 1
        M = math.prod(mods)
        assert M < 2 ** 160
        for kp in (1, 7, 64, 4096, 100000):
            lk = math.ceil(math.log2(kp))
            if M.bit_length() - 2 - lk < 2:
                with pytest.raises(ValueError):
                    ozaki2.beta_bits(n, kp)
                continue
            bet = ozaki2.beta_bits(n, kp)
            assert kp * 2 ** (2 * bet) <= M // 2
            if bet < 63:   # one more bit per operand would break the power-of-two bound
                assert 2 ** lk * 2 ** (2 * bet + 2) > 2 ** (M.bit_length() - 2)
    for m in (256, 255, 173):
        rs = [ozaki2.residue(x, m) for x in range(-600, 600)]
        assert min(rs) >= -128 and max(rs) <= 127
        assert all((x - r) % m == 0 for x, r in zip(range(-600, 600), rs))
    # the greedy choice from 256 downwards
    assert ozaki2.moduli(12) == [256, 255, 253, 251, 247, 241, 239, 233, 229, 227, 223, 217]


@pytest.mark.parametrize("n", [3, 10, 14, 20])
def test_garner_recovers_every_integer_of_the_balanced_range(n):
    mods = ozaki2.moduli(n)
    M = math.prod(mods)
    rng = np.random.default_rng(n)
    xs = [-(M // 2), M // 2 - 1, 0, 1, -1] + [int(rng.integers(-2 ** 62, 2 ** 62)) * int(
        rng.integers(1, 2 ** 62)) % M - M // 2 for _ in range(200)]
    for x in xs:
        assert ozaki2.garner([ozaki2.residue(x, m) for m in mods], mods) == x


def test_crt_product_equals_brute_force_integer_product():
    rng = np.random.default_rng(5)
    n = 12
    mods = ozaki2.moduli(n)
    kp = 37
    bet = ozaki2.beta_bits(n, kp)
    A = np.array([[int(rng.integers(-2 ** 40, 2 ** 40)) * 2 ** (bet - 41) for _ in range(kp)]
                  for _ in range(5)], dtype=object)
    B = np.array([[int(rng.integers(-2 ** 40, 2 ** 40)) * 2 ** (bet - 41) for _ in range(kp)]
                  for _ in range(4)], dtype=object)
    Cm = ozaki2.modular_products(A, B, mods)
    for i in range(5):
        for j in range(4):
            exact = sum(int(A[i, l]) * int(B[j, l]) for l in range(kp))
            assert ozaki2.garner([int(C[i, j]) for C in Cm], mods) == exact


def _exact_model(A, B, n):
    """The definition of Q2/Q5 evaluated with Fractions and Python ints, with
    complex products formed as (ar br - ai bi) + i (ar bi + ai br): no
    residues, no CRT, no interleaving."""
    cplx = np.iscomplexobj(A) or np.iscomplexobj(B)
    m, k = A.shape
    nn = B.shape[1]
    mag = (lambda z: max(abs(z.real), abs(z.imag))) if cplx else abs
    e = [math.frexp(max(mag(A[i, l]) for l in range(k)))[1] for i in range(m)]
    f = [math.frexp(max(mag(B[l, j]) for l in range(k)))[1] for j in range(nn)]
    bet = ozaki2.beta_bits(n, 2 * k if cplx else k)
    conv = lambda x, ex: int(Fraction(float(x)) * Fraction(2) ** (bet - ex))   # trunc toward 0
    out = np.zeros((m, nn), dtype=np.complex128 if cplx else np.float64)
    for i in range(m):
        for j in range(nn):
            if cplx:
                re = sum(conv(A[i, l].real, e[i]) * conv(B[l, j].real, f[j])
                         - conv(A[i, l].imag, e[i]) * conv(B[l, j].imag, f[j]) for l in range(k))
                im = sum(conv(A[i, l].real, e[i]) * conv(B[l, j].imag, f[j])
                         + conv(A[i, l].imag, e[i]) * conv(B[l, j].real, f[j]) for l in range(k))
                sc = e[i] + f[j] - 2 * bet
                out[i, j] = complex(math.ldexp(float(re), sc), math.ldexp(float(im), sc))
            else:
                c = sum(conv(A[i, l], e[i]) * conv(B[l, j], f[j]) for l in range(k))
                out[i, j] = math.ldexp(float(c), e[i] + f[j] - 2 * bet)
    return out


@pytest.mark.parametrize("complex_,n", [(False, 6), (False, 14), (True, 9), (True, 16), (False, 20)])
def test_model_equals_exact_rational_definition(complex_, n):
    A, B = uniform_binade(7, 5, 11, seed=40 + n, complex_=complex_)
    A[2, 3] = 5e-324                                    # a subnormal entry
    got = ozaki2.ozaki2_gemm("N", "N", A, B, n)
    want = _exact_model(A, B, n)
    assert np.array_equal(got.view(np.float64), want.view(np.float64))


@pytest.mark.parametrize("complex_", [False, True])
def test_error_falls_with_moduli_to_fp64_level(complex_):
    A, B = uniform_binade(24, 20, 30, seed=3, complex_=complex_)
    hi, lo = dd.dd_gemm("N", "N", A, B)
    den = metrics.abs_product("N", "N", A, B)
    errs = {n: metrics.err_comp(ozaki2.ozaki2_gemm("N", "N", A, B, n), hi, lo, den)
            for n in (6, 8, 10, 12, 14, 16)}
    for a, b in ((6, 8), (8, 10), (10, 12), (12, 14)):
        assert errs[b] < errs[a] / 50              # two moduli add ~8 bits per operand
    assert errs[14] < 1e-13 and errs[16] < 2 ** -52


def test_integer_inputs_give_the_exact_product():
    rng = np.random.default_rng(8)
    A = rng.integers(-1000, 1001, (9, 40)).astype(np.float64)
    B = rng.integers(-1000, 1001, (40, 6)).astype(np.float64)
    exact = (A.astype(np.int64) @ B.astype(np.int64)).astype(np.float64)
    assert np.array_equal(ozaki2.ozaki2_gemm("N", "N", A, B, 12), exact)


def test_power_of_two_equivariance_and_nonfinite_rows():
    A, B = uniform_binade(10, 8, 12, seed=9, complex_=True)
    r = np.random.default_rng(10).integers(-30, 31, 10)
    C1 = ozaki2.ozaki2_gemm("N", "N", A, B, 10)
    C2 = ozaki2.ozaki2_gemm("N", "N", A * np.ldexp(1.0, r)[:, None], B, 10)
    assert np.array_equal(C2, C1 * np.ldexp(1.0, r)[:, None])
    A[4, 2] = np.inf
    C3 = ozaki2.ozaki2_gemm("N", "N", A, B, 10)
    assert np.all(np.isnan(C3[4])) and np.array_equal(np.delete(C3, 4, 0), np.delete(C1, 4, 0))
