"""GPU parity of the Ozaki-II (CRT) path against its CPU oracle, through the C
ABI. The integer conversion, the residues, the modular products and the CRT
rebuild are exact, and the rounding and alpha/beta are fixed by the model, so
the results must match bit for bit."""
import sys

import numpy as np
import pytest

from oracle import dd, metrics, ozaki2
from tests.gpu_util import bits_equal, dev, host, mismatch_report, require_gpu, torch
from workloads import kkr_operands, uniform_binade

import paper_2603_29975_amd as oz

pytestmark = pytest.mark.gpu


@pytest.fixture(autouse=True)
def _gpu():
    require_gpu()
    yield
    torch.cuda.synchronize()


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _stored(X, trans):
    t = trans.upper()
    if t == "N":
        return X
    if t == "T":
        return np.ascontiguousarray(X.T)
    return np.ascontiguousarray(np.conj(X.T))


def _operands(kind, m, n, k, seed, nasty=False):
    A, B = uniform_binade(m, n, k, seed=seed, complex_=kind == "z")
    if nasty:
        rng = np.random.default_rng(seed + 1)
        A[rng.integers(0, m)] = 0.0                      # zero row
        B[:, rng.integers(0, n)] = 0.0                   # zero column
        A[rng.integers(0, m)] *= 2.0 ** -1060            # tiny row (subnormal entries)
        B[:, rng.integers(0, n)] *= 2.0 ** 900           # huge column
        A[rng.integers(0, m), rng.integers(0, k)] = 5e-324
    return A, B


def _run(kind, ta, tb, A, B, nmod, alpha=1.0, beta=0.0, C0=None):
    m, k = A.shape
    n = B.shape[1]
    Ad, lda = dev(_stored(A, ta))
    Bd, ldb = dev(_stored(B, tb))
    dt = np.complex128 if kind == "z" else np.float64
    if C0 is None:
        C0 = np.full((m, n), np.nan, dtype=dt)           # beta == 0 must not read C
    Cd, ldc = dev(C0.astype(dt))
    fn = oz.ozaki2_zgemm if kind == "z" else oz.ozaki2_dgemm
    rc = fn(ta, tb, m, n, k, alpha, Ad, lda, Bd, ldb, beta, Cd, ldc, nmod)
    assert rc == 0, oz.ozaki_status_string(rc)
    return host(Cd, m, n)


@pytest.mark.parametrize("kind", ["d", "z"])
@pytest.mark.parametrize("ta,tb,nmod", [("N", "N", 14), ("T", "N", 10), ("N", "C", 16),
                                        ("C", "T", 6), ("T", "T", 20), ("N", "N", 2)])
def test_ozaki2_bit_exact(kind, ta, tb, nmod):
    # several 64 x 64 residue tiles and 256-row rebuild blocks with ragged tails
    m, n, k = (300, 90, 140) if kind == "d" else (270, 70, 100)
    A, B = _operands(kind, m, n, k, seed=900 + nmod, nasty=True)
    _say("ozaki2", kind, ta, tb, nmod)
    got = _run(kind, ta, tb, A, B, nmod)
    ref = ozaki2.ozaki2_gemm("N", "N", A, B, nmod)
    assert bits_equal(got, ref), mismatch_report(got, ref)


@pytest.mark.parametrize("kind", ["d", "z"])
def test_ozaki2_alpha_beta_bit_exact(kind):
    m, n, k = 97, 130, 65
    A, B = _operands(kind, m, n, k, seed=910)
    rng = np.random.default_rng(911)
    C0 = rng.standard_normal((m, n))
    if kind == "z":
        C0 = C0 + 1j * rng.standard_normal((m, n))
        cases = [(0.5 - 1.25j, -2.0 + 0.5j), (1.0, 0.0), (1j, 1.0), (-0.3, 0.7j)]
    else:
        cases = [(0.5, -2.0), (1.0, 0.0), (-1.7, 1.0), (3.1, 0.25)]
    for alpha, beta in cases:
        _say("ozaki2 alpha/beta", kind, alpha, beta)
        got = _run(kind, "N", "N", A, B, 12, alpha, beta, C0 if beta != 0 else None)
        ref = ozaki2.ozaki2_gemm("N", "N", A, B, 12, alpha, beta, C0)
        assert bits_equal(got, ref), mismatch_report(got, ref)


@pytest.mark.parametrize("kind", ["d", "z"])
def test_ozaki2_quick_returns_nonfinite_and_tiny_shapes(kind):
    m, n, k = 33, 20, 17
    A, B = _operands(kind, m, n, k, seed=920)
    dt = np.complex128 if kind == "z" else np.float64
    C0 = (np.arange(m * n).reshape(m, n) + 0.5).astype(dt)
    got = _run(kind, "N", "N", A, B, 14, 0.0, 2.0, C0)
    assert bits_equal(got, ozaki2.ozaki2_gemm("N", "N", A, B, 14, 0.0, 2.0, C0))
    got = _run(kind, "N", "N", A[:, :0], B[:0, :], 14, 1.0, 3.0, C0)
    assert bits_equal(got, ozaki2.ozaki2_gemm("N", "N", A[:, :0], B[:0, :], 14, 1.0, 3.0, C0))
    A2, B2 = _operands(kind, 70, 90, 40, seed=921)
    A2[3, 7] = np.inf
    A2[60, 0] = np.nan
    B2[5, 80] = -np.inf
    got = _run(kind, "N", "N", A2, B2, 14)
    ref = ozaki2.ozaki2_gemm("N", "N", A2, B2, 14)
    assert bits_equal(got, ref), mismatch_report(got, ref)
    assert np.all(np.isnan(got[3])) and np.all(np.isnan(got[:, 80]))
    for (mm, nn, kk) in [(1, 1, 1), (1, 5, 3), (7, 1, 2), (3, 4, 1), (65, 257, 65)]:
        A3, B3 = _operands(kind, mm, nn, kk, seed=mm * 100 + nn * 10 + kk)
        got = _run(kind, "N", "N", A3, B3, 8)
        assert bits_equal(got, ozaki2.ozaki2_gemm("N", "N", A3, B3, 8)), (mm, nn, kk)


def test_ozaki2_integer_inputs_exact_and_accuracy_sweep():
    rng = np.random.default_rng(930)
    A = rng.integers(-1000, 1001, (70, 300)).astype(np.float64)
    B = rng.integers(-1000, 1001, (300, 50)).astype(np.float64)
    exact = (A.astype(np.int64) @ B.astype(np.int64)).astype(np.float64)
    assert np.array_equal(_run("d", "N", "N", A, B, 12), exact)
    # 160^3 DGEMM, entries u * 2^e, e in [-4, 4]: error falls with the moduli
    A, B = uniform_binade(160, 160, 160, seed=1001)
    hi, lo = dd.dd_gemm("N", "N", A, B)
    den = metrics.abs_product("N", "N", A, B)
    errs = {}
    for nmod in (8, 10, 12, 14, 16):
        got = _run("d", "N", "N", A, B, nmod)
        assert bits_equal(got, ozaki2.ozaki2_gemm("N", "N", A, B, nmod)), nmod
        errs[nmod] = metrics.err_comp(got, hi, lo, den)
    _say("ozaki2 err_comp", errs)
    assert all(errs[b] < errs[a] for a, b in ((8, 10), (10, 12), (12, 14), (14, 16)))
    assert errs[14] <= 1e-12


def test_ozaki2_kkr_2048_sampled_bit_exact_and_accuracy():
    # Full-size complex KKR workload (64 blocks of 32) at 14 moduli: the GPU
    # result equals the oracle on sampled rows/columns (the model is separable
    # by rows of op(A) and columns of op(B): exponents per row/column, beta
    # from N and K' only) and meets 1e-12 componentwise.
    A, B = kkr_operands(64, seed=1002)
    m = n = 2048
    got = _run("z", "N", "N", A, B, 14)
    rng = np.random.default_rng(78)
    rows = np.sort(rng.choice(m, 16, replace=False))
    cols = np.sort(rng.choice(n, 16, replace=False))
    ref = ozaki2.ozaki2_gemm("N", "N", A[rows], B[:, cols], 14)
    sub = got[np.ix_(rows, cols)]
    assert bits_equal(sub, ref), mismatch_report(sub, ref)
    ri, cj = np.meshgrid(rows, cols, indexing="ij")
    hi, lo = dd.dd_entries("N", "N", A, B, ri.ravel(), cj.ravel())
    den = metrics.denom_entries("N", "N", A, B, ri.ravel(), cj.ravel())
    err = metrics.err_comp(sub.ravel(), hi, lo, den)
    _say("kkr 2048 ozaki2 N=14 err_comp (sampled)", err)
    assert err <= 1e-12
