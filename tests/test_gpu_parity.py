"""GPU parity of the HIP path against the CPU oracle, through the C ABI.

Integer work (exponents, digits, diagonal sums) must match bit for bit; the
emulated GEMM must match the oracle's model bit for bit too, because every
FP64 operation of the recombination and of alpha/beta is fixed by the model.
Accuracy against the double-double reference is checked separately.
"""
import sys

import numpy as np
import pytest

from oracle import dd, metrics, ozaki
from tests.gpu_util import bits_equal, dev, host, mismatch_report, require_gpu, torch
from workloads import kkr_operands, scaled_gaussian, uniform_binade

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
    """The stored matrix whose op(.) under `trans` is X."""
    t = trans.upper()
    if t == "N":
        return X
    if t == "T":
        return np.ascontiguousarray(X.T)
    return np.ascontiguousarray(np.conj(X.T))


def _operands(kind, m, n, k, seed, nasty=False):
    cplx = kind == "z"
    A, B = uniform_binade(m, n, k, seed=seed, complex_=cplx)
    if nasty:
        rng = np.random.default_rng(seed + 1)
        A[rng.integers(0, m)] = 0.0                      # zero row
        B[:, rng.integers(0, n)] = 0.0                   # zero column
        A[rng.integers(0, m)] *= 2.0 ** -1060            # tiny row (subnormal entries)
        B[:, rng.integers(0, n)] *= 2.0 ** 900           # huge column
        A[rng.integers(0, m), rng.integers(0, k)] = 5e-324
    return A, B


# ------------------------------------------------------------------ exponents
@pytest.mark.parametrize("kind", ["d", "z"])
@pytest.mark.parametrize("side", ["A", "B"])
@pytest.mark.parametrize("trans", ["N", "T", "C"])
def test_exponents_bit_exact(kind, side, trans):
    rows, L = 150, 77
    A, _ = _operands(kind, rows, 1, L, seed=200, nasty=True)
    A[5, 3] = np.nan
    A[9, 0] = -np.inf
    opX = A if side == "A" else np.ascontiguousarray(A.T)   # side B: columns are the rows
    X = _stored(opX, trans)
    Xd, ldx = dev(X)
    exps = torch.zeros(rows, dtype=torch.int32, device="cuda")
    flags = torch.zeros(rows, dtype=torch.uint8, device="cuda")
    _say("exponents", kind, side, trans)
    rc = oz.ozaki_debug_exponents(kind, side, trans, rows, L, Xd, ldx, exps, flags)
    assert rc == 0
    e_ref, bad_ref = ozaki.row_exponents(A)
    torch.cuda.synchronize()
    assert np.array_equal(exps.cpu().numpy(), e_ref.astype(np.int32))
    assert np.array_equal(flags.cpu().numpy().astype(bool), bad_ref)


# ------------------------------------------------------------------ digits
@pytest.mark.parametrize("kind", ["d", "z"])
@pytest.mark.parametrize("side", ["A", "B"])
@pytest.mark.parametrize("trans,s", [("N", 7), ("T", 3), ("C", 12), ("N", 1)])
def test_split_bit_exact(kind, side, trans, s):
    rows, L = 131, 70
    A, _ = _operands(kind, rows, 1, L, seed=300 + s, nasty=True)
    opX = A if side == "A" else np.ascontiguousarray(A.T)
    X = _stored(opX, trans)
    Xd, ldx = dev(X)
    c = 2 if kind == "z" else 1
    digits = torch.zeros(s * rows * L * c, dtype=torch.int8, device="cuda")
    _say("split", kind, side, trans, s)
    assert oz.ozaki_debug_split(kind, side, trans, rows, L, Xd, ldx, s, digits) == 0
    e, bad = ozaki.row_exponents(A)
    ref = ozaki.split_operand(A, e, s, bad)
    got = digits.cpu().numpy().reshape(s, rows, L, c)
    for part in range(c):
        assert np.array_equal(got[..., part], ref[part]), mismatch_report(got[..., part], ref[part])


# ------------------------------------------------------------------ diagonals
def _gpu_diagonals(kind, ta, tb, A, B, s):
    opA, opB = A, B
    m, k = opA.shape
    n = opB.shape[1]
    Ad, lda = dev(_stored(opA, ta))
    Bd, ldb = dev(_stored(opB, tb))
    c = 2 if kind == "z" else 1
    out = torch.zeros(s * n * m * c, dtype=torch.int64, device="cuda")
    assert oz.ozaki_debug_diagonals(kind, ta, tb, m, n, k, Ad, lda, Bd, ldb, s, out) == 0
    raw = out.cpu().numpy().reshape(s, n, m, c)
    res = {}
    for t in range(2, s + 2):
        if c == 2:
            res[t] = raw[t - 2, :, :, 0].T.astype(np.float64) + 1j * raw[t - 2, :, :, 1].T.astype(np.float64)
        else:
            res[t] = raw[t - 2, :, :, 0].T.astype(np.float64)
    return res


def _ref_diagonals(A, B, s):
    e, bad_r = ozaki.row_exponents(A)
    f, bad_c = ozaki.col_exponents(B)
    return ozaki.diagonals(ozaki.split_operand(A, e, s, bad_r), ozaki.split_operand(B.T, f, s, bad_c), s)


@pytest.mark.parametrize("kind", ["d", "z"])
@pytest.mark.parametrize("ta,tb,s", [("N", "N", 1), ("N", "N", 7), ("T", "N", 4), ("N", "T", 9),
                                     ("C", "C", 12), ("T", "C", 10)])
def test_diagonals_bit_exact(kind, ta, tb, s):
    m, n, k = (200, 300, 130) if kind == "d" else (130, 70, 100)
    A, B = _operands(kind, m, n, k, seed=400 + s, nasty=True)
    _say("diagonals", kind, ta, tb, s, (m, n, k))
    got = _gpu_diagonals(kind, ta, tb, A, B, s)
    ref = _ref_diagonals(A, B, s)
    for t in ref:
        assert np.array_equal(got[t], ref[t]), f"t={t}\n" + mismatch_report(got[t], ref[t])


@pytest.mark.parametrize("kind,s,k", [("d", 7, 19100), ("z", 7, 9600), ("d", 12, 11200), ("z", 12, 5600)])
def test_diagonals_chunked_contraction_bit_exact(kind, s, k):
    # contraction long enough that the INT32 accumulators are carried into int64
    m, n = 40, 36
    cplx = kind == "z"
    A, B = scaled_gaussian(m, n, k, seed=450 + s, rmax=20, complex_=cplx)
    _say("chunked diagonals", kind, s, k)
    got = _gpu_diagonals(kind, "N", "N", A, B, s)
    ref = _ref_diagonals(A, B, s)
    for t in ref:
        assert np.array_equal(got[t], ref[t]), f"t={t}\n" + mismatch_report(got[t], ref[t])


# ------------------------------------------------------------------ full GEMM
def _run_gemm(kind, ta, tb, A, B, s, alpha=1.0, beta=0.0, C0=None):
    m, k = A.shape
    n = B.shape[1]
    Ad, lda = dev(_stored(A, ta))
    Bd, ldb = dev(_stored(B, tb))
    dt = np.complex128 if kind == "z" else np.float64
    if C0 is None:
        C0 = np.full((m, n), np.nan, dtype=dt)       # beta == 0 must not read C
    Cd, ldc = dev(C0.astype(dt))
    fn = oz.ozaki_zgemm if kind == "z" else oz.ozaki_dgemm
    rc = fn(ta, tb, m, n, k, alpha, Ad, lda, Bd, ldb, beta, Cd, ldc, s)
    assert rc == 0, oz.ozaki_status_string(rc)
    return host(Cd, m, n)


@pytest.mark.parametrize("kind", ["d", "z"])
@pytest.mark.parametrize("ta,tb,s", [("N", "N", 3), ("N", "N", 7), ("T", "N", 5), ("N", "C", 8),
                                     ("C", "T", 6), ("T", "T", 9), ("N", "N", 11)])
def test_gemm_bit_exact(kind, ta, tb, s):
    m, n, k = (200, 300, 130) if kind == "d" else (130, 70, 100)
    A, B = _operands(kind, m, n, k, seed=500 + s, nasty=True)
    _say("gemm", kind, ta, tb, s)
    got = _run_gemm(kind, ta, tb, A, B, s)
    ref = ozaki.ozaki_gemm("N", "N", A, B, s)
    assert bits_equal(got, ref), mismatch_report(got, ref)


@pytest.mark.parametrize("kind", ["d", "z"])
def test_gemm_alpha_beta_bit_exact(kind):
    m, n, k = 97, 130, 65
    A, B = _operands(kind, m, n, k, seed=600)
    rng = np.random.default_rng(601)
    C0 = rng.standard_normal((m, n))
    if kind == "z":
        C0 = C0 + 1j * rng.standard_normal((m, n))
        cases = [(0.5 - 1.25j, -2.0 + 0.5j), (1.0, 0.0), (1j, 1.0), (-0.3, 0.7j)]
    else:
        cases = [(0.5, -2.0), (1.0, 0.0), (-1.7, 1.0), (3.1, 0.25)]
    for alpha, beta in cases:
        _say("alpha/beta", kind, alpha, beta)
        got = _run_gemm(kind, "N", "N", A, B, 6, alpha, beta, C0 if beta != 0 else None)
        ref = ozaki.ozaki_gemm("N", "N", A, B, 6, alpha, beta, C0)
        assert bits_equal(got, ref), mismatch_report(got, ref)


@pytest.mark.parametrize("kind", ["d", "z"])
def test_quick_returns(kind):
    m, n, k = 33, 20, 17
    A, B = _operands(kind, m, n, k, seed=650)
    dt = np.complex128 if kind == "z" else np.float64
    C0 = (np.arange(m * n).reshape(m, n) + 0.5).astype(dt)
    # alpha = 0: C <- beta C; beta = 0 then gives zeros even over NaN
    got = _run_gemm(kind, "N", "N", A, B, 5, 0.0, 2.0, C0)
    assert bits_equal(got, ozaki.ozaki_gemm("N", "N", A, B, 5, 0.0, 2.0, C0))
    got = _run_gemm(kind, "N", "N", A, B, 5, 0.0, 0.0, np.full((m, n), np.nan, dtype=dt))
    assert np.all(got == 0)
    got = _run_gemm(kind, "N", "N", A, B, 5, 0.0, 1.0, C0)
    assert bits_equal(got, C0)
    # k = 0
    got = _run_gemm(kind, "N", "N", A[:, :0], B[:0, :], 5, 1.0, 3.0, C0)
    assert bits_equal(got, ozaki.ozaki_gemm("N", "N", A[:, :0], B[:0, :], 5, 1.0, 3.0, C0))


@pytest.mark.parametrize("kind", ["d", "z"])
def test_nonfinite_rows_and_columns(kind):
    m, n, k = 70, 90, 40
    A, B = _operands(kind, m, n, k, seed=700)
    A[3, 7] = np.inf
    A[60, 0] = np.nan
    B[5, 80] = -np.inf
    got = _run_gemm(kind, "N", "N", A, B, 7)
    ref = ozaki.ozaki_gemm("N", "N", A, B, 7)
    assert bits_equal(got, ref), mismatch_report(got, ref)
    assert np.all(np.isnan(got[3])) and np.all(np.isnan(got[:, 80]))


def test_tiny_and_single_element_shapes():
    for (m, n, k) in [(1, 1, 1), (1, 5, 3), (7, 1, 2), (3, 4, 1), (33, 129, 65)]:
        for kind in ("d", "z"):
            A, B = _operands(kind, m, n, k, seed=m * 100 + n * 10 + k)
            got = _run_gemm(kind, "N", "N", A, B, 4)
            ref = ozaki.ozaki_gemm("N", "N", A, B, 4)
            assert bits_equal(got, ref), (m, n, k, kind)


# ------------------------------------------------------------------ accuracy
def test_uniform_binade_256_accuracy_sweep():
    # 256^3 DGEMM, entries u * 2^e, e in [-4, 4]; error falls with s and s = 7
    # reaches the 1e-12 componentwise target.
    A, B = uniform_binade(256, 256, 256, seed=1001)
    hi, lo = dd.dd_gemm("N", "N", A, B)
    den = metrics.abs_product("N", "N", A, B)
    errs = {}
    for s in range(3, 9):
        got = _run_gemm("d", "N", "N", A, B, s)
        assert bits_equal(got, ozaki.ozaki_gemm("N", "N", A, B, s)), s
        errs[s] = metrics.err_comp(got, hi, lo, den)
    _say("err_comp", errs)
    assert all(errs[s + 1] < errs[s] for s in range(3, 8))
    assert errs[7] <= 1e-12 < errs[6]


def test_native_gemm_accuracy():
    for kind, (m, n, k) in (("d", (200, 300, 130)), ("z", (130, 70, 100)), ("d", (1, 1, 1)),
                            ("z", (257, 129, 33))):
        A, B = _operands(kind, m, n, k, seed=800 + m)
        for ta, tb in (("N", "N"), ("T", "C")):
            Ad, lda = dev(_stored(A, ta))
            Bd, ldb = dev(_stored(B, tb))
            dt = np.complex128 if kind == "z" else np.float64
            Cd, ldc = dev(np.full((m, n), np.nan, dtype=dt))
            fn = oz.ozaki_native_zgemm if kind == "z" else oz.ozaki_native_dgemm
            assert fn(ta, tb, m, n, k, 1.0, Ad, lda, Bd, ldb, 0.0, Cd, ldc) == 0
            got = host(Cd, m, n)
            hi, lo = dd.dd_gemm("N", "N", A, B)
            err = metrics.err_comp(got, hi, lo, metrics.abs_product("N", "N", A, B))
            _say("native", kind, ta, tb, err)
            assert err < 4 * k * 2.0 ** -53


def test_kkr_2048_sampled_bit_exact_and_accuracy():
    # Full-size complex KKR workload (64 blocks of 32): the GPU result must
    # equal the oracle on sampled rows/columns (the model is separable by rows
    # of A and columns of B) and meet 1e-12 componentwise at s = 7.
    A, B = kkr_operands(64, seed=1002)
    m = n = k = 2048
    got = _run_gemm("z", "N", "N", A, B, 7)
    rng = np.random.default_rng(77)
    rows = np.sort(rng.choice(m, 48, replace=False))
    cols = np.sort(rng.choice(n, 48, replace=False))
    ref = ozaki.ozaki_gemm("N", "N", A[rows], B[:, cols], 7)
    sub = got[np.ix_(rows, cols)]
    assert bits_equal(sub, ref), mismatch_report(sub, ref)
    ri, cj = np.meshgrid(rows, cols, indexing="ij")
    hi, lo = dd.dd_entries("N", "N", A, B, ri.ravel(), cj.ravel())
    den = metrics.denom_entries("N", "N", A, B, ri.ravel(), cj.ravel())
    err = metrics.err_comp(sub.ravel(), hi, lo, den)
    _say("kkr 2048 s=7 err_comp (sampled)", err)
    assert err <= 1e-12
