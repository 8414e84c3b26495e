"""GPU parity of the blocked LU / inverse (ozaki_zgetrf, ozaki_zgetri) against
the CPU model oracle/lu.py: factors, pivots and inverse bit for bit with
emulated trailing updates (both slice kinds), close to it with the native FP64
updates, and the inverse's error against the native path falling with s on a
KKR-shaped matrix."""
import sys

import numpy as np
import pytest

from oracle import lu
from tests.gpu_util import bits_equal, dev, host, mismatch_report, require_gpu, torch
from workloads import kkr_operands

import paper_2603_29975_amd as oz

pytestmark = pytest.mark.gpu


@pytest.fixture(autouse=True)
def _gpu():
    require_gpu()
    yield
    torch.cuda.synchronize()
    oz.ozaki_set_split("t7")


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _gpu_lu_inv(A, nb, slices):
    n = A.shape[0]
    Ad, lda = dev(A)
    ipiv = torch.zeros(max(n, 1), dtype=torch.int64, device="cuda")
    rc = oz.ozaki_zgetrf(n, Ad, lda, ipiv, nb, slices)
    assert rc == 0, oz.ozaki_status_string(rc)
    Xd, ldx = dev(np.zeros((n, n), dtype=np.complex128))
    rc = oz.ozaki_zgetri(n, Ad, lda, ipiv, Xd, ldx, nb, slices)
    assert rc == 0, oz.ozaki_status_string(rc)
    return host(Ad, n, n), ipiv.cpu().numpy()[:n], host(Xd, n, n)


def _matrix(n, seed):
    rng = np.random.default_rng(seed)
    return rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n))


@pytest.mark.parametrize("kind,s,n,nb", [("b8", 6, 200, 64), ("t7", 5, 200, 64), ("b8", 4, 130, 32),
                                         ("t7", 7, 96, 96), ("b8", 6, 300, 128), ("t7", 6, 250, 100)])
def test_lu_and_inverse_bit_exact(kind, s, n, nb):
    A = _matrix(n, 1600 + n + s)
    assert oz.ozaki_set_split(kind) == 0
    _say("lu", kind, s, n, nb)
    LU, ipiv, X = _gpu_lu_inv(A, nb, s)
    upd = lu.update_model(kind, s)
    LU_ref, ipiv_ref, singular = lu.zgetrf(A, nb, upd)
    assert not singular
    assert np.array_equal(ipiv, ipiv_ref)
    assert bits_equal(LU, LU_ref), mismatch_report(LU, LU_ref)
    X_ref = lu.zgetri(LU_ref, ipiv_ref, nb, upd)
    assert bits_equal(X, X_ref), mismatch_report(X, X_ref)


@pytest.mark.parametrize("mode", ["columns", "leaf8", "leaf4", "leaf2", "auto"])
def test_lu_panel_modes_bit_exact(mode, monkeypatch):
    # the panel by columns (one pivot and one update launch each) and by leaves
    # of each width held in registers: the same factors, pivots and inverse bit
    # for bit. nb = 36 leaves a ragged last leaf in every panel (36 = 4*8 + 4),
    # and the NaN entry makes one pivot a NaN row.
    monkeypatch.setenv("OZAKI_LU_PANEL", mode)
    n, nb = 150, 36
    A = _matrix(n, 1790)
    A[97, 40] = np.nan
    assert oz.ozaki_set_split("t7") == 0
    _say("lu panel mode", mode)
    Ad, lda = dev(A)
    ipiv = torch.zeros(n, dtype=torch.int64, device="cuda")
    rc = oz.ozaki_zgetrf(n, Ad, lda, ipiv, nb, 5)
    assert rc == 8, oz.ozaki_status_string(rc)       # OZAKI_ERR_SINGULAR: a NaN pivot
    upd = lu.update_model("t7", 5)
    LU_ref, ipiv_ref, singular = lu.zgetrf(A, nb, upd)
    assert singular
    assert np.array_equal(ipiv.cpu().numpy(), ipiv_ref)
    assert bits_equal(host(Ad, n, n), LU_ref)
    B = _matrix(n, 1791)
    LU, ipiv, X = _gpu_lu_inv(B, nb, 5)
    LU_ref, ipiv_ref, singular = lu.zgetrf(B, nb, upd)
    assert not singular
    assert np.array_equal(ipiv, ipiv_ref)
    assert bits_equal(LU, LU_ref), mismatch_report(LU, LU_ref)
    assert bits_equal(X, lu.zgetri(LU_ref, ipiv_ref, nb, upd))


def test_lu_native_updates_close_to_the_model():
    n, nb = 180, 64
    A = _matrix(n, 1700)
    LU, ipiv, X = _gpu_lu_inv(A, nb, 0)
    LU_ref, ipiv_ref, _ = lu.zgetrf(A, nb, lu.update_model("native", 0))
    assert np.array_equal(ipiv, ipiv_ref)
    assert np.max(np.abs(LU - LU_ref)) <= 1e-12 * np.max(np.abs(LU_ref))
    inv = np.linalg.inv(A)
    assert np.max(np.abs(X - inv)) <= 1e-10 * np.max(np.abs(inv))


def test_lu_singular_is_reported_and_tiny_sizes():
    A = _matrix(40, 1710)
    A[:, 7] = 0.0
    Ad, lda = dev(A)
    ipiv = torch.zeros(40, dtype=torch.int64, device="cuda")
    assert oz.ozaki_zgetrf(40, Ad, lda, ipiv, 16, 6) == 8        # OZAKI_ERR_SINGULAR
    for n in (1, 2, 5):
        A1 = _matrix(n, 1720 + n)
        LU, ipiv1, X = _gpu_lu_inv(A1, 4, 6)
        LU_ref, ipiv_ref, _ = lu.zgetrf(A1, 4, lu.update_model("t7", 6))
        assert np.array_equal(ipiv1, ipiv_ref) and bits_equal(LU, LU_ref)


def test_kkr_inverse_error_falls_with_s():
    # KKR-shaped I - T G of 16 blocks of 32: inverse through emulated updates
    # against the same blocked algorithm with native FP64 updates
    A, _ = kkr_operands(16, seed=1730)
    _, _, X_nat = _gpu_lu_inv(A, 128, 0)
    scale = np.max(np.abs(X_nat))
    errs = {}
    assert oz.ozaki_set_split("b8") == 0
    for s in (3, 4, 5, 6, 7):
        _, _, X = _gpu_lu_inv(A, 128, s)
        errs[s] = float(np.max(np.abs(X - X_nat)) / scale)
    # the FP64 floor: how far two FP64 inverses of this matrix lie apart (ours
    # with native updates and LAPACK's through numpy)
    floor = float(np.max(np.abs(X_nat - np.linalg.inv(A))) / scale)
    _say("kkr 512 inverse error vs native (b8)", errs, "fp64 floor", floor)
    assert all(errs[s + 1] < errs[s] / 20 for s in (3, 4, 5, 6))
    # s = 7 with 8-bit slices: 1.2e-12 on this matrix (the floor is 2.5e-13, so
    # the product's error still shows; each further slice divides it by ~256)
    assert errs[7] < 2e-12


def _sequential_interchanges(n, ipiv):
    perm = np.arange(n)
    for c in range(n):
        p = int(ipiv[c])
        perm[c], perm[p] = perm[p], perm[c]
    return perm


@pytest.mark.parametrize("n,nb,seed", [(300, 64, 1740), (257, 1, 1741), (96, 96, 1742), (1030, 1024, 1743)])
def test_interchanges_as_gathers(n, nb, seed):
    # with LU = I (L and U both the identity) the inverse is X = P I exactly:
    # row r of X is row perm[r] of I for the interchanges applied in turn.
    # Pivot sequences with chains, repeats and rows far below the block.
    rng = np.random.default_rng(seed)
    ipiv = np.arange(n, dtype=np.int64)
    for c in range(n):
        mode = rng.integers(0, 4)
        if mode == 1:
            ipiv[c] = int(rng.integers(c, min(n, c + 3)))
        elif mode >= 2:
            ipiv[c] = int(rng.integers(c, n))
    Id, lda = dev(np.eye(n, dtype=np.complex128))
    piv = torch.from_numpy(ipiv).to("cuda")
    Xd, ldx = dev(np.zeros((n, n), dtype=np.complex128))
    _say("interchanges", n, nb)
    rc = oz.ozaki_zgetri(n, Id, lda, piv, Xd, ldx, nb, 0)
    assert rc == 0, oz.ozaki_status_string(rc)
    X = host(Xd, n, n)
    perm = _sequential_interchanges(n, ipiv)
    assert np.array_equal(X, np.eye(n)[perm])


def test_nan_entry_is_the_pivot_like_the_model():
    # a NaN counts as the largest |Re| + |Im| (the first NaN row wins), so every
    # pivot stays inside the column and the factorization reports a singular pivot
    n, nb = 40, 16
    A = _matrix(n, 1750)
    A[5, 3] = complex(np.nan, 0.0)
    assert oz.ozaki_set_split("t7") == 0
    Ad, lda = dev(A)
    ipiv = torch.zeros(n, dtype=torch.int64, device="cuda")
    _say("lu nan pivot")
    assert oz.ozaki_zgetrf(n, Ad, lda, ipiv, nb, 6) == 8        # OZAKI_ERR_SINGULAR
    _, ipiv_ref, singular = lu.zgetrf(A, nb, lu.update_model("t7", 6))
    assert singular
    assert np.array_equal(ipiv.cpu().numpy(), ipiv_ref)


def test_lu_taller_than_one_pivot_batch():
    # more than 2048 rows below the diagonal (the pivot workgroup's second
    # batch of rows) for the first columns: factors and pivots bit-exact
    n, nb = 2100, 64
    A = _matrix(n, 1770)
    assert oz.ozaki_set_split("t7") == 0
    Ad, lda = dev(A)
    ipiv = torch.zeros(n, dtype=torch.int64, device="cuda")
    _say("lu tall", n, nb)
    rc = oz.ozaki_zgetrf(n, Ad, lda, ipiv, nb, 3)
    assert rc == 0, oz.ozaki_status_string(rc)
    LU = host(Ad, n, n)
    LU_ref, ipiv_ref, singular = lu.zgetrf(A, nb, lu.update_model("t7", 3))
    assert not singular
    assert np.array_equal(ipiv.cpu().numpy(), ipiv_ref)
    assert bits_equal(LU, LU_ref), mismatch_report(LU, LU_ref)
