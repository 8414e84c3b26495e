"""Pins of the blocked LU / inverse model (CPU): with plain FP64 updates it
reproduces LAPACK's pivot sequence (scipy.linalg.lu_factor, same izamax
measure) and factors, and numpy's inverse; the emulated updates converge to
it as the slice count grows."""
import numpy as np
import pytest

from oracle import lu
from workloads import kkr_operands

scipy_linalg = pytest.importorskip("scipy.linalg")


def _matrix(n, seed):
    rng = np.random.default_rng(seed)
    return rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n))


@pytest.mark.parametrize("n,nb", [(1, 4), (37, 8), (96, 32), (130, 64)])
def test_native_updates_match_lapack_pivots_factors_and_inverse(n, nb):
    A = _matrix(n, n)
    LU, ipiv, singular = lu.zgetrf(A, nb, lu.update_model("native", 0))
    lu_ref, piv_ref = scipy_linalg.lu_factor(A)
    assert not singular
    assert np.array_equal(ipiv, piv_ref)
    assert np.max(np.abs(LU - lu_ref)) <= 1e-12 * max(1.0, np.max(np.abs(lu_ref)))
    X = lu.zgetri(LU, ipiv, nb, lu.update_model("native", 0))
    inv = np.linalg.inv(A)
    assert np.max(np.abs(X - inv)) <= 1e-10 * np.max(np.abs(inv))
    assert np.max(np.abs(X @ A - np.eye(n))) <= 1e-10


def test_singular_matrix_is_flagged():
    A = _matrix(12, 3)
    A[:, 5] = 0.0
    _, _, singular = lu.zgetrf(A, 4, lu.update_model("native", 0))
    assert singular


@pytest.mark.parametrize("kind", ["t7", "b8"])
def test_emulated_updates_converge_to_fp64(kind):
    A, _ = kkr_operands(4, seed=21)                 # 128 x 128 KKR-shaped
    ref = np.linalg.inv(A)
    errs = {}
    for s in (3, 4, 5, 6, 7):
        LU, ipiv, _ = lu.zgetrf(A, 32, lu.update_model(kind, s))
        X = lu.zgetri(LU, ipiv, 32, lu.update_model(kind, s))
        errs[s] = np.max(np.abs(X - ref)) / np.max(np.abs(ref))
    # condition number ~3e3: the inverse carries the product error times ~cond
    assert all(errs[s + 1] < errs[s] / 20 for s in (3, 4, 5, 6))
    assert errs[7] < (1e-10 if kind == "t7" else 1e-12)


def test_nan_counts_as_the_largest_pivot():
    # reading L2 for non-finite input: the first NaN row of the column is the
    # pivot, and the factorization is flagged singular
    A = _matrix(12, 1760)
    A[7, 0] = complex(np.nan, 1.0)
    A[9, 0] = complex(0.0, np.nan)
    A[4, 0] = 1e300
    _, ipiv, singular = lu.zgetrf(A, 4, lu.update_model("native", 0))
    assert singular
    assert ipiv[0] == 7
    assert all(ipiv[c] == c for c in range(1, 12))   # NaN everywhere below: the first row
