"""GPU tests of the Fortran-BLAS interposer: DGEMM/ZGEMM on host arrays give
the oracle's model bit for bit (Ozaki-I by default, Ozaki-II when
configured), leave the rows of C beyond m untouched, and follow alpha/beta."""
import sys

import numpy as np
import pytest

from oracle import ozaki, ozaki2
from tests.gpu_util import bits_equal, mismatch_report, require_gpu, torch
from workloads import uniform_binade

pytestmark = pytest.mark.gpu


@pytest.fixture(autouse=True)
def _gpu():
    require_gpu()
    from paper_2603_29975_amd import blas
    blas.ozaki_blas_config(0, 0)
    yield
    blas.ozaki_blas_config(0, 0)
    torch.cuda.synchronize()


def _fortran(X, ld):
    """Column-major buffer with leading dimension ld >= rows holding X; the
    padding rows hold a marker value."""
    rows, cols = X.shape
    buf = np.full((ld, cols), 7.25, dtype=X.dtype, order="F")
    buf[:rows, :] = X
    return buf


def _stored(X, trans):
    t = trans.upper()
    if t == "N":
        return X
    if t == "T":
        return np.ascontiguousarray(X.T)
    return np.ascontiguousarray(np.conj(X.T))


@pytest.mark.parametrize("kind", ["d", "z"])
@pytest.mark.parametrize("ta,tb,cfg", [("N", "N", ("s", 7)), ("T", "C", ("s", 5)),
                                       ("N", "T", ("n", 14)), ("C", "N", ("n", 10))])
def test_interposer_matches_the_model(kind, ta, tb, cfg):
    from paper_2603_29975_amd import blas
    m, n, k = 150, 90, 70
    A, B = uniform_binade(m, n, k, seed=1200 + len(ta + tb), complex_=kind == "z")
    rng = np.random.default_rng(1201)
    C0 = rng.standard_normal((m, n))
    if kind == "z":
        C0 = C0 + 1j * rng.standard_normal((m, n))
    alpha, beta = (0.75 - 0.5j, 1.5 + 0.25j) if kind == "z" else (0.75, -1.5)
    As, Bs = _stored(A, ta), _stored(B, tb)
    Af, Bf, Cf = _fortran(As, As.shape[0] + 3), _fortran(Bs, Bs.shape[0] + 1), _fortran(C0, m + 5)
    if cfg[0] == "s":
        assert blas.ozaki_blas_config(cfg[1], 0) == 0
        ref = ozaki.ozaki_gemm("N", "N", A, B, cfg[1], alpha, beta, C0)
    else:
        assert blas.ozaki_blas_config(0, cfg[1]) == 0
        ref = ozaki2.ozaki2_gemm("N", "N", A, B, cfg[1], alpha, beta, C0)
    fn = blas.zgemm_ if kind == "z" else blas.dgemm_
    print("interposer", kind, ta, tb, cfg, flush=True)
    fn(ta, tb, m, n, k, alpha, Af, Af.shape[0], Bf, Bf.shape[0], beta, Cf, Cf.shape[0])
    got = Cf[:m]
    assert bits_equal(got, ref), mismatch_report(got, ref)
    assert np.all(Cf[m:] == 7.25)                        # rows beyond m untouched


def test_interposer_environment_and_beta_zero(monkeypatch):
    from paper_2603_29975_amd import blas
    m, n, k = 33, 20, 17
    A, B = uniform_binade(m, n, k, seed=1210, complex_=True)
    C = np.full((m, n), np.nan, dtype=np.complex128, order="F")   # beta = 0: C not read
    monkeypatch.setenv("OZAKI_BLAS_SLICES", "6")
    blas.zgemm_("N", "N", m, n, k, 1.0, np.asfortranarray(A), m, np.asfortranarray(B), k, 0.0, C, m)
    assert bits_equal(C, ozaki.ozaki_gemm("N", "N", A, B, 6))
    monkeypatch.setenv("OZAKI_BLAS_MODULI", "12")
    blas.zgemm_("N", "N", m, n, k, 1.0, np.asfortranarray(A), m, np.asfortranarray(B), k, 0.0, C, m)
    assert bits_equal(C, ozaki2.ozaki2_gemm("N", "N", A, B, 12))
    assert blas.ozaki_blas_release() == 0
