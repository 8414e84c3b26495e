"""Residual probe on the GPU against the oracle's exact-rational definition."""
import numpy as np
import pytest

from oracle import ozaki
from oracle.probe import probe_est
from tests.gpu_util import dev, require_gpu, torch
from workloads import kkr_operands, uniform_binade

import paper_2603_29975_amd as oz

pytestmark = pytest.mark.gpu


@pytest.fixture(autouse=True)
def _gpu():
    require_gpu()
    yield
    torch.cuda.synchronize()


def _stored(X, trans):
    t = trans.upper()
    if t == "N":
        return X
    if t == "T":
        return np.ascontiguousarray(X.T)
    return np.ascontiguousarray(np.conj(X.T))


def _gpu_est(kind, ta, tb, A, B, C, nvec, seed):
    m, k = A.shape
    n = B.shape[1]
    Ad, lda = dev(_stored(A, ta))
    Bd, ldb = dev(_stored(B, tb))
    Cd, ldc = dev(C)
    est = torch.full((m,), -1.0, dtype=torch.float64, device="cuda")
    rc = oz.ozaki_probe(kind, ta, tb, m, n, k, Ad, lda, Bd, ldb, Cd, ldc, nvec, seed, est)
    assert rc == 0, oz.ozaki_status_string(rc)
    torch.cuda.synchronize()
    return est.cpu().numpy()


@pytest.mark.parametrize("kind,ta,tb,s,nvec", [("d", "N", "N", 4, 1), ("d", "T", "N", 7, 3),
                                               ("z", "N", "C", 5, 2), ("z", "C", "T", 8, 4)])
def test_probe_matches_oracle(kind, ta, tb, s, nvec):
    m, n, k = 70, 45, 60
    A, B = uniform_binade(m, n, k, seed=900 + s, complex_=(kind == "z"))
    A[3] = 0.0                                    # a zero row: est 0 there
    C = ozaki.ozaki_gemm("N", "N", A, B, s)
    got = _gpu_est(kind, ta, tb, A, B, C, nvec, seed=1234 + s)
    ref = probe_est("N", "N", A, B, C, nvec, seed=1234 + s)
    assert got[3] == 0.0 and ref[3] == 0.0
    assert np.allclose(got, ref, rtol=1e-9, atol=0), np.max(np.abs(got - ref) / np.maximum(ref, 1e-300))


def test_probe_planted_error_closed_form():
    n = 64
    A = np.eye(n)
    C = np.eye(n)
    C[10, 50] = 3e-11
    got = _gpu_est("d", "N", "N", A, A, C, 2, seed=7)
    want = np.zeros(n)
    want[10] = 3e-11 * np.sqrt(n)
    assert np.allclose(got, want, rtol=1e-12, atol=0)


def test_probe_on_kkr_emulation_tracks_slices():
    A, B = kkr_operands(4, seed=1002)            # 128 x 128 complex
    ests = []
    for s in (4, 6, 8):
        C = ozaki.ozaki_gemm("N", "N", A, B, s)
        ests.append(_gpu_est("z", "N", "N", A, B, C, 2, seed=3).max())
    assert ests[0] > 1e3 * ests[1] > 1e6 * ests[2]
