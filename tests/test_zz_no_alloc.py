"""ozaki_zgemm_noalloc, the emulated ZGEMM whose scratch is a fixed device
array: bit for bit equal to ozaki_zgemm on the same inputs, over calls in a row
whose sizes shrink (so the array holds the previous call's larger contents),
for both slice kinds and trans combinations, and the size limit and argument
errors reported without a launch."""
import numpy as np
import pytest

from tests.gpu_util import bits_equal, dev, host, mismatch_report, require_gpu, torch
from workloads import scaled_gaussian

import paper_2603_29975_amd as oz

pytestmark = pytest.mark.gpu

OZAKI_ERR_TOO_LARGE = 9
SCRATCH = 64 << 20


@pytest.fixture(autouse=True)
def _gpu():
    require_gpu()
    yield
    torch.cuda.synchronize()
    oz.ozaki_set_split("t7")


def _pair(m, n, k, s, seed, alpha=1.0, beta=0.0, trans=("N", "N")):
    """One product through ozaki_zgemm and through ozaki_zgemm_noalloc; both
    results on the host."""
    ta, tb = trans
    A, B = scaled_gaussian(m, n, k, seed=seed, rmax=12, complex_=True)
    if ta != "N":
        A = np.ascontiguousarray(A.T.conj() if ta == "C" else A.T)
    if tb != "N":
        B = np.ascontiguousarray(B.T.conj() if tb == "C" else B.T)
    C0 = np.random.default_rng(seed + 1).standard_normal((m, n)).astype(np.complex128)
    Ad, lda = dev(A)
    Bd, ldb = dev(B)
    out = []
    for fn in (oz.ozaki_zgemm, oz.ozaki_zgemm_noalloc):
        Cd, ldc = dev(C0)
        rc = fn(ta, tb, m, n, k, alpha, Ad, lda, Bd, ldb, beta, Cd, ldc, s)
        assert rc == 0, (fn.__name__, oz.ozaki_status_string(rc))
        out.append(host(Cd, m, n))
    return out


@pytest.mark.parametrize("split", ["t7", "b8"])
def test_noalloc_equals_zgemm_shrinking_calls(split):
    assert oz.ozaki_set_split(split) == 0
    s = 6
    # three products in a row, each smaller than the one before
    cases = [(200, 180, 3000, ("N", "N"), 0.5 - 0.25j, -1.0 + 0.5j),
             (300, 260, 700, ("T", "C"), 1.0, 0.0),
             (37, 45, 129, ("C", "N"), -2.0 + 1.0j, 0.75j)]
    for i, (m, n, k, trans, alpha, beta) in enumerate(cases):
        assert oz.ozaki_workspace_bytes("z", m, n, k, s) <= SCRATCH
        ref, got = _pair(m, n, k, s, seed=960 + i, alpha=alpha, beta=beta, trans=trans)
        torch.cuda.synchronize()
        assert bits_equal(got, ref), f"call {i} {(m, n, k)}\n" + mismatch_report(got, ref)


def test_noalloc_twice_smaller_second():
    """The required pair: a call, then a smaller one, each equal to ozaki_zgemm."""
    for i, (m, n, k) in enumerate([(512, 384, 1000), (70, 33, 65)]):
        ref, got = _pair(m, n, k, 7, seed=970 + i)
        assert bits_equal(got, ref), f"call {i}\n" + mismatch_report(got, ref)


def test_noalloc_limit_and_arguments():
    m = n = k = 1536
    assert oz.ozaki_workspace_bytes("z", m, n, k, 7) > SCRATCH
    C = torch.zeros((n, m), dtype=torch.complex128, device="cuda")
    A = torch.zeros((k, m), dtype=torch.complex128, device="cuda")
    B = torch.zeros((n, k), dtype=torch.complex128, device="cuda")
    assert oz.ozaki_zgemm_noalloc("N", "N", m, n, k, 1.0, A, m, B, k, 0.0, C, m, 7) == \
        OZAKI_ERR_TOO_LARGE
    assert oz.ozaki_zgemm_noalloc("X", "N", m, n, k, 1.0, A, m, B, k, 0.0, C, m, 7) == -1
    assert oz.ozaki_zgemm_noalloc("N", "N", 4, 5, 6, 1.0, A, 3, B, 6, 0.0, C, 4, 7) == -8
    assert oz.ozaki_zgemm_noalloc("N", "N", 4, 5, 6, 1.0, A, 4, B, 6, 0.0, C, 4, 0) == -14
    # a product that fits right after a rejected one is still correct
    ref, got = _pair(64, 64, 64, 7, seed=980)
    assert bits_equal(got, ref), mismatch_report(got, ref)
