"""Long contractions: the INT32 accumulators carried exactly into int64 across
contraction chunks, with each persistent workgroup walking many output tiles
in turn (so its carry space is reused), for every tuning id and both slice
kinds; and the 16384^3 ill-conditioned complex product at full size, checked
bit for bit against the oracle on sampled rows and columns and against the
double-double reference on sampled entries."""
import os
import sys

import numpy as np
import pytest

from oracle import ozaki, ozaki_b8
from oracle.sampled import SampledReference
from tests.gpu_util import bits_equal, dev, host, mismatch_report, require_gpu, torch
from workloads import illcond_operands, scaled_gaussian

import paper_2603_29975_amd as oz

pytestmark = pytest.mark.gpu

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
TUNE_TABLE = os.path.join(ROOT, "paper_2603_29975_amd", "tune_gfx950.json")


@pytest.fixture(autouse=True)
def _gpu():
    require_gpu()
    oz.ozaki_tune_clear()
    yield
    torch.cuda.synchronize()
    oz.ozaki_tune_clear()
    oz.ozaki_set_grid_limit(0)
    oz.ozaki_set_split("t7")


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _model(split):
    return ozaki_b8.ozaki_gemm_b8 if split == "b8" else ozaki.ozaki_gemm


def _gemm(kind, A, B, s, alpha=1.0, beta=0.0, C0=None):
    m, k = A.shape
    n = B.shape[1]
    Ad, lda = dev(A)
    Bd, ldb = dev(B)
    dt = np.complex128 if kind == "z" else np.float64
    if C0 is None:
        C0 = np.full((m, n), np.nan, dtype=dt)
    Cd, ldc = dev(C0.astype(dt))
    fn = oz.ozaki_zgemm if kind == "z" else oz.ozaki_dgemm
    rc = fn("N", "N", m, n, k, alpha, Ad, lda, Bd, ldb, beta, Cd, ldc, s)
    assert rc == 0, oz.ozaki_status_string(rc)
    return host(Cd, m, n)


# Shapes: nkb = K'/32 above the chunk bound (693 blocks for trunc-7 s = 6, 682
# for 8-bit s = 6, 832 for s = 5), ragged in every dimension; with a grid of 3
# workgroups each walks 5..9 tiles of 128 x 128 (configuration 6) or more.
@pytest.mark.parametrize("split", ["t7", "b8"])
@pytest.mark.parametrize("kind,m,n,k,s", [("z", 300, 260, 13500, 6), ("z", 161, 97, 13500, 5),
                                          ("d", 200, 300, 26700, 6)])
def test_chunked_carry_many_tiles_every_id(split, kind, m, n, k, s):
    assert oz.ozaki_set_split(split) == 0
    A, B = scaled_gaussian(m, n, k, seed=820 + s + (kind == "z"), rmax=20, complex_=kind == "z")
    rng = np.random.default_rng(821)
    dt = np.complex128 if kind == "z" else np.float64
    C0 = rng.standard_normal((m, n)).astype(dt)
    alpha, beta = (0.75 - 0.5j, -1.0 + 0.25j) if kind == "z" else (0.75, -1.5)
    ref = _model(split)("N", "N", A, B, s, alpha, beta, C0)
    for limit in (3, 0):
        assert oz.ozaki_set_grid_limit(limit) == 0
        for tid in range(oz.ozaki_tune_configs()):
            assert oz.ozaki_tune_set(kind, m, n, k, s, tid) == 0
            _say(f"chunked {split} {kind} {(m, n, k)} s={s} grid limit {limit} tuning id {tid}")
            got = _gemm(kind, A, B, s, alpha, beta, C0)
            assert bits_equal(got, ref), f"id {tid} limit {limit}\n" + mismatch_report(got, ref)


# Contractions beyond the reach of the split accumulation (each diagonal's
# pairs over two INT32 sets: 1040 blocks for trunc-7 s = 7, 1365 for 8-bit
# s = 6, 1386 for trunc-7 s = 5), so every configuration takes the int64 carry;
# the shapes above are within it, where the configurations with one A' block
# per wave split instead of carrying.
@pytest.mark.parametrize("split,kind,m,n,k,s", [("t7", "z", 48, 40, 17000, 7),
                                                ("b8", "z", 40, 33, 22000, 6),
                                                ("t7", "d", 37, 29, 45000, 5)])
def test_chunked_beyond_split_reach_every_id(split, kind, m, n, k, s):
    assert oz.ozaki_set_split(split) == 0
    A, B = scaled_gaussian(m, n, k, seed=830 + s, rmax=20, complex_=kind == "z")
    rng = np.random.default_rng(831)
    dt = np.complex128 if kind == "z" else np.float64
    C0 = rng.standard_normal((m, n)).astype(dt)
    alpha, beta = (0.5 + 0.25j, 0.5 - 1.0j) if kind == "z" else (-0.75, 2.0)
    ref = _model(split)("N", "N", A, B, s, alpha, beta, C0)
    for tid in range(oz.ozaki_tune_configs()):
        assert oz.ozaki_tune_set(kind, m, n, k, s, tid) == 0
        _say(f"chunked beyond split {split} {kind} {(m, n, k)} s={s} tuning id {tid}")
        got = _gemm(kind, A, B, s, alpha, beta, C0)
        assert bits_equal(got, ref), f"id {tid}\n" + mismatch_report(got, ref)


def test_grid_limit_rejects_negative():
    assert oz.ozaki_set_grid_limit(-1) == -1
    assert oz.ozaki_set_grid_limit(0) == 0


def _upload_colmajor(X: np.ndarray):
    """Column-major device copy of the row-major host matrix X (rows x cols):
    uploaded as it is and transposed on the device."""
    t = torch.from_numpy(X).cuda()
    out = t.t().contiguous()
    del t
    return out


@pytest.mark.parametrize("split,s", [("b8", 6), ("t7", 7)])
def test_illcond_16384_full_size(split, s):
    """The 16384^3 ill-conditioned complex product (rows of A and columns of B
    scaled by 2^r, r in [-30, 30]; seed 1004) at the slice counts that meet
    1e-12, with the tuned tile table: 24 x 24 sampled entries of C bit for bit
    against the oracle model, and err_comp <= 1e-12 against double-double on
    4096 random entries plus 2 whole rows and 2 whole columns."""
    N = 16384
    _say(f"illcond 16384 {split} s={s}: generating operands")
    A, B = illcond_operands(N, N, N, seed=1004)
    Ad = _upload_colmajor(A)
    Bd = _upload_colmajor(B)
    Cd = torch.empty((N, N), dtype=torch.complex128, device="cuda")
    assert oz.ozaki_tune_load(TUNE_TABLE) == 0
    assert oz.ozaki_set_split(split) == 0
    _say(f"illcond 16384 {split} s={s}: tuning id {oz.ozaki_tune_get('z', N, N, N, s)}")
    rc = oz.ozaki_zgemm("N", "N", N, N, N, 1.0, Ad, N, Bd, N, 0.0, Cd, N, s)
    assert rc == 0, oz.ozaki_status_string(rc)
    torch.cuda.synchronize()
    _say("  product done; checking")
    rng = np.random.default_rng(1100 + s)
    rows = np.sort(np.concatenate([rng.choice(N, 22, replace=False), [0, N - 1]]))
    cols = np.sort(np.concatenate([rng.choice(N, 22, replace=False), [0, N - 1]]))
    got = Cd[torch.from_numpy(cols).cuda()][:, torch.from_numpy(rows).cuda()].cpu().numpy().T
    ref = _model(split)("N", "N", A[rows], B[:, cols], s)
    assert bits_equal(got, ref), mismatch_report(got, ref)
    Bt = Bd.cpu().numpy()
    sref = SampledReference(A, Bt=Bt, nrand=4096, nrows=2, ncols=2, seed=1200 + s)
    ri = torch.from_numpy(sref.ri).cuda()
    cj = torch.from_numpy(sref.cj).cuda()
    vals = Cd[cj, ri].cpu().numpy()
    err = sref.err_comp(vals)
    _say(f"  err_comp on {sref.count} entries: {err:.3e}")
    assert err <= 1e-12
    del Ad, Bd, Cd
    torch.cuda.empty_cache()
