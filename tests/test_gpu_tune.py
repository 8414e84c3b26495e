"""Tile autotuner of the fused slice GEMM: every tuning id gives the oracle's
result bit for bit; autotune, lookup and the JSON cache round trip."""
import json
import os
import sys

import numpy as np
import pytest

from oracle import ozaki
from tests.gpu_util import bits_equal, dev, host, mismatch_report, require_gpu, torch
from workloads import scaled_gaussian, uniform_binade

import paper_2603_29975_amd as oz

pytestmark = pytest.mark.gpu


@pytest.fixture(autouse=True)
def _gpu():
    require_gpu()
    oz.ozaki_tune_clear()
    yield
    torch.cuda.synchronize()
    oz.ozaki_tune_clear()


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


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


@pytest.mark.parametrize("kind,m,n,k,s", [("d", 200, 300, 130, 7), ("z", 130, 70, 100, 5),
                                          ("z", 257, 129, 190, 9), ("d", 65, 33, 700, 12)])
def test_every_tuning_id_bit_exact(kind, m, n, k, s):
    A, B = uniform_binade(m, n, k, seed=700 + s, complex_=kind == "z")
    ref = ozaki.ozaki_gemm("N", "N", A, B, s)
    for tid in range(oz.ozaki_tune_configs()):
        assert oz.ozaki_tune_set(kind, m, n, k, s, tid) == 0
        assert oz.ozaki_tune_get(kind, m, n, k, s) == tid
        _say("tuning id", tid, kind, (m, n, k), s)
        got = _gemm(kind, A, B, s)
        assert bits_equal(got, ref), f"id {tid}\n" + mismatch_report(got, ref)


@pytest.mark.parametrize("kind,s,k", [("d", 12, 11200), ("z", 7, 9600)])
def test_every_tuning_id_chunked_contraction(kind, s, k):
    # INT32 partial sums carried into int64 across contraction chunks
    m, n = 40, 36
    A, B = scaled_gaussian(m, n, k, seed=750 + s, rmax=20, complex_=kind == "z")
    ref = ozaki.ozaki_gemm("N", "N", A, B, s)
    for tid in range(oz.ozaki_tune_configs()):
        assert oz.ozaki_tune_set(kind, m, n, k, s, tid) == 0
        _say("chunked tuning id", tid, kind, k, s)
        got = _gemm(kind, A, B, s)
        assert bits_equal(got, ref), f"id {tid}\n" + mismatch_report(got, ref)


def test_every_tuning_id_alpha_beta():
    m, n, k, s = 97, 130, 65, 6
    A, B = uniform_binade(m, n, k, seed=780, complex_=True)
    rng = np.random.default_rng(781)
    C0 = rng.standard_normal((m, n)) + 1j * rng.standard_normal((m, n))
    alpha, beta = 0.5 - 1.25j, -2.0 + 0.5j
    ref = ozaki.ozaki_gemm("N", "N", A, B, s, alpha, beta, C0)
    for tid in range(oz.ozaki_tune_configs()):
        assert oz.ozaki_tune_set("z", m, n, k, s, tid) == 0
        got = _gemm("z", A, B, s, alpha, beta, C0)
        assert bits_equal(got, ref), f"id {tid}\n" + mismatch_report(got, ref)


def test_autotune_records_fastest_and_cache_round_trip(tmp_path):
    rc, best, ms = oz.ozaki_autotune("z", 512, 512, 512, 7, reps=5)
    assert rc == 0, oz.ozaki_status_string(rc)
    assert 0 <= best < oz.ozaki_tune_configs() and ms > 0
    _say("autotune 512 z s=7: id", best, "ms", ms)
    assert oz.ozaki_tune_get("z", 512, 512, 512, 7) == best
    path = str(tmp_path / "tune.json")
    assert oz.ozaki_tune_save(path) == 0
    doc = json.load(open(path))
    assert doc["format"] == "ozaki-tune-1"
    assert doc["arch"].startswith("gfx")
    assert doc["entries"] == [{"kind": "z", "slices": 7, "mb": 9, "nb": 10, "kb": 5, "id": best,
                               "ms": pytest.approx(ms, rel=1e-5, abs=1e-6)}]
    assert oz.ozaki_tune_clear() == 0
    assert oz.ozaki_tune_get("z", 512, 512, 512, 7) == 0
    assert oz.ozaki_tune_load(path) == 0
    assert oz.ozaki_tune_get("z", 512, 512, 512, 7) == best
    # another architecture's entries are ignored
    other = dict(doc, arch="gfx000")
    other["entries"] = [dict(doc["entries"][0], slices=6, id=oz.ozaki_tune_configs() - 1)]
    p2 = str(tmp_path / "other.json")
    with open(p2, "w") as f:
        f.write('{"format": "ozaki-tune-1", "arch": "gfx000", "entries": [\n')
        f.write(" " + json.dumps(other["entries"][0]) + "\n]}\n")
    assert oz.ozaki_tune_load(p2) == 0
    assert oz.ozaki_tune_get("z", 512, 512, 512, 6) == 0
    # malformed and missing files
    p3 = str(tmp_path / "bad.json")
    with open(p3, "w") as f:
        f.write('{"format": "ozaki-tune-1", "arch": "gfx950", "entries": [\n {"kind": "z", "slices": 99}\n]}\n')
    assert oz.ozaki_tune_load(p3) == 7
    assert oz.ozaki_tune_load(str(tmp_path / "missing.json")) == 7
    assert not os.path.exists(str(tmp_path / "missing.json"))


def test_autotuned_id_is_used_and_exact():
    m = n = k = 320
    s = 8
    A, B = uniform_binade(m, n, k, seed=790, complex_=True)
    rc, best, _ = oz.ozaki_autotune("z", m, n, k, s, reps=3)
    assert rc == 0
    assert oz.ozaki_tune_get("z", m, n, k, s) == best
    got = _gemm("z", A, B, s)
    ref = ozaki.ozaki_gemm("N", "N", A, B, s)
    assert bits_equal(got, ref), mismatch_report(got, ref)


@pytest.mark.parametrize("kind", ["d", "z"])
def test_diagonals_in_both_tile_orders(kind):
    # the raw-diagonal hook keeps the tuned tile order (configuration 0)
    from tests.test_gpu_parity import _gpu_diagonals, _ref_diagonals
    m, n, k, s = (200, 300, 130, 7) if kind == "d" else (130, 70, 100, 6)
    A, B = uniform_binade(m, n, k, seed=795, complex_=kind == "z")
    ref = _ref_diagonals(A, B, s)
    for tid in range(oz.ozaki_tune_configs()):
        assert oz.ozaki_tune_set(kind, m, n, k, s, tid) == 0
        got = _gpu_diagonals(kind, "N", "N", A, B, s)
        for t in ref:
            assert np.array_equal(got[t], ref[t]), f"id {tid} t={t}\n" + mismatch_report(got[t], ref[t])
