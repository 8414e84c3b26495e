"""What the learned slice selector gains, checked against the double-double
oracle: the trained network (with the residual probe as fallback, at the
safety factor calibrated on held-out pairs) meets the 1e-11 target on every
problem of the 512-product batch with fewer INT8 operations than the smallest
uniform slice count that meets it; and the labels the network was trained on
(taken on the GPU against its native FP64 product) agree with labels taken
against double-double on a subsample of the training distribution."""
import os
import sys

import numpy as np
import pytest

from oracle import dd, metrics
from tests.gpu_util import require_gpu, torch
from workloads import batched_problems

import paper_2603_29975_amd as oz
from paper_2603_29975_amd import selector

pytestmark = pytest.mark.gpu

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
WEIGHTS = os.path.join(ROOT, "paper_2603_29975_amd", "selector_weights.npz")
TARGET = 1e-11


@pytest.fixture(autouse=True)
def _gpu():
    require_gpu()
    yield
    torch.cuda.synchronize()


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _dd_refs(pairs):
    """(hi, lo, |A||B|) of every pair on the host."""
    out = []
    for A, B in pairs:
        hi, lo = dd.dd_gemm("N", "N", A, B)
        out.append((hi, lo, metrics.abs_product("N", "N", A, B)))
    return out


def _run_batch(db, nb, slices, used=None):
    out = torch.zeros(db.nc, dtype=torch.complex128, device="cuda")
    pa, pb = db.ptrs(db.A, db.oa, 16), db.ptrs(db.B, db.ob, 16)
    po = db.ptrs(out, db.oc, 16)
    rc = oz.ozaki_zgemm_batched(["N"] * nb, ["N"] * nb, db.m, db.n, db.k, [1.0] * nb, pa, db.m,
                                pb, db.k, [0.0] * nb, po, db.m, nb, slices, used)
    assert rc == 0, oz.ozaki_status_string(rc)
    torch.cuda.synchronize()
    host = out.cpu().numpy()
    return [host[db.oc[b]:db.oc[b + 1]].reshape(int(db.n[b]), int(db.m[b])).T for b in range(nb)]


def _errs(results, refs):
    return np.array([metrics.err_comp(C, hi, lo, den) for C, (hi, lo, den) in zip(results, refs)])


@pytest.mark.timeout(900)
def test_learned_selector_meets_target_with_less_work():
    theta, margin, target, meta = selector.load(WEIGHTS, with_meta=True)
    assert target == TARGET
    kappa = float(meta["kappa"])
    pairs, _ = batched_problems(512, 1003)
    nb = len(pairs)
    _say(f"double-double references of {nb} products")
    refs = _dd_refs(pairs)
    db = selector.DeviceBatch(pairs)
    work = 8.0 * db.m * db.n * db.k
    tri = lambda s: s * (s + 1) // 2
    # the smallest uniform slice count meeting the target on every problem
    s_fixed = None
    for s in range(6, 13):
        err = _errs(_run_batch(db, nb, [s] * nb), refs)
        _say(f"fixed s = {s}: max err_comp {err.max():.3e}, {int(np.sum(err > TARGET))} over")
        if np.all(err <= TARGET):
            s_fixed = s
            break
    assert s_fixed is not None
    assert oz.ozaki_load_selector(theta, margin, target, kappa) == 0
    used = []
    res = _run_batch(db, nb, None, used)
    used = np.array(used)
    err = _errs(res, refs)
    ops_learned = float(np.sum(np.array([tri(s) for s in used]) * work))
    ops_fixed = float(tri(s_fixed) * np.sum(work))
    _say(f"learned: mean s {used.mean():.3f} (min {used.min()}, max {used.max()}), max err_comp "
         f"{err.max():.3e}, INT8 work {ops_learned / ops_fixed:.3f} of fixed s = {s_fixed}, "
         f"kappa {kappa:.2f}")
    assert np.all(err <= TARGET), (np.argmax(err), err.max(), used[np.argmax(err)])
    assert ops_learned < ops_fixed


@pytest.mark.timeout(900)
def test_labels_agree_with_double_double_subsample():
    # 1000 pairs of the training distribution (another seed), both size
    # families: the GPU's labels against its native FP64 product, and the
    # labels against double-double from the same emulated products
    rng_pairs = selector.generate_pairs(900, 2006) + selector.generate_pairs(100, 2007, mn_law=True)
    lab_gpu, errs_gpu = selector.label_pairs(rng_pairs, TARGET)
    refs = _dd_refs(rng_pairs)
    db = selector.DeviceBatch(rng_pairs)
    nb = len(rng_pairs)
    lab_dd = np.full(nb, selector.S_HI + 1)
    err_dd = np.zeros((nb, selector.S_HI - selector.S_LO + 1))
    for s in range(selector.S_LO, selector.S_HI + 1):
        err_dd[:, s - selector.S_LO] = _errs(_run_batch(db, nb, [s] * nb), refs)
    ok = err_dd <= TARGET
    lab_dd = np.where(ok.any(axis=1), ok.argmax(axis=1) + selector.S_LO, selector.S_HI + 1)
    agree = np.mean(lab_dd == lab_gpu)
    _say(f"labels: {agree:.4f} identical; histogram gpu {np.bincount(lab_gpu, minlength=14)[3:]}, "
         f"dd {np.bincount(lab_dd, minlength=14)[3:]}")
    # the native product's own componentwise error is at most 2k u (u = 2^-53)
    # per entry, so the two error tables differ by at most that much
    kmax = max(A.shape[1] for A, _ in rng_pairs)
    assert np.all(np.abs(err_dd - errs_gpu) <= 2 * 2 * kmax * 2.0 ** -53 + 1e-3 * err_dd)
    assert agree >= 0.995
    diff = np.nonzero(lab_dd != lab_gpu)[0]
    for i in diff:          # a label may move only where an error sits at the target
        s = min(lab_gpu[i], lab_dd[i])
        assert abs(err_dd[i, s - selector.S_LO] - TARGET) <= 0.05 * TARGET, i
