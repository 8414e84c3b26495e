"""Batched ZGEMM (one batched scan, one batched split, grouped persistent GEMM,
captured HIP graph) against the CPU oracle, problem by problem, bit for bit."""
import os
import sys

import numpy as np
import pytest

from oracle import ozaki
from tests.gpu_util import bits_equal, dev, host, mismatch_report, require_gpu, torch
from workloads import batched_problems

import paper_2603_29975_amd as oz

pytestmark = pytest.mark.gpu


@pytest.fixture(autouse=True)
def _gpu():
    require_gpu()
    yield
    torch.cuda.synchronize()
    oz.ozaki_batched_graphs(True)
    oz.ozaki_batched_cache_clear()


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


class Batch:
    """Host operands, device buffers and oracle references of a batch."""

    def __init__(self, probs, trans, alphas, betas, C0s, slices):
        self.probs, self.trans, self.alphas, self.betas, self.C0s, self.slices = \
            probs, trans, alphas, betas, C0s, slices
        self.Ad, self.Bd, self.Cd = [], [], []
        self.lda, self.ldb, self.ldc = [], [], []
        for (A, B), (ta, tb), C0 in zip(probs, trans, C0s):
            a, la = dev(_stored(A, ta))
            b, lb = dev(_stored(B, tb))
            c, lc = dev(C0)
            self.Ad.append(a)
            self.Bd.append(b)
            self.Cd.append(c)
            self.lda.append(la)
            self.ldb.append(lb)
            self.ldc.append(lc)

    def reset_c(self):
        for c, C0 in zip(self.Cd, self.C0s):
            c.copy_(torch.from_numpy(np.ascontiguousarray(C0.T)).to(c.device))

    def run(self):
        nb = len(self.probs)
        ms = [A.shape[0] for A, _ in self.probs]
        ns = [B.shape[1] for _, B in self.probs]
        ks = [A.shape[1] for A, _ in self.probs]
        used = []
        rc = oz.ozaki_zgemm_batched([t[0] for t in self.trans], [t[1] for t in self.trans], ms, ns,
                                    ks, self.alphas, self.Ad, self.lda, self.Bd, self.ldb,
                                    self.betas, self.Cd, self.ldc, nb, self.slices, used)
        assert rc == 0, oz.ozaki_status_string(rc)
        assert used == list(self.slices)
        return [host(c, m, n) for c, m, n in zip(self.Cd, ms, ns)]

    def reference(self, b):
        A, B = self.probs[b]
        return ozaki.ozaki_gemm("N", "N", A, B, self.slices[b], self.alphas[b], self.betas[b],
                                self.C0s[b])


def _small_batch(seed=11, count=24):
    rng = np.random.default_rng(seed)
    sizes = []
    for b in range(count):
        m, n, k = (int(x) for x in rng.choice([1, 17, 32, 33, 64, 70, 96, 128, 160, 257], 3))
        sizes.append((m, n, k))
    ms, ns, ks = (np.array(x) for x in zip(*sizes))
    probs, _ = batched_problems(count, seed, max_spread=12.0, sizes=(ms, ns, ks))
    trans = [tuple(rng.choice(["N", "T", "C"], 2)) for _ in range(count)]
    alphas = [complex(*rng.standard_normal(2)) if b % 3 == 0 else 1.0 for b in range(count)]
    betas = [complex(*rng.standard_normal(2)) if b % 4 == 1 else 0.0 for b in range(count)]
    C0s = [(rng.standard_normal((m, n)) + 1j * rng.standard_normal((m, n))) for m, n, _ in sizes]
    slices = [int(rng.choice([5, 7, 9])) for _ in range(count)]
    return Batch(probs, trans, alphas, betas, C0s, slices)


def test_batched_bit_exact_mixed_sizes_trans_and_slices():
    bt = _small_batch()
    _say("batched small: slices", sorted(set(bt.slices)))
    got = bt.run()
    for b in range(len(bt.probs)):
        ref = bt.reference(b)
        assert bits_equal(got[b], ref), f"problem {b}\n" + mismatch_report(got[b], ref)


def test_batched_graph_replays_match_eager():
    bt = _small_batch(seed=12, count=16)
    refs = [bt.reference(b) for b in range(len(bt.probs))]
    for rep in range(3):
        bt.reset_c()
        # unrelated eager work between replays
        x = torch.randn(1 << 20, dtype=torch.float64, device="cuda")
        float((x * x).sum())
        got = bt.run()
        for b in range(len(bt.probs)):
            assert bits_equal(got[b], refs[b]), f"replay {rep} problem {b}"
    oz.ozaki_batched_graphs(False)
    bt.reset_c()
    got = bt.run()
    for b in range(len(bt.probs)):
        assert bits_equal(got[b], refs[b]), f"eager problem {b}"


def test_batched_quick_return_problems():
    rng = np.random.default_rng(13)
    probs, _ = batched_problems(4, 13, sizes=([40, 0, 33, 20], [30, 10, 0, 21], [50, 5, 7, 0]))
    C0s = [rng.standard_normal((A.shape[0], B.shape[1])) + 0j for A, B in probs]
    bt = Batch(probs, [("N", "N")] * 4, [1.0, 1.0, 0.0, 1.0], [0.5, 0.0, 2.0, 3.0], C0s, [7] * 4)
    got = bt.run()
    for b in range(4):
        ref = bt.reference(b)
        assert bits_equal(got[b], ref), b


def test_batched_full_size_sampled_problems():
    # The 512-problem workload (m, n, k in 32..1024, log-uniform; per-matrix
    # exponent spread up to 20 binades) at s = 7; eight problems are checked
    # in full against the oracle.
    probs, (ms, ns, ks) = batched_problems(512, 1003)
    nb = len(probs)
    bt = Batch(probs, [("N", "N")] * nb, [1.0] * nb, [0.0] * nb,
               [np.zeros((A.shape[0], B.shape[1]), dtype=np.complex128) for A, B in probs], [7] * nb)
    got = bt.run()
    rng = np.random.default_rng(5)
    order = np.argsort(ms * ns * ks)
    pick = list(rng.choice(nb, 6, replace=False)) + [int(order[-1]), int(order[0])]
    for b in pick:
        ref = bt.reference(b)
        assert bits_equal(got[b], ref), f"problem {b} ({ms[b]}x{ns[b]}x{ks[b]})"
    _say("batched 512: checked", pick)


def selector_weights():
    return os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))),
                        "paper_2603_29975_amd", "selector_weights.npz")


def _const_selector(value):
    from oracle import selector as sel
    theta = np.zeros(sel.P, dtype=np.float32)
    theta[sel.OFFS["b3"][0]] = value
    return theta


def test_automatic_slices_probe_raises_and_matches_fixed_model():
    # A selector that always predicts 3 slices: the residual probe must raise
    # every problem until its estimate meets the target; the result must equal
    # the model at the final slice count bit for bit.
    from oracle import dd, metrics
    from paper_2603_29975_amd import selector
    bt = _small_batch(seed=21, count=12)
    bt.slices = None
    target = 1e-11
    # the probe's safety factor calibrated on held-out pairs with the weights
    _, _, _, meta = selector.load(selector_weights(), with_meta=True)
    kappa = float(meta["kappa"])
    assert oz.ozaki_load_selector(_const_selector(3.0), 0.0, target, kappa) == 0
    nb = len(bt.probs)
    ms = [A.shape[0] for A, _ in bt.probs]
    ns = [B.shape[1] for _, B in bt.probs]
    ks = [A.shape[1] for A, _ in bt.probs]
    used = []
    bt.reset_c()
    rc = oz.ozaki_zgemm_batched([t[0] for t in bt.trans], [t[1] for t in bt.trans], ms, ns, ks,
                                bt.alphas, bt.Ad, bt.lda, bt.Bd, bt.ldb, bt.betas, bt.Cd, bt.ldc, nb,
                                None, used)
    assert rc == 0, oz.ozaki_status_string(rc)
    _say("automatic slices used", used)
    assert min(used) >= 3 and max(used) > 3
    for b in range(nb):
        got = host(bt.Cd[b], ms[b], ns[b])
        A, B = bt.probs[b]
        ref = ozaki.ozaki_gemm("N", "N", A, B, used[b], bt.alphas[b], bt.betas[b], bt.C0s[b])
        assert bits_equal(got, ref), f"problem {b}"
        if used[b] < 12 and bt.alphas[b] == 1.0 and bt.betas[b] == 0.0:
            hi, lo = dd.dd_gemm("N", "N", A, B)
            err = metrics.err_comp(got, hi, lo, metrics.abs_product("N", "N", A, B))
            assert err <= target, (b, used[b], err)


def test_automatic_slices_constant_twelve():
    bt = _small_batch(seed=22, count=6)
    assert oz.ozaki_load_selector(_const_selector(12.0), 0.5, 1e-11, 8.0) == 0
    nb = len(bt.probs)
    ms = [A.shape[0] for A, _ in bt.probs]
    ns = [B.shape[1] for _, B in bt.probs]
    ks = [A.shape[1] for A, _ in bt.probs]
    used = []
    rc = oz.ozaki_zgemm_batched([t[0] for t in bt.trans], [t[1] for t in bt.trans], ms, ns, ks,
                                bt.alphas, bt.Ad, bt.lda, bt.Bd, bt.ldb, bt.betas, bt.Cd, bt.ldc, nb,
                                None, used)
    assert rc == 0 and used == [12] * nb
