"""Training and evaluation of the learned slice-count selector.

Data come from the emulator itself: for each generated (A, B) pair the GPU
forms the emulated product at every slice count s = S_LO..12 (the batched
entry point) and the native FP64 matrix-core product as the reference; the
label is the smallest s whose componentwise error max |C_s - C_ref| /
(|A||B|) reaches the target (|A||B| is formed by the native kernel too). The
features are the library's (ozaki_features). Training runs the library's BF16
MLP kernels (forward, backward, Adam); PyTorch only holds device buffers and
does the elementwise bookkeeping of the labels (differences, ratios, maxima).

The paper tunes the emulation precision by hand per run (Sections 3.2 and 4:
mantissa bits 31..63, moduli 10..18) and notes that accuracy depends on the
operator as well as the precision; the selector makes that choice per product.
"""
from __future__ import annotations

import math
import time

import numpy as np

from . import (MLP_PARAMS, OzakiError, ozaki_features, ozaki_mlp_adam, ozaki_mlp_backward,
               ozaki_mlp_forward, ozaki_mlp_init, ozaki_mlp_scratch_bytes, ozaki_mlp_state_bytes,
               ozaki_native_dgemm, ozaki_native_zgemm, ozaki_zgemm_batched)

S_LO = 3
S_HI = 12
KAPPA = 8.0      # probe safety factor used when the weights file stores none
# What a weights file was trained on: the library's feature vector and network.
# A file stores it as `feature_spec`; load() refuses a file without it or with
# another one (weights trained on other features would be read as if they fit).
FEATURE_SPEC = ("ozaki-selector/1: features = op(A) row exponent offsets, bins 0..30 + zero "
                "(32); op(B) column offsets, bins 0..29 + zero (31); log2(k)/16; "
                f"network 64-128-128-1 ReLU, BF16 products, {MLP_PARAMS} FP32 parameters")


def pair_sizes(rng, count, mn_choices=(32, 64), kmax_j=32, mn_law=False):
    """k = 32 j with P(j) ~ 1/j (the batched law); m, n from mn_choices, or
    with mn_law from the same law as k (32..1024, the sizes of the batch)."""
    j = np.arange(1, kmax_j + 1)
    p = (1.0 / j) / np.sum(1.0 / j)
    if mn_law:
        m = rng.choice(j, count, p=p) * 32
        n = rng.choice(j, count, p=p) * 32
    else:
        m = rng.choice(mn_choices, count)
        n = rng.choice(mn_choices, count)
    k = rng.choice(j, count, p=p) * 32
    return m.astype(np.int64), n.astype(np.int64), k.astype(np.int64)


def kkr_rows(m, n, k, seed, block=32):
    """The first m rows of a KKR-shaped A = I - T G (k x k, blocks of 32: T
    block diagonal with entries of magnitude 10^U[-3,0] and uniform phase, G
    complex Gaussian decaying as 1 / (1 + block distance)) and a complex
    Gaussian B (k x n); only the needed block rows are drawn."""
    from workloads import complex_normal
    rng = np.random.default_rng(seed)
    rows = -(-m // block) * block
    G = complex_normal(rng, (rows, k))
    bi = np.arange(rows) // block
    bj = np.arange(k) // block
    G = G / (1.0 + np.abs(bi[:, None] - bj[None, :]))
    A = np.zeros((rows, k), dtype=np.complex128)
    A[np.arange(min(rows, k)), np.arange(min(rows, k))] = 1.0
    for I in range(rows // block):
        T = 10.0 ** rng.uniform(-3, 0, (block, block)) * np.exp(1j * rng.uniform(0, 2 * np.pi, (block, block)))
        sl = slice(I * block, (I + 1) * block)
        A[sl] -= T @ G[sl]
    B = complex_normal(rng, (k, n))
    return A[:m], B


def generate_pairs(count: int, seed: int, mn_choices=(32, 64), mn_law=False):
    """Complex (A, B) pairs from four families: per-entry binade spread,
    per-matrix exponent spread with row/column scaling, Gaussian with
    power-of-two row/column scaling, and KKR-shaped blocks."""
    from workloads import batched_problems, complex_normal
    rng = np.random.default_rng(seed)
    ms, ns, ks = pair_sizes(rng, count, mn_choices, mn_law=mn_law)
    fam = rng.integers(0, 4, count)
    pairs = []
    for i in range(count):
        m, n, k = int(ms[i]), int(ns[i]), int(ks[i])
        f = fam[i]
        sub = int(rng.integers(0, 2 ** 31))
        if f == 0:
            w = int(rng.integers(0, 13))
            r = np.random.default_rng(sub)
            A = (r.uniform(-1, 1, (m, k)) + 1j * r.uniform(-1, 1, (m, k))) * np.ldexp(1.0, r.integers(-w, w + 1, (m, k)))
            B = (r.uniform(-1, 1, (k, n)) + 1j * r.uniform(-1, 1, (k, n))) * np.ldexp(1.0, r.integers(-w, w + 1, (k, n)))
        elif f == 1:
            (A, B), = batched_problems(1, sub, sizes=([m], [n], [k]))[0]
        elif f == 2:
            r = np.random.default_rng(sub)
            A = complex_normal(r, (m, k)) * np.ldexp(1.0, r.integers(-30, 31, m))[:, None]
            B = complex_normal(r, (k, n)) * np.ldexp(1.0, r.integers(-30, 31, n))[None, :]
        else:
            A, B = kkr_rows(m, n, k, sub)
        pairs.append((np.ascontiguousarray(A, dtype=np.complex128),
                      np.ascontiguousarray(B, dtype=np.complex128)))
    return pairs


def generate_pairs_device(count: int, seed: int, mn_choices=(32, 64), mn_law=False):
    """The same four families as generate_pairs, drawn on the GPU with a seeded
    torch generator (training data only; the oracle-checked workloads use the
    numpy generators). Returns a list of (A, B) complex128 CUDA tensors."""
    import torch
    rng = np.random.default_rng(seed)
    gen = torch.Generator(device="cuda")
    gen.manual_seed(int(seed))
    ms, ns, ks = pair_sizes(rng, count, mn_choices, mn_law=mn_law)
    fam = rng.integers(0, 4, count)
    two = torch.tensor(2.0, dtype=torch.float64, device="cuda")

    def cn(shape):
        re = torch.randn(shape, generator=gen, dtype=torch.float64, device="cuda")
        im = torch.randn(shape, generator=gen, dtype=torch.float64, device="cuda")
        return torch.complex(re, im) / math.sqrt(2.0)

    def uni(shape, lo, hi):
        return torch.rand(shape, generator=gen, dtype=torch.float64, device="cuda") * (hi - lo) + lo

    def ints(shape, lo, hi):
        return torch.randint(lo, hi + 1, shape, generator=gen, device="cuda").to(torch.float64)

    out = []
    for i in range(count):
        m, n, k = int(ms[i]), int(ns[i]), int(ks[i])
        f = fam[i]
        if f == 0:
            w = int(rng.integers(0, 13))
            A = torch.complex(uni((m, k), -1, 1), uni((m, k), -1, 1)) * two.pow(ints((m, k), -w, w))
            B = torch.complex(uni((k, n), -1, 1), uni((k, n), -1, 1)) * two.pow(ints((k, n), -w, w))
        elif f == 1:
            sa, sb = rng.uniform(0.0, 20.0, 2)
            A = cn((m, k)) * two.pow(-torch.floor(sa * uni((m, k), 0, 1)))
            A = A * two.pow(ints((m,), 0, int(sa)))[:, None]
            B = cn((k, n)) * two.pow(-torch.floor(sb * uni((k, n), 0, 1)))
            B = B * two.pow(ints((n,), 0, int(sb)))[None, :]
        elif f == 2:
            A = cn((m, k)) * two.pow(ints((m,), -30, 30))[:, None]
            B = cn((k, n)) * two.pow(ints((n,), -30, 30))[None, :]
        else:
            rows = -(-m // 32) * 32
            bi = torch.arange(rows, device="cuda") // 32
            bj = torch.arange(k, device="cuda") // 32
            G = cn((rows, k)) / (1.0 + (bi[:, None] - bj[None, :]).abs().to(torch.float64))
            nbr = rows // 32
            mag = torch.pow(10.0, uni((nbr, 32, 32), -3, 0))
            ph = uni((nbr, 32, 32), 0, 2 * math.pi)
            T = torch.polar(mag, ph)
            TG = torch.bmm(T, G.reshape(nbr, 32, k).contiguous()).reshape(rows, k)
            eye = torch.zeros((rows, k), dtype=torch.complex128, device="cuda")
            d = min(rows, k)
            eye[torch.arange(d), torch.arange(d)] = 1.0
            A = (eye - TG)[:m]
            B = cn((k, n))
        out.append((A.contiguous(), B.contiguous()))
    return out


class DeviceBatch:
    """Column-major device copies of a list of complex pairs in flat buffers
    (pairs of numpy arrays or of CUDA tensors)."""

    def __init__(self, pairs):
        import torch
        self.pairs = pairs
        self.m = np.array([A.shape[0] for A, _ in pairs], dtype=np.int64)
        self.k = np.array([A.shape[1] for A, _ in pairs], dtype=np.int64)
        self.n = np.array([B.shape[1] for _, B in pairs], dtype=np.int64)
        sa, sb, sc = self.m * self.k, self.k * self.n, self.m * self.n
        self.oa = np.concatenate([[0], np.cumsum(sa)])
        self.ob = np.concatenate([[0], np.cumsum(sb)])
        self.oc = np.concatenate([[0], np.cumsum(sc)])
        if isinstance(pairs[0][0], np.ndarray):
            self.A = torch.from_numpy(np.concatenate([A.T.ravel() for A, _ in pairs])).cuda()
            self.B = torch.from_numpy(np.concatenate([B.T.ravel() for _, B in pairs])).cuda()
        else:
            self.A = torch.cat([A.t().contiguous().reshape(-1) for A, _ in pairs])
            self.B = torch.cat([B.t().contiguous().reshape(-1) for _, B in pairs])
        self.Aabs = self.A.abs()
        self.Babs = self.B.abs()
        self.nc = int(self.oc[-1])
        self.seg = torch.from_numpy(np.repeat(np.arange(len(pairs)), sc)).cuda()

    def ptrs(self, t, off, elem):
        base = t.data_ptr()
        return [base + int(o) * elem for o in off[:-1]]


def label_pairs(pairs, target: float, s_lo: int = S_LO, s_hi: int = S_HI, chunk: int = 2048,
                with_features: bool = False):
    """Smallest s in [s_lo, s_hi] with componentwise error <= target for each
    pair (s_hi + 1 when none reaches it), the error table err[pair, s] and,
    if asked, the features of every pair (a CUDA tensor)."""
    import torch
    labels = np.zeros(len(pairs), dtype=np.int64)
    errs = np.zeros((len(pairs), s_hi - s_lo + 1))
    feats = torch.zeros((len(pairs), 64), dtype=torch.float32, device="cuda") if with_features else None
    for c0 in range(0, len(pairs), chunk):
        sub = pairs[c0:c0 + chunk]
        db = DeviceBatch(sub)
        nb = len(sub)
        if with_features:
            pa0, pb0 = db.ptrs(db.A, db.oa, 16), db.ptrs(db.B, db.ob, 16)
            for b in range(nb):
                m, n, k = int(db.m[b]), int(db.n[b]), int(db.k[b])
                rc = ozaki_features("z", "N", "N", m, n, k, pa0[b], m, pb0[b], k, feats[c0 + b])
                if rc:
                    raise OzakiError(rc, "ozaki_features")
        ref = torch.zeros(db.nc, dtype=torch.complex128, device="cuda")
        den = torch.zeros(db.nc, dtype=torch.float64, device="cuda")
        pa, pb = db.ptrs(db.A, db.oa, 16), db.ptrs(db.B, db.ob, 16)
        paa, pba = db.ptrs(db.Aabs, db.oa, 8), db.ptrs(db.Babs, db.ob, 8)
        pr, pd = db.ptrs(ref, db.oc, 16), db.ptrs(den, db.oc, 8)
        for b in range(nb):
            m, n, k = int(db.m[b]), int(db.n[b]), int(db.k[b])
            rc = ozaki_native_zgemm("N", "N", m, n, k, 1.0, pa[b], m, pb[b], k, 0.0, pr[b], m)
            rc |= ozaki_native_dgemm("N", "N", m, n, k, 1.0, paa[b], m, pba[b], k, 0.0, pd[b], m)
            if rc:
                raise OzakiError(rc, "native reference")
        out = torch.zeros(db.nc, dtype=torch.complex128, device="cuda")
        po = db.ptrs(out, db.oc, 16)
        big = torch.full((nb,), 0.0, dtype=torch.float64, device="cuda")
        for s in range(s_lo, s_hi + 1):
            rc = ozaki_zgemm_batched(["N"] * nb, ["N"] * nb, db.m, db.n, db.k, [1.0] * nb, pa,
                                     db.m, pb, db.k, [0.0] * nb, po, db.m, nb, [s] * nb)
            if rc:
                raise OzakiError(rc, "ozaki_zgemm_batched")
            ratio = (out - ref).abs() / den
            ratio = torch.where(den > 0, ratio, torch.where((out - ref).abs() > 0,
                                                              torch.full_like(ratio, math.inf),
                                                              torch.zeros_like(ratio)))
            e = big.clone().scatter_reduce_(0, db.seg, ratio, reduce="amax", include_self=True)
            errs[c0:c0 + nb, s - s_lo] = e.cpu().numpy()
        ok = errs[c0:c0 + nb] <= target
        first = np.where(ok.any(axis=1), ok.argmax(axis=1) + s_lo, s_hi + 1)
        labels[c0:c0 + nb] = first
    if with_features:
        return labels, errs, feats
    return labels, errs


def features_of(pairs):
    import torch
    feats = torch.zeros((len(pairs), 64), dtype=torch.float32, device="cuda")
    for i, (A, B) in enumerate(pairs):
        m, k = A.shape
        n = B.shape[1]
        Ad = torch.from_numpy(np.ascontiguousarray(A.T)).cuda()
        Bd = torch.from_numpy(np.ascontiguousarray(B.T)).cuda()
        rc = ozaki_features("z", "N", "N", m, n, k, Ad, m, Bd, k, feats[i])
        if rc:
            raise OzakiError(rc, "ozaki_features")
    return feats


def train(feats, labels, epochs=20, batch=256, lr=1e-3, under=4.0, seed=1005, log=None):
    """Adam on the asymmetric squared loss; returns the FP32 parameters."""
    import torch
    n = feats.shape[0]
    y_t = torch.from_numpy(np.asarray(labels, dtype=np.float32)).cuda()
    state = torch.zeros(ozaki_mlp_state_bytes() // 4 + 16, dtype=torch.float32, device="cuda")
    if ozaki_mlp_init(state, seed):
        raise RuntimeError("mlp init")
    scratch = torch.zeros(ozaki_mlp_scratch_bytes(batch) // 4 + 64, dtype=torch.float32, device="cuda")
    out = torch.zeros(batch, dtype=torch.float32, device="cuda")
    loss = torch.zeros(1, dtype=torch.float32, device="cuda")
    rng = np.random.default_rng(seed)
    step = 0
    for ep in range(epochs):
        perm = torch.from_numpy(rng.permutation(n)).cuda()
        tot = 0.0
        nb = 0
        for s0 in range(0, n - batch + 1, batch):
            idx = perm[s0:s0 + batch]
            X = feats[idx].contiguous()
            t = y_t[idx].contiguous()
            step += 1
            rc = ozaki_mlp_forward(state, batch, X, out, scratch)
            rc |= ozaki_mlp_backward(state, batch, out, t, under, loss, scratch)
            rc |= ozaki_mlp_adam(state, lr, 0.9, 0.999, 1e-8, step)
            if rc:
                raise RuntimeError("mlp step failed")
            if s0 % (batch * 64) == 0:
                tot += loss.item()
                nb += 1
        if log:
            log(f"epoch {ep}: loss {tot / max(nb, 1):.4f}")
    return state[:MLP_PARAMS].cpu().numpy().copy()


def predict(theta, feats):
    import torch
    n = feats.shape[0]
    state = torch.zeros(ozaki_mlp_state_bytes() // 4 + 16, dtype=torch.float32, device="cuda")
    state[:MLP_PARAMS] = torch.from_numpy(np.asarray(theta, dtype=np.float32)).cuda()
    from . import ozaki_mlp_refresh
    ozaki_mlp_refresh(state)
    scratch = torch.zeros(ozaki_mlp_scratch_bytes(n) // 4 + 64, dtype=torch.float32, device="cuda")
    out = torch.zeros(n, dtype=torch.float32, device="cuda")
    if ozaki_mlp_forward(state, n, feats.contiguous(), out, scratch):
        raise RuntimeError("mlp forward")
    return out.cpu().numpy()


def calibrate_margin(pred, labels, coverage=0.99):
    """Smallest margin (multiple of 0.05 in [-2, 6]) with ceil(pred + margin) >=
    label for at least `coverage` of the pairs."""
    for mg in np.arange(-2.0, 6.0001, 0.05):
        s = np.clip(np.ceil(pred + mg), 1, S_HI)
        if np.mean(s >= np.minimum(labels, S_HI)) >= coverage:
            return float(mg)
    return 6.0


PROBE_SEED = 0x5EED0000   # the automatic mode probes round r with seed PROBE_SEED + r
PROBE_VECTORS = 2


def probe_table(pairs, slices, seeds):
    """For each pair, the emulated product at slices[i] (the batched entry
    point, alpha = 1, beta = 0) and, for every r in `seeds`, the residual
    probe's largest row estimate with the automatic mode's probe
    (PROBE_VECTORS sign vectors, seed PROBE_SEED + r). Returns an array
    (len(pairs), len(seeds))."""
    import torch
    from . import ozaki_probe
    db = DeviceBatch(pairs)
    nb = len(pairs)
    pa, pb = db.ptrs(db.A, db.oa, 16), db.ptrs(db.B, db.ob, 16)
    out = torch.zeros(db.nc, dtype=torch.complex128, device="cuda")
    po = db.ptrs(out, db.oc, 16)
    rc = ozaki_zgemm_batched(["N"] * nb, ["N"] * nb, db.m, db.n, db.k, [1.0] * nb, pa, db.m, pb,
                             db.k, [0.0] * nb, po, db.m, nb, [int(x) for x in slices])
    if rc:
        raise OzakiError(rc, "ozaki_zgemm_batched")
    est = torch.zeros((len(seeds), int(db.m.max())), dtype=torch.float64, device="cuda")
    res = torch.zeros((nb, len(seeds)), dtype=torch.float64, device="cuda")
    for b in range(nb):
        m, n, k = int(db.m[b]), int(db.n[b]), int(db.k[b])
        for x, r in enumerate(seeds):
            rc = ozaki_probe("z", "N", "N", m, n, k, pa[b], m, pb[b], k, po[b], m, PROBE_VECTORS,
                             PROBE_SEED + r, est[x])
            if rc:
                raise OzakiError(rc, "ozaki_probe")
        res[b] = est[:, :m].max(dim=1).values
    return res.cpu().numpy()


def simulate_auto(pred, margin, kappa, errs, est, target, s_lo=S_LO):
    """The automatic mode on labelled pairs, from tables: errs[i, s - s_lo]
    (componentwise error at s slices) and est[i, s - s_lo, r] (the probe's
    largest row estimate at s with seed PROBE_SEED + r). Pass p starts at
    s_p (s_0 = ceil(pred + margin)), probes with seed 2p, raises to s_p + 1
    if est * kappa > target, probes that with seed 2p + 1, and if the target is
    still missed starts pass p + 1 at s_p + 2 (up to S_HI). Returns the final
    slice counts and whether each pair then meets the target."""
    n = len(pred)
    s = np.clip(np.ceil(pred + margin), 1, S_HI).astype(int)
    s = np.maximum(s, s_lo)
    final = s.copy()
    active = np.ones(n, dtype=bool)
    idx = np.arange(n)
    for p in range(4):
        if not active.any():
            break
        r0 = min(2 * p, est.shape[2] - 1)
        r1 = min(2 * p + 1, est.shape[2] - 1)
        e0 = est[idx, final - s_lo, r0]
        raise0 = active & (e0 * kappa > target) & (final < S_HI)
        final = np.where(raise0, final + 1, final)
        e1 = est[idx, final - s_lo, r1]
        again = raise0 & (e1 * kappa > target) & (final < S_HI)
        final = np.where(again, np.minimum(final + 1, S_HI), final)
        active = again
    ok = errs[idx, final - s_lo] <= target
    return final, ok


def calibrate_auto(pred, errs, est, work, target, log=None):
    """Margin and probe safety factor kappa for the automatic mode, from
    held-out labelled pairs: among margins in [-1, 3] (steps of 0.05) and
    kappa in {1, 2, 4, ..., 2^14}, the setting with the least INT8 work
    (sum of s(s+1)/2 x work[i]) under which every pair meets the target
    after the mode's raises (simulate_auto). Returns (margin, kappa, stats)."""
    best = None
    tri = lambda v: v * (v + 1) / 2.0
    for margin in np.arange(-1.0, 3.0001, 0.05):
        for kappa in 2.0 ** np.arange(0, 15):
            final, ok = simulate_auto(pred, margin, kappa, errs, est, target)
            if not ok.all():
                continue
            w = float(np.sum(tri(final) * work))
            if best is None or w < best[0]:
                best = (w, float(margin), float(kappa), float(final.mean()))
            break   # a larger kappa only raises more
    if best is None:
        raise RuntimeError("no margin and kappa meet the target on every held-out pair")
    w, margin, kappa, mean_s = best
    if log:
        log(f"auto calibration: margin {margin:.2f}, kappa {kappa:g}, mean final s {mean_s:.3f}")
    return margin, kappa, {"mean_final_s": mean_s, "int8_work": w}


def save(path, theta, margin, target, meta):
    meta = {k: v for k, v in meta.items() if k != "feature_spec"}
    np.savez(path, theta=np.asarray(theta, dtype=np.float32), margin=np.float32(margin),
             target=np.float64(target), feature_spec=np.asarray(FEATURE_SPEC),
             **{k: np.asarray(v) for k, v in meta.items()})


def load(path, with_meta=False):
    """(theta, margin, target) of a saved selector, plus the dict of its other
    stored values when with_meta is set."""
    z = np.load(path, allow_pickle=False)
    spec = str(z["feature_spec"]) if "feature_spec" in z.files else None
    if spec != FEATURE_SPEC:
        raise ValueError(f"{path}: selector weights for features {spec!r}, the library computes "
                         f"{FEATURE_SPEC!r}")
    if z["theta"].size != MLP_PARAMS:
        raise ValueError(f"{path}: {z['theta'].size} parameters, the network has {MLP_PARAMS}")
    out = (z["theta"], float(z["margin"]), float(z["target"]))
    if with_meta:
        meta = {key: (z[key].item() if z[key].ndim == 0 else z[key]) for key in z.files
                if key not in ("theta", "margin", "target", "feature_spec")}
        return out + (meta,)
    return out


def evaluate_gain(theta, margin, target, kappa=8.0, pairs=None, steps=5, log=None):
    """Learned selector + probe versus the best fixed slice count on a batch.

    The fixed policy uses the smallest uniform s with every problem within the
    target (known from the true errors against the native FP64 product); the
    learned policy is ozaki_zgemm_batched in automatic mode. Returns a dict
    with slice counts, INT8 work, times and whether every problem meets the
    target at the slice count it got."""
    import torch
    from . import ozaki_load_selector, ozaki_status_string
    from workloads import batched_problems
    if pairs is None:
        pairs, _ = batched_problems(512, 1003)
    labels, errs = label_pairs(pairs, target)
    nb = len(pairs)
    m = np.array([A.shape[0] for A, _ in pairs])
    n = np.array([B.shape[1] for _, B in pairs])
    k = np.array([A.shape[1] for A, _ in pairs])
    work = 8.0 * m * n * k
    s_fixed = int(min(labels.max(), S_HI))
    db = DeviceBatch(pairs)
    pa, pb = db.ptrs(db.A, db.oa, 16), db.ptrs(db.B, db.ob, 16)
    out = torch.zeros(db.nc, dtype=torch.complex128, device="cuda")
    po = db.ptrs(out, db.oc, 16)
    rc = ozaki_load_selector(theta, margin, target, kappa)
    if rc:
        raise OzakiError(rc, "ozaki_load_selector")
    used = []

    def run_auto():
        r = ozaki_zgemm_batched(["N"] * nb, ["N"] * nb, m, n, k, [1.0] * nb, pa, m, pb, k,
                                [0.0] * nb, po, m, nb, None, used)
        if r:
            raise RuntimeError(ozaki_status_string(r))

    def run_fixed():
        r = ozaki_zgemm_batched(["N"] * nb, ["N"] * nb, m, n, k, [1.0] * nb, pa, m, pb, k,
                                [0.0] * nb, po, m, nb, [s_fixed] * nb)
        if r:
            raise RuntimeError(ozaki_status_string(r))

    def timed(fn):
        fn()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            fn()
        torch.cuda.synchronize()
        return (time.perf_counter() - t0) * 1e3 / steps

    t_auto = timed(run_auto)
    s_auto = np.array(used)
    t_fixed = timed(run_fixed)
    err_auto = np.array([errs[b, min(s_auto[b], S_HI) - S_LO] if s_auto[b] >= S_LO else np.inf
                         for b in range(nb)])
    pairs_of = lambda s: s * (s + 1) / 2
    res = {
        "problems": nb, "target": target, "s_fixed": s_fixed,
        "mean_s_learned": float(s_auto.mean()), "mean_label": float(np.minimum(labels, S_HI).mean()),
        "int8_ops_learned": float(np.sum(pairs_of(s_auto) * work)),
        "int8_ops_fixed": float(np.sum(pairs_of(s_fixed) * work)),
        "ms_learned": t_auto, "ms_fixed": t_fixed,
        "all_within_target_learned": bool(np.all(err_auto <= target)),
        "max_err_learned": float(err_auto.max()),
        "problems_raised_by_probe_or_over_label": int(np.sum(s_auto > np.minimum(labels, S_HI))),
        "problems_below_label": int(np.sum(s_auto < np.minimum(labels, S_HI))),
        "problems_over_target": int(np.sum(err_auto > target)),
        "kappa": kappa,
    }
    res["int8_work_ratio_learned_over_fixed"] = res["int8_ops_learned"] / res["int8_ops_fixed"]
    if log:
        log(res)
    return res


LAW_S_LO, LAW_S_HI = 5, 11   # label range of the pairs with batch-sized m, n


def labelled_set(count, seed, target, law_frac, chunk=4096, log=None, keep_pairs=False):
    """`count` generated pairs (a fraction law_frac of each chunk with m, n
    from the batch's size law, the rest with m, n in {32, 64}), labelled and
    featurised on the GPU. Returns (features, labels) and, with keep_pairs,
    the error table over S_LO..S_HI and the pairs."""
    import torch
    feats_l, labels_l, errs_l, kept = [], [], [], []
    for c0 in range(0, count, chunk):
        cnt = min(chunk, count - c0)
        nlaw = int(round(cnt * law_frac))
        for part, (num, law) in enumerate(((cnt - nlaw, False), (nlaw, True))):
            if num == 0:
                continue
            pairs = generate_pairs_device(num, seed * 1000003 + 2 * c0 + part, mn_law=law)
            lo, hi = (LAW_S_LO, LAW_S_HI) if law else (S_LO, S_HI)
            lab, err, f = label_pairs(pairs, target, s_lo=lo, s_hi=hi, with_features=True)
            feats_l.append(f)
            labels_l.append(lab)
            # errors over S_LO..S_HI: below lo counted as misses, above hi as at hi
            full = np.full((len(pairs), S_HI - S_LO + 1), np.inf)
            full[:, lo - S_LO:hi - S_LO + 1] = err
            full[:, hi - S_LO + 1:] = err[:, -1:]
            errs_l.append(full)
            if keep_pairs:
                kept += pairs
            del pairs
        if log and (c0 // chunk) % 8 == 0:
            log(f"{c0 + cnt} pairs labelled")
    out = (torch.cat(feats_l), np.concatenate(labels_l))
    if keep_pairs:
        out = out + (np.concatenate(errs_l), kept)
    return out


def main(argv=None):
    import argparse
    ap = argparse.ArgumentParser(description="train the slice-count selector on the GPU")
    ap.add_argument("--pairs", type=int, default=200_000)
    ap.add_argument("--law-frac", type=float, default=0.1,
                    help="share of pairs whose m, n follow the batch's size law (32..1024)")
    ap.add_argument("--kappa-pairs", type=int, default=16384,
                    help="held-out pairs (seed + 1) that calibrate the probe's safety factor")
    ap.add_argument("--target", type=float, default=1e-11)
    ap.add_argument("--epochs", type=int, default=20)
    ap.add_argument("--out", required=True)
    ap.add_argument("--seed", type=int, default=1005)
    args = ap.parse_args(argv)
    t0 = time.time()

    def log(*a):
        print(f"[{time.time() - t0:7.1f}s]", *a, flush=True)

    from . import ozaki_batched_graphs
    ozaki_batched_graphs(False)          # one-off batches: no graph capture
    feats, labels = labelled_set(args.pairs, args.seed, args.target, args.law_frac, log=log)
    # chunks mix both size families, so a random split keeps both in validation
    perm = np.random.default_rng(args.seed).permutation(len(labels))
    ntrain = int(len(labels) * 0.9)
    tr, va = perm[:ntrain], perm[ntrain:]
    import torch
    tr_d, va_d = torch.from_numpy(tr).cuda(), torch.from_numpy(va).cuda()
    log(f"label histogram (s = {S_LO}..{S_HI + 1}) {np.bincount(labels, minlength=S_HI + 2)[S_LO:]}")
    log("training")
    theta = train(feats[tr_d], labels[tr], epochs=args.epochs, seed=args.seed, log=log)
    pred = predict(theta, feats[va_d])
    margin = calibrate_margin(pred, labels[va])
    s_val = np.clip(np.ceil(pred + margin), 1, S_HI)
    cov = float(np.mean(s_val >= np.minimum(labels[va], S_HI)))
    log(f"validation: margin {margin:.2f}, coverage {cov:.4f}, "
        f"mean predicted s {s_val.mean():.3f}, mean label {labels[va].mean():.3f}")
    # the automatic mode's margin and probe safety factor from pairs of another
    # seed: the mode simulated from their error tables and probe estimates
    kfeat, klab, kerrs, kpairs = labelled_set(args.kappa_pairs, args.seed + 1, args.target,
                                              args.law_frac, keep_pairs=True)
    kpred = predict(theta, kfeat)
    nk = len(kpairs)
    est = np.full((nk, S_HI - S_LO + 1, 4), np.inf)
    for sv in range(S_LO, S_HI + 1):
        est[:, sv - S_LO, :] = probe_table(kpairs, [sv] * nk, seeds=(0, 1, 2, 3))
    work = np.array([8.0 * A.shape[0] * B.shape[1] * A.shape[1] for A, B in kpairs])
    auto_margin, kappa, st = calibrate_auto(kpred, kerrs, est, work, args.target, log=log)
    s_pred = np.clip(np.ceil(kpred + auto_margin), 1, S_HI)
    log(f"held-out pairs {nk}: mean label {np.mean(np.minimum(klab, S_HI)):.3f}, mean predicted s "
        f"{s_pred.mean():.3f}, mean final s {st['mean_final_s']:.3f}")
    ozaki_batched_graphs(True)
    save(args.out, theta, auto_margin, args.target,
         {"pairs": args.pairs, "seed": args.seed, "law_frac": args.law_frac, "val_coverage": cov,
          "coverage_margin": margin, "val_mean_s": s_val.mean(),
          "val_mean_label": labels[va].mean(), "kappa": kappa, "kappa_pairs": nk,
          "calib_mean_final_s": st["mean_final_s"]})
    log(f"saved {args.out}")


if __name__ == "__main__":
    main()
