"""Per-element tolerances for the BF16 selector MLP's gradient (test helper).

The GPU kernels and the CPU mirror (oracle/selector.py) round the same
quantities to BF16 at the same points, but the GPU accumulates in FP32 (in its
own order) where the mirror uses FP64. Two results can therefore differ only
through (a) FP32 accumulation errors, (b) a BF16 rounding of slightly different
inputs landing on different neighbours and (c) a ReLU mask or the loss weight
decided differently for an input within the accumulation error of zero. This
module propagates an absolute bound U on the GPU-minus-mirror difference of
every intermediate through the forward and backward pass (first order plus the
U*U cross terms of products), so that each gradient entry gets a tolerance
derived from the arithmetic alone:
  FP32 sums of n terms:       gamma(n) * sum |terms|, gamma(n) = n u32 / (1 - n u32)
  BF16 rounding of b, |b - a| <= U:  bf is monotone, so |bf(b) - bf(a)| <=
                              bf(a + U) - bf(a - U), which is 0 unless a rounding
                              tie lies within U of a (then one BF16 step)
  ambiguous mask / weight:    the whole term that the decision switches
with u32 = 2^-24 (unit roundoff of FP32).
"""
from __future__ import annotations

import numpy as np

from oracle import selector as sel

U32 = 2.0 ** -24


def gamma(n):
    return n * U32 / (1.0 - n * U32)


def _bf_bound(val, U):
    """Bound on |bf(b) - bf(a)| over every b with |b - a| <= U (a = val): the
    spread of the BF16 roundings of the interval's ends (the rounding is
    monotone)."""
    return sel.bf16(val + U) - sel.bf16(val - U)


def gradient_bounds(theta, X, t, under):
    """(g_ref, U): the mirror's quantised gradient and the per-entry bound on
    |g_gpu - g_ref| (both packed like theta)."""
    p = sel.unpack(theta)
    q = sel.bf16
    B = X.shape[0]
    X16 = q(X)
    W1h, W2h, w3h = q(p["W1"]), q(p["W2"]), q(p["w3"])
    aW1, aW2, aw3 = np.abs(W1h), np.abs(W2h), np.abs(w3h)

    # forward
    H1pre = X16 @ W1h.T + p["b1"]
    U_H1 = gamma(X.shape[1] + 1) * (np.abs(X16) @ aW1.T + np.abs(p["b1"]))
    H1 = np.maximum(H1pre, 0.0)
    amb1 = np.abs(H1pre) <= U_H1                      # ReLU / mask decided within the error
    U_H1 = np.where(H1pre < -U_H1, 0.0, U_H1)         # clearly negative: 0 on both sides
    H1h = q(H1)
    U_H1h = _bf_bound(H1, U_H1)
    H2pre = H1h @ W2h.T + p["b2"]
    aH1h = np.abs(H1h)
    U_H2 = U_H1h @ aW2.T + gamma(129) * (aH1h @ aW2.T + np.abs(p["b2"]))
    H2 = np.maximum(H2pre, 0.0)
    amb2 = np.abs(H2pre) <= U_H2
    U_H2 = np.where(H2pre < -U_H2, 0.0, U_H2)
    y = H2 @ w3h + p["b3"][0]
    U_y = U_H2 @ aw3 + gamma(129) * (H2 @ aw3 + abs(p["b3"][0]))

    # loss head
    e = y - t
    w = np.where(y < t, under, 1.0)
    ambw = np.abs(e) <= U_y
    wmax = max(under, 1.0)
    dy = 2.0 * w * e / B
    U_dy = 2.0 / B * (wmax * U_y + np.where(ambw, abs(under - 1.0) * (np.abs(e) + U_y), 0.0))
    U_dy = U_dy + 4.0 * U32 * np.abs(dy)

    G2 = dy[:, None] * w3h[None, :] * (H2 > 0)
    full2 = np.abs(dy)[:, None] * aw3[None, :]
    U_G2 = U_dy[:, None] * aw3[None, :] + U32 * full2
    U_G2 = np.where(amb2, U_G2 + full2 + U_dy[:, None] * aw3[None, :], U_G2)
    dH2h = q(G2)
    U_dH2h = _bf_bound(G2, U_G2)
    adH2h = np.abs(dH2h)

    # parameter gradients
    gW2 = dH2h.T @ H1h
    U_gW2 = adH2h.T @ U_H1h + U_dH2h.T @ aH1h + U_dH2h.T @ U_H1h + gamma(B) * (adH2h.T @ aH1h)
    gb2 = dH2h.sum(axis=0)
    U_gb2 = U_dH2h.sum(axis=0) + gamma(B) * adH2h.sum(axis=0)
    gw3 = dy @ H2
    U_gw3 = np.abs(dy) @ U_H2 + U_dy @ H2 + U_dy @ U_H2 + gamma(B) * (np.abs(dy) @ H2)
    gb3 = np.array([dy.sum()])
    U_gb3 = np.array([U_dy.sum() + gamma(B) * np.abs(dy).sum()])

    G1 = dH2h @ W2h
    aG1 = adH2h @ aW2
    U_G1 = U_dH2h @ aW2 + gamma(128) * aG1
    G1m = G1 * (H1 > 0)
    U_G1m = np.where(amb1, U_G1 + aG1, U_G1)
    dH1h = q(G1m)
    U_dH1h = _bf_bound(G1m, U_G1m)
    adH1h = np.abs(dH1h)
    aX = np.abs(X16)
    gW1 = dH1h.T @ X16
    U_gW1 = U_dH1h.T @ aX + gamma(B) * (adH1h.T @ aX)
    gb1 = dH1h.sum(axis=0)
    U_gb1 = U_dH1h.sum(axis=0) + gamma(B) * adH1h.sum(axis=0)

    g = sel.pack({"W1": gW1, "b1": gb1, "W2": gW2, "b2": gb2, "w3": gw3, "b3": gb3})
    U = sel.pack({"W1": U_gW1, "b1": U_gb1, "W2": U_gW2, "b2": U_gb2, "w3": U_gw3, "b3": U_gb3})
    return g, U


def _regions(batch):
    """Byte offsets of the scratch regions (layout documented with
    ozaki_mlp_scratch_bytes in the C header)."""
    bp = (batch + 31) // 32 * 32
    sizes = [("xh", bp * 64 * 2), ("xht", bp * 64 * 2), ("h1", bp * 128 * 4), ("h1h", bp * 128 * 2),
             ("h1ht", bp * 128 * 2), ("h2", bp * 128 * 4), ("h2h", bp * 128 * 2),
             ("h2ht", bp * 128 * 2), ("dh2h", bp * 128 * 2), ("dh2ht", bp * 128 * 2),
             ("dh1h", bp * 128 * 2), ("dh1ht", bp * 128 * 2)]
    out, off = {}, 0
    for name, size in sizes:
        out[name] = off
        off += (size + 255) // 256 * 256
    return out, bp


def read_scratch(raw: np.ndarray, batch: int):
    """The GPU's intermediates as float64 arrays (rows < batch) from the raw
    scratch bytes."""
    offs, bp = _regions(batch)
    raw = raw.view(np.uint8)

    def bf(name, cols):
        u = raw[offs[name]: offs[name] + bp * cols * 2].view(np.uint16).astype(np.uint32) << 16
        return u.view(np.float32).astype(np.float64).reshape(bp, cols)[:batch]

    def f32(name, cols):
        return raw[offs[name]: offs[name] + bp * cols * 4].view(np.float32).astype(np.float64) \
            .reshape(bp, cols)[:batch]

    return dict(Xh=bf("xh", 64), H1=f32("h1", 128), H1h=bf("h1h", 128), H2=f32("h2", 128),
                dH2h=bf("dh2h", 128), dH1h=bf("dh1h", 128))


def stage_violations(theta, X, t, under, y_gpu, g_gpu, gpu):
    """Each GPU stage against the CPU mirror evaluated on that stage's GPU
    inputs (so that a BF16 tie decided differently upstream cannot spread):
    the tolerance of a stage is its own FP32 accumulation bound, and a BF16
    output may differ from the mirror's only where a rounding tie lies within
    that bound. Returns a list of (stage, worst excess) for violated stages."""
    p = sel.unpack(theta)
    q = sel.bf16
    W1h, W2h, w3h = q(p["W1"]), q(p["W2"]), q(p["w3"])
    aW2, aw3 = np.abs(W2h), np.abs(w3h)
    bad = []

    def check(name, got, ref, U):
        ex = np.abs(got - ref) - U
        if np.any(ex > 0):
            bad.append((name, float(ex.max())))

    Xh, H1, H1h, H2 = gpu["Xh"], gpu["H1"], gpu["H1h"], gpu["H2"]
    check("Xh", Xh, q(X), 0.0)
    pre1 = Xh @ W1h.T + p["b1"]
    check("H1", H1, np.maximum(pre1, 0.0), gamma(65) * (np.abs(Xh) @ np.abs(W1h).T + np.abs(p["b1"])))
    check("H1h", H1h, q(H1), 0.0)
    pre2 = H1h @ W2h.T + p["b2"]
    check("H2", H2, np.maximum(pre2, 0.0), gamma(129) * (np.abs(H1h) @ aW2.T + np.abs(p["b2"])))
    check("y", y_gpu, H2 @ w3h + p["b3"][0], gamma(129) * (H2 @ aw3 + abs(p["b3"][0])))
    c = dict(X16=Xh, H1=H1, H1h=H1h, H2=H2, W2h=W2h, w3h=w3h)
    g_ref, st = sel.backward_stages(y_gpu, c, t, under)
    dy = st["dy"]
    U_dy = 4.0 * U32 * np.abs(dy)                      # the GPU's FP32 e, w e, 2 w e / B
    G2 = dy[:, None] * w3h[None, :] * (H2 > 0)
    check("dH2h", gpu["dH2h"], st["dH2h"], _bf_bound(G2, U_dy[:, None] * aw3[None, :] + U32 * np.abs(G2)))
    dH2h = gpu["dH2h"]
    G1 = (dH2h @ W2h) * (H1 > 0)
    check("dH1h", gpu["dH1h"], q(G1), _bf_bound(G1, gamma(128) * (np.abs(dH2h) @ aW2)))
    # parameter gradients from the GPU's own BF16 inputs
    dH1h = gpu["dH1h"]
    B = X.shape[0]
    bp = (B + 31) // 32 * 32
    ref = sel.pack({"W1": dH1h.T @ Xh, "b1": dH1h.sum(axis=0), "W2": dH2h.T @ H1h,
                    "b2": dH2h.sum(axis=0), "w3": dy @ H2, "b3": np.array([dy.sum()])})
    U = sel.pack({"W1": gamma(bp) * (np.abs(dH1h).T @ np.abs(Xh)),
                  "b1": gamma(bp) * np.abs(dH1h).sum(axis=0),
                  "W2": gamma(bp) * (np.abs(dH2h).T @ np.abs(H1h)),
                  "b2": gamma(bp) * np.abs(dH2h).sum(axis=0),
                  "w3": np.abs(U_dy) @ H2 + gamma(B) * (np.abs(dy) @ H2),
                  "b3": np.array([U_dy.sum() + gamma(B) * np.abs(dy).sum()])})
    del g_ref
    check("gradient", g_gpu, ref, U)
    return bad
