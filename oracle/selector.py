"""Selector features and MLP: the plain CPU definitions.

TEST INFRASTRUCTURE ONLY.

Features of a product op(A) op(B) (64 floats):
  [0..31]   fraction of entries of op(A) with delta = e_i - E(a) in bin
            min(delta, 30); bin 31 counts zero entries
  [32..62]  the same for the columns of op(B): bins min(delta, 29), bin 30 zeros
  [63]      log2(k) / 16
E(a) is the frexp exponent of the entry (the larger over real and imaginary
parts for complex data); e_i is the row exponent of the emulation model.

MLP 64 -> 128 -> 128 -> 1 with ReLU. The GPU runs the matrix products on BF16
matrix cores; this mirror rounds the same quantities to BF16 (round to nearest
even, via FP32) at the same points and computes everything else in FP64:
  X16 = bf(X), W1h = bf(W1), W2h = bf(W2), w3h = bf(w3)
  H1 = relu(X16 W1h^T + b1),  H1h = bf(H1)
  H2 = relu(H1h W2h^T + b2),  y = H2 w3h + b3
Backward of L = mean(w (y - t)^2), w = under where y < t else 1:
  dy = 2 w (y - t) / B
  dH2h = bf(dy w3h [H2 > 0]);  gW3 = dy^T H2, gb3 = sum dy
  gW2 = dH2h^T H1h, gb2 = sum dH2h
  dH1h = bf((dH2h W2h) [H1 > 0]);  gW1 = dH1h^T X16, gb1 = sum dH1h
(the BF16 roundings are treated as identities in the backward pass).
With quantize=False every bf() is the identity: the exact gradient of the
unquantized network, which the finite-difference pin checks.
"""
from __future__ import annotations

import numpy as np

from .ozaki import op

IN, H = 64, 128
P = H * IN + H + H * H + H + H + 1
OFFS = {"W1": (0, (H, IN)), "b1": (H * IN, (H,)), "W2": (H * IN + H, (H, H)),
        "b2": (H * IN + H + H * H, (H,)), "w3": (H * IN + 2 * H + H * H, (H,)),
        "b3": (H * IN + 3 * H + H * H, (1,))}


def unpack(theta):
    theta = np.asarray(theta, dtype=np.float64)
    return {k: theta[o:o + int(np.prod(s))].reshape(s) for k, (o, s) in OFFS.items()}


def pack(parts):
    out = np.zeros(P)
    for k, (o, s) in OFFS.items():
        out[o:o + int(np.prod(s))] = np.asarray(parts[k], dtype=np.float64).ravel()
    return out


def bf16(x):
    """Round to BF16 (nearest even) through FP32, returned as float64."""
    f = np.asarray(x, dtype=np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    r = ((u + 0x7FFF + ((u >> 16) & 1)) >> 16) << 16
    return (r & 0xFFFFFFFF).astype(np.uint32).view(np.float32).astype(np.float64)


def _codes(X):
    """frexp exponent per entry (larger of Re and Im), 0 marks zero entries."""
    if np.iscomplexobj(X):
        a, b = np.abs(X.real), np.abs(X.imag)
        _, ea = np.frexp(a)
        _, eb = np.frexp(b)
        e = np.where(a == 0, eb, np.where(b == 0, ea, np.maximum(ea, eb)))
        zero = (a == 0) & (b == 0)
    else:
        _, e = np.frexp(np.abs(X))
        zero = X == 0
    return e.astype(np.int64), zero


def _hist(rows, nbins):
    """Histogram of delta over the rows of `rows` (row exponent from the row
    maximum, as the emulation model's exponent step)."""
    e, zero = _codes(rows)
    ee = np.where(zero, np.iinfo(np.int64).min, e)
    rmax = ee.max(axis=1)
    delta = rmax[:, None] - e
    bins = np.where(zero, nbins - 1, np.clip(delta, 0, nbins - 2))
    return np.bincount(bins.ravel(), minlength=nbins)[:nbins]


def features(transa, transb, A, B) -> np.ndarray:
    cplx = np.iscomplexobj(A) or np.iscomplexobj(B)
    dt = np.complex128 if cplx else np.float64
    opA = op(np.asarray(A, dtype=dt), transa)
    opB = op(np.asarray(B, dtype=dt), transb)
    m, k = opA.shape
    n = opB.shape[1]
    out = np.zeros(64, dtype=np.float32)
    out[:32] = _hist(opA, 32).astype(np.float32) / np.float32(m * k)
    out[32:63] = _hist(opB.T, 31).astype(np.float32) / np.float32(k * n)
    out[63] = np.float32(np.log2(float(k)) / 16.0)
    return out


def forward(theta, X, quantize=True):
    q = bf16 if quantize else (lambda v: np.asarray(v, dtype=np.float64))
    p = unpack(theta)
    X16 = q(X)
    W1h, W2h, w3h = q(p["W1"]), q(p["W2"]), q(p["w3"])
    H1 = np.maximum(X16 @ W1h.T + p["b1"], 0.0)
    H1h = q(H1)
    H2 = np.maximum(H1h @ W2h.T + p["b2"], 0.0)
    y = H2 @ w3h + p["b3"][0]
    return y, dict(X16=X16, H1=H1, H1h=H1h, H2=H2, W2h=W2h, w3h=w3h)


def loss(y, t, under):
    e = y - t
    w = np.where(y < t, under, 1.0)
    return float(np.mean(w * e * e))


def backward_stages(y, c, t, under, quantize=True):
    """The backward pass from the forward values y and c (X16, H1, H1h, H2,
    W2h, w3h as forward() returns them): the gradient (packed like theta) and
    the intermediates dy, dH2h, dH1h."""
    q = bf16 if quantize else (lambda v: np.asarray(v, dtype=np.float64))
    B = y.shape[0]
    e = y - t
    w = np.where(y < t, under, 1.0)
    dy = 2.0 * w * e / B
    dH2h = q(dy[:, None] * c["w3h"][None, :] * (c["H2"] > 0))
    gw3 = dy @ c["H2"]
    gb3 = np.array([dy.sum()])
    gW2 = dH2h.T @ c["H1h"]
    gb2 = dH2h.sum(axis=0)
    dH1h = q((dH2h @ c["W2h"]) * (c["H1"] > 0))
    gW1 = dH1h.T @ c["X16"]
    gb1 = dH1h.sum(axis=0)
    g = pack({"W1": gW1, "b1": gb1, "W2": gW2, "b2": gb2, "w3": gw3, "b3": gb3})
    return g, dict(dy=dy, dH2h=dH2h, dH1h=dH1h)


def backward(theta, X, t, under, quantize=True):
    y, c = forward(theta, X, quantize)
    g, _ = backward_stages(y, c, t, under, quantize)
    return g, loss(y, t, under)


def adam(theta, m, v, grad, lr, b1, b2, eps, step):
    """One Adam step (Kingma and Ba 2015) with bias correction."""
    m = b1 * m + (1 - b1) * grad
    v = b2 * v + (1 - b2) * grad * grad
    mh = m / (1 - b1 ** step)
    vh = v / (1 - b2 ** step)
    return theta - lr * mh / (np.sqrt(vh) + eps), m, v
