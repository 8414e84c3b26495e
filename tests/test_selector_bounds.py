"""CPU checks of the per-element gradient tolerances used by the GPU MLP test:
they hold for an independent FP32 implementation of the same network (other
summation orders, BF16 at the same points), and a planted mistake in the
mirror's backward pass (a transposed weight, a dropped factor, a wrong mask,
a wrong weight of the loss) breaks them."""
import numpy as np
import pytest

from oracle import selector as sel
from tests.selector_bounds import gradient_bounds, stage_violations


def _theta(seed):
    rng = np.random.default_rng(seed)
    parts = {"W1": rng.standard_normal((128, 64)) * np.sqrt(2 / 64),
             "b1": rng.standard_normal(128) * 0.1,
             "W2": rng.standard_normal((128, 128)) * np.sqrt(2 / 128),
             "b2": rng.standard_normal(128) * 0.1,
             "w3": rng.standard_normal(128) * 0.3, "b3": np.array([5.0])}
    return sel.pack(parts).astype(np.float32).astype(np.float64)


def _inputs(batch, seed):
    rng = np.random.default_rng(seed)
    X = rng.uniform(0, 1, (batch, 64)).astype(np.float32).astype(np.float64)
    t = rng.uniform(3, 10, batch).astype(np.float32).astype(np.float64)
    return X, t


def _fp32_backward(theta, X, t, under, stages=False, plant=None):
    """The network in FP32 with BF16 roundings at the mirror's points, summing
    in an order of its own (reversed contraction, pairwise column sums); with
    stages, also y and the intermediates as the GPU's scratch holds them."""
    f = np.float32
    q = lambda v: sel.bf16(np.asarray(v, dtype=np.float32)).astype(np.float32)
    p = {k: np.asarray(v, dtype=np.float32) for k, v in sel.unpack(theta).items()}
    B = X.shape[0]
    X16 = q(X)
    W1h, W2h, w3h = q(p["W1"]), q(p["W2"]), q(p["w3"])
    H1 = np.maximum((X16[:, ::-1] @ W1h[:, ::-1].T).astype(f) + p["b1"], f(0))
    H1h = q(H1)
    H2 = np.maximum((H1h[:, ::-1] @ W2h[:, ::-1].T).astype(f) + p["b2"], f(0))
    y = np.zeros(B, dtype=f)
    for k in range(127, -1, -1):
        y = (y + w3h[k] * H2[:, k]).astype(f)
    y = y + p["b3"][0]
    t32 = t.astype(f)
    e = y - t32
    w = np.where(y < t32, f(under), f(1))
    dy = (f(2) * w * e / f(B)).astype(f)
    dH2h = q(dy[:, None] * w3h[None, :] * (H2 > 0))
    gW2 = dH2h[::-1].T @ H1h[::-1]
    gb2 = np.add.reduce(dH2h[::-1], axis=0, dtype=f)
    gw3 = dy[::-1] @ H2[::-1]
    gb3 = np.array([np.sum(dy[::-1], dtype=f)])
    dH1h = q(((dH2h @ (W2h.T if plant == "transposed_W2" else W2h)).astype(f)) * (H1 > 0))
    gW1 = dH1h[::-1].T @ X16[::-1]
    gb1 = np.add.reduce(dH1h[::-1], axis=0, dtype=f)
    g = sel.pack({"W1": gW1, "b1": gb1, "W2": gW2, "b2": gb2, "w3": gw3, "b3": gb3})
    if not stages:
        return g
    d = lambda v: np.asarray(v, dtype=np.float64)
    return g, d(y), dict(Xh=d(X16), H1=d(H1), H1h=d(H1h), H2=d(H2), dH2h=d(dH2h), dH1h=d(dH1h))


@pytest.mark.parametrize("batch", [1, 37, 256])
def test_bounds_mirror_and_fp32_implementation(batch):
    theta = _theta(10 + batch)
    X, t = _inputs(batch, batch)
    g_ref, U = gradient_bounds(theta, X, t, 4.0)
    g_mirror, _ = sel.backward(theta, X, t, 4.0)
    assert np.array_equal(g_ref, g_mirror)
    g32 = _fp32_backward(theta, X, t, 4.0)
    assert np.all(np.abs(g32 - g_ref) <= U), np.max(np.abs(g32 - g_ref) - U)
    # the end-to-end tolerance of the second layer and the head is a small
    # fraction of the entries it guards (the first layer's is wider: one BF16
    # tie in H1 moves a whole row of the backward pass; its stages are
    # checked one by one on the GPU's own intermediates)
    for name in ("W2", "w3"):
        o, shape = sel.OFFS[name]
        sz = int(np.prod(shape))
        gg, uu = np.abs(g_ref[o:o + sz]), U[o:o + sz]
        nz = gg > 0
        assert np.median(uu[nz] / gg[nz]) < 0.05, name


def _planted(theta, X, t, under, mistake):
    """The mirror's backward pass with one planted mistake."""
    q = sel.bf16
    y, c = sel.forward(theta, X)
    B = X.shape[0]
    e = y - t
    w = np.where(y < t, under, 1.0)
    if mistake == "no_under_weight":
        w = np.ones_like(w)
    dy = 2.0 * w * e / B
    if mistake == "dropped_two":
        dy = w * e / B
    mask2 = c["H2"] > 0
    if mistake == "mask_of_h1":
        mask2 = c["H1"] > 0
    dH2h = q(dy[:, None] * c["w3h"][None, :] * mask2)
    gw3 = dy @ c["H2"]
    gb3 = np.array([dy.sum()])
    gW2 = dH2h.T @ c["H1h"]
    if mistake == "transposed_gW2":
        gW2 = gW2.T
    gb2 = dH2h.sum(axis=0)
    W2 = c["W2h"].T if mistake == "transposed_W2" else c["W2h"]
    dH1h = q((dH2h @ W2) * (c["H1"] > 0))
    gW1 = dH1h.T @ c["X16"]
    gb1 = dH1h.sum(axis=0)
    return sel.pack({"W1": gW1, "b1": gb1, "W2": gW2, "b2": gb2, "w3": gw3, "b3": gb3})


@pytest.mark.parametrize("mistake", ["no_under_weight", "dropped_two", "mask_of_h1",
                                     "transposed_gW2", "transposed_W2"])
def test_planted_mistake_breaks_bounds(mistake):
    theta = _theta(300)
    X, t = _inputs(256, 301)
    g_ref, U = gradient_bounds(theta, X, t, 4.0)
    assert np.array_equal(_planted(theta, X, t, 4.0, None), g_ref)
    bad = _planted(theta, X, t, 4.0, mistake)
    assert np.any(np.abs(bad - g_ref) > U)


@pytest.mark.parametrize("batch", [1, 37, 256])
def test_stage_checks_accept_fp32_implementation(batch):
    theta = _theta(20 + batch)
    X, t = _inputs(batch, 50 + batch)
    g, y, inter = _fp32_backward(theta, X, t, 4.0, stages=True)
    assert stage_violations(theta, X, t, 4.0, y, g, inter) == []


def test_stage_checks_reject_planted_mistakes():
    theta = _theta(400)
    X, t = _inputs(256, 401)
    g, y, inter = _fp32_backward(theta, X, t, 4.0, stages=True, plant="transposed_W2")
    assert [name for name, _ in stage_violations(theta, X, t, 4.0, y, g, inter)] == ["dH1h"]
    g, y, inter = _fp32_backward(theta, X, t, 4.0, stages=True)
    inter = dict(inter)
    H1h = inter["H1h"].copy()
    H1h[3, 7] = -H1h[3, 7] if H1h[3, 7] != 0 else 1.0          # one wrong activation
    inter["H1h"] = H1h
    assert "H1h" in [name for name, _ in stage_violations(theta, X, t, 4.0, y, g, inter)]
    g2 = g.copy()
    o = sel.OFFS["W2"][0]
    g2[o + 5] *= 1.01                                            # one gradient entry off by 1%
    _, y, inter = _fp32_backward(theta, X, t, 4.0, stages=True)
    assert [name for name, _ in stage_violations(theta, X, t, 4.0, y, g2, inter)] == ["gradient"]
