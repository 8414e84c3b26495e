"""Selector features and BF16 MLP kernels against the CPU oracle."""
import numpy as np
import pytest

from oracle import selector as sel
from tests.gpu_util import dev, require_gpu, torch
from tests.selector_bounds import gradient_bounds, read_scratch, stage_violations
from workloads import batched_problems, kkr_operands, uniform_binade

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


@pytest.mark.parametrize("case", ["binade_d", "kkr_z", "spread_z_T", "spread_z_C"])
def test_features_match_oracle(case):
    if case == "binade_d":
        A, B = uniform_binade(70, 40, 90, seed=3)
        ta = tb = "N"
    elif case == "kkr_z":
        A, B = kkr_operands(3, seed=4)
        ta = tb = "N"
    else:
        (A, B), = batched_problems(1, 5, sizes=([66], [33], [130]))[0]
        ta, tb = ("T", "N") if case == "spread_z_T" else ("C", "C")
    A[1, :5] = 0
    kind = "z" if np.iscomplexobj(A) else "d"
    m, k = A.shape
    n = B.shape[1]
    Ad, lda = dev(_stored(A, ta))
    Bd, ldb = dev(_stored(B, tb))
    feat = torch.zeros(64, dtype=torch.float32, device="cuda")
    assert oz.ozaki_features(kind, ta, tb, m, n, k, Ad, lda, Bd, ldb, feat) == 0
    got = feat.cpu().numpy()
    ref = sel.features("N", "N", A, B)
    assert np.array_equal(got[:63], ref[:63])
    assert abs(got[63] - ref[63]) <= 1e-7


def _state_with(theta):
    st = torch.zeros(oz.ozaki_mlp_state_bytes() // 4 + 16, dtype=torch.float32, device="cuda")
    st[: sel.P] = torch.from_numpy(theta.astype(np.float32)).cuda()
    assert oz.ozaki_mlp_refresh(st) == 0
    return st


def _theta(seed):
    rng = np.random.default_rng(seed)
    th = np.zeros(sel.P)
    p = sel.unpack(th)
    parts = {"W1": rng.standard_normal((128, 64)) * np.sqrt(2 / 64),
             "b1": rng.standard_normal(128) * 0.1,
             "W2": rng.standard_normal((128, 128)) * np.sqrt(2 / 128),
             "b2": rng.standard_normal(128) * 0.1,
             "w3": rng.standard_normal(128) * 0.3, "b3": np.array([5.0])}
    del p
    return sel.pack(parts).astype(np.float32).astype(np.float64)


@pytest.mark.parametrize("batch", [1, 37, 256])
def test_mlp_forward_backward_match_oracle(batch):
    rng = np.random.default_rng(batch)
    theta = _theta(10 + batch)
    X = rng.uniform(0, 1, (batch, 64)).astype(np.float32).astype(np.float64)
    t = rng.uniform(3, 10, batch).astype(np.float32).astype(np.float64)
    st = _state_with(theta)
    Xd = torch.from_numpy(X.astype(np.float32)).cuda()
    td = torch.from_numpy(t.astype(np.float32)).cuda()
    y = torch.zeros(batch, dtype=torch.float32, device="cuda")
    scratch = torch.zeros(oz.ozaki_mlp_scratch_bytes(batch) // 4 + 64, dtype=torch.float32, device="cuda")
    loss = torch.zeros(1, dtype=torch.float32, device="cuda")
    assert oz.ozaki_mlp_forward(st, batch, Xd, y, scratch) == 0
    assert oz.ozaki_mlp_backward(st, batch, y, td, 4.0, loss, scratch) == 0
    torch.cuda.synchronize()
    y_gpu = y.cpu().numpy().astype(np.float64)
    g = st[3 * sel.P: 4 * sel.P].cpu().numpy().astype(np.float64)
    # end to end, element by element, within the bound propagated from FP32
    # accumulation and BF16 ties through the whole network
    g_ref, U = gradient_bounds(theta, X, t, 4.0)
    g_mirror, L_ref = sel.backward(theta, X, t, 4.0)
    assert np.array_equal(g_ref, g_mirror)
    assert np.all(np.abs(g - g_ref) <= U), np.max(np.abs(g - g_ref) - U)
    y_ref, _ = sel.forward(theta, X)
    assert np.allclose(y_gpu, y_ref, rtol=2e-3, atol=2e-3)
    assert abs(loss.item() - L_ref) <= 5e-3 * L_ref
    # every stage on the GPU's own inputs, with that stage's tolerance only
    inter = read_scratch(scratch.cpu().numpy(), batch)
    assert stage_violations(theta, X, t, 4.0, y_gpu, g, inter) == []


def test_adam_step_matches_oracle():
    theta = _theta(3)
    st = _state_with(theta)
    rng = np.random.default_rng(4)
    X = rng.uniform(0, 1, (64, 64)).astype(np.float32)
    t = rng.uniform(3, 10, 64).astype(np.float32)
    scratch = torch.zeros(oz.ozaki_mlp_scratch_bytes(64) // 4 + 64, dtype=torch.float32, device="cuda")
    y = torch.zeros(64, dtype=torch.float32, device="cuda")
    Xd, td = torch.from_numpy(X).cuda(), torch.from_numpy(t).cuda()
    assert oz.ozaki_mlp_forward(st, 64, Xd, y, scratch) == 0
    assert oz.ozaki_mlp_backward(st, 64, y, td, 4.0, None, scratch) == 0
    torch.cuda.synchronize()
    g = st[3 * sel.P: 4 * sel.P].cpu().numpy().astype(np.float64)
    assert oz.ozaki_mlp_adam(st, 1e-3, 0.9, 0.999, 1e-8, 1) == 0
    torch.cuda.synchronize()
    th_ref, _, _ = sel.adam(theta, np.zeros(sel.P), np.zeros(sel.P), g, 1e-3, 0.9, 0.999, 1e-8, 1)
    th = st[: sel.P].cpu().numpy().astype(np.float64)
    assert np.allclose(th, th_ref, rtol=1e-5, atol=1e-7)


def test_training_reduces_loss():
    # a smooth target of the features: the network must fit it with Adam
    rng = np.random.default_rng(6)
    X = rng.uniform(0, 1, (512, 64)).astype(np.float32)
    t = (3 + 4 * X[:, :8].mean(axis=1) + 2 * X[:, 40]).astype(np.float32)
    st = torch.zeros(oz.ozaki_mlp_state_bytes() // 4 + 16, dtype=torch.float32, device="cuda")
    assert oz.ozaki_mlp_init(st, 1234) == 0
    scratch = torch.zeros(oz.ozaki_mlp_scratch_bytes(512) // 4 + 64, dtype=torch.float32, device="cuda")
    Xd, td = torch.from_numpy(X).cuda(), torch.from_numpy(t).cuda()
    y = torch.zeros(512, dtype=torch.float32, device="cuda")
    loss = torch.zeros(1, dtype=torch.float32, device="cuda")
    losses = []
    for step in range(1, 301):
        assert oz.ozaki_mlp_forward(st, 512, Xd, y, scratch) == 0
        assert oz.ozaki_mlp_backward(st, 512, y, td, 1.0, loss, scratch) == 0
        assert oz.ozaki_mlp_adam(st, 3e-3, 0.9, 0.999, 1e-8, step) == 0
        if step in (1, 300):
            losses.append(loss.item())
    assert losses[1] < losses[0] / 20, losses
