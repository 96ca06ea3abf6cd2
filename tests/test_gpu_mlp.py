"""Step-model kernels against the FP64 oracle (same binary16-rounded weights
and inputs), the matrix-instruction lane layout, Adam and training."""
from __future__ import annotations

import numpy as np
import pytest

import oracle

pytestmark = pytest.mark.gpu

# parameter tensors of the MLP: name, offset, size
TENSORS = [("W1", 0, 256), ("b1", 256, 32), ("W2", 288, 1024), ("b2", 1312, 32), ("w3", 1344, 32), ("b3", 1376, 1)]


def _st():
    from paper_2304_09673_amd import st
    return st


def _random_problem(seed, n, target_spread=True):
    rng = np.random.default_rng(seed)
    w = np.zeros(1377, dtype=np.float32)
    w[0:256] = rng.normal(0, 0.5, 256)
    w[256:288] = rng.normal(0, 0.1, 32)
    w[288:1312] = rng.normal(0, 0.25, 1024)
    w[1312:1344] = rng.normal(0, 0.1, 32)
    w[1344:1376] = rng.normal(0, 0.3, 32)
    w[1376] = 0.1
    x = rng.normal(0, 1, (n, 8)).astype(np.float32) * np.array([0.1, 1, 0.01, 3, 0.5, 2, 1.5, 2], np.float32) \
        + np.array([0.05, 0.9, 0.01, 4, -0.3, 3, 3.0, 2], np.float32)
    mu = x.mean(axis=0)
    inv = 1.0 / np.maximum(x.std(axis=0), 1e-3)
    norm = np.concatenate([mu, inv]).astype(np.float32)
    t = rng.uniform(1.0, 4.0, n).astype(np.float32) if target_spread else np.full(n, 2.0, np.float32)
    return w, norm, x, t


def _oracle_inputs(w, norm, x):
    """The device's inputs to the arithmetic: binary16 weights and standardised
    features computed in FP32, clamped to [-3, 3], then rounded to binary16."""
    xs = np.clip(((x - norm[:8]) * norm[8:]).astype(np.float32), -3.0, 3.0)
    return oracle.round_half(w.astype(np.float64)), oracle.round_half(xs.astype(np.float64))


def _rel_l2(a, b):
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-30))


def test_mfma_lane_layout():
    """One 32x32x8 binary16 product with small integers (exact in FP32)
    read back through the accumulator-row formula the inference relies on."""
    import torch
    st = _st()
    rng = np.random.default_rng(5)
    a = rng.integers(-4, 5, (32, 8)).astype(np.float32)
    b = rng.integers(-4, 5, (8, 32)).astype(np.float32)
    d = st.debug_mfma_probe(torch.as_tensor(a).cuda(), torch.as_tensor(b).cuda()).cpu().numpy()
    np.testing.assert_array_equal(d, a @ b)


@pytest.mark.parametrize("n", [1, 63, 64, 1000, 4099])
def test_forward_matches_oracle(n):
    import torch
    st = _st()
    w, norm, x, t = _random_problem(11 + n, n)
    tab = st.mlp_pack(torch.as_tensor(w).cuda(), torch.as_tensor(norm).cuda())
    om = st.mlp_forward(tab, torch.as_tensor(x).cuda()).cpu().numpy().astype(np.float64)
    wr, xr = _oracle_inputs(w, norm, x)
    _, om_ref, _ = oracle.mlp(wr, xr, t.astype(np.float64), grad=False)
    assert np.all((om >= 1.0) & (om <= 4.0))
    # binary16 hidden activations: a rounding-boundary tie may move one
    # activation by one binary16 step, so the bound is relative L2 plus a max
    assert _rel_l2(om, om_ref) <= 1e-3
    assert np.max(np.abs(om - om_ref)) <= 1e-2


@pytest.mark.parametrize("n,over", [(256, 4.0), (5000, 4.0), (5000, 16.0)])
def test_gradients_match_oracle(n, over):
    import torch
    st = _st()
    w, norm, x, t = _random_problem(101 + n, n)
    g, loss = st.mlp_grad(torch.as_tensor(w).cuda(), torch.as_tensor(norm).cuda(), torch.as_tensor(x).cuda(),
                          torch.as_tensor(t).cuda(), over_weight=over)
    g = g.cpu().numpy().astype(np.float64)
    wr, xr = _oracle_inputs(w, norm, x)
    loss_ref, _, g_ref = oracle.mlp(wr, xr, t.astype(np.float64), grad=True, over_weight=over)
    assert abs(float(loss.cpu()) - loss_ref) <= 1e-4 * abs(loss_ref)
    for name, off, size in TENSORS:
        e = _rel_l2(g[off:off + size], g_ref[off:off + size])
        assert e <= 1e-3, (name, e)


def test_empty_batch_zeroes_gradient():
    import torch
    st = _st()
    w, norm, x, t = _random_problem(3, 4)
    grad = torch.full((1377,), 7.0, device="cuda")
    loss = torch.full((1,), 7.0, device="cuda")
    st.mlp_grad(torch.as_tensor(w).cuda(), torch.as_tensor(norm).cuda(), torch.as_tensor(x[:0]).cuda(),
                torch.as_tensor(t[:0]).cuda(), grad=grad, loss=loss)
    assert float(grad.abs().max().cpu()) == 0.0 and float(loss.cpu()) == 0.0


def test_adam_update():
    """Adam (Kingma and Ba 2015) with bias correction, two updates."""
    import torch
    st = _st()
    rng = np.random.default_rng(8)
    n = 1377
    w0 = rng.normal(0, 1, n).astype(np.float32)
    g1 = rng.normal(0, 1, n).astype(np.float32)
    g2 = rng.normal(0, 1, n).astype(np.float32)
    w = torch.as_tensor(w0).cuda()
    m = torch.zeros_like(w)
    v = torch.zeros_like(w)
    lr, b1, b2, eps = 1e-2, 0.9, 0.999, 1e-8
    for k, g in enumerate((g1, g2), start=1):
        st.mlp_adam(w, m, v, torch.as_tensor(g).cuda(), k, lr=lr, beta1=b1, beta2=b2, eps=eps)
    wr = w0.astype(np.float64)
    mr = np.zeros(n)
    vr = np.zeros(n)
    for k, g in enumerate((g1, g2), start=1):
        mr = b1 * mr + (1 - b1) * g
        vr = b2 * vr + (1 - b2) * g.astype(np.float64) ** 2
        wr = wr - lr * (mr / (1 - b1 ** k)) / (np.sqrt(vr / (1 - b2 ** k)) + eps)
    np.testing.assert_allclose(w.cpu().numpy(), wr, rtol=0, atol=1e-5)


def test_forward_clamps_outlying_features():
    """Features far outside the standardisation range give a finite omega in
    [1, 4] equal to that of the clamped features."""
    import torch
    st = _st()
    w, norm, x, t = _random_problem(77, 256)
    x_far = x.copy()
    x_far[::2, 3] = 1e30
    x_far[1::2, 6] = -1e30
    tab = st.mlp_pack(torch.as_tensor(w).cuda(), torch.as_tensor(norm).cuda())
    om = st.mlp_forward(tab, torch.as_tensor(x_far).cuda()).cpu().numpy().astype(np.float64)
    assert np.isfinite(om).all() and np.all((om >= 1.0) & (om <= 4.0))
    wr, xr = _oracle_inputs(w, norm, x_far)
    _, om_ref, _ = oracle.mlp(wr, xr, t.astype(np.float64), grad=False)
    assert _rel_l2(om, om_ref) <= 1e-3


def test_training_reduces_loss():
    """A learnable target (a smooth function of two features) is fitted by the
    device kernels: the loss falls well below that of the initial model."""
    from paper_2304_09673_amd import stepmodel
    rng = np.random.default_rng(21)
    n = 32768
    x = rng.normal(0, 1, (n, 8)).astype(np.float32)
    t = (1.0 + 3.0 / (1.0 + np.exp(-(1.5 * x[:, 0] - x[:, 3])))).astype(np.float32)
    w, norm, losses = stepmodel.fit(x, t, epochs=12, batch=4096, lr=1e-2, seed=1)
    assert losses[-1] < 0.2 * losses[0], losses


def test_train_step_model_standardisation_and_loss():
    """st_train_step_model: the standardisation equals the FP64 host one, the
    trained model's loss (recomputed by st_mlp_grad) is below that of the
    initial model, the reported epoch losses fall, and a batch larger than
    the sample count trains on one batch."""
    import torch
    st = _st()
    from paper_2304_09673_amd import stepmodel
    rng = np.random.default_rng(5)
    n = 20000
    x = (rng.normal(0, 1, (n, 8)) * np.array([0.1, 1, 0.01, 3, 0.5, 2, 1.5, 2])
         + np.array([0.05, 0.9, 0.01, 4, -0.3, 3, 3.0, 2])).astype(np.float32)
    t = (1.0 + 3.0 / (1.0 + np.exp(-(1.5 * (x[:, 1] - 0.9) - (x[:, 3] - 4) / 3)))).astype(np.float32)
    xd, td = torch.as_tensor(x).cuda(), torch.as_tensor(t).cuda()
    w, norm, losses = st.train_step_model(xd, td, epochs=6, batch=2048, lr=1e-2, seed=3)
    np.testing.assert_allclose(norm.cpu().numpy(), stepmodel.standardisation(x), rtol=1e-5)
    assert len(losses) == 6 and losses[-1] < 0.5 * losses[0], losses
    _, l_end = st.mlp_grad(w, norm, xd, td)
    assert float(l_end.cpu()) < losses[0]
    w1, _, l1 = st.train_step_model(xd[:100], td[:100], epochs=2, batch=4096, lr=1e-2, seed=3)
    assert len(l1) == 2 and np.isfinite(w1.cpu().numpy()).all()
