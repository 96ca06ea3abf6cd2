"""Training of the step model for the learned step (not in the paper).

Orchestration only: samples come from the device dump of the plain tracer
(st_trace_dump), gradients and updates from the library's kernels
(st_mlp_grad, st_mlp_adam).  The host draws the initial weights, computes the
feature standardisation once and shuffles the sample order once; PyTorch
provides the device buffers.
"""
from __future__ import annotations

import numpy as np

from . import st

OMEGA_MAX = 4.0


def collect(scenes, cap_per_scene: int = 1 << 20, tuning=None):
    """Runs the dump tracer over scenegen scenes; returns host arrays (X [n, 8], T [n])."""
    import torch
    xs, ts = [], []
    for sc in scenes:
        s = st.Scene(sc)
        s.build_abuffer(sc.camera, tuning)
        feats = torch.empty((cap_per_scene, 8), dtype=torch.float32, device="cuda")
        targ = torch.empty(cap_per_scene, dtype=torch.float32, device="cuda")
        n, _, _ = s.trace_dump(feats, targ)
        n = min(n, cap_per_scene)
        x = feats[:n].cpu().numpy()
        t = targ[:n].cpu().numpy()
        # the dump's slot order follows the device's scheduling: sort the
        # samples so that a training run depends on the samples only
        order = np.lexsort(np.concatenate([x, t[:, None]], axis=1).T[::-1])
        xs.append(x[order])
        ts.append(t[order])
        s.close()
    return np.concatenate(xs), np.concatenate(ts)


def init_weights(seed: int = 0) -> np.ndarray:
    """He-normal hidden layers, small output layer, b3 so that omega starts near 1.5."""
    rng = np.random.default_rng(seed)
    w = np.zeros(st.MLP_PARAMS, dtype=np.float32)
    w[0:256] = rng.normal(0.0, np.sqrt(2.0 / 8), 256)
    w[288:1312] = rng.normal(0.0, np.sqrt(2.0 / 32), 1024)
    w[1344:1376] = rng.normal(0.0, 0.1 / np.sqrt(32), 32)
    w[1376] = np.log(0.5 / (OMEGA_MAX - 1.0 - 0.5))   # sigmoid^-1((1.5 - 1) / 3)
    return w


def standardisation(X: np.ndarray) -> np.ndarray:
    """norm[16] = feature means, inverse standard deviations (floor 1e-6)."""
    X = np.asarray(X, dtype=np.float64)
    mu = X.mean(axis=0)
    sd = np.maximum(X.std(axis=0), 1e-6)
    return np.concatenate([mu, 1.0 / sd]).astype(np.float32)


def fit(X, T, epochs: int = 8, batch: int = 8192, lr: float = 3e-3, seed: int = 0, log=None,
        over_weight: float = 4.0):
    """Adam on the weighted squared error; returns (weights [1377], norm [16], losses per epoch)."""
    import torch
    rng = np.random.default_rng(seed)
    order = rng.permutation(X.shape[0])
    Xd = torch.as_tensor(np.ascontiguousarray(X[order], dtype=np.float32)).cuda()
    Td = torch.as_tensor(np.ascontiguousarray(T[order], dtype=np.float32)).cuda()
    norm = torch.as_tensor(standardisation(X)).cuda()
    w = torch.as_tensor(init_weights(seed)).cuda()
    m = torch.zeros_like(w)
    v = torch.zeros_like(w)
    grad = torch.empty_like(w)
    loss = torch.empty(1, dtype=torch.float32, device="cuda")
    n = Xd.shape[0]
    nb = max(1, n // batch)
    losses = []
    step = 0
    for ep in range(epochs):
        acc = torch.zeros(1, dtype=torch.float64)
        for b in range(nb):
            lo, hi = b * batch, min(n, (b + 1) * batch)
            st.mlp_grad(w, norm, Xd[lo:hi], Td[lo:hi], grad=grad, loss=loss, over_weight=over_weight)
            step += 1
            st.mlp_adam(w, m, v, grad, step, lr=lr)
            acc += loss.cpu().double() if b % 16 == 0 else 0.0
        losses.append(float(acc) / max(1, (nb + 15) // 16))
        if log:
            log(f"epoch {ep}: loss {losses[-1]:.4f}")
    return w, norm, losses


def save(path, weights, norm, meta: dict | None = None):
    """Weights and standardisation as a .npz (plain arrays, no pickled objects)."""
    import json
    np.savez(path, weights=np.asarray(weights.cpu() if hasattr(weights, "cpu") else weights, dtype=np.float32),
             norm=np.asarray(norm.cpu() if hasattr(norm, "cpu") else norm, dtype=np.float32),
             meta=np.frombuffer(json.dumps(meta or {}).encode(), dtype=np.uint8))


def load(path):
    import json
    z = np.load(path, allow_pickle=False)
    return z["weights"], z["norm"], json.loads(bytes(z["meta"]).decode() or "{}")
