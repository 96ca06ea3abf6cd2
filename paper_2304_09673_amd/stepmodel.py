"""Training of the step model for the learned step (not in the paper).

Orchestration only: samples come from the device dump of the plain tracer
(st_trace_dump) and the training loop runs in the library
(st_train_step_model: standardisation, initial weights, sample order, Adam
over the gradient kernel).  PyTorch provides the device buffers.
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


def standardisation(X: np.ndarray) -> np.ndarray:
    """norm[16] = feature means, inverse standard deviations (floor 1e-6), as
    st_train_step_model computes them on the device (host check)."""
    X = np.asarray(X, dtype=np.float64)
    mu = X.mean(axis=0)
    sd = np.maximum(X.std(axis=0), 1e-6)
    return np.concatenate([mu, 1.0 / sd]).astype(np.float32)


def fit(X, T, epochs: int = 8, batch: int = 8192, lr: float = 3e-3, seed: int = 0, log=None,
        over_weight: float = 4.0):
    """Adam on the weighted squared error, on the device (st_train_step_model);
    returns (weights [1377], norm [16] CUDA tensors, losses per epoch)."""
    import torch
    Xd = torch.as_tensor(np.ascontiguousarray(X, dtype=np.float32)).cuda()
    Td = torch.as_tensor(np.ascontiguousarray(T, dtype=np.float32)).cuda()
    w, norm, losses = st.train_step_model(Xd, Td, epochs=epochs, batch=batch, lr=lr, over_weight=over_weight,
                                          seed=seed)
    if log:
        for ep, v in enumerate(losses):
            log(f"epoch {ep}: loss {v:.4f}")
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
