"""Rank predictor for the interpolative decompositions (not part of the paper).

An MLP 8 -> 64 -> 64 -> 1 (FP32) maps box geometry features to log2(1 + k),
where k is the rank the library's own pivoted QR finds at the handle's eps.
Training data comes from plain builds of smaller seeded problems; training
runs on the device through the library's gradient and Adam kernels
(h2_mlp_train_step).  A trained model is passed to h2_build as
params.rank_model: every box's basis buffer is then sized from the
prediction (plus a margin) before compression, and a box whose rank exceeds
its capacity falls back to a buffer of its own (h2_stats.rank_fallbacks).
"""
from __future__ import annotations

import numpy as np

from . import h2

NPARAM = 4801


def init_weights(seed: int = 7) -> np.ndarray:
    """He-uniform weights, zero biases (row-major W1 b1 W2 b2 W3 b3), float32."""
    rng = np.random.default_rng(seed)
    parts = []
    for shape in [(64, 8), (64,), (64, 64), (64,), (1, 64), (1,)]:
        if len(shape) == 2:
            lim = np.sqrt(6.0 / shape[1])
            parts.append(rng.uniform(-lim, lim, shape).ravel())
        else:
            parts.append(np.zeros(shape))
    return np.concatenate(parts).astype(np.float32)


def collect(problems) -> tuple[np.ndarray, np.ndarray]:
    """(features, log2(1 + k)) of every box of plain builds of `problems`."""
    import torch
    xs, ys = [], []
    for p in problems:
        H = h2.build(p.points, p.kernel, p.leaf, p.eta, p.eps, p.perm(), s_far=p.s_far,
                     s_near=p.s_near)
        f = H.box_features().cpu().numpy()
        _, ranks, _, _ = H.structure()
        xs.append(f)
        ys.append(np.log2(1.0 + ranks.astype(np.float64)).astype(np.float32))
        H.close()
        torch.cuda.synchronize()
    return np.concatenate(xs), np.concatenate(ys)


def train(X: np.ndarray, y: np.ndarray, steps: int = 2000, lr: float = 3e-3,
          seed: int = 7) -> tuple[np.ndarray, list]:
    """Full-batch Adam on the device; returns (weights, loss history)."""
    import torch
    dev = lambda a: torch.from_numpy(np.ascontiguousarray(a)).cuda()
    w = dev(init_weights(seed))
    m = torch.zeros_like(w)
    v = torch.zeros_like(w)
    g = torch.zeros_like(w)
    loss = torch.zeros(1, dtype=torch.float32, device="cuda")
    Xd, yd = dev(X.astype(np.float32)), dev(y.astype(np.float32))
    hist = []
    for s in range(1, steps + 1):
        h2.mlp_train_step(w, m, v, g, Xd, yd, s, lr, loss)
        if s == 1 or s % 100 == 0:
            hist.append(float(loss.item()))
    return w.cpu().numpy(), hist


def predict(w: np.ndarray, X: np.ndarray) -> np.ndarray:
    """Predicted ranks 2^y - 1 (float) for feature rows X."""
    import torch
    y = h2.mlp_forward(torch.from_numpy(np.ascontiguousarray(w)).cuda(),
                       torch.from_numpy(np.ascontiguousarray(X.astype(np.float32))).cuda())
    return np.exp2(y.cpu().numpy().astype(np.float64)) - 1.0
