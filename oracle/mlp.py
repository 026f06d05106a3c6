"""FP64 reference of the rank-predictor network (not part of the paper).

A multilayer perceptron 8 -> 64 -> 64 -> 1 with ReLU activations predicts
log2(1 + k_i) of a box from eight geometry features, trained with a
mean-squared-error loss and Adam (Kingma & Ba 2015).  Weights are row-major
W1 (64x8), b1 (64), W2 (64x64), b2 (64), W3 (1x64), b3 (1), packed in that
order into one flat vector of 4801 numbers.

Features of box i at level l (all computed from the cluster tree):
  0  l / L
  1  log2(number of points in the box)
  2  log(rho_i / ell), ell = kernel length scale (1 for Laplace/Yukawa)
  3  e_mid / e_max     (sorted bounding-box extents; 0 for a 2-D box's missing axis)
  4  e_min / e_max
  5  number of near boxes (j != i) at level l
  6  log2(1 + number of points in boxes that are not near at level l)
  7  -log10(eps)
"""
from __future__ import annotations

import math

import numpy as np

SIZES = [(64, 8), (64,), (64, 64), (64,), (1, 64), (1,)]
NPARAM = sum(int(np.prod(s)) for s in SIZES)


def unpack(theta: np.ndarray):
    out, o = [], 0
    for s in SIZES:
        n = int(np.prod(s))
        out.append(theta[o:o + n].reshape(s))
        o += n
    return out


def init(seed: int = 7) -> np.ndarray:
    """He-uniform weights, zero biases, from a PCG64 stream."""
    rng = np.random.default_rng(seed)
    parts = []
    for s in SIZES:
        if len(s) == 2:
            lim = math.sqrt(6.0 / s[1])
            parts.append(rng.uniform(-lim, lim, s).ravel())
        else:
            parts.append(np.zeros(s))
    return np.concatenate(parts)


def forward(theta: np.ndarray, X: np.ndarray):
    W1, b1, W2, b2, W3, b3 = unpack(theta)
    z1 = X @ W1.T + b1
    h1 = np.maximum(z1, 0.0)
    z2 = h1 @ W2.T + b2
    h2 = np.maximum(z2, 0.0)
    y = (h2 @ W3.T + b3)[:, 0]
    return y, (X, z1, h1, z2, h2)


def loss_and_grad(theta: np.ndarray, X: np.ndarray, t: np.ndarray):
    """MSE loss mean((y - t)^2) and its gradient w.r.t. the flat parameters."""
    W1, b1, W2, b2, W3, b3 = unpack(theta)
    y, (X, z1, h1, z2, h2) = forward(theta, X)
    n = X.shape[0]
    dy = 2.0 * (y - t) / n
    loss = float(np.mean((y - t) ** 2))
    gW3 = dy[None, :] @ h2
    gb3 = np.array([dy.sum()])
    dh2 = dy[:, None] * W3
    dz2 = dh2 * (z2 > 0)
    gW2 = dz2.T @ h1
    gb2 = dz2.sum(0)
    dh1 = dz2 @ W2
    dz1 = dh1 * (z1 > 0)
    gW1 = dz1.T @ X
    gb1 = dz1.sum(0)
    g = np.concatenate([gW1.ravel(), gb1, gW2.ravel(), gb2, gW3.ravel(), gb3])
    return loss, g


def adam_step(theta, g, m, v, step, lr=1e-3, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam update (step counts from 1); returns new (theta, m, v)."""
    m = b1 * m + (1.0 - b1) * g
    v = b2 * v + (1.0 - b2) * g * g
    mh = m / (1.0 - b1 ** step)
    vh = v / (1.0 - b2 ** step)
    return theta - lr * mh / (np.sqrt(vh) + eps), m, v


def features(tree, ell: float, eps: float) -> list:
    """Per level l = 1..L the (2^l, 8) feature matrix described above."""
    out = [None]
    n = tree.n
    for l in range(1, tree.L + 1):
        nb = 1 << l
        near = tree.near_of(l)
        sizes = np.array([e - s for (s, e) in tree.ranges[l]], dtype=np.float64)
        F = np.zeros((nb, 8))
        for i in range(nb):
            s, e = tree.ranges[l][i]
            ext = np.sort(np.pad(tree.extent[l][i], (0, 3 - tree.dim)))
            emax = ext[2] if ext[2] > 0 else 1.0
            near_pts = sum(sizes[j] for j in near[i])
            F[i] = [l / tree.L, math.log2(sizes[i]),
                    math.log(max(tree.radius[l][i], 1e-300) / ell),
                    ext[1] / emax, ext[0] / emax, len(near[i]) - 1,
                    math.log2(1.0 + n - near_pts), -math.log10(eps)]
        out.append(F)
    return out

