"""Kernel functions G(x, y) of the dense matrices being solved.

Section 6.2 (Eq. 35): Laplace Green's function with 1e3 on the diagonal;
Section 6.4 (Eq. 36): Yukawa potential with all constants 1 and 1e3 on the
diagonal.  The regularised forms 1/(r+delta) and exp(-kappa r)/(r+delta) with
delta = 1e-3 give exactly that diagonal value at r = 0.  The Gaussian and
Matern-3/2 covariance kernels take a nugget added where the two point indices
are equal (by index, not by distance).

Distance: r = sqrt(sum_d (x_d - y_d)^2), summed over axes 0..d-1 in order.
"""
from __future__ import annotations

import math

import numpy as np

LAPLACE, YUKAWA, GAUSSIAN, MATERN32 = 0, 1, 2, 3


def distances(X: np.ndarray, Y: np.ndarray) -> np.ndarray:
    """Euclidean distance matrix r_ij = ||X_i - Y_j||_2 (float64)."""
    s = np.zeros((X.shape[0], Y.shape[0]))
    for d in range(X.shape[1]):
        diff = X[:, d][:, None] - Y[:, d][None, :]
        s += diff * diff
    return np.sqrt(s)


def evaluate(kernel, X: np.ndarray, Y: np.ndarray,
             ix: np.ndarray | None = None, iy: np.ndarray | None = None) -> np.ndarray:
    """G(X, Y) for kernel ``kernel`` (an object with id, delta, kappa, ell, nugget).

    ``ix``/``iy`` are the global point indices of the rows/columns; the nugget
    is added where they coincide.
    """
    r = distances(X, Y)
    kid = kernel.id
    if kid == LAPLACE:
        v = 1.0 / (r + kernel.delta)
    elif kid == YUKAWA:
        v = np.exp(-kernel.kappa * r) / (r + kernel.delta)
    elif kid == GAUSSIAN:
        v = np.exp(-(r * r) / (kernel.ell * kernel.ell))
    elif kid == MATERN32:
        a = math.sqrt(3.0) * r / kernel.ell
        v = (1.0 + a) * np.exp(-a)
    else:
        raise ValueError(f"unknown kernel id {kid}")
    if kernel.nugget != 0.0 and ix is not None and iy is not None:
        v = v + kernel.nugget * (ix[:, None] == iy[None, :])
    return v


def dense(kernel, X: np.ndarray) -> np.ndarray:
    """The full N x N kernel matrix A_ij = G(x_i, x_j)."""
    idx = np.arange(X.shape[0])
    return evaluate(kernel, X, X, idx, idx)
