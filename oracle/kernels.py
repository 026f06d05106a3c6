"""Kernel functions G(x, y) of the dense matrices being solved.

Section 6.2 (Eq. 35): Laplace Green's function with 1e3 on the diagonal;
Section 6.4 (Eq. 36): Yukawa potential with all constants 1 and 1e3 on the
diagonal.  The regularised forms 1/(r+delta) and exp(-kappa r)/(r+delta) with
delta = 1e-3 give exactly that diagonal value at r = 0.  The Gaussian and
Matern-3/2 covariance kernels take a nugget added where the two point indices
are equal (by index, not by distance).

Distance: r = sqrt(sum_d (x_d - y_d)^2), summed over axes 0..d-1 in order.

A non-symmetric kernel for the LU variant (not in the paper, whose method is
stated for symmetric positive definite matrices): the Yukawa kernel with a
drift along the first axis,
    G(x, y) = exp(-kappa r) / (r + delta) * (1 + beta (x_0 - y_0) / (r + delta)).
Its symmetric part is the Yukawa kernel and the rest is skew-symmetric, so
x^T A x = x^T A_sym x: where the Yukawa matrix is positive definite, every
leading principal block of A is non-singular and an LU factorization without
pivoting exists.
"""
from __future__ import annotations

import math

import numpy as np

LAPLACE, YUKAWA, GAUSSIAN, MATERN32, YUKAWA_DRIFT = 0, 1, 2, 3, 4


def symmetric(kernel) -> bool:
    """Whether G(x, y) = G(y, x) for this kernel."""
    return kernel.id != YUKAWA_DRIFT or getattr(kernel, "beta", 0.0) == 0.0


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
    elif kid == YUKAWA_DRIFT:
        dx = X[:, 0][:, None] - Y[:, 0][None, :]
        v = np.exp(-kernel.kappa * r) / (r + kernel.delta) * (1.0 + kernel.beta * dx / (r + kernel.delta))
    else:
        raise ValueError(f"unknown kernel id {kid}")
    if kernel.nugget != 0.0 and ix is not None and iy is not None:
        v = v + kernel.nugget * (ix[:, None] == iy[None, :])
    return v


def dense(kernel, X: np.ndarray) -> np.ndarray:
    """The full N x N kernel matrix A_ij = G(x_i, x_j)."""
    idx = np.arange(X.shape[0])
    return evaluate(kernel, X, X, idx, idx)
