"""Seeded synthetic inputs for the H^2-ULV solver.

This module holds only random-number draws and point layouts: no kernel
evaluation, no clustering, no linear algebra of the method.  Both the
independent CPU oracle (``oracle/``) and the HIP library's callers
(``tests/``, ``bench.py``) take their inputs from here, so that the two sides
see identical points, right-hand sides and sampling permutations.

Workloads (the geometry families the paper evaluates on, Section 6):
  * ``cube``   -- points uniform in the unit cube / square (seeded PCG64).
  * ``sphere`` -- a Fibonacci lattice on the unit sphere surface with a small
    uniform jitter; a stand-in for the paper's "evenly spaced points on a
    sphere surface" Laplace experiment (Section 6.2, Eq. 35).  The paper's
    hemoglobin meshes (Section 6.4) are not available; uniform cubes stand
    in for them.

Kernel identifiers follow the C ABI (``include/h2.h``):
  0 = regularised Laplace 1/(r+delta)
  1 = regularised Yukawa  exp(-kappa r)/(r+delta)
  2 = Gaussian            exp(-r^2/ell^2) + nugget [i==j]
  3 = Matern nu=3/2       (1+sqrt3 r/ell) exp(-sqrt3 r/ell) + nugget [i==j]
  4 = Yukawa with drift   exp(-kappa r)/(r+delta) (1 + beta (x_0 - y_0)/(r+delta))
                          (non-symmetric for beta != 0)
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np

LAPLACE, YUKAWA, GAUSSIAN, MATERN32, YUKAWA_DRIFT = 0, 1, 2, 3, 4


@dataclasses.dataclass(frozen=True)
class Kernel:
    id: int
    delta: float = 1e-3
    kappa: float = 1.0
    ell: float = 1.0
    nugget: float = 0.0
    beta: float = 0.0    # drift strength of the non-symmetric kernel (id 4)


def cube_points(n: int, dim: int = 3, seed: int = 0) -> np.ndarray:
    """n points uniform in [0,1)^dim, float64, row-major (n, dim)."""
    return np.random.default_rng(seed).random((n, dim))


def sphere_points(n: int, seed: int = 0, jitter: float = 1e-3) -> np.ndarray:
    """Fibonacci lattice on the unit sphere plus uniform jitter in [-j, j]^3.

    z_k = 1 - (2k+1)/n, phi_k = k * pi * (3 - sqrt 5); the jittered points are
    not projected back onto the sphere.
    """
    k = np.arange(n, dtype=np.float64)
    z = 1.0 - (2.0 * k + 1.0) / n
    phi = k * math.pi * (3.0 - math.sqrt(5.0))
    s = np.sqrt(np.maximum(0.0, 1.0 - z * z))
    p = np.stack([s * np.cos(phi), s * np.sin(phi), z], axis=1)
    p += np.random.default_rng(seed).uniform(-jitter, jitter, (n, 3))
    return p


def sample_perm(n: int, seed: int = 2) -> np.ndarray:
    """The sampling permutation pi of 0..n-1 (int64)."""
    return np.random.default_rng(seed).permutation(n).astype(np.int64)


def rhs(n: int, nrhs: int = 1, seed: int = 1) -> np.ndarray:
    """Standard-normal right-hand sides, (n, nrhs) float64."""
    return np.random.default_rng(seed).standard_normal((n, nrhs))


@dataclasses.dataclass
class Problem:
    """One kernel-matrix system: points, kernel and method parameters."""
    name: str
    points: np.ndarray
    kernel: Kernel
    leaf: int
    eta: float
    eps: float
    nrhs: int
    s_far: int = -1      # -1: take every candidate point (no sampling)
    s_near: int = -1
    max_rank: int = 0    # 0: no cap

    @property
    def n(self) -> int:
        return self.points.shape[0]

    @property
    def dim(self) -> int:
        return self.points.shape[1]

    def perm(self) -> np.ndarray:
        return sample_perm(self.n)

    def b(self) -> np.ndarray:
        return rhs(self.n, self.nrhs)


def laplace_cube(n: int = 2048, leaf: int = 128, eps: float = 1e-10,
                 eta: float = 1.0, s: int = -1) -> Problem:
    """Uniform cube, 1/(r+1e-3): the small plain-FP64 case (N=2048 default)."""
    return Problem("laplace_cube", cube_points(n, 3, 0), Kernel(LAPLACE, delta=1e-3),
                   leaf, eta, eps, 1, s, s)


def laplace_sphere(n: int = 65536, leaf: int = 256, eps: float = 1e-8,
                   eta: float = 1.0, nrhs: int = 16, s: int | None = None) -> Problem:
    """Sphere-surface Laplace 1/(r+1e-3), 16 RHS by default (N=65536)."""
    if s is None:
        s = 2 * leaf
    return Problem("laplace_sphere", sphere_points(n, 0), Kernel(LAPLACE, delta=1e-3),
                   leaf, eta, eps, nrhs, s, s)


def yukawa_cube(n: int = 262144, leaf: int = 256, eps: float = 1e-8,
                eta: float = 1.0, nrhs: int = 4, s: int | None = None) -> Problem:
    """Uniform cube, exp(-r)/(r+1e-3), 4 RHS (N=262144 default)."""
    if s is None:
        s = 2 * leaf
    return Problem("yukawa_cube", cube_points(n, 3, 0),
                   Kernel(YUKAWA, delta=1e-3, kappa=1.0), leaf, eta, eps, nrhs, s, s)


def yukawa_drift_cube(n: int = 4096, leaf: int = 128, eps: float = 1e-8, beta: float = 0.5,
                      eta: float = 1.0, nrhs: int = 1, s: int | None = None) -> Problem:
    """Uniform cube, the non-symmetric Yukawa kernel with a drift of strength
    beta along the first axis (the LU variant's test problem)."""
    if s is None:
        s = 2 * leaf
    return Problem("yukawa_drift_cube", cube_points(n, 3, 0),
                   Kernel(YUKAWA_DRIFT, delta=1e-3, kappa=1.0, beta=beta), leaf, eta, eps, nrhs, s, s)


def matern_cube(n: int = 1 << 20, leaf: int = 256, eps: float = 1e-6,
                eta: float = 1.0, nrhs: int = 1, s: int | None = None) -> Problem:
    """Uniform cube, Matern-3/2 with ell=0.2 plus 1e-4 I (N=2^20 default)."""
    if s is None:
        s = 2 * leaf
    return Problem("matern_cube", cube_points(n, 3, 0),
                   Kernel(MATERN32, ell=0.2, nugget=1e-4), leaf, eta, eps, nrhs, s, s)


def gaussian_batch(n_inst: int = 64, n_min: int = 4096, n_max: int = 32768,
                   leaf: int = 128, eps: float = 1e-6, eta: float = 1.0,
                   s: int | None = None, seed: int = 4) -> list[Problem]:
    """Independent 2-D Gaussian covariance systems.

    For each instance t, from one PCG64 stream seeded ``seed``: ell_t ~
    U[0.1, 0.5], N_t ~ U{n_min..n_max} (inclusive), then N_t points uniform in
    the unit square; Gaussian kernel exp(-r^2/ell_t^2) + 1e-4 [i==j].
    """
    if s is None:
        s = 2 * leaf
    rng = np.random.default_rng(seed)
    ells = rng.uniform(0.1, 0.5, n_inst)
    ns = rng.integers(n_min, n_max, n_inst, endpoint=True)
    out = []
    for t in range(n_inst):
        pts = rng.random((int(ns[t]), 2))
        out.append(Problem(f"gaussian_{t}", pts,
                           Kernel(GAUSSIAN, ell=float(ells[t]), nugget=1e-4),
                           leaf, eta, eps, 1, s, s))
    return out
