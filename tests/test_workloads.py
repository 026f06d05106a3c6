"""The seeded input generators (workloads.py), which both the oracle and the
library's callers draw from: shapes, domains and the documented structure of
each family, and determinism per seed."""
import numpy as np

import workloads as W


def test_cube_points_are_uniform_in_the_unit_cube():
    P = W.cube_points(20000, 3, 0)
    assert P.shape == (20000, 3) and P.dtype == np.float64
    assert (P >= 0).all() and (P < 1).all()
    # a uniform draw: every octant holds about an eighth of the points
    occ = np.bincount(((P > 0.5) * [1, 2, 4]).sum(axis=1), minlength=8)
    assert np.all(np.abs(occ / 20000 - 0.125) < 0.01)
    assert np.array_equal(P, W.cube_points(20000, 3, 0))
    assert not np.array_equal(P, W.cube_points(20000, 3, 1))
    assert W.cube_points(100, 2, 0).shape == (100, 2)


def test_sphere_points_lie_within_the_jitter_of_the_unit_sphere():
    n, j = 4096, 1e-3
    P = W.sphere_points(n, 0, j)
    assert P.shape == (n, 3)
    r = np.linalg.norm(P, axis=1)
    assert np.all(np.abs(r - 1.0) <= np.sqrt(3) * j + 1e-12)
    # the lattice: z strictly decreasing in k up to the jitter, spanning (-1, 1)
    assert P[0, 2] > 1 - 2 / n - 2 * j and P[-1, 2] < -1 + 2 / n + 2 * j
    assert np.all(np.diff(P[:, 2]) < 2 * j)
    # without jitter the points are on the sphere
    assert np.allclose(np.linalg.norm(W.sphere_points(n, 0, 0.0), axis=1), 1.0, atol=1e-14)


def test_sampling_permutation_and_rhs():
    pi = W.sample_perm(1000)
    assert pi.dtype == np.int64 and np.array_equal(np.sort(pi), np.arange(1000))
    assert np.array_equal(pi, W.sample_perm(1000))
    b = W.rhs(500, 3, 1)
    assert b.shape == (500, 3) and np.isfinite(b).all()
    assert abs(b.mean()) < 0.1 and abs(b.std() - 1) < 0.1


def test_problem_families():
    p = W.yukawa_cube(n=4096, leaf=64, eps=1e-6, s=128)
    assert (p.n, p.dim, p.leaf, p.s_far, p.s_near) == (4096, 3, 64, 128, 128)
    assert p.kernel.id == W.YUKAWA and p.b().shape == (4096, p.nrhs)
    assert np.array_equal(np.sort(p.perm()), np.arange(4096))
    d = W.yukawa_drift_cube(n=2048, beta=0.5)
    assert d.kernel.id == W.YUKAWA_DRIFT and d.kernel.beta == 0.5
    m = W.matern_cube(n=1024)
    assert m.kernel.id == W.MATERN32 and m.kernel.ell == 0.2 and m.kernel.nugget == 1e-4
    s = W.laplace_sphere(n=2048, leaf=128)
    assert s.nrhs == 16 and s.s_far == 256


def test_gaussian_batch_draws():
    ps = W.gaussian_batch(n_inst=16, n_min=100, n_max=300, seed=4)
    assert len(ps) == 16
    for p in ps:
        assert 100 <= p.n <= 300 and p.dim == 2
        assert 0.1 <= p.kernel.ell <= 0.5 and p.kernel.nugget == 1e-4
        assert p.kernel.id == W.GAUSSIAN
        assert (p.points >= 0).all() and (p.points < 1).all()
    again = W.gaussian_batch(n_inst=16, n_min=100, n_max=300, seed=4)
    assert all(np.array_equal(a.points, b.points) for a, b in zip(ps, again))
    assert len({p.n for p in ps}) > 1   # varying sizes
