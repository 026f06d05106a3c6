"""Pins of the oracle's Gauss-Seidel approximation of A_cc^{-1} (Section
3.5) against independent formulas: one forward sweep from zero is the solve
with the lower triangle (D + L)^{-1} B, two sweeps are
(D + L)^{-1} (B - U (D + L)^{-1} B), and many sweeps on an SPD matrix converge
to the Cholesky solve; a diagonal matrix is solved exactly in one sweep."""
import numpy as np
import scipy.linalg as sla

from oracle import kernels
from oracle.construct import gauss_seidel
import workloads as W


def _spd(n, seed):
    rng = np.random.default_rng(seed)
    M = rng.standard_normal((n, n))
    return M @ M.T + n * np.eye(n), rng.standard_normal((n, 5))


def test_one_sweep_is_lower_triangular_solve():
    A, B = _spd(40, 1)
    X = gauss_seidel(A, B, 1)
    ref = sla.solve_triangular(np.tril(A), B, lower=True)
    assert np.max(np.abs(X - ref)) <= 1e-13 * np.max(np.abs(ref))


def test_two_sweeps_closed_form():
    A, B = _spd(33, 2)
    X = gauss_seidel(A, B, 2)
    DL, U = np.tril(A), np.triu(A, 1)
    X1 = sla.solve_triangular(DL, B, lower=True)
    ref = sla.solve_triangular(DL, B - U @ X1, lower=True)
    assert np.max(np.abs(X - ref)) <= 1e-13 * np.max(np.abs(ref))


def test_converges_to_cholesky_solve_on_spd():
    A, B = _spd(25, 3)
    X = gauss_seidel(A, B, 200)
    ref = sla.cho_solve(sla.cho_factor(A, lower=True), B)
    assert np.max(np.abs(X - ref)) <= 1e-12 * np.max(np.abs(ref))


def test_diagonal_exact_in_one_sweep():
    rng = np.random.default_rng(4)
    d = rng.uniform(1, 3, 17)
    B = rng.standard_normal((17, 3))
    assert np.allclose(gauss_seidel(np.diag(d), B, 1), B / d[:, None], rtol=0, atol=1e-15)


def test_error_decreases_on_a_kernel_block():
    # a near-sample block of the Yukawa kernel (SPD): the error against the
    # exact solve falls with every sweep
    p = W.yukawa_cube(n=512, leaf=64, eps=1e-6, s=64)
    idx = np.arange(64)
    A = kernels.evaluate(p.kernel, p.points[idx], p.points[idx], idx, idx)
    B = kernels.evaluate(p.kernel, p.points[idx], p.points[100:130], idx, np.arange(100, 130))
    ref = sla.cho_solve(sla.cho_factor(A, lower=True), B)
    errs = [np.linalg.norm(gauss_seidel(A, B, s) - ref) for s in (1, 2, 4, 8)]
    assert all(e2 < e1 for e1, e2 in zip(errs, errs[1:]))
