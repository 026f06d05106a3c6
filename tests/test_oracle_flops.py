"""Pins of the canonical flop count (oracle/flops.py) to operation counts
taken from running implementations, not from the formulas themselves.

Each step of the per-box count is carried out here by a plain loop that adds
up the multiplications and additions it really performs (vector operations
counted by their length), on a random matrix, and its result is checked
against LAPACK's so the loop is the real algorithm:
  * unblocked Householder QR of an m x k matrix      vs GEQRF(m, k)
  * accumulation of the full m x m Q from k reflectors vs ORGQR_full(m, k)
  * Cholesky of an r x r SPD matrix                  vs r^3 / 3
  * B L^{-T} for B k x r, L r x r lower triangular   vs k r^2
The loop counts must agree with the formulas in their leading terms: the
difference is a lower-order term, at most a small multiple of m k (QR) or
of r^2 (Cholesky, triangular solve).  Finally the whole count of one
structure is compared with a sum of those loop counts.
"""
import numpy as np
import pytest
import scipy.linalg as sla

from oracle import flops


def _householder_qr(A):
    """Householder QR (LAPACK's reflector convention); returns (V, tau, R, flops)."""
    A = A.copy()
    m, k = A.shape
    V = np.zeros((m, k))
    tau = np.zeros(k)
    f = 0
    for j in range(k):
        x = A[j:, j]
        n = m - j
        nrm = np.sqrt(x @ x); f += 2 * n
        alpha = x[0]
        beta = -np.copysign(nrm, alpha)
        v = x.copy()
        v[0] = 1.0
        v[1:] = x[1:] / (alpha - beta); f += n - 1
        tau[j] = (beta - alpha) / beta
        A[j, j] = beta
        A[j + 1:, j] = 0.0
        if j + 1 < k:
            w = v @ A[j:, j + 1:]; f += 2 * n * (k - j - 1)
            A[j:, j + 1:] -= np.outer(tau[j] * v, w); f += 2 * n * (k - j - 1)
        V[j:, j] = v
    return V, tau, np.triu(A[:k]), f


def _orgqr_full(V, tau, m):
    """Q = H_0 H_1 ... H_{k-1} (m x m), accumulated from the last reflector."""
    k = V.shape[1]
    Q = np.eye(m)
    f = 0
    for j in range(k - 1, -1, -1):
        v = V[j:, j]
        n = m - j
        w = v @ Q[j:, j:]; f += 2 * n * n
        Q[j:, j:] -= np.outer(tau[j] * v, w); f += 2 * n * n
    return Q, f


def _cholesky(A):
    A = A.copy()
    r = A.shape[0]
    f = 0
    for j in range(r):
        A[j, j] = np.sqrt(A[j, j] - A[j, :j] @ A[j, :j]); f += 2 * j
        if j + 1 < r:
            A[j + 1:, j] = (A[j + 1:, j] - A[j + 1:, :j] @ A[j, :j]) / A[j, j]
            f += (r - j - 1) * (2 * j + 1)
    return np.tril(A), f


def _right_trsm_lt(B, L):
    """X = B L^{-T}: column j of X from the columns before it."""
    k, r = B.shape
    X = np.zeros_like(B)
    f = 0
    for j in range(r):
        X[:, j] = (B[:, j] - X[:, :j] @ L[j, :j]) / L[j, j]
        f += k * (2 * j + 1)
    return X, f


@pytest.mark.parametrize("m,k", [(40, 10), (64, 32), (96, 80), (50, 50)])
def test_geqrf_and_orgqr_counts(m, k):
    rng = np.random.default_rng(m * 1000 + k)
    W = rng.standard_normal((m, k))
    V, tau, R, fq = _householder_qr(W)
    Q, fo = _orgqr_full(V, tau, m)
    # the loops are a real QR: W = Q [R; 0] with Q orthogonal
    assert np.allclose(Q[:, :k] @ R, W, atol=1e-12 * np.abs(W).max() * m)
    assert np.allclose(Q.T @ Q, np.eye(m), atol=1e-13 * m)
    Rl = sla.qr(W, mode="r")[0][:k]
    assert np.allclose(np.abs(np.diag(R)), np.abs(np.diag(Rl)), rtol=1e-12)
    assert abs(fq - flops.geqrf(m, k)) <= 4 * m * k
    assert abs(fo - flops.orgqr_full(m, k)) <= 8 * m * m
    assert abs(fq - flops.geqrf(m, k)) / flops.geqrf(m, k) < 0.25


@pytest.mark.parametrize("k,r", [(10, 40), (32, 64), (80, 30)])
def test_cholesky_and_trsm_counts(k, r):
    rng = np.random.default_rng(k * 100 + r)
    G = rng.standard_normal((r, r))
    A = G @ G.T + r * np.eye(r)
    L, fc = _cholesky(A)
    assert np.allclose(L, sla.cholesky(A, lower=True), rtol=1e-12, atol=1e-12)
    B = rng.standard_normal((k, r))
    X, ft = _right_trsm_lt(B, L)
    assert np.allclose(X @ L.T, B, atol=1e-11)
    assert abs(fc - r ** 3 / 3.0) <= 2 * r * r
    assert abs(ft - k * r * r) <= k * r


def test_count_composes_the_step_counts():
    """One level with two boxes (m, k) = (60, 20), (50, 30), one near pair and
    one far pair, root n0 = 25: count() equals the per-step counts summed by
    hand from the loops above (leading terms; the loops carry lower-order
    terms that the canonical count leaves out)."""
    ms, ks = [None, [60, 50]], [None, [20, 30]]
    near = [None, [(0, 0), (0, 1), (1, 0), (1, 1)]]
    far = [None, []]
    ff, fs = flops.count(ms, ks, near, far, n0=25)
    exp = 0.0
    for m, k in zip(ms[1], ks[1]):
        r = m - k
        exp += flops.geqrf(m, k) + flops.orgqr_full(m, k)
        exp += 2 * (2.0 * m ** 3)                     # Q^T A Q: two m x m x m products
        exp += r ** 3 / 3 + k * r * r + k * k * r + m * r * r
    (m0, k0), (m1, k1) = (60, 20), (50, 30)
    r0, r1 = m0 - k0, m1 - k1
    exp += 2.0 * m1 * m0 * (m1 + m0)                  # Q_1^T A_10 Q_0, one unordered pair
    exp += k0 * r1 * r1 + k1 * r0 * r0                # L(s) of both orders
    exp += r1 * r0 * r0                               # L(r)_10
    exp += 25 ** 3 / 3.0
    assert abs(ff - exp) <= 1e-9 * exp
    # solve: 4 m^2 + 4 r^2 per box, 4 k_i r_j per ordered pair (diagonal
    # included), 4 r_1 r_0 for the pair below the diagonal, 2 n0^2
    es = sum(4.0 * m * m + 4.0 * (m - k) ** 2 for m, k in zip(ms[1], ks[1]))
    es += 4.0 * (k0 * r0 + k0 * r1 + k1 * r0 + k1 * r1) + 4.0 * r1 * r0 + 2.0 * 25 ** 2
    assert abs(fs - es) <= 1e-9 * es
