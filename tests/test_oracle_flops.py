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


def _lower_solve(L, B):
    """Y = L^{-1} B by forward substitution, column by column."""
    c, m = B.shape
    Y = np.zeros_like(B)
    f = 0
    for q in range(m):
        for i in range(c):
            Y[i, q] = (B[i, q] - L[i, :i] @ Y[:i, q]) / L[i, i]
            f += 2 * i + 1
    return Y, f


@pytest.mark.parametrize("c,m", [(30, 40), (64, 16), (17, 50)])
def test_prefactor_counts(c, m):
    """Section 3.5's pre-factorization of one box: Cholesky of A_cc and two
    triangular solves with the m columns of G(S_C, B_i), counted by loops
    that really solve A_cc X = G (checked against scipy), or Gauss-Seidel
    sweeps counted by a loop that reproduces oracle.construct.gauss_seidel."""
    from oracle import construct
    rng = np.random.default_rng(c * 100 + m)
    G = rng.standard_normal((c, c))
    A = G @ G.T + c * np.eye(c)
    B = rng.standard_normal((c, m))
    L, fc = _cholesky(A)
    Y, f1 = _lower_solve(L, B)
    Xr, f2 = _lower_solve(L[::-1, ::-1].T.copy(), Y[::-1].copy())   # L^T X = Y, reversed
    X = Xr[::-1]
    assert np.allclose(X, sla.cho_solve((sla.cholesky(A, lower=True), True), B), atol=1e-12)
    f = fc + f1 + f2
    assert abs(f - flops.prefactor_box(c, m)) <= 2 * c * c + 2 * c * m
    for sweeps in (1, 2, 3):
        Xg = np.zeros_like(B)
        fg = 0
        for _ in range(sweeps):
            for i in range(c):
                Xg[i] = (B[i] - A[i, :i] @ Xg[:i] - A[i, i + 1:] @ Xg[i + 1:]) / A[i, i]
                fg += (2 * (c - 1) + 1) * m
        assert np.allclose(Xg, construct.gauss_seidel(A, B, sweeps), rtol=1e-12, atol=1e-12)
        assert abs(fg - flops.prefactor_box(c, m, sweeps)) <= sweeps * c * m


def test_count_prefactor_follows_the_near_samples():
    """The per-box sample sizes the count uses are those the sampling rule
    gives (the first s_near candidates of the near boxes' active points, or
    all of them), and the total is the per-box formula summed over levels."""
    import workloads as W
    from oracle import construct
    p = W.laplace_cube(n=1024, leaf=64, eps=1e-6, s=96)
    h = construct.construct(p.points, p.kernel, p.leaf, p.eta, p.eps, p.perm(), p.s_far,
                            p.s_near)
    t = h.tree
    tot = 0.0
    for l in range(1, t.L + 1):
        near = t.near_of(l)
        for i, bb in enumerate(h.basis[l]):
            cands = sum(h.basis[l][j].m for j in near[i] if j != i)
            assert bb.sc == min(cands, p.s_near)
            tot += bb.sc ** 3 / 3.0 + 2.0 * bb.sc ** 2 * bb.m
    assert any(bb.sc == p.s_near for bb in h.basis[t.L])      # the sample bounds some boxes
    assert abs(flops.count_prefactor(h) - tot) <= 1e-9 * tot
    assert flops.count_prefactor(h, 2) > 0


def _lu_nopivot(A):
    """Doolittle elimination without row exchanges; returns (L, U, flops)."""
    U = A.copy()
    r = U.shape[0]
    L = np.eye(r)
    f = 0
    for j in range(r):
        if j + 1 < r:
            L[j + 1:, j] = U[j + 1:, j] / U[j, j]; f += r - j - 1
            U[j + 1:, j:] -= np.outer(L[j + 1:, j], U[j, j:]); f += 2 * (r - j - 1) * (r - j)
            U[j + 1:, j] = 0.0
    return L, np.triu(U), f


def _left_unit_lower_solve(L, B):
    """Y = L^{-1} B for unit lower L, by forward substitution."""
    r, k = B.shape
    Y = np.zeros_like(B)
    f = 0
    for i in range(r):
        Y[i] = B[i] - L[i, :i] @ Y[:i]
        f += 2 * i * k
    return Y, f


def _right_upper_solve(B, U):
    """X = B U^{-1}: column j of X from the columns before it."""
    k, r = B.shape
    X = np.zeros_like(B)
    f = 0
    for j in range(r):
        X[:, j] = (B[:, j] - X[:, :j] @ U[:j, j]) / U[j, j]
        f += k * (2 * j + 1)
    return X, f


@pytest.mark.parametrize("k,r", [(10, 40), (32, 64), (80, 30)])
def test_lu_and_its_triangular_solve_counts(k, r):
    """The LU variant's per-box steps: a pivot-free LU of the redundant block
    (checked against the oracle's and against L U = A), U(s) = L^{-1} RS and
    L(s) = SR U^{-1}, counted by the loops that perform them."""
    from oracle import ulv_lu
    rng = np.random.default_rng(k * 100 + r + 7)
    A = rng.standard_normal((r, r)) + r * np.eye(r)
    L, U, fl = _lu_nopivot(A)
    Lo, Uo = ulv_lu.lu_nopivot(A)
    assert np.allclose(L, Lo, atol=1e-13) and np.allclose(U, Uo, atol=1e-12)
    assert np.allclose(L @ U, A, atol=1e-12 * r)
    RS = rng.standard_normal((r, k))
    SR = rng.standard_normal((k, r))
    Y, f1 = _left_unit_lower_solve(L, RS)
    X, f2 = _right_upper_solve(SR, U)
    assert np.allclose(L @ Y, RS, atol=1e-11) and np.allclose(X @ U, SR, atol=1e-11)
    assert abs(fl - 2.0 * r ** 3 / 3.0) <= 2 * r * r
    assert abs(f1 - k * r * r) <= k * r and abs(f2 - k * r * r) <= k * r


def test_count_lu_composes_the_step_counts():
    """count_lu on one level with two boxes (m, k) = (60, 20), (50, 30), both
    orders of their near pair and root n0 = 25, against the per-step counts
    summed by hand (each ordered pair transformed on its own; L(s), U(s)
    and one of L(r) / U(r) per ordered pair; LU and both bases per box)."""
    ms, ks = [None, [60, 50]], [None, [20, 30]]
    near = [None, [(0, 0), (0, 1), (1, 0), (1, 1)]]
    far = [None, []]
    ff, fs = flops.count_lu(ms, ks, near, far, n0=25)
    exp = 0.0
    for m, k in zip(ms[1], ks[1]):
        r = m - k
        exp += flops.geqrf(m, k) + flops.orgqr_full(m, k) + 4.0 * m ** 3
        exp += 2 * r ** 3 / 3 + 2 * k * r * r + 2 * k * k * r + 2 * m * r * r
    (m0, k0), (m1, k1) = (60, 20), (50, 30)
    r0, r1 = m0 - k0, m1 - k1
    exp += 2 * (2.0 * m1 * m0 * (m1 + m0))            # P_1^T A_10 P'_0 and P_0^T A_01 P'_1
    exp += k1 * r0 * r0 + r1 * r1 * k0 + r1 * r0 * r0  # (1, 0): L(s), U(s), L(r)
    exp += k0 * r1 * r1 + r0 * r0 * k1 + r0 * r0 * r1  # (0, 1): L(s), U(s), U(r)
    exp += 2 * 25 ** 3 / 3.0
    assert abs(ff - exp) <= 1e-9 * exp
    es = sum(4.0 * m * m + 4.0 * (m - k) ** 2 + 4.0 * k * (m - k) for m, k in zip(ms[1], ks[1]))
    es += 2 * (2.0 * k1 * r0 + 2.0 * r1 * k0 + 2.0 * r1 * r0) + 2.0 * 25 ** 2
    assert abs(fs - es) <= 1e-9 * es
    # on a symmetric structure the LU count exceeds the Cholesky count by the
    # extra triangular work and the second transform of every pair
    fc, _ = flops.count(ms, ks, near, far, n0=25)
    assert ff > fc
