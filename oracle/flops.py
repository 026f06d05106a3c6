"""Canonical algorithmic flop counts of the factorization and the solve.

Counted on the actual (unpadded) sizes of an H^2 structure.  Per level, with
m, k, r = m - k per box:
  boxes:      GEQRF(m,k) + ORGQR_full(m,k)       basis completion (step 1)
              + 4 m^3                            Q^T A_ii Q (step 2)
              + r^3/3 + k r^2 + k^2 r + m r^2    Cholesky, TRSM for L(s)_ii,
                                                 Schur update, V_i (steps 3-6)
  near pairs: 2 m_i m_j (m_i + m_j) per unordered pair (the two-sided basis
              transform, Algorithm 4 line 10); k_i r_j^2 per ordered pair
              (L(s)_ij); r_i r_j^2 for i > j (L(r)_ij)
  far pairs:  k_i k_j (k_i + k_j) per unordered pair (R_i S_ij R_j^T)
  root:       n_0^3 / 3
with GEQRF(m,k) = 2 m k^2 - 2/3 k^3 and ORGQR_full(m,k) = 4 m^2 k - 4 m k^2
+ 4/3 k^3, the leading terms of the operation counts LAPACK Working Note 41
tabulates for xGEQRF (m x k, m >= k) and xORGQR (an m x n Q from k
reflectors: 4 m n k - 2 (m + n) k^2 + 4/3 k^3, here with n = m).  The solve,
per right-hand side: 4 m^2 + 4 r^2 per box, 4 r_i r_j per near pair i > j,
4 k_i r_j per ordered near pair (i == j included), 2 n_0^2 at the root.

The pre-factorization of the construction (Section 3.5, Algorithm 1), per
box with a near-field sample S_C of size c and m active points: the
Cholesky factorization of A_cc (c^3 / 3) and two triangular solves with the
m columns of G(S_C, B_i) (2 c^2 m), or, with Gauss-Seidel sweeps in place of
the factorization, 2 c^2 m per sweep (every off-diagonal entry of A_cc once
per column; Section 3.5's iterative variant).

The LU variant (oracle/ulv_lu.py; count_lu): per box the same QR and
diagonal transform, 2 r^3/3 for the pivot-free LU of the redundant block,
2 k r^2 for L(s)_ii = SR U^{-1} and U(s)_ii = L^{-1} RS, 2 k^2 r for
SS -= L(s)_ii U(s)_ii and 2 m r^2 for the two bases; per ordered near pair
i != j the transform 2 m_i m_j (m_i + m_j), k_i r_j^2 (L(s)_ij), r_i^2 k_j
(U(s)_ij) and r_i r_j^2 (i > j, L(r)_ij) or r_i^2 r_j (i < j, U(r)_ij); per
ordered far pair k_i k_j (k_i + k_j); the root 2 n_0^3 / 3.  Its solve, per
right-hand side: 4 m^2 + 4 r^2 per box, 4 k_i r_i per diagonal block, and
2 k_i r_j + 2 r_i k_j + 2 r_i r_j per ordered near pair i != j.

Pinned by tests/test_oracle_flops.py against the operations that running
Householder QR, Q accumulation, Cholesky, pivot-free LU and triangular-solve
loops perform.
"""
from __future__ import annotations


def geqrf(m: int, k: int) -> float:
    return 2.0 * m * k * k - 2.0 / 3.0 * k ** 3


def orgqr_full(m: int, k: int) -> float:
    return 4.0 * m * m * k - 4.0 * m * k * k + 4.0 / 3.0 * k ** 3


def count(ms: list, ks: list, near: list, far: list, n0: int, nrhs: int = 1):
    """ms[l][i], ks[l][i] for l = 1..L (index 0 unused); near[l], far[l] the
    ordered pair lists.  Returns (factor_flops, solve_flops)."""
    ff = 0.0
    fs = 0.0
    for l in range(1, len(ms)):
        m, k = ms[l], ks[l]
        for i in range(len(m)):
            r = m[i] - k[i]
            ff += geqrf(m[i], k[i]) + orgqr_full(m[i], k[i]) + 4.0 * m[i] ** 3
            ff += r ** 3 / 3.0 + k[i] * r * r + k[i] * k[i] * r + m[i] * r * r
            fs += 4.0 * m[i] ** 2 + 4.0 * r * r
        for (i, j) in near[l]:
            ri, rj = m[i] - k[i], m[j] - k[j]
            fs += 4.0 * k[i] * rj
            if i == j:
                continue
            ff += k[i] * rj * rj
            if i > j:
                ff += 2.0 * m[i] * m[j] * (m[i] + m[j])
                ff += ri * rj * rj
                fs += 4.0 * ri * rj
        for (i, j) in far[l]:
            if i > j:
                ff += k[i] * k[j] * (k[i] + k[j])
    ff += n0 ** 3 / 3.0
    fs += 2.0 * n0 * n0
    return ff, fs * nrhs


def count_lu(ms: list, ks: list, near: list, far: list, n0: int, nrhs: int = 1):
    """The LU variant's counts on the same inputs as count()."""
    ff = 0.0
    fs = 0.0
    for l in range(1, len(ms)):
        m, k = ms[l], ks[l]
        for i in range(len(m)):
            r = m[i] - k[i]
            ff += geqrf(m[i], k[i]) + orgqr_full(m[i], k[i]) + 4.0 * m[i] ** 3
            ff += 2.0 * r ** 3 / 3.0 + 2.0 * k[i] * r * r + 2.0 * k[i] * k[i] * r + 2.0 * m[i] * r * r
            fs += 4.0 * m[i] ** 2 + 4.0 * r * r
        for (i, j) in near[l]:
            ri, rj = m[i] - k[i], m[j] - k[j]
            if i == j:
                fs += 4.0 * k[i] * ri
                continue
            ff += 2.0 * m[i] * m[j] * (m[i] + m[j]) + k[i] * rj * rj + ri * ri * k[j]
            ff += ri * rj * rj if i > j else ri * ri * rj
            fs += 2.0 * k[i] * rj + 2.0 * ri * k[j] + 2.0 * ri * rj
        for (i, j) in far[l]:
            ff += k[i] * k[j] * (k[i] + k[j])
    ff += 2.0 * n0 ** 3 / 3.0
    fs += 2.0 * n0 * n0
    return ff, fs * nrhs


def count_h2_lu(h2, nrhs: int = 1):
    t = h2.tree
    ms = [None] + [[bb.m for bb in h2.basis[l]] for l in range(1, t.L + 1)]
    ks = [None] + [[bb.k for bb in h2.basis[l]] for l in range(1, t.L + 1)]
    return count_lu(ms, ks, t.near, t.far, len(h2.root_B), nrhs)


def count_h2(h2, nrhs: int = 1):
    t = h2.tree
    ms = [None] + [[bb.m for bb in h2.basis[l]] for l in range(1, t.L + 1)]
    ks = [None] + [[bb.k for bb in h2.basis[l]] for l in range(1, t.L + 1)]
    n0 = len(h2.root_B)
    return count(ms, ks, t.near, t.far, n0, nrhs)


def prefactor_box(c: int, m: int, gs_sweeps: int = 0) -> float:
    """Pre-factorization flops of one box (see the module docstring)."""
    if c == 0:
        return 0.0
    if gs_sweeps > 0:
        return gs_sweeps * 2.0 * c * c * m
    return c ** 3 / 3.0 + 2.0 * c * c * m


def count_prefactor(h2, gs_sweeps: int = 0) -> float:
    """Pre-factorization flops of a whole construction (every level)."""
    t = h2.tree
    return sum(prefactor_box(bb.sc, bb.m, gs_sweeps)
               for l in range(1, t.L + 1) for bb in h2.basis[l])
