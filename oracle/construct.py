"""H^2 construction with pre-factorization (Algorithm 1, Sections 3.4-3.5).

For each level l from the leaves up to 1 and each box i of that level:
  * S_F: sample of the far field, the active points of every box j at level l
    that is not near i (boxes whose ancestors were already far included);
  * S_C: sample of the near field, the active points of every near box j != i
    (box i itself excluded, otherwise A_Close would hold identity rows);
  * A_cc = G(S_C, S_C), A_Far = G(B_i, S_F), A_Close = G(B_i, S_C) A_cc^{-1}
    (the pre-factorization of Section 3.5: an exact Cholesky solve, or the
    paper's Gauss-Seidel approximation with a given number of sweeps);
  * (U_i, SK_i) = ID([A_Far, A_Close]) -- a row interpolative decomposition
    by column-pivoted QR of the transpose (rank k_i: the leading pivots with
    |R_jj| > eps |R_11|, optionally capped), U_i having identity rows at the
    skeleton.
Then the near blocks A_ij = G(B_i, B_j) at the leaves, the couplings
S_ij = G(SK_i, SK_j) for far pairs, and the parent's active points
B_I = (SK_2I, SK_2I+1).

Sampling reading: S_F (resp. S_C) holds the s_far (resp. s_near) candidates
that come first in the order of a given permutation pi of all points; a
negative sample size takes every candidate.  Candidates are ordered by their
position in pi.
"""
from __future__ import annotations

import dataclasses

import numpy as np
import scipy.linalg as sla

from . import kernels
from .tree import ClusterTree


@dataclasses.dataclass
class BoxBasis:
    B: np.ndarray          # active point ids (global, original numbering), length m
    SK: np.ndarray         # skeleton point ids, length k (pivot order)
    U: np.ndarray          # m x k interpolation basis, identity rows at the skeleton
    piv: np.ndarray        # CPQR pivot order (positions into B), length m
    R_diag: np.ndarray     # |R_jj| of the pivoted QR (diagnostics)
    sc: int = 0            # size of the near-field sample S_C (pre-factorization)

    @property
    def m(self) -> int:
        return len(self.B)

    @property
    def k(self) -> int:
        return len(self.SK)


@dataclasses.dataclass
class H2Matrix:
    tree: ClusterTree
    kernel: object
    X: np.ndarray
    basis: list            # basis[l][i]: BoxBasis, for l = 1..L (basis[0] unused)
    S: dict                # (l, i, j) -> k_i x k_j coupling, (i, j) in far[l]
    D: dict                # (i, j) -> leaf near block, (i, j) in near[L]
    root_B: np.ndarray     # active points of the root


def interpolative_decomposition(M: np.ndarray, eps: float, max_rank: int = 0):
    """Row ID of M (m x s) by column-pivoted QR of M^T (LAPACK dgeqp3).

    Returns (piv, k, T, rdiag): M[piv[k:]] ~= T^T M[piv[:k]] with
    T = R_11^{-1} R_12.  k counts the leading |R_jj| > eps |R_00|.
    """
    m, s = M.shape
    if m == 0:
        return np.zeros(0, dtype=np.int64), 0, np.zeros((0, 0)), np.zeros(0)
    if s == 0:
        return np.arange(m, dtype=np.int64), 0, np.zeros((0, m)), np.zeros(0)
    R, piv = sla.qr(M.T, mode="r", pivoting=True)
    rd = np.abs(np.diag(R))
    k = 0
    if rd.size and rd[0] > 0.0:
        thr = eps * rd[0]
        while k < rd.size and rd[k] > thr:
            k += 1
    if max_rank > 0:
        k = min(k, max_rank)
    T = sla.solve_triangular(R[:k, :k], R[:k, k:], lower=False) if k > 0 else np.zeros((0, m))
    return piv.astype(np.int64), k, T, rd


def build_basis(piv: np.ndarray, k: int, T: np.ndarray, m: int) -> np.ndarray:
    """U (m x k) with U[piv[t], t] = 1 and U[piv[k+q], :] = T[:, q]."""
    U = np.zeros((m, k))
    if k:
        U[piv[:k], np.arange(k)] = 1.0
        U[piv[k:], :] = T.T
    return U


def gauss_seidel(A: np.ndarray, B: np.ndarray, sweeps: int) -> np.ndarray:
    """Approximate A^{-1} B by forward Gauss-Seidel sweeps from X = 0 (the
    Section 3.5 replacement of the factorization of A_cc): in each sweep the
    rows i = 0, 1, ... of X become (B_i - sum_{j != i} A_ij X_j) / A_ii,
    using the rows already replaced in the same sweep."""
    X = np.zeros_like(B, dtype=np.float64)
    for _ in range(sweeps):
        for i in range(A.shape[0]):
            s = B[i] - A[i] @ X + A[i, i] * X[i]
            X[i] = s / A[i, i]
    return X


def _sample(cands: np.ndarray, pirank: np.ndarray, count: int) -> np.ndarray:
    o = np.argsort(pirank[cands], kind="stable")
    c = cands[o]
    return c if count < 0 else c[:count]


def construct(X: np.ndarray, kernel, leaf: int, eta: float, eps: float,
              pi: np.ndarray, s_far: int = -1, s_near: int = -1,
              max_rank: int = 0, skeletons: dict | None = None,
              gs_sweeps: int = 0) -> H2Matrix:
    """Algorithm 1.  ``skeletons`` optionally fixes, per (l, i), the skeleton
    (positions into B_i, in pivot order; its length is the rank) instead of
    running the pivoted QR; the remaining rows follow in increasing position.
    Used to build an H^2 matrix with a prescribed skeleton selection.
    ``gs_sweeps`` > 0 replaces the exact solve with A_cc by that many
    Gauss-Seidel sweeps (Section 3.5).

    Non-symmetric kernels (the LU variant; the paper treats symmetric
    matrices only): box i keeps one basis for its rows and its columns, so the
    interpolative decomposition runs on [G(B_i,S_F), G(S_F,B_i)^T,
    G(B_i,S_C) A_cc^{-1}, (A_cc^{-1} G(S_C,B_i))^T], the far field and the
    fill-in seen from both sides (A_cc by an LU factorization, or Gauss-Seidel
    sweeps on A_cc^T and A_cc); couplings and near blocks are evaluated for
    every ordered pair, as for symmetric kernels."""
    tree = ClusterTree(X, leaf, eta)
    L = tree.L
    sym = kernels.symmetric(kernel)
    n = X.shape[0]
    pirank = np.empty(n, dtype=np.int64)
    pirank[pi] = np.arange(n)
    basis: list = [None] * (L + 1)
    S: dict = {}
    D: dict = {}

    # Active points per box at the current level; leaves: tree-order points.
    B = [tree.perm[s:e].copy() for (s, e) in tree.ranges[L]]
    for l in range(L, 0, -1):
        nb = 1 << l
        near = tree.near_of(l)
        lvl = []
        for i in range(nb):
            nset = set(near[i])
            far_c = [B[j] for j in range(nb) if j not in nset]
            near_c = [B[j] for j in near[i] if j != i]
            F = np.concatenate(far_c) if far_c else np.zeros(0, dtype=np.int64)
            C = np.concatenate(near_c) if near_c else np.zeros(0, dtype=np.int64)
            SF = _sample(F, pirank, s_far)
            SC = _sample(C, pirank, s_near)
            Bi = B[i]
            A_far = kernels.evaluate(kernel, X[Bi], X[SF], Bi, SF)
            if SC.size:
                A_cc = kernels.evaluate(kernel, X[SC], X[SC], SC, SC)
                G_bc = kernels.evaluate(kernel, X[Bi], X[SC], Bi, SC)
                if not sym:
                    # the column side of the fill-in, A_cc^{-1} G(S_C, B_i)
                    G_cb = kernels.evaluate(kernel, X[SC], X[Bi], SC, Bi)
                    if gs_sweeps > 0:
                        A_close = gauss_seidel(A_cc.T, G_bc.T, gs_sweeps).T
                        A_close_c = gauss_seidel(A_cc, G_cb, gs_sweeps).T
                    else:
                        lf = sla.lu_factor(A_cc)
                        A_close = sla.lu_solve(lf, G_bc.T, trans=1).T   # G(B_i,S_C) A_cc^{-1}
                        A_close_c = sla.lu_solve(lf, G_cb).T            # (A_cc^{-1} G(S_C,B_i))^T
                elif gs_sweeps > 0:
                    A_close = gauss_seidel(A_cc, G_bc.T, gs_sweeps).T
                else:
                    cf = sla.cho_factor(A_cc, lower=True)
                    A_close = sla.cho_solve(cf, G_bc.T).T   # G(B_i,S_C) A_cc^{-1}
            else:
                A_close = np.zeros((Bi.size, 0))
                A_close_c = np.zeros((Bi.size, 0))
            if sym:
                M = np.hstack([A_far, A_close])
            else:
                # one shared basis for the rows and the columns of box i: the
                # far field seen from both sides and both sides of the fill-in
                A_far_c = kernels.evaluate(kernel, X[SF], X[Bi], SF, Bi).T
                M = np.hstack([A_far, A_far_c, A_close, A_close_c])
            if skeletons is not None:
                sk = np.asarray(skeletons[(l, i)], dtype=np.int64)
                k = sk.size
                rest = np.setdiff1d(np.arange(Bi.size), sk)
                piv = np.concatenate([sk, rest]).astype(np.int64)
                T, rd = _forced_id(M, piv, k)
            else:
                piv, k, T, rd = interpolative_decomposition(M, eps, max_rank)
            U = build_basis(piv, k, T, Bi.size)
            lvl.append(BoxBasis(Bi, Bi[piv[:k]], U, piv, rd, sc=int(SC.size)))
        basis[l] = lvl
        for (i, j) in tree.far[l]:
            S[(l, i, j)] = kernels.evaluate(kernel, X[lvl[i].SK], X[lvl[j].SK],
                                            lvl[i].SK, lvl[j].SK)
        if l == L:
            for (i, j) in tree.near[L]:
                D[(i, j)] = kernels.evaluate(kernel, X[B[i]], X[B[j]], B[i], B[j])
        B = [np.concatenate([lvl[2 * I].SK, lvl[2 * I + 1].SK]) for I in range(nb // 2)]
    if L == 0:
        D[(0, 0)] = kernels.evaluate(kernel, X[B[0]], X[B[0]], B[0], B[0])
    return H2Matrix(tree, kernel, X, basis, S, D, B[0])


def _forced_id(M: np.ndarray, piv: np.ndarray, k: int):
    """ID coefficients for a prescribed pivot order: Householder QR of the
    column-permuted M^T, then T = R_11^{-1} R_12 (same algebra as the pivoted
    QR with the pivot choices given)."""
    m = M.shape[0]
    if k == 0:
        return np.zeros((0, m)), np.zeros(0)
    R = sla.qr(M.T[:, piv], mode="r")[0]
    T = sla.solve_triangular(R[:k, :k], R[:k, k:], lower=False)
    return T, np.abs(np.diag(R))
