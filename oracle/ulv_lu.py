"""LU variant of the H^2-ULV factorization and substitution, for non-symmetric
kernel matrices.

The paper states the method for symmetric positive definite matrices
(Section 3.6, Algorithms 2 and 4: Cholesky of the redundant blocks, Eq. 21
the only trailing update; Section 3.7, Eq. 31 and its transpose for the
substitution).  This variant keeps every structural step and replaces the
Cholesky factorization of each redundant block by an LU factorization
without pivoting, so that the symmetric case reduces to the Cholesky variant
(up to how the diagonal is split between the two triangles, which the solve
does not see).  Readings taken here (the paper is silent on the LU form):

* one basis Q_i per box for its rows and its columns (the construction
  spans the far field and the fill-in seen from both sides);
* per level and box, with A^_ij = Q_i^T A_ij Q_j split into SS, SR, RS, RR:
      L(r)_ii U(r)_ii = RR_ii                         (pivot-free LU, unit L)
      L(s)_ii = SR_ii U(r)_ii^{-1},  U(s)_ii = L(r)_ii^{-1} RS_ii
      SS_ii   = SS_ii - L(s)_ii U(s)_ii                (the Eq. 21 update)
  and for near i != j
      L(s)_ij = SR_ij U(r)_jj^{-1},  U(s)_ij = L(r)_ii^{-1} RS_ij
      L(r)_ij = RR_ij U(r)_jj^{-1}   (i > j, the lower factor's block)
      U(r)_ij = L(r)_ii^{-1} RR_ij   (i < j, the upper factor's block)
      SS_ij   = SS_ij;
  far couplings and the merge as in the Cholesky variant;
* the forward sweep is Eq. 31 with these L blocks, the backward sweep the
  same form with the U blocks in place of the transposed L blocks:
      u_i = U(r)_ii^{-1} t_i,  v_j = t_j - sum_{i>j} U(r)_ji u_i,
      x_j^R = U(r)_jj^{-1} v_j,  with t_j = y_j^R - sum_i U(s)_ji x_i^S.
Refinement is stationary (PCG needs a symmetric operator).
"""
from __future__ import annotations

import dataclasses

import numpy as np
import scipy.linalg as sla

from .construct import H2Matrix
from .h2matrix import matvec
from .ulv import _complete


class LUBreakdown(Exception):
    def __init__(self, level: int, box: int):
        super().__init__(f"zero pivot in the LU of level {level}, box {box}")
        self.level, self.box = level, box


def lu_nopivot(A: np.ndarray, level: int = -1, box: int = -1):
    """A = L U with L unit lower and U upper triangular, no row exchanges
    (Doolittle's elimination, one column at a time)."""
    n = A.shape[0]
    U = A.astype(np.float64).copy()
    Lm = np.eye(n)
    for j in range(n):
        p = U[j, j]
        if not np.isfinite(p) or p == 0.0:
            raise LUBreakdown(level, box)
        if j + 1 < n:
            f = U[j + 1:, j] / p
            Lm[j + 1:, j] = f
            U[j + 1:, j:] -= np.outer(f, U[j, j:])
            U[j + 1:, j] = 0.0
    return Lm, np.triu(U)


def _right_solve_upper(B: np.ndarray, U: np.ndarray) -> np.ndarray:
    """B U^{-1}."""
    if U.shape[0] == 0 or B.shape[0] == 0:
        return np.zeros((B.shape[0], U.shape[0]))
    return sla.solve_triangular(U, B.T, trans="T", lower=False).T


def _left_solve_lower(Lm: np.ndarray, B: np.ndarray) -> np.ndarray:
    """L^{-1} B."""
    if Lm.shape[0] == 0 or B.shape[1] == 0:
        return np.zeros((Lm.shape[0], B.shape[1]))
    return sla.solve_triangular(Lm, B, lower=True, unit_diagonal=True)


@dataclasses.dataclass
class LULevel:
    k: list
    m: list
    Q: list          # m x m orthogonal completions
    R: list          # k x k triangular factors of D_i U_i
    Lr: list         # r x r unit lower factors of RR_ii
    Ur: list         # r x r upper factors of RR_ii
    Ls: dict         # (i, j) near, i == j included -> k_i x r_j
    Us: dict         # (i, j) near, i == j included -> r_i x k_j
    Lro: dict        # (i, j) near with i > j -> r_i x r_j
    Uro: dict        # (i, j) near with i < j -> r_i x r_j
    SS: dict         # (i, j) near or far -> k_i x k_j
    near: list


@dataclasses.dataclass
class LUFactor:
    h2: H2Matrix
    levels: list
    A_root: np.ndarray
    L00: np.ndarray
    U00: np.ndarray


def factor(h2: H2Matrix) -> LUFactor:
    t = h2.tree
    L = t.L
    A = {key: blk.copy() for key, blk in h2.D.items()}
    levels: list = [None] * (L + 1)
    Rchild = None
    for l in range(L, 0, -1):
        nb = 1 << l
        bas = h2.basis[l]
        ks = [bb.k for bb in bas]
        ms = [bb.m for bb in bas]
        Q, R = [], []
        for i in range(nb):
            W = bas[i].U if l == L else sla.block_diag(Rchild[2 * i], Rchild[2 * i + 1]) @ bas[i].U
            Qi, Ri = _complete(W, ks[i])
            Q.append(Qi)
            R.append(Ri)
        Lr, Ur = [], []
        Ls, Us, Lro, Uro, SS = {}, {}, {}, {}, {}
        for i in range(nb):
            k = ks[i]
            Ah = Q[i].T @ A[(i, i)] @ Q[i]
            Li, Ui = lu_nopivot(Ah[k:, k:], l, i)
            Lr.append(Li)
            Ur.append(Ui)
            Ls[(i, i)] = _right_solve_upper(Ah[:k, k:], Ui)
            Us[(i, i)] = _left_solve_lower(Li, Ah[k:, :k])
            SS[(i, i)] = Ah[:k, :k] - Ls[(i, i)] @ Us[(i, i)]
        for (i, j) in t.near[l]:
            if i == j:
                continue
            ki, kj = ks[i], ks[j]
            Ah = Q[i].T @ A[(i, j)] @ Q[j]
            SS[(i, j)] = Ah[:ki, :kj]
            Ls[(i, j)] = _right_solve_upper(Ah[:ki, kj:], Ur[j])
            Us[(i, j)] = _left_solve_lower(Lr[i], Ah[ki:, :kj])
            if i > j:
                Lro[(i, j)] = _right_solve_upper(Ah[ki:, kj:], Ur[j])
            else:
                Uro[(i, j)] = _left_solve_lower(Lr[i], Ah[ki:, kj:])
        for (i, j) in t.far[l]:
            SS[(i, j)] = R[i] @ h2.S[(l, i, j)] @ R[j].T
        levels[l] = LULevel(ks, ms, Q, R, Lr, Ur, Ls, Us, Lro, Uro, SS, t.near_of(l))
        Anew = {}
        for (I, J) in t.near[l - 1]:
            Anew[(I, J)] = np.block([[SS[(2 * I, 2 * J)], SS[(2 * I, 2 * J + 1)]],
                                     [SS[(2 * I + 1, 2 * J)], SS[(2 * I + 1, 2 * J + 1)]]])
        A = Anew
        Rchild = R
    A00 = A[(0, 0)]
    L00, U00 = lu_nopivot(A00, 0, 0) if A00.shape[0] else (np.zeros((0, 0)), np.zeros((0, 0)))
    return LUFactor(h2, levels, A00, L00, U00)


def _lsolve(Lm: np.ndarray, b: np.ndarray) -> np.ndarray:
    return sla.solve_triangular(Lm, b, lower=True, unit_diagonal=True) if Lm.shape[0] else b.copy()


def _usolve(Um: np.ndarray, b: np.ndarray) -> np.ndarray:
    return sla.solve_triangular(Um, b, lower=False) if Um.shape[0] else b.copy()


def solve(fac: LUFactor, b: np.ndarray) -> np.ndarray:
    """x = U^{-1} L^{-1} b: the forward sweep of Eq. 31 with the L blocks, the
    root, and the backward sweep in the same parallel form with the U blocks."""
    h2 = fac.h2
    t = h2.tree
    L = t.L
    b2 = b.reshape(t.n, -1)
    cur = [b2[t.perm][s:e] for (s, e) in t.ranges[L]]
    yRs: list = [None] * (L + 1)
    for l in range(L, 0, -1):
        lv = fac.levels[l]
        nb = 1 << l
        c = [lv.Q[i].T @ cur[i] for i in range(nb)]
        z = [_lsolve(lv.Lr[j], c[j][lv.k[j]:]) for j in range(nb)]
        yR = []
        for i in range(nb):
            w = c[i][lv.k[i]:].copy()
            for j in lv.near[i]:
                if j < i:
                    w -= lv.Lro[(i, j)] @ z[j]
            yR.append(_lsolve(lv.Lr[i], w))
        cS = []
        for i in range(nb):
            v = c[i][:lv.k[i]].copy()
            for j in lv.near[i]:
                v -= lv.Ls[(i, j)] @ yR[j]
            cS.append(v)
        yRs[l] = yR
        cur = [np.vstack([cS[2 * I], cS[2 * I + 1]]) for I in range(nb // 2)]
    x0 = _usolve(fac.U00, _lsolve(fac.L00, cur[0]))
    xs = [x0]
    for l in range(1, L + 1):
        lv = fac.levels[l]
        nb = 1 << l
        xS = []
        for I in range(nb // 2):
            k0 = lv.k[2 * I]
            xS += [xs[I][:k0], xs[I][k0:]]
        tv = []
        for j in range(nb):
            v = yRs[l][j].copy()
            for i in lv.near[j]:
                v -= lv.Us[(j, i)] @ xS[i]
            tv.append(v)
        u = [_usolve(lv.Ur[i], tv[i]) for i in range(nb)]
        xR = []
        for j in range(nb):
            v = tv[j].copy()
            for i in lv.near[j]:
                if i > j:
                    v -= lv.Uro[(j, i)] @ u[i]
            xR.append(_usolve(lv.Ur[j], v))
        xs = [lv.Q[j] @ np.vstack([xS[j], xR[j]]) for j in range(nb)]
    xt = np.vstack(xs)
    x = np.empty_like(xt)
    x[t.perm] = xt
    return x.reshape(b.shape)


def refine(fac: LUFactor, b: np.ndarray, tol: float, max_iter: int):
    """Stationary refinement x <- x + M^{-1}(b - A~ x) with the LU-ULV solve,
    stopped when the largest relative column residual against A~ reaches tol."""
    h2 = fac.h2
    b2 = b.reshape(h2.tree.n, -1)
    bn = np.linalg.norm(b2, axis=0)

    def res(x):
        r = (b - matvec(h2, x)).reshape(h2.tree.n, -1)
        return float(np.max(np.linalg.norm(r, axis=0) / bn))

    x = solve(fac, b)
    hist = [res(x)]
    it = 0
    while hist[-1] > tol and it < max_iter:
        x = x + solve(fac, b - matvec(h2, x))
        hist.append(res(x))
        it += 1
    return x, hist
