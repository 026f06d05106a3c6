"""H^2-ULV factorization and substitution.

Factorization: Algorithm 4 (the improved form of Algorithm 2 that reuses
V_j = U_j^R L(r)_jj^{-T}, Eq. 32), with the shared basis completed to a full
orthogonal matrix by Householder QR.  At level l box i has m_i active rows,
rank k_i and r_i = m_i - k_i redundant rows.  With D_i = I at the leaves and
D_i = blockdiag(R_2i, R_2i+1) above them:
  (1) D_i U_i = Q_i [R_i; 0]          (full Q_i = [Q_i^S | Q_i^R], S first)
  (2) A^_ii = Q_i^T A_ii Q_i            split into SS, SR, RS, RR
  (3) L(r)_ii = chol(A^_ii^RR)
  (4) L(s)_ii = A^_ii^SR L(r)_ii^{-T}
  (5) SS_ii  = A^_ii^SS - L(s)_ii L(s)_ii^T   (the only trailing update, Eq. 21)
  (6) V_i = Q_i^R L(r)_ii^{-T}
  (7) near i != j:  Q_i^T A_ij [Q_j^S | V_j] gives SS_ij, L(s)_ij (S rows, R
      columns) and, for i > j, L(r)_ij (R rows, R columns)   (Eq. 32)
  (8) far (i, j):   SS_ij = R_i S_ij R_j^T  -- the coupling expressed in the
      orthogonal skeleton coordinates (the paper writes SS <- S_ij for its
      interpolative completion; with a QR completion the R factors appear)
  (9) merge: the parent block A_IJ is the 2x2 grid of the children's SS blocks
Root: L_00 = chol(A_00).

Substitution: the forward sweep applies L^{-1} in the form of Eq. 31
(Section 3.7), (L^{-1})_ii = L_ii^{-1} and (L^{-1})_ij = -L_ii^{-1} L_ij L_jj^{-1}
for i > j, which drops the second-order terms that Eq. 21 makes zero; the
backward sweep applies the transpose of the same operator.  The naive block
substitution of Algorithm 3 (and its transpose) is kept as a comparator.
"""
from __future__ import annotations

import dataclasses

import numpy as np
import scipy.linalg as sla

from .construct import H2Matrix
from .h2matrix import matvec


class NotSPD(Exception):
    def __init__(self, level: int, box: int):
        super().__init__(f"Cholesky breakdown at level {level}, box {box}")
        self.level, self.box = level, box


@dataclasses.dataclass
class LevelFactor:
    k: list          # ranks
    m: list          # active sizes
    Q: list          # m x m orthogonal completions
    R: list          # k x k triangular factors of D_i U_i
    Lr: list         # r x r lower Cholesky factors of A^_ii^RR
    V: list          # m x r, Q^R L(r)^{-T}
    Ls: dict         # (i, j) near (i == j included) -> k_i x r_j
    Lro: dict        # (i, j) near with i > j -> r_i x r_j
    SS: dict         # (i, j) near or far -> k_i x k_j (what is merged upward)
    near: list       # near[i]: sorted list of near boxes


@dataclasses.dataclass
class ULVFactor:
    h2: H2Matrix
    levels: list     # levels[l] for l = 1..L
    A_root: np.ndarray
    L00: np.ndarray


def _chol(A: np.ndarray, level: int, box: int) -> np.ndarray:
    if A.shape[0] == 0:
        return np.zeros((0, 0))
    try:
        return sla.cholesky(A, lower=True)
    except np.linalg.LinAlgError:
        raise NotSPD(level, box) from None


def _trsm_right_lt(B: np.ndarray, Lr: np.ndarray) -> np.ndarray:
    """B L^{-T} for lower-triangular L."""
    if Lr.shape[0] == 0 or B.shape[0] == 0:
        return np.zeros((B.shape[0], Lr.shape[0]))
    return sla.solve_triangular(Lr, B.T, lower=True).T


def _complete(W: np.ndarray, k: int):
    """Householder QR W = Q [R; 0] with the full square Q."""
    m = W.shape[0]
    if k == 0:
        return np.eye(m), np.zeros((0, 0))
    Q, Rf = sla.qr(W, mode="full")
    return Q, Rf[:k, :k]


def factor(h2: H2Matrix) -> ULVFactor:
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
        Q, R, Lr, V = [], [], [], []
        for i in range(nb):
            W = bas[i].U if l == L else sla.block_diag(Rchild[2 * i], Rchild[2 * i + 1]) @ bas[i].U
            Qi, Ri = _complete(W, ks[i])
            Q.append(Qi)
            R.append(Ri)
        Ls, Lro, SS = {}, {}, {}
        for i in range(nb):
            k = ks[i]
            Ah = Q[i].T @ A[(i, i)] @ Q[i]
            Lri = _chol(Ah[k:, k:], l, i)
            Lsi = _trsm_right_lt(Ah[:k, k:], Lri)
            SS[(i, i)] = Ah[:k, :k] - Lsi @ Lsi.T
            Ls[(i, i)] = Lsi
            Lr.append(Lri)
            V.append(_trsm_right_lt(Q[i][:, k:], Lri))
        for (i, j) in t.near[l]:
            if i == j:
                continue
            ki, kj = ks[i], ks[j]
            T = Q[i].T @ A[(i, j)] @ np.hstack([Q[j][:, :kj], V[j]])
            SS[(i, j)] = T[:ki, :kj]
            Ls[(i, j)] = T[:ki, kj:]
            if i > j:
                Lro[(i, j)] = T[ki:, kj:]
        for (i, j) in t.far[l]:
            SS[(i, j)] = R[i] @ h2.S[(l, i, j)] @ R[j].T
        levels[l] = LevelFactor(ks, ms, Q, R, Lr, V, Ls, Lro, SS, t.near_of(l))
        Anew = {}
        for (I, J) in t.near[l - 1]:
            Anew[(I, J)] = np.block([[SS[(2 * I, 2 * J)], SS[(2 * I, 2 * J + 1)]],
                                     [SS[(2 * I + 1, 2 * J)], SS[(2 * I + 1, 2 * J + 1)]]])
        A = Anew
        Rchild = R
    A00 = A[(0, 0)]
    return ULVFactor(h2, levels, A00, _chol(A00, 0, 0))


def _lsolve(Lm: np.ndarray, b: np.ndarray) -> np.ndarray:
    return sla.solve_triangular(Lm, b, lower=True) if Lm.shape[0] else b.copy()


def _ltsolve(Lm: np.ndarray, b: np.ndarray) -> np.ndarray:
    return sla.solve_triangular(Lm.T, b, lower=False) if Lm.shape[0] else b.copy()


def _sweep(fac: ULVFactor, b: np.ndarray, parallel: bool) -> np.ndarray:
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
        yR = [None] * nb
        if parallel:
            # Eq. 31: y_i = L_ii^{-1} c_i - sum_{j<i} L_ii^{-1} L_ij L_jj^{-1} c_j
            z = [_lsolve(lv.Lr[j], c[j][lv.k[j]:]) for j in range(nb)]
            for i in range(nb):
                w = c[i][lv.k[i]:].copy()
                for j in lv.near[i]:
                    if j < i:
                        w -= lv.Lro[(i, j)] @ z[j]
                yR[i] = _lsolve(lv.Lr[i], w)
        else:
            # Algorithm 3: block forward substitution in box order.
            for i in range(nb):
                w = c[i][lv.k[i]:].copy()
                for j in lv.near[i]:
                    if j < i:
                        w -= lv.Lro[(i, j)] @ yR[j]
                yR[i] = _lsolve(lv.Lr[i], w)
        cS = []
        for i in range(nb):
            v = c[i][:lv.k[i]].copy()
            for j in lv.near[i]:
                v -= lv.Ls[(i, j)] @ yR[j]
            cS.append(v)
        yRs[l] = yR
        cur = [np.vstack([cS[2 * I], cS[2 * I + 1]]) for I in range(nb // 2)]
    x0 = _ltsolve(fac.L00, _lsolve(fac.L00, cur[0]))
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
                v -= lv.Ls[(i, j)].T @ xS[i]
            tv.append(v)
        xR = [None] * nb
        if parallel:
            # Transpose of Eq. 31: x_j = L_jj^{-T} (t_j - sum_{i>j} L_ij^T L_ii^{-T} t_i)
            u = [_ltsolve(lv.Lr[i], tv[i]) for i in range(nb)]
            for j in range(nb):
                v = tv[j].copy()
                for i in lv.near[j]:
                    if i > j:
                        v -= lv.Lro[(i, j)].T @ u[i]
                xR[j] = _ltsolve(lv.Lr[j], v)
        else:
            for j in range(nb - 1, -1, -1):
                v = tv[j].copy()
                for i in lv.near[j]:
                    if i > j:
                        v -= lv.Lro[(i, j)].T @ xR[i]
                xR[j] = _ltsolve(lv.Lr[j], v)
        xs = [lv.Q[j] @ np.vstack([xS[j], xR[j]]) for j in range(nb)]
    xt = np.vstack(xs)
    x = np.empty_like(xt)
    x[t.perm] = xt
    return x.reshape(b.shape)


def solve(fac: ULVFactor, b: np.ndarray) -> np.ndarray:
    """x = (L^T)^{-1} L^{-1} b through the parallel form of Eq. 31."""
    return _sweep(fac, b, parallel=True)


def solve_naive(fac: ULVFactor, b: np.ndarray) -> np.ndarray:
    """The same solve by block forward/backward substitution (Algorithm 3)."""
    return _sweep(fac, b, parallel=False)


def rel_residual(h2: H2Matrix, x: np.ndarray, b: np.ndarray) -> float:
    """max over columns of ||b - A~ x||_2 / ||b||_2."""
    r = (b - matvec(h2, x)).reshape(h2.tree.n, -1)
    bn = np.linalg.norm(b.reshape(h2.tree.n, -1), axis=0)
    return float(np.max(np.linalg.norm(r, axis=0) / bn))


def refine(fac: ULVFactor, b: np.ndarray, tol: float, max_iter: int):
    """Iterative refinement x <- x + M^{-1}(b - A~ x), M^{-1} the ULV solve,
    stopped when the relative residual against A~ reaches ``tol``."""
    h2 = fac.h2
    x = solve(fac, b)
    hist = [rel_residual(h2, x, b)]
    it = 0
    while hist[-1] > tol and it < max_iter:
        x = x + solve(fac, b - matvec(h2, x))
        hist.append(rel_residual(h2, x, b))
        it += 1
    return x, hist


def pcg(fac: ULVFactor, b: np.ndarray, tol: float, max_iter: int):
    """Preconditioned conjugate gradients on A~ x = b (one column at a time),
    preconditioner the ULV solve, which is symmetric positive definite since the
    backward sweep is the transpose of the forward one."""
    h2 = fac.h2
    b2 = b.reshape(h2.tree.n, -1)
    X = np.zeros_like(b2)
    iters = []
    for c in range(b2.shape[1]):
        bc = b2[:, c]
        bn = np.linalg.norm(bc)
        x = solve(fac, bc)
        r = bc - matvec(h2, x)
        z = solve(fac, r)
        p = z.copy()
        rz = r @ z
        it = 0
        while np.linalg.norm(r) / bn > tol and it < max_iter:
            Ap = matvec(h2, p)
            alpha = rz / (p @ Ap)
            x = x + alpha * p
            r = r - alpha * Ap
            z = solve(fac, r)
            rz_new = r @ z
            p = z + (rz_new / rz) * p
            rz = rz_new
            it += 1
        X[:, c] = x
        iters.append(it)
    return X.reshape(b.shape), iters
