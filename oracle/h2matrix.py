"""The H^2 operator defined by a construction: nested bases, dense assembly
and the matrix-vector product.

The approximant is
    A~ = sum_{(i,j) near at the leaves} E_i A_ij E_j^T
       + sum_l sum_{(i,j) far at l}   Uhat_i S_ij Uhat_j^T,
with the nested basis Uhat_i = U_i at the leaves and
Uhat_I = blockdiag(Uhat_2I, Uhat_2I+1) U_I above them (Algorithm 1: parents
inherit the children's skeletons, so U_I is a transfer matrix).
"""
from __future__ import annotations

import numpy as np
import scipy.linalg as sla

from .construct import H2Matrix


def nested_bases(h2: H2Matrix) -> list:
    """Uhat[l][i] with rows in tree order of box i's points, for l = 1..L."""
    t = h2.tree
    L = t.L
    Uh: list = [None] * (L + 1)
    if L == 0:
        return Uh
    Uh[L] = [bb.U for bb in h2.basis[L]]
    for l in range(L - 1, 0, -1):
        Uh[l] = [sla.block_diag(Uh[l + 1][2 * I], Uh[l + 1][2 * I + 1]) @ h2.basis[l][I].U
                 for I in range(1 << l)]
    return Uh


def assemble_dense(h2: H2Matrix) -> np.ndarray:
    """A~ as a dense N x N matrix in the original point order."""
    t = h2.tree
    n, L = t.n, t.L
    A = np.full((n, n), np.nan)
    if L == 0:
        A[np.ix_(h2.root_B, h2.root_B)] = h2.D[(0, 0)]
        return A
    Uh = nested_bases(h2)
    for (i, j), blk in h2.D.items():
        bi = h2.basis[L][i].B
        bj = h2.basis[L][j].B
        A[np.ix_(bi, bj)] = blk
    for (l, i, j), S in h2.S.items():
        si, ei = t.ranges[l][i]
        sj, ej = t.ranges[l][j]
        A[np.ix_(t.perm[si:ei], t.perm[sj:ej])] = Uh[l][i] @ S @ Uh[l][j].T
    return A


def matvec(h2: H2Matrix, x: np.ndarray) -> np.ndarray:
    """y = A~ x by the upward pass, couplings, downward pass and near field."""
    t = h2.tree
    L = t.L
    x2 = x.reshape(t.n, -1)
    xt = x2[t.perm]
    yt = np.zeros_like(xt)
    if L == 0:
        yt = h2.D[(0, 0)] @ xt
    else:
        xh: list = [None] * (L + 1)
        xh[L] = [h2.basis[L][i].U.T @ xt[s:e] for i, (s, e) in enumerate(t.ranges[L])]
        for l in range(L - 1, 0, -1):
            xh[l] = [h2.basis[l][I].U.T @ np.vstack([xh[l + 1][2 * I], xh[l + 1][2 * I + 1]])
                     for I in range(1 << l)]
        yh: list = [None] * (L + 1)
        for l in range(1, L + 1):
            yh[l] = [np.zeros((h2.basis[l][i].k, xt.shape[1])) for i in range(1 << l)]
            for (i, j) in t.far[l]:
                yh[l][i] += h2.S[(l, i, j)] @ xh[l][j]
        for l in range(1, L):
            for I in range(1 << l):
                v = h2.basis[l][I].U @ yh[l][I]
                k0 = h2.basis[l + 1][2 * I].k
                yh[l + 1][2 * I] += v[:k0]
                yh[l + 1][2 * I + 1] += v[k0:]
        for i, (s, e) in enumerate(t.ranges[L]):
            yt[s:e] += h2.basis[L][i].U @ yh[L][i]
        for (i, j), blk in h2.D.items():
            si, ei = t.ranges[L][i]
            sj, ej = t.ranges[L][j]
            yt[si:ei] += blk @ xt[sj:ej]
    y = np.empty_like(yt)
    y[t.perm] = yt
    return y.reshape(x.shape)


def near_block_count(h2: H2Matrix) -> int:
    """N_NZB: the number of dense near blocks at the leaves (Section 6.2)."""
    return len(h2.D)
