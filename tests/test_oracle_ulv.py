"""Pins of the oracle's ULV factorization and substitution.

Independent references: the dense assembly of the H^2 operator transformed
by the block-diagonal orthogonal bases (every stored factor block must satisfy
its defining identity against it), the dense Schur complement, exact solves
where the method is exact (HSS admissibility, no truncation), dense LU on the
small Laplace case, and refinement converging to the dense solve of A~.
"""
import numpy as np
import pytest
import scipy.linalg as sla

import workloads as W
from oracle import construct, flops, h2matrix, kernels, ulv


def _build(p, **kw):
    return construct.construct(p.points, p.kernel, p.leaf, p.eta, p.eps, p.perm(),
                               p.s_far, p.s_near, **kw)


@pytest.fixture(scope="module")
def compressed():
    # eta = 1, sampled, truncated: off-diagonal redundant blocks are non-zero.
    p = W.laplace_cube(n=2048, leaf=64, eps=1e-6, s=128)
    h2 = _build(p)
    return p, h2, ulv.factor(h2)


def test_bases_orthogonal_and_span(compressed):
    p, h2, fac = compressed
    for l in range(1, h2.tree.L + 1):
        lv = fac.levels[l]
        for i in range(1 << l):
            Q, k = lv.Q[i], lv.k[i]
            assert np.linalg.norm(Q.T @ Q - np.eye(Q.shape[0])) < 1e-13 * Q.shape[0]
            W_ = h2.basis[l][i].U if l == h2.tree.L else \
                sla.block_diag(fac.levels[l + 1].R[2 * i], fac.levels[l + 1].R[2 * i + 1]) @ h2.basis[l][i].U
            assert np.allclose(Q[:, :k] @ lv.R[i], W_, atol=1e-12 * max(1, np.abs(W_).max()))


def test_leaf_factor_blocks_against_dense_transform(compressed):
    p, h2, fac = compressed
    t = h2.tree
    L = t.L
    lv = fac.levels[L]
    At = h2matrix.assemble_dense(h2)[np.ix_(t.perm, t.perm)]     # tree order
    Qb = sla.block_diag(*lv.Q)
    Ah = Qb.T @ At @ Qb
    off = np.cumsum([0] + lv.m)
    blk = lambda i, j: Ah[off[i]:off[i + 1], off[j]:off[j + 1]]
    scale = np.abs(Ah).max()
    tol = 1e-12 * scale
    for i in range(1 << L):
        ki = lv.k[i]
        A_ii = blk(i, i)
        Lr = lv.Lr[i]
        assert np.abs(Lr @ Lr.T - A_ii[ki:, ki:]).max() < tol
        assert np.abs(lv.Ls[(i, i)] @ Lr.T - A_ii[:ki, ki:]).max() < tol
        # Schur identity: SS - SR RR^{-1} RS
        schur = A_ii[:ki, :ki] - A_ii[:ki, ki:] @ np.linalg.solve(A_ii[ki:, ki:], A_ii[ki:, :ki])
        assert np.abs(lv.SS[(i, i)] - schur).max() < 1e-10 * scale
    for (i, j) in t.near[L]:
        if i == j:
            continue
        ki, kj = lv.k[i], lv.k[j]
        Aij = blk(i, j)
        Lrj = lv.Lr[j]
        assert np.abs(lv.Ls[(i, j)] @ Lrj.T - Aij[:ki, kj:]).max() < tol
        assert np.abs(lv.SS[(i, j)] - Aij[:ki, :kj]).max() < tol
        if i > j:
            assert np.abs(lv.Lro[(i, j)] @ Lrj.T - Aij[ki:, kj:]).max() < tol
    for (i, j) in t.far[L]:
        ki, kj = lv.k[i], lv.k[j]
        Aij = blk(i, j)
        assert np.abs(lv.SS[(i, j)] - Aij[:ki, :kj]).max() < tol
        # a far block has no redundant part in the orthogonal coordinates
        assert np.abs(Aij[ki:, :]).max() < tol and np.abs(Aij[:, kj:]).max() < tol
    # some off-diagonal redundant couplings are genuinely non-zero here
    assert max(np.abs(v).max() for v in lv.Lro.values()) > 1e-6 * scale


def test_merge_places_children_blocks(compressed):
    p, h2, fac = compressed
    t = h2.tree
    L = t.L
    lv = fac.levels[L]
    parent = fac.levels[L - 1]
    # parent diagonal transform equals Q^T (merged block) Q; rebuild merged blocks
    for (I, J) in t.near[L - 1]:
        M = np.block([[lv.SS[(2 * I, 2 * J)], lv.SS[(2 * I, 2 * J + 1)]],
                      [lv.SS[(2 * I + 1, 2 * J)], lv.SS[(2 * I + 1, 2 * J + 1)]]])
        if I == J:
            kI = parent.k[I]
            Ah = parent.Q[I].T @ M @ parent.Q[I]
            Lr = parent.Lr[I]
            assert np.allclose(Lr @ Lr.T, Ah[kI:, kI:], atol=1e-11 * np.abs(Ah).max())


def test_flop_count_hand_case():
    # two boxes of m = 2, k = 1, near each other; root n0 = 2
    ff, fs = flops.count([None, [2, 2]], [None, [1, 1]],
                         [[(0, 0)], [(0, 0), (0, 1), (1, 0), (1, 1)]], [[], []], 2, nrhs=3)
    per_box = flops.geqrf(2, 1) + flops.orgqr_full(2, 1) + 4 * 8 + 1 / 3 + 1 + 1 + 2
    assert ff == pytest.approx(2 * per_box + 2 * 1 + 2 * 2 * 2 * 4 + 1 + 8 / 3)
    assert fs == pytest.approx(3 * (2 * (16 + 4) + 4 * 4 + 4 + 8))
    assert flops.geqrf(5, 5) == pytest.approx(2 * 125 - 2 / 3 * 125)


@pytest.mark.parametrize("kern", ["laplace", "matern"])
def test_hss_is_exact(kern):
    # eta = 0: no near off-diagonal blocks, nothing is dropped (HSS-ULV).
    # (with eta = 0 every adjacent box is "far": a far-field sample cannot
    # represent it, so no sampling here)
    if kern == "laplace":
        p = W.laplace_cube(n=1024, leaf=64, eps=1e-5, eta=0.0, s=-1)
    else:
        p = W.matern_cube(n=1024, leaf=64, eps=1e-5, eta=0.0, s=-1)
    h2 = _build(p)
    fac = ulv.factor(h2)
    b = W.rhs(1024, 3, 1)
    x = ulv.solve(fac, b)
    At = h2matrix.assemble_dense(h2)
    xe = np.linalg.solve(At, b)
    cond = np.linalg.cond(At)
    assert np.linalg.norm(x - xe) / np.linalg.norm(xe) < 1e-15 * cond * 100
    assert np.array_equal(ulv.solve_naive(fac, b), x)


def test_no_truncation_equals_dense_cholesky():
    p = W.yukawa_cube(n=1024, leaf=64, eps=0.0, s=-1)
    h2 = _build(p)
    fac = ulv.factor(h2)
    b = W.rhs(1024, 2, 1)
    A = kernels.dense(p.kernel, p.points)
    xe = sla.cho_solve(sla.cho_factor(A), b)
    assert np.linalg.norm(ulv.solve(fac, b) - xe) / np.linalg.norm(xe) < 1e-12


def test_laplace_2048_against_dense_lu():
    p = W.laplace_cube()          # N=2048, leaf 128, eta 1, eps 1e-10, no sampling
    h2 = _build(p)
    fac = ulv.factor(h2)
    b = p.b()
    A = kernels.dense(p.kernel, p.points)
    xl = sla.lu_solve(sla.lu_factor(A), b)
    assert np.linalg.norm(ulv.solve(fac, b) - xl) / np.linalg.norm(xl) < 1e-8


def test_parallel_and_naive_substitution_agree_to_dropped_terms(compressed):
    p, h2, fac = compressed
    b = W.rhs(2048, 2, 1)
    x = ulv.solve(fac, b)
    xn = ulv.solve_naive(fac, b)
    d = np.linalg.norm(x - xn) / np.linalg.norm(x)
    assert 0 < d < 1e-4
    # the parallel form is Eq. 31 exactly: on one level with the dense factors,
    # y = F c with F_ii = L_ii^{-1}, F_ij = -L_ii^{-1} L_ij L_jj^{-1} (i > j near)
    L = h2.tree.L
    lv = fac.levels[L]
    nb = 1 << L
    r = [lv.m[i] - lv.k[i] for i in range(nb)]
    ro = np.cumsum([0] + r)
    F = np.zeros((ro[-1], ro[-1]))
    for i in range(nb):
        Li = np.linalg.inv(lv.Lr[i])
        F[ro[i]:ro[i + 1], ro[i]:ro[i + 1]] = Li
        for j in lv.near[i]:
            if j < i:
                F[ro[i]:ro[i + 1], ro[j]:ro[j + 1]] = -Li @ lv.Lro[(i, j)] @ np.linalg.inv(lv.Lr[j])
    c = np.random.default_rng(5).standard_normal(ro[-1])
    z = [sla.solve_triangular(lv.Lr[j], c[ro[j]:ro[j + 1]], lower=True) for j in range(nb)]
    y = []
    for i in range(nb):
        w = c[ro[i]:ro[i + 1]].copy()
        for j in lv.near[i]:
            if j < i:
                w -= lv.Lro[(i, j)] @ z[j]
        y.append(sla.solve_triangular(lv.Lr[i], w, lower=True))
    assert np.allclose(np.concatenate(y), F @ c, rtol=1e-10, atol=1e-12)


def test_refinement_converges_to_dense_solve(compressed):
    p, h2, fac = compressed
    b = W.rhs(2048, 1, 1)
    x, hist = ulv.refine(fac, b, 1e-12, 20)
    assert hist[-1] <= 1e-12 and len(hist) <= 8
    At = h2matrix.assemble_dense(h2)
    xe = np.linalg.solve(At, b)
    assert np.linalg.norm(x - xe) / np.linalg.norm(xe) < 1e-10
    xp, its = ulv.pcg(fac, b, 1e-12, 50)
    assert np.linalg.norm(xp - xe) / np.linalg.norm(xe) < 1e-10


def test_residual_tracks_eps():
    res = []
    for eps in (1e-3, 1e-6, 1e-9):
        p = W.laplace_cube(n=1024, leaf=64, eps=eps, s=256)
        h2 = _build(p)
        fac = ulv.factor(h2)
        b = p.b()
        A = kernels.dense(p.kernel, p.points)
        x = ulv.solve(fac, b)
        res.append(np.linalg.norm(b - A @ x) / np.linalg.norm(b))
    assert res[0] > res[1] > res[2]
    assert res[2] < 1e-6


def test_not_spd_is_reported():
    p = W.laplace_cube(n=512, leaf=64, eps=1e-6, s=64)
    bad = W.Kernel(0, delta=-1e-3)      # 1/(r - 1e-3): negative diagonal
    h2 = construct.construct(p.points, W.Kernel(0, delta=1e-3), p.leaf, p.eta, p.eps, p.perm(), 64, 64)
    for key in h2.D:
        if key[0] == key[1]:
            h2.D[key] = h2.D[key] - 2000.0 * np.eye(h2.D[key].shape[0])
    with pytest.raises(ulv.NotSPD) as e:
        ulv.factor(h2)
    assert e.value.level == h2.tree.L
    del bad


def test_single_box_is_dense_cholesky():
    p = W.matern_cube(n=60, leaf=64, eps=1e-6)
    h2 = _build(p)
    fac = ulv.factor(h2)
    A = kernels.dense(p.kernel, p.points)
    b = W.rhs(60, 2, 1)
    assert np.allclose(ulv.solve(fac, b), sla.cho_solve(sla.cho_factor(A), b), rtol=1e-9)
