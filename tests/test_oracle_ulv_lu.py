"""Pins of the oracle's LU variant (non-symmetric kernel matrices).

Independent references: the definition of a pivot-free LU factorization;
the structure of the drift kernel (its symmetric part is the Yukawa kernel);
dense LU solves where the method is exact (no truncation, HSS admissibility);
the Cholesky variant, to which the LU variant must reduce on symmetric
matrices; the stored factor blocks against their defining identities with
the dense transformed blocks; and stationary refinement converging to the
dense solve of the compressed operator.
"""
import numpy as np
import pytest
import scipy.linalg as sla

import workloads as W
from oracle import construct, h2matrix, kernels, ulv, ulv_lu


def _build(p, **kw):
    return construct.construct(p.points, p.kernel, p.leaf, p.eta, p.eps, p.perm(),
                               p.s_far, p.s_near, **kw)


def _rel(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def test_lu_nopivot_is_an_lu_factorization():
    rng = np.random.default_rng(3)
    A = rng.standard_normal((40, 40)) + 40 * np.eye(40)
    Lm, U = ulv_lu.lu_nopivot(A)
    assert np.array_equal(np.diag(Lm), np.ones(40))
    assert np.array_equal(Lm, np.tril(Lm)) and np.array_equal(U, np.triu(U))
    assert np.allclose(Lm @ U, A, rtol=0, atol=1e-12 * np.abs(A).max())
    # without row exchanges it must agree with scipy's LU wherever scipy does
    # not pivot (a diagonally dominant matrix)
    P, Ls, Us = sla.lu(A)
    assert np.array_equal(P, np.eye(40))
    assert np.allclose(Ls, Lm, atol=1e-13) and np.allclose(Us, U, atol=1e-11)
    B = A.copy()
    B[0, 0] = 0.0
    with pytest.raises(ulv_lu.LUBreakdown):
        ulv_lu.lu_nopivot(B, 2, 5)


def test_drift_kernel_is_yukawa_plus_skew():
    p = W.yukawa_drift_cube(n=300, leaf=64, beta=0.5)
    A = kernels.dense(p.kernel, p.points)
    Y = kernels.dense(W.Kernel(W.YUKAWA, delta=1e-3, kappa=1.0), p.points)
    assert np.allclose((A + A.T) / 2, Y, rtol=1e-14, atol=0)
    assert not kernels.symmetric(p.kernel)
    assert np.linalg.norm(A - A.T) > 1e-2 * np.linalg.norm(A)
    # x^T A x = x^T Y x: where Y is positive definite every pivot-free LU exists
    assert np.linalg.eigvalsh(Y).min() > 0
    assert kernels.symmetric(W.Kernel(W.YUKAWA_DRIFT, beta=0.0))


def test_no_truncation_equals_dense_lu():
    p = W.yukawa_drift_cube(n=1024, leaf=64, eps=0.0, beta=0.5, s=-1)
    fac = ulv_lu.factor(_build(p))
    b = W.rhs(1024, 2, 1)
    A = kernels.dense(p.kernel, p.points)
    xe = sla.lu_solve(sla.lu_factor(A), b)
    assert _rel(ulv_lu.solve(fac, b), xe) < 1e-12


def test_hss_is_exact():
    # eta = 0: no near off-diagonal blocks, nothing is dropped
    p = W.yukawa_drift_cube(n=1024, leaf=64, eps=1e-5, beta=0.5, eta=0.0, s=-1)
    h2 = _build(p)
    fac = ulv_lu.factor(h2)
    b = W.rhs(1024, 3, 1)
    At = h2matrix.assemble_dense(h2)
    xe = np.linalg.solve(At, b)
    assert _rel(ulv_lu.solve(fac, b), xe) < 1e-13 * np.linalg.cond(At)


@pytest.mark.parametrize("kern", ["laplace", "drift_beta0"])
def test_reduces_to_the_cholesky_variant(kern):
    # a symmetric matrix: the same H^2 matrix factored both ways gives the same
    # solution (the split of the diagonal between L and U does not reach x)
    if kern == "laplace":
        p = W.laplace_cube(n=2048, leaf=64, eps=1e-6, s=128)
    else:
        p = W.yukawa_drift_cube(n=1024, leaf=64, eps=1e-6, beta=0.0, s=128)
    h2 = _build(p)
    b = W.rhs(p.n, 2, 1)
    assert _rel(ulv_lu.solve(ulv_lu.factor(h2), b), ulv.solve(ulv.factor(h2), b)) < 1e-12


@pytest.fixture(scope="module")
def drift():
    p = W.yukawa_drift_cube(n=1024, leaf=64, eps=1e-6, beta=0.5, s=128)
    h2 = _build(p)
    return p, h2, ulv_lu.factor(h2)


def test_leaf_factor_blocks_against_dense_transform(drift):
    p, h2, fac = drift
    L = h2.tree.L
    lv = fac.levels[L]
    for i in range(1 << L):
        k = lv.k[i]
        Ah = lv.Q[i].T @ h2.D[(i, i)] @ lv.Q[i]
        assert np.allclose(lv.Lr[i] @ lv.Ur[i], Ah[k:, k:], atol=1e-10 * np.abs(Ah).max())
        assert np.allclose(lv.Ls[(i, i)] @ lv.Ur[i], Ah[:k, k:], atol=1e-10 * np.abs(Ah).max())
        assert np.allclose(lv.Lr[i] @ lv.Us[(i, i)], Ah[k:, :k], atol=1e-10 * np.abs(Ah).max())
    checked = 0
    for (i, j) in h2.tree.near[L]:
        if i == j:
            continue
        ki, kj = lv.k[i], lv.k[j]
        Ah = lv.Q[i].T @ h2.D[(i, j)] @ lv.Q[j]
        tol = 1e-10 * np.abs(Ah).max()
        assert np.allclose(lv.Ls[(i, j)] @ lv.Ur[j], Ah[:ki, kj:], atol=tol)
        assert np.allclose(lv.Lr[i] @ lv.Us[(i, j)], Ah[ki:, :kj], atol=tol)
        if i > j:
            assert np.allclose(lv.Lro[(i, j)] @ lv.Ur[j], Ah[ki:, kj:], atol=tol)
        else:
            assert np.allclose(lv.Lr[i] @ lv.Uro[(i, j)], Ah[ki:, kj:], atol=tol)
        assert np.array_equal(fac.levels[L].SS[(i, j)], Ah[:ki, :kj])
        checked += 1
    assert checked > 0


def test_refinement_converges_to_dense_solve(drift):
    p, h2, fac = drift
    b = W.rhs(1024, 2, 1)
    x, hist = ulv_lu.refine(fac, b, 1e-12, 20)
    assert hist[-1] <= 1e-12 and len(hist) <= 6
    At = h2matrix.assemble_dense(h2)
    assert _rel(x, np.linalg.solve(At, b)) < 1e-10
    # the unrefined solve is within the compression error of the dense solve
    A = kernels.dense(p.kernel, p.points)
    assert _rel(ulv_lu.solve(fac, b), np.linalg.solve(A, b)) < 1e-3


def test_shared_basis_spans_rows_and_columns():
    # every far point sampled, eps = 1e-6: the truncated leaf basis must carry
    # the far field of box i as rows (A(B_i, F)) and as columns (A(F, B_i)^T)
    # to about eps (a basis built from the rows alone leaves 2-6e-5 of the
    # column side here)
    p = W.yukawa_drift_cube(n=2048, leaf=128, eps=1e-6, beta=0.5, s=-1)
    p.s_near = 64
    h2 = _build(p)
    t = h2.tree
    L = t.L
    A = kernels.dense(p.kernel, p.points)
    near = t.near_of(L)
    for i in (0, 5, (1 << L) - 1):
        bb = h2.basis[L][i]
        F = np.concatenate([h2.basis[L][j].B for j in range(1 << L) if j not in near[i]])
        assert bb.k < bb.m
        Qu, _ = np.linalg.qr(bb.U)
        for blk in (A[np.ix_(bb.B, F)], A[np.ix_(F, bb.B)].T):
            assert np.linalg.norm(blk - Qu @ (Qu.T @ blk)) <= 2e-6 * np.linalg.norm(blk)
