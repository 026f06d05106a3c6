"""Pins of the oracle's H^2 construction (Algorithm 1): the ID against the
matrix it compresses, exactness of the approximant when nothing is truncated,
accuracy tracking eps, the sampling rule, and the dense matrix-vector product."""
import numpy as np
import pytest
import scipy.linalg as sla

import workloads as W
from oracle import construct, h2matrix, kernels


def _build(p, pi=None, **kw):
    pi = p.perm() if pi is None else pi
    return construct.construct(p.points, p.kernel, p.leaf, p.eta, p.eps, pi,
                               p.s_far, p.s_near, **kw)


def test_id_reproduces_matrix_within_eps():
    rng = np.random.default_rng(0)
    # numerically low-rank M with a decaying spectrum
    m, s = 80, 120
    Uo, _ = np.linalg.qr(rng.standard_normal((m, m)))
    Vo, _ = np.linalg.qr(rng.standard_normal((s, m)))
    M = (Uo * (10.0 ** -np.linspace(0, 14, m))) @ Vo.T
    for eps in (1e-3, 1e-6, 1e-10):
        piv, k, T, rd = construct.interpolative_decomposition(M, eps)
        assert 0 < k < m
        err = np.linalg.norm(M[piv[k:]] - T.T @ M[piv[:k]], 2)
        assert err <= 10 * np.sqrt(m) * eps * np.linalg.norm(M, 2) * 10
        # leading-count rank: the first dropped pivot is below the threshold
        assert rd[k] <= eps * rd[0] and rd[k - 1] > eps * rd[0]
        U = construct.build_basis(piv, k, T, m)
        assert np.array_equal(U[piv[:k]], np.eye(k))


def test_id_full_rank_when_eps_zero():
    M = np.random.default_rng(1).standard_normal((30, 50))
    piv, k, T, rd = construct.interpolative_decomposition(M, 0.0)
    assert k == 30
    assert sorted(piv.tolist()) == list(range(30))


def test_id_zero_matrix_has_rank_zero():
    piv, k, T, rd = construct.interpolative_decomposition(np.zeros((10, 7)), 1e-8)
    assert k == 0


@pytest.mark.parametrize("eta", [0.0, 1.0])
def test_exact_when_nothing_truncated(eta):
    # eps = 0 and no sampling: every shared basis spans its whole off-diagonal
    # row block, so the H^2 approximant reproduces A to rounding.
    p = W.laplace_cube(n=1024, leaf=64, eps=0.0, eta=eta)
    h2 = _build(p)
    A = kernels.dense(p.kernel, p.points)
    At = h2matrix.assemble_dense(h2)
    assert not np.isnan(At).any()
    assert np.linalg.norm(At - A) / np.linalg.norm(A) < 1e-12


def test_approximation_tracks_eps():
    errs = []
    for eps in (1e-2, 1e-4, 1e-6, 1e-8):
        p = W.yukawa_cube(n=1024, leaf=64, eps=eps, s=256)
        h2 = _build(p)
        A = kernels.dense(p.kernel, p.points)
        errs.append(np.linalg.norm(h2matrix.assemble_dense(h2) - A) / np.linalg.norm(A))
    assert all(b < a for a, b in zip(errs, errs[1:]))
    for eps, e in zip((1e-2, 1e-4, 1e-6, 1e-8), errs):
        assert e < 10 * eps


def test_nested_skeletons_and_couplings():
    p = W.laplace_cube(n=1024, leaf=64, eps=1e-6, s=128)
    h2 = _build(p)
    t = h2.tree
    for l in range(1, t.L):
        for I in range(1 << l):
            B = h2.basis[l][I].B
            kids = np.concatenate([h2.basis[l + 1][2 * I].SK, h2.basis[l + 1][2 * I + 1].SK])
            assert np.array_equal(B, kids)
            assert set(h2.basis[l][I].SK) <= set(B)
    for (l, i, j), S in h2.S.items():
        Si, Sj = h2.basis[l][i].SK, h2.basis[l][j].SK
        assert np.allclose(S, kernels.evaluate(p.kernel, p.points[Si], p.points[Sj], Si, Sj), rtol=0, atol=0)


def test_sampling_takes_earliest_in_pi():
    p = W.laplace_cube(n=512, leaf=32, eps=1e-6, s=40)
    pi = p.perm()
    pirank = np.empty_like(pi)
    pirank[pi] = np.arange(len(pi))
    cands = np.random.default_rng(9).choice(512, 200, replace=False)
    got = construct._sample(cands, pirank, 40)
    brute = [q for q in pi if q in set(cands.tolist())][:40]
    assert got.tolist() == brute
    assert construct._sample(cands, pirank, -1).size == 200


def test_forced_skeletons_reproduce_free_construction():
    p = W.laplace_cube(n=1024, leaf=64, eps=1e-7, s=128)
    h2 = _build(p)
    sk = {}
    for l in range(1, h2.tree.L + 1):
        for i, bb in enumerate(h2.basis[l]):
            sk[(l, i)] = bb.piv[:bb.k]
    h2f = _build(p, skeletons=sk)
    for l in range(1, h2.tree.L + 1):
        for a, b in zip(h2.basis[l], h2f.basis[l]):
            assert np.array_equal(a.SK, b.SK)
            # T = R_11^{-1} R_12 is as sensitive as cond(R_11) ~ 1/eps
            if a.k:
                assert np.linalg.norm(a.U - b.U) <= 1e-6 * np.linalg.norm(a.U)


def test_matvec_equals_dense_assembly():
    p = W.matern_cube(n=1024, leaf=64, eps=1e-6, s=128)
    h2 = _build(p)
    At = h2matrix.assemble_dense(h2)
    x = np.random.default_rng(3).standard_normal((1024, 3))
    y = h2matrix.matvec(h2, x)
    assert np.linalg.norm(y - At @ x) / np.linalg.norm(At @ x) < 1e-14


def test_root_only_when_n_below_leaf():
    p = W.laplace_cube(n=50, leaf=64, eps=1e-8)
    h2 = _build(p)
    assert h2.tree.L == 0
    A = kernels.dense(p.kernel, p.points)
    assert np.array_equal(h2matrix.assemble_dense(h2), A)


def test_kernel_values_closed_form():
    X = np.array([[0.0, 0.0, 0.0], [0.3, 0.4, 0.0]])
    idx = np.arange(2)
    lap = kernels.evaluate(W.Kernel(0, delta=1e-3), X, X, idx, idx)
    assert lap[0, 0] == pytest.approx(1000.0) and lap[0, 1] == pytest.approx(1 / 0.501)
    yuk = kernels.evaluate(W.Kernel(1, delta=1e-3, kappa=1.0), X, X, idx, idx)
    assert yuk[0, 1] == pytest.approx(np.exp(-0.5) / 0.501)
    gau = kernels.evaluate(W.Kernel(2, ell=0.5, nugget=1e-4), X, X, idx, idx)
    assert gau[0, 0] == pytest.approx(1.0 + 1e-4) and gau[0, 1] == pytest.approx(np.exp(-1.0))
    mat = kernels.evaluate(W.Kernel(3, ell=0.2, nugget=1e-4), X, X, idx, idx)
    a = np.sqrt(3) * 0.5 / 0.2
    assert mat[0, 1] == pytest.approx((1 + a) * np.exp(-a)) and mat[1, 1] == pytest.approx(1 + 1e-4)
    # positive definiteness of the kernels (Schoenberg / Matern): all eigenvalues > 0
    P = W.cube_points(300, 3, 1)
    for kern in (W.Kernel(0, delta=1e-3), W.Kernel(1, delta=1e-3, kappa=1.0),
                 W.Kernel(2, ell=0.3, nugget=1e-4), W.Kernel(3, ell=0.2, nugget=1e-4)):
        assert np.linalg.eigvalsh(kernels.dense(kern, P))[0] > 0
