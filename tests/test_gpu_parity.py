"""Parity of the HIP library against the CPU oracle, through the C ABI.

Same-H^2 cases give the library the oracle's skeleton selection
(h2_build_fixed), so both sides factor the same H^2 matrix: x must agree to
max(1e-10, 100 kappa(A~) u) relative (FP64 on both sides, u the unit
roundoff), in norm and element by element (max |x - x_o| / max |x_o|), the
residual against A~ must match the oracle's, the matvec must agree to 1e-12
(norm and element-wise), the library's canonical flop counts must equal the
oracle's, the leaf factor blocks V_i V_i^T = Q_i^R (A^_ii^RR)^{-1} Q_i^R^T
(independent of how the complement basis is chosen) must agree, and the
assembled root block must have the same spectrum.  Free cases let the
library pick its own skeletons by its pivoted QR: the structure must agree
exactly, most ranks must agree, and the residual against the exact kernel
matrix must stay within the oracle's own accuracy.

Tolerances that depend on eps: both sides compute the interpolation
coefficients T = R_11^{-1} R_12 from sampled blocks M that differ by rounding,
|dM| <= u |R_00| (u the unit roundoff, |R_00| the largest column norm).  To
first order dT = R_11^{-1} (dR_12 - dR_11 T), and the pivoted QR keeps
sigma_min(R_11) near its last retained pivot, which is above eps |R_00|; so
|dT| <~ (1 + |T|) u / eps.  U_i moves by that much, and so does the projector
onto its complement (U_i has identity rows: sigma_min(U_i) >= 1).  The root
block, expressed in the skeleton coordinates, inherits the perturbation:
its spectrum agrees to max(tol, g u / eps) relative, g = max_i (1 + |T_i|_2)
over the oracle's boxes.  The leaf blocks V V^T = Q^R (A^RR)^{-1} Q^R^T add
the inverse of the redundant block, which amplifies the projector's change by
at most kappa(A^RR) <= kappa(A~) (a compression keeps the eigenvalues inside
A~'s range): 4 kappa(A~) g u / eps.  x, a function of A~ alone, keeps the
tight bound.
"""
import dataclasses

import numpy as np
import pytest
import scipy.linalg as sla

import workloads as W
from oracle import construct, flops, h2matrix, kernels, ulv

pytestmark = pytest.mark.gpu


def _oracle(p, skeletons=None):
    h2 = construct.construct(p.points, p.kernel, p.leaf, p.eta, p.eps, p.perm(), p.s_far,
                             p.s_near, skeletons=skeletons)
    return h2


def _skeletons(h2):
    """(dict for the oracle, ranks and positions in levels L..1 order)."""
    sk, ranks, pos = {}, [], []
    for l in range(h2.tree.L, 0, -1):
        for i, bb in enumerate(h2.basis[l]):
            sk[(l, i)] = bb.piv[:bb.k]
            ranks.append(bb.k)
            pos.extend(bb.piv[:bb.k].tolist())
    return sk, np.array(ranks, dtype=np.int32), np.array(pos, dtype=np.int32)


def _rel(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


CASES = {
    # name: (problem factory, nrhs)
    "laplace2048_full": (lambda: W.laplace_cube(), 1),
    "laplace4096_sampled": (lambda: W.laplace_cube(n=4096, leaf=64, eps=1e-6, s=128), 3),
    "yukawa_ragged": (lambda: W.yukawa_cube(n=3001, leaf=100, eps=1e-7, s=150), 2),
    "sphere_hss": (lambda: W.laplace_sphere(n=2048, leaf=64, eps=1e-6, eta=0.0, s=-1, nrhs=1), 1),
    "gauss2d": (lambda: _gauss2d(), 1),
    "matern_full": (lambda: W.matern_cube(n=1500, leaf=64, eps=1e-8, s=-1), 2),
    # near-field sampling variants (Section 3.5): a near sample smaller than
    # the far one, and every near candidate with a sampled far field
    "yukawa_near_sampled": (lambda: dataclasses.replace(
        W.yukawa_cube(n=4096, leaf=64, eps=1e-7, nrhs=1, s=256), s_near=48), 1),
    "laplace_near_all": (lambda: dataclasses.replace(
        W.laplace_cube(n=2048, leaf=128, eps=1e-7, s=128), s_near=-1), 1),
    "root_only": (lambda: W.laplace_cube(n=100, leaf=128, eps=1e-8), 2),
    # the right-hand-side counts of the 16-RHS configuration and of the
    # chunking beyond the 16 columns one pass carries
    "laplace4096_16rhs": (lambda: W.laplace_cube(n=4096, leaf=64, eps=1e-6, s=128), 16),
    "sphere_17rhs": (lambda: W.laplace_sphere(n=4096, leaf=128, eps=1e-7, s=256, nrhs=17), 17),
}


def _gauss2d():
    p = W.gaussian_batch(n_inst=1, n_min=1500, n_max=1500, leaf=64, eps=1e-8, s=-1)[0]
    return p


@pytest.mark.parametrize("name", list(CASES))
def test_same_h2_solve_matches_oracle(lib, name):
    import torch
    factory, nrhs = CASES[name]
    p = factory()
    print(f"[case {name}] n={p.n} leaf={p.leaf} eps={p.eps} eta={p.eta}", flush=True)
    h2o = _oracle(p)
    sk, ranks, pos = _skeletons(h2o)
    h2f = _oracle(p, skeletons=sk)
    fac = ulv.factor(h2f)
    b = W.rhs(p.n, nrhs, 1)
    xo = ulv.solve(fac, b)
    H = lib.build_fixed(p.points, p.kernel, p.leaf, p.eta, p.eps, p.perm(), ranks, pos,
                        s_far=p.s_far, s_near=p.s_near)
    perm, gr, gm, gsk = H.structure()
    assert np.array_equal(perm, h2o.tree.perm)
    assert np.array_equal(gr, ranks)
    H.factor()
    bt = torch.from_numpy(b).cuda()
    x = H.solve(bt).cpu().numpy()
    # both sides are FP64 on the same H^2 matrix: x agrees to rounding times the
    # condition number of A~, and both residuals against A~ are equally small
    At = h2matrix.assemble_dense(h2f)
    kappa = np.linalg.cond(At)
    u = np.finfo(float).eps / 2
    tol = max(1e-10, 100 * kappa * 2 * u)
    ew = float(np.abs(x - xo).max() / np.abs(xo).max())
    print(f"[{name}] x: norm {_rel(x, xo):.2e} element-wise {ew:.2e} (tol {tol:.1e}, "
          f"kappa {kappa:.1f})", flush=True)
    assert _rel(x, xo) < tol, (_rel(x, xo), kappa)
    assert ew < tol, (ew, kappa)
    res_g = np.linalg.norm(b - At @ x) / np.linalg.norm(b)
    res_o = np.linalg.norm(b - At @ xo) / np.linalg.norm(b)
    assert res_g <= max(10 * res_o, 1e-13), (res_g, res_o)
    # the H^2 operator itself
    y = H.matvec(bt).cpu().numpy()
    yo = h2matrix.matvec(h2f, b)
    assert _rel(y, yo) < 1e-12, _rel(y, yo)
    # component by component against the rounding bound of a product,
    # |y - y_o| <= gamma_n |A~| |b| (gamma_n = n u / (1 - n u) < 1e-12 for the
    # n <= 4096 terms of a row here)
    cw = float(np.max(np.abs(y - yo) / (np.abs(At) @ np.abs(b))))
    assert cw < 1e-12, cw
    # the library's canonical flop count against the oracle's, on the same
    # structure
    st = H.stats()
    ff_o, fs_o = flops.count_h2(h2f)
    assert abs(st["flops_factor"] - ff_o) <= 1e-12 * ff_o, (st["flops_factor"], ff_o)
    assert abs(st["flops_solve"] - fs_o) <= 1e-12 * fs_o, (st["flops_solve"], fs_o)
    L = h2f.tree.L
    if L > 0:
        g = _id_growth(h2f)
        # leaf factor blocks V V^T, box by box, norm and element-wise
        lv = fac.levels[L]
        tol_v = max(1e-12, 4 * kappa * g * u / max(p.eps, 1e-300))
        worst = 0.0
        for i in range(1 << L):
            P, k = H.basis(L, i)
            assert k == lv.k[i]
            Vg = P[:, k:]
            Vo = lv.V[i]
            if Vo.shape[1] == 0:
                continue
            Go, Gg = Vo @ Vo.T, Vg @ Vg.T
            worst = max(worst, float(np.abs(Gg - Go).max() / np.abs(Go).max()),
                        float(np.linalg.norm(Gg - Go) / np.linalg.norm(Go)))
        print(f"[{name}] leaf V V^T worst deviation {worst:.2e} (tol {tol_v:.1e})", flush=True)
        assert worst < tol_v, (worst, tol_v)
        # the assembled root block's spectrum (Weyl: |d lambda_i| <=
        # ||root_gpu - root_oracle||_2), see the module docstring
        ro = fac.A_root
        rg = H.root()
        ev_o = np.linalg.eigvalsh((ro + ro.T) / 2)
        ev_g = np.linalg.eigvalsh((rg + rg.T) / 2)
        dev = np.abs(ev_g - ev_o).max() / np.abs(ev_o).max()
        tol_root = max(tol, g * u / max(p.eps, 1e-300))
        print(f"[{name}] root spectrum deviation {dev:.2e} (tol {tol_root:.1e})", flush=True)
        assert dev < tol_root, (dev, kappa, tol_root)
    H.close()


def _id_growth(h2):
    """max over boxes of 1 + ||T_i||_2, T_i^T being the rows of U_i outside
    the skeleton."""
    g = 1.0
    for l in range(1, h2.tree.L + 1):
        for bb in h2.basis[l]:
            if bb.k and bb.m > bb.k:
                g = max(g, 1.0 + float(np.linalg.norm(bb.U[bb.piv[bb.k:]], 2)))
    return g


def _power(op, n, iters=30, seed=5):
    """Largest eigenvalue of a symmetric positive operator by the power method
    (Rayleigh quotient of the last iterate)."""
    v = np.random.default_rng(seed).standard_normal(n)
    v /= np.linalg.norm(v)
    lam = 0.0
    for _ in range(iters):
        w = op(v)
        lam = float(v @ w)
        v = w / np.linalg.norm(w)
    return lam


def test_deep_tree_same_h2(lib):
    """Nine levels (N = 16384, leaf 32, 64-point samples), so that every tree
    height the library's gather planner distinguishes (plain, wide, 128- and
    32-column segments) meets the oracle.  kappa(A~) is estimated without
    assembling A~: lambda_max(A~) by the power method on the oracle's H^2
    matvec, 1/lambda_min by the power method on the oracle's ULV solve (an
    approximate inverse of A~; the estimate is doubled for the difference)."""
    import torch
    p = W.yukawa_cube(n=16384, leaf=32, eps=1e-6, nrhs=2, s=64)
    print(f"[case deep] n={p.n} leaf={p.leaf}", flush=True)
    h2o = _oracle(p)
    assert h2o.tree.L == 9
    sk, ranks, pos = _skeletons(h2o)
    h2f = _oracle(p, skeletons=sk)
    fac = ulv.factor(h2f)
    b = W.rhs(p.n, 2, 1)
    xo = ulv.solve(fac, b)
    lmax = _power(lambda v: h2matrix.matvec(h2f, v), p.n)
    linv = _power(lambda v: ulv.solve(fac, v), p.n)
    kappa = 2.0 * lmax * linv
    H = lib.build_fixed(p.points, p.kernel, p.leaf, p.eta, p.eps, p.perm(), ranks, pos,
                        s_far=p.s_far, s_near=p.s_near)
    H.factor()
    bt = torch.from_numpy(b).cuda()
    x = H.solve(bt).cpu().numpy()
    tol = max(1e-10, 100 * kappa * np.finfo(float).eps)
    ew = float(np.abs(x - xo).max() / np.abs(xo).max())
    print(f"[deep] kappa est {kappa:.1f}; x norm {_rel(x, xo):.2e} element-wise {ew:.2e}",
          flush=True)
    assert _rel(x, xo) < tol and ew < tol
    y = H.matvec(bt).cpu().numpy()
    yo = h2matrix.matvec(h2f, b)
    assert _rel(y, yo) < 1e-12
    assert np.abs(y - yo).max() / np.abs(yo).max() < 1e-12
    H.close()


def test_plain_fp64_config_against_dense_lu(lib):
    """The plain FP64 configuration at N = 2048 (uniform cube, 1/(r + 1e-3),
    leaf 128, eta 1, eps 1e-10, every candidate sampled), built by the
    library's own pivoted QR, against dense FP64 LU: relative difference at
    most 1e-8."""
    import torch
    p = W.laplace_cube()
    H = lib.build(p.points, p.kernel, p.leaf, p.eta, p.eps, p.perm(), s_far=p.s_far,
                  s_near=p.s_near)
    H.factor()
    b = p.b()
    x = H.solve(torch.from_numpy(b).cuda()).cpu().numpy()
    A = kernels.dense(p.kernel, p.points)
    x_lu = sla.lu_solve(sla.lu_factor(A), b)
    err = _rel(x, x_lu)
    print(f"[cfg dense LU] ||x - x_LU|| / ||x_LU|| = {err:.2e}", flush=True)
    assert err <= 1e-8
    H.close()


def test_structure_matches_oracle(lib):
    p = W.laplace_sphere(n=8192, leaf=64, eps=1e-6, s=128, nrhs=1)
    h2o_tree = __import__("oracle.tree", fromlist=["ClusterTree"]).ClusterTree(p.points, p.leaf, p.eta)
    H = lib.build(p.points, p.kernel, p.leaf, p.eta, p.eps, p.perm(), s_far=p.s_far, s_near=p.s_near)
    perm, ranks, ms, skel = H.structure()
    assert np.array_equal(perm, h2o_tree.perm)
    for l in range(h2o_tree.L + 1):
        assert H.pairs(l, False) == h2o_tree.near[l]
        assert H.pairs(l, True) == h2o_tree.far[l]
    st = H.stats()
    assert st["levels"] == h2o_tree.L
    assert st["leaf_near_blocks"] == len(h2o_tree.near[h2o_tree.L])
    H.close()


@pytest.mark.parametrize("kern", ["laplace", "yukawa"])
def test_free_build_end_to_end(lib, kern):
    import torch
    if kern == "laplace":
        p = W.laplace_cube(n=4096, leaf=64, eps=1e-7, s=128)
    else:
        p = W.yukawa_cube(n=4096, leaf=64, eps=1e-7, s=128)
    h2o = _oracle(p)
    H = lib.build(p.points, p.kernel, p.leaf, p.eta, p.eps, p.perm(), s_far=p.s_far,
                  s_near=p.s_near)
    perm, ranks, ms, skel = H.structure()
    o_ranks = np.array([bb.k for l in range(h2o.tree.L, 0, -1) for bb in h2o.basis[l]])
    # pivot near-ties may differ; ranks agree almost everywhere and within a few
    assert np.mean(ranks == o_ranks) > 0.7
    assert np.max(np.abs(ranks - o_ranks)) <= 3
    H.factor()
    b = p.b()
    x = H.solve(torch.from_numpy(b).cuda()).cpu().numpy()
    A = kernels.dense(p.kernel, p.points)
    res_g = np.linalg.norm(b - A @ x) / np.linalg.norm(b)
    xo = ulv.solve(ulv.factor(h2o), b)
    res_o = np.linalg.norm(b - A @ xo) / np.linalg.norm(b)
    assert res_g <= max(10 * res_o, 1e-12), (res_g, res_o)
    H.close()


def test_refinement_reaches_tolerance(lib):
    import torch
    p = W.laplace_cube(n=4096, leaf=64, eps=1e-5, s=128)
    H = lib.build(p.points, p.kernel, p.leaf, p.eta, p.eps, p.perm(), s_far=p.s_far,
                  s_near=p.s_near, ir_max_iter=30, ir_tol=1e-12)
    H.factor()
    b = W.rhs(p.n, 2, 1)
    bt = torch.from_numpy(b).cuda()
    x = H.solve(bt)
    st = H.stats()
    assert st["ir_residual"] <= 1e-12 and st["ir_iters"] >= 1
    r = bt - H.matvec(x)
    assert float(torch.linalg.norm(r) / torch.linalg.norm(bt)) <= 2e-12
    H.close()
    Hp = lib.build(p.points, p.kernel, p.leaf, p.eta, p.eps, p.perm(), s_far=p.s_far,
                   s_near=p.s_near, ir_max_iter=30, ir_tol=1e-12, use_pcg=True)
    Hp.factor()
    xp = Hp.solve(bt)
    assert Hp.stats()["ir_residual"] <= 1e-12
    assert float(torch.linalg.norm(xp - x) / torch.linalg.norm(x)) < 1e-9
    Hp.close()


def test_gauss_seidel_prefactorization_matches_oracle(lib):
    """Section 3.5's Gauss-Seidel replacement of the near-sample solve: the
    library's build with two sweeps against the oracle's with two sweeps
    (ranks agree almost everywhere; the solve keeps the oracle's accuracy),
    and the exact build for comparison."""
    import torch
    p = W.yukawa_cube(n=4096, leaf=64, eps=1e-7, s=128)
    h2o = construct.construct(p.points, p.kernel, p.leaf, p.eta, p.eps, p.perm(), p.s_far,
                              p.s_near, gs_sweeps=2)
    H = lib.build(p.points, p.kernel, p.leaf, p.eta, p.eps, p.perm(), s_far=p.s_far,
                  s_near=p.s_near, gs_sweeps=2)
    print(f"[case gauss_seidel] n={p.n} sweeps=2", flush=True)
    _, ranks, _, _ = H.structure()
    o_ranks = np.array([bb.k for l in range(h2o.tree.L, 0, -1) for bb in h2o.basis[l]])
    assert np.mean(ranks == o_ranks) > 0.7
    assert np.max(np.abs(ranks - o_ranks)) <= 3
    H.factor()
    b = p.b()
    x = H.solve(torch.from_numpy(b).cuda()).cpu().numpy()
    A = kernels.dense(p.kernel, p.points)
    res_g = np.linalg.norm(b - A @ x) / np.linalg.norm(b)
    xo = ulv.solve(ulv.factor(h2o), b)
    res_o = np.linalg.norm(b - A @ xo) / np.linalg.norm(b)
    print(f"[gauss_seidel] residual gpu {res_g:.2e} oracle {res_o:.2e}", flush=True)
    assert res_g <= max(10 * res_o, 1e-12), (res_g, res_o)
    H.close()


def test_gauss_seidel_same_h2_matches_oracle(lib):
    """The Gauss-Seidel construction with the oracle's skeleton selection: both
    sides build the same H^2 matrix (interpolation from the sampled blocks with
    one sweep in place of the near-sample solve), so the solve, the matvec and
    the residual follow the same bounds as the exact same-H^2 cases."""
    import torch
    p = W.yukawa_cube(n=3001, leaf=100, eps=1e-7, nrhs=2, s=150)
    print(f"[case gauss_seidel_same_h2] n={p.n} sweeps=1", flush=True)
    h2o = construct.construct(p.points, p.kernel, p.leaf, p.eta, p.eps, p.perm(), p.s_far,
                              p.s_near, gs_sweeps=1)
    sk, ranks, pos = _skeletons(h2o)
    h2f = construct.construct(p.points, p.kernel, p.leaf, p.eta, p.eps, p.perm(), p.s_far,
                              p.s_near, skeletons=sk, gs_sweeps=1)
    b = W.rhs(p.n, 2, 1)
    xo = ulv.solve(ulv.factor(h2f), b)
    H = lib.build_fixed(p.points, p.kernel, p.leaf, p.eta, p.eps, p.perm(), ranks, pos,
                        s_far=p.s_far, s_near=p.s_near, gs_sweeps=1)
    H.factor()
    bt = torch.from_numpy(b).cuda()
    x = H.solve(bt).cpu().numpy()
    At = h2matrix.assemble_dense(h2f)
    kappa = np.linalg.cond(At)
    tol = max(1e-10, 100 * kappa * np.finfo(float).eps)
    print(f"[gauss_seidel_same_h2] x rel {_rel(x, xo):.2e} kappa {kappa:.1e}", flush=True)
    assert _rel(x, xo) < tol, (_rel(x, xo), kappa)
    y = H.matvec(bt).cpu().numpy()
    assert _rel(y, h2matrix.matvec(h2f, b)) < 1e-12
    H.close()
