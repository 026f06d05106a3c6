"""Parity of the HIP library against the CPU oracle, through the C ABI.

Same-H^2 cases give the library the oracle's skeleton selection
(h2_build_fixed), so both sides factor the same H^2 matrix: x must agree to
max(1e-10, 100 kappa(A~) u) relative (FP64 on both sides, u the unit
roundoff), the residual against A~ must match the oracle's, the matvec must
agree to 1e-12 and the assembled root block must have the same spectrum.  Free cases
let the library pick its own skeletons by its pivoted QR: the structure must
agree exactly, most ranks must agree, and the residual against the exact
kernel matrix must stay within the oracle's own accuracy.
"""
import dataclasses

import numpy as np
import pytest

import workloads as W
from oracle import construct, h2matrix, kernels, ulv

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
    tol = max(1e-10, 100 * kappa * np.finfo(float).eps)
    assert _rel(x, xo) < tol, (_rel(x, xo), kappa)
    res_g = np.linalg.norm(b - At @ x) / np.linalg.norm(b)
    res_o = np.linalg.norm(b - At @ xo) / np.linalg.norm(b)
    assert res_g <= max(10 * res_o, 1e-13), (res_g, res_o)
    # the H^2 operator itself
    y = H.matvec(bt).cpu().numpy()
    yo = h2matrix.matvec(h2f, b)
    assert _rel(y, yo) < 1e-12, _rel(y, yo)
    # the assembled root block
    if h2f.tree.L > 0:
        ro = fac.A_root
        rg = H.root()
        ev_o = np.linalg.eigvalsh((ro + ro.T) / 2)
        ev_g = np.linalg.eigvalsh((rg + rg.T) / 2)
        # Weyl: |d lambda_i| <= ||root_gpu - root_oracle||_2.  Unlike x, the
        # root is expressed in the skeleton bases, and the interpolation
        # coefficients T = R_11^{-1} R_12 solve a system whose retained pivots
        # go down to eps |R_00|: rounding differences in the sample matrix can
        # move T (hence the root) by up to u / eps relative, even when the H^2
        # operator itself agrees to 1e-12.
        dev = np.abs(ev_g - ev_o).max() / np.abs(ev_o).max()
        tol_root = max(tol, np.finfo(float).eps / p.eps)
        assert dev < tol_root, (dev, kappa, tol_root)
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
