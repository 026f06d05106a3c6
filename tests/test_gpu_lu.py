"""The LU variant on the GPU (non-symmetric kernels) against the oracle's LU
variant, through the C ABI.

Same-H^2 cases give the library the oracle's skeleton selection
(h2_build_fixed) for the drift kernel, so both sides factor the same
non-symmetric H^2 matrix with the same pivot-free LU steps: x agrees to
max(1e-10, 100 kappa(A~) u) relative, in norm and element by element, the
residual against A~ matches the oracle's, the matvec agrees to 1e-12
(norm, and component by component against the rounding bound of a product),
and the library's canonical flop counts equal the oracle's LU counts.
The forced LU variant on a symmetric kernel must reproduce the Cholesky
path's x.  The free build picks its own skeletons from the two-sided sample;
its structure must equal the oracle's and its ranks agree almost everywhere.
"""
import dataclasses

import numpy as np
import pytest

import workloads as W
from oracle import construct, flops, h2matrix, kernels, ulv_lu

pytestmark = pytest.mark.gpu


def _oracle(p, skeletons=None, gs_sweeps=0):
    return construct.construct(p.points, p.kernel, p.leaf, p.eta, p.eps, p.perm(), p.s_far,
                               p.s_near, skeletons=skeletons, gs_sweeps=gs_sweeps)


def _skeletons(h2):
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
    "drift2048_sampled": (lambda: W.yukawa_drift_cube(n=2048, leaf=64, eps=1e-6, beta=0.5, s=128), 2),
    "drift_ragged": (lambda: W.yukawa_drift_cube(n=3001, leaf=100, eps=1e-7, beta=0.8, s=150), 1),
    "drift_unsampled": (lambda: W.yukawa_drift_cube(n=1024, leaf=64, eps=1e-6, beta=0.5, s=-1), 3),
    "drift_hss": (lambda: W.yukawa_drift_cube(n=1024, leaf=64, eps=1e-6, beta=0.5, eta=0.0, s=-1), 1),
    # wide boxes: the redundant blocks span several 64-wide LU panels
    "drift_leaf256": (lambda: W.yukawa_drift_cube(n=4096, leaf=256, eps=1e-7, beta=0.5, s=256), 1),
    "drift_root_only": (lambda: W.yukawa_drift_cube(n=100, leaf=128, eps=1e-8, beta=0.5), 2),
}


def _same_h2(lib, p, nrhs, name, gs_sweeps=0):
    import torch
    print(f"[case {name}] n={p.n} leaf={p.leaf} eps={p.eps} eta={p.eta} "
          f"beta={p.kernel.beta} gs={gs_sweeps}", flush=True)
    h2o = _oracle(p, gs_sweeps=gs_sweeps)
    sk, ranks, pos = _skeletons(h2o)
    h2f = _oracle(p, skeletons=sk, gs_sweeps=gs_sweeps)
    fac = ulv_lu.factor(h2f)
    b = W.rhs(p.n, nrhs, 1)
    xo = ulv_lu.solve(fac, b)
    H = lib.build_fixed(p.points, p.kernel, p.leaf, p.eta, p.eps, p.perm(), ranks, pos,
                        s_far=p.s_far, s_near=p.s_near, gs_sweeps=gs_sweeps)
    assert H.stats()["lu_variant"] == 1
    perm, gr, gm, gsk = H.structure()
    assert np.array_equal(perm, h2o.tree.perm)
    assert np.array_equal(gr, ranks)
    H.factor()
    bt = torch.from_numpy(b).cuda()
    x = H.solve(bt).cpu().numpy()
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
    # the non-symmetric H^2 operator
    y = H.matvec(bt).cpu().numpy()
    yo = h2matrix.matvec(h2f, b)
    assert _rel(y, yo) < 1e-12, _rel(y, yo)
    cw = float(np.max(np.abs(y - yo) / (np.abs(At) @ np.abs(b))))
    assert cw < 1e-12, cw
    # the library's canonical LU flop counts against the oracle's
    st = H.stats()
    ff_o, fs_o = flops.count_h2_lu(h2f)
    assert abs(st["flops_factor"] - ff_o) <= 1e-12 * ff_o, (st["flops_factor"], ff_o)
    assert abs(st["flops_solve"] - fs_o) <= 1e-12 * fs_o, (st["flops_solve"], fs_o)
    H.close()
    return h2f


@pytest.mark.parametrize("name", list(CASES))
def test_same_h2_lu_matches_oracle(lib, name):
    factory, nrhs = CASES[name]
    _same_h2(lib, factory(), nrhs, name)


def test_same_h2_lu_gauss_seidel(lib):
    """The pre-factorization by Gauss-Seidel sweeps on both sides of the
    fill-in (A_cc and A_cc^T), the same sweeps on both sides."""
    p = W.yukawa_drift_cube(n=2048, leaf=64, eps=1e-6, beta=0.5, s=128)
    _same_h2(lib, p, 1, "drift_gs2", gs_sweeps=2)


def test_lu_refinement_matches_oracle(lib):
    """Stationary refinement to 1e-12 against A~ on both sides."""
    import torch
    p = W.yukawa_drift_cube(n=2048, leaf=64, eps=1e-5, beta=0.5, s=128)
    h2o = _oracle(p)
    sk, ranks, pos = _skeletons(h2o)
    h2f = _oracle(p, skeletons=sk)
    b = W.rhs(p.n, 2, 3)
    xo, hist = ulv_lu.refine(ulv_lu.factor(h2f), b, 1e-12, 30)
    assert hist[-1] <= 1e-12
    H = lib.build_fixed(p.points, p.kernel, p.leaf, p.eta, p.eps, p.perm(), ranks, pos,
                        s_far=p.s_far, s_near=p.s_near, ir_max_iter=30, ir_tol=1e-12)
    H.factor()
    x = H.solve(torch.from_numpy(b).cuda()).cpu().numpy()
    st = H.stats()
    print(f"[refine] gpu {st['ir_iters']} iterations residual {st['ir_residual']:.2e}; "
          f"oracle {len(hist) - 1} iterations", flush=True)
    assert H.last_solve_status == lib.OK
    assert st["ir_residual"] <= 1e-12
    At = h2matrix.assemble_dense(h2f)
    kappa = np.linalg.cond(At)
    # both solutions are within kappa times their residual of A~^{-1} b
    assert _rel(x, xo) < 2 * kappa * 1e-12 + 1e-13, _rel(x, xo)
    H.close()


def test_forced_lu_on_symmetric_kernel_matches_cholesky(lib):
    """The LU variant reduces to the Cholesky variant on a symmetric matrix:
    the same H^2 matrix factored both ways gives the same x."""
    import torch
    p = W.yukawa_cube(n=4096, leaf=64, eps=1e-7, s=128)
    h2o = _oracle(p)
    sk, ranks, pos = _skeletons(h2o)
    b = W.rhs(p.n, 2, 1)
    bt = torch.from_numpy(b).cuda()
    xs = {}
    for lu in (False, True):
        H = lib.build_fixed(p.points, p.kernel, p.leaf, p.eta, p.eps, p.perm(), ranks, pos,
                            s_far=p.s_far, s_near=p.s_near, factor_lu=lu)
        assert H.stats()["lu_variant"] == int(lu)
        H.factor()
        xs[lu] = H.solve(bt).cpu().numpy()
        H.close()
    h2f = _oracle(p, skeletons=sk)
    xo = ulv_lu.solve(ulv_lu.factor(h2f), b)
    kappa = np.linalg.cond(h2matrix.assemble_dense(h2f))
    tol = max(1e-10, 100 * kappa * np.finfo(float).eps)
    print(f"[forced lu] vs cholesky {_rel(xs[True], xs[False]):.2e}, vs oracle "
          f"{_rel(xs[True], xo):.2e} (tol {tol:.1e})", flush=True)
    assert _rel(xs[True], xs[False]) < tol
    assert _rel(xs[True], xo) < tol


def test_free_lu_build_end_to_end(lib):
    """The library's own two-sided construction (pivoted QR on the stacked
    row and column samples) against the oracle's free construction."""
    import torch
    p = W.yukawa_drift_cube(n=4096, leaf=64, eps=1e-7, beta=0.5, s=128)
    h2o = _oracle(p)
    H = lib.build(p.points, p.kernel, p.leaf, p.eta, p.eps, p.perm(), s_far=p.s_far,
                  s_near=p.s_near)
    perm, ranks, ms, skel = H.structure()
    assert np.array_equal(perm, h2o.tree.perm)
    o_ranks = np.array([bb.k for l in range(h2o.tree.L, 0, -1) for bb in h2o.basis[l]])
    print(f"[free lu] rank agreement {np.mean(ranks == o_ranks):.3f}, max diff "
          f"{np.max(np.abs(ranks - o_ranks))}", flush=True)
    assert np.mean(ranks == o_ranks) > 0.7
    assert np.max(np.abs(ranks - o_ranks)) <= 3
    H.factor()
    b = W.rhs(p.n, 1, 2)
    x = H.solve(torch.from_numpy(b).cuda()).cpu().numpy()
    A = kernels.dense(p.kernel, p.points)
    res_g = np.linalg.norm(b - A @ x) / np.linalg.norm(b)
    xo = ulv_lu.solve(ulv_lu.factor(h2o), b)
    res_o = np.linalg.norm(b - A @ xo) / np.linalg.norm(b)
    print(f"[free lu] residual vs dense: gpu {res_g:.2e} oracle {res_o:.2e}", flush=True)
    assert res_g <= max(10 * res_o, 1e-12), (res_g, res_o)
    H.close()


def test_lu_rejects_bf16_copies_and_pcg(lib):
    p = W.yukawa_drift_cube(n=512, leaf=64, eps=1e-6, beta=0.5)
    for kw in ({"solve_prec": lib.PREC_BF16}, {"matvec_prec": lib.PREC_FP32},
               {"use_pcg": True}):
        with pytest.raises(lib.H2Error) as ei:
            lib.build(p.points, p.kernel, p.leaf, p.eta, p.eps, p.perm(), **kw)
        assert ei.value.status == lib.ERR_ARG
    # beta = 0: the drift kernel is symmetric and takes the Cholesky path
    q = dataclasses.replace(p, kernel=dataclasses.replace(p.kernel, beta=0.0))
    H = lib.build(q.points, q.kernel, q.leaf, q.eta, q.eps, q.perm())
    assert H.stats()["lu_variant"] == 0
    H.close()


@pytest.mark.parametrize("gp,sp", [("fp32", "fp64"), ("bf16x3", "fp32")])
def test_lu_precision_split_against_oracle(lib, gp, sp):
    """The LU variant with reduced-precision transforms (FP32, or split BF16
    on the BF16 matrix cores) and FP64 or FP32 substitution copies, refined
    by stationary iterations against the FP64 H^2 operator on the oracle's
    H^2 matrix: the refined x meets 2 kappa(A~) max(res, res_o) of the
    oracle's refined x (both residuals against A~ at most 1.1e-10), and the
    iterations stay few (the preconditioner's error is that of its
    precision)."""
    import torch
    P = {"fp64": lib.PREC_FP64, "fp32": lib.PREC_FP32, "bf16x3": lib.PREC_BF16X3}
    p = W.yukawa_drift_cube(n=4096, leaf=128, eps=1e-8, beta=0.5, s=256)
    h2o = _oracle(p)
    sk, ranks, pos = _skeletons(h2o)
    h2f = _oracle(p, skeletons=sk)
    b = W.rhs(p.n, 2, 5)
    xo, hist = ulv_lu.refine(ulv_lu.factor(h2f), b, 1e-10, 30)
    At = h2matrix.assemble_dense(h2f)
    kappa = np.linalg.cond(At)
    res_o = np.linalg.norm(b - At @ xo, axis=0) / np.linalg.norm(b, axis=0)
    H = lib.build_fixed(p.points, p.kernel, p.leaf, p.eta, p.eps, p.perm(), ranks, pos,
                        s_far=p.s_far, s_near=p.s_near, gemm_prec=P[gp], solve_prec=P[sp],
                        ir_max_iter=30, ir_tol=1e-10)
    assert H.stats()["lu_variant"] == 1
    H.factor()
    x = H.solve(torch.from_numpy(b).cuda()).cpu().numpy()
    st = H.stats()
    res = np.linalg.norm(b - At @ x, axis=0) / np.linalg.norm(b, axis=0)
    print(f"[lu {gp} transforms, {sp} copies] {st['ir_iters']} steps (oracle FP64 "
          f"{len(hist) - 1}), residual {res.max():.2e}, x vs oracle {_rel(x, xo):.2e}", flush=True)
    assert H.last_solve_status == lib.OK
    assert st["ir_residual"] <= 1e-10 and res.max() <= 1.1e-10
    assert _rel(x, xo) <= 2 * kappa * max(res.max(), res_o.max())
    assert st["ir_iters"] <= 3 * max(len(hist) - 1, 1) + 4
    H.close()


def test_lu_batched_graph_and_noalloc(lib):
    """The LU variant through the other entry points: several non-symmetric
    instances in one handle, the factorization captured in a hipGraph, and
    the no-allocation solve.  Each batched instance has its own build's
    structure and agrees with its own build to rounding (1e-13 relative;
    measured 0 to 1e-15: the batched work lists may sum a few products in
    another order); the graph's replays are bitwise equal to its capture and
    agree with a plain handle to rounding; the no-allocation solve is bitwise
    equal to the plain solve on the same handle."""
    import torch
    ps = [W.yukawa_drift_cube(n=n, leaf=64, eps=1e-6, beta=bt, s=128)
          for n, bt in ((1500, 0.5), (2600, 0.8), (900, 0.3))]
    Hb = lib.build_batched([p.points for p in ps], [p.kernel for p in ps], 64, 1.0, 1e-6,
                           perms=[p.perm() for p in ps], s_far=128, s_near=128)
    assert Hb.stats()["lu_variant"] == 1
    perm_b, ranks_b, _, _ = Hb.structure()
    Hb.factor()
    bs = [W.rhs(p.n, 1, 7) for p in ps]
    bcat = torch.from_numpy(np.concatenate(bs, axis=0)).cuda()
    xb = Hb.solve(bcat).cpu().numpy()
    yb = Hb.matvec(bcat).cpu().numpy()
    off = 0
    nranks = 0
    for p, b in zip(ps, bs):
        H = lib.build(p.points, p.kernel, 64, 1.0, 1e-6, p.perm(), s_far=128, s_near=128)
        perm, ranks, _, _ = H.structure()
        assert np.array_equal(perm, perm_b[off:off + p.n])
        nranks += ranks.sum()
        H.factor()
        bt = torch.from_numpy(b).cuda()
        x = H.solve(bt).cpu().numpy()
        y = H.matvec(bt).cpu().numpy()
        dx = _rel(xb[off:off + p.n], x)
        dy = _rel(yb[off:off + p.n], y)
        A = kernels.dense(p.kernel, p.points)
        print(f"[lu batched] n={p.n} beta={p.kernel.beta} x vs own build {dx:.1e}, y {dy:.1e}, "
              f"residual vs dense {np.linalg.norm(b - A @ x) / np.linalg.norm(b):.2e}", flush=True)
        assert dx < 1e-13 and dy < 1e-13
        H.close()
        off += p.n
    assert nranks == ranks_b.sum()
    Hb.close()
    p = ps[1]
    b = torch.from_numpy(W.rhs(p.n, 2, 9)).cuda()
    Hp = lib.build(p.points, p.kernel, 64, 1.0, 1e-6, p.perm(), s_far=128, s_near=128)
    Hp.factor()
    x_plain = Hp.solve(b).cpu().numpy()
    cols_b = b.t().contiguous()
    cols_x = torch.empty_like(cols_b)
    assert Hp.solve_noalloc_into(cols_b, cols_x) == lib.OK
    torch.cuda.synchronize()
    assert np.array_equal(cols_x.t().cpu().numpy(), x_plain)
    Hp.close()
    Hg = lib.build(p.points, p.kernel, 64, 1.0, 1e-6, p.perm(), s_far=128, s_near=128,
                   use_graph=True)
    xg = []
    for _ in range(3):  # capture, then replays
        Hg.factor()
        xg.append(Hg.solve(b).cpu().numpy())
    assert np.array_equal(xg[0], xg[1]) and np.array_equal(xg[0], xg[2])
    assert _rel(xg[0], x_plain) < 1e-13
    Hg.close()
