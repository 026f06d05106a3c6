"""Status paths of the C ABI, each forced from the host so that every kernel
still runs to completion: a Cholesky breakdown (H2_ERR_NOT_SPD with its
location), refinement that cannot reach its tolerance and a non-finite
residual (H2_ERR_NOCONV), allocation failures at chosen calls of the caller's
allocator (H2_ERR_ALLOC, with every buffer handed back), and a zero
right-hand-side column next to non-zero ones under PCG."""
import ctypes

import numpy as np
import pytest

import workloads as W
from oracle import construct, ulv

pytestmark = pytest.mark.gpu


def _skeletons(h2):
    ranks, pos = [], []
    for l in range(h2.tree.L, 0, -1):
        for bb in h2.basis[l]:
            ranks.append(bb.k)
            pos.extend(bb.piv[:bb.k].tolist())
    return np.array(ranks, dtype=np.int32), np.array(pos, dtype=np.int32)


def test_not_spd_reports_the_oracles_breakdown(lib):
    """Matern-3/2 with a 1e-4 nugget at eps = 1e-6 (the rank-predictor
    configuration's kernel, at N = 4096): the oracle's factorization breaks
    down at level 3, box 0 (smallest eigenvalue of the redundant block
    -8.7e-3 against a largest of 2.7, far from rounding).  The library, given
    the same skeletons, must stop there with H2_ERR_NOT_SPD and the same
    location, and then refuse to solve."""
    import torch
    p = W.matern_cube(n=4096, leaf=128, eps=1e-6, s=256)
    h2o = construct.construct(p.points, p.kernel, p.leaf, p.eta, p.eps, p.perm(), p.s_far,
                              p.s_near)
    with pytest.raises(ulv.NotSPD) as ei:
        ulv.factor(h2o)
    lvl, box = ei.value.level, ei.value.box
    ranks, pos = _skeletons(h2o)
    H = lib.build_fixed(p.points, p.kernel, p.leaf, p.eta, p.eps, p.perm(), ranks, pos,
                        s_far=p.s_far, s_near=p.s_near)
    print(f"[not_spd] oracle breakdown at level {lvl}, box {box}", flush=True)
    L = lib.load()
    assert L.h2_factor(H._h, lib._stream(None)) == lib.ERR_NOT_SPD
    st = H.stats()
    assert (st["fail_level"], st["fail_box"], st["fail_inst"]) == (lvl, box, 0)
    b = torch.from_numpy(p.b()).cuda().t().contiguous()
    x = torch.empty_like(b)
    assert H.solve_into(b, x) == lib.ERR_STATE
    assert L.h2_factor(H._h, lib._stream(None)) == lib.ERR_STATE
    H.close()


def test_noconv_and_non_finite_residual(lib):
    import torch
    p = W.laplace_cube(n=4096, leaf=64, eps=1e-5, s=128)
    H = lib.build(p.points, p.kernel, p.leaf, p.eta, p.eps, p.perm(), s_far=p.s_far,
                  s_near=p.s_near, ir_max_iter=1, ir_tol=1e-15)
    H.factor()
    b = torch.from_numpy(W.rhs(p.n, 2, 1)).cuda().t().contiguous()
    x = torch.empty_like(b)
    assert H.solve_into(b, x) == lib.ERR_NOCONV
    st = H.stats()
    assert st["ir_iters"] == 1 and 1e-15 < st["ir_residual"] < 1e-3
    assert bool(torch.isfinite(x).all())
    # a NaN in one column: the residual is not finite, which is reported as
    # non-convergence rather than as success
    H2 = lib.build(p.points, p.kernel, p.leaf, p.eta, p.eps, p.perm(), s_far=p.s_far,
                   s_near=p.s_near, ir_max_iter=5, ir_tol=1e-12)
    H2.factor()
    bn = b.clone()
    bn[1, 17] = float("nan")
    assert H2.solve_into(bn, x) == lib.ERR_NOCONV
    assert not np.isfinite(H2.stats()["ir_residual"])
    H.close()
    H2.close()


def test_pcg_with_a_zero_column(lib):
    import torch
    p = W.yukawa_cube(n=4096, leaf=64, eps=1e-6, s=128)
    H = lib.build(p.points, p.kernel, p.leaf, p.eta, p.eps, p.perm(), s_far=p.s_far,
                  s_near=p.s_near, ir_max_iter=30, ir_tol=1e-12, use_pcg=True)
    H.factor()
    b = W.rhs(p.n, 3, 1)
    b[:, 1] = 0.0
    x = H.solve(torch.from_numpy(b).cuda())
    assert H.last_solve_status == lib.OK
    xs = x.cpu().numpy()
    assert np.isfinite(xs).all()
    assert np.all(xs[:, 1] == 0.0)
    assert H.stats()["ir_residual"] <= 1e-12
    y = H.matvec(x).cpu().numpy()
    for c in (0, 2):
        assert np.linalg.norm(b[:, c] - y[:, c]) <= 2e-12 * np.linalg.norm(b[:, c])
    H.close()


@pytest.mark.parametrize("fail_at", [1, 2, 7, 40, 400])
def test_allocation_failure_releases_everything(lib, fail_at):
    import torch
    p = W.laplace_cube(n=4096, leaf=64, eps=1e-6, s=128)
    ref = lib.TorchAllocator()
    H = lib.build(p.points, p.kernel, p.leaf, p.eta, p.eps, p.perm(), s_far=p.s_far,
                  s_near=p.s_near, allocator=ref)
    total = ref.calls
    assert total > 400
    H.factor()
    x_ref = H.solve(torch.from_numpy(p.b()).cuda()).cpu().numpy()
    H.close()
    assert ref.live == 0
    al = lib.TorchAllocator(fail_at=fail_at)
    print(f"[alloc] failing call {fail_at} of {total}", flush=True)
    with pytest.raises(lib.H2Error) as ei:
        lib.build(p.points, p.kernel, p.leaf, p.eta, p.eps, p.perm(), s_far=p.s_far,
                  s_near=p.s_near, allocator=al)
    assert ei.value.status == lib.ERR_ALLOC
    assert al.live == 0 and al.calls == fail_at
    # the same allocator object keeps working once it stops failing
    H = lib.build(p.points, p.kernel, p.leaf, p.eta, p.eps, p.perm(), s_far=p.s_far,
                  s_near=p.s_near, allocator=al)
    H.factor()
    x = H.solve(torch.from_numpy(p.b()).cuda()).cpu().numpy()
    assert np.array_equal(x, x_ref)
    H.close()
    assert al.live == 0


def test_library_allocator_and_torch_allocator_agree(lib):
    """hipMalloc inside the library (allocator=None) and PyTorch's caching
    allocator give the same bits."""
    import torch
    p = W.yukawa_cube(n=3001, leaf=100, eps=1e-7, s=150)
    b = torch.from_numpy(p.b()).cuda()
    xs = []
    for al in (None, lib.TorchAllocator()):
        H = lib.build(p.points, p.kernel, p.leaf, p.eta, p.eps, p.perm(), s_far=p.s_far,
                      s_near=p.s_near, allocator=al)
        H.factor()
        xs.append(H.solve(b).cpu().numpy())
        H.close()
    assert np.array_equal(xs[0], xs[1])
