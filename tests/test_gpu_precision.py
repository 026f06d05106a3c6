"""Precision split: basis-transform and Schur-update GEMMs in FP32 or BF16
(FP32 accumulation) with FP64 Cholesky factors, FP64 root and an FP64 H^2
matvec for refinement.  The refined solution must reach the FP64 tolerance and
agree with the plain FP64 path; the unrefined error is reported per precision
and must stay within what the GEMM precision allows."""
import numpy as np
import pytest

import workloads as W

pytestmark = pytest.mark.gpu


# Unrefined bounds: the inputs of every transform are rounded to the GEMM
# precision (unit roundoff 6e-8 for FP32, 3.9e-3 for BF16) and the error is
# amplified by the conditioning of the regularised Yukawa matrix (diagonal
# 1/delta = 1e3 against off-diagonal entries of order 1).  Measured: FP32
# 5.2e-4, BF16 below 0.5.  The real claim is the refined result.
@pytest.mark.parametrize("prec,unrefined_max", [(1, 5e-3), (2, 5e-1)])
def test_mixed_precision_refines_to_fp64(lib, prec, unrefined_max):
    import torch
    p = W.yukawa_cube(n=16384, leaf=128, eps=1e-8, nrhs=4, s=256)
    b = torch.from_numpy(p.b()).cuda()
    H64 = lib.build(p.points, p.kernel, p.leaf, p.eta, p.eps, p.perm(), s_far=p.s_far,
                    s_near=p.s_near, ir_max_iter=30, ir_tol=1e-10)
    H64.factor()
    x64 = H64.solve(b)
    assert H64.stats()["ir_residual"] <= 1e-10
    Hd = lib.build(p.points, p.kernel, p.leaf, p.eta, p.eps, p.perm(), s_far=p.s_far,
                   s_near=p.s_near, gemm_prec=prec)
    Hd.factor()
    xd = Hd.solve(b)
    err_direct = float(torch.linalg.norm(xd - x64) / torch.linalg.norm(x64))
    print(f"[prec {prec}] unrefined rel. error vs FP64 refined: {err_direct:.2e}")
    assert err_direct < unrefined_max
    Hm = lib.build(p.points, p.kernel, p.leaf, p.eta, p.eps, p.perm(), s_far=p.s_far,
                   s_near=p.s_near, gemm_prec=prec, ir_max_iter=60, ir_tol=1e-10)
    Hm.factor()
    xm = Hm.solve(b)
    st = Hm.stats()
    print(f"[prec {prec}] refinement steps {st['ir_iters']}, residual {st['ir_residual']:.2e}")
    assert st["ir_residual"] <= 1e-10
    r = b - H64.matvec(xm)
    assert float(torch.linalg.norm(r) / torch.linalg.norm(b)) <= 2e-10
    assert float(torch.linalg.norm(xm - x64) / torch.linalg.norm(x64)) < 1e-8
    for H in (H64, Hd, Hm):
        H.close()


def test_fp32_substitution_copies_refine_to_fp64(lib):
    """The substitution reading FP32 copies of the transformed blocks and bases
    is still a fixed symmetric preconditioner: PCG against the FP64 H^2
    operator reaches the FP64 tolerance and the FP64 path's solution."""
    import torch
    p = W.yukawa_cube(n=16384, leaf=128, eps=1e-8, nrhs=4, s=256)
    b = torch.from_numpy(p.b()).cuda()
    kw = dict(s_far=p.s_far, s_near=p.s_near, ir_max_iter=60, ir_tol=1e-10, use_pcg=True)
    H64 = lib.build(p.points, p.kernel, p.leaf, p.eta, p.eps, p.perm(), **kw)
    H64.factor()
    x64 = H64.solve(b)
    H32 = lib.build(p.points, p.kernel, p.leaf, p.eta, p.eps, p.perm(), solve_prec=lib.PREC_FP32,
                    **kw)
    H32.factor()
    x32 = H32.solve(b)
    st64, st32 = H64.stats(), H32.stats()
    print(f"[solve fp32] iterations {st32['ir_iters']} (fp64 {st64['ir_iters']}), "
          f"residual {st32['ir_residual']:.2e}")
    assert st32["ir_residual"] <= 1e-10
    r = b - H64.matvec(x32)
    assert float(torch.linalg.norm(r) / torch.linalg.norm(b)) <= 2e-10
    assert float(torch.linalg.norm(x32 - x64) / torch.linalg.norm(x64)) < 1e-8
    assert st32["ir_iters"] <= st64["ir_iters"] + 2
    H64.close()
    H32.close()
