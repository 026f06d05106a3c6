"""The measured configuration at full size: Yukawa cube, N = 2^20, leaf 256,
eps 1e-6, 512-point samples, FP32 transforms with FP32 copies for the
substitution, PCG against the FP64 H^2 operator to 1e-8 (the launch
configuration bench.py times, without the rank predictor).

The oracle cannot build an H^2 matrix of this size, so the checks are the
ones that hold at any size plus rows the oracle computes one by one:
  * PCG reaches the 1e-8 relative residual against the FP64 H^2 operator, and
    the library's H^2 matvec confirms it;
  * on 32 seeded rows, the H^2 matvec agrees with the dense kernel matrix
    (oracle kernel evaluation, FP64) to the compression accuracy, and so does
    the solution's residual b_i - (A x)_i.
Bounds: the row ID keeps pivots above eps |R_00| = 1e-6 of each sampled
block, so every far-field block is represented to about 1e-6 of its own size;
summed over the far field of a row and measured against sum_j |A_ij x_j|
that stays below 1e-5 (observed values are printed).  A solution with a
1e-8 residual against A~ then has a dense residual of the same order."""
import numpy as np
import pytest

import workloads as W
from oracle import kernels

pytestmark = pytest.mark.gpu


def test_fullsize_measured_configuration(lib):
    import torch
    p = W.yukawa_cube(n=1 << 20, leaf=256, eps=1e-6, nrhs=1, s=512)
    print(f"[case fullsize] n={p.n} leaf={p.leaf} eps={p.eps} s={p.s_far}", flush=True)
    H = lib.build(p.points, p.kernel, p.leaf, p.eta, p.eps, p.perm(), s_far=p.s_far,
                  s_near=p.s_near, gemm_prec=lib.PREC_FP32, solve_prec=lib.PREC_FP32,
                  ir_max_iter=100, ir_tol=1e-8, use_pcg=True)
    H.factor()
    bnp = p.b()
    b = torch.from_numpy(bnp).cuda()
    x = H.solve(b)
    st = H.stats()
    print(f"[fullsize] PCG iterations {st['ir_iters']}, residual {st['ir_residual']:.2e}", flush=True)
    assert st["ir_residual"] <= 1e-8
    y = H.matvec(x)
    rel = float(torch.linalg.norm(b - y) / torch.linalg.norm(b))
    assert rel <= 1.01e-8
    xs = x.cpu().numpy()[:, 0]
    ys = y.cpu().numpy()[:, 0]
    rows = np.random.default_rng(7).choice(p.n, size=32, replace=False)
    A = kernels.evaluate(p.kernel, p.points[rows], p.points, rows, np.arange(p.n))
    ax = A @ xs
    scale = np.abs(A) @ np.abs(xs)
    err_mv = np.max(np.abs(ys[rows] - ax) / scale)
    err_res = np.max(np.abs(bnp[rows, 0] - ax) / scale)
    print(f"[fullsize] sampled rows: H^2 matvec vs dense {err_mv:.2e}, dense residual {err_res:.2e}",
          flush=True)
    assert err_mv <= 1e-5
    assert err_res <= 1e-5
    H.close()
