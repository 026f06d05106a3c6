"""Captured solves (use_graph): the substitution and the H^2 products of an
untimed h2_solve are captured once per shape and replayed.  Every replay, with
eager work and synchronizations between them, must equal the eager solve on
the same handle bit for bit (h2_solve_noalloc never captures), for PCG on the
target-path precisions, several right-hand sides, and the LU variant's
stationary refinement."""
import numpy as np
import pytest

import workloads as W

pytestmark = pytest.mark.gpu


def _eager(lib, H, b):
    import torch
    cols_b = b.t().contiguous()
    cols_x = torch.empty_like(cols_b)
    assert H.solve_noalloc_into(cols_b, cols_x) == lib.OK
    torch.cuda.synchronize()
    return cols_x.t().cpu().numpy()


@pytest.mark.parametrize("case", ["pcg_mixed", "lu_stationary"])
def test_captured_solve_replays_equal_eager(lib, case):
    import torch
    if case == "pcg_mixed":
        p = W.yukawa_cube(n=8192, leaf=64, eps=1e-6, s=128)
        kw = dict(gemm_prec=lib.PREC_BF16X3, solve_prec=lib.PREC_BF16,
                  matvec_prec=lib.PREC_FP32, use_pcg=True)
    else:
        p = W.yukawa_drift_cube(n=4096, leaf=64, eps=1e-6, beta=0.5, s=128)
        kw = dict(gemm_prec=lib.PREC_BF16X3, solve_prec=lib.PREC_FP32)
    H = lib.build(p.points, p.kernel, p.leaf, p.eta, p.eps, p.perm(), s_far=p.s_far,
                  s_near=p.s_near, ir_max_iter=50, ir_tol=1e-10, use_graph=True, **kw)
    H.factor()
    for nrhs in (1, 3):
        b = torch.from_numpy(W.rhs(p.n, nrhs, 11)).cuda()
        x_eager = _eager(lib, H, b)
        for rep in range(3):
            x = H.solve(b).cpu().numpy()
            assert H.last_solve_status == lib.OK
            st = H.stats()
            print(f"[{case}] nrhs={nrhs} replay {rep}: {st['ir_iters']} iterations, residual "
                  f"{st['ir_residual']:.2e}", flush=True)
            assert st["ir_residual"] <= 1e-10
            assert np.array_equal(x, x_eager)
            # eager work between the replays
            y = H.matvec(b)
            torch.cuda.synchronize()
            assert bool(torch.isfinite(y).all())
    H.close()
