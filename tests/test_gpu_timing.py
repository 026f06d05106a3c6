"""The per-launch timing the measurements rest on (params.timing): every
gather launch is timed by its own dispatch's start and end events, the sums
are consistent with the solve's wall time, and the counts match the plan."""
import numpy as np
import pytest

import workloads as W

pytestmark = pytest.mark.gpu


def test_gather_launch_times_are_consistent(lib):
    import torch
    p = W.yukawa_cube(n=8192, leaf=64, eps=1e-6, s=128)
    H = lib.build(p.points, p.kernel, p.leaf, p.eta, p.eps, p.perm(), s_far=p.s_far,
                  s_near=p.s_near, timing=True, ir_max_iter=20, ir_tol=1e-10, use_pcg=True,
                  solve_prec=lib.PREC_BF16, matvec_prec=lib.PREC_FP32)
    H.factor()
    b = torch.from_numpy(W.rhs(p.n, 1, 1)).cuda()
    H.solve(b)
    st = H.stats()
    it = st["ir_iters"]
    print(f"[timing] iterations {it}, solve {st['t_solve']:.4f}s, gathers {st['t_gather']}, "
          f"launches {st['gather_launches']}, PCG products {st['t_gather_mv32']:.4f}s "
          f"({st['gather_launches_mv32']})", flush=True)
    assert it > 0
    # FP64 gathers (the FP64 operator's products and the bases' products),
    # BF16 chunks, reductions, and per PCG iteration one product on the FP32
    # copies of the near blocks and couplings
    assert all(n > 0 for n in st["gather_launches"])
    assert 1 <= st["gather_launches_mv32"] <= it + 1
    # every chunk launch has its reduction launch
    assert st["gather_launches"][2] == (st["gather_launches"][0] + st["gather_launches"][1]
                                        + st["gather_launches_mv32"])
    t = sum(st["t_gather"]) + st["t_gather_mv32"]
    assert all(x > 0 for x in st["t_gather"]) and st["t_gather_mv32"] > 0
    assert t < st["t_solve"], (t, st["t_solve"])
    assert all(x > 0 for x in st["bytes_gather"]) and st["bytes_gather_mv32"] > 0
    H.close()
