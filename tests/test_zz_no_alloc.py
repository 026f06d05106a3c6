"""h2_solve_noalloc, the solve for callers that cannot allocate device memory,
against h2_solve through the C ABI: two calls in a row on one GPU, the second
with a smaller input (fewer points and fewer right-hand sides), so that the
second call runs on the fixed partials array that the first one left full.
Both entry points run the same kernels in the same order on the same data,
so their solutions agree bit for bit; the oracle is not needed here."""
import ctypes

import numpy as np
import pytest

import workloads as W

pytestmark = pytest.mark.gpu

NOALLOC_PARTIALS = 1 << 23  # H2_NOALLOC_PARTIALS in include/h2.h


def _solve_both(lib, H, b_np):
    """(x from h2_solve, x from h2_solve_noalloc, statuses) for (n, nrhs) b."""
    import torch
    L = lib.load()
    b = torch.from_numpy(np.ascontiguousarray(b_np.T)).cuda()  # (nrhs, n): column-major n x nrhs
    x_ref = torch.full_like(b, np.nan)
    x_na = torch.full_like(b, np.nan)
    st = lib._stream(None)
    s_ref = L.h2_solve(H._h, ctypes.c_void_p(b.data_ptr()), ctypes.c_void_p(x_ref.data_ptr()),
                       b.shape[0], H.n, st)
    s_na = L.h2_solve_noalloc(H._h, ctypes.c_void_p(b.data_ptr()),
                              ctypes.c_void_p(x_na.data_ptr()), b.shape[0], H.n, st)
    torch.cuda.synchronize()
    return x_ref.cpu().numpy(), x_na.cpu().numpy(), s_ref, s_na


def test_noalloc_solve_matches_solve_on_two_calls(lib):
    # first call: N = 4096, three right-hand sides, PCG refinement
    p1 = W.laplace_cube(n=4096, leaf=64, eps=1e-6, s=128)
    H1 = lib.build(p1.points, p1.kernel, p1.leaf, p1.eta, p1.eps, p1.perm(), s_far=p1.s_far,
                   s_near=p1.s_near, ir_max_iter=50, ir_tol=1e-10, use_pcg=True)
    H1.factor()
    st1 = H1.stats()
    print(f"[noalloc] N=4096 nrhs=3 partials/rhs={st1['gather_partials']}", flush=True)
    assert 0 < st1["gather_partials"] <= NOALLOC_PARTIALS
    b1 = W.rhs(p1.n, 3, seed=11)
    x_ref, x_na, s_ref, s_na = _solve_both(lib, H1, b1)
    assert s_ref == lib.OK and s_na == lib.OK
    assert np.all(np.isfinite(x_ref))
    assert np.array_equal(x_ref, x_na)

    # second call: N = 2048, one right-hand side, direct solve
    p2 = W.laplace_cube(n=2048, leaf=128, eps=1e-7, s=256)
    H2 = lib.build(p2.points, p2.kernel, p2.leaf, p2.eta, p2.eps, p2.perm(), s_far=p2.s_far,
                   s_near=p2.s_near)
    H2.factor()
    st2 = H2.stats()
    print(f"[noalloc] N=2048 nrhs=1 partials/rhs={st2['gather_partials']}", flush=True)
    assert 0 < st2["gather_partials"] <= NOALLOC_PARTIALS
    b2 = W.rhs(p2.n, 1, seed=12)
    x_ref2, x_na2, s_ref2, s_na2 = _solve_both(lib, H2, b2)
    assert s_ref2 == lib.OK and s_na2 == lib.OK
    assert np.all(np.isfinite(x_ref2))
    assert np.array_equal(x_ref2, x_na2)

    # and the larger handle again after the smaller one (b == x in place)
    import torch
    b = torch.from_numpy(np.ascontiguousarray(b1.T)).cuda()
    L = lib.load()
    assert L.h2_solve_noalloc(H1._h, ctypes.c_void_p(b.data_ptr()), ctypes.c_void_p(b.data_ptr()),
                              b.shape[0], H1.n, lib._stream(None)) == lib.OK
    torch.cuda.synchronize()
    assert np.array_equal(b.cpu().numpy(), x_ref)
    H1.close()
    H2.close()


def test_noalloc_argument_and_state_errors(lib):
    import torch
    L = lib.load()
    p = W.laplace_cube(n=2048, leaf=128, eps=1e-7, s=256)
    H = lib.build(p.points, p.kernel, p.leaf, p.eta, p.eps, p.perm(), s_far=p.s_far,
                  s_near=p.s_near)
    b = torch.zeros((1, p.n), dtype=torch.float64, device="cuda")
    x = torch.zeros_like(b)
    st = lib._stream(None)
    bp, xp = ctypes.c_void_p(b.data_ptr()), ctypes.c_void_p(x.data_ptr())
    assert L.h2_solve_noalloc(H._h, bp, xp, 1, H.n, st) == lib.ERR_STATE  # before factor
    H.factor()
    assert L.h2_solve_noalloc(H._h, bp, xp, 0, H.n, st) == lib.ERR_ARG
    assert L.h2_solve_noalloc(H._h, bp, xp, 1, H.n - 1, st) == lib.ERR_ARG
    assert L.h2_solve_noalloc(H._h, None, xp, 1, H.n, st) == lib.ERR_ARG
    assert L.h2_solve_noalloc(H._h, bp, xp, 1, H.n, st) == lib.OK
    torch.cuda.synchronize()
    assert float(x.abs().max()) == 0.0  # zero right-hand side, zero solution
    H.close()
