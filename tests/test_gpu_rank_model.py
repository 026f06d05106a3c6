"""The learned rank predictor end to end: trained on the device by the
library's own kernels on ranks from plain builds of smaller seeded problems,
then used to size the basis buffers of a build of a held-out problem.

A/B against the plain build: the decompositions themselves are unchanged
(same ranks, same skeletons, bitwise-identical solution), the basis memory
shrinks, and the fallbacks stay rare."""
import numpy as np
import pytest

import workloads as W

pytestmark = pytest.mark.gpu


def _problem(seed, n=8192):
    p = W.yukawa_cube(n=n, leaf=128, eps=1e-6, nrhs=1, s=256)
    p.points = W.cube_points(n, 3, seed)
    return p


def test_predictor_sizes_buffers_without_changing_results(lib):
    import torch
    from paper_2502_02395_amd import rank_model
    X, y = rank_model.collect([_problem(s) for s in (100, 101, 102)])
    w, hist = rank_model.train(X, y, steps=1500, lr=3e-3)
    assert hist[-1] < 0.1 * hist[0]
    p = _problem(200)
    b = torch.from_numpy(p.b()).cuda()
    Hp = lib.build(p.points, p.kernel, p.leaf, p.eta, p.eps, p.perm(), s_far=p.s_far,
                   s_near=p.s_near)
    Hm = lib.build(p.points, p.kernel, p.leaf, p.eta, p.eps, p.perm(), s_far=p.s_far,
                   s_near=p.s_near, rank_model=w, rank_margin=0.25)
    _, rp, mp, skp = Hp.structure()
    _, rm, mm, skm = Hm.structure()
    assert np.array_equal(rp, rm) and np.array_equal(skp, skm)
    sp, sm = Hp.stats(), Hm.stats()
    nbox = len(rp)
    assert sm["rank_fallbacks"] <= 0.05 * nbox + 1
    assert sm["bytes_basis"] < sp["bytes_basis"]
    Hp.factor()
    Hm.factor()
    assert np.array_equal(Hp.solve(b).cpu().numpy(), Hm.solve(b).cpu().numpy())
    Hp.close()
    Hm.close()


def test_forced_fallback_with_a_useless_model(lib):
    import torch
    p = _problem(201, n=4096)
    w = np.zeros(4801, dtype=np.float32)          # predicts rank 0 everywhere
    Hp = lib.build(p.points, p.kernel, p.leaf, p.eta, p.eps, p.perm(), s_far=p.s_far,
                   s_near=p.s_near)
    Hm = lib.build(p.points, p.kernel, p.leaf, p.eta, p.eps, p.perm(), s_far=p.s_far,
                   s_near=p.s_near, rank_model=w, rank_margin=0.0)
    _, rp, _, _ = Hp.structure()
    _, rm, _, _ = Hm.structure()
    assert np.array_equal(rp, rm)
    assert Hm.stats()["rank_fallbacks"] == int(np.sum(rp > 4))
    b = torch.from_numpy(p.b()).cuda()
    Hp.factor()
    Hm.factor()
    assert np.array_equal(Hp.solve(b).cpu().numpy(), Hm.solve(b).cpu().numpy())
    Hp.close()
    Hm.close()
