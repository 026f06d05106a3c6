"""The single-node studies' counts against the oracle's tree and counts:
the pre-factorization and factorization flops vs the admissibility eta
(Section 6.2, Fig. 17; HSS at eta = 0 has no near field, so no
pre-factorization) and the fixed-rank construction of the HSS / H^2
comparison (Section 6.3, Figs. 18-19: no far sampling, every rank at the cap
unless the block is smaller)."""
import numpy as np
import pytest

import workloads as W
from oracle import construct, flops

pytestmark = pytest.mark.gpu


def _skeletons(h2o):
    ranks, pos = [], []
    for l in range(h2o.tree.L, 0, -1):
        for bb in h2o.basis[l]:
            ranks.append(bb.k)
            pos.extend(bb.piv[:bb.k].tolist())
    return np.array(ranks, dtype=np.int32), np.array(pos, dtype=np.int32)


@pytest.mark.parametrize("eta,sweeps", [(0.0, 0), (0.5, 0), (1.0, 0), (1.0, 2), (2.0, 0)])
def test_eta_study_counts_match_oracle(lib, eta, sweeps):
    p = W.laplace_sphere(n=2048, leaf=64, eps=1e-6, eta=eta, nrhs=1, s=96)
    print(f"[eta study] n={p.n} leaf={p.leaf} eta={eta} sweeps={sweeps}", flush=True)
    h2o = construct.construct(p.points, p.kernel, p.leaf, p.eta, p.eps, p.perm(), p.s_far,
                              p.s_near, gs_sweeps=sweeps)
    ranks, pos = _skeletons(h2o)
    H = lib.build_fixed(p.points, p.kernel, p.leaf, p.eta, p.eps, p.perm(), ranks, pos,
                        s_far=p.s_far, s_near=p.s_near, gs_sweeps=sweeps)
    st = H.stats()
    H.close()
    t = h2o.tree
    assert st["near_pairs"] == sum(1 for l in range(1, t.L + 1) for (i, j) in t.near[l] if i >= j)
    assert st["far_pairs"] == sum(1 for l in range(1, t.L + 1) for (i, j) in t.far[l] if i > j)
    assert st["leaf_near_blocks"] == len(t.near[t.L])
    ff_o, _ = flops.count_h2(h2o)
    pre_o = flops.count_prefactor(h2o, sweeps)
    assert abs(st["flops_factor"] - ff_o) <= 1e-12 * ff_o
    assert abs(st["flops_prefactor"] - pre_o) <= 1e-12 * max(pre_o, 1.0)
    if eta == 0.0:
        assert pre_o == 0.0          # weak admissibility: no near boxes to sample
    else:
        assert pre_o > 0.0
    print(f"[eta study] eta={eta}: prefactor share "
          f"{pre_o / (pre_o + ff_o):.3f} (oracle count), near pairs {st['near_pairs']}",
          flush=True)


@pytest.mark.parametrize("eta", [0.0, 1.0])
def test_fixed_rank_construction_matches_oracle(lib, eta):
    """max_rank with eps = 0 and every far point: each rank is
    min(max_rank, m, samples), the same on both sides."""
    p = W.laplace_sphere(n=2048, leaf=128, eps=0.0, eta=eta, nrhs=1, s=-1)
    r = 24
    print(f"[fixed rank] n={p.n} leaf=128 eta={eta} rank={r}", flush=True)
    h2o = construct.construct(p.points, p.kernel, p.leaf, p.eta, 0.0, p.perm(), -1, 512,
                              max_rank=r)
    H = lib.build(p.points, p.kernel, p.leaf, p.eta, 0.0, p.perm(), s_far=-1, s_near=512,
                  max_rank=r)
    _, ranks, ms, _ = H.structure()
    st = H.stats()
    H.close()
    ro, mo = _skeletons(h2o)[0], []
    for l in range(h2o.tree.L, 0, -1):
        mo.extend(bb.m for bb in h2o.basis[l])
    assert np.array_equal(ranks, ro)
    assert np.array_equal(ms, np.array(mo))
    assert ranks.max() == r
    assert st["root_n"] == len(h2o.root_B)
