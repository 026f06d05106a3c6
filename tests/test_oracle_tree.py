"""Pins of the oracle's cluster tree and block lists against brute-force
invariants: a partition of the points, the halving sizes, symmetric lists,
an exact tiling of the N x N index set, and the admissibility definition."""
import itertools

import numpy as np
import pytest

import workloads as W
from oracle.tree import ClusterTree, num_levels


@pytest.mark.parametrize("n,leaf,dim", [(2048, 128, 3), (1000, 64, 3), (777, 50, 2), (64, 64, 3), (5, 2, 2)])
def test_partition_and_sizes(n, leaf, dim):
    X = W.cube_points(n, dim, 3)
    t = ClusterTree(X, leaf, 1.0)
    assert sorted(t.perm.tolist()) == list(range(n))
    assert t.L == num_levels(n, leaf)
    assert -(-n // (1 << t.L)) <= leaf and (t.L == 0 or -(-n // (1 << (t.L - 1))) > leaf)
    for l in range(t.L + 1):
        sizes = [e - s for (s, e) in t.ranges[l]]
        assert set(sizes) <= {n >> l, -(-n // (1 << l))}
        assert sum(sizes) == n
        # contiguous and ordered
        assert t.ranges[l][0][0] == 0 and t.ranges[l][-1][1] == n
        for a, b in zip(t.ranges[l], t.ranges[l][1:]):
            assert a[1] == b[0]


def test_split_is_median_on_longest_axis():
    X = W.cube_points(512, 3, 5) * np.array([1.0, 3.0, 0.5])  # y is the longest axis
    t = ClusterTree(X, 256, 1.0)
    left = X[t.perm[:256]]
    right = X[t.perm[256:]]
    assert left[:, 1].max() <= right[:, 1].min()


def _tiles(t):
    """Every (row point, col point) pair covered by a leaf near block or a far block."""
    n = t.n
    cover = np.zeros((n, n), dtype=np.int32)
    for (i, j) in t.near[t.L]:
        si, ei = t.ranges[t.L][i]
        sj, ej = t.ranges[t.L][j]
        cover[si:ei, sj:ej] += 1
    for l in range(1, t.L + 1):
        for (i, j) in t.far[l]:
            si, ei = t.ranges[l][i]
            sj, ej = t.ranges[l][j]
            cover[si:ei, sj:ej] += 1
    return cover


@pytest.mark.parametrize("eta", [0.0, 0.7, 1.0, 2.0])
def test_lists_symmetric_and_tile_exactly_once(eta):
    X = W.cube_points(1024, 3, 1)
    t = ClusterTree(X, 64, eta)
    for l in range(t.L + 1):
        assert set(t.near[l]) == {(j, i) for (i, j) in t.near[l]}
        assert set(t.far[l]) == {(j, i) for (i, j) in t.far[l]}
        assert not (set(t.near[l]) & set(t.far[l]))
        assert all((i, i) in set(t.near[l]) for i in range(1 << l))
    assert np.all(_tiles(t) == 1)


def test_eta_zero_is_hss():
    t = ClusterTree(W.cube_points(1024, 3, 2), 64, 0.0)
    for l in range(t.L + 1):
        assert sorted(t.near[l]) == [(i, i) for i in range(1 << l)]


def test_admissibility_brute_force():
    X = W.cube_points(2048, 3, 4)
    t = ClusterTree(X, 64, 1.0)
    for l in range(1, t.L + 1):
        nearset = set(t.near[l])
        farset = set(t.far[l])
        parent_near = set(t.near[l - 1])
        for a, b in itertools.product(range(1 << l), repeat=2):
            if (a // 2, b // 2) not in parent_near:
                assert (a, b) not in nearset and (a, b) not in farset
                continue
            Pa = X[t.perm[slice(*t.ranges[l][a])]]
            Pb = X[t.perm[slice(*t.ranges[l][b])]]
            ca = 0.5 * (Pa.max(0) + Pa.min(0))
            cb = 0.5 * (Pb.max(0) + Pb.min(0))
            ra = 0.5 * np.linalg.norm(Pa.max(0) - Pa.min(0))
            rb = 0.5 * np.linalg.norm(Pb.max(0) - Pb.min(0))
            is_far = a != b and np.linalg.norm(ca - cb) > 1.0 * (ra + rb)
            assert ((a, b) in farset) == is_far
            assert ((a, b) in nearset) == (not is_far)


def test_face_neighbours_stay_dense_at_eta_one():
    # A regular 16^3 lattice split into 4x4x4-point cubes: cubes sharing a
    # face must be near at eta = 1 (Section 3.3 / Figure 5).
    g = (np.arange(16) + 0.5) / 16
    X = np.array(list(itertools.product(g, g, g)))
    t = ClusterTree(X, 64, 1.0)
    L = t.L
    c = t.center[L]
    nearset = set(t.near[L])
    for a in range(1 << L):
        for b in range(1 << L):
            d = np.abs(c[a] - c[b])
            if np.isclose(d.sum(), 0.25) and np.count_nonzero(d > 1e-9) == 1:  # face neighbours
                assert (a, b) in nearset
