"""The library's host-side cluster tree, admissibility lists and sample
selection (csrc/tree.cpp) against the oracle's (oracle/tree.py; the sampling
rule of Algorithm 1 as oracle/construct.py applies it) on the CPU, bit for
bit: permutation, box ranges, box centres, extents and radii, the near and
far lists of every level, and the far and near samples of every box.  Point
sets: the workloads' cube and sphere, 1-D and 2-D sets, and degenerate ones
(duplicated coordinates, a set of identical points, sizes at the leaf size),
at admissibility 0 (HSS), 0.5, 1 and 2, built on one and on several threads
(boxes of 2^16 points and more sort in parallel runs).  The tree source is
compiled with the flags the library uses for it, into a helper loaded
through ctypes."""
import ctypes
import os
import shutil
import subprocess

import numpy as np
import pytest

from oracle import construct as oc
from oracle import tree as ot

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = [os.path.join(ROOT, "tests", "host", "tree_check.cpp"),
       os.path.join(ROOT, "paper_2502_02395_amd", "csrc", "tree.cpp")]

i64p = ctypes.POINTER(ctypes.c_int64)
i32p = ctypes.POINTER(ctypes.c_int32)
f64p = ctypes.POINTER(ctypes.c_double)


@pytest.fixture(scope="module")
def tc(tmp_path_factory):
    if shutil.which("g++") is None:
        pytest.skip("needs g++")
    so = str(tmp_path_factory.mktemp("tree") / "libtree_check.so")
    # the flags the library builds csrc/tree.cpp with
    r = subprocess.run(["g++", "-O2", "-std=c++17", "-fPIC", "-ffp-contract=off", "-pthread",
                        "-shared"] + SRC + ["-o", so], capture_output=True, text=True, timeout=300)
    assert r.returncode == 0, r.stderr[-3000:]
    lib = ctypes.CDLL(so)
    lib.tc_build.argtypes = [f64p, ctypes.c_int64, ctypes.c_int, ctypes.c_int, ctypes.c_double,
                             ctypes.c_int]
    lib.tc_build.restype = ctypes.c_int
    lib.tc_perm.argtypes = [i64p]
    lib.tc_level.argtypes = [ctypes.c_int, i64p, f64p, f64p, f64p]
    lib.tc_npairs.argtypes = [ctypes.c_int, ctypes.c_int]
    lib.tc_npairs.restype = ctypes.c_int64
    lib.tc_pairs.argtypes = [ctypes.c_int, ctypes.c_int, i32p]
    lib.tc_sample.argtypes = [ctypes.c_int, i64p, i64p, i32p, i64p, i64p, ctypes.c_int64,
                              ctypes.c_int, ctypes.c_int, ctypes.c_int]
    lib.tc_sample_size.argtypes = [ctypes.c_int, ctypes.c_int]
    lib.tc_sample_size.restype = ctypes.c_int64
    lib.tc_sample_get.argtypes = [ctypes.c_int, ctypes.c_int, i64p]
    return lib


def _p(a, t):
    return a.ctypes.data_as(t)


def _points(kind, n, rng):
    if kind == "cube":
        return rng.random((n, 3))
    if kind == "sphere":
        v = rng.standard_normal((n, 3))
        return v / np.linalg.norm(v, axis=1, keepdims=True)
    if kind == "plane":
        return rng.random((n, 2))
    if kind == "line":
        return rng.random((n, 1))
    if kind == "grid_dups":       # coarse grid: many equal coordinates and equal points
        return rng.integers(0, 5, size=(n, 3)).astype(np.float64) * 0.25
    if kind == "identical":
        return np.full((n, 3), 0.5)
    if kind == "flat_slab":       # one axis constant, the others tied in extent
        P = rng.random((n, 3))
        P[:, 2] = 0.0
        P[:, 1] = P[:, 0]
        return P
    raise ValueError(kind)


CASES = [
    ("cube", 3000, 64, 1.0),
    ("cube", 2048, 32, 0.0),
    ("cube", 1500, 100, 2.0),
    ("sphere", 4096, 128, 1.0),
    ("sphere", 1000, 16, 0.5),
    ("plane", 2500, 50, 1.0),
    ("line", 777, 20, 1.0),
    ("grid_dups", 3000, 40, 1.0),
    ("identical", 300, 16, 1.0),
    ("flat_slab", 1200, 30, 1.0),
    ("cube", 64, 64, 1.0),        # n = leaf: the root is the only box
    ("cube", 65, 64, 1.0),        # one split
    ("cube", 2, 2, 1.0),
    # boxes of 2^16 points and more: their keys are sorted in parallel runs
    # and merged (with ties in grid_dups)
    ("cube", 131072, 2048, 1.0),
    ("grid_dups", 131072, 4096, 1.0),
]


@pytest.mark.parametrize("threads", [1, 3, 5])
@pytest.mark.parametrize("kind,n,leaf,eta", CASES,
                         ids=[f"{c[0]}-{c[1]}-leaf{c[2]}-eta{c[3]}" for c in CASES])
def test_tree_and_lists_equal_the_oracle(tc, kind, n, leaf, eta, threads):
    rng = np.random.default_rng(n * 31 + leaf)
    X = np.ascontiguousarray(_points(kind, n, rng))
    dim = X.shape[1]
    o = ot.ClusterTree(X, leaf, eta)
    L = tc.tc_build(_p(X, f64p), n, dim, leaf, eta, threads)
    assert L == o.L
    perm = np.empty(n, np.int64)
    tc.tc_perm(_p(perm, i64p))
    assert np.array_equal(perm, o.perm)
    for l in range(L + 1):
        nb = 1 << l
        st = np.empty(nb + 1, np.int64)
        c = np.empty((nb, dim))
        ex = np.empty((nb, dim))
        r = np.empty(nb)
        tc.tc_level(l, _p(st, i64p), _p(c, f64p), _p(ex, f64p), _p(r, f64p))
        assert np.array_equal(st[:-1], [s for s, _ in o.ranges[l]]) and st[-1] == n
        assert np.array_equal(st[1:], [e for _, e in o.ranges[l]])
        # geometry bit for bit (same operations in the same order)
        assert np.array_equal(c, o.center[l]), l
        assert np.array_equal(ex, o.extent[l]), l
        assert np.array_equal(r, o.radius[l]), l
        for far, ref in ((0, o.near[l]), (1, o.far[l])):
            m = tc.tc_npairs(l, far)
            pr = np.empty((m, 2), np.int32)
            if m:
                tc.tc_pairs(l, far, _p(pr, i32p))
            assert [tuple(map(int, x)) for x in pr] == [tuple(x) for x in ref], (l, far)
    # every ordered pair of boxes is covered once at the finest level where
    # its ancestors were near (a partition of the matrix)
    if L <= 6 and n <= 8192:
        cover = np.zeros((n, n), np.int32)
        pos = np.empty(n, np.int64)
        pos[o.perm] = np.arange(n)
        for l in range(L + 1):
            blocks = list(o.far[l]) + (list(o.near[l]) if l == L else [])
            for (i, j) in blocks:
                (a0, a1), (b0, b1) = o.ranges[l][i], o.ranges[l][j]
                cover[a0:a1, b0:b1] += 1
        assert (cover == 1).all()


@pytest.mark.parametrize("s_far,s_near", [(-1, -1), (0, 0), (7, 3), (64, 16), (10 ** 6, 10 ** 6)])
def test_samples_equal_the_oracle(tc, s_far, s_near):
    """At each level, active sets as the construction would have them (random
    subsets of each box's points standing in for the children's skeletons);
    samples by the oracle's rule: the first s points in pi order among the
    non-near boxes' (far) and the other near boxes' (near) active points."""
    rng = np.random.default_rng(5)
    n, leaf, eta = 4096, 64, 1.0
    X = np.ascontiguousarray(rng.random((n, 3)))
    o = ot.ClusterTree(X, leaf, eta)
    id_base = 1000       # ids offset as in a batched handle
    pi = rng.permutation(n)
    rank = np.empty(n, np.int64)
    rank[pi] = np.arange(n)
    for l in range(1, o.L + 1):
        nb = 1 << l
        B = []
        for (s, e) in o.ranges[l]:
            pts = o.perm[s:e]
            keep = rng.random(pts.size) < (1.0 if l == o.L else 0.4)
            B.append(rng.permutation(pts[keep]))
        near = o.near_of(l)
        ids = np.concatenate(B).astype(np.int64) + id_base
        ids_off = np.concatenate([[0], np.cumsum([b.size for b in B])]).astype(np.int64)
        nflat = np.concatenate([np.asarray(x, np.int32) for x in near])
        near_off = np.concatenate([[0], np.cumsum([len(x) for x in near])]).astype(np.int64)
        tc.tc_sample(nb, _p(ids, i64p), _p(ids_off, i64p), _p(nflat, i32p), _p(near_off, i64p),
                     _p(rank, i64p), id_base, s_far, s_near, 3)
        for i in range(nb):
            nset = set(near[i])
            far_c = [B[j] for j in range(nb) if j not in nset]
            near_c = [B[j] for j in near[i] if j != i]
            F = np.concatenate(far_c) if far_c else np.zeros(0, np.int64)
            C = np.concatenate(near_c) if near_c else np.zeros(0, np.int64)
            for which, cands, cnt in ((0, F, s_far), (1, C, s_near)):
                want = oc._sample(cands.astype(np.int64), rank, cnt) + id_base
                m = tc.tc_sample_size(i, which)
                got = np.empty(m, np.int64)
                if m:
                    tc.tc_sample_get(i, which, _p(got, i64p))
                assert np.array_equal(got, want), (l, i, which)
