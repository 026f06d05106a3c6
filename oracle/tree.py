"""Binary cluster tree, box geometry and the near/far block lists.

The paper uses a binary tree whose box i has children 2i and 2i+1 (Algorithm 1
merge step, Algorithm 2 merge step) and loops over levels from the leaves to
level 1.  It does not state how points are split; this oracle reads it as a
median bisection along the longest axis of the box's bounding box.

Admissibility (Section 6.2): the admissibility number eta is the accepted
ratio of box radius to centre distance, eta = 0 gives HSS (weak
admissibility), and at eta = 1 boxes sharing a face stay dense (Section 3.3,
Figure 5).  Reading: a pair (a, b), a != b, is far (low-rank) iff
    ||c_a - c_b||_2 > eta * (rho_a + rho_b),
with c the bounding-box midpoint and rho half the bounding-box diagonal.
Only children of near pairs are tested (nested block cluster tree).
"""
from __future__ import annotations

import numpy as np


def num_levels(n: int, leaf: int) -> int:
    """Smallest L with ceil(n / 2^L) <= leaf."""
    L = 0
    while -(-n // (1 << L)) > leaf:
        L += 1
    return L


class ClusterTree:
    """Level l (0 = root, L = leaves) has 2^l boxes; box i covers the
    contiguous tree-order positions ranges[l][i] = (start, end).
    ``perm[t]`` is the original index of the point at tree position t."""

    def __init__(self, X: np.ndarray, leaf: int, eta: float):
        if leaf < 2:
            raise ValueError("leaf must be >= 2")
        n, d = X.shape
        self.n, self.dim, self.leaf, self.eta = n, d, leaf, eta
        self.L = num_levels(n, leaf)
        order = np.arange(n)
        self.ranges = [[(0, n)]]
        for l in range(self.L):
            nxt = []
            for (s, e) in self.ranges[l]:
                idx = order[s:e]
                P = X[idx]
                ext = P.max(axis=0) - P.min(axis=0)
                axis = int(np.argmax(ext))           # ties -> lowest axis
                o = np.argsort(P[:, axis], kind="stable")
                order[s:e] = idx[o]
                h = (e - s) // 2                      # left child takes floor(n/2)
                nxt.append((s, s + h))
                nxt.append((s + h, e))
            self.ranges.append(nxt)
        self.perm = order.copy()

        # Geometry of every box from all of its original points.
        self.center, self.radius, self.extent = [], [], []
        for l in range(self.L + 1):
            c = np.zeros((1 << l, d))
            r = np.zeros(1 << l)
            ex = np.zeros((1 << l, d))
            for i, (s, e) in enumerate(self.ranges[l]):
                P = X[self.perm[s:e]]
                mx, mn = P.max(axis=0), P.min(axis=0)
                c[i] = 0.5 * (mx + mn)
                diag = mx - mn
                ex[i] = diag
                r[i] = 0.5 * np.sqrt(np.sum(diag * diag))
            self.center.append(c)
            self.radius.append(r)
            self.extent.append(ex)

        # Near/far lists, ordered pairs (both (i,j) and (j,i) appear).
        self.near = [[(0, 0)]]
        self.far = [[]]
        for l in range(1, self.L + 1):
            near, far = [], []
            c, r = self.center[l], self.radius[l]
            for (I, J) in self.near[l - 1]:
                for a in (2 * I, 2 * I + 1):
                    for b in (2 * J, 2 * J + 1):
                        if a == b:
                            near.append((a, b))
                            continue
                        diff = c[a] - c[b]
                        dist = np.sqrt(np.sum(diff * diff))
                        if dist > eta * (r[a] + r[b]):
                            far.append((a, b))
                        else:
                            near.append((a, b))
            near.sort()
            far.sort()
            self.near.append(near)
            self.far.append(far)

    def nboxes(self, l: int) -> int:
        return 1 << l

    def near_of(self, l: int) -> list[list[int]]:
        """For each box i at level l, the sorted list of j with (i, j) near."""
        out = [[] for _ in range(1 << l)]
        for (i, j) in self.near[l]:
            out[i].append(j)
        return out

    def far_of(self, l: int) -> list[list[int]]:
        out = [[] for _ in range(1 << l)]
        for (i, j) in self.far[l]:
            out[i].append(j)
        return out
