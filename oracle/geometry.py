"""Recursive domain partition and knot sets (Sec. 2.2, Sec. 2.5).

The domain D (an interval for d = 1, a rectangle for d = 2) is split
recursively into J subregions per level, levels m = 0..M.  Region (m, i)
is the i-th region at level m; its children are (m+1, J*i + j), j = 0..J-1,
so the digits of i in base J are the path j_1..j_m from the root.

Readings where the paper leaves the choice open (it fixes only that the
partition and knots are known, Sec. 2.2, and recommends equal-area splits and
equidistant knots, Sec. 2.5):
  * d = 2, J = 4: quadrant split at the midpoint 0.5*(a+b) of each side;
    child j = 2*[y >= ymid] + [x >= xmid] (points on a split line go to the
    upper child).
  * d = 1, J >= 2: split points t_j = a + ((b - a) * j) / J, j = 1..J-1;
    child = number of split points <= x.
  * J = 1: every region has one child equal to itself (test configuration).
  * default knots of an internal region: cell-centred equidistant grid,
    d = 2: g x g with g = sqrt(r), x_i = a + ((b - a) * (2i + 1)) / (2g),
    index iy*g + ix; d = 1: x_i = a + ((b - a) * (2i + 1)) / (2r).
  * the knots of level M are the observations of each leaf (Sec. 2.2).
"""
from __future__ import annotations

import math

import numpy as np


class Geometry:
    """Partition, knots and the leaf assignment of observation locations.

    Attributes
      d, M, J, r, lo, hi
      bounds[m]   (J^m, d, 2) region boxes
      knots[m]    (J^m, r, d) knot coordinates of internal levels m < M
      leaf        (n,) leaf index of each observation (original order)
      perm        (n,) observation indices sorted by (leaf, original index)
      offsets     (J^M + 1,) CSR offsets of the sorted observations per leaf
    """

    def __init__(self, locs, d, M, J, r, lo=None, hi=None, knots=None):
        locs = np.asarray(locs, dtype=np.float64).reshape(-1, d)
        self.d, self.M, self.J, self.r = d, M, J, r
        self.lo = np.zeros(d) if lo is None else np.asarray(lo, dtype=np.float64)
        self.hi = np.ones(d) if hi is None else np.asarray(hi, dtype=np.float64)
        if d == 2 and J not in (1, 4):
            raise ValueError("d = 2 supports J in {1, 4}")
        if d not in (1, 2):
            raise ValueError("d must be 1 or 2")
        if ((locs < self.lo) | (locs > self.hi)).any() or not np.isfinite(locs).all():
            raise ValueError("locations outside the domain box")
        self.bounds = [np.stack([self.lo, self.hi], axis=1)[None]]
        for m in range(M):
            self.bounds.append(self._split(self.bounds[-1]))
        self.knots = []
        for m in range(M):
            if knots is not None:
                kk = np.asarray(knots[m], dtype=np.float64).reshape(J ** m, r, d)
            else:
                kk = self._grid_knots(self.bounds[m])
            self.knots.append(kk)
        self.leaf = self.leaf_of(locs)
        self.perm = np.lexsort((np.arange(locs.shape[0]), self.leaf))
        counts = np.bincount(self.leaf, minlength=J ** M)
        self.offsets = np.concatenate([[0], np.cumsum(counts)])
        self.locs = locs

    # -- partition --------------------------------------------------------
    def _split(self, b):
        """Children boxes of every box in b (level-major, child-minor)."""
        J, d = self.J, self.d
        out = np.empty((b.shape[0] * J, d, 2))
        for i in range(b.shape[0]):
            for j in range(J):
                out[i * J + j] = self._child_box(b[i], j)
        return out

    def _child_box(self, box, j):
        J, d = self.J, self.d
        c = box.copy()
        if J == 1:
            return c
        if d == 2:
            bx, by = j & 1, j >> 1
            for ax, bit in ((0, bx), (1, by)):
                a, b = box[ax]
                mid = 0.5 * (a + b)
                c[ax] = (mid, b) if bit else (a, mid)
            return c
        a, b = box[0]
        t = [a] + [a + ((b - a) * k) / J for k in range(1, J)] + [b]
        c[0] = (t[j], t[j + 1])
        return c

    def _child_of(self, box, x):
        """Child index of point x inside box."""
        J, d = self.J, self.d
        if J == 1:
            return 0
        if d == 2:
            xm = 0.5 * (box[0, 0] + box[0, 1])
            ym = 0.5 * (box[1, 0] + box[1, 1])
            return 2 * int(x[1] >= ym) + int(x[0] >= xm)
        a, b = box[0]
        return sum(1 for k in range(1, J) if x[0] >= a + ((b - a) * k) / J)

    def leaf_of(self, pts):
        """Leaf (level-M region) index of every point, by descending the tree
        one level at a time (vectorised form of _child_of)."""
        pts = np.asarray(pts, dtype=np.float64).reshape(-1, self.d)
        i = np.zeros(pts.shape[0], dtype=np.int64)
        J, d = self.J, self.d
        for m in range(self.M):
            if J == 1:
                continue
            b = self.bounds[m][i]                      # (n, d, 2)
            if d == 2:
                xm = 0.5 * (b[:, 0, 0] + b[:, 0, 1])
                ym = 0.5 * (b[:, 1, 0] + b[:, 1, 1])
                ch = 2 * (pts[:, 1] >= ym).astype(np.int64) + (pts[:, 0] >= xm).astype(np.int64)
            else:
                a, bb = b[:, 0, 0], b[:, 0, 1]
                ch = np.zeros(pts.shape[0], dtype=np.int64)
                for k in range(1, J):
                    ch += (pts[:, 0] >= a + ((bb - a) * k) / J).astype(np.int64)
            i = i * J + ch
        return i

    def _grid_knots(self, boxes):
        r, d = self.r, self.d
        out = np.empty((boxes.shape[0], r, d))
        if r == 0:
            return out
        if d == 2:
            g = int(round(math.sqrt(r)))
            if g * g != r:
                raise ValueError("default 2-D knots need r to be a perfect square")
            for i, b in enumerate(boxes):
                for iy in range(g):
                    for ix in range(g):
                        out[i, iy * g + ix, 0] = b[0, 0] + ((b[0, 1] - b[0, 0]) * (2 * ix + 1)) / (2 * g)
                        out[i, iy * g + ix, 1] = b[1, 0] + ((b[1, 1] - b[1, 0]) * (2 * iy + 1)) / (2 * g)
        else:
            for i, b in enumerate(boxes):
                for k in range(r):
                    out[i, k, 0] = b[0, 0] + ((b[0, 1] - b[0, 0]) * (2 * k + 1)) / (2 * r)
        return out

    # -- helpers ----------------------------------------------------------
    def ancestors(self, m, i):
        """[a_0, ..., a_m]: index at level l of the level-l ancestor of (m, i)."""
        return [i // (self.J ** (m - l)) for l in range(m + 1)]

    def leaf_obs(self, i):
        """Indices (original order) of the observations in leaf i, sorted."""
        return self.perm[self.offsets[i]:self.offsets[i + 1]]

    def region_points(self, m, i):
        """Q_{(m,i)}: knots for m < M, observation locations for m = M."""
        if m < self.M:
            return self.knots[m][i]
        return self.locs[self.leaf_obs(i)]
