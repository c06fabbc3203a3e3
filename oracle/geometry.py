"""Recursive domain partition and knot sets (Sec. 2.2, Sec. 2.5).

The domain D (an interval for d = 1, a rectangle for d = 2) is split
recursively, levels m = 0..M.  Every region of level m - 1 has J_m children
(Sec. 2.2 writes one J for all levels; the satellite application of Sec. 4.2
uses J_m = (2, 2, 4, 8, 8, 16)), and every region of level m < M holds r_m
knots.  Region (m, i) is the i-th region at level m; its children are
(m+1, J_{m+1} i + j), j = 0..J_{m+1}-1.

Readings where the paper leaves the choice open (it fixes only that the
partition and knots are known, Sec. 2.2, recommends equal-area splits and
equidistant knots for roughly uniform data and other partitions for
far-from-uniform data, Sec. 2.5):
  * a split into J children is a grid of g_x x g_y cells: d = 1: g_x = J;
    d = 2: J = 1, 2, 4, 8, 16 as 1x1, 2x1, 2x2, 4x2, 4x4 with the larger
    count on the longer side of the box (x when the sides are equal);
  * the box is first cut along y into g_y slabs, then every slab along x
    into g_x cells; child j = iy * g_x + ix, where iy counts the y split
    values <= y and ix the slab's x split values <= x (points on a split
    line go to the upper child);
  * equal-area split values: a + ((b - a) * k) / g, k = 1..g-1, except
    0.5 * (a + b) for two-way splits in d = 2;
  * data-adaptive splits (Sec. 2.5's "more complicated partitioning
    schemes" for non-uniform data): the split values are quantiles of the
    observation locations in the region (the y values of the region, then
    the x values of each slab): t_k = 0.5 * (v[i - 1] + v[i]) with v the
    sorted values and i = (k * len(v)) // g; a region (or slab) with fewer
    than g observations is split into equal parts;
  * default knots of a region of level m: cell-centred equidistant grid,
    d = 2: g x g with g = sqrt(r_m), x_i = a + ((b - a) * (2i + 1)) / (2g),
    index iy*g + ix; d = 1: x_i = a + ((b - a) * (2i + 1)) / (2 r_m);
  * the knots of level M are the observations of each leaf (Sec. 2.2).
"""
from __future__ import annotations

import math

import numpy as np


def grid_shape(d, J, box):
    """(g_x, g_y) of a split of `box` ((d, 2) bounds) into J children."""
    if d == 1:
        return J, 1
    if J in (1, 4, 16):
        g = int(round(math.sqrt(J)))
        return g, g
    if J in (2, 8):
        hi, lo = (2, 1) if J == 2 else (4, 2)
        wide = (box[0, 1] - box[0, 0]) >= (box[1, 1] - box[1, 0])
        return (hi, lo) if wide else (lo, hi)
    raise ValueError("d = 2 supports J in {1, 2, 4, 8, 16}")


def split_values(a, b, g, d, vals=None):
    """Split values of [a, b] into g parts: equal-area, or quantiles of vals."""
    if g <= 1:
        return []
    if vals is not None and len(vals) >= g:
        v = np.sort(np.asarray(vals, dtype=np.float64))
        return [0.5 * (v[(k * len(v)) // g - 1] + v[(k * len(v)) // g]) for k in range(1, g)]
    if d == 2 and g == 2:
        return [0.5 * (a + b)]
    return [a + ((b - a) * k) / g for k in range(1, g)]


class Geometry:
    """Partition, knots and the leaf assignment of observation locations.

    Attributes
      d, M, lo, hi, adaptive
      Jl[m]       children per region of level m - 1 (m = 1..M; Jl[0] = 1)
      rl[m]       knots per region of level m (m = 0..M-1)
      J, r        the common J and r when they do not vary (else None)
      nreg[m]     regions at level m
      bounds[m]   (nreg[m], d, 2) region boxes
      knots[m]    (nreg[m], r_m, d) knot coordinates of internal levels m < M
      leaf        (n,) leaf index of each observation (original order)
      perm        (n,) observation indices sorted by (leaf, original index)
      offsets     (nreg[M] + 1,) CSR offsets of the sorted observations per leaf
    """

    def __init__(self, locs, d, M, J, r, lo=None, hi=None, knots=None, J_levels=None, r_levels=None,
                 adaptive=False):
        locs = np.asarray(locs, dtype=np.float64).reshape(-1, d)
        if d not in (1, 2):
            raise ValueError("d must be 1 or 2")
        self.d, self.M = d, M
        self.adaptive = bool(adaptive)
        self.Jl = [1] + [int(x) for x in (J_levels if J_levels is not None else [J] * M)]
        self.rl = [int(x) for x in (r_levels if r_levels is not None else [r] * M)]
        if len(self.Jl) != M + 1 or len(self.rl) != M:
            raise ValueError("J_levels and r_levels need M entries")
        self.J = self.Jl[1] if M > 0 and len(set(self.Jl[1:])) == 1 else (J if M == 0 else None)
        self.r = self.rl[0] if M > 0 and len(set(self.rl)) == 1 else (r if M == 0 else None)
        self.lo = np.zeros(d) if lo is None else np.asarray(lo, dtype=np.float64)
        self.hi = np.ones(d) if hi is None else np.asarray(hi, dtype=np.float64)
        if ((locs < self.lo) | (locs > self.hi)).any() or not np.isfinite(locs).all():
            raise ValueError("locations outside the domain box")
        self.nreg = [1]
        for m in range(1, M + 1):
            self.nreg.append(self.nreg[-1] * self.Jl[m])
        # boxes and split values, level by level; the observations of each
        # region drive the adaptive splits
        self.bounds = [np.stack([self.lo, self.hi], axis=1)[None]]
        self.splits = []            # splits[m][i] = (gx, ysplits, [xsplits per slab])
        reg = np.zeros(locs.shape[0], dtype=np.int64)
        for m in range(M):
            J1 = self.Jl[m + 1]
            boxes = np.empty((self.nreg[m + 1], d, 2))
            spl = []
            for i in range(self.nreg[m]):
                box = self.bounds[m][i]
                pts = locs[reg == i] if self.adaptive else None
                gx, gy = grid_shape(d, J1, box)
                if d == 1:
                    ys = []
                    xs = [split_values(box[0, 0], box[0, 1], gx, d, None if pts is None else pts[:, 0])]
                else:
                    ys = split_values(box[1, 0], box[1, 1], gy, d, None if pts is None else pts[:, 1])
                    xs = []
                    for iy in range(gy):
                        sub = None
                        if pts is not None:
                            cy = np.zeros(pts.shape[0], dtype=np.int64)
                            for t in ys:
                                cy += (pts[:, 1] >= t)
                            sub = pts[cy == iy, 0]
                        xs.append(split_values(box[0, 0], box[0, 1], gx, d, sub))
                spl.append((gx, ys, xs))
                yb = [box[1, 0]] + list(ys) + [box[1, 1]] if d == 2 else None
                for iy in range(gy):
                    xb = [box[0, 0]] + list(xs[iy]) + [box[0, 1]]
                    for ix in range(gx):
                        c = boxes[i * J1 + iy * gx + ix]
                        c[0] = (xb[ix], xb[ix + 1])
                        if d == 2:
                            c[1] = (yb[iy], yb[iy + 1])
            self.splits.append(spl)
            self.bounds.append(boxes)
            reg = self._descend(locs, reg, m)
        self.knots = []
        for m in range(M):
            if knots is not None:
                kk = np.asarray(knots[m], dtype=np.float64).reshape(self.nreg[m], self.rl[m], d)
            else:
                kk = self._grid_knots(self.bounds[m], self.rl[m])
            self.knots.append(kk)
        self.leaf = reg
        self.perm = np.lexsort((np.arange(locs.shape[0]), self.leaf))
        counts = np.bincount(self.leaf, minlength=self.nreg[M])
        self.offsets = np.concatenate([[0], np.cumsum(counts)])
        self.locs = locs

    # -- partition --------------------------------------------------------
    def _descend(self, pts, reg, m):
        """Region indices at level m + 1 of points in regions reg of level m."""
        out = np.empty_like(reg)
        J1 = self.Jl[m + 1]
        for i in np.unique(reg):
            sel = np.flatnonzero(reg == i)
            gx, ys, xs = self.splits[m][int(i)]
            iy = np.zeros(sel.size, dtype=np.int64)
            if self.d == 2:
                for t in ys:
                    iy += (pts[sel, 1] >= t)
            ix = np.zeros(sel.size, dtype=np.int64)
            for y in np.unique(iy):
                s2 = iy == y
                for t in xs[int(y)]:
                    ix[s2] += (pts[sel[s2], 0] >= t)
            out[sel] = int(i) * J1 + iy * gx + ix
        return out

    def leaf_of(self, pts):
        """Leaf (level-M region) index of every point, by descending the tree
        one level at a time with the regions' split values."""
        pts = np.asarray(pts, dtype=np.float64).reshape(-1, self.d)
        reg = np.zeros(pts.shape[0], dtype=np.int64)
        for m in range(self.M):
            reg = self._descend(pts, reg, m)
        return reg

    def _grid_knots(self, boxes, r):
        d = self.d
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
    def parent(self, m, i):
        """Index at level m - 1 of the parent of region (m, i)."""
        return i // self.Jl[m]

    def ancestors(self, m, i):
        """[a_0, ..., a_m]: index at level l of the level-l ancestor of (m, i)."""
        out = [i]
        for l in range(m, 0, -1):
            out.append(out[-1] // self.Jl[l])
        return out[::-1]

    def ancestor_index(self, leaves, m):
        """Vectorised: level-m ancestor of every leaf index in `leaves`."""
        a = np.asarray(leaves, dtype=np.int64).copy()
        for l in range(self.M, m, -1):
            a //= self.Jl[l]
        return a

    def leaf_obs(self, i):
        """Indices (original order) of the observations in leaf i, sorted."""
        return self.perm[self.offsets[i]:self.offsets[i + 1]]

    def region_points(self, m, i):
        """Q_{(m,i)}: knots for m < M, observation locations for m = M."""
        if m < self.M:
            return self.knots[m][i]
        return self.locs[self.leaf_obs(i)]
