"""The oracle's partition and knots against the definitions of Sec. 2.2.

Checks by brute force: every observation lies in the box of its leaf and of
each of its ancestors, the children of a region tile it, the default knots
lie inside their region and never repeat an ancestor's knot (which would make
K^{-1} singular), and the observation order is the stable sort by leaf.
"""
import numpy as np
import pytest

from oracle.geometry import Geometry
from paper_1507_04789_amd import workloads as wl


def _inside(p, box):
    return all(box[a, 0] <= p[a] <= box[a, 1] for a in range(box.shape[0]))


@pytest.mark.parametrize("d,J,M,r", [(2, 4, 3, 16), (2, 4, 5, 4), (1, 2, 6, 3), (1, 3, 4, 2), (2, 1, 3, 4)])
def test_leaf_boxes_and_children(d, J, M, r):
    g0 = np.random.default_rng(1)
    locs = g0.random((500, d))
    locs[:3] = 0.5        # on split lines
    locs[3] = 1.0         # on the outer edge
    kn = None
    if J == 1:
        kn = [g0.random((1, r, d)) for _ in range(M)]
    g = Geometry(locs, d, M, J, r, knots=kn)
    for p in range(locs.shape[0]):
        i = int(g.leaf[p])
        for m in range(M, -1, -1):
            assert _inside(locs[p], g.bounds[m][g.ancestor_index([i], m)[0]])
    # children tile their parent (volume and containment)
    for m in range(M):
        for i in range(J ** m):
            par = g.bounds[m][i]
            vol = np.prod(par[:, 1] - par[:, 0])
            ch = g.bounds[m + 1][i * J:(i + 1) * J]
            cv = np.prod(ch[:, :, 1] - ch[:, :, 0], axis=1)
            if J > 1:
                assert abs(cv.sum() - vol) <= 1e-15
            for c in ch:
                assert (c[:, 0] >= par[:, 0]).all() and (c[:, 1] <= par[:, 1]).all()
    # points on a split line go to the upper child
    if d == 2 and J == 4:
        assert g.leaf[0] == g.leaf_of(np.array([[0.5, 0.5]]))[0]
        b = g.bounds[M][g.leaf[0]]
        assert b[0, 0] == 0.5 and b[1, 0] == 0.5
    # stable sort by leaf
    order = np.lexsort((np.arange(len(locs)), g.leaf))
    assert (g.perm == order).all()
    assert g.offsets[-1] == len(locs)


@pytest.mark.parametrize("d,J,M,r", [(2, 4, 6, 64), (2, 4, 4, 16), (1, 2, 8, 4)])
def test_default_knots_inside_and_distinct(d, J, M, r):
    g = Geometry(np.zeros((1, d)) + 0.25, d, M, J, r)
    for m in range(M):
        for i in range(J ** m):
            box = g.bounds[m][i]
            for q in g.knots[m][i]:
                assert _inside(q, box)
            anc = g.ancestors(m, i)
            chain = np.concatenate([g.knots[l][anc[l]] for l in range(m + 1)])
            # no two chain knots coincide
            u = np.unique(chain, axis=0)
            assert u.shape[0] == chain.shape[0]


def test_clustered_workload_shape():
    w = wl.clustered(n=8192, M=4)
    g = Geometry(w.locs, 2, w.M, w.J, w.r)
    c = np.diff(g.offsets)
    assert c.sum() == 8192 and c.max() > 2.5 * c.mean()   # uneven leaves
    assert ((w.locs >= 0) & (w.locs <= 1)).all()


def test_swath_workload_shape():
    geom = wl.swath_geometry(5)
    pts = wl.swath_locations(geom, 20000, 6)
    gp = wl.swath_locations(geom, 5000, 7, in_gaps=True)
    assert ((pts >= 0) & (pts <= 1)).all() and ((gp >= 0) & (gp <= 1)).all()
    # every point is within half a strip width of some line x - y = c
    dist = np.abs((pts[:, 0] - pts[:, 1])[:, None] - geom.centers[None, :]) / np.sqrt(2)
    assert (dist.min(axis=1) <= geom.width / 2 + 1e-12).all()


@pytest.mark.parametrize("Jl,adaptive", [((2, 2, 4, 8), False), ((2, 8, 16), False), ((2, 2, 4, 8), True),
                                         ((4, 4, 4), True), ((8, 2), True)])
def test_mixed_and_adaptive_partitions(Jl, adaptive):
    """Level-dependent J_m and data-adaptive splits: every point lies in the
    boxes of its leaf and ancestors, the children of a region tile it (area
    and containment), split values of adaptive splits are quantiles of the
    region's points, and the leaf assignment of prediction points agrees
    with that of the observations."""
    w = wl.clustered(n=6000, M=len(Jl))
    M = len(Jl)
    g = Geometry(w.locs, 2, M, 4, 4, J_levels=Jl, r_levels=[4] * M, adaptive=adaptive)
    for p in range(0, 6000, 7):
        i = int(g.leaf[p])
        for m in range(M, -1, -1):
            assert _inside(w.locs[p], g.bounds[m][g.ancestor_index([i], m)[0]])
    for m in range(M):
        J = Jl[m]
        for i in range(g.nreg[m]):
            par = g.bounds[m][i]
            ch = g.bounds[m + 1][i * J:(i + 1) * J]
            cv = np.prod(ch[:, :, 1] - ch[:, :, 0], axis=1)
            assert abs(cv.sum() - np.prod(par[:, 1] - par[:, 0])) <= 1e-12
            for c in ch:
                assert (c[:, 0] >= par[:, 0]).all() and (c[:, 1] <= par[:, 1]).all()
    assert (g.leaf_of(w.locs) == g.leaf).all()
    if adaptive:
        # each split divides its region's points into (nearly) equal parts
        m0 = np.bincount(g.ancestor_index(g.leaf, 1), minlength=Jl[0])
        assert m0.max() - m0.min() <= Jl[0]
