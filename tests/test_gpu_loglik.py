"""GPU parity of the M-RA log-likelihood against the CPU oracle.

Every case runs the HIP path through the C ABI and the oracle on the same
seeded inputs and compares element by element: relative error <= 1e-10 on
the log-likelihood.  Cases span several tiles and ragged tails: leaves
with 0, 1 and several hundred observations, r below the 64-wide tile, one-
dimensional domains, J = 1, M = 0 (exact GP), several parameter vectors in
one launch, the plain one-launch-per-task form, and the failure path.
"""
import math

import numpy as np
import pytest

from oracle import mra
from oracle.geometry import Geometry
from paper_1507_04789_amd import Plan, MRAError, MRA_PLAIN, MRA_SYNC
from paper_1507_04789_amd import workloads as wl

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

RTOL = 1e-10


def _th(s2, k, t2):
    return np.array([math.log(s2), math.log(k), math.log(t2)])


def _oracle(locs, z, kind, th, M, J, r, d=2, knots=None):
    g = Geometry(locs, d, M, J, r, knots=knots)
    return mra.loglik(g, z, kind, th)[0]


def _case(locs, z, kind, th, M, J, r, d=2, knots=None, flags=MRA_SYNC):
    print("case n=%d M=%d J=%d r=%d d=%d %s" % (len(z), M, J, r, d, kind), flush=True)
    p = Plan(locs, M=M, J=J, r=r, cov=kind, d=d, knots=knots, flags=flags)
    got = p.loglik(z, th).cpu().numpy()[0]
    ref = _oracle(locs, z, kind, th, M, J, r, d, knots)
    assert abs(got - ref) <= RTOL * abs(ref), (got, ref, (got - ref) / abs(ref))
    return p, got


def test_exact_gp_m0():
    g = np.random.default_rng(0)
    locs = g.random((300, 2))
    z = g.standard_normal(300)
    _case(locs, z, "matern32", _th(1.2, 0.2, 0.05), 0, 4, 16)


@pytest.mark.parametrize("kind", ["matern32", "exponential"])
@pytest.mark.parametrize("M,r,n", [(1, 16, 1000), (2, 9, 1500), (3, 25, 2500)])
def test_small_uniform(kind, M, r, n):
    g = np.random.default_rng(M)
    locs = g.random((n, 2))
    z = g.standard_normal(n)
    _case(locs, z, kind, _th(0.9, 0.15, 0.03), M, 4, r)


def test_uniform_exponential_m3_r16():
    w = wl.small_uniform()
    _case(w.locs, w.z, w.cov, w.theta, w.M, w.J, w.r)


def test_clustered_r64_m4():
    w = wl.clustered(n=16384, M=4)
    _case(w.locs, w.z, w.cov, w.theta, w.M, w.J, w.r)


def test_empty_single_and_large_leaves():
    g = np.random.default_rng(5)
    locs = np.concatenate([g.random((700, 2)) * 0.25, g.random((40, 2)) * 0.5 + 0.5, [[0.99, 0.01]]])
    z = g.standard_normal(locs.shape[0])
    p, _ = _case(locs, z, "matern32", _th(1.0, 0.1, 0.01), 3, 4, 16)
    assert p.info["max_leaf"] > 128


@pytest.mark.parametrize("J,r,M", [(2, 1, 5), (3, 2, 4)])
def test_one_dimensional(J, r, M):
    g = np.random.default_rng(7)
    locs = g.random((400, 1))
    z = g.standard_normal(400)
    knots = None
    if J == 3:
        knots = []
        for m in range(M):
            w = 1.0 / J ** m
            knots.append(np.array([[[i * w + w * k / J] for k in range(1, J)] for i in range(J ** m)]))
    _case(locs, z, "exponential", _th(1.0, 0.3, 0.05), M, J, r, d=1, knots=knots)


def test_single_child_partition():
    g = np.random.default_rng(8)
    locs = g.random((200, 2))
    z = g.standard_normal(200)
    knots = [g.random((1, 6, 2)) for _ in range(3)]
    _case(locs, z, "matern32", _th(1.0, 0.2, 0.05), 3, 1, 6, knots=knots)


def test_theta_batch_plain_and_repeat():
    w = wl.clustered(n=8192, M=3)
    ths = wl.theta_draws(4, 31)
    p = Plan(w.locs, M=w.M, J=w.J, r=w.r, cov=w.cov, max_theta=4)
    batch = p.loglik(w.z, ths).cpu().numpy()
    for q in range(4):
        one = p.loglik(w.z, ths[q]).cpu().numpy()[0]
        assert one == batch[q]                       # bitwise: same kernels
        ref = _oracle(w.locs, w.z, w.cov, ths[q], w.M, w.J, w.r)
        assert abs(batch[q] - ref) <= RTOL * abs(ref)
    again = p.loglik(w.z, ths).cpu().numpy()
    assert (again == batch).all()                     # deterministic (no atomics)
    pp = Plan(w.locs, M=w.M, J=w.J, r=w.r, cov=w.cov, max_theta=4, flags=MRA_SYNC | MRA_PLAIN)
    plain = pp.loglik(w.z, ths).cpu().numpy()
    assert (plain == batch).all()


def test_failure_reports_theta():
    g = np.random.default_rng(9)
    locs = g.random((500, 2))
    z = g.standard_normal(500)
    p = Plan(locs, M=2, J=4, r=16, cov="matern32", max_theta=3)
    ths = np.stack([_th(1, 0.1, 0.01), [np.nan, math.log(0.1), math.log(0.01)], _th(2, 0.2, 0.02)])
    with pytest.raises(MRAError) as e:
        p.loglik(z, ths)
    assert "theta 1" in str(e.value)
    # the other entries stay valid without the sync check
    p2 = Plan(locs, M=2, J=4, r=16, cov="matern32", max_theta=3, flags=0)
    out = p2.loglik(z, ths).cpu().numpy()
    assert math.isnan(out[1]) and np.isfinite(out[[0, 2]]).all()
    ref = _oracle(locs, z, "matern32", ths[2], 2, 4, 16)
    assert abs(out[2] - ref) <= RTOL * abs(ref)


def _last_failure(p):
    import ctypes as C
    from paper_1507_04789_amd import _lib
    th, lv, rg = C.c_int32(), C.c_int32(), C.c_int64()
    _lib.lib().mra_last_failure(p._h, C.byref(th), C.byref(lv), C.byref(rg), p._stream())
    return th.value, lv.value, rg.value


@pytest.mark.parametrize("case", ["huge_range_root", "duplicate_leaf_points"])
def test_breakdown_matches_oracle(case):
    """Singular inputs where the oracle's Cholesky raises LinAlgError: a range
    so large that the root's K^{-1} is numerically rank one (failure at level
    0, region 0), and 21 copies of one location in a leaf with a negligible
    nugget (failure at level M, that leaf).  The library returns MRA_ENOTPD
    and names the same parameter row, level and region; the other rows of
    the batch keep their values."""
    from numpy.linalg import LinAlgError
    from paper_1507_04789_amd import _lib
    g = np.random.default_rng(90)
    locs = g.random((800, 2))
    z = g.standard_normal(800)
    geo = Geometry(locs, 2, 3, 4, 16)
    bad = _th(1.0, math.exp(16.0), 0.01)
    where = (0, 0)
    if case == "duplicate_leaf_points":
        leaf = int(np.bincount(geo.leaf).argmax())
        idx = np.flatnonzero(geo.leaf == leaf)
        locs[idx[1:21]] = locs[idx[0]]
        geo = Geometry(locs, 2, 3, 4, 16)
        bad = np.array([0.0, math.log(0.1), -200.0])
        where = (3, leaf)
    print("breakdown case %s" % case, flush=True)
    with pytest.raises(LinAlgError):
        mra.loglik(geo, z, "matern32", bad)
    ths = np.stack([_th(1, 0.1, 0.01), bad, _th(2, 0.2, 0.02)])
    for flags in (MRA_SYNC, MRA_SYNC | MRA_PLAIN):
        p = Plan(locs, M=3, J=4, r=16, cov="matern32", max_theta=3, flags=flags)
        with pytest.raises(MRAError) as e:
            p.loglik_grad(z, ths)
        assert e.value.status == _lib.MRA_ENOTPD
        assert _last_failure(p) == (1, where[0], where[1])
    q = Plan(locs, M=3, J=4, r=16, cov="matern32", max_theta=3, flags=0)
    ll, gr = q.loglik_grad(z, ths)
    ll, gr = ll.cpu().numpy(), gr.cpu().numpy()
    assert math.isnan(ll[1]) and np.isnan(gr[1]).all()
    for i in (0, 2):
        ref = _oracle(locs, z, "matern32", ths[i], 3, 4, 16)
        assert abs(ll[i] - ref) <= RTOL * abs(ref)


def test_knots_equal_to_ancestor_knots_break_down():
    """Eight knots of level-1 region 2 placed on root knots: that region's
    prior K^{-1} is singular for every parameter vector (its rows for those
    knots vanish once the root is conditioned on).  The oracle raises
    LinAlgError; the library names row 0, level 1, region 2, and without
    MRA_SYNC every row reads NaN."""
    from numpy.linalg import LinAlgError
    from paper_1507_04789_amd import _lib
    g = np.random.default_rng(90)
    locs = g.random((800, 2))
    z = g.standard_normal(800)
    kn = [np.array(k, copy=True) for k in Geometry(locs, 2, 3, 4, 16).knots]
    kn[1][2][:8] = kn[0][0][8:16]
    geo = Geometry(locs, 2, 3, 4, 16, knots=kn)
    ths = np.stack([_th(1, 0.1, 0.01), _th(2, 0.2, 0.02), _th(1, 0.3, 0.05)])
    for th in ths:
        with pytest.raises(LinAlgError):
            mra.loglik(geo, z, "matern32", th)
    print("breakdown case: knots on ancestor knots", flush=True)
    p = Plan(locs, M=3, J=4, r=16, cov="matern32", knots=kn, max_theta=3, flags=MRA_SYNC)
    with pytest.raises(MRAError) as e:
        p.loglik_grad(z, ths)
    assert e.value.status == _lib.MRA_ENOTPD
    assert _last_failure(p) == (0, 1, 2)
    q = Plan(locs, M=3, J=4, r=16, cov="matern32", knots=kn, max_theta=3, flags=0)
    ll, gr = q.loglik_grad(z, ths)
    assert torch.isnan(ll).all() and torch.isnan(gr).all()


def test_no_grad_plan_matches_and_refuses_gradient():
    from paper_1507_04789_amd import MRA_NO_GRAD
    w = wl.clustered(n=32768, M=4, r=64)
    print("case: clustered n=%d M=%d, loglik-only plan" % (len(w.z), w.M), flush=True)
    full = Plan(w.locs, M=w.M, J=w.J, r=w.r, cov=w.cov, max_theta=2)
    lean = Plan(w.locs, M=w.M, J=w.J, r=w.r, cov=w.cov, max_theta=2, flags=MRA_SYNC | MRA_NO_GRAD)
    assert lean.work_bytes < full.work_bytes
    z = w.z
    ths = wl.theta_draws(2, 9)
    a = full.loglik(z, ths).cpu().numpy()
    b = lean.loglik(z, ths).cpu().numpy()
    assert np.array_equal(a, b)
    # the gradient call on the full plan leaves the loglik-only results unchanged
    ll, _ = full.loglik_grad(z, ths[:1])
    assert float(ll[0]) == a[0]
    with pytest.raises(MRAError):
        lean.loglik_grad(z, ths[:1])
