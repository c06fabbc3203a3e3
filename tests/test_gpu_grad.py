"""GPU parity of the reverse-pass gradient against the oracle's forward-mode
gradient (a different algorithm), and against central finite differences of
the GPU log-likelihood.  Bar: |g - g_oracle| <= 1e-6 |g_oracle| per
component (plus 1e-9 of the largest component for entries near zero)."""
import math

import numpy as np
import pytest

from oracle import mra
from oracle.geometry import Geometry
from paper_1507_04789_amd import MRALogLik, Plan, MRA_PLAIN, MRA_SYNC
from paper_1507_04789_amd import workloads as wl

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def _th(s2, k, t2):
    return np.array([math.log(s2), math.log(k), math.log(t2)])


def _check_grad(g, ref):
    tol = 1e-6 * np.abs(ref) + 1e-9 * np.abs(ref).max()
    assert (np.abs(g - ref) <= tol).all(), (g, ref, (g - ref) / np.abs(ref))


def _case(locs, z, kind, th, M, J, r, d=2, knots=None):
    print("grad case n=%d M=%d J=%d r=%d d=%d %s" % (len(z), M, J, r, d, kind), flush=True)
    p = Plan(locs, M=M, J=J, r=r, cov=kind, d=d, knots=knots)
    ll, g = p.loglik_grad(z, th)
    ll, g = ll.cpu().numpy()[0], g.cpu().numpy()[0]
    geo = Geometry(locs, d, M, J, r, knots=knots)
    rll, rg, st = mra.loglik(geo, z, kind, th, grad=True)
    assert abs(ll - rll) <= 1e-10 * abs(rll)
    _check_grad(g, rg)
    # sigma^2 / tau^2 scale identity: g0 + g2 = -(n - u)/2
    u = float(st.u[(0, 0)].v)
    assert abs(g[0] + g[2] + 0.5 * (len(z) - u)) <= 1e-8 * len(z)
    return p, g


def test_grad_m0():
    g = np.random.default_rng(0)
    locs = g.random((300, 2))
    z = g.standard_normal(300)
    _case(locs, z, "matern32", _th(1.2, 0.2, 0.05), 0, 4, 16)


@pytest.mark.parametrize("kind", ["matern32", "exponential"])
@pytest.mark.parametrize("M,r,n", [(1, 16, 1000), (2, 9, 1500), (3, 25, 2500)])
def test_grad_small(kind, M, r, n):
    g = np.random.default_rng(10 + M)
    locs = g.random((n, 2))
    z = g.standard_normal(n)
    _case(locs, z, kind, _th(0.9, 0.15, 0.03), M, 4, r)


def test_grad_uniform_exponential_m3_r16():
    w = wl.small_uniform()
    _case(w.locs, w.z, w.cov, w.theta, w.M, w.J, w.r)


def test_grad_clustered_r64_m4():
    w = wl.clustered(n=16384, M=4)
    _case(w.locs, w.z, w.cov, w.theta, w.M, w.J, w.r)


def test_grad_empty_single_and_large_leaves():
    g = np.random.default_rng(5)
    locs = np.concatenate([g.random((700, 2)) * 0.25, g.random((40, 2)) * 0.5 + 0.5, [[0.99, 0.01]]])
    z = g.standard_normal(locs.shape[0])
    _case(locs, z, "matern32", _th(1.0, 0.1, 0.01), 3, 4, 16)


@pytest.mark.parametrize("J,r,M", [(2, 1, 5), (3, 2, 4)])
def test_grad_one_dimensional(J, r, M):
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


def test_grad_single_child_partition():
    g = np.random.default_rng(8)
    locs = g.random((200, 2))
    z = g.standard_normal(200)
    knots = [g.random((1, 6, 2)) for _ in range(3)]
    _case(locs, z, "matern32", _th(1.0, 0.2, 0.05), 3, 1, 6, knots=knots)


def test_grad_batch_plain_fd_and_autograd():
    w = wl.clustered(n=8192, M=3)
    ths = wl.theta_draws(4, 31)
    p = Plan(w.locs, M=w.M, J=w.J, r=w.r, cov=w.cov, max_theta=4)
    ll, g = p.loglik_grad(w.z, ths)
    ll, g = ll.cpu().numpy(), g.cpu().numpy()
    geo = Geometry(w.locs, 2, w.M, w.J, w.r)
    for q in range(4):
        rll, rg, _ = mra.loglik(geo, w.z, w.cov, ths[q], grad=True)
        assert abs(ll[q] - rll) <= 1e-10 * abs(rll)
        _check_grad(g[q], rg)
        one_ll, one_g = p.loglik_grad(w.z, ths[q])
        assert (one_g.cpu().numpy()[0] == g[q]).all()
    pp = Plan(w.locs, M=w.M, J=w.J, r=w.r, cov=w.cov, max_theta=4, flags=MRA_SYNC | MRA_PLAIN)
    _, gp = pp.loglik_grad(w.z, ths)
    assert (gp.cpu().numpy() == g).all()
    # central finite differences of the GPU log-likelihood, h = 1e-5
    h = 1e-5
    for q in range(2):
        fd = []
        for c in range(3):
            e = np.zeros(3)
            e[c] = h
            lp = p.loglik(w.z, ths[q] + e).cpu().numpy()[0]
            lm = p.loglik(w.z, ths[q] - e).cpu().numpy()[0]
            fd.append((lp - lm) / (2 * h))
        fd = np.array(fd)
        assert (np.abs(fd - g[q]) <= 1e-5 * np.abs(g[q]) + 1e-6 * np.abs(g[q]).max()).all(), (fd, g[q])
    # torch.autograd.Function
    th = torch.tensor(ths, dtype=torch.float64, requires_grad=True)
    out = MRALogLik.apply(th, p, torch.tensor(w.z, device="cuda"))
    (out * torch.arange(1, 5, dtype=torch.float64, device="cuda")).sum().backward()
    np.testing.assert_array_equal(th.grad.numpy(), g * np.arange(1, 5)[:, None])


def test_grad_swath_pruned_regions():
    geom = wl.swath_geometry(5)
    locs = wl.swath_locations(geom, 6000, 6)
    z = np.random.default_rng(9).standard_normal(6000)
    _case(locs, z, "matern32", _th(1.0, 0.08, 0.02), 6, 4, 9)
