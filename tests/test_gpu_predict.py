"""GPU parity of the kriging pass (Prop. 2) against the oracle: posterior
predictive mean and marginal variance of the latent process, relative error
<= 1e-10 (variances compared relative to sigma^2, the prior variance); at
r = 64, M = 6 (stored oracle values) entry by entry."""
import json
import math
import os

import numpy as np
import pytest

from oracle import predict
from oracle.geometry import Geometry
from paper_1507_04789_amd import Plan
from paper_1507_04789_amd import workloads as wl

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def _th(s2, k, t2):
    return np.array([math.log(s2), math.log(k), math.log(t2)])


def _case(locs, z, pred, kind, th, M, J, r, d=2, knots=None):
    print("predict case n=%d np=%d M=%d J=%d r=%d d=%d %s" % (len(z), len(pred), M, J, r, d, kind), flush=True)
    p = Plan(locs, M=M, J=J, r=r, cov=kind, d=d, knots=knots, pred=pred)
    mu, var = p.predict(z, th)
    mu, var = mu.cpu().numpy(), var.cpu().numpy()
    geo = Geometry(locs, d, M, J, r, knots=knots)
    rmu, rvar = predict.predict(geo, z, kind, th, pred)
    s2 = math.exp(th[0])
    # entry by entry, with a floor for means and variances near zero
    em, ev = np.abs(mu - rmu), np.abs(var - rvar)
    assert (em <= 1e-10 * np.abs(rmu) + 1e-12 * np.abs(rmu).max()).all(), (em / np.abs(rmu)).max()
    assert (ev <= 1e-10 * np.abs(rvar) + 1e-12 * s2).all(), (ev / np.abs(rvar)).max()
    assert (var > 0).all()


def test_predict_uniform_exponential_m3_r16():
    w = wl.small_uniform()
    _case(w.locs, w.z, w.pred, w.cov, w.theta, w.M, w.J, w.r)


@pytest.mark.parametrize("M,r", [(0, 16), (1, 16), (2, 9)])
def test_predict_small(M, r):
    g = np.random.default_rng(20 + M)
    locs = g.random((900, 2))
    z = g.standard_normal(900)
    pred = g.random((300, 2))
    _case(locs, z, pred, "matern32", _th(1.1, 0.12, 0.02), M, 4, r)


def test_predict_empty_leaves_and_large_leaf():
    g = np.random.default_rng(6)
    locs = np.concatenate([g.random((500, 2)) * 0.25, g.random((30, 2)) * 0.5 + 0.5])
    z = g.standard_normal(locs.shape[0])
    pred = g.random((400, 2))            # many fall in empty leaves
    _case(locs, z, pred, "matern32", _th(1.0, 0.1, 0.01), 3, 4, 16)


def test_predict_clustered_r64():
    w = wl.clustered(n=16384, M=4)
    pred = np.random.default_rng(3).random((2000, 2))
    _case(w.locs, w.z, pred, w.cov, w.theta, w.M, w.J, w.r)


def test_predict_one_dimensional_exact():
    g = np.random.default_rng(7)
    locs = g.random((300, 1))
    z = g.standard_normal(300)
    pred = g.random((100, 1))
    _case(locs, z, pred, "exponential", _th(1.0, 0.3, 0.05), 5, 2, 1, d=1)


def test_predict_swath_gaps_pruned_regions():
    # satellite-swath scatter at a small size: most regions below level 2 hold
    # no observation (pruned from the posterior) and the prediction points lie
    # in the gaps (regions kept for the prior only)
    geom = wl.swath_geometry(5)
    locs = wl.swath_locations(geom, 6000, 6)
    pred = wl.swath_locations(geom, 1500, 7, in_gaps=True)
    z = np.random.default_rng(8).standard_normal(6000)
    p = Plan(locs, M=6, J=4, r=9, cov="matern32", pred=pred)
    leaves = np.diff(p.geometry()[1])
    assert (leaves == 0).mean() > 0.5
    _case(locs, z, pred, "matern32", _th(1.0, 0.08, 0.02), 6, 4, 9)


PRED_GOLD = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "predict_n65536_M6_r64.json")


@pytest.mark.parametrize("case", ["swath", "clustered"])
def test_predict_r64_m6_per_entry(case):
    """The kernel's full shape (M = 6, r = 64, Matern) on 2^16 locations,
    against the oracle's kriging stored by tests/golden/make_golden.py
    --predict: satellite swaths with most leaves empty (pruned regions) and
    prediction points in the gaps plus uniform ones (regions kept for the
    prior only), and the clustered scatter.  Entry by entry: |mean error| <=
    1e-10 |mean| + 1e-12 max|mean|, |var error| <= 1e-10 var + 1e-12 sigma^2."""
    import importlib.util
    spec = importlib.util.spec_from_file_location(
        "make_golden", os.path.join(os.path.dirname(PRED_GOLD), "make_golden.py"))
    mg = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mg)
    with open(PRED_GOLD) as f:
        gold = {c["case"]: c for c in json.load(f)["cases"]}[case]
    name, locs, z, pred, theta = [c for c in mg.predict_cases() if c[0] == case][0]
    assert len(z) == gold["n"] and len(pred) == gold["n_pred"] and np.array_equal(theta, gold["theta"])
    print("predict r64 M6 per entry: %s n=%d n_pred=%d" % (case, len(z), len(pred)), flush=True)
    p = Plan(locs, M=6, J=4, r=64, cov="matern32", pred=pred)
    mu, var = p.predict(z, theta)
    mu, var = mu.cpu().numpy(), var.cpu().numpy()
    rmu, rvar = np.asarray(gold["mean"]), np.asarray(gold["var"])
    s2 = math.exp(theta[0])
    em, ev = np.abs(mu - rmu), np.abs(var - rvar)
    print("  worst relative: mean %.2e var %.2e" % ((em / np.abs(rmu)).max(), (ev / rvar).max()), flush=True)
    assert (em <= 1e-10 * np.abs(rmu) + 1e-12 * np.abs(rmu).max()).all(), (em / np.abs(rmu)).max()
    assert (ev <= 1e-10 * rvar + 1e-12 * s2).all(), (ev / rvar).max()
    assert (var > 0).all()
