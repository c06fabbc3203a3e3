"""Full-size GPU parity: the clustered workload (n = 2^18, M = 6, J = 4,
r = 64, Matern nu = 1.5) in the launch configuration the benchmark times
(asynchronous plan, one parameter vector per call), and as one batched call
over three parameter vectors, against oracle values stored in
tests/golden/clustered_n262144.json (written by tests/golden/make_golden.py,
which calls only the oracle).  Bar: 1e-10 relative on the log-likelihood,
1e-6 relative per gradient component."""
import json
import os

import numpy as np
import pytest

from paper_1507_04789_amd import Plan
from paper_1507_04789_amd import workloads as wl

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

GOLD = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "clustered_n262144.json")


@pytest.fixture(scope="module")
def data():
    with open(GOLD) as f:
        gold = json.load(f)
    w = wl.clustered()
    assert len(w.z) == gold["n"] and (w.M, w.J, w.r, w.cov) == (gold["M"], gold["J"], gold["r"], gold["cov"])
    assert np.allclose(w.theta, gold["points"][0]["theta"], rtol=0, atol=0)
    return w, gold


def _check(ll, g, pt):
    rll, rg = pt["loglik"], np.asarray(pt["grad"])
    assert abs(ll - rll) <= 1e-10 * abs(rll), (ll, rll)
    assert (np.abs(g - rg) <= 1e-6 * np.abs(rg)).all(), (g, rg, (g - rg) / rg)


def test_full_size_bench_configuration(data):
    w, gold = data
    print("full-size case: n=%d M=%d one theta per call, async plan" % (len(w.z), w.M), flush=True)
    p = Plan(w.locs, M=w.M, J=w.J, r=w.r, cov=w.cov, flags=0)
    p.bind("cuda:0")
    z = torch.tensor(w.z, device="cuda:0")
    for pt in gold["points"]:
        th = torch.tensor(pt["theta"], dtype=torch.float64, device="cuda:0").reshape(1, 3)
        ll, g = p.loglik_grad(z, th)
        ll1 = p.loglik(z, th)
        torch.cuda.synchronize()
        _check(float(ll[0]), g[0].cpu().numpy(), pt)
        assert abs(float(ll1[0]) - float(ll[0])) <= 1e-12 * abs(float(ll[0]))
    del p
    torch.cuda.empty_cache()


def test_full_size_theta_batch(data):
    w, gold = data
    k = len(gold["points"])
    print("full-size case: n=%d M=%d %d thetas in one call" % (len(w.z), w.M, k), flush=True)
    p = Plan(w.locs, M=w.M, J=w.J, r=w.r, cov=w.cov, max_theta=k)
    p.bind("cuda:0")
    z = torch.tensor(w.z, device="cuda:0")
    th = torch.tensor([pt["theta"] for pt in gold["points"]], dtype=torch.float64, device="cuda:0")
    ll, g = p.loglik_grad(z, th)
    ll, g = ll.cpu().numpy(), g.cpu().numpy()
    for i, pt in enumerate(gold["points"]):
        _check(float(ll[i]), g[i], pt)
    del p
    torch.cuda.empty_cache()


def test_swath_full_size_properties():
    """Satellite-swath workload at full size (n = 2^22 in 24 strips with
    gaps, M = 9, r = 64, 73% of the leaves empty; 2^20 prediction points in
    the gaps).  The oracle cannot run at this size, so the checks are
    properties that hold at any size: the scale identity
    loglik(s z; s^2 sigma^2, kappa, s^2 tau^2) = loglik(z; theta) - n log s,
    mean(s z) = s mean(z) and var scaled by s^2, and the gradient against
    central differences of the GPU log-likelihood."""
    import math
    torch.cuda.empty_cache()
    w = wl.swaths()
    z = w.z - (0.5 + w.locs[:, 0] - w.locs[:, 1])     # the caller removes the mean trend
    print("full-size swath case: n=%d M=%d n_pred=%d" % (len(z), w.M, len(w.pred)), flush=True)
    p = Plan(w.locs, M=w.M, J=w.J, r=w.r, cov=w.cov, pred=w.pred, flags=0)
    p.bind("cuda:0")
    zt = torch.tensor(z, device="cuda:0")
    th = torch.tensor(w.theta, dtype=torch.float64, device="cuda:0").reshape(1, 3)
    ll, g = p.loglik_grad(zt, th)
    ll, g = float(ll[0]), g[0].cpu().numpy()
    assert math.isfinite(ll) and np.isfinite(g).all()
    s = 2.0
    shift = torch.tensor([[2 * math.log(s), 0.0, 2 * math.log(s)]], dtype=torch.float64, device="cuda:0")
    l2 = float(p.loglik(zt * s, th + shift)[0])
    assert abs(l2 - (ll - len(z) * math.log(s))) <= 1e-10 * abs(ll)
    mu, var = p.predict(zt, th)
    mu2, var2 = p.predict(zt * s, th + shift)
    assert (var > 0).all()
    assert float((mu2 - s * mu).abs().max()) <= 1e-10 * s * float(mu.abs().max())
    assert float((var2 - s * s * var).abs().max()) <= 1e-10 * s * s * float(var.max())
    h = 1e-4
    for a in range(3):
        e = torch.zeros(1, 3, dtype=torch.float64, device="cuda:0")
        e[0, a] = h
        fd = (float(p.loglik(zt, th + e)[0]) - float(p.loglik(zt, th - e)[0])) / (2 * h)
        assert abs(fd - g[a]) <= 1e-5 * abs(g[a]) + 1e-3, (a, fd, g[a])
    del p
    torch.cuda.empty_cache()
