"""Host logic of the maximum-likelihood driver (L-BFGS with a batched line
search) on functions whose maximiser is known, and on the oracle's
log-likelihood of a small M-RA against scipy's L-BFGS-B on the same
function.  No GPU: the driver only sees an evaluate(thetas) callback."""
import math

import numpy as np
import pytest
from scipy.optimize import minimize

from oracle import mra
from oracle.covariance import Covariance
from oracle.geometry import Geometry
from paper_1507_04789_amd import mle


def _quadratic(c, A):
    def ev(th):
        d = th - c[None, :]
        return -0.5 * np.einsum("ki,ij,kj->k", d, A, d), -(d @ A)
    return ev


@pytest.mark.parametrize("batch", [1, 3, 6])
def test_concave_quadratic_ill_conditioned(batch):
    g = np.random.default_rng(0)
    Q, _ = np.linalg.qr(g.standard_normal((3, 3)))
    A = Q @ np.diag([1e3, 1.0, 1e-1]) @ Q.T
    c = np.array([0.3, -1.2, 2.0])
    r = mle.maximize(_quadratic(c, A), np.zeros(3), batch=batch, gtol=1e-12)
    assert r.converged, r.message
    np.testing.assert_allclose(r.theta, c, atol=1e-8)
    assert r.evaluations == 1 + batch * (r.calls - 1)
    # log-likelihood never decreases along the accepted iterates
    lls = [h[1] for h in r.history]
    assert all(b >= a for a, b in zip(lls, lls[1:]))


def test_rosenbrock_3d():
    def ev(th):
        x = th
        f = 100 * (x[:, 1] - x[:, 0] ** 2) ** 2 + (1 - x[:, 0]) ** 2 + 100 * (x[:, 2] - x[:, 1] ** 2) ** 2 + (1 - x[:, 1]) ** 2
        gx = np.zeros_like(x)
        gx[:, 0] = -400 * x[:, 0] * (x[:, 1] - x[:, 0] ** 2) - 2 * (1 - x[:, 0])
        gx[:, 1] = 200 * (x[:, 1] - x[:, 0] ** 2) - 400 * x[:, 1] * (x[:, 2] - x[:, 1] ** 2) - 2 * (1 - x[:, 1])
        gx[:, 2] = 200 * (x[:, 2] - x[:, 1] ** 2)
        return -f, -gx
    r = mle.maximize(ev, np.array([-1.0, 1.5, 0.5]), batch=4, max_iter=500, gtol=1e-10, ftol=0.0)
    assert r.converged, r.message
    np.testing.assert_allclose(r.theta, np.ones(3), atol=1e-6)


def test_failed_evaluations_are_rejected():
    """NaN (a factorisation breakdown) beyond a wall: the line search backs
    off and the maximiser just inside the wall is still found."""
    c = np.array([0.0, 0.0, -2.0])
    base = _quadratic(c, np.diag([1.0, 2.0, 4.0]))

    def ev(th):
        ll, g = base(th)
        bad = th[:, 2] < -2.5
        ll = np.where(bad, np.nan, ll)
        g = np.where(bad[:, None], np.nan, g)
        return ll, g
    r = mle.maximize(ev, np.array([3.0, -2.0, 1.0]), batch=2, max_step=10.0, gtol=1e-12)
    assert r.converged, r.message
    np.testing.assert_allclose(r.theta, c, atol=1e-8)


def test_start_not_finite_and_bad_arguments():
    r = mle.maximize(lambda th: (np.full(len(th), np.nan), np.zeros((len(th), 3))), np.zeros(3))
    assert not r.converged and r.iterations == 0
    with pytest.raises(ValueError):
        mle.maximize(_quadratic(np.zeros(3), np.eye(3)), np.zeros(3), batch=0)


def test_oracle_mra_likelihood_matches_scipy():
    """The driver and scipy's L-BFGS-B reach the same maximum-likelihood
    estimate on the oracle's M-RA log-likelihood (n = 300, M = 2, r = 9)."""
    g = np.random.default_rng(3)
    locs = g.random((300, 2))
    cov = Covariance("matern32", np.array([math.log(1.0), math.log(0.15), math.log(0.05)]))
    z = np.linalg.cholesky(cov(locs, locs) + cov.tau2 * np.eye(300)) @ g.standard_normal(300)
    geo = Geometry(locs, 2, 2, 4, 9)

    def ev(th):
        out = [mra.loglik(geo, z, "matern32", t, grad=True)[:2] for t in th]
        return np.array([o[0] for o in out]), np.array([o[1] for o in out])
    th0 = np.array([0.0, math.log(0.2), math.log(0.1)])
    r = mle.maximize(ev, th0, batch=3, gtol=1e-9)
    assert r.converged, r.message
    ref = minimize(lambda t: -ev(t[None])[0][0], th0, jac=lambda t: -ev(t[None])[1][0], method="L-BFGS-B",
                   options={"gtol": 1e-10, "ftol": 1e-15, "maxiter": 500})
    assert r.loglik >= -ref.fun - 1e-9 * abs(ref.fun)
    np.testing.assert_allclose(r.theta, ref.x, atol=2e-4)
    assert np.abs(r.grad).max() <= 1e-9 * max(1.0, abs(r.loglik))
