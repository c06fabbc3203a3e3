"""Brute-force dense checks for small n.

The M-RA covariance between two locations is assembled from the closed form
of Sec. 2.4 ("Quality of the covariance approximation"): if s and s' lie in
the same region at resolution M, C_M(s, s') = C_0(s, s'); if they share a
region only up to resolution m* < M, C_M(s, s') is the sum over l <= m* of
b_{a_l}(s)' K_{a_l} b_{a_l}(s').  Along one chain of regions a_0, ..., a_{m*}
every point involved lies in every region of the chain, so v_l restricted to
that chain is the covariance of y_0 conditional on the knots of a_0..a_{l-1}
(eq. msadetails, by induction on l), and the sum telescopes to the
predictive-process covariance given all chain knots Q_c = Q_{a_0} u ... u
Q_{a_{m*}}:
    C_M(s, s') = C_0(s, Q_c) C_0(Q_c, Q_c)^{-1} C_0(Q_c, s').
This uses none of eq. priorw or the posterior recursion, so it checks them.
The data covariance is C_M(S, S) + tau^2 I (Sec. 4.2).
"""
from __future__ import annotations

import math

import numpy as np

from .covariance import Covariance
from .geometry import Geometry


def _chain_knots(geom: Geometry, m: int, i: int):
    anc = geom.ancestors(m, i)
    return np.concatenate([geom.knots[l][anc[l]] for l in range(m + 1)], axis=0)


def mra_cross(geom: Geometry, cov: Covariance, X, leafX, Y, leafY, grad=False):
    """C_M(X, Y) (and its (3, ...) tangents) by the chain closed form.

    leafX, leafY: leaf indices of the points.  Returns (value, tangents)."""
    M = geom.M
    X = np.atleast_2d(X)
    Y = np.atleast_2d(Y)
    out = np.zeros((X.shape[0], Y.shape[0]))
    tout = np.zeros((3,) + out.shape) if grad else None
    # deepest common level of every pair
    mstar = np.full(out.shape, M, dtype=np.int64)
    for m in range(M - 1, -1, -1):
        ax = geom.ancestor_index(leafX, m)
        ay = geom.ancestor_index(leafY, m)
        ax1 = geom.ancestor_index(leafX, m + 1)
        ay1 = geom.ancestor_index(leafY, m + 1)
        sel = (ax[:, None] == ay[None, :]) & (ax1[:, None] != ay1[None, :])
        mstar[sel] = m
    same = mstar == M
    if same.any():
        t = cov.tangents(X, Y)
        out[same] = t[0][same]
        if grad:
            tout[:, same] = t[:, same]
    for m in range(M):
        axm, aym = geom.ancestor_index(leafX, m), geom.ancestor_index(leafY, m)
        for i in range(geom.nreg[m]):
            ix = np.flatnonzero(axm == i)
            iy = np.flatnonzero(aym == i)
            if ix.size == 0 or iy.size == 0:
                continue
            blk = mstar[np.ix_(ix, iy)] == m
            if not blk.any():
                continue
            Qc = _chain_knots(geom, m, i)
            if Qc.shape[0] == 0:
                continue
            cx = cov.tangents(Qc, X[ix])
            cy = cov.tangents(Qc, Y[iy])
            G = cov.tangents(Qc, Qc)
            Gi_cy = np.linalg.solve(G[0], cy[0])
            Gi_cx = np.linalg.solve(G[0], cx[0])
            val = cx[0].T @ Gi_cy
            sub = out[np.ix_(ix, iy)]
            sub[blk] = val[blk]
            out[np.ix_(ix, iy)] = sub
            if grad:
                for p in range(3):
                    dv = cx[p].T @ Gi_cy + Gi_cx.T @ cy[p] - Gi_cx.T @ G[p] @ Gi_cy
                    s = tout[p][np.ix_(ix, iy)]
                    s[blk] = dv[blk]
                    tout[p][np.ix_(ix, iy)] = s
    return out, tout


def data_covariance(geom: Geometry, cov: Covariance, grad=False):
    """Sigma = C_M(S, S) + tau^2 I in the original order of geom.locs."""
    S = geom.locs
    V, T = mra_cross(geom, cov, S, geom.leaf, S, geom.leaf, grad)
    n = S.shape[0]
    V = V + cov.tau2 * np.eye(n)
    if grad:
        T[2] = T[2] + cov.tau2 * np.eye(n)
    return V, T


def gauss_loglik(Sigma, z, dSigma=None):
    """log N(z; 0, Sigma) by a dense Cholesky, with the gradient
    -1/2 [tr(Sigma^{-1} dSigma) - a' dSigma a], a = Sigma^{-1} z."""
    n = z.shape[0]
    L = np.linalg.cholesky(Sigma)
    w = np.linalg.solve(L, z)
    ll = -np.log(np.diag(L)).sum() - 0.5 * w @ w - 0.5 * n * math.log(2 * math.pi)
    if dSigma is None:
        return ll, None
    Si = np.linalg.inv(Sigma)
    a = Si @ z
    g = np.array([-0.5 * (np.sum(Si * dSigma[p]) - a @ dSigma[p] @ a) for p in range(dSigma.shape[0])])
    return ll, g


def mra_loglik_dense(geom, z, cov_kind, theta, grad=False):
    cov = Covariance(cov_kind, theta)
    V, T = data_covariance(geom, cov, grad)
    return gauss_loglik(V, np.asarray(z, dtype=np.float64), T)


def exact_loglik(locs, z, cov_kind, theta, grad=False):
    """The original process (0-RA): z ~ N(0, C_0(S, S) + tau^2 I)."""
    cov = Covariance(cov_kind, theta)
    t = cov.tangents(locs, locs)
    n = locs.shape[0]
    V = t[0] + cov.tau2 * np.eye(n)
    t[2] = cov.tau2 * np.eye(n)
    return gauss_loglik(V, np.asarray(z, dtype=np.float64), t if grad else None)


def mra_krige_dense(geom, z, cov_kind, theta, pred):
    """Posterior mean and variance of the latent M-RA process at pred."""
    cov = Covariance(cov_kind, theta)
    V, _ = data_covariance(geom, cov)
    leafP = geom.leaf_of(pred)
    Cps, _ = mra_cross(geom, cov, pred, leafP, geom.locs, geom.leaf)
    a = np.linalg.solve(V, np.asarray(z, dtype=np.float64))
    mean = Cps @ a
    var = cov.sigma2 - np.einsum("ij,ji->i", Cps, np.linalg.solve(V, Cps.T))
    return mean, var


def exact_krige(locs, z, cov_kind, theta, pred):
    """Simple kriging under the original process."""
    cov = Covariance(cov_kind, theta)
    V = cov(locs, locs) + cov.tau2 * np.eye(locs.shape[0])
    Cps = cov(pred, locs)
    mean = Cps @ np.linalg.solve(V, z)
    var = cov.sigma2 - np.einsum("ij,ji->i", Cps, np.linalg.solve(V, Cps.T))
    return mean, var


def mra_krige_joint_dense(geom, z, cov_kind, theta, pred):
    """Posterior predictive mean and joint covariance of the latent M-RA
    process at pred: C_M(P, S) Sigma^{-1} z and
    C_M(P, P) - C_M(P, S) Sigma^{-1} C_M(S, P), all from the chain closed form."""
    cov = Covariance(cov_kind, theta)
    V, _ = data_covariance(geom, cov)
    leafP = geom.leaf_of(pred)
    Cps, _ = mra_cross(geom, cov, pred, leafP, geom.locs, geom.leaf)
    Cpp, _ = mra_cross(geom, cov, pred, leafP, pred, leafP)
    mean = Cps @ np.linalg.solve(V, np.asarray(z, dtype=np.float64))
    Psi = Cpp - Cps @ np.linalg.solve(V, Cps.T)
    return mean, 0.5 * (Psi + Psi.T)


def exact_krige_joint(locs, z, cov_kind, theta, pred):
    """Joint simple kriging under the original process."""
    cov = Covariance(cov_kind, theta)
    V = cov(locs, locs) + cov.tau2 * np.eye(locs.shape[0])
    Cps = cov(pred, locs)
    mean = Cps @ np.linalg.solve(V, z)
    Psi = cov(pred, pred) - Cps @ np.linalg.solve(V, Cps.T)
    return mean, Psi
