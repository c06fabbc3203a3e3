"""Covariance functions C_0(s, s') = sigma^2 * rho(||s - s'|| / kappa).

Matern with smoothness 1.5: rho(h) = (1 + sqrt(3) h) exp(-sqrt(3) h)
(eq. mat15, Sec. 4.1; the form used for the satellite data, Sec. 4.2).
Exponential: rho(h) = exp(-h) (Sec. 4.1's two-dimensional study names an
"exponential covariance function" without a formula; read as the nu = 1/2
member of the same Matern family).

Parameters are theta = (log sigma^2, log kappa, log tau^2); tau^2 is the
measurement-error variance added to the leaf covariances only (Sec. 4.2).

Derivatives with respect to log kappa: with h = dist / kappa,
dh/dlog kappa = -h, so
  Matern 1.5:  dC/dlog kappa = sigma^2 * 3 h^2 exp(-sqrt(3) h)
  exponential: dC/dlog kappa = sigma^2 * h exp(-h)
and dC/dlog sigma^2 = C.
"""
from __future__ import annotations

import math

import numpy as np

SQRT3 = math.sqrt(3.0)


def _dist(X, Y):
    X = np.atleast_2d(X)
    Y = np.atleast_2d(Y)
    diff = X[:, None, :] - Y[None, :, :]
    return np.sqrt((diff * diff).sum(axis=-1))


class Covariance:
    def __init__(self, kind: str, theta):
        if kind not in ("matern32", "exponential"):
            raise ValueError("unknown covariance " + kind)
        theta = np.asarray(theta, dtype=np.float64)
        if not np.isfinite(theta).all():
            raise ValueError("non-finite parameter")
        self.kind = kind
        self.sigma2 = math.exp(theta[0])
        self.kappa = math.exp(theta[1])
        self.tau2 = math.exp(theta[2])

    def rho(self, h):
        if self.kind == "matern32":
            return (1.0 + SQRT3 * h) * np.exp(-SQRT3 * h)
        return np.exp(-h)

    def drho_dlogkappa(self, h):
        if self.kind == "matern32":
            return 3.0 * h * h * np.exp(-SQRT3 * h)
        return h * np.exp(-h)

    def __call__(self, X, Y):
        """C_0(X, Y), shape (len(X), len(Y))."""
        return self.sigma2 * self.rho(_dist(X, Y) / self.kappa)

    def tangents(self, X, Y):
        """(3, len(X), len(Y)): dC_0/d(log sigma^2, log kappa, log tau^2)."""
        h = _dist(X, Y) / self.kappa
        c = self.sigma2 * self.rho(h)
        dk = self.sigma2 * self.drho_dlogkappa(h)
        return np.stack([c, dk, np.zeros_like(c)])
