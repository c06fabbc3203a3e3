"""Posterior predictive mean and variance of the latent M-RA process
(Sec. 3.4 and Prop. 2), in the paper's notation.

For prediction locations S^P in leaf R = (M, i) with ancestors a_0..a_M = R:
  U^l   = C_0(S^P, Q_{a_l}) - sum_{k<l} U^k K_{a_k} W^k_{a_l}',  l = 0..M,
          where Q_{a_M} = S_R and W^k_{a_M} = B^k_R;   L^M = U^M
  V^P   = C_0(S^P, S^P) - sum_{k=0}^{M-1} U^k K_{a_k} U^k'
          (the sum's upper limit is printed as l-1 with l undefined; read as M-1)
  B~^{M,k} = U^k - L^M Sigma_R^{-1} B^k_R                      (eq. bfrecursion, l = M)
  B~^{l,k} = B~^{l+1,k} - B~^{l+1,l} K~_{a_l} A^{l,k}_{a_l},  l = M-1..1, k < l
  mean  = sum_{m<M} B~^{m+1,m} K~_{a_m} w^m_{a_m} + L^M Sigma_R^{-1} z_R
  var   = diag( sum_{m<M} B~^{m+1,m} K~_{a_m} B~^{m+1,m}' + V^P - L^M Sigma_R^{-1} L^M' )
(eq. prediction: weights eta~_m ~ N(K~ w^m, K~), remainder delta~ with the
mean and covariance of Prop. 2).  predict() returns the marginal variances,
predict_joint() the joint covariance matrix.
"""
from __future__ import annotations

import numpy as np
from scipy.linalg import cho_solve

from .covariance import Covariance
from .geometry import Geometry
from .mra import loglik


def predict(geom: Geometry, z, cov_kind, theta, pred):
    """(mean, var) of y_M at pred given z (Prop. 2)."""
    cov = Covariance(cov_kind, theta)
    _, _, st = loglik(geom, z, cov_kind, theta, grad=False, keep=True)
    M = geom.M
    z = np.asarray(z, dtype=np.float64)
    pred = np.atleast_2d(np.asarray(pred, dtype=np.float64))
    leafP = geom.leaf_of(pred)
    mean = np.zeros(pred.shape[0])
    var = np.zeros(pred.shape[0])
    for i in np.unique(leafP):
        ip = np.flatnonzero(leafP == i)
        SP = pred[ip]
        anc = geom.ancestors(M, int(i))
        SR = geom.region_points(M, int(i))
        zR = z[geom.leaf_obs(int(i))]
        WR = st.W[(M, int(i))]
        U = []
        for l in range(M + 1):
            Ql = SR if l == M else geom.knots[l][anc[l]]
            u = cov(SP, Ql)
            for k in range(l):
                Wk_al = WR[k] if l == M else st.W[(l, anc[l])][k]
                u = u - U[k] @ cho_solve(st.Kinv[(k, anc[k])].c, Wk_al.v.T) \
                    if st.Kinv[(k, anc[k])].c is not None else u
            U.append(u)
        LM = U[M]
        VP = np.diag(cov(SP, SP)).copy()
        for k in range(M):
            if st.Kinv[(k, anc[k])].c is None:
                continue
            VP -= np.einsum("ij,ji->i", U[k], cho_solve(st.Kinv[(k, anc[k])].c, U[k].T))
        Sig = st.Sigma[int(i)]
        if Sig is not None and Sig.c is not None:
            SiB = [cho_solve(Sig.c, WR[k].v) for k in range(M)]
            Siz = cho_solve(Sig.c, zR)
            SiL = cho_solve(Sig.c, LM.T)
            Bt = {(M, k): U[k] - LM @ SiB[k] for k in range(M)}
            m_leaf = LM @ Siz
            v_leaf = VP - np.einsum("ij,ji->i", LM, SiL)
        else:
            Bt = {(M, k): U[k] for k in range(M)}
            m_leaf = np.zeros(SP.shape[0])
            v_leaf = VP
        for l in range(M - 1, 0, -1):
            Kt = st.Ktilde[(l, anc[l])]
            for k in range(l):
                Bt[(l, k)] = Bt[(l + 1, k)] - Bt[(l + 1, l)] @ cho_solve(Kt.c, st.A[(l, anc[l])][(l, k)].v) \
                    if Kt.c is not None else Bt[(l + 1, k)]
        mu = m_leaf.copy()
        vv = v_leaf.copy()
        for m in range(M):
            Kt = st.Ktilde[(m, anc[m])]
            if Kt.c is None:
                continue
            Bm = Bt[(m + 1, m)]
            mu += (Bm @ cho_solve(Kt.c, st.omega[(m, anc[m])][m].v)).ravel()
            vv += np.einsum("ij,ji->i", Bm, cho_solve(Kt.c, Bm.T))
        mean[ip] = mu
        var[ip] = vv
    return mean, var


def predict_joint(geom: Geometry, z, cov_kind, theta, pred):
    """(mean, Psi): posterior predictive mean and JOINT covariance of y_M at
    pred given z, from Prop. 2.  The posterior predictive has the M-RA form
    sum_{m<M} B~^{m+1,m} eta~_{a_m} + delta~ with independent weights
    eta~_{a_m} ~ N(K~ w^m, K~) per region and an independent remainder
    delta~ ~ N(L^M Sigma^{-1} z_R, V^P - L^M Sigma^{-1} L^M') per leaf, so
      Psi(s, s') = sum over the levels m < M at which s and s' share the
                   region a_m of  B~^{m+1,m}(s) K~_{a_m} B~^{m+1,m}(s')'
                 + [s, s' in the same leaf] (V^P - L^M Sigma^{-1} L^M')(s, s'),
    with V^P the full block C_0(S^P, S^P) - sum_{k<M} U^k K_{a_k} U^k' (the
    printed upper limit of that sum read as M - 1).  The quantities are those
    of predict(), kept as full blocks instead of diagonals."""
    cov = Covariance(cov_kind, theta)
    _, _, st = loglik(geom, z, cov_kind, theta, grad=False, keep=True)
    M = geom.M
    z = np.asarray(z, dtype=np.float64)
    pred = np.atleast_2d(np.asarray(pred, dtype=np.float64))
    leafP = geom.leaf_of(pred)
    npred = pred.shape[0]
    mean = np.zeros(npred)
    Psi = np.zeros((npred, npred))
    leaves = np.unique(leafP)
    idx = {}
    fac = {}     # leaf -> [B~^{m+1,m} for m < M]
    for i in leaves:
        i = int(i)
        ip = np.flatnonzero(leafP == i)
        idx[i] = ip
        SP = pred[ip]
        anc = geom.ancestors(M, i)
        SR = geom.region_points(M, i)
        zR = z[geom.leaf_obs(i)]
        WR = st.W[(M, i)]
        U = []
        for l in range(M + 1):
            Ql = SR if l == M else geom.knots[l][anc[l]]
            u = cov(SP, Ql)
            for k in range(l):
                Wk_al = WR[k] if l == M else st.W[(l, anc[l])][k]
                u = u - U[k] @ cho_solve(st.Kinv[(k, anc[k])].c, Wk_al.v.T)
            U.append(u)
        LM = U[M]
        VP = cov(SP, SP)
        for k in range(M):
            VP = VP - U[k] @ cho_solve(st.Kinv[(k, anc[k])].c, U[k].T)
        Sig = st.Sigma[i]
        if Sig is not None and Sig.c is not None:
            Bt = {(M, k): U[k] - LM @ cho_solve(Sig.c, WR[k].v) for k in range(M)}
            m_leaf = LM @ cho_solve(Sig.c, zR)
            C_leaf = VP - LM @ cho_solve(Sig.c, LM.T)
        else:
            Bt = {(M, k): U[k] for k in range(M)}
            m_leaf = np.zeros(SP.shape[0])
            C_leaf = VP
        for l in range(M - 1, 0, -1):
            Kt = st.Ktilde[(l, anc[l])] if (l, anc[l]) in st.Ktilde else None
            for k in range(l):
                Bt[(l, k)] = (Bt[(l + 1, k)] - Bt[(l + 1, l)] @ cho_solve(Kt.c, st.A[(l, anc[l])][(l, k)].v)
                              if Kt is not None and Kt.c is not None else Bt[(l + 1, k)])
        mu = m_leaf.copy()
        for m in range(M):
            Kt = st.Ktilde[(m, anc[m])]
            if Kt.c is None:
                continue
            mu += (Bt[(m + 1, m)] @ cho_solve(Kt.c, st.omega[(m, anc[m])][m].v)).ravel()
        mean[ip] = mu
        Psi[np.ix_(ip, ip)] += C_leaf
        fac[i] = [Bt[(m + 1, m)] for m in range(M)]
    for i in leaves:
        i = int(i)
        for j in leaves:
            j = int(j)
            ai, aj = geom.ancestors(M, i), geom.ancestors(M, j)
            for m in range(M):
                if ai[m] != aj[m]:
                    break
                Kt = st.Ktilde[(m, ai[m])]
                Psi[np.ix_(idx[i], idx[j])] += fac[i][m] @ cho_solve(Kt.c, fac[j][m].T)
    return mean, Psi


def data_gradient(geom: Geometry, z, cov_kind, theta, idx=None):
    """d loglik / d z = -Sigma^{-1} z at the observations idx (all when None).

    Sigma = C_M(S, S) + tau^2 I is the M-RA data covariance (measurement
    error as in Sec. 4.2), and C_M(S, S) is the covariance of the latent
    y_M at S.  The posterior mean of Prop. 2 at the observed locations is
    therefore E[y_M(S) | z] = C_M(S, S) Sigma^{-1} z = z - tau^2 Sigma^{-1} z,
    so -Sigma^{-1} z = (E[y_M(S) | z] - z) / tau^2: the gradient is the
    scaled residual of the kriging pass (Sec. 3.4) run at S itself.
    """
    z = np.asarray(z, dtype=np.float64)
    idx = np.arange(z.shape[0]) if idx is None else np.asarray(idx, dtype=np.int64)
    cov = Covariance(cov_kind, theta)
    mean, _ = predict(geom, z, cov_kind, theta, geom.locs[idx])
    return (mean - z[idx]) / cov.tau2


def gls(geom: Geometry, z, X, cov_kind, theta):
    """Generalised least squares for a mean trend z = X beta + (M-RA field
    with measurement error): beta = (X' Sigma^{-1} X)^{-1} X' Sigma^{-1} z,
    the profile log-likelihood loglik(z - X beta; theta) and its gradient in
    the log-parameters.  The paper removes the mean before the M-RA and
    states the model for a zero-mean field; a linear trend is the usual
    estimator of that mean.  By the envelope theorem the profile gradient is
    the gradient at the fixed residual (beta maximises the likelihood for
    every theta).  Sigma^{-1} v comes from data_gradient (Prop. 2), the
    likelihood and its gradient from mra.loglik (Sec. 3.3).

    Returns (beta, loglik, grad, XtSiX).
    """
    z = np.asarray(z, dtype=np.float64)
    X = np.asarray(X, dtype=np.float64).reshape(z.shape[0], -1)
    SiX = np.stack([-data_gradient(geom, X[:, j], cov_kind, theta) for j in range(X.shape[1])], axis=1)
    XtSiX = X.T @ SiX
    XtSiz = SiX.T @ z
    beta = np.linalg.solve(XtSiX, XtSiz)
    ll, g, _ = loglik(geom, z - X @ beta, cov_kind, theta, grad=True)
    return beta, ll, g, XtSiX
