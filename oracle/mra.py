"""M-RA prior quantities, posterior recursion and log-likelihood (Sec. 3.1-3.3),
with an optional forward-mode (tangent) gradient.

Notation follows the paper.  For region R = (m, i) with ancestors
a_0, ..., a_m = R and point set Q_R (knots for m < M, the observations S_R
for m = M):

  eq. priorw      W^l_R = C_0(Q_R, Q_{a_l}) - sum_{k<l} W^k_R K_{a_k} W^k_{a_l}',
                  l = 0..m, with K_R^{-1} = W^m_R (m < M), B^l_R = W^l_R (l < M)
                  and, with measurement error (Sec. 4.2),
                  Sigma_R = W^M_R + tau^2 I at the leaves.
  eq. helpquantities at m = M (computed from the definition):
                  A~^{k,l} = B^k' Sigma^{-1} B^l, w~^k = B^k' Sigma^{-1} z,
                  d = log|Sigma|, u = z' Sigma^{-1} z.
  eq. mainquantities: A^{k,l}_R = sum over children of A~^{k,l},
                  w^k_R = sum over children of w~^k.
  eq. posterior:  K~^{-1} = K^{-1} + A^{m,m}.
  Sec. 3.3:       d_R = log|K~^{-1}| - log|K^{-1}| + sum_children d,
                  u_R = -w^m' K~ w^m + sum_children u.
  eq. helpquantities (recursive form):
                  A~^{k,l} = A^{k,l} - A^{k,m} K~ A^{m,l},
                  w~^k = w^k - A^{k,m} K~ w^m,   k >= l, k, l < m.
  Sec. 3.3:       -2 log L = d_root + u_root; the returned log-likelihood
                  also carries the Gaussian constant -(n/2) log(2 pi).

K is applied through Cholesky solves of K^{-1} (never an explicit inverse).

The gradient with respect to theta = (log sigma^2, log kappa, log tau^2) is
propagated forward: every quantity carries its three tangents, updated with
d(XY) = dX Y + X dY, d(K Y) = K (dY - d(K^{-1}) K Y),
d log|A| = tr(A^{-1} dA), dC_0/dlog sigma^2 = C_0, dC_0/dlog kappa from
covariance.py and dSigma_R/dlog tau^2 = tau^2 I.
"""
from __future__ import annotations

import math

import numpy as np
from scipy.linalg import cho_factor, cho_solve

from .covariance import Covariance
from .geometry import Geometry

P = 3  # number of parameters


class Dual:
    """A value and (optionally) its P tangents, shape (P, *value.shape)."""
    __slots__ = ("v", "t")

    def __init__(self, v, t=None):
        self.v = v
        self.t = t

    @property
    def T(self):
        return Dual(self.v.T, None if self.t is None else np.swapaxes(self.t, -1, -2))

    def __add__(self, o):
        return Dual(self.v + o.v, _tadd(self.t, o.t))

    def __sub__(self, o):
        return Dual(self.v - o.v, _tadd(self.t, None if o.t is None else -o.t))

    def __matmul__(self, o):
        t = None
        if self.t is not None:
            t = self.t @ o.v
        if o.t is not None:
            t = _tadd(t, self.v @ o.t)
        return Dual(self.v @ o.v, t)

    def __neg__(self):
        return Dual(-self.v, None if self.t is None else -self.t)


def _tadd(a, b):
    if a is None:
        return b
    if b is None:
        return a
    return a + b


class SPD:
    """A symmetric positive-definite Dual matrix A kept as its Cholesky
    factorisation, for applying A^{-1} and taking log|A|."""

    def __init__(self, A: Dual):
        self.A = A
        self.empty = A.v.shape[0] == 0
        self.c = None if self.empty else cho_factor(A.v, lower=True)

    def solve(self, Y: Dual) -> Dual:
        """A^{-1} Y with tangent A^{-1} (dY - dA A^{-1} Y)."""
        if self.empty:
            return Dual(np.zeros(Y.v.shape), None if Y.t is None else np.zeros(Y.t.shape))
        X = cho_solve(self.c, Y.v)
        t = None
        if Y.t is not None or self.A.t is not None:
            rhs = np.zeros((P,) + X.shape) if Y.t is None else Y.t.copy()
            if self.A.t is not None:
                rhs = rhs - self.A.t @ X
            t = np.stack([cho_solve(self.c, rhs[p]) for p in range(P)])
        return Dual(X, t)

    def logdet(self) -> Dual:
        if self.empty:
            return Dual(np.float64(0.0), None if self.A.t is None else np.zeros(P))
        v = 2.0 * np.log(np.diag(self.c[0])).sum()
        t = None
        if self.A.t is not None:
            t = np.array([np.trace(cho_solve(self.c, self.A.t[p])) for p in range(P)])
        return Dual(np.float64(v), t)


def _cov_dual(cov: Covariance, X, Y, grad: bool) -> Dual:
    if grad:
        t = cov.tangents(X, Y)
        return Dual(t[0].copy(), t)
    return Dual(cov(X, Y))


class MRAState:
    """Everything the recursion produced (for prediction and inspection)."""

    def __init__(self):
        self.W = {}        # (m, i) -> [W^0..W^m] (Dual)
        self.Kinv = {}     # (m, i) -> SPD(W^m), m < M
        self.Sigma = {}    # leaf i -> SPD(Sigma_R)
        self.A = {}        # (m, i) -> {(k, l): A^{k,l}}, m < M
        self.omega = {}    # (m, i) -> [w^0..w^m]
        self.Ktilde = {}   # (m, i) -> SPD(K~^{-1})
        self.d = {}        # (m, i) -> Dual scalar
        self.u = {}


def prior_region(geom: Geometry, cov: Covariance, st: MRAState, m: int, i: int, grad: bool):
    """eq. priorw for region (m, i); ancestors' W and K must be present."""
    anc = geom.ancestors(m, i)
    Q = geom.region_points(m, i)
    Ws = []
    for l in range(m + 1):
        Ql = Q if l == m else geom.knots[l][anc[l]]
        w = _cov_dual(cov, Q, Ql, grad)
        for k in range(l):
            Wk_al = Ws[k] if l == m else st.W[(l, anc[l])][k]
            w = w - Ws[k] @ st.Kinv[(k, anc[k])].solve(Wk_al.T)
        Ws.append(w)
    return Ws


def leaf_quantities(geom, cov, Ws, zR, grad):
    """eq. helpquantities at m = M from the definition, plus d and u."""
    M = geom.M
    nR = zR.shape[0]
    tau2 = Dual(cov.tau2 * np.eye(nR),
                np.stack([np.zeros((nR, nR)), np.zeros((nR, nR)), cov.tau2 * np.eye(nR)]) if grad else None)
    Sig = SPD(Ws[M] + tau2)
    zD = Dual(zR.reshape(-1, 1))
    Sz = Sig.solve(zD)
    SB = [Sig.solve(Ws[l]) for l in range(M)]
    At = {}
    for k in range(M):
        for l in range(k + 1):
            At[(k, l)] = Ws[k].T @ SB[l]
    om = [Ws[k].T @ Sz for k in range(M)]
    u = zD.T @ Sz
    return Sig, At, om, Sig.logdet(), Dual(u.v[0, 0], None if u.t is None else u.t[:, 0, 0])


def _zero_like_blocks(M, rl, grad):
    """Leaf quantities of an empty leaf: A~^{k,l} (r_k x r_l), w~^k (r_k), d, u."""
    def z(shape):
        return Dual(np.zeros(shape), np.zeros((P,) + shape) if grad else None)
    At = {(k, l): z((rl[k], rl[l])) for k in range(M) for l in range(k + 1)}
    om = [z((rl[k], 1)) for k in range(M)]
    return At, om, z(()), z(())


def loglik(geom: Geometry, z, cov_kind: str, theta, grad: bool = False, keep: bool = False,
           child_order: str = "forward"):
    """M-RA log-likelihood (and its gradient in log-parameters).

    Returns (loglik, grad or None, state).  z is in the original order of
    the locations given to geom.  state holds the recursion's quantities when
    keep is True (prediction needs them).  child_order = "reversed" visits
    the regions of each level, and so sums every parent's children, in the
    opposite order: an equally valid operation order, used to measure the
    rounding spread of the result.
    """
    if child_order not in ("forward", "reversed"):
        raise ValueError("child_order must be 'forward' or 'reversed'")
    order = (lambda n: range(n)) if child_order == "forward" else (lambda n: range(n - 1, -1, -1))
    cov = Covariance(cov_kind, theta)
    M, nreg = geom.M, geom.nreg
    z = np.asarray(z, dtype=np.float64)
    st = MRAState()
    # prior quantities of the internal levels, top-down (eq. priorw)
    for m in range(M):
        for i in range(nreg[m]):
            Ws = prior_region(geom, cov, st, m, i, grad)
            st.W[(m, i)] = Ws
            st.Kinv[(m, i)] = SPD(Ws[m])
    # leaves and the first posterior level: each level-(M-1) region sums its
    # children's leaf quantities (eq. mainquantities)
    child_sum = {}
    for i in order(nreg[M]):
        Ws = prior_region(geom, cov, st, M, i, grad)
        zR = z[geom.leaf_obs(i)]
        if zR.shape[0] == 0:
            At, om, dR, uR = _zero_like_blocks(M, geom.rl, grad)
            Sig = None
        else:
            Sig, At, om, dR, uR = leaf_quantities(geom, cov, Ws, zR, grad)
        if keep:
            st.W[(M, i)] = Ws
            st.Sigma[i] = Sig
        st.d[(M, i)], st.u[(M, i)] = dR, uR
        _accumulate(child_sum, (M - 1, geom.parent(M, i)) if M > 0 else None, At, om, dR, uR)
    if M == 0:
        ll = -0.5 * (st.d[(0, 0)] + st.u[(0, 0)]).v - 0.5 * geom.locs.shape[0] * math.log(2 * math.pi)
        g = None if not grad else -0.5 * (st.d[(0, 0)].t + st.u[(0, 0)].t)
        return ll, g, st
    # posterior recursion, bottom-up (eq. posterior, helpquantities, Sec. 3.3)
    for m in range(M - 1, -1, -1):
        for i in order(nreg[m]):
            A, om, dsum, usum = child_sum.pop((m, i))
            Kinv = st.Kinv[(m, i)]
            Kt = SPD(Kinv.A + A[(m, m)])
            dR = Kt.logdet() - Kinv.logdet() + dsum
            Ktw = Kt.solve(om[m])
            uq = om[m].T @ Ktw
            uR = Dual(-uq.v[0, 0], None if uq.t is None else -uq.t[:, 0, 0]) + usum
            st.d[(m, i)], st.u[(m, i)] = dR, uR
            if keep:
                st.A[(m, i)], st.omega[(m, i)], st.Ktilde[(m, i)] = A, om, Kt
            if m == 0:
                continue
            Am = [A[(m, l)] for l in range(m)]           # A^{m,l}, l < m
            KtAm = [Kt.solve(Am[l]) for l in range(m)]   # K~ A^{m,l}
            At = {}
            for k in range(m):
                for l in range(k + 1):
                    At[(k, l)] = A[(k, l)] - Am[k].T @ KtAm[l]
            omt = [om[k] - Am[k].T @ Ktw for k in range(m)]
            _accumulate(child_sum, (m - 1, geom.parent(m, i)), At, omt, dR, uR)
    root_d, root_u = st.d[(0, 0)], st.u[(0, 0)]
    n = geom.locs.shape[0]
    ll = -0.5 * (root_d.v + root_u.v) - 0.5 * n * math.log(2 * math.pi)
    g = None if not grad else -0.5 * (root_d.t + root_u.t)
    return float(ll), g, st


def _accumulate(child_sum, key, At, om, dR, uR):
    """Sum of children in child order (eq. mainquantities and the d, u sums)."""
    if key is None:
        return
    if key not in child_sum:
        child_sum[key] = ({kl: Dual(v.v.copy(), None if v.t is None else v.t.copy()) for kl, v in At.items()},
                          [Dual(w.v.copy(), None if w.t is None else w.t.copy()) for w in om],
                          dR, uR)
        return
    A, o, d, u = child_sum[key]
    for kl in A:
        A[kl] = A[kl] + At[kl]
    for k in range(len(o)):
        o[k] = o[k] + om[k]
    child_sum[key] = (A, o, d + dR, u + uR)


def _dual_scalar_add(a: Dual, b: Dual) -> Dual:
    return Dual(a.v + b.v, _tadd(a.t, b.t))


def d_u(geom, z, cov_kind, theta):
    """(d_root, u_root): the two parts of -2 log L without the constant."""
    _, _, st = loglik(geom, z, cov_kind, theta, grad=False)
    return float(st.d[(0, 0)].v), float(st.u[(0, 0)].v)
