"""Maximum-likelihood estimation of theta = (log sigma^2, log kappa,
log tau^2) for the M-RA.  The paper infers the covariance parameters by
numerically maximising the log-likelihood of Sec. 3.3; this driver does so
with the library's log-likelihood and reverse-pass gradient.

Method: limited-memory BFGS (Nocedal and Wright, Numerical Optimization,
2nd ed., Sec. 7.2: the two-loop recursion with the scaled initial matrix
gamma I, gamma = s'y / y'y) on f = -loglik, with a batched backtracking line
search.  Each iteration evaluates the log-likelihood and gradient at k step
lengths alpha_j = alpha_0 shrink^j, j = 0..k-1, in one call (the parameter
batch of the library), and keeps the best trial point that satisfies the
Armijo condition f(theta + alpha d) <= f(theta) + c1 alpha grad f' d.  The
accepted point arrives with its gradient, so an iteration costs one call
unless no trial passes (then a further batch of shorter steps).  A trial
whose factorisation breaks down (NaN log-likelihood) counts as failing.

Only host logic over 3-vectors lives here; every likelihood evaluation runs
in the library's kernels.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np


@dataclass
class FitResult:
    theta: np.ndarray            # (3,) maximiser found
    loglik: float
    grad: np.ndarray             # (3,) gradient at theta
    iterations: int
    calls: int                   # batched evaluation calls
    evaluations: int             # parameter vectors evaluated
    converged: bool
    message: str
    history: list = field(default_factory=list)   # (iteration, loglik, max |grad|)


def maximize(evaluate, theta0, *, batch: int = 4, memory: int = 8, max_iter: int = 100, gtol: float = 1e-9,
             ftol: float = 1e-14, c1: float = 1e-4, shrink: float = 0.5, max_step: float = 2.0,
             max_backtracks: int = 4) -> FitResult:
    """Maximise a log-likelihood by L-BFGS with a batched line search.

    evaluate(thetas) takes a (k, 3) float64 array and returns (loglik [k],
    grad [k, 3]) as numpy arrays; NaN entries mark failed evaluations.
    Stops when max |grad| <= gtol max(1, |loglik|), when an accepted step
    changes the log-likelihood by at most ftol max(1, |loglik|), or after
    max_iter iterations.  max_step bounds the largest component of a trial
    step (log scale), batch the trial points per call.
    """
    if batch < 1 or memory < 1 or not (0.0 < shrink < 1.0) or max_step <= 0.0:
        raise ValueError("batch >= 1, memory >= 1, 0 < shrink < 1 and max_step > 0 are required")
    theta = np.asarray(theta0, dtype=np.float64).reshape(3).copy()
    ll, g = evaluate(theta[None])
    ll, g = float(ll[0]), np.asarray(g[0], dtype=np.float64)
    calls, evals = 1, 1
    if not np.isfinite(ll) or not np.isfinite(g).all():
        return FitResult(theta, ll, g, 0, calls, evals, False, "log-likelihood not finite at the start")
    S, Y = [], []   # curvature pairs of f = -loglik: s = step, y = change of grad f
    hist = [(0, ll, float(np.abs(g).max()))]
    it = 0
    msg = "maximum number of iterations reached"
    converged = False
    while it < max_iter:
        if np.abs(g).max() <= gtol * max(1.0, abs(ll)):
            converged, msg = True, "gradient tolerance reached"
            break
        # two-loop recursion: d = -H grad f = H g
        q = -g.copy()
        alphas = []
        for s, y in zip(reversed(S), reversed(Y)):
            a = (s @ q) / (y @ s)
            alphas.append(a)
            q -= a * y
        gamma = (S[-1] @ Y[-1]) / (Y[-1] @ Y[-1]) if S else 1.0 / max(np.abs(g).max(), 1e-300)
        r = gamma * q
        for (s, y), a in zip(zip(S, Y), reversed(alphas)):
            b = (y @ r) / (y @ s)
            r += (a - b) * s
        d = -r
        slope = g @ d                          # directional derivative of loglik, > 0 for ascent
        if not slope > 0.0:                    # not an ascent direction: restart from the gradient
            S.clear()
            Y.clear()
            d = g / max(np.abs(g).max(), 1e-300)
            slope = g @ d
        a0 = min(1.0, max_step / np.abs(d).max())
        accepted = None
        for _ in range(max_backtracks):
            steps = a0 * shrink ** np.arange(batch)
            trial = theta[None, :] + steps[:, None] * d[None, :]
            tl, tg = evaluate(trial)
            calls += 1
            evals += batch
            tl = np.asarray(tl, dtype=np.float64)
            ok = np.isfinite(tl) & (tl >= ll + c1 * steps * slope) & np.isfinite(np.asarray(tg)).all(axis=1)
            if ok.any():
                j = int(np.flatnonzero(ok)[np.argmax(tl[ok])])
                accepted = (trial[j], float(tl[j]), np.asarray(tg[j], dtype=np.float64))
                break
            a0 = steps[-1] * shrink
        if accepted is None:
            msg = "line search found no point of sufficient increase"
            break
        it += 1
        th_new, ll_new, g_new = accepted
        s = th_new - theta
        y = -(g_new - g)
        if s @ y > 1e-12 * np.linalg.norm(s) * np.linalg.norm(y):
            S.append(s)
            Y.append(y)
            if len(S) > memory:
                S.pop(0)
                Y.pop(0)
        dl = ll_new - ll
        theta, ll, g = th_new, ll_new, g_new
        hist.append((it, ll, float(np.abs(g).max())))
        if abs(dl) <= ftol * max(1.0, abs(ll)):
            converged, msg = True, "relative change of the log-likelihood below ftol"
            break
    if not converged and np.abs(g).max() <= gtol * max(1.0, abs(ll)):
        converged, msg = True, "gradient tolerance reached"
    return FitResult(theta, ll, g, it, calls, evals, converged, msg, hist)
