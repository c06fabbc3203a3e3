"""MI355X-native multi-resolution approximation (M-RA) of Gaussian processes.

FP64 log-likelihood, its gradient in (log sigma^2, log kappa, log tau^2) and
kriging for the M-RA of Katzfuss (JASA 2017, arXiv 1507.04789), computed by
hand-written HIP kernels for gfx950 behind the C ABI of include/mra.h.  This
module only marshals arguments: device memory and streams come from torch.
"""
from __future__ import annotations

import ctypes as C
import math

import numpy as np

from . import _lib
from ._lib import MRA_CHECKPOINT, MRA_GRAPH, MRA_JOINT, MRA_NO_GRAD, MRA_PLAIN, MRA_SYNC, MRAError

__all__ = ["Plan", "MRALogLik", "MRAError", "MRA_SYNC", "MRA_PLAIN", "MRA_GRAPH", "MRA_NO_GRAD", "MRA_CHECKPOINT",
           "MRA_JOINT"]

_COV = {"exponential": _lib.MRA_COV_EXPONENTIAL, "matern32": _lib.MRA_COV_MATERN32}


def _torch():
    import torch
    return torch


class Plan:
    """A built M-RA plan.

    locs: (n, d) float64 observation locations; pred: optional (n_pred, d)
    prediction locations; knots: optional explicit knots, a list over levels
    m < M of arrays (regions of level m, r_m, d); chunks: leaf chunks of an
    MRA_CHECKPOINT plan (0: the library's default); J_levels (J_1..J_M) and
    r_levels (r_0..r_{M-1}): children and knots per level instead of J and
    r; adaptive: split values at quantiles of the observations (see
    mra_config in include/mra.h).  The geometry is built on the host; device
    arenas are allocated with torch and bound on first use (or bind()).
    """

    def __init__(self, locs, *, M: int, J: int, r: int, cov: str, d: int | None = None,
                 lo=None, hi=None, pred=None, knots=None, max_theta: int = 1,
                 flags: int = MRA_SYNC, chunks: int = 0, J_levels=None, r_levels=None,
                 adaptive: bool = False):
        L = _lib.lib()
        locs = np.ascontiguousarray(np.asarray(locs, dtype=np.float64))
        if locs.ndim == 1:
            locs = locs[:, None]
        d = locs.shape[1] if d is None else d
        self.n, self.d, self.M, self.J, self.r = locs.shape[0], d, M, J, r
        cfg = _lib.Config()
        cfg.d, cfg.M, cfg.J, cfg.r = d, M, J, r
        lo = [0.0] * d if lo is None else list(lo)
        hi = [1.0] * d if hi is None else list(hi)
        for a in range(2):
            cfg.lo[a] = lo[a] if a < d else 0.0
            cfg.hi[a] = hi[a] if a < d else 0.0
        cfg.cov = _COV[cov]
        cfg.max_theta = max_theta
        cfg.flags = flags
        cfg.chunks = chunks
        self.Jl = [1] + [int(x) for x in (J_levels if J_levels is not None else [J] * M)]
        self.rl = [int(x) for x in (r_levels if r_levels is not None else [r] * M)]
        if len(self.Jl) != M + 1 or len(self.rl) != M or M > 12:
            raise ValueError("J_levels and r_levels need M entries (M <= 11)")
        for m in range(M):
            cfg.J_level[m] = self.Jl[m + 1]
            cfg.r_level[m] = self.rl[m]
        cfg.adaptive = 1 if adaptive else 0
        self.nreg = [1]
        for m in range(1, M + 1):
            self.nreg.append(self.nreg[-1] * self.Jl[m])
        self.cfg = cfg
        self.cov = cov
        self.max_theta = max_theta
        self.flags = flags
        if pred is not None:
            pred = np.ascontiguousarray(np.asarray(pred, dtype=np.float64).reshape(-1, d))
        self.n_pred = 0 if pred is None else pred.shape[0]
        kn = None
        if knots is not None:
            kn = np.ascontiguousarray(np.concatenate([np.asarray(k, dtype=np.float64).reshape(-1) for k in knots]))
        h = C.c_void_p()
        s = L.mra_build(C.byref(cfg), locs.ctypes.data, self.n,
                        None if pred is None else pred.ctypes.data, self.n_pred,
                        None if kn is None else kn.ctypes.data, C.byref(h))
        _lib.check(s, "mra_build")
        self._h = h
        g, w = C.c_size_t(), C.c_size_t()
        _lib.check(L.mra_requirements(h, C.byref(g), C.byref(w)), "mra_requirements")
        self.geom_bytes, self.work_bytes = g.value, w.value
        info = _lib.Info()
        _lib.check(L.mra_get_info(h, C.byref(info)), "mra_get_info")
        self.info = {f: getattr(info, f) for f, _ in _lib.Info._fields_}
        self._geom = self._work = None
        self.device = None

    # -- host-side queries --------------------------------------------------
    def geometry(self):
        """(perm, leaf_offsets, knots) as built by the library; knots is a
        list over levels m < M of arrays (regions of level m, r_m, d)."""
        L = _lib.lib()
        perm = np.empty(self.n, dtype=np.int64)
        off = np.empty(self.nreg[self.M] + 1, dtype=np.int64)
        sizes = [self.nreg[m] * self.rl[m] * self.d for m in range(self.M)]
        kn = np.empty(max(sum(sizes), 1), dtype=np.float64)
        _lib.check(L.mra_get_geometry(self._h, perm.ctypes.data, off.ctypes.data, kn.ctypes.data), "mra_get_geometry")
        out, q = [], 0
        for m in range(self.M):
            out.append(kn[q:q + sizes[m]].reshape(self.nreg[m], self.rl[m], self.d))
            q += sizes[m]
        return perm, off, out

    # -- device ---------------------------------------------------------------
    def bind(self, device="cuda", work: bool = True):
        """Allocate the arenas on `device` and bind them.  work=False binds
        the geometry only (no work arena): then only loglik_grad_noalloc
        computes."""
        torch = _torch()
        dev = torch.device(device)
        if dev.type != "cuda":
            raise RuntimeError("the M-RA library runs on a GPU device only")
        self._geom = torch.empty(self.geom_bytes + 256, dtype=torch.uint8, device=dev)
        self._work = torch.empty(self.work_bytes + 256, dtype=torch.uint8, device=dev) if work else None
        gp = (self._geom.data_ptr() + 255) // 256 * 256
        wp = (self._work.data_ptr() + 255) // 256 * 256 if work else None
        st = torch.cuda.current_stream(dev).cuda_stream
        _lib.check(_lib.lib().mra_bind(self._h, gp, self.geom_bytes, wp, self.work_bytes if work else 0, st),
                   "mra_bind")
        self.device = dev
        return self

    def _ensure(self, t):
        if self.device is None:
            self.bind(t.device if t.is_cuda else "cuda")

    def _stream(self):
        return _torch().cuda.current_stream(self.device).cuda_stream

    def _prep(self, y, theta, rows=False):
        """Device tensors for (y, theta).  With rows=True, y may be (k, n):
        one data vector per parameter row (k = theta rows)."""
        torch = _torch()
        for name, t in (("y", y), ("theta", theta)):
            if isinstance(t, torch.Tensor) and t.dtype != torch.float64:
                raise TypeError("%s is %s: the library computes in FP64 and takes float64 tensors "
                                "(a narrower tensor has already lost precision)" % (name, t.dtype))
        y = torch.as_tensor(y, dtype=torch.float64)
        theta = torch.as_tensor(theta, dtype=torch.float64)
        if not y.is_cuda:
            y = y.to("cuda")
        self._ensure(y)
        y = y.to(self.device).contiguous()
        theta = theta.to(self.device).reshape(-1, 3).contiguous()
        if rows and y.dim() == 2 and y.shape[0] > 1:
            if y.shape != (theta.shape[0], self.n):
                raise ValueError("y rows %s do not match %d parameter rows x %d locations"
                                 % (tuple(y.shape), theta.shape[0], self.n))
        elif y.numel() != self.n:
            raise ValueError("y has %d entries, plan has %d locations" % (y.numel(), self.n))
        if theta.shape[0] > self.max_theta:
            raise ValueError("%d parameter vectors exceed max_theta=%d" % (theta.shape[0], self.max_theta))
        return y, theta

    def _fail(self, s, where):
        if s == _lib.MRA_ENOTPD:
            th, lv, rg = C.c_int32(), C.c_int32(), C.c_int64()
            _lib.lib().mra_last_failure(self._h, C.byref(th), C.byref(lv), C.byref(rg), self._stream())
            raise MRAError(s, where, ": theta %d, level %d, region %d" % (th.value, lv.value, rg.value))
        _lib.check(s, where)

    def _out(self, t, shape):
        torch = _torch()
        if t is None:
            return torch.empty(shape, dtype=torch.float64, device=self.device)
        if t.dtype != torch.float64 or tuple(t.shape) != tuple(shape) or not t.is_contiguous() or t.device != self.device:
            raise ValueError("output tensor must be contiguous float64 of shape %s on %s" % (shape, self.device))
        return t

    def loglik(self, y, theta, out=None):
        """Log-likelihood for each row of theta (n_theta x 3); `out`
        optionally names the output tensor (stable buffers let MRA_GRAPH
        plans replay one captured graph)."""
        y, theta = self._prep(y, theta)
        out = self._out(out, (theta.shape[0],))
        s = _lib.lib().mra_loglik(self._h, y.data_ptr(), theta.data_ptr(), theta.shape[0], out.data_ptr(),
                                  self._stream())
        self._fail(s, "mra_loglik")
        return out

    def loglik_grad(self, y, theta, out=None):
        """(loglik [n_theta], grad [n_theta, 3]); out = (loglik, grad)
        optionally names the output tensors."""
        y, theta = self._prep(y, theta)
        out, g = (None, None) if out is None else out
        out = self._out(out, (theta.shape[0],))
        g = self._out(g, (theta.shape[0], 3))
        s = _lib.lib().mra_loglik_grad(self._h, y.data_ptr(), theta.data_ptr(), theta.shape[0], out.data_ptr(),
                                       g.data_ptr(), self._stream())
        self._fail(s, "mra_loglik_grad")
        return out, g

    def loglik_grad_noalloc(self, y, theta, out):
        """As loglik_grad, through mra_loglik_grad_noalloc: the library's own
        scratch array stands in for the work arena and the call allocates
        nothing, so the outputs must be given: out = (loglik [n_theta],
        grad [n_theta, 3]) on the plan's device."""
        y, theta = self._prep(y, theta)
        ll, g = out
        ll = self._out(ll, (theta.shape[0],))
        g = self._out(g, (theta.shape[0], 3))
        s = _lib.lib().mra_loglik_grad_noalloc(self._h, y.data_ptr(), theta.data_ptr(), theta.shape[0],
                                               ll.data_ptr(), g.data_ptr(), self._stream())
        self._fail(s, "mra_loglik_grad_noalloc")
        return ll, g

    def loglik_grad_data(self, y, theta, out=None):
        """(loglik [n_theta], grad [n_theta, 3], grad_y [n_theta, n]), where
        grad_y = d loglik / d y = -Sigma^{-1} y in the caller's order, from
        the same reverse pass.  y is one data vector (n,) for all parameter
        rows, or (n_theta, n): one data vector per row.  out = (loglik, grad,
        grad_y) optionally names the output tensors."""
        y, theta = self._prep(y, theta, rows=True)
        stride = self.n if y.dim() == 2 and y.shape[0] > 1 else 0
        out, g, gy = (None, None, None) if out is None else out
        out = self._out(out, (theta.shape[0],))
        g = self._out(g, (theta.shape[0], 3))
        gy = self._out(gy, (theta.shape[0], self.n))
        s = _lib.lib().mra_loglik_grad_data(self._h, y.data_ptr(), stride, theta.data_ptr(), theta.shape[0],
                                            out.data_ptr(), g.data_ptr(), gy.data_ptr(), self._stream())
        self._fail(s, "mra_loglik_grad_data")
        return out, g, gy

    def gls(self, y, X, theta):
        """Generalised least-squares mean trend for data y = X beta + (M-RA
        field with measurement error) at one parameter vector theta (3,),
        through mra_gls: beta = (X' Sigma^{-1} X)^{-1} X' Sigma^{-1} y, the
        profile log-likelihood loglik(y - X beta; theta) and its gradient
        (the gradient at the fixed residual), from one forward pass that
        carries the trend columns beside y and one reverse pass.  X is
        (n, p) with 1 <= p <= 63.  Returns a dict of device tensors: beta
        (p,), loglik (1,), grad (3,), resid (n,), XtSiX (p, p)."""
        torch = _torch()
        y, theta = self._prep(y, theta)
        X = torch.as_tensor(X, dtype=torch.float64)
        if X.dim() == 1:
            X = X[:, None]
        if X.shape[0] != self.n:
            raise ValueError("X has %d rows, plan has %d locations" % (X.shape[0], self.n))
        p = X.shape[1]
        Xt = X.to(self.device).t().contiguous()      # [p][n]
        out = {"beta": torch.empty(p, dtype=torch.float64, device=self.device),
               "loglik": torch.empty(1, dtype=torch.float64, device=self.device),
               "grad": torch.empty(3, dtype=torch.float64, device=self.device),
               "resid": torch.empty(self.n, dtype=torch.float64, device=self.device),
               "XtSiX": torch.empty(p, p, dtype=torch.float64, device=self.device)}
        s = _lib.lib().mra_gls(self._h, y.data_ptr(), Xt.data_ptr(), p, theta[:1].data_ptr(),
                               out["beta"].data_ptr(), out["loglik"].data_ptr(), out["grad"].data_ptr(),
                               out["resid"].data_ptr(), out["XtSiX"].data_ptr(), self._stream())
        self._fail(s, "mra_gls")
        return out

    def fit(self, y, theta0, *, batch: int | None = None, **kw):
        """Maximum-likelihood estimate of (log sigma^2, log kappa, log tau^2)
        from theta0 by L-BFGS with a batched line search (mle.maximize):
        each iteration evaluates `batch` step lengths (default max_theta, at
        most 8) in one loglik_grad call.  Keyword arguments go to
        mle.maximize; returns its FitResult."""
        from . import mle
        torch = _torch()
        k = min(self.max_theta, 8) if batch is None else int(batch)
        if not 1 <= k <= self.max_theta:
            raise ValueError("batch must lie in 1..max_theta (%d)" % self.max_theta)
        y, _ = self._prep(y, np.zeros(3))
        bufs = {}

        def evaluate(th):
            m = th.shape[0]
            if m not in bufs:
                bufs[m] = tuple(torch.empty(s, dtype=torch.float64, device=self.device) for s in ((m, 3), (m,), (m, 3)))
            tb, lb, gb = bufs[m]
            tb.copy_(torch.from_numpy(np.ascontiguousarray(th, dtype=np.float64)))
            try:
                self.loglik_grad(y, tb, out=(lb, gb))
            except MRAError as e:   # a failed factorisation leaves NaN in its entries only
                if e.status != _lib.MRA_ENOTPD:
                    raise
            return lb.cpu().numpy(), gb.cpu().numpy()

        return mle.maximize(evaluate, theta0, batch=k, **kw)

    def predict(self, y, theta, out=None):
        """Posterior predictive (mean, var) of the latent process at the
        plan's prediction locations, for one parameter vector; out =
        (mean, var) optionally names the output tensors."""
        y, theta = self._prep(y, theta)
        mean, var = (None, None) if out is None else out
        mean = self._out(mean, (self.n_pred,))
        var = self._out(var, (self.n_pred,))
        s = _lib.lib().mra_predict(self._h, y.data_ptr(), theta[:1].data_ptr(), mean.data_ptr(), var.data_ptr(),
                                   self._stream())
        self._fail(s, "mra_predict")
        return mean, var

    def predict_cov(self, y, theta):
        """(mean [n_pred], cov [n_pred, n_pred]): posterior predictive mean
        and joint covariance of the latent process at the prediction
        locations (Prop. 2), for one parameter vector; needs an MRA_JOINT
        plan."""
        torch = _torch()
        y, theta = self._prep(y, theta)
        mean = torch.empty(self.n_pred, dtype=torch.float64, device=self.device)
        cov = torch.empty(self.n_pred, self.n_pred, dtype=torch.float64, device=self.device)
        s = _lib.lib().mra_predict_cov(self._h, y.data_ptr(), theta[:1].data_ptr(), mean.data_ptr(), cov.data_ptr(),
                                       self._stream())
        self._fail(s, "mra_predict_cov")
        return mean, cov

    def simulate(self, y, theta, eps):
        """Conditional draws of the latent process at the prediction
        locations given y (Prop. 2), one per row of the standard normals
        eps (n_draws <= 64, each row info["n_sim_normals"] long: 64 per
        region below level M, then one per prediction location); returns
        (n_draws, n_pred).  Needs an MRA_JOINT plan."""
        torch = _torch()
        y, theta = self._prep(y, theta)
        eps = torch.as_tensor(eps, dtype=torch.float64).to(self.device)
        if eps.dim() == 1:
            eps = eps[None]
        eps = eps.contiguous()
        out = torch.empty(eps.shape[0], self.n_pred, dtype=torch.float64, device=self.device)
        s = _lib.lib().mra_simulate(self._h, y.data_ptr(), theta[:1].data_ptr(), eps.data_ptr(), eps.shape[1],
                                    eps.shape[0], out.data_ptr(), self._stream())
        self._fail(s, "mra_simulate")
        return out

    # -- autotuning -------------------------------------------------------------
    def autotune(self, y, theta, reps: int = 3):
        """Time the launch shapes of every kernel family on this data and keep
        the fastest (results do not depend on the shapes); returns the table."""
        import json
        torch = _torch()
        y, theta = self._prep(y, theta)
        ll = torch.empty(theta.shape[0], dtype=torch.float64, device=self.device)
        g = torch.empty(theta.shape[0], 3, dtype=torch.float64, device=self.device)
        buf = C.create_string_buffer(8192)
        n = C.c_size_t()
        s = _lib.lib().mra_autotune(self._h, y.data_ptr(), theta.data_ptr(), theta.shape[0], ll.data_ptr(),
                                    g.data_ptr(), reps, buf, len(buf), C.byref(n), self._stream())
        self._fail(s, "mra_autotune")
        return json.loads(buf.value.decode())

    def tuning(self):
        """The current tuning table."""
        import json
        buf = C.create_string_buffer(8192)
        n = C.c_size_t()
        _lib.check(_lib.lib().mra_get_tuning(self._h, buf, len(buf), C.byref(n)), "mra_get_tuning")
        return json.loads(buf.value.decode())

    def set_tuning(self, table):
        """Apply a table from autotune() / tuning() (dict or JSON text)."""
        import json
        text = table if isinstance(table, str) else json.dumps(table)
        _lib.check(_lib.lib().mra_set_tuning(self._h, text.encode()), "mra_set_tuning")

    # -- tracing ----------------------------------------------------------------
    def profile(self, enable: bool = True):
        """Enable (and clear) or disable per-kernel HIP-event timing."""
        _lib.check(_lib.lib().mra_profile(self._h, 1 if enable else 0), "mra_profile")

    def profile_read(self):
        """Aggregated per-kernel timings since the last read:
        list of dicts (name, level, groups, launches, total_ms, flops)."""
        cap = 256
        buf = (_lib.PhaseStat * cap)()
        cnt = C.c_int32()
        st = self._stream() if self.device is not None else None
        _lib.check(_lib.lib().mra_profile_read(self._h, buf, cap, C.byref(cnt), st), "mra_profile_read")
        return [{"name": b.name.decode(), "level": b.level, "groups": b.groups, "launches": b.launches,
                 "total_ms": b.total_ms, "flops": b.flops} for b in buf[:min(cnt.value, cap)]]

    def __del__(self):
        h = getattr(self, "_h", None)
        L = getattr(_lib, "_lib", None) if _lib is not None else None   # None at interpreter shutdown
        if h is not None and L is not None:
            L.mra_destroy(h)
            self._h = None


def _make_autograd():
    torch = _torch()

    class MRALogLik(torch.autograd.Function):
        """loglik(theta) with the library's reverse-pass gradient.

        forward(theta [n_theta, 3], plan, y) -> loglik [n_theta]; y is one
        data vector (n,) shared by every parameter row, or (n_theta, n) with
        one data vector per row.  When y requires grad, its gradient comes
        from the same reverse pass: for a shared y the rows' gradients are
        summed (loglik[b] depends on y through every row), for per-row data
        row b's gradient goes to y[b] alone."""

        @staticmethod
        def forward(ctx, theta, plan, y):
            per_row = y.dim() == 2 and y.shape[0] > 1
            if per_row and not ctx.needs_input_grad[2]:
                raise ValueError("per-row data (n_theta, n) goes through the data-gradient call; "
                                 "give y requires_grad=True or pass one data vector")
            if ctx.needs_input_grad[2]:
                ll, g, gy = plan.loglik_grad_data(y.detach(), theta.detach())
            else:
                (ll, g), gy = plan.loglik_grad(y, theta.detach()), None
            ctx.save_for_backward(g, gy)
            ctx.theta_device = theta.device
            ctx.y_device = y.device
            ctx.y_shape = tuple(y.shape)
            ctx.per_row = per_row
            return ll

        @staticmethod
        def backward(ctx, gout):
            g, gy = ctx.saved_tensors
            go = gout.to(g.device)
            dtheta = (go[:, None] * g).to(ctx.theta_device)
            dy = None
            if gy is not None:
                dy = go[:, None] * gy if ctx.per_row else go @ gy
                dy = dy.reshape(ctx.y_shape).to(ctx.y_device)
            return dtheta, None, dy

    return MRALogLik


class _Lazy:
    _cls = None

    def __getattr__(self, k):
        if _Lazy._cls is None:
            _Lazy._cls = _make_autograd()
        return getattr(_Lazy._cls, k)


MRALogLik = _Lazy()
