"""Seeded synthetic inputs for the M-RA workloads (locations, data, parameters).

This module is shared by the HIP path's callers (bench, tests) and by the
CPU oracle's callers.  It holds none of the M-RA arithmetic: no covariance
evaluation, no partitioning, no linear algebra of the method.  It only draws
numbers from ``numpy.random.Generator(PCG64(seed))``.

Workload shapes follow the paper's settings:
  * irregular 2-D locations on the unit square (Sec. 2.1 allows any
    non-gridded domain; Sec. 4.1 uses equidistant grids, which are replaced
    here by uniform and clustered scatters so that leaf sizes are uneven);
  * satellite-swath geometry with gaps standing in for the MIRS total
    precipitable water data of Sec. 4.2 (not available here);
  * data drawn from a stationary Gaussian field of the paper's covariance
    families (exponential, Matern nu=1.5, eq. mat15) by random Fourier
    features, plus white measurement error (Sec. 4.2).

The data field is an approximation of the exact Gaussian process; the
likelihood, gradient and kriging computed from it are exact functions of
whatever data they are given, so parity does not depend on how it was drawn.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np


def _rng(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(seed))


# --------------------------------------------------------------------------
# locations
# --------------------------------------------------------------------------

def uniform_locations(n: int, seed: int, d: int = 2) -> np.ndarray:
    """n locations uniform on [0,1]^d, shape (n, d), float64."""
    return _rng(seed).random((n, d))


def clustered_locations(n_uniform: int, n_clustered: int, n_centers: int,
                        sd: float, seed: int) -> np.ndarray:
    """Half-uniform, half-clustered scatter on [0,1]^2.

    Cluster centres are uniform; each clustered point picks a centre
    uniformly and adds an isotropic N(0, sd^2 I) offset; offsets that leave
    the unit square are redrawn.  Gives the uneven leaf counts of a satellite
    or sensor network.
    """
    g = _rng(seed)
    uni = g.random((n_uniform, 2))
    centers = g.random((n_centers, 2))
    ids = g.integers(0, n_centers, size=n_clustered)
    pts = centers[ids] + sd * g.standard_normal((n_clustered, 2))
    bad = np.flatnonzero((pts < 0.0).any(axis=1) | (pts > 1.0).any(axis=1))
    while bad.size:
        pts[bad] = centers[ids[bad]] + sd * g.standard_normal((bad.size, 2))
        bad = bad[(pts[bad] < 0.0).any(axis=1) | (pts[bad] > 1.0).any(axis=1)]
    return np.concatenate([uni, pts], axis=0)


@dataclass
class SwathGeometry:
    centers: np.ndarray          # c_i of the lines x - y = c_i
    width: float
    gaps: np.ndarray             # (n_strips, n_gaps, 2) along-track [t0, t1) in [0,1]


def _swath_segment(c: float):
    """End points of the line x - y = c inside the unit square."""
    p0 = np.array([max(0.0, c), max(0.0, -c)])
    p1 = np.array([min(1.0, 1.0 + c), min(1.0, 1.0 - c)])
    return p0, p1


def swath_geometry(seed: int, n_strips: int = 24, width: float = 0.02,
                   n_gaps: int = 3, gap_frac: float = 0.10) -> SwathGeometry:
    """Diagonal strips x - y = c_i, c_i = -1 + (i + 1/2)/(n_strips/2), each
    with n_gaps non-overlapping contiguous gaps of gap_frac of its length."""
    g = _rng(seed)
    centers = np.array([-1.0 + (i + 0.5) / (n_strips / 2.0) for i in range(n_strips)])
    gaps = np.zeros((n_strips, n_gaps, 2))
    free = 1.0 - n_gaps * gap_frac
    for s in range(n_strips):
        # n_gaps gap starts placed in the free length, sorted, then shifted so
        # gaps never overlap (stick-breaking of the free length)
        cuts = np.sort(g.random(n_gaps)) * free
        for k in range(n_gaps):
            t0 = cuts[k] + k * gap_frac
            gaps[s, k] = (t0, t0 + gap_frac)
    return SwathGeometry(centers=centers, width=width, gaps=gaps)


def _in_gap(t: np.ndarray, gaps: np.ndarray) -> np.ndarray:
    m = np.zeros(t.shape, dtype=bool)
    for t0, t1 in gaps:
        m |= (t >= t0) & (t < t1)
    return m


def swath_locations(geom: SwathGeometry, n: int, seed: int, in_gaps: bool = False) -> np.ndarray:
    """n points uniform over the kept parts of the strips (or over the gaps
    when in_gaps), clipped to the unit square by rejection."""
    g = _rng(seed)
    p0s, p1s = zip(*[_swath_segment(c) for c in geom.centers])
    p0s, p1s = np.array(p0s), np.array(p1s)
    lens = np.linalg.norm(p1s - p0s, axis=1)
    gap_total = (geom.gaps[:, :, 1] - geom.gaps[:, :, 0]).sum(axis=1)
    frac = gap_total if in_gaps else 1.0 - gap_total
    w = lens * frac
    w = w / w.sum()
    out = np.empty((0, 2))
    while out.shape[0] < n:
        m = int((n - out.shape[0]) * 1.3) + 1024
        sid = g.choice(len(w), size=m, p=w)
        t = g.random(m)
        keep = _strip_mask(sid, t, geom.gaps, in_gaps)
        sid, t = sid[keep], t[keep]
        off = (g.random(sid.size) - 0.5) * geom.width
        d = p1s[sid] - p0s[sid]
        u = d / np.linalg.norm(d, axis=1, keepdims=True)
        nrm = np.stack([-u[:, 1], u[:, 0]], axis=1)
        pts = p0s[sid] + t[:, None] * d + off[:, None] * nrm
        ok = (pts >= 0.0).all(axis=1) & (pts <= 1.0).all(axis=1)
        out = np.concatenate([out, pts[ok]], axis=0)
    return out[:n]


def _strip_mask(sid, t, gaps, in_gaps):
    m = np.zeros(t.shape, dtype=bool)
    for s in np.unique(sid):
        sel = sid == s
        m[sel] = _in_gap(t[sel], gaps[s])
    return m if in_gaps else ~m


# --------------------------------------------------------------------------
# data
# --------------------------------------------------------------------------

def normals(n: int, seed: int) -> np.ndarray:
    return _rng(seed).standard_normal(n)


def rff_field(locs: np.ndarray, sigma2: float, kappa: float, nu: float,
              tau2: float, seed: int, n_features: int = 1024,
              chunk: int = 65536) -> np.ndarray:
    """Draw of a stationary Gaussian field plus white noise at locs.

    Random Fourier features: frequencies from the spectral measure of the
    Matern family with smoothness nu and length kappa (for nu = 1/2 the
    exponential model, for nu = 3/2 the paper's eq. mat15), which is a
    multivariate Student-t with 2*nu degrees of freedom and scale 1/kappa.
    Returns sigma * sqrt(2/F) * sum_f cos(w_f . s + b_f) + sqrt(tau2) * eps.
    """
    g = _rng(seed)
    n, d = locs.shape
    F = n_features
    dof = 2.0 * nu
    gauss = g.standard_normal((F, d))
    chi = g.chisquare(dof, size=F)
    w = gauss / np.sqrt(chi / dof)[:, None] / kappa
    b = g.random(F) * 2.0 * math.pi
    eps = g.standard_normal(n)
    out = np.empty(n)
    amp = math.sqrt(sigma2) * math.sqrt(2.0 / F)
    for s in range(0, n, chunk):
        ph = locs[s:s + chunk] @ w.T + b
        out[s:s + chunk] = amp * np.cos(ph).sum(axis=1)
    return out + math.sqrt(tau2) * eps


def theta_draws(k: int, seed: int) -> np.ndarray:
    """k parameter vectors (log sigma^2, log kappa, log tau^2):
    log sigma^2 ~ U[-1, 1], log kappa ~ U[log 0.02, log 0.3],
    log tau^2 ~ U[-6, -2]."""
    g = _rng(seed)
    ls2 = g.uniform(-1.0, 1.0, size=k)
    lk = g.uniform(math.log(0.02), math.log(0.3), size=k)
    lt2 = g.uniform(-6.0, -2.0, size=k)
    return np.stack([ls2, lk, lt2], axis=1)


# --------------------------------------------------------------------------
# named workloads
# --------------------------------------------------------------------------

@dataclass
class Workload:
    name: str
    locs: np.ndarray
    z: np.ndarray
    theta: np.ndarray             # (3,) log sigma^2, log kappa, log tau^2
    cov: str                      # "exponential" | "matern32"
    M: int
    J: int
    r: int
    d: int = 2
    pred: np.ndarray | None = None
    extra: dict = field(default_factory=dict)


def _theta(sigma2, kappa, tau2):
    return np.array([math.log(sigma2), math.log(kappa), math.log(tau2)])


def small_uniform(n: int = 4096, seed: int = 1, n_pred: int = 1000) -> Workload:
    """n uniform locations, exponential covariance sigma^2=1, kappa=0.05,
    tau^2=0.05; M=3, J=4 (64 leaves of ~n/64), r=16; n_pred uniform
    prediction locations."""
    locs = uniform_locations(n, seed)
    z = rff_field(locs, 1.0, 0.05, 0.5, 0.05, seed + 100)
    pred = uniform_locations(n_pred, seed + 1000)
    return Workload("uniform_n%d_exp_M3_r16" % n, locs, z, _theta(1.0, 0.05, 0.05),
                    "exponential", 3, 4, 16, pred=pred)


def clustered(n: int = 262144, seed: int = 2, M: int = 6, r: int = 64) -> Workload:
    """n locations, half uniform and half from 200 Gaussian clusters with
    sd 0.01; Matern nu=1.5, sigma^2=1, kappa=0.1, tau^2=0.01; J=4."""
    locs = clustered_locations(n // 2, n - n // 2, 200, 0.01, seed)
    z = rff_field(locs, 1.0, 0.1, 1.5, 0.01, seed + 100)
    return Workload("clustered_n%d_matern32_M%d_r%d" % (n, M, r), locs, z,
                    _theta(1.0, 0.1, 0.01), "matern32", M, 4, r)


def swaths(n: int = 4194304, n_pred: int = 1048576, seed: int = 5,
           M: int = 9, r: int = 64) -> Workload:
    """Satellite-swath scatter: 24 diagonal strips of width 0.02 with 30% of
    each removed in 3 contiguous gaps; Matern nu=1.5, sigma^2=1, kappa=0.08,
    tau^2=0.02, plus a linear mean 0.5 + x - y (to be removed by the caller);
    prediction locations in the gaps."""
    geom = swath_geometry(seed)
    locs = swath_locations(geom, n, seed + 1)
    pred = swath_locations(geom, n_pred, seed + 2, in_gaps=True)
    z = rff_field(locs, 1.0, 0.08, 1.5, 0.02, seed + 100)
    z = z + 0.5 + locs[:, 0] - locs[:, 1]
    return Workload("swaths_n%d_matern32_M%d_r%d" % (n, M, r), locs, z,
                    _theta(1.0, 0.08, 0.02), "matern32", M, 4, r, pred=pred,
                    extra={"trend": (0.5, 1.0, -1.0)})
