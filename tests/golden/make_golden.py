#!/usr/bin/env python3
"""Write the stored oracle values of the full-size GPU parity tests.

Only the CPU oracle (oracle/) and the seeded input generators are called;
nothing here touches the GPU library.

    python tests/golden/make_golden.py [--jobs 3]
    python tests/golden/make_golden.py --sweep [--jobs 6]
    python tests/golden/make_golden.py --predict [--jobs 2]
    python tests/golden/make_golden.py --data-grad

The first writes tests/golden/clustered_n262144.json: the oracle log-likelihood and
its forward-mode gradient on the clustered workload (n = 2^18 locations,
half uniform, half in 200 Gaussian clusters of sd 0.01; Matern nu = 1.5;
M = 6, J = 4, r = 64; data a random-Fourier-feature draw of the Matern
field plus noise) at the workload's
own parameter vector and at two vectors drawn from the multi-parameter
distribution (seed 31).  Single-threaded BLAS per job; about three minutes
per parameter vector.  The second writes
tests/golden/clustered_n262144_grad_data.json: the oracle's data gradient
d loglik / d z = -Sigma^{-1} z (kriging residual at the observed locations)
at 512 observations drawn with seed 77, at the workload's own parameters.

--sweep writes tests/golden/clustered_n262144_sweep.json: the same
workload at the eight finite-difference points (theta_draws(8, 31)) and at
the worst-conditioned vectors of the 64-vector batch (theta_draws(64, 41):
the largest range kappa, draws 58, 36 and 4, and the smallest nugget tau^2,
draws 63 and 29).  At the five extreme vectors the oracle also runs with its
children summed in reverse order (an equally valid operation order), and the
relative spread of the two runs is stored as the oracle's noise floor there.

--predict writes tests/golden/predict_n65536_M6_r64.json: the oracle's
kriging mean and variance (Prop. 2) with M = 6, J = 4, r = 64, Matern
nu = 1.5 at two scatters of 2^16 locations: satellite swaths (seed 5
geometry, locations seed 6, most leaves empty) with 2048 prediction points
in the gaps and 512 uniform ones (regions kept for the prior only), and the
clustered scatter (seed 2) with 2048 uniform prediction points.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time
from concurrent.futures import ProcessPoolExecutor

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "clustered_n262144.json")


def _thetas():
    from paper_1507_04789_amd import workloads as wl
    w = wl.clustered()
    return [list(map(float, w.theta))] + [list(map(float, t)) for t in wl.theta_draws(2, 31)]


def _one(theta):
    from threadpoolctl import threadpool_limits
    import numpy as np
    from oracle import mra
    from oracle.geometry import Geometry
    from paper_1507_04789_amd import workloads as wl
    w = wl.clustered()
    with threadpool_limits(1):
        geo = Geometry(w.locs, 2, w.M, w.J, w.r)
        t0 = time.perf_counter()
        ll, g, _ = mra.loglik(geo, w.z, w.cov, np.asarray(theta), grad=True)
        dt = time.perf_counter() - t0
    return {"theta": theta, "loglik": float(ll), "grad": [float(x) for x in g], "oracle_s": dt}


OUT_SWEEP = os.path.join(os.path.dirname(os.path.abspath(__file__)), "clustered_n262144_sweep.json")
EXTREME = [58, 36, 4, 63, 29]


def _sweep_one(job):
    from threadpoolctl import threadpool_limits
    import numpy as np
    from oracle import mra
    from oracle.geometry import Geometry
    from paper_1507_04789_amd import workloads as wl
    theta, order = job
    w = wl.clustered()
    with threadpool_limits(1):
        geo = Geometry(w.locs, 2, w.M, w.J, w.r)
        t0 = time.perf_counter()
        ll, g, _ = mra.loglik(geo, w.z, w.cov, np.asarray(theta), grad=True, child_order=order)
        dt = time.perf_counter() - t0
    return {"theta": list(map(float, theta)), "loglik": float(ll), "grad": [float(x) for x in g], "oracle_s": dt}


def sweep(jobs):
    from paper_1507_04789_amd import workloads as wl
    fd = [list(map(float, t)) for t in wl.theta_draws(8, 31)]
    d64 = wl.theta_draws(64, 41)
    ext = [list(map(float, d64[i])) for i in EXTREME]
    work = [(t, "forward") for t in fd + ext] + [(t, "reversed") for t in ext]
    with ProcessPoolExecutor(max_workers=jobs) as ex:
        res = list(ex.map(_sweep_one, work))
    fwd, rev = res[:len(fd) + len(ext)], res[len(fd) + len(ext):]
    for p, q in zip(fwd[len(fd):], rev):
        p["noise_loglik"] = abs(p["loglik"] - q["loglik"]) / abs(p["loglik"])
        p["noise_grad"] = [abs(a - b) / abs(a) for a, b in zip(p["grad"], q["grad"])]
    for p in fwd[:len(fd)]:
        p["set"] = "finite-difference points, theta_draws(8, 31)"
    for p, i in zip(fwd[len(fd):], EXTREME):
        p["set"] = "theta_draws(64, 41)[%d]" % i
    out = {"workload": "as clustered_n262144.json", "n": 262144, "M": 6, "J": 4, "r": 64, "cov": "matern32",
           "values": "oracle.mra.loglik(grad=True); at the extreme draws also child_order='reversed', whose "
                     "relative difference is stored as noise_loglik / noise_grad",
           "points": fwd}
    with open(OUT_SWEEP, "w") as f:
        json.dump(out, f, indent=1)
    print("wrote", OUT_SWEEP)


OUT_PRED = os.path.join(os.path.dirname(os.path.abspath(__file__)), "predict_n65536_M6_r64.json")


def predict_cases():
    """(name, locs, z, pred, theta) of the two kriging cases."""
    import math
    import numpy as np
    from paper_1507_04789_amd import workloads as wl
    geom = wl.swath_geometry(5)
    sl = wl.swath_locations(geom, 65536, 6)
    sp = np.concatenate([wl.swath_locations(geom, 2048, 7, in_gaps=True), wl.uniform_locations(512, 9)])
    sz = wl.rff_field(sl, 1.0, 0.08, 1.5, 0.02, 105)
    st = np.array([0.0, math.log(0.08), math.log(0.02)])
    c = wl.clustered(n=65536)
    cp = wl.uniform_locations(2048, 10)
    return [("swath", sl, sz, sp, st), ("clustered", c.locs, c.z, cp, np.asarray(c.theta))]


def _pred_one(k):
    from threadpoolctl import threadpool_limits
    from oracle import predict
    from oracle.geometry import Geometry
    name, locs, z, pred, theta = predict_cases()[k]
    with threadpool_limits(1):
        t0 = time.perf_counter()
        mu, var = predict.predict(Geometry(locs, 2, 6, 4, 64), z, "matern32", theta, pred)
        dt = time.perf_counter() - t0
    return {"case": name, "theta": list(map(float, theta)), "n": int(len(z)), "n_pred": int(len(pred)),
            "mean": [float(x) for x in mu], "var": [float(x) for x in var], "oracle_s": dt}


def predict_golden(jobs):
    with ProcessPoolExecutor(max_workers=jobs) as ex:
        res = list(ex.map(_pred_one, range(2)))
    out = {"M": 6, "J": 4, "r": 64, "cov": "matern32",
           "generator": "predict_cases() in this script (paper_1507_04789_amd.workloads generators)",
           "values": "oracle.predict.predict: Prop. 2 posterior predictive mean and marginal variance of y_M",
           "cases": res}
    with open(OUT_PRED, "w") as f:
        json.dump(out, f)
    print("wrote", OUT_PRED, [r["oracle_s"] for r in res])


OUT_DATA = os.path.join(os.path.dirname(os.path.abspath(__file__)), "clustered_n262144_grad_data.json")


def data_grad():
    import numpy as np
    from oracle import predict
    from oracle.geometry import Geometry
    from paper_1507_04789_amd import workloads as wl
    w = wl.clustered()
    idx = np.sort(np.random.default_rng(77).choice(len(w.z), 512, replace=False))
    geo = Geometry(w.locs, 2, w.M, w.J, w.r)
    t0 = time.perf_counter()
    gz = predict.data_gradient(geo, w.z, w.cov, np.asarray(w.theta), idx)
    out = {"workload": "as clustered_n262144.json", "theta": list(map(float, w.theta)),
           "values": "oracle.predict.data_gradient: (E[y_M(S_i) | z] - z_i) / tau^2 = -(Sigma^{-1} z)_i, "
                     "Prop. 2 posterior mean at the observed locations",
           "index": [int(i) for i in idx], "grad_y": [float(x) for x in gz],
           "oracle_s": time.perf_counter() - t0}
    with open(OUT_DATA, "w") as f:
        json.dump(out, f, indent=1)
    print("wrote", OUT_DATA, "in %.1f s" % out["oracle_s"])


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--jobs", type=int, default=3)
    ap.add_argument("--data-grad", action="store_true")
    ap.add_argument("--sweep", action="store_true")
    ap.add_argument("--predict", action="store_true")
    a = ap.parse_args()
    if a.sweep:
        sweep(a.jobs)
        return
    if a.predict:
        predict_golden(a.jobs)
        return
    if a.data_grad:
        data_grad()
        return
    from paper_1507_04789_amd import workloads as wl
    w = wl.clustered()
    ths = _thetas()
    with ProcessPoolExecutor(max_workers=a.jobs) as ex:
        res = list(ex.map(_one, ths))
    out = {"workload": "clustered n=262144 (131072 uniform + 131072 in 200 clusters, sd 0.01), seed 2, "
                       "Matern nu=1.5, M=6, J=4, r=64, z a random-Fourier-feature Matern draw plus noise",
           "n": int(len(w.z)), "M": w.M, "J": w.J, "r": w.r, "cov": w.cov,
           "generator": "paper_1507_04789_amd.workloads.clustered()",
           "values": "oracle.mra.loglik(grad=True): eq. priorw, helpquantities, posterior in FP64",
           "points": res}
    with open(OUT, "w") as f:
        json.dump(out, f, indent=1)
    print(json.dumps(out, indent=1))


if __name__ == "__main__":
    main()
