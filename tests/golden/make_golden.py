#!/usr/bin/env python3
"""Write the stored oracle values of the full-size GPU parity tests.

Only the CPU oracle (oracle/) and the seeded input generators are called;
nothing here touches the GPU library.

    python tests/golden/make_golden.py [--jobs 3]
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
    a = ap.parse_args()
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
