#!/usr/bin/env python3
"""Write the stored oracle values of the full-size GPU parity tests.

Only the CPU oracle (oracle/) and the seeded input generators are called;
nothing here touches the GPU library.

    python tests/golden/make_golden.py [--jobs 3]

writes tests/golden/clustered_n262144.json: the oracle log-likelihood and
its forward-mode gradient on the clustered workload (n = 2^18 locations,
half uniform, half in 200 Gaussian clusters of sd 0.01; Matern nu = 1.5;
M = 6, J = 4, r = 64; data a random-Fourier-feature draw of the Matern
field plus noise) at the workload's
own parameter vector and at two vectors drawn from the multi-parameter
distribution (seed 31).  Single-threaded BLAS per job; about three minutes
per parameter vector.
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


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--jobs", type=int, default=3)
    a = ap.parse_args()
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
