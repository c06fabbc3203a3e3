#!/usr/bin/env python3
"""Benchmark of the M-RA FP64 log-likelihood + gradient on one MI355X.

Workload: n = 2^18 locations (half uniform, half in 200 Gaussian clusters of
sd 0.01) on the unit square, Matern nu = 1.5 with sigma^2 = 1, kappa = 0.1,
tau^2 = 0.01; M = 6 levels of quadrant splits (4096 leaves of uneven size),
r = 64 knots per region.  One step is one log-likelihood plus its reverse-
pass gradient in (log sigma^2, log kappa, log tau^2), with the data resident
in HBM.  Printed as one JSON line; see --help.
"""
from __future__ import annotations

import argparse
import json
import math
import re
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_FP64_TFLOPS = 78.6      # MI355X dense FP64 (matrix and vector)
PEAK_HBM_GBPS = 8000.0       # MI355X HBM3E
PROFILE_SUMMARY = "clustered_n262144_loglik_grad_counters.txt"
METRIC = "M-RA loglik+grad evals/s at n=2^18 (batched vs plain, 1 GPU); FP64 MFMA % peak"


def _dominant(stats):
    """Aggregate per-kernel records over levels; pick the kernel with the
    largest summed time."""
    fam = {}
    for s in stats:
        f = fam.setdefault(s["name"], {"name": s["name"], "groups": 0, "launches": 0, "total_ms": 0.0, "flops": 0.0})
        for k in ("groups", "launches", "total_ms", "flops"):
            f[k] += s[k]
    ranked = sorted(fam.values(), key=lambda f: -f["total_ms"])
    return ranked


def _oracle_sample(job):
    """One oracle loglik + forward-mode gradient on the bounded sample,
    single-threaded BLAS; returns its wall time (seconds)."""
    n, M, theta = job
    import numpy as np
    from threadpoolctl import threadpool_limits
    from oracle import mra
    from oracle.geometry import Geometry
    from paper_1507_04789_amd import workloads as wl
    w = wl.clustered(n=n, M=M)
    with threadpool_limits(1):
        geo = Geometry(w.locs, 2, w.M, w.J, w.r)
        t0 = time.perf_counter()
        mra.loglik(geo, w.z, w.cov, np.asarray(theta if theta is not None else w.theta), grad=True)
        return time.perf_counter() - t0


def _host_cores():
    """Cores this process may run on, capped at 16 (one GPU's share of the
    host on the benchmark machines)."""
    try:
        c = len(os.sched_getaffinity(0))
    except AttributeError:  # pragma: no cover
        c = os.cpu_count() or 1
    return max(1, min(c, 16))


def cpu_baseline(sample_n: int, sample_M: int, full_flops: float):
    """The oracle (loglik + forward-mode gradient), unchanged, on a bounded
    sample of the same workload family: the clustered generator at
    n = sample_n with M = sample_M (about 64 observations per leaf, as the
    full workload).  Two modes: one process with single-threaded BLAS, and
    C processes (C = the host cores available, at most 16) each evaluating
    its own parameter vector, the CPU form of the multi-parameter batch.
    Rates are scaled to the full workload by the ratio of algorithmic flops
    (sample / full).  Runs before the GPU is touched, so the worker
    processes fork from a process without a GPU context."""
    import multiprocessing as mp
    from concurrent.futures import ProcessPoolExecutor
    from paper_1507_04789_amd import Plan
    from paper_1507_04789_amd import workloads as wl
    w = wl.clustered(n=sample_n, M=sample_M)
    sp = Plan(w.locs, M=w.M, J=w.J, r=w.r, cov=w.cov)
    ratio = sp.info["flops_grad"] / full_flops
    dt1 = _oracle_sample((sample_n, sample_M, None))
    cores = _host_cores()
    ths = wl.theta_draws(cores, 41)
    t0 = time.perf_counter()
    with ProcessPoolExecutor(max_workers=cores, mp_context=mp.get_context("fork")) as ex:
        per = list(ex.map(_oracle_sample, [(sample_n, sample_M, list(t)) for t in ths]))
    wall = time.perf_counter() - t0
    return {"value": cores * ratio / wall, "unit": "evals/s", "cores": cores, "kind": "oracle",
            "sample": "oracle loglik + forward-mode gradient, unchanged, on the clustered generator at n=%d, M=%d "
                      "(about 64 obs per leaf, as the full workload): %d processes with single-threaded BLAS, one "
                      "parameter vector each (theta_draws(%d, 41)), %.2f s wall (%.2f-%.2f s per evaluation); "
                      "rate scaled to n=2^18, M=6 by the algorithmic flop ratio %.4g"
                      % (sample_n, sample_M, cores, cores, wall, min(per), max(per), ratio),
            "single_thread": {"value": ratio / dt1, "cores": 1, "sample_s": dt1},
            "cpu": _cpu_name(), "host_cpus_visible": os.cpu_count()}


def _src_digest() -> str:
    """sha256 over the library's HIP/C++ sources: ties a stored counter
    summary to the kernels it was taken on."""
    import hashlib
    d = os.path.join(ROOT, "paper_1507_04789_amd", "csrc")
    h = hashlib.sha256()
    for f in sorted(os.listdir(d)):
        # the kernels, their headers and the plan (task lists); not the ABI
        # glue (api.cpp), the scratch array of the no-allocation call or the
        # stand-alone engine probe
        if f.endswith((".hip", ".hpp", ".cpp", ".h")) and f not in ("api.cpp", "noalloc.hip", "engine_probe.hip"):
            h.update(f.encode())
            h.update(open(os.path.join(d, f), "rb").read())
    return h.hexdigest()[:16]


def _stored_traffic(kernel: str):
    """HBM bytes per launch of `kernel` from the committed counter summary,
    or None when the summary is missing, names another kernel, or was taken
    on other sources."""
    path = os.path.join(ROOT, "profiles", PROFILE_SUMMARY)
    if not os.path.exists(path):
        return None
    vals = {}
    for line in open(path):
        m = re.match(r"^traffic\s+(\S+)\s+(\S+)\s+src\s+(\S+)", line.strip())
        if m:
            vals[m.group(1)] = (float(m.group(2)), m.group(3))
    if kernel not in vals or vals[kernel][1] != _src_digest():
        return None
    return vals[kernel][0]


def _stored_mfma(kernel: str):
    """(executed FP64 MFMA flops per launch, MFMA busy %) of `kernel` from
    the committed counter summary, or None when missing or taken on other
    sources."""
    path = os.path.join(ROOT, "profiles", PROFILE_SUMMARY)
    if not os.path.exists(path):
        return None
    for line in open(path):
        m = re.match(r"^mfma\s+(\S+)\s+(\S+)\s+(\S+)\s+src\s+(\S+)", line.strip())
        if m and m.group(1) == kernel and m.group(4) == _src_digest():
            return float(m.group(2)), float(m.group(3))
    return None


def copy_probe(nbytes: int, reps: int = 3):
    """A plain device-to-device copy of known size, for scaling the HBM
    byte counters (each launch reads and writes nbytes)."""
    import torch
    n = nbytes // 8
    a = torch.ones(n, dtype=torch.float64, device="cuda:0")
    b = torch.empty_like(a)
    for _ in range(reps):
        b.copy_(a)
    torch.cuda.synchronize()
    print(json.dumps({"copy_probe_bytes": n * 8, "reps": reps}))


def _csv(path):
    import csv
    with open(path) as f:
        return list(csv.DictReader(f))


def _short(name: str) -> str:
    m = re.match(r"^(?:void )?mra::k_(\w+)(<\w+>)?", name)
    return m.group(1) + (m.group(2) or "") if m else name[:40]


def summarize_profiles(root: str, copy_bytes: int):
    """Text summary of a profiling directory: root/trace (kernel trace +
    stats of a bench run), root/fetch and root/write (FETCH_SIZE and
    WRITE_SIZE of the same run), root/copy_fetch and root/copy_write (the
    same counters on copy_probe).  Commands are read from root/commands.txt."""
    out = []
    cmds = os.path.join(root, "commands.txt")
    if os.path.exists(cmds):
        out.append("commands:")
        out += ["  " + l.rstrip() for l in open(cmds) if l.strip()]
    out.append("source digest: %s" % _src_digest())

    def find(sub, suffix):
        d = os.path.join(root, sub)
        for dp, _, fs in os.walk(d):
            for f in fs:
                if f.endswith(suffix):
                    return os.path.join(dp, f)
        raise FileNotFoundError("%s/*%s" % (d, suffix))

    stats = _csv(find("trace", "kernel_stats.csv"))
    out.append("")
    out.append("kernel stats (rocprofv3 --kernel-trace --stats):")
    out.append("%-18s %6s %12s %12s %6s" % ("kernel", "calls", "total_ms", "avg_us", "pct"))
    for r in stats[:20]:
        out.append("%-18s %6s %12.3f %12.2f %6s" % (_short(r["Name"]), r["Calls"],
                                                     float(r["TotalDurationNs"]) / 1e6,
                                                     float(r["AverageNs"]) / 1e3, r["Percentage"]))

    def counter(sub):
        per = {}
        for r in _csv(find(sub, "counter_collection.csv")):
            per.setdefault(r["Kernel_Name"], []).append(float(r["Counter_Value"]))
        return per

    def copy_factor(sub):
        per = counter(sub)
        # the largest dispatch is the probe's copy
        vals = max((v for vs in per.values() for v in vs))
        return copy_bytes / vals, vals

    ff, fv = copy_factor("copy_fetch")
    wf, wv = copy_factor("copy_write")
    out.append("")
    out.append("copy calibration: %d bytes read and written per copy; FETCH_SIZE %.1f, WRITE_SIZE %.1f "
               "per dispatch -> %.2f and %.2f bytes per counter unit" % (copy_bytes, fv, wv, ff, wf))
    fetch, write = counter("fetch"), counter("write")
    out.append("")
    out.append("HBM traffic per dispatch (counter x calibration), averaged over dispatches:")
    out.append("%-18s %6s %12s %12s %12s" % ("kernel", "disp", "fetch_MB", "write_MB", "total_MB"))
    rows = []
    for k in fetch:
        fb = ff * sum(fetch[k]) / len(fetch[k])
        wb = wf * (sum(write.get(k, [0.0])) / max(len(write.get(k, [])), 1))
        rows.append((_short(k), len(fetch[k]), fb, wb))
    rows.sort(key=lambda x: -(x[2] + x[3]) * x[1])
    for name, nd, fb, wb in rows:
        out.append("%-18s %6d %12.2f %12.2f %12.2f" % (name, nd, fb / 1e6, wb / 1e6, (fb + wb) / 1e6))
    out.append("")
    out.append("machine-readable (kernel, HBM bytes per launch, source digest):")
    for name, nd, fb, wb in rows:
        out.append("traffic %s %.6g src %s" % (name, fb + wb, _src_digest()))
    # executed FP64 MFMA work: derived counters MfmaFlopsF64
    # (SQ_INSTS_VALU_MFMA_MOPS_F64 x 512) and MfmaUtil (busy MFMA cycles over
    # GPU-active cycles times SIMDs), one pass of their own
    try:
        mf = _csv(find("mfma", "counter_collection.csv"))
    except FileNotFoundError:
        mf = []
    if mf:
        per = {}
        for r in mf:
            per.setdefault(r["Kernel_Name"], {}).setdefault(r["Counter_Name"], []).append(float(r["Counter_Value"]))
        avg_ns = {_short(r["Name"]): float(r["AverageNs"]) for r in stats}
        out.append("")
        out.append("executed FP64 MFMA per dispatch (MfmaFlopsF64, MfmaUtil), with the kernel-trace average duration:")
        out.append("%-18s %6s %14s %12s %12s" % ("kernel", "disp", "exec_GFLOP", "exec_TF/s", "mfma_busy%"))
        mrows = []
        for k, c in per.items():
            fl = c.get("MfmaFlopsF64", [0.0])
            ut = c.get("MfmaUtil", [0.0])
            e = sum(fl) / len(fl)
            u = sum(ut) / len(ut)
            ns = avg_ns.get(_short(k))
            mrows.append((_short(k), len(fl), e, (e / ns / 1e3) if ns else float("nan"), u))
        mrows.sort(key=lambda x: -x[2] * x[1])
        for name, nd, e, tf, u in mrows:
            out.append("%-18s %6d %14.3f %12.2f %12.2f" % (name, nd, e / 1e9, tf, u))
        out.append("")
        out.append("machine-readable (kernel, executed FP64 MFMA flops per launch, MFMA busy %, source digest):")
        for name, nd, e, tf, u in mrows:
            out.append("mfma %s %.6g %.4g src %s" % (name, e, u, _src_digest()))
    out += _timeline(find("trace", "kernel_trace.csv"))
    print("\n".join(out))


def _timeline(path: str, step: int = 2):
    """Launch timeline of one step of the traced run: every kernel's start
    and end relative to the step's first launch, with its hardware queue
    (kernels in order of their start times, a step from one call's first
    kernel to the next call's).
    Step 2 of a `--steps 3 --warmup 1` run is the second timed graph replay
    (step 0 is the warm-up, steps 4..6 the eager profiled pass)."""
    rows = sorted((r for r in _csv(path) if "mra::k_" in r["Kernel_Name"]), key=lambda r: int(r["Start_Timestamp"]))
    # a gradient call starts by clearing its partial sums, a log-likelihood call with init
    names = [_short(r["Kernel_Name"]) for r in rows]
    marker = "zero_gpart" if "zero_gpart" in names else "init"
    starts = [i for i, nm in enumerate(names) if nm == marker]
    if len(starts) <= step:
        return []
    a = starts[step]
    b = starts[step + 1] if step + 1 < len(starts) else len(rows)
    st = rows[a:b]
    t0 = min(int(r["Start_Timestamp"]) for r in st)
    t1 = max(int(r["End_Timestamp"]) for r in st)
    out = ["", "timeline of step %d of the traced run (a timed graph replay): %.3f ms from first start to last end"
           % (step, (t1 - t0) / 1e6),
           "%-16s %5s %10s %10s %9s %9s" % ("kernel", "queue", "start_us", "end_us", "dur_us", "blocks")]
    for r in sorted(st, key=lambda r: int(r["Start_Timestamp"])):
        s0 = (int(r["Start_Timestamp"]) - t0) / 1e3
        s1 = (int(r["End_Timestamp"]) - t0) / 1e3
        out.append("%-16s %5s %10.1f %10.1f %9.1f %9d" % (_short(r["Kernel_Name"]), r["Queue_Id"], s0, s1, s1 - s0,
                                                        int(r["Grid_Size_X"]) // 256))
    return out


def summarize_engine(root: str):
    """Text summary of the tile-engine probe run: root/engine.log (the
    probe's own HIP-event timings) and root/engine (rocprofv3 kernel stats of
    the same run)."""
    out = ["command:",
           "  rocprofv3 --kernel-trace --stats --output-format csv -d %s/engine -o run -- "
           "./paper_1507_04789_amd/engine_probe" % root,
           "",
           "probe output (tile variants: HIP events over 10 launches after a warm-up, FP64 TFLOP/s of the tile "
           "products; MFMA peak: 5 launches; factorisation: in-kernel wall clock over 99 calls):"]
    for line in open(os.path.join(root, "engine.log")):
        if re.match(r"^(library|A row|A k|B transposed|MFMA peak|factorisation)", line):
            out.append("  " + line.rstrip())
    stats = None
    for dp, _, fs in os.walk(os.path.join(root, "engine")):
        for f in fs:
            if f.endswith("kernel_stats.csv"):
                stats = _csv(os.path.join(dp, f))
    if stats:
        out += ["", "rocprofv3 --stats (all launches of each kernel, both segment counts):",
                "%-40s %6s %12s" % ("kernel", "calls", "avg_us")]
        for r in stats:
            name = re.sub(r"\(anonymous namespace\)::|\(double const\*.*$", "", r["Name"]).replace("void ", "")
            out.append("%-40s %6s %12.1f" % (name[:40], r["Calls"], float(r["AverageNs"]) / 1e3))
    print("\n".join(out))


def _hbm_side(traffic, avg_ms: float):
    """The dominant kernel against the HBM roof as well: its measured L2-miss
    traffic per launch (FETCH_SIZE + WRITE_SIZE, copy-calibrated; this also
    counts reads served by the Infinity Cache) over its mean launch time."""
    if traffic is None or avg_ms <= 0:
        return None
    gbps = traffic / (avg_ms * 1e-3) / 1e9
    return {"achieved": gbps, "peak": PEAK_HBM_GBPS, "unit": "GB/s", "frac": gbps / PEAK_HBM_GBPS}


def _executed(kernel: str, alg_flops: float, avg_ms: float):
    """Executed FP64 MFMA work of the dominant kernel from the committed
    counters (padding, zero columns and recomputation included), at the
    launch duration measured in this run; None when the counters were
    taken on other sources."""
    got = _stored_mfma(kernel)
    if got is None:
        return None
    e, busy = got
    tf = e / (avg_ms * 1e-3) / 1e12
    return {"flops_per_launch": e, "tflops": tf, "frac": tf / PEAK_FP64_TFLOPS, "mfma_busy_pct": busy,
            "executed_over_algorithmic": e / alg_flops}


def _time_calls(fn, steps, warmup=2):
    import torch
    for _ in range(warmup):
        fn()
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(steps):
        fn()
    e1.record()
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / steps


def secondary_configs(dev, w2, theta_batch):
    """The other measured workloads, each on captured-graph replays:
    the small uniform case (n = 4096, exponential, M = 3, r = 16, 1000
    prediction points; latency of one loglik+grad and one kriging call),
    the clustered n = 2^18 log-likelihood alone, and 64 parameter vectors on
    the clustered data (log kappa ~ U[log 0.02, log 0.3], log sigma^2 ~
    U[-1, 1], log tau^2 ~ U[-6, -2], seed 41) in batches of theta_batch
    vectors per call (one launch per level for the whole batch), the GLS
    trend call, and the clustered data partitioned by quantile splits."""
    import torch
    from paper_1507_04789_amd import MRA_GRAPH, MRA_NO_GRAD, Plan
    from paper_1507_04789_amd import workloads as wl
    res = {}
    w1 = wl.small_uniform()
    p1 = Plan(w1.locs, M=w1.M, J=w1.J, r=w1.r, cov=w1.cov, pred=w1.pred, flags=MRA_GRAPH)
    p1.bind(dev)
    z1 = torch.tensor(w1.z, device=dev)
    t1 = torch.tensor(w1.theta, device=dev).reshape(1, 3)
    o1 = (torch.empty(1, dtype=torch.float64, device=dev), torch.empty(1, 3, dtype=torch.float64, device=dev))
    pr = (torch.empty(w1.pred.shape[0], dtype=torch.float64, device=dev),
          torch.empty(w1.pred.shape[0], dtype=torch.float64, device=dev))
    ms_g = _time_calls(lambda: p1.loglik_grad(z1, t1, out=o1), 50)
    ms_p = _time_calls(lambda: p1.predict(z1, t1, out=pr), 50)
    res["uniform_n4096_exp_M3_r16"] = {"loglik_grad_ms": ms_g, "predict_ms": ms_p, "n_pred": int(w1.pred.shape[0]),
                                       "flops_grad": p1.info["flops_grad"], "flops_predict": p1.info["flops_predict"]}
    del p1
    z2 = torch.tensor(w2.z, device=dev)
    p2 = Plan(w2.locs, M=w2.M, J=w2.J, r=w2.r, cov=w2.cov, flags=MRA_GRAPH | MRA_NO_GRAD)
    p2.bind(dev)
    t2 = torch.tensor(w2.theta, device=dev).reshape(1, 3)
    o2 = torch.empty(1, dtype=torch.float64, device=dev)
    ms_l = _time_calls(lambda: p2.loglik(z2, t2, out=o2), 10)
    res["clustered_n262144_loglik"] = {"ms": ms_l, "evals_per_s": 1000.0 / ms_l,
                                       "fp64_pct_peak": 100.0 * p2.info["flops_loglik"] / (ms_l * 1e-3) /
                                       (PEAK_FP64_TFLOPS * 1e12)}
    del p2
    torch.cuda.empty_cache()
    # GLS with the linear trend (1, x, y) in one library call, against one
    # loglik + gradient call on the same plan (both launched eagerly)
    pg = Plan(w2.locs, M=w2.M, J=w2.J, r=w2.r, cov=w2.cov, flags=0)
    pg.bind(dev)
    X = torch.stack([torch.ones(len(w2.z), dtype=torch.float64), torch.tensor(w2.locs[:, 0]),
                     torch.tensor(w2.locs[:, 1])], dim=1).to(dev)
    zt = z2 + X @ torch.tensor([0.5, 1.0, -1.0], dtype=torch.float64, device=dev)
    og = (torch.empty(1, dtype=torch.float64, device=dev), torch.empty(1, 3, dtype=torch.float64, device=dev))
    ms_gls = _time_calls(lambda: pg.gls(zt, X, t2), 10)
    ms_lg = _time_calls(lambda: pg.loglik_grad(zt, t2, out=og), 10)
    beta = pg.gls(zt, X, t2)["beta"].tolist()
    res["clustered_n262144_gls_trend3"] = {"gls_ms": ms_gls, "loglik_grad_ms_eager": ms_lg,
                                           "ratio": ms_gls / ms_lg, "beta": beta}
    del pg
    torch.cuda.empty_cache()
    ths = torch.tensor(wl.theta_draws(64, 41), device=dev)
    B = max(1, min(theta_batch, 64))
    p4 = Plan(w2.locs, M=w2.M, J=w2.J, r=w2.r, cov=w2.cov, max_theta=B, flags=MRA_GRAPH)
    p4.bind(dev)
    chunks = [ths[i:i + B].contiguous() for i in range(0, 64, B)]
    outs = [(torch.empty(c.shape[0], dtype=torch.float64, device=dev),
             torch.empty(c.shape[0], 3, dtype=torch.float64, device=dev)) for c in chunks]

    def all64():
        for c, o in zip(chunks, outs):
            p4.loglik_grad(z2, c, out=o)
    ms4 = _time_calls(all64, 2, warmup=1)
    lls = torch.cat([o[0] for o in outs])
    grads = torch.cat([o[1] for o in outs])
    res["clustered_n262144_64theta_loglik_grad"] = {
        "ms_for_64": ms4, "evals_per_s": 64 * 1000.0 / ms4, "theta_per_call": B,
        "fp64_pct_peak": 100.0 * 64 * p4.info["flops_grad"] / (ms4 * 1e-3) / (PEAK_FP64_TFLOPS * 1e12),
        "finite": bool(torch.isfinite(lls).all() and torch.isfinite(grads).all())}
    del p4
    torch.cuda.empty_cache()
    # the same clustered data with data-adaptive (quantile) splits: equal
    # leaf counts instead of the quadrants' 0..542, so less padding and no
    # large leaves; its own algorithmic flop count
    pa = Plan(w2.locs, M=w2.M, J=w2.J, r=w2.r, cov=w2.cov, adaptive=True, flags=MRA_GRAPH)
    pa.bind(dev)
    oa = (torch.empty(1, dtype=torch.float64, device=dev), torch.empty(1, 3, dtype=torch.float64, device=dev))
    ms_a = _time_calls(lambda: pa.loglik_grad(z2, t2, out=oa), 10)
    res["clustered_n262144_adaptive_splits_loglik_grad"] = {
        "ms": ms_a, "evals_per_s": 1000.0 / ms_a, "max_leaf": int(pa.info["max_leaf"]),
        "fp64_pct_peak": 100.0 * pa.info["flops_grad"] / (ms_a * 1e-3) / (PEAK_FP64_TFLOPS * 1e12),
        "loglik": float(oa[0][0])}
    del pa
    torch.cuda.empty_cache()
    return res


def swath_config(dev):
    """The satellite-swath workload at full size: n = 2^22 in 24 diagonal
    strips of width 0.02 with three 10% gaps each, Matern nu = 1.5 with a
    linear trend removed by the caller, M = 9, J = 4, r = 64 (73% of the
    leaves empty, their regions pruned), kriging at 2^20 points in the gaps.
    Graph replays; generation of the data takes about a minute on the host."""
    import torch
    from paper_1507_04789_amd import MRA_GRAPH, Plan
    from paper_1507_04789_amd import workloads as wl
    t0 = time.perf_counter()
    w = wl.swaths()
    z = w.z - (0.5 + w.locs[:, 0] - w.locs[:, 1])
    gen_s = time.perf_counter() - t0
    p = Plan(w.locs, M=w.M, J=w.J, r=w.r, cov=w.cov, pred=w.pred, flags=MRA_GRAPH)
    p.bind(dev)
    zt = torch.tensor(z, device=dev)
    th = torch.tensor(w.theta, device=dev).reshape(1, 3)
    ll = torch.empty(1, dtype=torch.float64, device=dev)
    g = torch.empty(1, 3, dtype=torch.float64, device=dev)
    mu = torch.empty(w.pred.shape[0], dtype=torch.float64, device=dev)
    var = torch.empty_like(mu)
    ms_g = _time_calls(lambda: p.loglik_grad(zt, th, out=(ll, g)), 3, warmup=1)
    ms_l = _time_calls(lambda: p.loglik(zt, th, out=ll), 3, warmup=1)
    ms_p = _time_calls(lambda: p.predict(zt, th, out=(mu, var)), 3, warmup=1)
    from paper_1507_04789_amd import MRA_CHECKPOINT
    ckpt_bytes = Plan(w.locs, M=w.M, J=w.J, r=w.r, cov=w.cov, pred=w.pred, flags=MRA_CHECKPOINT).work_bytes
    res = {"workload": "swaths_n4194304_matern32_M9_J4_r64_pred1048576",
           "work_arena_gb": p.work_bytes / 1e9, "work_arena_gb_checkpoint": ckpt_bytes / 1e9,
           "generation_s": gen_s,
           "loglik_grad_ms": ms_g, "loglik_grad_evals_per_s": 1000.0 / ms_g,
           "loglik_grad_fp64_pct_peak": 100.0 * p.info["flops_grad"] / (ms_g * 1e-3) / (PEAK_FP64_TFLOPS * 1e12),
           "loglik_ms": ms_l,
           "loglik_fp64_pct_peak": 100.0 * p.info["flops_loglik"] / (ms_l * 1e-3) / (PEAK_FP64_TFLOPS * 1e12),
           "predict_ms": ms_p, "n_pred": int(w.pred.shape[0]),
           "loglik": float(ll[0]), "finite": bool(torch.isfinite(g).all() and torch.isfinite(mu).all())}
    del p
    torch.cuda.empty_cache()
    return res


def _cpu_name():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def main():
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--n", type=int, default=262144)
    ap.add_argument("--M", type=int, default=6)
    ap.add_argument("--plain-steps", type=int, default=2, help="steps of the one-launch-per-task form (0: skip)")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--checkpoint-steps", type=int, default=10,
                    help="steps of the checkpointed form (MRA_CHECKPOINT; 0: skip)")
    ap.add_argument("--eager", action="store_true", help="time eager launches instead of captured-graph replays")
    ap.add_argument("--no-secondary", action="store_true",
                    help="skip the secondary workloads (small uniform case, loglik only, 64-vector batch)")
    ap.add_argument("--no-tune", action="store_true", help="keep the built-in launch shapes (no autotuning)")
    ap.add_argument("--swath", action="store_true",
                    help="also run the n = 2^22 satellite-swath workload (about 250 GB of HBM, a minute of host time)")
    ap.add_argument("--theta-batch", type=int, default=16, help="parameter vectors per call in the 64-vector case")
    ap.add_argument("--copy-probe", type=int, default=0, metavar="BYTES",
                    help="only run a plain copy of BYTES (counter calibration)")
    ap.add_argument("--summarize-profiles", metavar="DIR",
                    help="print the text summary of a profiling directory and exit")
    ap.add_argument("--copy-bytes", type=int, default=1 << 30)
    ap.add_argument("--summarize-engine", metavar="DIR",
                    help="print the text summary of a tile-engine probe run (DIR/engine.log, DIR/engine) and exit")
    args = ap.parse_args()
    if args.summarize_profiles:
        summarize_profiles(args.summarize_profiles, args.copy_bytes)
        return
    if args.summarize_engine:
        summarize_engine(args.summarize_engine)
        return
    if args.copy_probe:
        copy_probe(args.copy_probe)
        return
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU: the M-RA path here runs on a single MI355X "
              "(multi-GPU sharding is a design note, not built)", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_1507_04789_amd import MRA_GRAPH, Plan
    from paper_1507_04789_amd import workloads as wl

    dev = torch.device("cuda:0")
    w = wl.clustered(n=args.n, M=args.M)
    plan = Plan(w.locs, M=w.M, J=w.J, r=w.r, cov=w.cov, flags=0 if args.eager else MRA_GRAPH)
    cpu = None
    if not args.no_cpu:
        # host-only work first: the oracle's worker processes fork from a
        # process that has not touched the GPU
        print("cpu baseline: oracle on the bounded sample", file=sys.stderr, flush=True)
        cpu = cpu_baseline(65536, max(args.M - 1, 1), plan.info["flops_grad"])
    plan.bind(dev)
    z = torch.tensor(w.z, device=dev)
    th = torch.tensor(w.theta, device=dev).reshape(1, 3)
    ll = torch.empty(1, dtype=torch.float64, device=dev)
    g = torch.empty(1, 3, dtype=torch.float64, device=dev)
    flops = plan.info["flops_grad"]

    def timed(steps, profile=False):
        if profile:
            plan.profile(True)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        e0.record()
        for _ in range(steps):
            plan.loglik_grad(z, th, out=(ll, g))
        e1.record()
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        stats = None
        if profile:
            stats = plan.profile_read()
            plan.profile(False)
        return e0.elapsed_time(e1) / steps, wall, stats

    tuning = None
    if not args.no_tune:
        t0 = time.perf_counter()
        tuning = plan.autotune(z, th, reps=2)
        tuning["tuning_s"] = time.perf_counter() - t0
    for _ in range(args.warmup):
        plan.loglik_grad(z, th, out=(ll, g))
    torch.cuda.synchronize()
    # the timed region: captured-graph replays (or eager launches with --eager)
    ms, wall, _ = timed(args.steps)
    # per-kernel HIP-event timings: the same steps launched eagerly with
    # events around every launch group (graph replays carry no events)
    prof_steps = min(args.steps, 10)
    ms_prof, _, stats = timed(prof_steps, profile=True)
    llv, gv = float(ll[0]), g[0].tolist()
    if not (math.isfinite(llv) and all(math.isfinite(x) for x in gv)):
        raise RuntimeError("non-finite result: loglik %r grad %r" % (llv, gv))
    fam = _dominant(stats)
    dom = fam[0]
    per_launch_flops = dom["flops"] / dom["groups"]
    avg_ms = dom["total_ms"] / dom["groups"]
    achieved = per_launch_flops / (avg_ms * 1e-3) / 1e12

    plain = None
    if args.plain_steps > 0:
        pplan = Plan(w.locs, M=w.M, J=w.J, r=w.r, cov=w.cov, flags=2)
        pplan.bind(dev)
        pplan.loglik_grad(z, th)
        torch.cuda.synchronize()
        p0, p1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        p0.record()
        for _ in range(args.plain_steps):
            pll, pg = pplan.loglik_grad(z, th)
        p1.record()
        torch.cuda.synchronize()
        pms = p0.elapsed_time(p1) / args.plain_steps
        plain = {"value": 1000.0 / pms, "ms_per_step": pms, "steps": args.plain_steps,
                 "same_result": bool(float(pll[0]) == llv and pg[0].tolist() == gv)}
        del pplan
        torch.cuda.empty_cache()

    # the checkpointed form (MRA_CHECKPOINT): leaf phase in chunks, leaf
    # planes recomputed for the reverse pass; same workload, graph replays
    checkpoint = None
    if args.checkpoint_steps > 0:
        from paper_1507_04789_amd import MRA_CHECKPOINT
        work_stored = plan.work_bytes
        cplan = Plan(w.locs, M=w.M, J=w.J, r=w.r, cov=w.cov, flags=MRA_CHECKPOINT | (0 if args.eager else MRA_GRAPH))
        cplan.bind(dev)
        if tuning is not None:
            cplan.set_tuning({"families": tuning["families"]})
        cll = torch.empty(1, dtype=torch.float64, device=dev)
        cg = torch.empty(1, 3, dtype=torch.float64, device=dev)
        cms = _time_calls(lambda: cplan.loglik_grad(z, th, out=(cll, cg)), args.checkpoint_steps)
        checkpoint = {"value": 1000.0 / cms, "ms_per_step": cms, "steps": args.checkpoint_steps,
                      "work_bytes": cplan.work_bytes, "work_bytes_stored_form": work_stored,
                      "chunks": 8,
                      "same_result": bool(float(cll[0]) == llv and cg[0].tolist() == gv)}
        del cplan
        torch.cuda.empty_cache()

    secondary = None
    if not args.no_secondary:
        del plan
        torch.cuda.empty_cache()
        secondary = secondary_configs(dev, w, args.theta_batch)
        if args.swath:
            secondary["swaths_n4194304"] = swath_config(dev)

    out = {
        "metric": METRIC,
        "value": 1000.0 / ms,
        "unit": "evals/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": "clustered_n%d_matern32_M%d_J4_r64_loglik_grad" % (args.n, args.M),
                   "n": args.n, "M": args.M, "J": 4, "r": 64, "cov": "matern32",
                   "theta": {"sigma2": 1.0, "kappa": 0.1, "tau2": 0.01}, "batch_theta": 1},
        "fp64_pct_peak_step": 100.0 * flops / (ms * 1e-3) / (PEAK_FP64_TFLOPS * 1e12),
        "algorithmic_flops_per_step": flops,
        "roofline": {"bound": "mfma", "kernel": dom["name"], "achieved": achieved, "peak": PEAK_FP64_TFLOPS,
                     "unit": "TFLOP/s", "frac": achieved / PEAK_FP64_TFLOPS,
                     "traffic": _stored_traffic(dom["name"]), "traffic_unit": "bytes",
                     "flops_per_launch": per_launch_flops, "avg_launch_ms": avg_ms,
                     "executed": _executed(dom["name"], per_launch_flops, avg_ms),
                     "hbm": _hbm_side(_stored_traffic(dom["name"]), avg_ms)},
        "kernels": [{"name": f["name"], "ms_per_step": f["total_ms"] / prof_steps,
                     "tflops": (f["flops"] / (f["total_ms"] * 1e-3) / 1e12) if f["total_ms"] > 0 else None}
                    for f in fam],
        "form": "eager" if args.eager else "hipgraph",
        "tuning": tuning,
        "profiled_pass": {"steps": prof_steps, "ms_per_step": ms_prof,
                          "note": "eager launches with HIP events around every launch group; source of the "
                                  "kernel table and the roofline"},
        "plain": plain,
        "checkpoint": checkpoint,
        "secondary": secondary,
        "result": {"loglik": llv, "grad": gv},
        "wall_s_timed": wall,
    }
    if cpu is not None:
        out["cpu_baseline"] = cpu
    print(json.dumps(out))


if __name__ == "__main__":
    main()
