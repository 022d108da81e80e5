#!/usr/bin/env python3
"""Throughput of the random-tree Monte Carlo hot path on one MI355X.

Workload (default): the 1-D Fisher equation u_t = u_xx + u - u^2 with the travelling-wave initial data
(1 + e^{x/sqrt6})^-2, 64 points in [-10, 10] times t in {0.5, 1, 2} (192 queries), 1e6 trees per point,
series order 12 with pruning, Pade [6/6], FP32 paths with FP64 clock, products and moments.

One step = one run of the whole path (tree walk, per-bin moment reduction, FP64 finalize with Pade)
over all 192 points, captured once into a HIP graph on a created stream and replayed, with the inputs
already resident in HBM.

Prints one JSON line on stdout (progress goes to stderr):
  value          trees per second over the timed steps (whole job)
  latency_ms     p50/p99 of per-step latency (one step answers the 192 point queries)
  roofline       the walker kernel: algorithmic VALU operations per launch / its average duration
                 (HIP events on the launch stream), against the FP32 vector peak expressed in ops
  cpu_baseline   the CPU oracle timed on a bounded sample of the same trees, on the host's cores
  parity         the sampled trees compared with the oracle (shape bit-exact, value within tolerance)
  pade_parity    when the sample is the whole workload: the Pade values against the oracle's, point by
                 point, and both against the exact travelling wave
"""
from __future__ import annotations

import argparse
import hashlib
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "random trees/sec at fixed error vs oracle; p50/p99 point-query latency"

# Algorithmic work per tree node, in 32-bit VALU lane operations (a 32x32->64 product counts 2, an FP64
# operation 1, a transcendental 1).  Per node: Philox4x32-10 80 (10 rounds x (2 wide products = 4,
# 2 three-input xors = 4)); uniform conversions 8; clock product and test 2; Box-Muller 7 (log, scale,
# sqrt, sin, cos, two products); exponential time 2; Brownian step 3 + 2 d; then either a vertex
# (count, prune test, time left and clamp, arity product and lookup, weight exponent, exp, two
# products: 12) or a leaf (initial data: about 9 for the logistic families), counted as 10 on average.
OPS_PER_NODE = {1: 114, 2: 116}
# FP32 vector peak of MI355X expressed in operations: 157.3 TFLOP/s counts an FMA as 2 flops, i.e.
# 78.6 T lane-operations/s (256 CUs x 4 SIMDs x 32 lanes per cycle x 2.4 GHz).  Plain, non-packed VALU
# code reaches it: a microbenchmark of independent FMA chains measured 62.6 T FMA/s on an MI355X.
PEAK_TOPS = 78.6


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def workload(name):
    from paper_2402_06491_amd import inputs

    if name == "fisher":
        return inputs.fisher()
    if name == "kpp":
        return inputs.kpp()
    if name == "cubic_2d":
        return inputs.cubic_2d()
    if name == "poly_batch":
        return inputs.poly_batch()
    raise SystemExit(f"unknown workload {name}")


def describe(wl):
    if wl["name"] == "fisher_1d":
        return ("fisher_1d: u_t=u_xx+u-u^2, u0=(1+e^{x/sqrt6})^-2, 64 x in [-10,10] x t in {0.5,1,2}, "
                "1e6 trees/point, order 12 pruned, Pade [6/6], FP32 paths, FP64 clock/products/moments")
    return wl["name"]


def cpu_threads():
    """Worker threads for the CPU oracle: the host cores this process may use, at most 16 (the CPU share
    of one GPU on the benchmark machines)."""
    try:
        n = len(os.sched_getaffinity(0))
    except AttributeError:
        n = os.cpu_count() or 1
    return max(1, min(n, 16))


def cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(wl, gpu_meta, gpu_f, target_s):
    """Time the oracle on the first S trees of every point (a calibration run as warm-up, then the median
    of 3 timed runs); compare the trees of the first timed run with the GPU records.  Returns the
    baseline, the tree parity and the oracle's records (for the Pade parity)."""
    import oracle

    oracle.build(force=False)
    threads = cpu_threads()
    npts = len(wl["t"])
    n_trees = np.asarray(wl["n_trees"], dtype=np.int64)
    base = np.concatenate([[0], np.cumsum(n_trees)])
    prob = wl["problems"][0]

    def run(S):
        t0 = time.perf_counter()
        recs = []
        for p in range(npts):
            r = oracle.walk_point(prob, wl["mc"], wl["x"][p], float(wl["t"][p]), p, S, nthreads=threads)
            recs.append(r)
        return time.perf_counter() - t0, recs

    dt, _ = run(2000)  # calibration and warm-up
    rate = npts * 2000 / max(dt, 1e-6)
    S = int(min(n_trees.min(), max(1000, rate * target_s / npts)))
    log(f"cpu baseline: {threads} threads of {os.cpu_count()} ({cpu_model()}), calibrated {rate:.3g} trees/s, "
        f"sample {S} trees x {npts} points, median of 3")
    times = []
    recs = None
    for rep in range(3):
        dt, r = run(S)
        times.append(dt)
        if rep == 0:
            recs = r
        del r
    dt = float(np.median(times))
    # parity of the sampled trees: shapes bit-exact; values within tol |F| + 1e-6 max_point |F|
    tol = 2e-4 if wl["mc"]["precision"] == 32 else 1e-12
    max_rel, mism, checked, worst_ratio, worst = 0.0, 0, 0, 0.0, []
    for p, r in enumerate(recs):
        sl = slice(int(base[p]), int(base[p]) + S)
        m = gpu_meta[sl].astype(np.uint32)
        mism += int(np.sum((m & 0xFF) != np.minimum(r["ne"], 255)))
        mism += int(np.sum((m >> 11) != r["nodes"]))
        fl = ((m >> 8) & 1) + 2 * ((m >> 9) & 1)
        mism += int(np.sum(fl != r["flags"]))
        absF = np.abs(r["F"])
        diff = np.abs(gpu_f[sl] - r["F"])
        floor = (1e-6 * absF.max()) if wl["mc"]["precision"] == 32 else 1e-300
        ratio = diff / (tol * absF + floor + 1e-300)
        k = int(np.argmax(ratio))
        if ratio[k] > worst_ratio:
            worst_ratio = float(ratio[k])
            worst = [p, k, int(r["ne"][k]), int(r["nodes"][k]), float(gpu_f[sl][k]), float(r["F"][k])]
        big = absF > 1e-3 * max(absF.max(), 1e-300)
        if big.any():
            max_rel = max(max_rel, float((diff[big] / absF[big]).max()))
        checked += S
    return ({"value": npts * S / dt, "unit": "trees/s", "cores": threads, "nproc": os.cpu_count(),
             "cpu_model": cpu_model(), "runs_s": times, "kind": "oracle",
             "sample": f"first {S} trees of each of the {npts} points ({npts * S} trees, median {dt:.1f} s of 3 "
                       f"runs after a warm-up)"},
            {"trees_checked": checked, "shape_mismatches": mism, "max_rel_tree_diff_big": max_rel,
             "tree_tol": tol, "worst_err_over_bound": worst_ratio,
             "worst_tree": dict(zip(["point", "tree", "ne", "nodes", "F_gpu", "F_oracle"], worst))},
            recs if S == int(n_trees.min()) == int(n_trees.max()) else None)


def describe_extra(wl):
    if wl["name"] == "kpp_1d":
        return ("kpp_1d: u_t=0.5u_xx+u^2-u, u0=1/(1+e^x), 16 x in [-4,4], t=1, 1e5 trees/point, unpruned "
                "(bins 0..63 + tail), node cap 2^16, FP64")
    if wl["name"] == "poly_batch":
        return (f"poly_batch: 4096 points of 8 PDEs (f of degree 2..5, coefficients U[-1,1]), t log-uniform "
                f"in [0.25,4], 1e4..1e6 trees/point (log-uniform), order 12 pruned, Pade [6/6], "
                f"FP{wl['mc']['precision']} paths")
    return wl["name"]


def cpu_sample_rate(wl, target_s):
    """The oracle on a proportional sample of a workload (the first ceil(f n_i) trees of every point, so
    the sample has the workload's mix of points): a calibration run as warm-up, then the median of 3."""
    import oracle

    oracle.build(force=False)
    threads = cpu_threads()
    n_trees = np.asarray(wl["n_trees"], dtype=np.int64)
    pid = np.asarray(wl.get("problem_id", np.zeros(len(n_trees), np.uint32)))

    def run(f):
        k = np.maximum(1, np.ceil(f * n_trees)).astype(np.int64)
        t0 = time.perf_counter()
        for p in range(len(n_trees)):
            oracle.walk_point(wl["problems"][int(pid[p])], wl["mc"], wl["x"][p], float(wl["t"][p]), p, int(k[p]),
                              nthreads=threads)
        return time.perf_counter() - t0, int(k.sum())

    f = min(1.0, 2e5 / max(1, n_trees.sum()))
    dt, n = run(f)
    f = min(1.0, f * target_s / max(dt, 1e-3))
    times = []
    for _ in range(3):
        dt, n = run(f)
        times.append(dt)
    dt = float(np.median(times))
    return {"value": n / dt, "unit": "trees/s", "cores": threads, "nproc": os.cpu_count(), "cpu_model": cpu_model(),
            "runs_s": times, "kind": "oracle",
            "sample": f"first {f:.4g} of every point's trees ({n} trees, the workload's mix), median {dt:.2f} s of 3 "
                      f"runs after a warm-up"}


def config_bench(ctx, wl, steps, warmup, cpu_s):
    """Throughput of one more workload: the same step (walk, reduce, finalize) replayed as a graph on a
    created stream, the walker's duration from HIP events in timing mode, and the oracle on a sample."""
    import tempfile

    import torch

    import paper_2402_06491_amd as brt

    tuned = ctx.autotune(wl["problems"], wl["mc"], wl["x"], wl["t"], wl["n_trees"], problem_id=wl.get("problem_id"),
                         cache_path=os.path.join(tempfile.gettempdir(), "brt_autotune.jsonl"))
    plan = brt.Plan(ctx, wl["problems"], wl["mc"], wl["x"], wl["t"], wl["n_trees"], problem_id=wl.get("problem_id"))
    out = plan.outputs(records=False)
    stream = torch.cuda.Stream()
    with torch.cuda.stream(stream):
        for _ in range(warmup):
            plan.execute(out, stream=stream)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    with torch.cuda.stream(stream):
        for _ in range(steps):
            plan.execute(out, stream=stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    graph = plan.graph_stats()
    plan.set_timing(True)
    with torch.cuda.stream(stream):
        for _ in range(steps):
            plan.execute(out, stream=stream)
    (walk_ms, red_ms, fin_ms), runs = plan.get_timing()
    plan.set_timing(False)
    nodes = int(out["nodes"].sum().item())
    flags = out["flags"].cpu().numpy()
    plan.close()
    del out
    total = int(np.sum(wl["n_trees"]))
    dim = int(wl["problems"][0]["dim"])
    walk_s = walk_ms / runs / 1e3
    achieved = nodes * OPS_PER_NODE[dim] / walk_s / 1e12
    res = {"workload": describe_extra(wl), "points": len(wl["t"]), "total_trees": total,
           "value": total * steps / wall, "unit": "trees/s", "ms_per_step": wall * 1e3 / steps, "steps": steps,
           "dtype": "f32" if wl["mc"]["precision"] == 32 else "f64", "launch": tuned, "graph": graph,
           "roofline": {"bound": "alu", "achieved": achieved, "peak": PEAK_TOPS, "unit": "Top/s",
                        "frac": achieved / PEAK_TOPS, "traffic": None, "kernel": "walk_kernel",
                        "kernel_ms": walk_s * 1e3, "nodes_per_launch": nodes, "ops_per_node": OPS_PER_NODE[dim],
                        "reduce_ms": red_ms / runs, "finalize_ms": fin_ms / runs},
           "pade": {"pole_flagged": int(((flags & 1) != 0).sum()), "sensitive_flagged": int(((flags & 32) != 0).sum()),
                    "lowered": int(((flags & 2) != 0).sum())}}
    log(f"{wl['name']} FP{wl['mc']['precision']}: {wall * 1e3 / steps:.3f} ms/step, {res['value']:.4g} trees/s, "
        f"walker {walk_s * 1e3:.3f} ms ({100 * achieved / PEAK_TOPS:.1f}% of peak), reduce {red_ms / runs:.3f} ms, "
        f"finalize {fin_ms / runs:.3f} ms")
    if cpu_s > 0:
        res["cpu_baseline"] = cpu_sample_rate(wl, cpu_s)
        log(f"{wl['name']} FP{wl['mc']['precision']} cpu baseline {res['cpu_baseline']['value']:.4g} trees/s "
            f"({res['cpu_baseline']['sample']})")
    return res


def pade_parity(wl, recs, gpu):
    """The headline's Pade values against the oracle's, from the oracle's walk of every tree of every
    point: the oracle's moments (exact sums), coefficients and Pade summary per point, then the same
    point-by-point rule as the parity tests (a point is exempt from the 1e-3 bound only when both sides
    flag it POLE or SENSITIVE), and the error of both against the exact travelling wave per t."""
    import oracle
    from paper_2402_06491_amd import inputs

    mc = wl["mc"]
    L, M, no = int(mc["pade_L"]), int(mc["pade_M"]), int(mc["max_order"])
    nz = oracle.normalize(wl["problems"][0], mc)
    rows = []
    for p, rec in enumerate(recs):
        mom = oracle.moments(rec, mc)
        a, cov = oracle.coefficients(mom, nz.mu, float(wl["t"][p]))
        summ = oracle.pade_summary(a[: no + 1], cov[: no + 1, : no + 1], L, M)
        fl = int(gpu["flags"][p])
        dev_flag = bool(fl & 33)
        orc_flag = summ["pole"] or summ["sensitive"]
        rows.append({"p": p, "t": float(wl["t"][p]), "du": abs(float(gpu["u"][p]) - summ["pade"]),
                     "both": dev_flag and orc_flag, "either": dev_flag or orc_flag,
                     "same_order": (int(gpu["pade_diag"][p][0]), int(gpu["pade_diag"][p][1])) == summ["pade_order"],
                     "u_gpu": float(gpu["u"][p]), "u_orc": summ["pade"],
                     "exact": float(inputs.fisher_exact(float(wl["x"][p][0]), float(wl["t"][p])))
                     if wl["name"] == "fisher_1d" else float("nan")})
    unf = [r for r in rows if not r["both"]]
    out = {"points": len(rows), "flagged_both": int(sum(r["both"] for r in rows)),
           "flagged_either": int(sum(r["either"] for r in rows)),
           "unflagged_max_abs_du": float(max((r["du"] for r in unf), default=0.0)),
           "unflagged_within_1e-3": int(sum(r["du"] <= 1e-3 for r in unf)), "unflagged": len(unf),
           "degree_mismatches": int(sum(not r["same_order"] for r in rows)),
           "rule": "|u_gpu - u_oracle| <= 1e-3 at every point unless the device and the oracle both flag it "
                   "(pole within 0.5 of [0, 1], or kappa = sum |du/da_k||a_k| > 100)"}
    if wl["name"] == "fisher_1d":
        per_t = {}
        for t in sorted(set(r["t"] for r in rows)):
            sel = [r for r in rows if r["t"] == t]
            ok = [r for r in sel if not r["either"]]
            per_t[str(t)] = {"points": len(sel), "unflagged": len(ok),
                             "gpu_max_abs_err_vs_exact_unflagged": float(max((abs(r["u_gpu"] - r["exact"]) for r in ok), default=float("nan"))),
                             "gpu_median_abs_err_vs_exact_unflagged": float(np.median([abs(r["u_gpu"] - r["exact"]) for r in ok])) if ok else None,
                             "oracle_median_abs_err_vs_exact_unflagged": float(np.median([abs(r["u_orc"] - r["exact"]) for r in ok])) if ok else None}
        out["vs_exact_wave"] = per_t
    return out


def pmc_record(kernel_src_sha, name="walk_fisher_pmc.json"):
    """A kernel's committed rocprofv3 counter summary, if it was taken on the current kernel source
    (else None)."""
    path = os.path.join(ROOT, "profiles", name)
    try:
        d = json.load(open(path))
    except (OSError, ValueError):
        return None
    return d if d.get("kernel_source_sha256") == kernel_src_sha else None


def pmc_traffic(kernel_src_sha, launch=None, name="walk_fisher_pmc.json"):
    """HBM bytes per launch of a kernel from its committed counter summary (None if stale), and the
    launch they were taken at: the summary's record for `launch` when it holds one, else its latest."""
    d = pmc_record(kernel_src_sha, name)
    if not d:
        return None, None
    for r in d.get("by_launch", []):
        if launch is not None and r.get("launch") == launch:
            return r["hbm_bytes_per_launch"], r["launch"]
    return d.get("hbm_bytes_per_launch"), d.get("launch")


def source_sha(files):
    h = hashlib.sha256()
    for f in files:
        h.update(open(os.path.join(ROOT, "paper_2402_06491_amd", "csrc", f), "rb").read())
    return h.hexdigest()


def walker_source_sha():
    return source_sha(("brt_kernels.hip", "brt_internal.h"))


def adi_source_sha():
    return source_sha(("brt_pdd.hip",))  # the ADI kernel and its launch live in this file alone


COPY_BYTES = 512 << 20  # the plain device copy of --pmc-calibration
FISHER_WALKER = "walk_kernel<float, 1, 1, 0, 0>"  # the headline's walker (1-D, logistic data, one problem, Strategy A)


def pmc_summary(fetch_dir, write_dir, command, launch=None, which="both"):
    """Write profiles/walk_fisher_pmc.json (and profiles/adi_pdd_cubic_2d_pmc.json when the runs include
    the domain-decomposition tail) from two rocprofv3 --pmc runs of this script (FETCH_SIZE, then
    WRITE_SIZE, with --pmc-calibration): the last dispatch of each kernel (the timed plan's last direct
    walker launch, the last 1000-step solve) and the calibration copy, whose known size gives each
    counter's scale."""
    import csv

    def read(d, counter, kernel="walk_kernel"):
        rows = []
        for root, _, files in os.walk(d):
            for f in files:
                if f.endswith("counter_collection.csv"):
                    rows += list(csv.DictReader(open(os.path.join(root, f))))
        per = {}
        for r in rows:
            if r["Counter_Name"] != counter:
                continue
            key = (int(r["Dispatch_Id"]), r["Kernel_Name"])
            per[key] = per.get(key, 0.0) + float(r["Counter_Value"])
        walk = [v for (i, k), v in sorted(per.items()) if kernel in k]
        copy = [v for (i, k), v in sorted(per.items()) if "copyBuffer(" in k or k.endswith("copyBuffer")]
        if not copy:
            copy = [v for (i, k), v in sorted(per.items()) if "copyBuffer" in k and "Rect" not in k]
        return (walk[-1] if walk else None), copy[-1]

    fw, fc = read(fetch_dir, "FETCH_SIZE", FISHER_WALKER)
    ww, wc = read(write_dir, "WRITE_SIZE", FISHER_WALKER)
    fs = COPY_BYTES / (fc * 1024.0)
    ws = COPY_BYTES / (wc * 1024.0)
    if which in ("both", "walker"):
        wl = workload("fisher")
        trees = int(np.sum(wl["n_trees"]))
        out = {"kernel": "walk_kernel", "workload": wl["name"], "kernel_source_sha256": walker_source_sha(),
               "fetch_kib_per_dispatch": fw, "write_kib_per_dispatch": ww,
               "copy_fetch_kib": fc, "copy_write_kib": wc, "copy_bytes": COPY_BYTES,
               "fetch_scale": fs, "write_scale": ws,
               "hbm_bytes_per_launch": fw * 1024.0 * fs + ww * 1024.0 * ws,
               "algorithmic_bytes_per_launch": 12 * trees, "command": command}
        if launch:
            out["launch"] = json.loads(launch)  # the walker launch the counter runs used
        # one record per launch shape taken on the current source (the spill traffic depends on it)
        path = os.path.join(ROOT, "profiles", "walk_fisher_pmc.json")
        prev = pmc_record(out["kernel_source_sha256"]) or {}
        keys = ("fetch_kib_per_dispatch", "write_kib_per_dispatch", "fetch_scale", "write_scale",
                "hbm_bytes_per_launch", "launch")
        out["by_launch"] = [r for r in prev.get("by_launch", []) if r.get("launch") != out.get("launch")]
        out["by_launch"].append({k: out.get(k) for k in keys})
        json.dump(out, open(path, "w"), indent=1)
        print(json.dumps(out))
    if which not in ("both", "adi"):
        return
    fa, _ = read(fetch_dir, "FETCH_SIZE", "adi_kernel")
    wa, _ = read(write_dir, "WRITE_SIZE", "adi_kernel")
    if fa is not None and wa is not None:
        from paper_2402_06491_amd import inputs

        g = inputs.pdd_cubic_2d()["grid"]
        interior = g["px"] * g["py"] * (g["cx"] - 1) * (g["cy"] - 1)
        adi = {"kernel": "adi_kernel", "workload": "pdd_cubic_2d", "kernel_source_sha256": adi_source_sha(),
               "steps_per_launch": g["n_steps"], "fetch_kib_per_dispatch": fa, "write_kib_per_dispatch": wa,
               "copy_fetch_kib": fc, "copy_write_kib": wc, "copy_bytes": COPY_BYTES,
               "fetch_scale": fs, "write_scale": ws,
               "hbm_bytes_per_launch": fa * 1024.0 * fs + wa * 1024.0 * ws,
               "algorithmic_bytes_per_launch": 40.0 * interior * g["n_steps"], "command": command}
        json.dump(adi, open(os.path.join(ROOT, "profiles", "adi_pdd_cubic_2d_pmc.json"), "w"), indent=1)
        print(json.dumps(adi))


def serve_stream(ctx, reqs, mc, opts, realtime=True):
    """Replay a request stream through a brt_server (in real time, or all requests at once); returns its
    statistics and every completed request's result."""
    import paper_2402_06491_amd as brt

    srv = brt.Server(ctx, 2, "gauss_sum", mc, **opts)
    pending, results, rejected = {}, {}, 0

    def collect():
        for tk, (rid, n) in list(pending.items()):
            r = srv.poll(tk, n)
            if r is not None:
                results[rid] = r
                del pending[tk]

    t0 = time.perf_counter()
    last_log = t0
    for r in reqs:
        while realtime and time.perf_counter() - t0 < r["arrival"]:
            collect()
            time.sleep(0.0005)
        try:
            pending[srv.submit(r["problem"], r["x"], r["t"], stream_id=r["id"])] = (r["id"], len(r["t"]))
        except brt.BrtError as e:
            if e.code != -4:
                raise
            rejected += 1
        if time.perf_counter() - last_log > 10.0:
            last_log = time.perf_counter()
            log(f"serving: {r['id'] + 1} requests submitted, {len(results)} completed")
    srv.drain(timeout_s=900.0)
    collect()
    st = srv.stats()
    srv.close()
    st["rejected_at_submit"] = rejected
    return st, results


def plain_per_request(ctx, reqs, results, mc):
    """The plain path: one brt_solve launch per request, in arrival order, each point with the trees the
    server gave it (the same Philox trees, so the same estimates and errors).  Latency from the measured
    service times with first-come-first-served queueing at the recorded arrival times."""
    import torch

    import paper_2402_06491_amd as brt

    finish, lat, trees = 0.0, [], 0
    t_first = reqs[0]["arrival"]
    for r in reqs:
        res = results[r["id"]]
        n = len(r["t"])
        nt = res["trees"].astype(np.int64)
        ids = (r["id"] * 1024 + np.arange(n)).astype(np.uint32)
        t0 = time.perf_counter()
        brt.solve(ctx, r["problem"], mc, r["x"], r["t"], nt, point_id=ids, records=False)
        torch.cuda.synchronize()
        svc = time.perf_counter() - t0
        start = max(finish, r["arrival"])
        finish = start + svc
        lat.append(finish - r["arrival"])
        trees += int(nt.sum())
    lat = np.array(lat)
    span = finish - t_first
    return {"requests": len(reqs), "trees": trees, "span_s": span, "trees_per_s": trees / span,
            "p50_latency_s": float(np.percentile(lat, 50)), "p99_latency_s": float(np.percentile(lat, 99)),
            "mean_latency_s": float(lat.mean())}


def family_plan_rate(ctx):
    """The plan rate on the served family: the 2-D cubic problem's 1536 interface points x 1e5 trees in
    one plan (FP32 paths, t = 1), replayed as a graph; trees and tree nodes per second (the served
    points' times differ, so their trees differ in size: nodes compare the two)."""
    import torch

    import paper_2402_06491_amd as brt
    from paper_2402_06491_amd import inputs

    wl = inputs.cubic_2d(n_trees=100_000)
    plan = brt.Plan(ctx, wl["problems"], wl["mc"], wl["x"], wl["t"], wl["n_trees"], problem_id=wl["problem_id"])
    out = plan.outputs(records=False)
    stream = torch.cuda.Stream()
    with torch.cuda.stream(stream):
        plan.execute(out, stream=stream)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(5):
            plan.execute(out, stream=stream)
        torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / 5
    nodes = int(out["nodes"].sum().item())
    plan.close()
    return int(np.sum(wl["n_trees"])) / dt, nodes / dt


def serve_bench(ctx, duration, rate, opts, plain_requests, saturated_requests):
    """The served mixed-size query stream (Poisson arrivals, 1..1024 points per request, target SE, tree
    cap): continuous batching in real time; the plain one-launch-per-request path on the stream's first
    requests; the server saturated with requests (all submitted at once) against the plan rate."""
    from paper_2402_06491_amd import inputs

    reqs = inputs.served_stream(rate=rate, duration=duration)
    mc = inputs.mc_params(seed=0, max_order=12, prune=1, precision=32)
    log(f"serving: {len(reqs)} requests over {duration} s ({sum(len(r['t']) for r in reqs)} points)")
    out = {"requests": len(reqs), "arrival_rate_per_s": rate, "duration_s": duration,
           "points": int(sum(len(r["t"]) for r in reqs)), **{k: v for k, v in opts.items()}}
    st, res = serve_stream(ctx, reqs, mc, opts)
    se = np.concatenate([res[r["id"]]["se"] for r in reqs if r["id"] in res])
    tr = np.concatenate([res[r["id"]]["trees"] for r in reqs if r["id"] in res]).astype(np.int64)
    out["batched"] = {"trees_per_s": st["trees_per_s"], "p50_latency_s": st["p50_latency_s"],
                      "p99_latency_s": st["p99_latency_s"], "mean_latency_s": st["mean_latency_s"],
                      "completed": st["completed"], "trees": st["trees"], "ticks": st["ticks"],
                      "span_s": st["span_s"], "device_busy_s": st["busy_s"],
                      "points_at_target_se": int(np.sum(se <= opts["target_se"])),
                      "points_at_tree_cap": int(np.sum((se > opts["target_se"]) & (tr >= opts["max_trees"]))),
                      "share_at_target_se": float(np.mean(se <= opts["target_se"])),
                      "mean_trees_per_point": float(tr.mean())}
    b = out["batched"]
    log(f"serving batched: {b['trees_per_s']:.4g} trees/s, p50 {b['p50_latency_s']:.3f} s, p99 "
        f"{b['p99_latency_s']:.3f} s, {b['completed']} completed in {b['span_s']:.2f} s; "
        f"{100 * b['share_at_target_se']:.1f}% of points reached SE <= {opts['target_se']}")
    head = [r for r in reqs if r["id"] in res][:plain_requests]
    if head:
        out["plain_one_launch_per_request"] = plain_per_request(ctx, head, res, mc)
        lat = np.array([res[r["id"]]["latency_s"] for r in head])
        out["batched_same_requests"] = {"requests": len(head), "p50_latency_s": float(np.percentile(lat, 50)),
                                        "p99_latency_s": float(np.percentile(lat, 99))}
        pl = out["plain_one_launch_per_request"]
        log(f"serving plain (first {len(head)} requests): {pl['trees_per_s']:.4g} trees/s, p50 "
            f"{pl['p50_latency_s']:.3f} s, p99 {pl['p99_latency_s']:.3f} s; batched on the same requests: p50 "
            f"{out['batched_same_requests']['p50_latency_s']:.3f} s, p99 {out['batched_same_requests']['p99_latency_s']:.3f} s")
    sat = reqs[:saturated_requests]
    if sat:
        st2, _ = serve_stream(ctx, sat, mc, opts, realtime=False)
        rate_plan, node_rate_plan = family_plan_rate(ctx)
        node_rate = st2["nodes"] / st2["span_s"]
        out["saturated"] = {"requests": len(sat), "trees_per_s": st2["trees_per_s"], "span_s": st2["span_s"],
                            "device_busy_s": st2["busy_s"], "plan_trees_per_s": rate_plan,
                            "fraction_of_plan_rate": st2["trees_per_s"] / rate_plan,
                            "nodes_per_s": node_rate, "plan_nodes_per_s": node_rate_plan,
                            "fraction_of_plan_node_rate": node_rate / node_rate_plan}
        log(f"serving saturated ({len(sat)} requests at once): {st2['trees_per_s']:.4g} trees/s = "
            f"{100 * st2['trees_per_s'] / rate_plan:.1f}% of the plan rate {rate_plan:.4g} trees/s; "
            f"{node_rate:.4g} nodes/s = {100 * node_rate / node_rate_plan:.1f}% of the plan's {node_rate_plan:.4g}")
    return out


def pdd_bench(ctx, trees_per_node, cpu_steps):
    """The domain-decomposition tail of the 2-D cubic workload: Monte Carlo at the 2640 line nodes,
    spline interpolation, 1000 ADI steps on 4 x 4 subdomains of 512^2 cells.  Reports stage times and
    the ADI kernel's rate against HBM (40 algorithmic bytes per interior node and step: the x phase
    reads u^n and u^{n-1} and writes the y phase's right-hand side, the y phase reads it and writes
    u^{n+1})."""
    import torch

    import paper_2402_06491_amd as brt
    from paper_2402_06491_amd import inputs

    wl = inputs.pdd_cubic_2d(n_trees=trees_per_node)
    g = wl["grid"]
    pd = brt.Pdd(ctx, wl["problem"], g)
    xy, t = pd.nodes()
    node_u = torch.empty(len(t), dtype=torch.float64, device="cuda")
    field = torch.empty((pd.NY + 1, pd.NX + 1), dtype=torch.float64, device="cuda")
    times = []
    stream = torch.cuda.Stream()
    with torch.cuda.stream(stream):  # a created stream: the nodes' plan is captured once and replayed
        for rep in range(3):  # the first run builds the nodes' plan and captures its graph
            pd.run(wl["mc"], trees_per_node, node_u=node_u, field=field)
            times.append(pd.timing())
    torch.cuda.synchronize()
    mc_ms, int_ms, solve_ms = (min(x[k] for x in times[1:]) for k in range(3))
    interior = g["px"] * g["py"] * (g["cx"] - 1) * (g["cy"] - 1)
    alg_bytes = 40.0 * interior * g["n_steps"]
    achieved = alg_bytes / (solve_ms * 1e-3) / 1e9
    n_groups, die_local = pd.barrier()
    u = field.cpu().numpy()
    res = {"workload": wl["name"], "nodes": int(len(t)), "trees_per_node": int(trees_per_node),
           "grid": {k: g[k] for k in ("px", "py", "cx", "cy", "n_steps", "ns_x", "nt")},
           "mc_ms": mc_ms, "interp_ms": int_ms, "solve_ms": solve_ms,
           "adi_us_per_step": solve_ms * 1e3 / g["n_steps"],
           "adi_roofline": {"bound": "hbm", "achieved": achieved, "peak": 8000.0, "unit": "GB/s",
                            "frac": achieved / 8000.0, "algorithmic_bytes": alg_bytes,
                            "traffic": pmc_traffic(adi_source_sha(), name="adi_pdd_cubic_2d_pmc.json")[0]},
           "barrier_groups": n_groups, "die_local_groups": die_local,
           "field_finite": bool(np.isfinite(u).all()), "field_max": float(np.abs(u).max())}
    pd.close()
    if cpu_steps > 0:
        from oracle import pdd as opdd

        og = opdd.Grid(**g)
        vals = opdd.g_grid(wl["problem"], xy[:, 0], xy[:, 1])  # stand-in node values: timing only
        bd = opdd.boundary_data(og, wl["problem"], vals)
        t0 = time.perf_counter()
        opdd.adi_solve(og, wl["problem"], bd, n_steps=cpu_steps)
        dt = time.perf_counter() - t0
        res["cpu_baseline"] = {"value": dt * 1e3 / cpu_steps, "unit": "ms/step", "kind": "oracle",
                               "cores": 1, "sample": f"first {cpu_steps} ADI steps of the same grid (numpy/LAPACK)"}
    log(f"pdd tail: MC {mc_ms:.2f} ms, interpolation {int_ms:.3f} ms, {g['n_steps']} ADI steps {solve_ms:.2f} ms "
        f"({achieved:.0f} GB/s algorithmic)")
    return res


def strategy_compare(ctx, wl, ms_a, se_a, qs=(0.4, 0.5, 0.6, 0.7), reps=5):
    """Strategy B (Sec. 2.2) on the same workload and trees, against Strategy A's step time and standard
    errors: the efficiency ratio (time x SE^2 of A) / (time x SE^2 of B) compares the two at equal error
    (the paper reports B 1.2-1.6x faster at equal maximum error)."""
    import torch

    import paper_2402_06491_amd as brt

    stream = torch.cuda.current_stream()
    rows = []
    for q in qs:
        mc = dict(wl["mc"], strategy=1, q=q)
        plan = brt.Plan(ctx, wl["problems"], mc, wl["x"], wl["t"], wl["n_trees"],
                        problem_id=wl.get("problem_id"), point_id=wl.get("point_id"))
        out = plan.outputs(records=True)
        plan.execute(out)
        ev = [torch.cuda.Event(enable_timing=True) for _ in range(2)]
        torch.cuda.synchronize()
        ev[0].record(stream)
        for _ in range(reps):
            plan.execute(out)
        ev[1].record(stream)
        torch.cuda.synchronize()
        ms_b = ev[0].elapsed_time(ev[1]) / reps
        se_b = out["se"].cpu().numpy()
        ok = np.isfinite(se_a) & np.isfinite(se_b) & (se_b > 0) & (se_a > 0)
        ratio = (ms_a * se_a[ok] ** 2) / (ms_b * se_b[ok] ** 2)
        rows.append({"q": q, "ms_per_step": ms_b, "trees_per_s": float(np.sum(wl["n_trees"])) / (ms_b * 1e-3),
                     "efficiency_vs_A_median": float(np.median(ratio)),
                     "efficiency_vs_A_total": float(ms_a * np.sum(se_a[ok] ** 2) / (ms_b * np.sum(se_b[ok] ** 2)))})
        log(f"strategy B q={q}: {ms_b:.3f} ms/step, efficiency vs A {rows[-1]['efficiency_vs_A_median']:.3f} (median), "
            f"{rows[-1]['efficiency_vs_A_total']:.3f} (total)")
        plan.close()
        del out
    return {"strategy_A_ms_per_step": ms_a, "strategy_B": rows,
            "what": "efficiency = (time x SE^2 of A) / (time x SE^2 of B) per point, same trees per point"}


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="fisher")
    ap.add_argument("--cpu-seconds", type=float, default=15.0,
                    help="upper bound of one timed oracle run (the whole workload when it fits)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--serve-seconds", type=float, default=60.0,
                    help="length of the served request stream replayed after the throughput steps (0: skip)")
    ap.add_argument("--serve-rate", type=float, default=200.0)
    ap.add_argument("--serve-max-trees", type=int, default=1 << 20)
    ap.add_argument("--serve-max-points", type=int, default=16384, help="the server's device slots")
    ap.add_argument("--serve-round-trees", type=int, default=32768, help="trees per point per tick")
    ap.add_argument("--serve-plain-requests", type=int, default=1000,
                    help="requests of the stream replayed through one brt_solve launch each")
    ap.add_argument("--serve-saturated-requests", type=int, default=1000,
                    help="requests of the stream submitted at once to measure the server's full rate")
    ap.add_argument("--pdd-trees", type=int, default=100_000,
                    help="trees per node of the domain-decomposition tail run after the steps (0: skip)")
    ap.add_argument("--pdd-cpu-steps", type=int, default=5)
    ap.add_argument("--no-strategy-b", action="store_true")
    ap.add_argument("--configs", default="kpp,poly_batch",
                    help="more workloads timed after the headline (comma list of kpp, poly_batch; empty: none)")
    ap.add_argument("--config-steps", type=int, default=5)
    ap.add_argument("--config-cpu-seconds", type=float, default=2.0)
    ap.add_argument("--pmc-calibration", action="store_true",
                    help="end with a plain 512 MiB device copy (scale of the rocprofv3 byte counters)")
    ap.add_argument("--pmc-summary", nargs=2, metavar=("FETCH_DIR", "WRITE_DIR"),
                    help="write the counter summaries under profiles/ from two rocprofv3 --pmc runs and exit")
    ap.add_argument("--pmc-command", default="", help="the command of the counter runs, recorded in the summary")
    ap.add_argument("--pmc-launch", default="", help="the walker launch of the counter runs (JSON), recorded in the summary")
    ap.add_argument("--launch", default="",
                    help="the headline walker's launch (JSON, e.g. for counter runs at a given launch) instead of "
                         "the autotuner's")
    ap.add_argument("--pmc-which", default="both", choices=("both", "walker", "adi"),
                    help="which kernels' summaries --pmc-summary writes")
    args = ap.parse_args()
    if args.pmc_summary:
        pmc_summary(args.pmc_summary[0], args.pmc_summary[1], args.pmc_command, args.pmc_launch or None,
                    args.pmc_which)
        return
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU only: the library has no multi-GPU path (run with --gpus 1)",
              file=sys.stderr)
        sys.exit(2)

    import torch

    import paper_2402_06491_amd as brt

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    wl = workload(args.workload)
    log(f"workload {wl['name']}: {len(wl['t'])} points, {int(np.sum(wl['n_trees']))} trees")
    ctx = brt.Context(0)
    import tempfile

    t_tune = time.perf_counter()
    if args.launch:
        ctx.set_launch(**json.loads(args.launch))
        tuned = ctx.get_launch()
        log(f"launch {tuned} (given)")
    else:
        tuned = ctx.autotune(wl["problems"], wl["mc"], wl["x"], wl["t"], wl["n_trees"],
                             problem_id=wl.get("problem_id"),
                             cache_path=os.path.join(tempfile.gettempdir(), "brt_autotune.jsonl"))
        log(f"autotuned launch {tuned} in {time.perf_counter() - t_tune:.1f} s")
    plan = brt.Plan(ctx, wl["problems"], wl["mc"], wl["x"], wl["t"], wl["n_trees"],
                    problem_id=wl.get("problem_id"), point_id=wl.get("point_id"))
    out = plan.outputs(records=True)
    # A created stream: brt_plan_execute captures the step (walk, reduce, finalize) into a HIP graph on
    # its first run and replays it afterwards (torch's default stream is NULL, where it would enqueue
    # kernel by kernel).
    stream = torch.cuda.Stream()
    with torch.cuda.stream(stream):
        for i in range(args.warmup):
            plan.execute(out, stream=stream)
    torch.cuda.synchronize()
    log(f"warmup done ({args.warmup} steps)")

    # ---- timed region: K graph replays ----
    starts = [torch.cuda.Event(enable_timing=True) for _ in range(args.steps)]
    ends = [torch.cuda.Event(enable_timing=True) for _ in range(args.steps)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    with torch.cuda.stream(stream):
        for i in range(args.steps):
            starts[i].record(stream)
            plan.execute(out, stream=stream)
            ends[i].record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    graph = plan.graph_stats()
    lat = np.array([s.elapsed_time(e) for s, e in zip(starts, ends)])
    total_trees = int(np.sum(wl["n_trees"]))
    value = total_trees * args.steps / wall
    log(f"timed {args.steps} steps: {wall * 1e3 / args.steps:.3f} ms/step, {value:.4g} trees/s; graph {graph}")

    # ---- walker kernel duration with HIP events on the launch stream (timing mode enqueues the
    # kernels one by one, with events between them) ----
    plan.set_timing(True)
    with torch.cuda.stream(stream):
        for i in range(args.steps):
            plan.execute(out, stream=stream)
    (walk_ms, red_ms, fin_ms), runs = plan.get_timing()
    plan.set_timing(False)
    walk_s = walk_ms / runs / 1e3
    nodes = int(out["nodes"].sum().item())
    dim = int(wl["problems"][0]["dim"])
    ops = nodes * OPS_PER_NODE[dim]
    achieved = ops / walk_s / 1e12
    sha = walker_source_sha()
    traffic, traffic_launch = pmc_traffic(sha, tuned)
    roofline = {"bound": "alu", "achieved": achieved, "peak": PEAK_TOPS, "unit": "Top/s",
                "frac": achieved / PEAK_TOPS, "traffic": traffic, "traffic_launch": traffic_launch,
                "kernel": "walk_kernel", "kernel_ms": walk_s * 1e3, "nodes_per_launch": nodes,
                "ops_per_node": OPS_PER_NODE[dim], "reduce_ms": red_ms / runs, "finalize_ms": fin_ms / runs}
    log(f"walk kernel {walk_s * 1e3:.3f} ms, {nodes} nodes, {achieved:.2f} Top/s "
        f"({100 * achieved / PEAK_TOPS:.1f}% of {PEAK_TOPS}); reduce {red_ms / runs:.3f} ms, "
        f"finalize {fin_ms / runs:.3f} ms")

    u = out["u"].cpu().numpy()
    flags = out["flags"].cpu().numpy()
    result = {
        "metric": METRIC, "value": value, "unit": "trees/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": wall * 1e3 / args.steps, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f32" if wl["mc"]["precision"] == 32 else "f64",
        "data": "synthetic",
        "config": {"workload": describe(wl), "points": len(wl["t"]), "total_trees": total_trees,
                   "nodes_per_step": nodes, "parallelism": "single GPU, persistent work-stealing launch",
                   "launch": tuned},
        "latency_ms": {"p50": float(np.percentile(lat, 50)), "p99": float(np.percentile(lat, 99)),
                       "what": "one step = all point queries of the workload"},
        "graph": dict(graph, what="HIP graphs instantiated / graph launches / kernel-by-kernel runs of the "
                                  "timed plan over warmup and timed steps"),
        "roofline": roofline,
        "pade": {"finite": int(np.isfinite(u).sum()), "pole_flagged": int(((flags & 1) != 0).sum()),
                 "sensitive_flagged": int(((flags & 32) != 0).sum()),
                 "lowered": int(((flags & 2) != 0).sum())},
    }
    if not args.no_cpu_baseline:
        meta = out["tree_meta"].cpu().numpy()
        f = out["tree_f"].cpu().numpy()
        cb, parity, recs = cpu_baseline(wl, meta, f, args.cpu_seconds)
        del meta, f
        result["cpu_baseline"] = cb
        result["parity"] = parity
        log(f"cpu baseline {cb['value']:.4g} trees/s on {cb['cores']} threads; parity {parity}")
        if recs is not None:
            gpu = {k: out[k].cpu().numpy() for k in ("u", "flags", "pade_diag")}
            t_pp = time.perf_counter()
            result["pade_parity"] = pade_parity(wl, recs, gpu)
            log(f"pade parity ({time.perf_counter() - t_pp:.1f} s): {result['pade_parity']}")
        del recs
    se_a = out["se"].cpu().numpy()
    plan.close()
    del out, starts, ends
    if not args.no_strategy_b:
        result["strategy_b"] = strategy_compare(ctx, wl, wall * 1e3 / args.steps, se_a)
    if args.configs:
        from paper_2402_06491_amd import inputs

        extra = {}
        headline_launch = ctx.get_launch()
        for name in [c for c in args.configs.split(",") if c]:
            if name == "kpp":
                extra["kpp_fp64"] = config_bench(ctx, inputs.kpp(), args.config_steps, 1, args.config_cpu_seconds)
            elif name == "poly_batch":
                for prec in (32, 64):
                    extra[f"poly_batch_fp{prec}"] = config_bench(ctx, inputs.poly_batch(precision=prec),
                                                                 args.config_steps, 1, args.config_cpu_seconds)
            else:
                raise SystemExit(f"unknown config {name}")
        ctx.set_launch(**headline_launch)  # the serving and tail legs below run with the headline's settings
        result["configs"] = extra
    if args.serve_seconds > 0:
        result["serving"] = serve_bench(ctx, args.serve_seconds, args.serve_rate,
                                        {"max_points": args.serve_max_points, "round_trees": args.serve_round_trees,
                                         "max_trees": args.serve_max_trees, "target_se": 1e-3,
                                         "queue_cap": 100_000}, args.serve_plain_requests,
                                        args.serve_saturated_requests)
    if args.pdd_trees > 0:
        result["pdd"] = pdd_bench(ctx, args.pdd_trees, args.pdd_cpu_steps)
    if args.pmc_calibration:
        a = torch.ones(COPY_BYTES // 8, dtype=torch.float64, device="cuda")
        b = torch.empty_like(a)
        b.copy_(a)
        torch.cuda.synchronize()
        del a, b
    # Explicit teardown while the HIP runtime (and a profiler attached to it) is still up: the library's
    # objects, then torch's cached device memory; nothing GPU-side is left for exit-time destructors.
    ctx.close()
    torch.cuda.synchronize()
    torch.cuda.empty_cache()
    print(json.dumps(result), flush=True)


if __name__ == "__main__":
    main()
