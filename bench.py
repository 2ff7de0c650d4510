"""Benchmark of the colour-coding DP on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload 2]

A step is one pass of the hot path over one batch: a fresh batch of random
colourings of the resident host graph (computed on the device) and the DP
over the pattern's nice tree decomposition for all of them (leaf,
introduce, forget and join nodes, root counts copied to the host).  The
graph upload and the decomposition are done once, before timing.

Prints one JSON line.  `value` is DP table entries per second: the sum over
all tree-decomposition nodes and colourings of |D_x| (the paper's nonzero
configurations) divided by the wall time of the steps.  The `roofline`
object is measured live with HIP events on the library's stream; the
`cpu_baseline` object times the CPU oracle on a bounded sample of the same
workload on this host's cores.
"""
import argparse
import concurrent.futures as cf
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

import paper_1908_11248_amd as cc  # noqa: E402
from paper_1908_11248_amd import workloads as W  # noqa: E402

HBM_PEAK_GBS = 8000.0
METRIC = "DP table entries/s; queries/s + p50/p99 latency, batched vs plain (bit-exact)"


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def kernel_source_hash():
    h = hashlib.sha256()
    for f in sorted(os.listdir(os.path.join(ROOT, "paper_1908_11248_amd", "csrc"))):
        with open(os.path.join(ROOT, "paper_1908_11248_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def traffic_for(kernel, workload, launches_algo_bytes):
    """HBM bytes per launch from the committed rocprofv3 counter summary, if
    it was taken on the current kernel sources; otherwise None."""
    path = os.path.join(ROOT, "profiles", "traffic_w%d.json" % workload)
    if not os.path.exists(path):
        return None
    with open(path) as fh:
        t = json.load(fh)
    if t.get("source_hash") != kernel_source_hash():
        return None
    k = t.get("kernels", {}).get(kernel)
    return None if k is None else k.get("bytes_per_launch")


def cpu_baseline(workload, g, pat, k, budget_s=15.0):
    """The oracle DP (single-threaded C) on a sample of colourings, one
    colouring per host thread."""
    import oracle as O

    w = W.workload(workload)
    cores = min(os.cpu_count() or 1, 16)
    td = None
    done = 0
    entries = 0
    t0 = time.perf_counter()
    nb = w.colorings

    def one(b):
        col = O.color_array(w.color_seed, b, g.n, k)
        r = O.dp_count(g, pat, k, col, td=td, sizes=True)
        return int(r["sizes"].sum())

    with cf.ThreadPoolExecutor(max_workers=cores) as ex:
        b = 0
        while b < nb and time.perf_counter() - t0 < budget_s:
            batch = list(range(b, min(nb, b + cores)))
            for e in ex.map(one, batch):
                entries += e
            done += len(batch)
            b += len(batch)
    dt = time.perf_counter() - t0
    return {"value": entries / dt, "unit": "entries/s", "cores": cores, "kind": "oracle",
            "sample": "%d of %d colourings of workload %d (%s), one colouring per thread, %.1f s"
                      % (done, nb, workload, w.name, dt)}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", type=int, default=2, choices=[1, 2, 3])
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--plain", type=int, default=4, help="colourings timed one at a time for the plain rate")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU: this build runs on a single MI355X; "
              "--gpus %d is not supported (multi-GPU sharding is described in DESIGN.md)" % args.gpus,
              file=sys.stderr)
        sys.exit(2)

    w = W.workload(args.workload)
    log("workload", w.index, w.name)
    g = W.workload_graph(args.workload)
    pat = W.workload_pattern(args.workload)
    ctx = cc.Context(0, arena_bytes=96 << 30)
    G = cc.load_graph(ctx, g.n, g.row_ptr, g.col)
    D = cc.build_decomposition(pat.n, pat.edges)

    def step(i):
        C = cc.color(ctx, G, w.k, w.color_seed + 1000003 * i, w.colorings)
        counts, ovf = cc.count(ctx, G, C, D)
        C.close()
        return counts

    for i in range(args.warmup):
        step(i)
        log("warmup", i, "done")
    ctx.profile_enable(True)
    entries = 0
    t0 = time.perf_counter()
    for i in range(args.steps):
        step(args.warmup + i)
        entries += int(ctx.last_table_sizes().sum())
    dt = time.perf_counter() - t0
    prof = ctx.profile_read()
    ctx.profile_enable(False)
    log("timed", args.steps, "steps in %.3f s" % dt)

    # plain path: the same colourings one at a time (the paper's single run)
    plain_rate = None
    if args.plain > 0:
        cols = [cc.color(ctx, G, w.k, w.color_seed + 7 + b, 1) for b in range(args.plain)]
        cc.count(ctx, G, cols[0], D)
        t1 = time.perf_counter()
        for C in cols:
            cc.count(ctx, G, C, D)
        plain_rate = args.plain / (time.perf_counter() - t1)

    dom = max(prof.items(), key=lambda kv: kv[1][1])
    name, (launches, ms, byts) = dom
    achieved = (byts / launches) / ((ms / launches) * 1e-3) / 1e9
    roofline = {"bound": "hbm", "kernel": name, "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
                "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
                "traffic": traffic_for(name, args.workload, byts / launches),
                "avg_launch_ms": round(ms / launches, 4), "algo_bytes_per_launch": round(byts / launches)}
    kernels = {k: {"launches": v[0], "ms": round(v[1], 3), "GBps": round(v[2] / (v[1] * 1e-3) / 1e9, 1) if v[1] else None}
               for k, v in sorted(prof.items(), key=lambda kv: -kv[1][1])}
    ms_per_step = dt / args.steps * 1e3
    out = {
        "metric": METRIC,
        "value": entries / dt,
        "unit": "entries/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u64",
        "data": "synthetic",
        "config": {"workload": w.name, "colorings_per_step": w.colorings, "k": w.k, "n_G": g.n, "m_G": g.m,
                   "pattern": pat.name, "pattern_edges": pat.edges, "width": D.width},
        "colorings_per_s": round(w.colorings * args.steps / dt, 2),
        "plain_colorings_per_s": round(plain_rate, 2) if plain_rate else None,
        "entries_per_step": entries // args.steps,
        "roofline": roofline,
        "kernels": kernels,
    }
    if not args.no_cpu_baseline:
        log("cpu baseline (oracle)")
        out["cpu_baseline"] = cpu_baseline(args.workload, g, pat, w.k)
    print(json.dumps(out), flush=True)
    ctx.close()


if __name__ == "__main__":
    main()
