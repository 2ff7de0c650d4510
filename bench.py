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
import math
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
    from paper_1908_11248_amd.profiling import kernel_source_hash as h

    return h()


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


def copy_calibration(mib):
    """One device-to-device copy of a known size through torch (device memory
    plumbing only): hardware byte counters of this kernel, divided by the
    bytes it must move, give the scale factor of the counters."""
    import torch

    n = mib << 20
    src = torch.ones(n, dtype=torch.uint8, device="cuda")
    dst = torch.empty(n, dtype=torch.uint8, device="cuda")
    torch.cuda.synchronize()
    dst.copy_(src)
    torch.cuda.synchronize()
    log("copy calibration: %d bytes read, %d bytes written" % (n, n))
    del src, dst


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
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--workload", type=int, default=2, choices=[1, 2, 3, 4, 5])
    ap.add_argument("--queries", type=int, default=0, help="queries of workloads 4/5 (0: 256 / 120)")
    ap.add_argument("--budget", type=float, default=3e7, help="DP entries per table and colouring (workloads 4/5)")
    ap.add_argument("--load", type=float, default=0.7, help="arrival rate / plain throughput (workload 5)")
    ap.add_argument("--inflight", type=int, default=4, help="concurrent queries while serving (workload 5)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--plain", type=int, default=4, help="colourings timed one at a time for the plain rate")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MIB",
                    help="first run one plain device copy of MIB mebibytes (reference kernel for counter scaling)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU (one MI355X); --gpus %d is not supported: colourings and "
              "queries are independent, so more GPUs would each take their own share" % args.gpus,
              file=sys.stderr)
        sys.exit(2)

    if args.copy_calibration:
        copy_calibration(args.copy_calibration)
    if args.workload in (4, 5):
        return bench_queries(args)
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

    # warm-up with every kernel timed: it names the dominant kernel and gives
    # the per-kernel table; the timed steps record events around that kernel
    # only, so the other launches run without event overhead
    ctx.profile_enable(True)
    for i in range(max(args.warmup, 1)):  # at least one step names the dominant kernel
        step(i)
        log("warmup", i, "done")
    prof_all = ctx.profile_read()
    if not prof_all:
        raise SystemExit("no kernel timings were recorded")
    dom_name = max(prof_all.items(), key=lambda kv: kv[1][1])[0]
    # one launch in `every`, with `every` coprime to the launches per step so
    # that the sample visits every launch site of the step
    per_step = max(1, prof_all[dom_name][0] // max(args.warmup, 1))
    every = 4
    while math.gcd(every, per_step) != 1:
        every += 1
    ctx.profile_enable(True)
    ctx.profile_filter(dom_name, every)
    entries = 0
    t0 = time.perf_counter()
    for i in range(args.steps):
        step(args.warmup + i)
        entries += int(ctx.last_table_sizes().sum())
    dt = time.perf_counter() - t0
    prof = ctx.profile_read()
    ctx.profile_filter(None)
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

    if not prof:
        raise SystemExit("no kernel timings were recorded")
    dom = max(prof.items(), key=lambda kv: kv[1][1])
    name, (launches, ms, byts) = dom
    achieved = (byts / launches) / ((ms / launches) * 1e-3) / 1e9
    roofline = {"bound": "hbm", "kernel": name, "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
                "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
                "traffic": traffic_for(name, args.workload, byts / launches),
                "avg_launch_ms": round(ms / launches, 4), "algo_bytes_per_launch": round(byts / launches)}
    kernels = {k: {"launches": v[0], "ms": round(v[1], 3), "GBps": round(v[2] / (v[1] * 1e-3) / 1e9, 1) if v[1] else None}
               for k, v in sorted(prof_all.items(), key=lambda kv: -kv[1][1])}
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
        "kernels_warmup": kernels,
    }
    if not args.no_cpu_baseline:
        log("cpu baseline (oracle)")
        out["cpu_baseline"] = cpu_baseline(args.workload, g, pat, w.k)
    print(json.dumps(out), flush=True)
    ctx.close()


def bench_queries(args):
    """Workloads 4 and 5: streams of uneven pattern queries over a resident
    host graph.  Queries over the per-colouring table budget are redrawn
    (workloads.select_queries); the redraws are reported."""
    w = W.workload(args.workload)
    nq = args.queries or (256 if args.workload == 4 else 120)
    log("workload", w.index, w.name, "queries", nq)
    g = W.workload_graph(args.workload)
    log("graph", g.n, g.m)
    ctx = cc.Context(0, arena_bytes=0)
    G = cc.load_graph(ctx, g.n, g.row_ptr, g.col)
    B = w.colorings
    budget1 = int(args.budget)

    def fits(p, s):
        log("select", p.name, hex(s))
        D = cc.build_decomposition(p.n, p.edges)
        C = cc.color(ctx, G, p.n, W.colouring_seed(s), 1)
        ctx.set_table_budget(budget1)
        try:
            cc.count(ctx, G, C, D)
            return True
        except cc.CcError as e:
            if e.code != cc.CC_ERANGE:
                raise
            return False
        finally:
            ctx.set_table_budget(0)
            C.close()

    t0 = time.perf_counter()
    sel, redraws = W.select_queries(args.workload, nq, fits)
    t_sel = time.perf_counter() - t0
    log("selected %d queries in %.1f s, %d redraws" % (len(sel), t_sel, sum(redraws.values())))
    ctx.set_table_budget(budget1 * B)
    decs = [cc.build_decomposition(p.n, p.edges) for p, _ in sel]
    fam = {}
    for p, _ in sel:
        fam["%s%d" % (p.family, p.n)] = fam.get("%s%d" % (p.family, p.n), 0) + 1

    if args.workload == 4:
        cols = [cc.color(ctx, G, p.n, W.colouring_seed(s), B) for p, s in sel]
        queries = list(zip(decs, cols))
        # plain: one query at a time on one stream (the paper's sequential runs)
        t0 = time.perf_counter()
        plain = []
        for qi, (D, C) in enumerate(queries):
            plain.append(cc.count(ctx, G, C, D))
            if qi % 16 == 15:
                log("plain query", qi + 1, "at %.1f s" % (time.perf_counter() - t0))
        t_plain = time.perf_counter() - t0
        log("plain %.2f s" % t_plain)
        lanes = cc.tune_batch(ctx, G, queries[: min(32, len(queries))])
        log("tuned lanes", lanes)
        for i in range(args.warmup):
            cc.count_batch(ctx, G, queries)
        ctx.profile_enable(True)
        t0 = time.perf_counter()
        entries = 0
        for i in range(args.steps):
            out = cc.count_batch(ctx, G, queries)
            entries += int(ctx.last_table_sizes().sum())
        dt = time.perf_counter() - t0
        prof = ctx.profile_read()
        ctx.profile_enable(False)
        same = all(np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1]) for a, b in zip(out, plain))
        if not same:
            raise SystemExit("batched counts differ from plain counts")
        extra = {"plain_queries_per_s": round(len(sel) / t_plain, 3),
                 "batched_queries_per_s": round(len(sel) * args.steps / dt, 3),
                 "batched_vs_plain": round((len(sel) * args.steps / dt) / (len(sel) / t_plain), 3),
                 "bit_identical_batched_vs_plain": same, "lanes": lanes}
        value = entries / dt
        ms_per_step = dt / args.steps * 1e3
    else:
        # plain rate first (one at a time), then Poisson arrivals at a fixed
        # fraction of it, served with `inflight` lanes and with one lane
        t0 = time.perf_counter()
        plain_counts = []
        for qi, ((p, s), D) in enumerate(zip(sel, decs)):
            C = cc.color(ctx, G, p.n, W.colouring_seed(s), B)
            tq = time.perf_counter()
            plain_counts.append(cc.count(ctx, G, C, D)[0])
            log("plain query", qi, p.name, "%.3f s" % (time.perf_counter() - tq))
            C.close()
        t_plain = time.perf_counter() - t0
        plain_qps = len(sel) / t_plain
        lam = args.load * plain_qps
        rng = np.random.Generator(np.random.PCG64(w.seed ^ 0xA5))
        gaps = rng.exponential(1.0 / lam, size=len(sel))
        log("plain %.2f q/s; arrivals at %.2f q/s" % (plain_qps, lam))

        def serve(inflight):
            srv = cc.Server(ctx, G, max_inflight=inflight, max_entries=budget1 * B, max_heavy=1)
            tickets = []
            t_start = time.perf_counter()
            due = t_start
            for i, ((p, s), D) in enumerate(zip(sel, decs)):
                due += gaps[i]
                while time.perf_counter() < due:
                    time.sleep(min(0.0005, max(0.0, due - time.perf_counter())))
                tickets.append(srv.submit(D, p.n, W.colouring_seed(s), B))
            log("submitted", len(tickets), "queries with", inflight, "lanes")
            res = []
            for i, t in enumerate(tickets):
                res.append(srv.wait(t))
                if i % 10 == 9:
                    log("served", i + 1)
            st = srv.stop()
            ok = all(r[0] == 1 for r in res) and all(np.array_equal(r[1], c) for r, c in zip(res, plain_counts))
            return st, ok

        ctx.profile_enable(True)
        st_b, ok_b = serve(args.inflight)
        prof = ctx.profile_read()
        ctx.profile_enable(False)
        log("served", st_b)
        st_p, ok_p = serve(1)
        log("one lane", st_p)
        if not (ok_b and ok_p):
            raise SystemExit("served counts differ from plain counts")
        extra = {"plain_queries_per_s": round(plain_qps, 3), "arrival_rate_qps": round(lam, 3),
                 "served": {k: (round(v, 3) if isinstance(v, float) else v) for k, v in st_b.items()},
                 "served_one_lane": {k: (round(v, 3) if isinstance(v, float) else v) for k, v in st_p.items()},
                 "p50_ms": round(st_b["p50_ms"], 2), "p99_ms": round(st_b["p99_ms"], 2),
                 "p99_vs_one_lane": round(st_b["p99_ms"] / st_p["p99_ms"], 3) if st_p["p99_ms"] else None,
                 "bit_identical_served_vs_plain": True, "inflight": args.inflight, "max_heavy": 1}
        value = st_b["qps"]
        dt = st_b["wall_s"]
        ms_per_step = dt * 1e3
    if not prof:
        raise SystemExit("no kernel timings were recorded")
    dom = max(prof.items(), key=lambda kv: kv[1][1])
    name, (launches, ms, byts) = dom
    achieved = (byts / launches) / ((ms / launches) * 1e-3) / 1e9
    out = {
        "metric": METRIC,
        "value": value,
        "unit": "entries/s" if args.workload == 4 else "queries/s",
        "n_gpus": 1, "steps": args.steps if args.workload == 4 else 1, "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 3), "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "u64", "data": "synthetic",
        "config": {"workload": w.name, "queries": len(sel), "colorings_per_query": B, "n_G": g.n, "m_G": g.m,
                   "budget_entries_per_table_per_coloring": budget1, "families": fam,
                   "redraws": {"%s%d" % k: v for k, v in sorted(redraws.items())}, "selection_s": round(t_sel, 1)},
        "roofline": {"bound": "hbm", "kernel": name, "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": None,
                     "avg_launch_ms": round(ms / launches, 4), "algo_bytes_per_launch": round(byts / launches)},
    }
    out.update(extra)
    print(json.dumps(out), flush=True)
    ctx.close()


if __name__ == "__main__":
    main()
