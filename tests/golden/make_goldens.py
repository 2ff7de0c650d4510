"""Writes the oracle's counts for the five standard workloads at their own
sizes into tests/golden/ (test infrastructure; calls only the CPU oracle and
the seeded input generators, never the HIP library).

    python tests/golden/make_goldens.py [2 3 4 5] [--workers N]

Files (one line per value, each with a header naming this command):
  w2_counts.txt   workload 2: all 64 colourings            b count overflow
  w3_counts.txt   workload 3: all 32 colourings            b count overflow
  w4_counts.txt   workload 4: colouring 0 of all 256 queries (selected under
                  the workload's admission rule); the 5-cycles, whose largest
                  table holds about 4e8 entries per colouring, by four
                  sampled ranges of the image of pattern vertex 0
                  q seed name b lo hi count overflow   (lo hi = 0 n: full count)
  w5_sample.txt   workload 5: colouring 0 of a seeded sample of 32 of the
                  first 200 queries of the stream       same format
"""
import argparse
import concurrent.futures as cf
import multiprocessing as mp
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import oracle as O  # noqa: E402
from paper_1908_11248_amd import workloads as W  # noqa: E402

W5_STREAM = 200
W5_SAMPLE = 32

_G = {}


def _graph(index):
    if index not in _G:
        _G[index] = W.workload_graph(index)
    return _G[index]


def _one(task):
    index, q, seed, name, k, edges, b, cseed, lo, hi = task
    g = _graph(index)
    pat = W.Pattern(k, [tuple(e) for e in edges], name)
    col = O.color_array(cseed, b, g.n, k)
    t0 = time.perf_counter()
    if lo == 0 and hi == g.n:
        r = O.dp_count(g, pat, k, col)
    else:
        r = O.dp_count_range(g, pat, k, col, lo, hi)
    return task, r["count"], int(r["overflow"]), time.perf_counter() - t0


def _run(tasks, workers, out_path, header, fmt):
    ctx = mp.get_context("fork")
    rows = {}
    t0 = time.perf_counter()
    with cf.ProcessPoolExecutor(max_workers=workers, mp_context=ctx) as ex:
        futs = [ex.submit(_one, t) for t in tasks]
        for i, f in enumerate(cf.as_completed(futs)):
            task, cnt, ovf, dt = f.result()
            rows[task] = (cnt, ovf)
            print("%s: %d/%d done (%.1f s, last %.1f s)" % (os.path.basename(out_path), i + 1, len(tasks),
                                                             time.perf_counter() - t0, dt), flush=True)
    with open(out_path, "w") as fh:
        fh.write(header)
        for t in tasks:
            fh.write(fmt(t, *rows[t]) + "\n")


def _hdr(what):
    return ("# %s\n# written by: python tests/golden/make_goldens.py (CPU oracle + seeded generators only)\n" % what)


def w_single(index, workers):
    w = W.workload(index)
    g = _graph(index)
    pat = W.workload_pattern(index)
    edges = tuple(tuple(e) for e in pat.edges)
    tasks = [(index, 0, 0, pat.name, w.k, edges, b, w.color_seed, 0, g.n) for b in range(w.colorings)]
    _run(tasks, workers, os.path.join(HERE, "w%d_counts.txt" % index),
         _hdr("workload %d (%s): oracle counts of all %d colourings\n# b count overflow" % (index, w.name, w.colorings)),
         lambda t, c, o: "%d %d %d" % (t[6], c, o))


def _ranges(g, seed):
    rng = np.random.Generator(np.random.PCG64(seed))
    x = int(rng.integers(0, g.n - 2000))
    return [(0, 64), (1000, 1500), (x, x + 2000), (g.n - 5000, g.n)]


def w_queries(index, workers):
    g = _graph(index)
    if index == 4:
        sel, _ = W.select_queries(4, 256)
        picked = list(range(len(sel)))
        what = "workload 4 (%s): colouring 0 of all %d queries" % (W.workload(4).name, len(sel))
        out = "w4_counts.txt"
    else:
        sel, _ = W.select_queries(5, W5_STREAM)
        rng = np.random.Generator(np.random.PCG64(W.workload(5).seed ^ 0x5A))
        picked = sorted(int(x) for x in rng.choice(len(sel), size=W5_SAMPLE, replace=False))
        what = ("workload 5 (%s): colouring 0 of a seeded sample of %d of the first %d queries"
                % (W.workload(5).name, W5_SAMPLE, W5_STREAM))
        out = "w5_sample.txt"
    tasks = []
    for q in picked:
        p, s = sel[q]
        cs = W.colouring_seed(s)
        if p.family == "cycle":
            for lo, hi in _ranges(g, s):
                tasks.append((index, q, s, p.name, p.n, tuple(tuple(e) for e in p.edges), 0, cs, lo, hi))
        else:
            tasks.append((index, q, s, p.name, p.n, tuple(tuple(e) for e in p.edges), 0, cs, 0, g.n))
    # the largest patterns first, so the pool drains evenly
    tasks.sort(key=lambda t: -t[4])
    _run(tasks, workers, os.path.join(HERE, out),
         _hdr(what + "\n# q seed name b lo hi count overflow (lo hi = 0 n_G: the full count)"),
         lambda t, c, o: "%d %d %s %d %d %d %d %d" % (t[1], t[2], t[3], t[6], t[8], t[9], c, o))
    # rewrite in query order
    path = os.path.join(HERE, out)
    lines = open(path).read().splitlines()
    head = [l for l in lines if l.startswith("#")]
    body = sorted((l for l in lines if not l.startswith("#")), key=lambda l: (int(l.split()[0]), int(l.split()[4])))
    with open(path, "w") as fh:
        fh.write("\n".join(head + body) + "\n")


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("which", nargs="*", type=int, default=[2, 3, 4, 5])
    ap.add_argument("--workers", type=int, default=0)
    a = ap.parse_args()
    for index in a.which:
        t0 = time.perf_counter()
        if index in (2, 3):
            w_single(index, a.workers or (8 if index == 2 else 6))
        else:
            w_queries(index, a.workers or (3 if index == 4 else 2))
        print("workload %d goldens in %.0f s" % (index, time.perf_counter() - t0), flush=True)


if __name__ == "__main__":
    main()
