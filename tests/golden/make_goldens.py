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
                  sampled ranges of the image of pattern vertex 0, and every
                  query whose full count exceeds the oracle's caps (12 GiB of
                  address space, 300 s) by two such ranges; a range over the
                  caps is listed in the header as skipped
                  q seed name b lo hi count overflow   (lo hi = 0 n: full count)
  w5_sample.txt   workload 5: colouring 0 of a seeded sample of 32 of the
                  first 200 queries of the stream, under caps of 12 GiB and
                  900 s per oracle run (one colouring of a 5-vertex partial
                  3-tree takes the oracle about 500 s on CL(10^6))
                                                        same format
"""
import argparse
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


MEM_CAP = 12 << 30  # address-space limit of one oracle process
TIME_CAP = 300.0  # seconds for one oracle task (--time-cap)


def _child(task, conn):
    import resource

    resource.setrlimit(resource.RLIMIT_AS, (MEM_CAP, MEM_CAP))
    try:
        conn.send(("ok",) + _one(task)[1:3])
    except Exception as e:  # ENOMEM of the oracle under the limit, or MemoryError
        conn.send(("fail", repr(e)))
    conn.close()


def _fallback(task, n):
    """Two anchor ranges of the image of pattern vertex 0 in place of a full
    count that exceeded the caps."""
    index, q, seed, name, k, edges, b, cseed, lo, hi = task
    rng = np.random.Generator(np.random.PCG64(seed ^ 0xA5))
    x = int(rng.integers(0, n - 500))
    return [(index, q, seed, name, k, edges, b, cseed, 0, 64), (index, q, seed, name, k, edges, b, cseed, x, x + 500)]


def _run(tasks, workers, out_path, header, fmt, n=None):
    """Runs the oracle tasks, each in a process of its own with MEM_CAP bytes
    of address space and TIME_CAP seconds, and writes one line per finished
    task.  A full count that exceeds either cap is replaced by two anchor
    ranges (_fallback); a range that exceeds them is recorded as skipped.
    Finished lines go to <out_path>.part as they come, so an interrupted run
    resumes where it stopped."""
    ctx = mp.get_context("fork")
    part = out_path + ".part"
    done = {}
    if os.path.exists(part):
        for line in open(part):
            key, val = line.rsplit("|", 1)
            done[key] = val.strip()
    rows, skipped = {}, []
    queue = list(tasks)
    todo = []
    while queue:
        t = queue.pop(0)
        v = done.get(repr(t))
        if v is None:
            todo.append(t)
        elif v == "skip":
            if n is not None and (t[8], t[9]) == (0, n):
                queue.extend(_fallback(t, n))
            else:
                skipped.append(t)
        else:
            c, o = v.split()
            rows[t] = (int(c), int(o))
    t0 = time.perf_counter()
    running = {}
    with open(part, "a") as ph:
        def record(t, val):
            ph.write("%r|%s\n" % (t, val))
            ph.flush()

        while todo or running:
            while todo and len(running) < workers:
                t = todo.pop(0)
                a, b_ = ctx.Pipe(duplex=False)
                pr = ctx.Process(target=_child, args=(t, b_))
                pr.start()
                b_.close()
                running[t] = (pr, a, time.perf_counter())
            time.sleep(0.2)
            for t in list(running):
                pr, a, ts = running[t]
                res = None
                if a.poll():
                    try:
                        res = a.recv()
                    except EOFError:
                        res = ("fail", "died")
                elif not pr.is_alive():
                    res = ("fail", "exit %s" % pr.exitcode)
                elif time.perf_counter() - ts > TIME_CAP:
                    pr.kill()
                    res = ("fail", "time cap")
                if res is None:
                    continue
                pr.join()
                a.close()
                del running[t]
                dt = time.perf_counter() - ts
                if res[0] == "ok":
                    rows[t] = (res[1], res[2])
                    record(t, "%d %d" % (res[1], res[2]))
                    what = "done"
                else:
                    record(t, "skip")
                    if n is not None and (t[8], t[9]) == (0, n):
                        todo.extend(_fallback(t, n))
                        what = "over the caps (%s): two ranges instead" % res[1]
                    else:
                        skipped.append(t)
                        what = "over the caps (%s): skipped" % res[1]
                print("%s: %d finished, %d queued, %d running (%.0f s; task q%d n_F %d [%d,%d) %.1f s) %s"
                      % (os.path.basename(out_path), len(rows), len(todo), len(running), time.perf_counter() - t0,
                         t[1], t[4], t[8], t[9], dt, what), flush=True)
    with open(out_path, "w") as fh:
        fh.write(header)
        for t in skipped:
            fh.write("# skipped: q %d %s [%d, %d) exceeds the oracle's caps\n" % (t[1], t[3], t[8], t[9]))
        for t in tasks + [x for x in rows if x not in tasks]:
            if t in rows:
                fh.write(fmt(t, *rows[t]) + "\n")
    os.remove(part)


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
    # the smallest patterns first
    tasks.sort(key=lambda t: (t[4], t[1]))
    _run(tasks, workers, os.path.join(HERE, out),
         _hdr(what + "\n# q seed name b lo hi count overflow (lo hi = 0 n_G: the full count)"),
         lambda t, c, o: "%d %d %s %d %d %d %d %d" % (t[1], t[2], t[3], t[6], t[8], t[9], c, o), n=g.n)
    # rewrite in query order
    path = os.path.join(HERE, out)
    lines = open(path).read().splitlines()
    head = [l for l in lines if l.startswith("#")]
    body = sorted(set(l for l in lines if not l.startswith("#")), key=lambda l: (int(l.split()[0]), int(l.split()[4])))
    with open(path, "w") as fh:
        fh.write("\n".join(head + body) + "\n")


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("which", nargs="*", type=int, default=[2, 3, 4, 5])
    ap.add_argument("--workers", type=int, default=0)
    ap.add_argument("--time-cap", type=float, default=0.0, help="seconds per oracle task (default 300; 900 for workload 5)")
    a = ap.parse_args()
    global TIME_CAP
    for index in a.which:
        t0 = time.perf_counter()
        if index in (2, 3):
            w_single(index, a.workers or (8 if index == 2 else 6))
        else:
            TIME_CAP = a.time_cap or (900.0 if index == 5 else 300.0)
            w_queries(index, a.workers or (3 if index == 5 else 4))
        print("workload %d goldens in %.0f s" % (index, time.perf_counter() - t0), flush=True)


if __name__ == "__main__":
    main()
