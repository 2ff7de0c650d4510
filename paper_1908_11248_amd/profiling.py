"""Summaries of rocprofv3 output for the profiles/ folder.

    python -m paper_1908_11248_amd.profiling stats  <kernel_stats.csv | results.db> <out.md> <command...>
    python -m paper_1908_11248_amd.profiling traffic <fetch_dir> <write_dir> <copy_mib> <out.json> <command...>
    python -m paper_1908_11248_amd.profiling window <results.db> <bench.json> <out.md>

`stats` turns a --kernel-trace --stats CSV (or the database rocprofv3 writes
by default) into a short table.  `window` appends to such a table the
dispatches of the bench line's roofline kernel (and its nested batched
line's) that ran inside the line's timed window (CLOCK_MONOTONIC
nanoseconds, the clock of the trace) and their mean duration beside the
bench's own HIP-event figure.  `traffic`
reads two --pmc runs (FETCH_SIZE, WRITE_SIZE; values in KiB per dispatch),
scales every dispatch by the factor measured on the calibration copy kernel
(bytes it must move / bytes counted) and writes bytes per launch per kernel,
keyed by the short kernel names the library's profiler uses, together with a
hash of the kernel sources the counters were taken on.
"""
import csv
import glob
import hashlib
import json
import os
import re
import sys
from collections import defaultdict

HERE = os.path.dirname(os.path.abspath(__file__))

# device kernel -> library profiler name
KERNEL_NAMES = [
    (r"k_slot_edge_push", "slot_edge_push"), (r"k_slot_edge_leaf", "slot_edge_leaf"), (r"k_slot_edge", "slot_edge"),
    (r"k_slot_leaf_join", "slot_leaf_join"), (r"k_slot_join", "slot_join"),
    (r"k_slot_root", "slot_root"),
    (r"k_slot_leaf", "slot_leaf"), (r"k_slot_counters", "slot_counters"),
    (r"k_edge<.*true, true>", "edge_emit"), (r"k_edge<.*true, false>", "edge_emit"),
    (r"k_edge<.*false, true>", "edge_count"), (r"k_edge<.*false, false>", "edge_count"),
    (r"k_join<.*true>", "join_emit"), (r"k_join<.*false>", "join_count"),
    (r"k_forget<.*true>", "forget_emit"), (r"k_forget<.*false>", "forget_count"),
    (r"k_expand_entry<.*true>", "entry_emit"), (r"k_expand_entry<.*false>", "entry_count"),
    (r"k_entry_seglen", "entry_seglen"), (r"k_push_seglen", "push_seglen"), (r"k_pull_seglen", "pull_seglen"),
    (r"k_expand_ball<.*true>", "ball_emit"), (r"k_expand_ball<.*false>", "ball_count"), (r"k_ball_seglen", "ball_seglen"),
    (r"k_join_pairs", "join_pairs"), (r"k_drop_last", "drop_last"), (r"k_reduce_runs", "reduce_runs"),
    (r"k_take_runs", "take_runs"), (r"k_expand_bounds", "expand_bounds"),
    (r"k_expand<.*true, true>", "pull_emit"), (r"k_expand<.*false, true>", "pull_count"),
    (r"k_expand<.*true, false>", "push_emit"), (r"k_expand<.*false, false>", "push_count"),
    (r"k_leaf_pull<.*true>", "leaf_pull_emit"), (r"k_leaf_pull<.*false>", "leaf_pull_count"),
    (r"k_tri<.*true>", "tri_emit"), (r"k_tri<.*false>", "tri_count"),
    (r"k_pull_index", "pull_index"), (r"k_root", "root"), (r"k_heads", "heads"),
    (r"k_group_starts", "group_starts"), (r"k_scan", "scan"), (r"k_radix", "radix_sort"),
    (r"k_permute", "permute"), (r"k_leaf_emit", "leaf_emit"), (r"k_leaf_count", "leaf_count"),
]


def short_name(full):
    for pat, name in KERNEL_NAMES:
        if re.search(pat, full):
            return name
    return None


def code_only(text):
    """C++/HIP source text without its comments, whitespace runs collapsed to
    one space (string and character literals kept as written), so that an
    edit of comments or layout leaves the code's hash unchanged."""
    out, i, n = [], 0, len(text)
    while i < n:
        c = text[i]
        if c in "\"'":
            j = i + 1
            while j < n and text[j] != c:
                j += 2 if text[j] == "\\" else 1
            out.append(text[i:j + 1])
            i = j + 1
        elif text.startswith("//", i):
            j = text.find("\n", i)
            i = n if j < 0 else j
        elif text.startswith("/*", i):
            j = text.find("*/", i + 2)
            i = n if j < 0 else j + 2
            out.append(" ")
        else:
            out.append(c)
            i += 1
    return " ".join("".join(out).split())


def kernel_source_hash(sources=None):
    """Hash of the library's sources (file name and code without comments);
    sources: {file name: text}, default the files of csrc/."""
    if sources is None:
        d = os.path.join(HERE, "csrc")
        sources = {}
        for f in os.listdir(d):
            with open(os.path.join(d, f), encoding="utf-8") as fh:
                sources[f] = fh.read()
    h = hashlib.sha256()
    for f in sorted(sources):
        h.update(f.encode() + b"\0" + code_only(sources[f]).encode() + b"\0")
    return h.hexdigest()[:16]


def _db_stats(db_path):
    """kernel_stats rows from a rocprofv3 database (its default output)."""
    import sqlite3

    db = sqlite3.connect(db_path)
    rows = db.execute("SELECT name, COUNT(*), SUM(end - start), AVG(end - start) FROM kernels "
                      "GROUP BY name ORDER BY SUM(end - start) DESC").fetchall()
    total = sum(r[2] for r in rows) or 1
    return [{"Name": r[0], "Calls": r[1], "TotalDurationNs": r[2], "AverageNs": r[3], "Percentage": 100.0 * r[2] / total}
            for r in rows]


def stats(csv_path, out_md, command):
    rows = _db_stats(csv_path) if csv_path.endswith(".db") else list(csv.DictReader(open(csv_path)))
    lines = ["# rocprofv3 kernel statistics", "", "Command:", "", "    " + command, "",
             "Durations are of the kernels alone (concurrent kernels overlap in time).", "",
             "| kernel | short name | calls | total ms | avg us | % |", "|---|---|---|---|---|---|"]
    for r in rows[:25]:
        name = r.get("Name") or r.get("KernelName") or r.get("Kernel_Name")
        calls = int(r.get("Calls") or r.get("TotalCalls") or 0)
        tot = float(r.get("TotalDurationNs") or r.get("TotalDuration") or 0)
        avg = float(r.get("AverageNs") or r.get("Average") or 0)
        pct = float(r.get("Percentage") or 0)
        lines.append("| %s | %s | %d | %.3f | %.1f | %.1f |" % (name.split("(")[0][:110], short_name(name) or "-", calls,
                                                               tot / 1e6, avg / 1e3, pct))
    open(out_md, "w").write("\n".join(lines) + "\n")


def _counter_rows(d):
    files = glob.glob(os.path.join(d, "**", "*counter_collection.csv"), recursive=True)
    out = []
    for f in files:
        out.extend(csv.DictReader(open(f)))
    return out


def _per_dispatch(rows):
    """(kernel name, dispatch id) -> counter value in bytes"""
    acc = defaultdict(float)
    for r in rows:
        name = r.get("Kernel_Name") or r.get("Kernel-Name") or r.get("KernelName")
        disp = r.get("Dispatch_Id") or r.get("Dispatch-Id") or r.get("DispatchId")
        acc[(name, disp)] += float(r.get("Counter_Value") or r.get("Counter-Value") or 0) * 1024.0
    return acc


def traffic(fetch_dir, write_dir, copy_mib, out_json, command):
    f = _per_dispatch(_counter_rows(fetch_dir))
    w = _per_dispatch(_counter_rows(write_dir))
    copy_bytes = float(copy_mib) * (1 << 20)
    # the calibration copy: the largest dispatch before the library's first
    # kernel (the bench runs it first; later runtime copies belong to the
    # library's own work)
    def calib(acc):
        lib_ids = [int(d) for (name, d) in acc if "ccg::" in name]
        first = min(lib_ids) if lib_ids else None
        cands = [(v, k) for k, v in acc.items() if "ccg::" not in k[0] and (first is None or int(k[1]) < first)]
        return max(cands)[0] if cands else None
    fc, wc = calib(f), calib(w)
    sf = copy_bytes / fc if fc else 1.0
    sw = copy_bytes / wc if wc else 1.0
    # A radix sort is one library launch of several dispatches (a histogram,
    # scans and a scatter per 8-bit pass): the dispatches from one radix
    # kernel up to the next kernel that is neither a radix nor a scan kernel
    # form one launch, scans included, as the library's profiler times it.
    # Each counter's run is grouped on its own (dispatch ids differ between
    # runs when lanes run concurrently).
    def grouped(acc, scale):
        names = {int(d): name for (name, d) in acc}
        vals = defaultdict(float)
        for (name, d), v in acc.items():
            vals[int(d)] += v
        total, launches = defaultdict(float), defaultdict(int)
        in_sort = False
        for d in sorted(names):
            sn = short_name(names[d])
            if sn == "radix_sort":
                if not in_sort:
                    launches[sn] += 1
                in_sort = True
                total[sn] += vals[d] * scale
            elif sn == "scan" and in_sort:
                total["radix_sort"] += vals[d] * scale
            else:
                in_sort = False
                if sn:
                    launches[sn] += 1
                    total[sn] += vals[d] * scale
        return total, launches

    ft, fl = grouped(f, sf)
    wt, wl = grouped(w, sw)
    per = {k: [ft[k], wt.get(k, 0.0), fl[k], wl.get(k, 0)] for k in ft}
    kernels = {k: {"fetch_bytes_per_launch": round(v[0] / max(v[2], 1)),
                   "write_bytes_per_launch": round(v[1] / max(v[3], 1)),
                   "bytes_per_launch": round(v[0] / max(v[2], 1) + v[1] / max(v[3], 1)), "launches": v[2]}
               for k, v in per.items()}
    out = {"command": command, "source_hash": kernel_source_hash(), "copy_calibration_bytes": copy_bytes,
           "fetch_scale": sf, "write_scale": sw, "kernels": kernels}
    json.dump(out, open(out_json, "w"), indent=1, sort_keys=True)


def window(db_path, bench_json, out_md):
    import sqlite3

    line = [l for l in open(bench_json).read().splitlines() if l.strip().startswith("{")][-1]
    b = json.loads(line)
    db = sqlite3.connect(db_path)
    rows = db.execute("SELECT name, start, end FROM kernels").fetchall()
    out = ["", "Dispatches inside the bench line's timed window (trace clock = CLOCK_MONOTONIC):", "",
           "| line | kernel | dispatches | trace ms, total | launches | mean us per launch (trace) | mean us per launch (bench, HIP events) |",
           "|---|---|---|---|---|---|---|"]
    for label, obj in (("main", b), ("batched_w4", b.get("batched_w4"))):
        if not obj or "timed_window_monotonic_ns" not in obj or "roofline" not in obj:
            continue
        t0, t1 = obj["timed_window_monotonic_ns"]
        k = obj["roofline"]["kernel"]
        d = [e - s0 for name, s0, e in rows if short_name(name) == k and s0 >= t0 and e <= t1]
        # a library launch of a composite (a radix sort: two kernels per
        # pass) spans several dispatches; the bench states its launches
        launches = obj["roofline"].get("launches_in_window", obj["roofline"].get("launches_timed", len(d)))
        mean = sum(d) / launches / 1e3 if launches else float("nan")
        out.append("| %s | %s | %d | %.1f | %d | %.1f | %.1f |" % (label, k, len(d), sum(d) / 1e6, launches, mean,
                                                                  1e3 * obj["roofline"]["avg_launch_ms"]))
    with open(out_md, "a") as fh:
        fh.write("\n".join(out) + "\n")


if __name__ == "__main__":
    if sys.argv[1] == "stats":
        stats(sys.argv[2], sys.argv[3], " ".join(sys.argv[4:]))
    elif sys.argv[1] == "window":
        window(sys.argv[2], sys.argv[3], sys.argv[4])
    elif sys.argv[1] == "traffic":
        traffic(sys.argv[2], sys.argv[3], int(sys.argv[4]), sys.argv[5], " ".join(sys.argv[6:]))
    else:
        raise SystemExit(__doc__)
