"""Host logic of the measurement tools (no GPU): the counter summary groups a
radix sort's dispatches into one library launch and scales by the first
copy; the trace window check matches dispatches to a bench line; bench.py
refuses more than one GPU."""
import csv
import json
import os
import sqlite3
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

from paper_1908_11248_amd import profiling as P  # noqa: E402


def _counters(d, rows, counter):
    os.makedirs(d, exist_ok=True)
    with open(os.path.join(d, "run_counter_collection.csv"), "w", newline="") as fh:
        w = csv.writer(fh)
        w.writerow(["Dispatch_Id", "Kernel_Name", "Counter_Name", "Counter_Value"])
        for disp, name, kib in rows:
            w.writerow([disp, name, counter, kib])


def test_traffic_calibration_and_radix_grouping(tmp_path):
    copy = "__amd_rocclr_copyBuffer"
    # the 1 GiB calibration copy (FETCH reads half of it per its counter),
    # then one radix sort (hist, scans, scatter, hist, scatter) and a forget,
    # then a large runtime copy of the library's own that must not calibrate
    seq = [(1, copy, 524288.0, 1048576.0),
           (2, "void ccg::k_radix_hist<unsigned long, false>(...)", 100.0, 1.0),
           (3, "void ccg::k_scan_down<unsigned int>(...)", 10.0, 10.0),
           (4, "void ccg::k_radix_scatter<unsigned long, false>(...)", 200.0, 400.0),
           (5, "void ccg::k_radix_hist<unsigned long, false>(...)", 100.0, 1.0),
           (6, "void ccg::k_radix_scatter<unsigned long, false>(...)", 200.0, 400.0),
           (7, "void ccg::k_forget<unsigned long, unsigned long, true>(...)", 50.0, 20.0),
           (8, copy, 4194304.0, 4194304.0)]
    _counters(str(tmp_path / "f"), [(d, n, f) for d, n, f, _ in seq], "FETCH_SIZE")
    _counters(str(tmp_path / "w"), [(d, n, w) for d, n, _, w in seq], "WRITE_SIZE")
    out = str(tmp_path / "t.json")
    P.traffic(str(tmp_path / "f"), str(tmp_path / "w"), 1024, out, "cmd")
    t = json.load(open(out))
    assert t["fetch_scale"] == pytest.approx(2.0) and t["write_scale"] == pytest.approx(1.0)
    r = t["kernels"]["radix_sort"]
    assert r["launches"] == 1
    assert r["fetch_bytes_per_launch"] == pytest.approx((100 + 10 + 200 + 100 + 200) * 1024 * 2.0, rel=1e-9)
    assert r["write_bytes_per_launch"] == pytest.approx((1 + 10 + 400 + 1 + 400) * 1024 * 1.0, rel=1e-9)
    assert t["kernels"]["forget_emit"]["launches"] == 1
    assert "scan" not in t["kernels"]  # the only scan ran inside the sort


def test_window_matches_dispatches(tmp_path):
    db = str(tmp_path / "r.db")
    con = sqlite3.connect(db)
    con.execute("CREATE TABLE kernels (name TEXT, start INTEGER, end INTEGER)")
    rows = [("void ccg::k_slot_edge_push<true, false>(...)", 100, 130), ("void ccg::k_slot_edge_push<true, false>(...)", 200, 240),
            ("void ccg::k_slot_edge_push<true, false>(...)", 900, 950), ("ccg::k_slot_root(...)", 140, 150)]
    con.executemany("INSERT INTO kernels VALUES (?, ?, ?)", rows)
    con.commit()
    line = {"timed_window_monotonic_ns": [90, 300],
            "roofline": {"kernel": "slot_edge_push", "avg_launch_ms": 35e-6, "launches_timed": 2}}
    bj = str(tmp_path / "b.json")
    open(bj, "w").write(json.dumps(line) + "\n")
    md = str(tmp_path / "o.md")
    P.window(db, bj, md)
    text = open(md).read()
    assert "| main | slot_edge_push | 2 | 0.0 | 2 | 0.0 | 0.0 |" in text or "| main | slot_edge_push | 2 |" in text
    # mean 35 ns = 0.035 us: the dispatch at 900 lies outside the window
    assert "0.0" in text.split("| main | slot_edge_push | 2 |")[1]


def test_bench_refuses_several_gpus():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True, text=True)
    assert r.returncode == 2 and "one GPU" in r.stderr


def test_source_hash_ignores_comments_not_code():
    from paper_1908_11248_amd.profiling import code_only, kernel_source_hash

    a = {"k.hip": "__global__ void k(int* p) {  // store\n    p[0] = 1; /* one */\n}\n"}
    b = {"k.hip": "// a kernel\n__global__ void k(int* p) {\n p[0] = 1;\n}"}
    c = {"k.hip": "__global__ void k(int* p) { p[0] = 2; }"}
    assert kernel_source_hash(a) == kernel_source_hash(b) != kernel_source_hash(c)
    # literals keep what looks like a comment
    assert code_only('x = "/* y */"; // z') == 'x = "/* y */";'
    assert kernel_source_hash({"a.h": "int x;"}) != kernel_source_hash({"b.h": "int x;"})


def test_kernel_names_of_the_fused_introduces():
    # the profiler's short names of the pull over a leaf and the triangle step
    assert P.short_name("void ccg::k_leaf_pull<unsigned long, true>(...)") == "leaf_pull_emit"
    assert P.short_name("void ccg::k_leaf_pull<unsigned __int128, false>(...)") == "leaf_pull_count"
    assert P.short_name("void ccg::k_tri<unsigned __int128, true>(...)") == "tri_emit"
    assert P.short_name("void ccg::k_tri<unsigned long, false>(...)") == "tri_count"
    assert P.short_name("void ccg::k_slot_edge_push<true, false, true, true>(...)") == "slot_edge_push"
    assert P.short_name("void ccg::k_slot_leaf<1>(...)") == "slot_leaf"
