"""Schedules and the autotuner: every schedule (lanes, introduce form
threshold, dense LDS accumulators against sorting in forget and join) gives
the oracle's counts; the tuner keeps one of the schedules it tried."""
import sys

import numpy as np
import pytest

import oracle as O
import paper_1908_11248_amd as cc
from paper_1908_11248_amd import workloads as W

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def test_schedules_agree_with_oracle_and_tuner_picks_one():
    g = W.barabasi_albert(2000, 3, 61)
    pats = [W.cycle(5), W.partial_3tree(7, 4), W.ladder(3), W.random_tree(7, 8), W.pattern_B(), W.complete(4)]
    with cc.Context(0, arena_bytes=8 << 30) as ctx:
        G = cc.load_graph(ctx, g.n, g.row_ptr, g.col)
        decs = [cc.build_decomposition(p.n, p.edges) for p in pats]
        cols = [cc.color(ctx, G, p.n, 40 + i, 2) for i, p in enumerate(pats)]
        ref = [[O.dp_count(g, p, p.n, O.color_array(40 + i, b, g.n, p.n))["count"] for b in range(2)]
               for i, p in enumerate(pats)]
        for sched in ({"lanes": 1, "entry_factor": 1, "sort_above_k": 12, "group_min": 1},
                      {"lanes": 4, "entry_factor": 8, "sort_above_k": 0, "group_min": 0},
                      {"lanes": 2, "entry_factor": 3, "sort_above_k": 6, "group_min": 2}):
            say("schedule", sched)
            ctx.set_schedule(**sched)
            assert ctx.schedule() == sched
            out = cc.count_batch(ctx, G, list(zip(decs, cols)))
            for i, (c, _) in enumerate(out):
                assert [int(x) for x in c] == ref[i], (sched, pats[i].name)
        ctx.set_schedule()
        best = cc.tune_batch(ctx, G, list(zip(decs, cols)))
        s = ctx.schedule()
        assert best == s["lanes"] and s["lanes"] in (1, 2, 4, 8)
        assert s["entry_factor"] in (1, 3, 8) and s["sort_above_k"] in (12, 8, 0) and s["group_min"] in (2, 0, 4)
        out = cc.count_batch(ctx, G, list(zip(decs, cols)))
        for i, (c, _) in enumerate(out):
            assert [int(x) for x in c] == ref[i], pats[i].name


def test_enumeration_under_a_sorting_schedule():
    # enumeration records contributors, which only the dense forget and join
    # produce: a schedule that sorts elsewhere leaves it unchanged
    g = W.er_pairs(80, 0.12, 5)
    pat = W.cycle(5)
    with cc.Context(0, arena_bytes=1 << 30) as ctx:
        ctx.set_schedule(lanes=1, entry_factor=3, sort_above_k=0)
        G = cc.load_graph(ctx, g.n, g.row_ptr, g.col)
        D = cc.build_decomposition(pat.n, pat.edges)
        C = cc.color(ctx, G, pat.n, 3, 1)
        sets, nmap = cc.vertex_sets(ctx, G, C, 0, D, 10**6)
        col = O.color_array(3, 0, g.n, pat.n)
        assert nmap == O.dp_count(g, pat, pat.n, col)["count"]
        assert [tuple(r) for r in sets] == O.vertex_sets(g, pat, pat.n, col)
