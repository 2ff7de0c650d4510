"""Batched and served queries give the same counts as one query at a time.

* cc_count_batch over uneven patterns (trees, cycles, partial 3-trees of
  5-10 vertices) on concurrent lanes equals one cc_count per query, with any
  lane count the tuner may pick, and coloring 0 of a sample equals the oracle.
* colouring waves under a per-table budget leave the counts unchanged; a
  single colouring over the budget fails with CC_ERANGE.
* the server's results for a query are the same alone and in a mix of
  concurrent queries, also when memory pressure forces re-runs.
"""
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


BUDGET = 2_000_000  # DP entries per table and colouring


@pytest.fixture(scope="module")
def env():
    ctx = cc.Context(0, arena_bytes=32 << 30)
    g = W.barabasi_albert(3000, 3, 77)
    G = cc.load_graph(ctx, g.n, g.row_ptr, g.col)
    yield ctx, g, G
    ctx.close()


def fits_budget(ctx, G, budget):
    def fits(p, s):
        D = cc.build_decomposition(p.n, p.edges)
        C = cc.color(ctx, G, p.n, W.colouring_seed(s), 1)
        ctx.set_table_budget(budget)
        try:
            cc.count(ctx, G, C, D)
            return True
        except cc.CcError as e:
            assert e.code == cc.CC_ERANGE
            return False
        finally:
            ctx.set_table_budget(0)
    return fits


def make_queries(ctx, G, n, B, seed0=5):
    sel, _ = W.select_queries(4, n + seed0, fits_budget(ctx, G, BUDGET))
    qs = []
    for p, s in sel[seed0:]:
        D = cc.build_decomposition(p.n, p.edges)
        C = cc.color(ctx, G, p.n, W.colouring_seed(s), B)
        qs.append((p, D, C, s))
    return qs


def test_batch_equals_individual_and_oracle(env):
    ctx, g, G = env
    qs = make_queries(ctx, G, 24, 4)
    ref = [cc.count(ctx, G, C, D) for _, D, C, _ in qs]
    for lanes in (1, 3, 8):
        say("batch lanes", lanes)
        ctx.set_batch_lanes(lanes)
        out = cc.count_batch(ctx, G, [(D, C) for _, D, C, _ in qs])
        for (c, o), (rc, ro) in zip(out, ref):
            assert np.array_equal(c, rc) and np.array_equal(o, ro)
    for p, D, C, s in qs[:6]:
        col = O.color_array(W.colouring_seed(s), 0, g.n, p.n)
        r = O.dp_count(g, p, p.n, col, td=D.export())
        c, o = cc.count(ctx, G, C, D)
        assert int(c[0]) == r["count"] and bool(o[0]) == r["overflow"], p.name


def test_tuner_picks_a_lane_count(env):
    ctx, g, G = env
    qs = make_queries(ctx, G, 8, 2, seed0=40)
    best = cc.tune_batch(ctx, G, [(D, C) for _, D, C, _ in qs])
    assert best in (1, 2, 4, 8)
    out = cc.count_batch(ctx, G, [(D, C) for _, D, C, _ in qs])
    for (c, _), (_, D, C, _) in zip(out, qs):
        assert np.array_equal(c, cc.count(ctx, G, C, D)[0])


def test_waves_under_budget(env):
    ctx, g, G = env
    p = W.cycle(5)
    D = cc.build_decomposition(p.n, p.edges)
    C = cc.color(ctx, G, 5, 99, 8)
    full, _ = cc.count(ctx, G, C, D)
    sizes = ctx.last_table_sizes()
    per_col_max = int(sizes.max()) // 8
    ctx.set_table_budget(max(1, per_col_max * 2))  # forces waves of about two colourings
    try:
        waves, _ = cc.count(ctx, G, C, D)
        assert np.array_equal(full, waves)
        ctx.set_table_budget(max(1, per_col_max // 50))
        with pytest.raises(cc.CcError) as ei:
            cc.count(ctx, G, C, D)
        assert ei.value.code == cc.CC_ERANGE
    finally:
        ctx.set_table_budget(0)


def test_server_alone_vs_mix(env):
    ctx, g, G = env
    qs = make_queries(ctx, G, 20, 4, seed0=60)
    alone = [cc.count(ctx, G, C, D)[0] for _, D, C, _ in qs]
    srv = cc.Server(ctx, G, max_inflight=4)
    tickets = [srv.submit(D, p.n, W.colouring_seed(s), 4) for p, D, _, s in qs]
    for t, ref in zip(tickets, alone):
        st, c, _ = srv.wait(t)
        assert st == 1 and np.array_equal(c, ref)
    stats = srv.stop()
    assert stats["completed"] == 20 and stats["failed"] == 0
    assert 0 < stats["p50_ms"] <= stats["p99_ms"] <= stats["max_ms"]


@pytest.mark.parametrize("tail", [0.5, 2.5])
def test_server_tail_protection(env, tail):
    """With tail protection the server holds admissions while a query runs
    long; every query still completes with the counts of its own run."""
    ctx, g, G = env
    qs = make_queries(ctx, G, 16, 4, seed0=90)
    alone = [cc.count(ctx, G, C, D)[0] for _, D, C, _ in qs]
    srv = cc.Server(ctx, G, max_inflight=4, tail_factor=tail)
    tickets = [srv.submit(D, p.n, W.colouring_seed(s), 4) for p, D, _, s in qs]
    for t, ref in zip(tickets, alone):
        st, c, _ = srv.wait(t)
        assert st == 1 and np.array_equal(c, ref)
    stats = srv.stop()
    assert stats["completed"] == 16 and stats["failed"] == 0


def test_server_under_memory_pressure():
    """A small arena: concurrent queries run out of memory, are re-queued to
    run alone, and still give the counts of the sequential runs."""
    ctx = cc.Context(0, arena_bytes=24 << 20)
    try:
        g = W.barabasi_albert(1500, 3, 78)
        G = cc.load_graph(ctx, g.n, g.row_ptr, g.col)
        qs = []
        for s in W.query_seeds(4, 40)[20:]:
            p = W.random_query(s)
            D = cc.build_decomposition(p.n, p.edges)
            C = cc.color(ctx, G, p.n, W.colouring_seed(s), 4)
            try:
                ref = cc.count(ctx, G, C, D)[0]
            except cc.CcError:
                continue  # does not fit even alone
            qs.append((p, D, s, ref))
        assert len(qs) >= 8
        srv = cc.Server(ctx, G, max_inflight=6)
        tickets = [srv.submit(D, p.n, W.colouring_seed(s), 4) for p, D, s, _ in qs]
        for t, (_, _, _, ref) in zip(tickets, qs):
            st, c, _ = srv.wait(t)
            assert st == 1 and np.array_equal(c, ref)
        stats = srv.stop()
        assert stats["completed"] == len(qs) and stats["failed"] == 0
        say("requeued", stats["requeued"])
    finally:
        ctx.close()
