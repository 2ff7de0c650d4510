"""Anchor-range chunks on the GPU against the oracle.

cc_count_range counts the mappings with Phi(0) in [lo, hi); the oracle's
dp_count_range is pinned (tests/test_oracle_count.py) against the brute force
with Phi(0) fixed and against the full count over partitions.  A per-table
budget small enough to force the executor to split one colouring into
anchor ranges must leave counts, overflow flags and every node's |D_x|
equal to the oracle's unsplit run.
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


@pytest.fixture(scope="module")
def ctx():
    c = cc.Context(0, arena_bytes=8 << 30)
    yield c
    c.close()


PATS = [W.cycle(5), W.cycle(6), W.pattern_B(), W.partial_3tree(7, 3), W.ladder(3), W.random_tree(7, 2)]


@pytest.mark.parametrize("pat", PATS, ids=lambda p: p.name)
def test_ranges_match_oracle_and_add_up(ctx, pat):
    g = W.er_pairs(300, 0.04, 41)
    G = cc.load_graph(ctx, g.n, g.row_ptr, g.col)
    D = cc.build_decomposition(pat.n, pat.edges)
    td = D.export()
    B = 3
    C = cc.color(ctx, G, pat.n, 77, B)
    full, full_ovf = cc.count(ctx, G, C, D)
    cuts = [0, 1, 57, 58, 150, 299, 300]
    acc = np.zeros(B, dtype=np.uint64)
    for lo, hi in zip(cuts[:-1], cuts[1:]):
        say("range", pat.name, lo, hi)
        got, _ = cc.count_range(ctx, G, C, D, lo, hi)
        sizes = ctx.last_table_sizes()
        ref_sizes = 0
        for b in range(B):
            col = O.color_array(77, b, g.n, pat.n)
            r = O.dp_count_range(g, pat, pat.n, col, lo, hi, td=td, sizes=True)
            assert int(got[b]) == r["count"], (pat.name, lo, hi, b)
            ref_sizes = ref_sizes + r["sizes"]
        assert np.array_equal(sizes, ref_sizes), (pat.name, lo, hi)
        acc += got
    assert np.array_equal(acc, full)
    empty, _ = cc.count_range(ctx, G, C, D, 10, 10)
    assert not empty.any()


@pytest.mark.parametrize("pat", PATS[:4], ids=lambda p: p.name)
def test_budget_forces_anchor_chunks(ctx, pat):
    g = W.er_skip(4000, 7.0 / 3999, 42)
    G = cc.load_graph(ctx, g.n, g.row_ptr, g.col)
    D = cc.build_decomposition(pat.n, pat.edges)
    td = D.export()
    for B in (1, 4):
        C = cc.color(ctx, G, pat.n, 5, B)
        ref = [O.dp_count(g, pat, pat.n, O.color_array(5, b, g.n, pat.n), td=td, sizes=True) for b in range(B)]
        # tables of nodes whose bag holds vertex 0 split over anchor ranges,
        # the others do not: a budget above the others and below a fifth of
        # the largest anchored table forces several ranges per colouring
        anchored = np.array([(int(td[5 + 5 * i]) & 1) == 1 for i in range(int(td[0]))])
        anchored[-1] = False  # the root
        big_a = max(int(r["sizes"][anchored].max()) for r in ref)
        big_o = max(int(r["sizes"][~anchored][:-1].max()) if (~anchored)[:-1].any() else 0 for r in ref)
        budget = max(big_o + 1, big_a // 5)
        if budget >= big_a:
            pytest.skip("tables without vertex 0 are as large as the anchored ones")
        ctx.set_table_budget(budget)
        try:
            say("chunks", pat.name, "B", B, "budget", budget)
            got, ovf = cc.count(ctx, G, C, D)
            chunks = ctx.last_chunk_count()
            sizes = ctx.last_table_sizes()
        finally:
            ctx.set_table_budget(0)
        assert chunks > B, (pat.name, B, chunks)
        for b in range(B):
            assert int(got[b]) == ref[b]["count"] and bool(ovf[b]) == ref[b]["overflow"], (pat.name, B, b)
        assert np.array_equal(sizes, sum(r["sizes"] for r in ref)), (pat.name, B)


def test_chunk_carry_sets_overflow(ctx):
    """Stars S8 around 8 hubs spread over the id range: each half of the
    range counts below 2^64 (exact, no flag) but the two halves add up to
    more, so a run split into anchor ranges must raise the flag from the
    carry of the final sum; the count is the true value mod 2^64."""
    k = 8
    per_colour = 135  # 7! * 135^7 per hub: four hubs stay below 2^64, eight do not
    n = 8 + 8 * per_colour
    hubs = np.arange(8) * (n // 8)
    leaves = np.setdiff1d(np.arange(n), hubs)
    a = np.repeat(hubs, leaves.size)
    b = np.tile(leaves, hubs.size)
    g = W.csr_from_edges(n, a, b)
    col = np.zeros(n, dtype=np.uint8)
    col[hubs] = np.arange(8)
    col[leaves] = np.arange(leaves.size) % k
    pat = W.star(k)
    ref = O.dp_count(g, pat, k, col)
    lo_half = O.dp_count_range(g, pat, k, col, 0, n // 2)
    hi_half = O.dp_count_range(g, pat, k, col, n // 2, n)
    assert not lo_half["overflow"] and not hi_half["overflow"]
    assert lo_half["count"] + hi_half["count"] >= 2**64
    assert ref["overflow"] and ref["count"] == (lo_half["count"] + hi_half["count"]) % 2**64
    G = cc.load_graph(ctx, g.n, g.row_ptr, g.col)
    C = cc.color_explicit(ctx, G, k, col)
    D = cc.build_decomposition(pat.n, pat.edges)
    got, ovf = cc.count(ctx, G, C, D, cc.CC_SPARSE_TABLES)
    assert int(got[0]) == ref["count"] and bool(ovf[0])
    part, part_ovf = cc.count_range(ctx, G, C, D, 0, n // 2, cc.CC_SPARSE_TABLES)
    assert int(part[0]) == lo_half["count"] and not bool(part_ovf[0])
    ctx.set_table_budget(int(ctx.last_table_sizes()[:-1].max()) // 3)
    try:
        got2, ovf2 = cc.count(ctx, G, C, D, cc.CC_SPARSE_TABLES)
        chunks = ctx.last_chunk_count()
    finally:
        ctx.set_table_budget(0)
    assert chunks > 1 and int(got2[0]) == ref["count"] and bool(ovf2[0])
