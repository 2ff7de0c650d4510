"""GPU parity of the dense one-column tables (tree patterns) and of the
sorted-list tables forced with CC_SPARSE_TABLES, against the oracle: counts,
overflow flags, per-vertex counts and the per-node table sizes |D_x| (summed
over colourings) must be identical, bit for bit, on both paths.

Batches of 9 colourings cover the XCD-interleaved block mapping with a
ragged last group; k = 12 with 7-vertex trees gives 462 slots per vertex,
more than one block's threads.  Trees with k <= 10 run the edge steps in
the push form where no count can wrap and in the gather form otherwise;
a graph with a hub covers their 64-bit variants.
"""
import sys

import numpy as np
import pytest

import oracle as O
import paper_1908_11248_amd as cc
from paper_1908_11248_amd import workloads as W

pytestmark = pytest.mark.gpu

SPARSE = cc.CC_SPARSE_TABLES


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def ctx():
    c = cc.Context(0, arena_bytes=16 << 30)
    yield c
    c.close()


GRAPHS = [("er40", lambda: W.er_pairs(40, 0.2, 4)), ("rgg300", lambda: W.rgg(300, 8, 6)),
          ("ba400", lambda: W.barabasi_albert(400, 3, 7))]
TREES = [W.Pattern(1, [], "K1"), W.path(2), W.path(4), W.star(5), W.random_tree(7, 1), W.pattern_A(),
         W.random_tree(8, 11)]


def run(ctx, G, C, D, flags):
    counts, ovf = cc.count(ctx, G, C, D, flags)
    return counts, ovf, ctx.last_table_sizes()


@pytest.mark.parametrize("gname,make", GRAPHS, ids=[x[0] for x in GRAPHS])
def test_trees_dense_and_sparse_match_oracle(ctx, gname, make):
    g = make()
    G = cc.load_graph(ctx, g.n, g.row_ptr, g.col)
    rng = np.random.default_rng(len(gname) + 100)
    for pat in TREES:
        for k in sorted({pat.n, min(pat.n + 2, 12), 12}):
            B = 9
            colors = rng.integers(0, k, size=(B, g.n)).astype(np.uint8)
            say("slots", gname, pat.name, "k", k)
            D = cc.build_decomposition(pat.n, pat.edges)
            td = D.export()
            C = cc.color_explicit(ctx, G, k, colors)
            cd, od, sd = run(ctx, G, C, D, 0)
            cs, os_, ss = run(ctx, G, C, D, SPARSE)
            ref_sizes = np.zeros(len(sd), dtype=np.int64)
            for b in range(B):
                ref = O.dp_count(g, pat, k, colors[b], td=td, sizes=True)
                assert int(cd[b]) == ref["count"], (gname, pat.name, k, b)
                assert bool(od[b]) == ref["overflow"]
                ref_sizes += ref["sizes"]
            assert np.array_equal(cd, cs) and np.array_equal(od, os_)
            assert np.array_equal(sd, ref_sizes), (gname, pat.name, k)
            assert np.array_equal(ss, ref_sizes), (gname, pat.name, k)
            C.close()


def hub_graph(n=2500, m=3000, seed=5):
    # vertex 0 adjacent to every other vertex, plus random edges: a degree
    # bound of 2499^(s-1) puts 4-vertex subtrees past 2^32, so the push form
    # of the edge step runs with 64-bit accumulators and the gather reads
    # both count planes
    rng = np.random.default_rng(seed)
    a, b = rng.integers(1, n, m), rng.integers(1, n, m)
    keep = a != b
    src = np.concatenate([np.zeros(n - 1, dtype=np.int64), a[keep]])
    dst = np.concatenate([np.arange(1, n), b[keep]])
    return W.csr_from_edges(n, src, dst)


@pytest.mark.parametrize("k", [8, 10])
@pytest.mark.parametrize("pat", [W.path(5), W.random_tree(6, 3), W.random_tree(7, 5)], ids=lambda p: p.name)
def test_hub_graph_dense_and_sparse_match_oracle(ctx, pat, k):
    g = hub_graph()
    G = cc.load_graph(ctx, g.n, g.row_ptr, g.col)
    rng = np.random.default_rng(pat.n + k)
    B = 5
    colors = rng.integers(0, k, size=(B, g.n)).astype(np.uint8)
    say("hub", pat.name, "k", k)
    D = cc.build_decomposition(pat.n, pat.edges)
    C = cc.color_explicit(ctx, G, k, colors)
    cd, od, sd = run(ctx, G, C, D, 0)
    cs, os_, ss = run(ctx, G, C, D, SPARSE)
    ref_sizes = np.zeros(len(sd), dtype=np.int64)
    for b in range(B):
        ref = O.dp_count(g, pat, k, colors[b], td=D.export(), sizes=True)
        assert int(cd[b]) == ref["count"] and bool(od[b]) == ref["overflow"], (pat.name, b)
        ref_sizes += ref["sizes"]
    assert np.array_equal(cd, cs) and np.array_equal(od, os_)
    assert np.array_equal(sd, ref_sizes) and np.array_equal(ss, ref_sizes)
    C.close()


@pytest.mark.parametrize("pat", [W.star(4), W.path(4)], ids=lambda p: p.name)
def test_degree_past_16_bits_matches_oracle(ctx, pat):
    # a hub of degree 65 599: the leaf steps and the fused leaf join count
    # neighbourhoods past 2^16, and the block holding the hub splits its
    # neighbour list over all of its threads
    n = 65600
    rng = np.random.default_rng(9)
    a, b = rng.integers(1, n, 2000), rng.integers(1, n, 2000)
    keep = a != b
    g = W.csr_from_edges(n, np.concatenate([np.zeros(n - 1, dtype=np.int64), a[keep]]),
                         np.concatenate([np.arange(1, n), b[keep]]))
    G = cc.load_graph(ctx, g.n, g.row_ptr, g.col)
    B, k = 2, 5
    colors = rng.integers(0, k, size=(B, g.n)).astype(np.uint8)
    say("hub 2^16", pat.name)
    D = cc.build_decomposition(pat.n, pat.edges)
    C = cc.color_explicit(ctx, G, k, colors)
    cd, od, sd = run(ctx, G, C, D, 0)
    ref_sizes = np.zeros(len(sd), dtype=np.int64)
    for bb in range(B):
        ref = O.dp_count(g, pat, k, colors[bb], td=D.export(), sizes=True)
        assert int(cd[bb]) == ref["count"] and bool(od[bb]) == ref["overflow"], (pat.name, bb)
        ref_sizes += ref["sizes"]
    assert np.array_equal(sd, ref_sizes)
    C.close()


# joins at a vertex computed in the push kernel of its deeper child's edge
# step (k <= 10, no count can wrap, the kernel's LDS fits): with the fused join of two leaf children
# ("LJ+"), or with one leaf and then another ("chain"); vertex orders decide
# which children the plan joins first.  On the hub graph the chain of a
# 4-vertex child runs with 64-bit accumulators.
PUSH_JOIN = [W.Pattern(5, [(0, 1), (0, 2), (0, 3), (3, 4)], "LJ+P2"),
             W.Pattern(6, [(0, 3), (3, 4), (4, 5), (0, 1), (0, 2)], "LJ+P3"),
             W.Pattern(7, [(0, 1), (1, 2), (1, 3), (1, 4), (4, 5), (0, 6)], "LJ+P2+chain1"),
             W.Pattern(5, [(0, 1), (1, 2), (0, 3), (0, 4)], "chain2-P3"),
             W.Pattern(6, [(0, 1), (1, 2), (2, 3), (0, 4), (0, 5)], "chain2-P4"),
             W.workload_pattern(2)]


@pytest.mark.parametrize("gname", ["er40", "rgg300", "ba400", "hub"])
def test_push_join_matches_oracle(ctx, gname):
    g = hub_graph() if gname == "hub" else dict(GRAPHS)[gname]()
    G = cc.load_graph(ctx, g.n, g.row_ptr, g.col)
    rng = np.random.default_rng(len(gname) + 7)
    for pat in PUSH_JOIN:
        # k = 10: some chains no longer fit a block's LDS and run unfused
        for k in sorted({pat.n, min(pat.n + 2, 10), 10}):
            B = 9 if gname != "hub" else 3
            colors = rng.integers(0, k, size=(B, g.n)).astype(np.uint8)
            say("push join", gname, pat.name, "k", k)
            D = cc.build_decomposition(pat.n, pat.edges)
            td = D.export()
            C = cc.color_explicit(ctx, G, k, colors)
            cd, od, sd = run(ctx, G, C, D, 0)
            ref_sizes = np.zeros(len(sd), dtype=np.int64)
            for b in range(B):
                ref = O.dp_count(g, pat, k, colors[b], td=td, sizes=True)
                assert int(cd[b]) == ref["count"] and bool(od[b]) == ref["overflow"], (gname, pat.name, k, b)
                ref_sizes += ref["sizes"]
            assert np.array_equal(sd, ref_sizes), (gname, pat.name, k)
            C.close()


def test_random_tree_sweep_matches_oracle(ctx):
    # 40 seeded random trees of 3-9 vertices at k from n_F to 10 on a graph
    # mixing a dense core with sparse periphery: many plan shapes, so the
    # push form, its joins (leaf joins, chains of one or two leaves) and
    # their fallbacks all meet the oracle's counts and node sizes, and the
    # sorted-list path agrees
    rng = np.random.default_rng(2024)
    n = 700
    a, b = rng.integers(0, n, 2600), rng.integers(0, n, 2600)
    core = rng.integers(0, 60, (2, 900))
    keep = a != b
    ck = core[0] != core[1]
    g = W.csr_from_edges(n, np.concatenate([a[keep], core[0][ck]]), np.concatenate([b[keep], core[1][ck]]))
    G = cc.load_graph(ctx, g.n, g.row_ptr, g.col)
    for t in range(40):
        nf = int(rng.integers(3, 10))
        pat = W.random_tree(nf, 1000 + t)
        k = int(rng.integers(nf, 11))
        B = 3
        colors = rng.integers(0, k, size=(B, g.n)).astype(np.uint8)
        say("sweep", t, pat.name, pat.edges, "k", k)
        D = cc.build_decomposition(pat.n, pat.edges)
        td = D.export()
        C = cc.color_explicit(ctx, G, k, colors)
        cd, od, sd = run(ctx, G, C, D, 0)
        cs, os_, ss = run(ctx, G, C, D, SPARSE)
        ref_sizes = np.zeros(len(sd), dtype=np.int64)
        for bb in range(B):
            ref = O.dp_count(g, pat, k, colors[bb], td=td, sizes=True)
            assert int(cd[bb]) == ref["count"] and bool(od[bb]) == ref["overflow"], (t, pat.edges, k, bb)
            ref_sizes += ref["sizes"]
        assert np.array_equal(sd, ref_sizes), (t, pat.edges, k)
        assert np.array_equal(cd, cs) and np.array_equal(od, os_) and np.array_equal(ss, ref_sizes), (t, k)
        C.close()


def test_overflow_on_both_paths(ctx):
    # a hub of degree 6000: the star S7 overflows 64 bits
    n = 6001
    g = W.csr_from_edges(n, np.zeros(n - 1, dtype=np.int64), np.arange(1, n))
    G = cc.load_graph(ctx, g.n, g.row_ptr, g.col)
    pat = W.star(7)
    colors = np.stack([(np.arange(n) % 7), (np.arange(n) * 3 % 7)]).astype(np.uint8)
    D = cc.build_decomposition(pat.n, pat.edges)
    C = cc.color_explicit(ctx, G, 7, colors)
    for flags in (0, SPARSE):
        counts, ovf = cc.count(ctx, G, C, D, flags)
        for b in range(2):
            ref = O.dp_count(g, pat, 7, colors[b], td=D.export())
            assert int(counts[b]) == ref["count"] and bool(ovf[b]) == ref["overflow"], (flags, b)
        assert ovf.all()


def test_per_vertex_on_both_paths(ctx):
    g = W.barabasi_albert(500, 3, 9)
    G = cc.load_graph(ctx, g.n, g.row_ptr, g.col)
    pat = W.random_tree(6, 4)
    C = cc.color(ctx, G, 6, 77, 3)
    D = cc.build_decomposition(pat.n, pat.edges)
    col = O.color_array(77, 2, g.n, 6)
    ref = O.dp_count(g, pat, 6, col, td=D.export(), per_root_vertex=True)
    for flags in (0, SPARSE):
        pv, total, ovf = cc.count_by_vertex(ctx, G, C, 2, D, flags)
        assert total == ref["count"] and not ovf
        assert np.array_equal(pv.astype(np.uint64), ref["per_root_vertex"]), flags


def test_degree_mask_off_on_both_paths(ctx):
    g = W.er_pairs(200, 0.04, 12)
    G = cc.load_graph(ctx, g.n, g.row_ptr, g.col)
    pat = W.random_tree(7, 8)
    C = cc.color(ctx, G, 7, 5, 4)
    D = cc.build_decomposition(pat.n, pat.edges)
    a, _ = cc.count(ctx, G, C, D, 0)
    sa = ctx.last_table_sizes()
    b, _ = cc.count(ctx, G, C, D, cc.CC_NO_DEGREE_MASK)
    sb = ctx.last_table_sizes()
    c, _ = cc.count(ctx, G, C, D, cc.CC_NO_DEGREE_MASK | SPARSE)
    sc = ctx.last_table_sizes()
    assert np.array_equal(a, b) and np.array_equal(b, c)
    assert np.array_equal(sb, sc) and (sb >= sa).all()


def test_budget_waves_on_both_paths(ctx):
    # a per-table budget that holds one colouring but not the batch: waves,
    # same counts; a budget below one colouring's table: CC_ERANGE on both
    g = W.er_pairs(400, 0.03, 2)
    G = cc.load_graph(ctx, g.n, g.row_ptr, g.col)
    pat = W.path(5)
    C = cc.color(ctx, G, 5, 3, 8)
    D = cc.build_decomposition(pat.n, pat.edges)
    full, _ = cc.count(ctx, G, C, D, SPARSE)
    sizes = ctx.last_table_sizes()
    per_col = int(sizes.max()) // 8
    try:
        for flags in (0, SPARSE):
            ctx.set_table_budget(3 * per_col)
            got, _ = cc.count(ctx, G, C, D, flags)
            assert np.array_equal(got, full), flags
            ctx.set_table_budget(1)
            with pytest.raises(cc.CcError) as e:
                cc.count(ctx, G, C, D, flags)
            assert e.value.code == cc.CC_ERANGE
    finally:
        ctx.set_table_budget(0)


def test_workload2_dense_matches_sparse(ctx):
    w = W.workload(2)
    g = W.workload_graph(2)
    pat = W.workload_pattern(2)
    G = cc.load_graph(ctx, g.n, g.row_ptr, g.col)
    C = cc.color(ctx, G, w.k, w.color_seed, w.colorings)
    D = cc.build_decomposition(pat.n, pat.edges)
    say("workload 2 dense")
    a, oa = cc.count(ctx, G, C, D, 0)
    sa = ctx.last_table_sizes()
    say("workload 2 sparse")
    b, ob = cc.count(ctx, G, C, D, SPARSE)
    sb = ctx.last_table_sizes()
    assert np.array_equal(a, b) and np.array_equal(oa, ob) and np.array_equal(sa, sb)
    col = O.color_array(w.color_seed, 33, g.n, w.k)
    ref = O.dp_count(g, pat, w.k, col, td=D.export())
    assert int(a[33]) == ref["count"]
