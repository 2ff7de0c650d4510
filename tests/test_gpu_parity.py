"""GPU parity: counts from the HIP path (through the C ABI) against the oracle.

The bar is bit-exactness: uint64 counts (mod 2^64) and overflow flags equal
to the oracle's on the same inputs and, for flags, the same decomposition.
Sizes: tiny zoo cases (several tiles, ragged tails, edge cases) checked in
full; the standard workloads at full size checked on sampled colourings and
sampled per-vertex counts the oracle computes one by one.
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
    c = cc.Context(0, arena_bytes=48 << 30)
    yield c
    c.close()


def gpu_graph(ctx, g):
    return cc.load_graph(ctx, g.n, g.row_ptr, g.col)


def run_gpu(ctx, g, pat, k, colors, td=None, flags=0):
    G = gpu_graph(ctx, g)
    C = cc.color_explicit(ctx, G, k, colors)
    D = cc.decomp_import(pat.n, pat.edges, td) if td is not None else cc.build_decomposition(pat.n, pat.edges)
    counts, ovf = cc.count(ctx, G, C, D, flags)
    return counts, ovf, D


ZOO_G = [("er12", lambda: W.er_pairs(12, 0.4, 3)), ("er40", lambda: W.er_pairs(40, 0.2, 4)),
         ("er120", lambda: W.er_pairs(120, 0.08, 5)), ("rgg300", lambda: W.rgg(300, 8, 6)),
         ("ba400", lambda: W.barabasi_albert(400, 3, 7))]
ZOO_P = [W.path(2), W.path(4), W.cycle(3), W.cycle(5), W.star(5), W.grid(2, 3), W.ladder(3), W.complete(4),
         W.pattern_A(), W.pattern_B(), W.pattern_D(), W.random_tree(7, 1), W.partial_3tree(7, 2),
         W.Pattern(1, [], "K1")]


@pytest.mark.parametrize("gname,make", ZOO_G, ids=[x[0] for x in ZOO_G])
def test_zoo_counts_match_oracle(ctx, gname, make):
    g = make()
    rng = np.random.default_rng(len(gname))
    for pat in ZOO_P:
        for k in sorted({pat.n, min(pat.n + 2, 12)}):
            B = 3
            colors = rng.integers(0, k, size=(B, g.n)).astype(np.uint8)
            say("zoo", gname, pat.name, "k", k)
            D = cc.build_decomposition(pat.n, pat.edges)
            td = D.export()
            counts, ovf, _ = run_gpu(ctx, g, pat, k, colors, td=td)
            sizes = ctx.last_table_sizes()
            ref_sizes = 0
            for b in range(B):
                ref = O.dp_count(g, pat, k, colors[b], td=td, sizes=True)
                assert int(counts[b]) == ref["count"], (gname, pat.name, k, b)
                assert bool(ovf[b]) == ref["overflow"]
                ref_sizes = ref_sizes + ref["sizes"]
            # |D_x| of every node, summed over the colourings
            assert np.array_equal(sizes, ref_sizes), (gname, pat.name, k)


def test_oracle_td_imported_gives_same_counts(ctx):
    g = W.er_pairs(150, 0.07, 9)
    rng = np.random.default_rng(1)
    for pat in [W.cycle(6), W.pattern_B(), W.pattern_C(), W.ladder(4), W.random_tree(8, 5)]:
        colors = rng.integers(0, pat.n, size=(2, g.n)).astype(np.uint8)
        td, _ = O.build_td(pat)
        say("oracle-td", pat.name)
        c1, _, _ = run_gpu(ctx, g, pat, pat.n, colors, td=td)
        c2, _, _ = run_gpu(ctx, g, pat, pat.n, colors)
        for b in range(2):
            assert int(c1[b]) == int(c2[b]) == O.dp_count(g, pat, pat.n, colors[b])["count"]


def test_degree_mask_off_same_counts(ctx):
    g = W.barabasi_albert(300, 2, 3)
    rng = np.random.default_rng(2)
    pat = W.star(5)
    colors = rng.integers(0, 5, size=(2, g.n)).astype(np.uint8)
    c1, _, _ = run_gpu(ctx, g, pat, 5, colors)
    c2, _, _ = run_gpu(ctx, g, pat, 5, colors, flags=cc.CC_NO_DEGREE_MASK)
    assert np.array_equal(c1, c2)


def test_overflow_flag_and_wraparound(ctx):
    n = 6001
    g = W.csr_from_edges(n, np.zeros(n - 1, dtype=np.int64), np.arange(1, n))
    pat = W.star(7)
    colors = (np.arange(n) % 7).astype(np.uint8)[None, :]
    D = cc.build_decomposition(pat.n, pat.edges)
    counts, ovf, _ = run_gpu(ctx, g, pat, 7, colors, td=D.export())
    ref = O.dp_count(g, pat, 7, colors[0], td=D.export())
    assert int(counts[0]) == ref["count"] and bool(ovf[0]) and ref["overflow"]


def test_wrapping_push_matches_oracle(ctx):
    # Paths of 10 vertices on K(200, 200) and on K(400): the count bound of
    # the late edge steps of the dense plan passes 2^64, so they run the push
    # form that tracks wraps (no gather launch).  On K(400) single slots pass
    # 2^64 as well (about (400/10)^9 9! colourful paths leave a vertex with a
    # given colour set), so sums wrap inside the push.
    pat = W.path(10)
    a = 200
    bip = W.csr_from_edges(2 * a, np.repeat(np.arange(a), a).astype(np.int64),
                           (a + np.tile(np.arange(a), a)).astype(np.int64))
    iu = np.triu_indices(400, 1)
    kn = W.csr_from_edges(400, iu[0].astype(np.int64), iu[1].astype(np.int64))
    for name, g in (("K200,200", bip), ("K400", kn)):
        col = np.random.default_rng(g.n).integers(0, 10, size=(1, g.n)).astype(np.uint8)
        ctx.profile_enable(True)
        counts, ovf, D = run_gpu(ctx, g, pat, 10, col)
        sizes = ctx.last_table_sizes()
        prof = ctx.profile_read()
        ctx.profile_enable(False)
        assert "slot_edge_push" in prof and "slot_edge" not in prof, (name, sorted(prof))
        ref = O.dp_count(g, pat, 10, col[0], td=D.export(), sizes=True)
        assert int(counts[0]) == ref["count"] and bool(ovf[0]) == ref["overflow"], name
        assert ref["overflow"], name
        assert np.array_equal(sizes, ref["sizes"]), name


def test_pull_over_a_leaf_matches_oracle(ctx):
    # K4, C5 and a partial 3-tree start by introducing a vertex next to a leaf
    # in pull form with no edge test: those entries come straight from the
    # edges (the leaf's table is never built); in K4 the next vertex closes a
    # triangle with them, whose entries come from the edges' common-neighbour
    # lists.  Counts and every node's size against the oracle, on a graph
    # with hubs and on one without.
    for g in (W.barabasi_albert(400, 3, 7), W.er_pairs(120, 0.08, 5)):
        for pat in (W.complete(4), W.cycle(5), W.partial_3tree(7, 2)):
            colors = np.random.default_rng(pat.n).integers(0, pat.n, size=(2, g.n)).astype(np.uint8)
            ctx.profile_enable(True)
            counts, ovf, D = run_gpu(ctx, g, pat, pat.n, colors)
            sizes = ctx.last_table_sizes()
            prof = ctx.profile_read()
            ctx.profile_enable(False)
            assert "leaf_pull_emit" in prof or "leaf_pull_count" in prof, (pat.name, sorted(prof))
            if pat.name == "K4":  # the next vertex closes a triangle: common-neighbour lists
                assert "tri_count" in prof, sorted(prof)
            ref_sizes = 0
            for b in range(2):
                ref = O.dp_count(g, pat, pat.n, colors[b], td=D.export(), sizes=True)
                assert int(counts[b]) == ref["count"] and bool(ovf[b]) == ref["overflow"], (pat.name, b)
                ref_sizes = ref_sizes + ref["sizes"]
            assert np.array_equal(sizes, ref_sizes), pat.name


def test_short_forget_runs_with_large_counts(ctx):
    # A hub joined to D vertices that are paired by edges: every pair closes a
    # triangle with the hub.  Pattern: triangle (0, 1, 2) with four leaves on
    # vertex 2.  Forgetting vertex 2 with 0 and 1 on a pair leaves runs of a
    # few colour sets whose counts, (D/7)^4 * 4! or so embeddings of the
    # leaves at the hub, exceed 2^28: the short-run forget must add them in
    # 64 bits.
    pat = W.Pattern(7, [(0, 1), (1, 2), (0, 2), (2, 3), (2, 4), (2, 5), (2, 6)], "triangle+4")
    for D in (600, 6000):
        src = np.concatenate([np.zeros(D, np.int64), np.arange(1, D, 2)])
        dst = np.concatenate([np.arange(1, D + 1), np.arange(2, D + 1, 2)])
        g = W.csr_from_edges(D + 1, src, dst)
        colors = np.random.default_rng(D).integers(0, 7, size=(3, g.n)).astype(np.uint8)
        counts, ovf, Dd = run_gpu(ctx, g, pat, 7, colors)
        for b in range(3):
            ref = O.dp_count(g, pat, 7, colors[b], td=Dd.export())
            assert ref["count"] > 1 << 32
            assert int(counts[b]) == ref["count"] and bool(ovf[b]) == ref["overflow"], (D, b)


def test_two_word_keys_match_oracle(ctx):
    # An ER(300) graph whose vertex ids are spread over 2^20 + 7 vertices: an
    # image takes 21 bits, so a bag of three or four columns, its colour set
    # and the colouring index need 128-bit keys, and every sorted-list kernel
    # runs its two-word form.
    g0 = W.er_pairs(300, 0.05, 21)
    n = (1 << 20) + 7
    ids = (np.arange(300, dtype=np.int64) * 3491 + 17) % n
    src = np.repeat(np.arange(300), np.diff(g0.row_ptr))
    m = src < g0.col
    g = W.csr_from_edges(n, ids[src[m]], ids[g0.col[m]])
    rng = np.random.default_rng(99)
    for pat in (W.cycle(5), W.ladder(3), W.partial_3tree(7, 2)):
        for k in (pat.n, pat.n + 1):
            colors = rng.integers(0, k, size=(3, g.n)).astype(np.uint8)
            say("two-word keys", pat.name, "k", k)
            counts, ovf, D = run_gpu(ctx, g, pat, k, colors)
            for b in range(3):
                ref = O.dp_count(g, pat, k, colors[b], td=D.export())
                assert int(counts[b]) == ref["count"] and bool(ovf[b]) == ref["overflow"], (pat.name, k, b)
            assert counts.any(), pat.name


def test_edge_cases(ctx):
    # graph without edges, pattern with edges: zero
    g = W.csr_from_edges(50, np.zeros(0, np.int64), np.zeros(0, np.int64))
    colors = np.zeros((1, 50), dtype=np.uint8)
    counts, _, _ = run_gpu(ctx, g, W.path(2), 2, colors)
    assert int(counts[0]) == 0
    # single-vertex pattern: every vertex
    counts, _, _ = run_gpu(ctx, g, W.Pattern(1, [], "K1"), 1, colors)
    assert int(counts[0]) == 50
    # pattern larger than the host graph
    g2 = W.er_pairs(4, 1.0, 1)
    counts, _, _ = run_gpu(ctx, g2, W.path(5), 5, np.zeros((1, 4), dtype=np.uint8))
    assert int(counts[0]) == 0
    # all vertices one colour: nothing colourful
    g3 = W.er_pairs(60, 0.2, 2)
    counts, _, _ = run_gpu(ctx, g3, W.cycle(4), 4, np.zeros((2, 60), dtype=np.uint8))
    assert counts.tolist() == [0, 0]


def test_device_colouring_matches_oracle_hash(ctx):
    g = W.er_pairs(1000, 0.01, 3)
    G = gpu_graph(ctx, g)
    C = cc.color(ctx, G, 7, 0xABCDEF, 5)
    for b in range(5):
        assert np.array_equal(C.download(b, g.n), O.color_array(0xABCDEF, b, g.n, 7))


def test_determinism(ctx):
    g = W.rgg(2000, 10, 4)
    G = gpu_graph(ctx, g)
    C = cc.color(ctx, G, 8, 5, 4)
    D = cc.build_decomposition(8, W.ladder(4).edges)
    a, _ = cc.count(ctx, G, C, D)
    b, _ = cc.count(ctx, G, C, D)
    assert np.array_equal(a, b)


# ---- the standard workloads at full size -------------------------------

def test_workload1_count(ctx):
    w = W.workload(1)
    g = W.workload_graph(1)
    pat = W.workload_pattern(1)
    G = gpu_graph(ctx, g)
    C = cc.color(ctx, G, w.k, w.color_seed, w.colorings)
    D = cc.build_decomposition(pat.n, pat.edges)
    counts, ovf = cc.count(ctx, G, C, D)
    col = O.color_array(w.color_seed, 0, g.n, w.k)
    assert int(counts[0]) == O.brute_count(g, pat, col) == O.dp_count(g, pat, w.k, col)["count"]
    assert not ovf[0]


def test_workload2_sampled_colourings(ctx):
    w = W.workload(2)
    g = W.workload_graph(2)
    pat = W.workload_pattern(2)
    G = gpu_graph(ctx, g)
    C = cc.color(ctx, G, w.k, w.color_seed, w.colorings)
    D = cc.build_decomposition(pat.n, pat.edges)
    say("workload 2 count, 64 colourings")
    counts, ovf = cc.count(ctx, G, C, D)
    for b in (0, 17, 63):
        col = O.color_array(w.color_seed, b, g.n, w.k)
        ref = O.dp_count(g, pat, w.k, col, td=D.export())
        assert int(counts[b]) == ref["count"] and bool(ovf[b]) == ref["overflow"]
    # the colourings in one batch equal the same colourings run alone
    say("workload 2 single colourings")
    for b in (5, 40):
        C1 = cc.color_explicit(ctx, G, w.k, O.color_array(w.color_seed, b, g.n, w.k))
        c1, _ = cc.count(ctx, G, C1, D)
        assert int(c1[0]) == int(counts[b])


def test_workload3_sampled_vertices(ctx):
    w = W.workload(3)
    g = W.workload_graph(3)
    pat = W.workload_pattern(3)
    G = gpu_graph(ctx, g)
    C = cc.color(ctx, G, w.k, w.color_seed, w.colorings)
    D = cc.build_decomposition(pat.n, pat.edges)
    say("workload 3 count, 32 colourings")
    counts, ovf = cc.count(ctx, G, C, D)
    assert not ovf.any()
    say("workload 3 per-vertex, colouring 1")
    pv, total, _ = cc.count_by_vertex(ctx, G, C, 1, D)
    assert total == int(counts[1]) and int(pv.sum()) == total
    col = O.color_array(w.color_seed, 1, g.n, w.k)
    rng = np.random.default_rng(0)
    for v in rng.choice(g.n, 40, replace=False):
        assert int(pv[v]) == O.brute_count(g, pat, col, fix0=int(v)), v


@pytest.mark.parametrize("gname,make", [("ba600", lambda: W.barabasi_albert(600, 3, 12)),
                                        ("rgg800", lambda: W.rgg(800, 8, 13)),
                                        ("cl1500", lambda: W.chung_lu(1500, 2.5, 6.0, 14))],
                         ids=["ba600", "rgg800", "cl1500"])
def test_entry_and_classic_introduce_match_oracle(ctx, gname, make):
    """Introduce nodes whose vertex has two or more bag neighbours: the
    entry-wise form (candidates from the lowest-degree neighbour's row, then
    a re-sort), per entry or per group of entries with equal bag images, and
    the fixed-column form give the oracle's counts, flags and per-node table
    sizes on heavy-tailed and clustered hosts."""
    g = make()
    pats = [W.complete(4), W.pattern_B(), W.ladder(4), W.cycle(6), W.partial_3tree(8, 5),
            W.partial_3tree(9, 21), W.partial_3tree(10, 8)]
    G = gpu_graph(ctx, g)
    for pat in pats:
        D = cc.build_decomposition(pat.n, pat.edges)
        td = D.export()
        C = cc.color(ctx, G, pat.n, 31, 2)
        ref = [O.dp_count(g, pat, pat.n, O.color_array(31, b, g.n, pat.n), td=td, sizes=True) for b in range(2)]
        # (flags, entry_factor, group_min): default; entry-wise whenever it
        # walks fewer candidates, always grouped; the same, never grouped;
        # the fixed-column forms only
        for flags, ef, gm in ((0, 3, 2), (0, 1, 1), (0, 1, 0), (cc.CC_CLASSIC_EXPAND, 3, 2)):
            say("introduce forms", gname, pat.name, "flags", flags, "entry_factor", ef, "group_min", gm)
            ctx.set_schedule(entry_factor=ef, group_min=gm)
            try:
                counts, ovf = cc.count(ctx, G, C, D, flags)
            finally:
                ctx.set_schedule()
            sizes = ctx.last_table_sizes()
            for b in range(2):
                assert int(counts[b]) == ref[b]["count"] and bool(ovf[b]) == ref[b]["overflow"], (gname, pat.name, flags, gm, b)
            assert np.array_equal(sizes, ref[0]["sizes"] + ref[1]["sizes"]), (gname, pat.name, flags, gm)


@pytest.mark.parametrize("gname,make", [("er150", lambda: W.er_pairs(150, 0.07, 9)),
                                        ("ba500", lambda: W.barabasi_albert(500, 3, 10)),
                                        ("rgg400", lambda: W.rgg(400, 8, 11))], ids=["er150", "ba500", "rgg400"])
def test_distance_bounded_introduce_matches_oracle(ctx, gname, make):
    """Pattern C's decomposition introduces vertices with no bag neighbour but
    a bag vertex at distance 2 (Sec. 3.2): their candidates are the walks of
    length <= 2 from that vertex's image, de-duplicated.  Same counts, flags
    and table sizes as the oracle with the same bound; with CC_CLASSIC_EXPAND
    the full scan, equal to the oracle without the bound."""
    g = make()
    pat = W.pattern_C()
    D = cc.build_decomposition(pat.n, pat.edges)
    assert "anchor=-1" in D.describe()
    td = D.export()
    G = gpu_graph(ctx, g)
    C = cc.color(ctx, G, pat.n, 57, 2)
    for flags in (0, cc.CC_CLASSIC_EXPAND):
        say("distance-bounded", gname, "flags", flags)
        # the full scan (CC_CLASSIC_EXPAND) keeps the entries the bound drops
        ref = [O.dp_count(g, pat, pat.n, O.color_array(57, b, g.n, pat.n), td=td, sizes=True,
                          distbound=(flags == 0)) for b in range(2)]
        counts, ovf = cc.count(ctx, G, C, D, flags)
        sizes = ctx.last_table_sizes()
        for b in range(2):
            assert int(counts[b]) == ref[b]["count"] and bool(ovf[b]) == ref[b]["overflow"], (gname, flags, b)
        assert np.array_equal(sizes, ref[0]["sizes"] + ref[1]["sizes"]), (gname, flags)


def test_wide_colour_sets_match_oracle(ctx):
    """k from 13 to 16 colours (the paper's masks allow n_F <= 32, Sec. 3.2):
    forget and join by sorting and adding up runs instead of the dense 2^k
    accumulators; paths up to P15 (the paper's largest pattern), trees with
    joins and a ladder, against the oracle, with flags.  Enumeration stays
    limited to k <= 12."""
    g = W.er_pairs(90, 0.1, 17)
    G = gpu_graph(ctx, g)
    cases = [(W.path(13), 13), (W.path(13), 14), (W.path(15), 15), (W.random_tree(14, 3), 14),
             (W.star(13), 13), (W.ladder(6), 13), (W.random_tree(16, 9), 16)]
    for pat, k in cases:
        say("wide colour sets", pat.name, "k", k)
        D = cc.build_decomposition(pat.n, pat.edges)
        td = D.export()
        C = cc.color(ctx, G, k, 5, 2)
        counts, ovf = cc.count(ctx, G, C, D)
        sizes = ctx.last_table_sizes()
        ref_sizes = 0
        for b in range(2):
            ref = O.dp_count(g, pat, k, O.color_array(5, b, g.n, k), td=td, sizes=True)
            assert int(counts[b]) == ref["count"] and bool(ovf[b]) == ref["overflow"], (pat.name, k, b)
            ref_sizes = ref_sizes + ref["sizes"]
        assert np.array_equal(sizes, ref_sizes), (pat.name, k)
    with pytest.raises(cc.CcError) as e:
        cc.enumerate(ctx, G, C, 0, D, 10)
    assert e.value.code == cc.CC_ERANGE
    with pytest.raises(cc.CcError) as e:
        cc.color(ctx, G, 17, 1, 1)
    assert e.value.code == cc.CC_ERANGE
