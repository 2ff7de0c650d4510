"""GPU parity of enumeration (Sec. 4): the rows the HIP path returns equal the
oracle's, bit for bit -- the lexicographically first min(count, cap)
colourful mappings (Phi(0), ..., Phi(n_F - 1)) of one colouring."""
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


PATS = [W.path(3), W.path(5), W.cycle(4), W.cycle(5), W.star(4), W.grid(2, 3), W.ladder(3), W.complete(4),
        W.pattern_B(), W.pattern_D(), W.random_tree(7, 3), W.partial_3tree(6, 1), W.Pattern(1, [], "K1")]


@pytest.mark.parametrize("pat", PATS, ids=lambda p: p.name)
def test_enumeration_matches_oracle(ctx, pat):
    g = W.er_pairs(60, 0.12, 11)
    G = cc.load_graph(ctx, g.n, g.row_ptr, g.col)
    rng = np.random.default_rng(pat.n)
    D = cc.build_decomposition(pat.n, pat.edges)
    for k in sorted({pat.n, min(pat.n + 1, 12)}):
        colors = rng.integers(0, k, size=(2, g.n)).astype(np.uint8)
        C = cc.color_explicit(ctx, G, k, colors)
        for b in range(2):
            say("enum", pat.name, "k", k, "b", b)
            ref = O.brute_enum(g, pat, colors[b], 10**7)
            rows, total = cc.enumerate(ctx, G, C, b, D, 10**7)
            assert total == len(ref)
            assert np.array_equal(rows, ref)
            if len(ref) > 3:
                cap = len(ref) // 3
                rows2, total2 = cc.enumerate(ctx, G, C, b, D, cap)
                assert total2 == len(ref) and np.array_equal(rows2, ref[:cap])
            rows0, total0 = cc.enumerate(ctx, G, C, b, D, 0)
            assert rows0.shape[0] == 0 and total0 == len(ref)


def test_enumeration_with_oracle_reconstruction(ctx):
    """Rows also equal the oracle's own R(x, M) reconstruction."""
    g = W.rgg(400, 8, 5)
    G = cc.load_graph(ctx, g.n, g.row_ptr, g.col)
    for pat in [W.cycle(5), W.pattern_B(), W.ladder(3)]:
        col = O.color_array(99, 0, g.n, pat.n)
        C = cc.color_explicit(ctx, G, pat.n, col)
        D = cc.build_decomposition(pat.n, pat.edges)
        rows, total = cc.enumerate(ctx, G, C, 0, D, 10**7)
        ref, tot = O.dp_enumerate(g, pat, pat.n, col, 10**7, td=D.export())
        assert total == tot and np.array_equal(rows, ref)


def test_workload1_full_enumeration(ctx):
    w = W.workload(1)
    g = W.workload_graph(1)
    pat = W.workload_pattern(1)
    G = cc.load_graph(ctx, g.n, g.row_ptr, g.col)
    C = cc.color(ctx, G, w.k, w.color_seed, w.colorings)
    D = cc.build_decomposition(pat.n, pat.edges)
    rows, total = cc.enumerate(ctx, G, C, 0, D, 10**8)
    col = O.color_array(w.color_seed, 0, g.n, w.k)
    ref = O.brute_enum(g, pat, col, 10**8)
    assert total == len(ref) == rows.shape[0]
    assert np.array_equal(rows, ref)


@pytest.mark.parametrize("b", [0, 13])
def test_workload3_capped_enumeration(ctx, b):
    w = W.workload(3)
    g = W.workload_graph(3)
    pat = W.workload_pattern(3)
    G = cc.load_graph(ctx, g.n, g.row_ptr, g.col)
    C = cc.color(ctx, G, w.k, w.color_seed, w.colorings)
    D = cc.build_decomposition(pat.n, pat.edges)
    say("workload 3 enumeration, colouring", b)
    rows, total = cc.enumerate(ctx, G, C, b, D, w.cap)
    col = O.color_array(w.color_seed, b, g.n, w.k)
    ref = O.brute_enum(g, pat, col, w.cap)
    assert rows.shape == ref.shape == (w.cap, 8)
    assert np.array_equal(rows, ref)
    counts, _ = cc.count(ctx, G, C, D)
    assert total == int(counts[b])


def test_enumeration_with_two_word_keys(ctx):
    """An ER(300) graph with its vertex ids spread over 2^20 + 7 vertices: the
    tables of a bag of three columns need 128-bit keys, and the rows still
    equal brute force's, capped or not."""
    g0 = W.er_pairs(300, 0.05, 21)
    n = (1 << 20) + 7
    ids = (np.arange(300, dtype=np.int64) * 3491 + 17) % n
    src = np.repeat(np.arange(300), np.diff(g0.row_ptr))
    m = src < g0.col
    g = W.csr_from_edges(n, ids[src[m]], ids[g0.col[m]])
    G = cc.load_graph(ctx, g.n, g.row_ptr, g.col)
    rng = np.random.default_rng(7)
    for pat in (W.cycle(5), W.ladder(3)):
        colors = rng.integers(0, pat.n, size=(1, g.n)).astype(np.uint8)
        C = cc.color_explicit(ctx, G, pat.n, colors)
        D = cc.build_decomposition(pat.n, pat.edges)
        say("enum two-word keys", pat.name)
        ref = O.brute_enum(g, pat, colors[0], 10**7)
        assert len(ref) > 0
        rows, total = cc.enumerate(ctx, G, C, 0, D, 10**7)
        assert total == len(ref) and np.array_equal(rows, ref)
        cap = len(ref) // 3
        rows2, total2 = cc.enumerate(ctx, G, C, 0, D, cap)
        assert total2 == len(ref) and np.array_equal(rows2, ref[:cap])
        C.close()
