"""cc_count_noalloc (the entry point for callers that cannot allocate) against
cc_count on the same inputs, through the C ABI: bit-equal counts and
overflow flags on two calls in a row (the second smaller than the first), on
both table forms (dense slot tables for trees, sorted lists otherwise), and
CC_ERANGE for inputs beyond its fixed 64 MiB device scratch."""
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
    c = cc.Context(0, arena_bytes=4 << 30)
    yield c
    c.close()


def _both(ctx, g, pat, k, seed, B, flags=0):
    G = cc.load_graph(ctx, g.n, g.row_ptr, g.col)
    C = cc.color(ctx, G, k, seed, B)
    D = cc.build_decomposition(pat.n, pat.edges)
    ref, ref_ovf = cc.count(ctx, G, C, D, flags)
    ref_sizes = ctx.last_table_sizes()
    got, got_ovf = cc.count_noalloc(ctx, G, C, D, flags)
    assert np.array_equal(got, ref), (pat.name, g.n, B)
    assert np.array_equal(got_ovf, ref_ovf)
    assert np.array_equal(ctx.last_table_sizes(), ref_sizes)
    return got


@pytest.mark.parametrize("flags", [0, cc.CC_SPARSE_TABLES])
def test_noalloc_equals_count_two_calls_second_smaller(ctx, flags):
    big = W.er_skip(1000, 5.0 / 999, 31)
    small = W.er_pairs(200, 0.05, W.workload(1).seed)
    for pat in (W.random_tree(8, 4), W.cycle(5), W.pattern_B()):
        say("noalloc", pat.name, "flags", flags, "first call: n", big.n, "B 8")
        _both(ctx, big, pat, pat.n, 17, 8, flags)
        say("noalloc", pat.name, "flags", flags, "second call: n", small.n, "B 2")
        got = _both(ctx, small, pat, pat.n, 18, 2, flags)
        for b in range(2):
            col = O.color_array(18, b, small.n, pat.n)
            assert int(got[b]) == O.dp_count(small, pat, pat.n, col)["count"]


def test_noalloc_rejects_inputs_beyond_its_scratch(ctx):
    say("noalloc: limits")
    g = W.er_skip(70000, 4.0 / 69999, 32)
    G = cc.load_graph(ctx, g.n, g.row_ptr, g.col)
    D = cc.build_decomposition(5, W.path(5).edges)
    C = cc.color(ctx, G, 5, 1, 64)  # 64 x 70000 x 16 bytes > 64 MiB
    with pytest.raises(cc.CcError) as e:
        cc.count_noalloc(ctx, G, C, D)
    assert e.value.code == cc.CC_ERANGE
    # fits the first check, but its tables outgrow the scratch during the run
    g2 = W.er_skip(20000, 12.0 / 19999, 33)
    G2 = cc.load_graph(ctx, g2.n, g2.row_ptr, g2.col)
    D6 = cc.build_decomposition(6, W.cycle(6).edges)
    C2 = cc.color(ctx, G2, 6, 2, 16)
    with pytest.raises(cc.CcError) as e:
        cc.count_noalloc(ctx, G2, C2, D6)
    assert e.value.code == cc.CC_ERANGE
    # and the next call that fits is still right
    _both(ctx, W.er_pairs(200, 0.05, 3), W.cycle(4), 4, 5, 3)
