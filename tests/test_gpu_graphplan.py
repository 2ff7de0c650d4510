"""Counts captured into HIP graphs (cc_plan_*) against eager cc_count and
the oracle: several replays with new seeds, with eager work of the same
context and synchronisations between them, every replay checked."""
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


@pytest.mark.parametrize("pat", [W.path(5), W.random_tree(8, 4), W.star(6), W.pattern_A()], ids=lambda p: p.name)
def test_plan_replays_equal_eager_and_oracle(ctx, pat):
    g = W.er_skip(3000, 6.0 / 2999, 51)
    G = cc.load_graph(ctx, g.n, g.row_ptr, g.col)
    D = cc.build_decomposition(pat.n, pat.edges)
    B = 8
    plan = cc.Plan(ctx, G, D, pat.n, B)
    other = cc.build_decomposition(5, W.cycle(5).edges)
    for rep, seed in enumerate((11, 12, 11, 99)):
        say("plan", pat.name, "replay", rep, "seed", seed)
        got, ovf = plan.count(seed)
        C = cc.color(ctx, G, pat.n, seed, B)
        ref, ref_ovf = cc.count(ctx, G, C, D)
        assert np.array_equal(got, ref) and np.array_equal(ovf, ref_ovf), (pat.name, rep)
        for b in (0, B - 1):
            assert int(got[b]) == O.dp_count(g, pat, pat.n, O.color_array(seed, b, g.n, pat.n))["count"]
        # eager work of another plan shape between replays
        C5 = cc.color(ctx, G, 5, seed, 2)
        cc.count(ctx, G, C5, other)
    plan.close()


def test_plan_refuses_sorted_list_plans(ctx):
    g = W.er_pairs(200, 0.05, 2)
    G = cc.load_graph(ctx, g.n, g.row_ptr, g.col)
    D = cc.build_decomposition(5, W.cycle(5).edges)
    with pytest.raises(cc.CcError) as e:
        cc.Plan(ctx, G, D, 5, 4)
    assert e.value.code == cc.CC_ERANGE
