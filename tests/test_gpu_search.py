"""The distinct-vertex-set mode and the repetition driver on the GPU against
the oracle's step-by-step versions (pinned in tests/test_oracle_count.py):
equal sets of solutions, equal numbers of colourings run."""
import math
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


@pytest.mark.parametrize("pat", [W.path(4), W.cycle(4), W.star(4), W.pattern_B(), W.cycle(5)], ids=lambda p: p.name)
def test_vertex_sets_match_oracle(ctx, pat):
    g = W.er_pairs(80, 0.12, 5)
    G = cc.load_graph(ctx, g.n, g.row_ptr, g.col)
    D = cc.build_decomposition(pat.n, pat.edges)
    C = cc.color(ctx, G, pat.n, 3, 3)
    for b in range(3):
        say("vertex sets", pat.name, "colouring", b)
        sets, nmap = cc.vertex_sets(ctx, G, C, b, D, 10**6)
        col = O.color_array(3, b, g.n, pat.n)
        ref = O.vertex_sets(g, pat, pat.n, col)
        assert nmap == O.dp_count(g, pat, pat.n, col)["count"]
        assert [tuple(r) for r in sets] == ref, (pat.name, b)
    # a cap below the mappings is an error
    if nmap > 1:
        with pytest.raises(cc.CcError) as e:
            cc.vertex_sets(ctx, G, C, 2, D, nmap - 1)
        assert e.value.code == cc.CC_ERANGE


@pytest.mark.parametrize("pat,maxsol,sets", [(W.path(3), 10**5, False), (W.cycle(4), 40, False),
                                             (W.path(4), 500, True), (W.pattern_B(), 25, False)],
                         ids=["P3-all", "C4-40", "P4-sets", "B-25"])
def test_search_matches_oracle(ctx, pat, maxsol, sets):
    g = W.er_pairs(40, 0.15, 6)
    G = cc.load_graph(ctx, g.n, g.row_ptr, g.col)
    D = cc.build_decomposition(pat.n, pat.edges)
    eps = 1 / math.e
    say("search", pat.name, "max", maxsol, "sets", sets)
    rows, run, planned = cc.search(ctx, G, D, eps, 11, maxsol, batch=8, distinct_sets=sets)
    ref, ref_run = O.search(g, pat, eps, 11, maxsol, distinct_sets=sets)
    assert planned == O.repetitions(pat.n, eps)
    assert run == ref_run
    assert [tuple(r) for r in rows] == ref
