"""CPU-side checks of the HIP library: it loads, exports every symbol the
header declares, and its host planner (exact-width nice tree decomposition,
Sec. 3 / Sec. 1.2) agrees with the oracle's treewidth and passes the oracle's
validator.  No compute call is made here (no GPU)."""
import os
import re

import numpy as np
import pytest

import oracle as O
import paper_1908_11248_amd as cc
from paper_1908_11248_amd import workloads as W

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def header_symbols():
    txt = open(os.path.join(ROOT, "include", "ccgpu.h")).read()
    return sorted(set(re.findall(r"\b(cc_[a-z_]+)\s*\(", txt)))


def test_library_exports_every_declared_symbol():
    L = cc.lib()
    syms = header_symbols()
    assert len(syms) >= 20
    for s in syms:
        assert hasattr(L, s), s
    assert sorted(cc.EXPORTS) == syms


PATTERNS = [W.path(2), W.path(5), W.cycle(3), W.cycle(6), W.cycle(10), W.star(6), W.ladder(4), W.grid(3, 3),
            W.complete(4), W.pattern_A(), W.pattern_B(), W.pattern_C(), W.pattern_D(),
            W.Pattern(1, [], "K1")] + [W.random_tree(n, n) for n in range(5, 11)] + \
           [W.partial_3tree(n, 7 * n) for n in range(5, 11)]


@pytest.mark.parametrize("pat", PATTERNS, ids=lambda p: p.name)
def test_planner_decomposition_valid_and_optimal(pat):
    d = cc.build_decomposition(pat.n, pat.edges)
    td = d.export()
    assert O.validate_td(pat, td) == 0
    assert d.width == O.treewidth(pat)
    # pattern vertex 0 is forgotten last: the node below the root holds {0}
    N = int(td[0])
    root_child = int(td[1 + 5 * (N - 1) + 2])
    assert int(td[5 + 5 * root_child]) == 1
    # re-import round trip
    d2 = cc.decomp_import(pat.n, pat.edges, td)
    assert np.array_equal(d2.export(), td)


def test_import_accepts_oracle_decompositions():
    for pat in PATTERNS:
        td, _ = O.build_td(pat)
        d = cc.decomp_import(pat.n, pat.edges, td)
        assert np.array_equal(d.export(), td)


def test_import_rejects_invalid_decompositions():
    pat = W.cycle(5)
    td, _ = O.build_td(pat)
    bad = td.copy()
    bad[5 + 5 * (int(td[0]) - 1)] = 1  # non-empty root
    with pytest.raises(cc.CcError):
        cc.decomp_import(pat.n, pat.edges, bad)
    with pytest.raises(cc.CcError):  # edges not covered
        cc.decomp_import(5, pat.edges + [(0, 2), (1, 3), (2, 4)], td)
    with pytest.raises(cc.CcError):
        cc.decomp_import(5, pat.edges, td[:-1])


def test_limits():
    with pytest.raises(cc.CcError):
        cc.build_decomposition(17, [(i, i + 1) for i in range(16)])
    with pytest.raises(cc.CcError):  # treewidth 4 exceeds the device bag limit
        cc.build_decomposition(5, W.complete(5).edges)
    with pytest.raises(cc.CcError):
        cc.build_decomposition(3, [(0, 3)])
