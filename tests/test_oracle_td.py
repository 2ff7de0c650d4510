"""Pins of the oracle's tree-decomposition side (Sec. 1.2 definitions, Sec. 3).

* splitmix64 against its published outputs (golden file).
* the colour map against colours derived by hand from those outputs (golden
  file).
* exact treewidth against the families' known values and Table `prop`
  (golden file), and against brute force over all elimination orderings.
* the nice-TD validator accepts the oracle's TDs and rejects planted mistakes.
"""
import itertools
import os

import numpy as np
import pytest

import oracle as O
from paper_1908_11248_amd import workloads as W

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def test_splitmix64_published_vectors():
    gamma = 0x9E3779B97F4A7C15
    n = 0
    for line in open(os.path.join(GOLDEN, "splitmix64_vectors.txt")):
        if line.startswith("#") or not line.strip():
            continue
        seed, i, out = (int(x) for x in line.split())
        assert O.splitmix64((seed + (i - 1) * gamma) % 2**64) == out
        n += 1
    assert n == 6


def test_colour_map_hand_derived_vectors():
    """Colours derived by hand from the published splitmix64 outputs
    (golden/colour_vectors.txt): pins the seed mixing, the high word and the
    multiply-shift, for b = 0 and b > 0 and vertex ids up to 2^31 - 1."""
    n = 0
    for line in open(os.path.join(GOLDEN, "colour_vectors.txt")):
        if line.startswith("#") or not line.strip():
            continue
        seed, b, v, k, colour = (int(x) for x in line.split("|")[0].split())
        assert O.color_of(seed, b, v, k) == colour, line
        if v < 200000:
            assert int(O.color_array(seed, b, v + 1, k)[v]) == colour, line
        n += 1
    assert n == 18


def test_colouring_range_and_uniformity():
    k = 7
    c = O.color_array(12345, 3, 70000, k)
    assert c.min() >= 0 and c.max() < k
    h = np.bincount(c, minlength=k)
    exp = c.size / k
    chi2 = float(((h - exp) ** 2 / exp).sum())
    assert chi2 < 30.0  # 6 degrees of freedom: p ~ 4e-5
    # different colourings / seeds differ
    assert (O.color_array(12345, 4, 1000, k) != c[:1000]).mean() > 0.5


def _by_name():
    return {"A": W.pattern_A(), "B": W.pattern_B(), "C": W.pattern_C(), "D": W.pattern_D()}


def _connected(p):
    adj = {v: set() for v in range(p.n)}
    for a, b in p.edges:
        adj[a].add(b)
        adj[b].add(a)
    seen = {0}
    st = [0]
    while st:
        x = st.pop()
        for y in adj[x]:
            if y not in seen:
                seen.add(y)
                st.append(y)
    return len(seen) == p.n


def test_table_prop_patterns():
    pats = _by_name()
    rows = 0
    for line in open(os.path.join(GOLDEN, "table_prop.txt")):
        if line.startswith("#") or not line.strip():
            continue
        name, nv, ne, tw, conn = line.split()
        p = pats[name]
        assert p.n == int(nv)
        assert len(set(map(frozenset, p.edges))) == int(ne)
        assert O.treewidth(p) == int(tw)
        assert _connected(p) == bool(int(conn))
        td, w = O.build_td(p)
        assert w == int(tw)
        assert O.validate_td(p, td) == 0
        rows += 1
    assert rows == 4


@pytest.mark.parametrize("n", [2, 3, 5, 8, 12])
def test_family_treewidths(n):
    assert O.treewidth(W.path(n)) == 1
    assert O.treewidth(W.star(n)) == 1
    if n >= 3:
        assert O.treewidth(W.cycle(n)) == 2
    if n <= 8:
        assert O.treewidth(W.complete(n)) == n - 1


@pytest.mark.parametrize("r,c", [(2, 2), (2, 4), (3, 3), (3, 4)])
def test_grid_treewidth(r, c):
    assert O.treewidth(W.grid(r, c)) == min(r, c)


def _width_of_order(n, edges, order):
    adj = {v: set() for v in range(n)}
    for a, b in edges:
        adj[a].add(b)
        adj[b].add(a)
    width = 0
    alive = set(range(n))
    for v in order:
        nb = adj[v] & alive - {v}
        width = max(width, len(nb))
        for a in nb:
            adj[a] |= nb - {a}
        alive.discard(v)
    return width


@pytest.mark.parametrize("seed", range(12))
def test_treewidth_vs_all_orderings(seed):
    rng = np.random.default_rng(seed)
    n = int(rng.integers(3, 7))
    p = float(rng.uniform(0.3, 0.8))
    edges = [(i, j) for i in range(n) for j in range(i + 1, n) if rng.random() < p]
    pat = W.Pattern(n, edges)
    best = min(_width_of_order(n, edges, o) for o in itertools.permutations(range(n)))
    assert O.treewidth(pat) == best
    td, w = O.build_td(pat)
    assert w == best
    assert O.validate_td(pat, td) == 0
    # the width realised by the nice TD's bags equals the treewidth
    N = int(td[0])
    bags = [int(td[5 + 5 * i]) & 0xFFFFFFFF for i in range(N)]
    assert max(bin(b).count("1") for b in bags) - 1 == max(best, 0)


def _mutate(td, i, field, value):
    t = td.copy()
    t[1 + 5 * i + field] = value
    return t


def test_validator_rejects_planted_mistakes():
    p = W.cycle(5)
    td, _ = O.build_td(p)
    assert O.validate_td(p, td) == 0
    N = int(td[0])
    # root must be empty
    assert O.validate_td(p, _mutate(td, N - 1, 4, 1)) != 0
    # an introduce node whose bag misses its vertex
    for i in range(N):
        if td[1 + 5 * i] == 1:
            assert O.validate_td(p, _mutate(td, i, 4, int(td[5 + 5 * i]) ^ (1 << int(td[2 + 5 * i])))) != 0
            break
    # a pattern with an extra edge is not covered by the cycle's TD
    q = W.Pattern(5, p.edges + [(0, 2), (1, 3), (2, 4), (0, 3)])
    assert O.validate_td(q, td) != 0
    # a forget node that forgets a vertex which is not in its child's bag
    for i in range(N):
        if td[1 + 5 * i] == 2:
            u = int(td[2 + 5 * i])
            other = (u + 1) % 5
            assert O.validate_td(p, _mutate(td, i, 1, other)) != 0
            break
