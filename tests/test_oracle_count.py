"""Pins of the oracle's counting DP (Sec. 3.1) and reconstruction (Sec. 4).

Nothing here re-types the oracle's own formulas.  The DP and the C brute
force are pinned against:
* the definition, evaluated by a pure-Python brute force over ALL mappings;
* the colourful-probability statement of Sec. 2.1 (a fixed injective copy is
  colourful with probability n_F!/n_F^n_F), summed exactly over every
  colouring of a tiny host;
* closed forms: single vertex, an edge, P3, stars (big integers), complete
  hosts;
* invariants: colour permutation, relabelling of G and of F, choice of the
  tree decomposition, the degree mask, |Aut(F)| divisibility, additivity over
  disjoint unions of G, and the split of a disconnected pattern over colour
  sets.
"""
import itertools
import math

import numpy as np
import pytest

import oracle as O
from oracle import brute as B
from paper_1908_11248_amd import workloads as W

U64 = 2**64


def zoo_graphs():
    gs = [W.er_pairs(8, 0.5, 11), W.er_pairs(10, 0.4, 12), W.er_pairs(12, 0.3, 13)]
    gs.append(W.csr_from_edges(6, np.arange(6), (np.arange(6) + 1) % 6, "C6"))  # host cycle
    a, b = np.triu_indices(6, 1)
    gs.append(W.csr_from_edges(6, a, b, "K6"))
    return gs


ZOO_PATTERNS = [W.path(2), W.path(3), W.path(4), W.cycle(3), W.cycle(4), W.star(4),
                W.grid(2, 2), W.Pattern(4, [(0, 1), (2, 3)], "2K2"),
                W.Pattern(4, [(0, 1), (1, 2), (0, 2), (2, 3)], "paw")]


def colours(rng, n, k):
    return rng.integers(0, k, size=n).astype(np.uint8)


@pytest.mark.parametrize("pi", range(len(ZOO_PATTERNS)))
def test_dp_and_brute_vs_definition(pi):
    pat = ZOO_PATTERNS[pi]
    rng = np.random.default_rng(100 + pi)
    for g in zoo_graphs():
        for k in {pat.n, pat.n + 1}:
            col = colours(rng, g.n, k)
            ref = B.all_mappings(g, pat, col)
            assert O.brute_count(g, pat, col) == len(ref)
            r = O.dp_count(g, pat, k, col)
            assert r["count"] == len(ref) and not r["overflow"]
            rows, tot = O.dp_enumerate(g, pat, k, col, 10**9)
            assert tot == len(ref)
            assert [tuple(x) for x in rows] == ref
            assert [tuple(x) for x in O.brute_enum(g, pat, col, 10**9)] == ref
            cap = max(1, len(ref) // 3)
            capped, tot2 = O.dp_enumerate(g, pat, k, col, cap)
            assert [tuple(x) for x in capped] == ref[:cap] and tot2 == len(ref)


@pytest.mark.parametrize("name", ["A", "B", "C", "D"])
def test_paper_patterns_vs_brute(name):
    pat = {"A": W.pattern_A, "B": W.pattern_B, "C": W.pattern_C, "D": W.pattern_D}[name]()
    rng = np.random.default_rng(7)
    g = W.er_pairs(40, 0.25, 3)
    for _ in range(3):
        col = colours(rng, g.n, pat.n)
        bc = O.brute_count(g, pat, col)
        assert O.dp_count(g, pat, pat.n, col)["count"] == bc
    if name in ("B", "D"):  # small enough to reconstruct
        rows, tot = O.dp_enumerate(g, pat, pat.n, col, 10**9)
        assert tot == bc
        assert [tuple(x) for x in rows] == [tuple(x) for x in O.brute_enum(g, pat, col, 10**9)]


@pytest.mark.parametrize("pat", [W.path(3), W.cycle(3), W.star(3), W.Pattern(3, [(0, 1)], "K2+K1")],
                         ids=lambda p: p.name)
def test_sum_over_all_colourings(pat):
    """Sum over all k^n colourings of the colourful count equals
    #injective copies x k(k-1)...(k-nF+1) x k^(n-nF): every fixed injective
    mapping is colourful in exactly that many colourings (Sec. 2.1)."""
    g = W.er_pairs(6, 0.6, 5)
    k = pat.n
    inj = B.injective_homomorphisms(g, pat)
    total = 0
    for col in itertools.product(range(k), repeat=g.n):
        total += O.dp_count(g, pat, k, np.asarray(col, dtype=np.uint8))["count"]
    falling = math.perm(k, pat.n)
    assert total == inj * falling * k ** (g.n - pat.n)


def test_single_vertex_pattern():
    g = W.er_pairs(30, 0.2, 9)
    col = np.zeros(g.n, dtype=np.uint8)
    assert O.dp_count(g, W.Pattern(1, [], "K1"), 1, col)["count"] == g.n


def _colour_hist(g, col, k):
    h = np.zeros((g.n, k), dtype=object)
    for v in range(g.n):
        for w in g.col[g.row_ptr[v]:g.row_ptr[v + 1]]:
            h[v, col[w]] += 1
    return h


def test_edge_and_p3_closed_forms():
    g = W.er_pairs(60, 0.15, 21)
    rng = np.random.default_rng(1)
    for _ in range(4):
        col = colours(rng, g.n, 2)
        a, b = W.edge_list(g)
        assert O.dp_count(g, W.path(2), 2, col)["count"] == 2 * int((col[a] != col[b]).sum())
        col = colours(rng, g.n, 3)
        h = _colour_hist(g, col, 3)
        ref = 0
        for v in range(g.n):
            hs = [h[v, c] for c in range(3) if c != col[v]]
            ref += sum(hs) ** 2 - sum(x * x for x in hs)
        assert O.dp_count(g, W.path(3), 3, col)["count"] == ref


@pytest.mark.parametrize("k", [3, 4, 5])
def test_star_closed_form_and_overflow(k):
    """Star S_k with k colours: sum_v (k-1)! prod_{c != col(v)} h_c(v); compared
    mod 2^64 (big integers on the Python side), overflow flag iff too big."""
    # a host with hubs so that counts get large for k = 5
    rng = np.random.default_rng(k)
    n = 400
    hubs = np.arange(4)
    a = np.concatenate([np.repeat(hubs, n - 4), rng.integers(4, n, 800)])
    b = np.concatenate([np.tile(np.arange(4, n), 4), rng.integers(4, n, 800)])
    g = W.csr_from_edges(n, a, b)
    col = colours(rng, n, k)
    h = _colour_hist(g, col, k)
    ref = 0
    for v in range(n):
        p = 1
        for c in range(k):
            if c != col[v]:
                p *= int(h[v, c])
        ref += math.factorial(k - 1) * p
    r = O.dp_count(g, W.star(k), k, col)
    assert r["count"] == ref % U64
    if ref < U64:
        assert not r["overflow"]


def test_star_overflow_flag_on_huge_counts():
    # one hub of degree 6000, S7: (k-1)! prod h_c ~ 720 * 1000^6 > 2^64
    n = 6001
    g = W.csr_from_edges(n, np.zeros(n - 1, dtype=np.int64), np.arange(1, n))
    k = 7
    col = (np.arange(n) % k).astype(np.uint8)
    col[0] = 0
    h = _colour_hist(g, col, k)
    ref = math.factorial(k - 1) * math.prod(int(h[0, c]) for c in range(1, k))
    assert ref >= U64
    r = O.dp_count(g, W.star(k), k, col)
    assert r["count"] == ref % U64
    assert r["overflow"]


@pytest.mark.parametrize("pat", [W.path(4), W.cycle(4), W.star(4), W.pattern_B()], ids=lambda p: p.name)
def test_complete_host_closed_form(pat):
    """G = K_N, n_F = k: count = k! prod_c N_c (N_c = vertices of colour c)."""
    N = 9
    a, b = np.triu_indices(N, 1)
    g = W.csr_from_edges(N, a, b)
    rng = np.random.default_rng(3)
    k = pat.n
    for _ in range(3):
        col = colours(rng, N, k)
        Nc = np.bincount(col, minlength=k)
        ref = math.factorial(k) * math.prod(int(x) for x in Nc)
        assert O.dp_count(g, pat, k, col)["count"] == ref


def test_invariants_relabel_permute_td_degmask():
    rng = np.random.default_rng(17)
    g = W.er_pairs(50, 0.12, 8)
    for pat in [W.path(5), W.cycle(5), W.pattern_B(), W.pattern_D(), W.random_tree(6, 4)]:
        k = pat.n
        col = colours(rng, g.n, k)
        base = O.dp_count(g, pat, k, col)["count"]
        # colour permutation
        perm = rng.permutation(k).astype(np.uint8)
        assert O.dp_count(g, pat, k, perm[col])["count"] == base
        # relabel G
        sigma = rng.permutation(g.n)
        g2 = W.relabel(g, sigma)
        col2 = np.empty_like(col)
        col2[sigma] = col
        assert O.dp_count(g2, pat, k, col2)["count"] == base
        # relabel F
        tau = rng.permutation(pat.n)
        pat2 = W.Pattern(pat.n, [(int(tau[a]), int(tau[b])) for a, b in pat.edges])
        assert O.dp_count(g, pat2, k, col)["count"] == base
        # a different TD: the relabelled pattern's TD mapped back to F
        td2, _ = O.build_td(pat2)
        inv = np.argsort(tau)
        td3 = td2.copy()
        N = int(td3[0])
        for i in range(N):
            u = int(td3[2 + 5 * i])
            if u >= 0:
                td3[2 + 5 * i] = inv[u]
            bag = int(td3[5 + 5 * i]) & 0xFFFFFFFF
            nb = 0
            for v in range(pat.n):
                if bag >> v & 1:
                    nb |= 1 << int(inv[v])
            td3[5 + 5 * i] = nb
        assert O.validate_td(pat, td3) == 0
        assert O.dp_count(g, pat, k, col, td=td3)["count"] == base
        # degree mask off
        assert O.dp_count(g, pat, k, col, degmask=False)["count"] == base


@pytest.mark.parametrize("pat", [W.path(4), W.cycle(4), W.cycle(5), W.star(5), W.grid(2, 3), W.ladder(3)],
                         ids=lambda p: p.name)
def test_automorphism_divisibility(pat):
    aut = B.automorphisms(pat)
    g = W.er_pairs(60, 0.2, 31)
    rng = np.random.default_rng(5)
    for _ in range(3):
        c = O.dp_count(g, pat, pat.n, colours(rng, g.n, pat.n))["count"]
        assert c % aut == 0


def test_disjoint_union_additivity():
    rng = np.random.default_rng(2)
    g1 = W.er_pairs(40, 0.15, 1)
    g2 = W.er_pairs(35, 0.2, 2)
    g = W.disjoint_union(g1, g2)
    for pat in [W.path(4), W.cycle(4), W.pattern_B()]:
        k = pat.n
        c1 = colours(rng, g1.n, k)
        c2 = colours(rng, g2.n, k)
        tot = O.dp_count(g, pat, k, np.concatenate([c1, c2]))["count"]
        assert tot == O.dp_count(g1, pat, k, c1)["count"] + O.dp_count(g2, pat, k, c2)["count"]


def test_disconnected_pattern_split_over_colour_sets():
    """F = F1 + F2 (disjoint): count = sum over colour sets S of size n1 of
    count_S(F1) * count_{[k] \\ S}(F2), where count_S counts colourful copies
    using exactly the colours S (brute force per side)."""
    g = W.er_pairs(14, 0.35, 4)
    F1, F2 = W.path(2), W.path(3)
    F = W.Pattern(5, [(0, 1), (2, 3), (3, 4)])
    rng = np.random.default_rng(8)
    col = colours(rng, g.n, 5)
    by1 = {}
    for phi in B.all_mappings(g, F1, col):
        s = frozenset(int(col[v]) for v in phi)
        by1[s] = by1.get(s, 0) + 1
    by2 = {}
    for phi in B.all_mappings(g, F2, col):
        s = frozenset(int(col[v]) for v in phi)
        by2[s] = by2.get(s, 0) + 1
    full = frozenset(range(5))
    ref = sum(c * by2.get(full - s, 0) for s, c in by1.items())
    assert O.dp_count(g, F, 5, col)["count"] == ref


def test_per_root_vertex_split():
    g = W.er_pairs(40, 0.2, 6)
    rng = np.random.default_rng(4)
    for pat in [W.path(4), W.cycle(4), W.pattern_B()]:
        col = colours(rng, g.n, pat.n)
        r = O.dp_count(g, pat, pat.n, col, per_root_vertex=True)
        prv = r["per_root_vertex"]
        assert int(prv.sum()) == r["count"]
        for v in rng.choice(g.n, 6, replace=False):
            assert int(prv[v]) == O.brute_count(g, pat, col, fix0=int(v))


def _td_nodes(td):
    N = int(td[0])
    return [(int(td[1 + 5 * i]), int(td[2 + 5 * i]), int(td[3 + 5 * i]), int(td[4 + 5 * i]),
             int(td[5 + 5 * i]) & 0xFFFFFFFF) for i in range(N)]


def _definition_table_sizes(g, pat, k, col, td, degmask=True):
    """|D_x| of every node straight from the definition of D(x, phi, C)
    (Sec. 3.1): the number of distinct pairs (phi, C) such that some mapping
    Phi of V_x (the vertices of the bags below x) preserves the edges of F
    among V_x, gives V_x pairwise distinct colours, restricts to phi on the
    bag and has colour set C; with the degree mask (Sec. 3.2) every image
    also has deg_G >= deg_F.  Plain backtracking over all such Phi."""
    adj = B.adjacency(g)
    fadj = {u: set() for u in range(pat.n)}
    for a, b in pat.edges:
        fadj[a].add(b)
        fadj[b].add(a)
    nodes = _td_nodes(td)
    below = []
    for t, u, c0, c1, bag in nodes:
        s = bag
        for c in (c0, c1):
            if c >= 0:
                s |= below[c]
        below.append(s)
    sizes = []
    for i, (t, u, c0, c1, bag) in enumerate(nodes):
        vx = [w for w in range(pat.n) if below[i] >> w & 1]
        bagv = [w for w in range(pat.n) if bag >> w & 1]
        seen = set()
        phi = {}

        def rec(j, used):
            if j == len(vx):
                seen.add((tuple(phi[w] for w in bagv), used))
                return
            w = vx[j]
            for v in range(g.n):
                c = int(col[v])
                if used >> c & 1:
                    continue
                if degmask and len(adj[v]) < len(fadj[w]):
                    continue
                if any(x in phi and phi[x] not in adj[v] for x in fadj[w]):
                    continue
                phi[w] = v
                rec(j + 1, used | (1 << c))
                del phi[w]

        rec(0, 0)
        sizes.append(len(seen))
    return sizes


@pytest.mark.parametrize("pat", [W.path(4), W.cycle(4), W.cycle(5), W.star(4), W.grid(2, 2),
                                 W.Pattern(4, [(0, 1), (2, 3)], "2K2"),
                                 W.Pattern(5, [(0, 1), (1, 2), (0, 2), (2, 3), (3, 4)], "tri+tail")],
                         ids=lambda p: p.name)
def test_node_table_sizes_vs_definition(pat):
    """The oracle's per-node |D_x| (dp_count sizes=True) equals the number of
    (phi, C) pairs the definition of D(x, phi, C) admits, node by node, with
    and without the degree mask, with k = n_F and k = n_F + 1."""
    rng = np.random.default_rng(77)
    td, _ = O.build_td(pat)
    for g in zoo_graphs()[:4]:
        for k in (pat.n, pat.n + 1):
            col = colours(rng, g.n, k)
            for dm in (True, False):
                got = O.dp_count(g, pat, k, col, td=td, degmask=dm, sizes=True, distbound=False)["sizes"]
                assert list(got) == _definition_table_sizes(g, pat, k, col, td, degmask=dm)


@pytest.mark.parametrize("pat", [W.cycle(5), W.pattern_B(), W.path(4), W.partial_3tree(6, 1)], ids=lambda p: p.name)
def test_anchor_ranges_partition_the_count(pat):
    """Counting only mappings with Phi(0) in [lo, hi): single-vertex ranges
    equal the brute force with Phi(0) fixed (the definition), and any
    partition of V(G) into ranges adds up to the full count; tables of nodes
    without pattern vertex 0 in their bag do not depend on the range."""
    g = W.er_pairs(40, 0.2, 8)
    rng = np.random.default_rng(5)
    col = colours(rng, g.n, pat.n)
    full = O.dp_count(g, pat, pat.n, col, sizes=True)
    td, _ = O.build_td(pat)
    for v in range(0, g.n, 7):
        assert O.dp_count_range(g, pat, pat.n, col, v, v + 1)["count"] == O.brute_count(g, pat, col, fix0=v)
    cuts = [0, 3, 11, 12, 29, g.n]
    total = 0
    nodes = _td_nodes(td)
    for lo, hi in zip(cuts[:-1], cuts[1:]):
        r = O.dp_count_range(g, pat, pat.n, col, lo, hi, td=td, sizes=True)
        total += r["count"]
        for i, node in enumerate(nodes[:-1]):
            if not node[4] & 1:
                assert r["sizes"][i] == full["sizes"][i]
    assert total % U64 == full["count"]
    assert O.dp_count_range(g, pat, pat.n, col, 0, g.n)["count"] == full["count"]
    assert O.dp_count_range(g, pat, pat.n, col, 5, 5)["count"] == 0


def test_vertex_sets_closed_forms():
    """A host that is a disjoint union of induced copies of F: every copy is
    one vertex set and |Aut(F)| mappings; with fewer vertex-set-distinct
    colourings the sets are exactly the colourful copies (brute force)."""
    for pat, aut in ((W.cycle(3), 6), (W.path(4), 2), (W.star(4), 6), (W.cycle(5), 10)):
        copies = 4
        a = np.concatenate([np.array([e[0] for e in pat.edges]) + pat.n * c for c in range(copies)])
        b = np.concatenate([np.array([e[1] for e in pat.edges]) + pat.n * c for c in range(copies)])
        g = W.csr_from_edges(pat.n * copies, a, b)
        col = np.tile(np.arange(pat.n), copies).astype(np.uint8)  # every copy colourful
        sets = O.vertex_sets(g, pat, pat.n, col)
        assert len(sets) == copies
        assert O.dp_count(g, pat, pat.n, col)["count"] == copies * aut
        assert B.automorphisms(pat) == aut
    # general hosts: the sets of the brute-force mappings
    rng = np.random.default_rng(9)
    for g in zoo_graphs():
        for pat in (W.path(3), W.cycle(4), W.star(4), W.grid(2, 2)):
            col = colours(rng, g.n, pat.n)
            ref = sorted({tuple(sorted(m)) for m in B.all_mappings(g, pat, col)})
            assert O.vertex_sets(g, pat, pat.n, col) == ref


def test_repetition_count_and_search_finds_every_occurrence():
    """ceil(e^{n_F} ln(1/eps)) colourings; with eps tiny the union of the
    colourful mappings of all runs is every injective adjacency-preserving
    mapping of a tiny host (each is colourful in a run with probability
    >= n_F!/n_F^{n_F})."""
    import math

    assert O.repetitions(5, 1 / math.e) == math.ceil(math.exp(5))
    assert O.repetitions(3, 1e-9) == math.ceil(math.exp(3) * math.log(1e9))
    g = W.er_pairs(9, 0.45, 4)
    for pat in (W.path(3), W.cycle(3)):
        every = set()
        adj = B.adjacency(g)
        for phi in itertools.permutations(range(g.n), pat.n):
            if all(phi[b] in adj[phi[a]] for a, b in pat.edges):
                every.add(phi)
        rows, run = O.search(g, pat, 1e-9, 77, 10**6)
        assert run == O.repetitions(pat.n, 1e-9)
        assert set(rows) == every
        sets, _ = O.search(g, pat, 1e-9, 77, 10**6, distinct_sets=True)
        assert set(sets) == {tuple(sorted(r)) for r in every}
        few, run2 = O.search(g, pat, 1e-9, 77, 3)
        assert len(few) == 3 and run2 <= run and few == sorted(few)


@pytest.mark.parametrize("pat", [W.pattern_C(), W.pattern_D(), W.Pattern(6, [(0, 1), (1, 2), (3, 4), (4, 5), (2, 3)], "P6")],
                         ids=lambda p: p.name)
def test_distance_bound_keeps_counts(pat):
    """The distance bound of Sec. 3.2 only drops entries that cannot
    complete: with it on and off, counts, flags and enumerated rows agree
    (brute force) on every decomposition tried, while the tables of
    introduce nodes with no bag neighbour can only shrink."""
    rng = np.random.default_rng(31)
    tds = [O.build_td(pat)[0]]
    import paper_1908_11248_amd as cc

    try:
        tds.append(cc.build_decomposition(pat.n, pat.edges).export())
    except Exception:
        pass
    for g in (W.er_pairs(14, 0.3, 3), W.er_pairs(30, 0.15, 4), W.rgg(40, 6, 5)):
        col = colours(rng, g.n, pat.n)
        ref = O.brute_count(g, pat, col)
        for td in tds:
            on = O.dp_count(g, pat, pat.n, col, td=td, sizes=True)
            off = O.dp_count(g, pat, pat.n, col, td=td, sizes=True, distbound=False)
            assert on["count"] == off["count"] == ref
            assert (on["sizes"] <= off["sizes"]).all()
        rows, _ = O.dp_enumerate(g, pat, pat.n, col, 10**6)
        assert [tuple(r) for r in rows] == [tuple(r) for r in O.brute_enum(g, pat, col, 10**6)]
