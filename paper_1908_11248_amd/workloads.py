"""Seeded synthetic workloads: host graphs G, pattern graphs F and query streams.

This module only draws inputs.  It holds none of the colour-coding method's
arithmetic (no colouring, no decomposition, no counting) and is shared by the
tests, the benchmark and the CPU oracle's callers.

Graphs are returned as ``Graph(n, row_ptr int64[n+1], col int32[2m])``: simple,
undirected (both directions stored), rows sorted ascending -- the input class
of the paper (Sec. 1.2: all graphs are undirected and simple).

The five standard workloads stand in for the paper's data sets (Images, Trans,
ICPR2014 and the Erdos-Renyi setup of Sec. 5), none of which ships here:
    1  ER G(200, 0.05), path P5, k = 5, one colouring, full enumeration
    2  ER n = 10 000, mean degree 8, uniform random labelled tree on 8 vertices,
       k = 8, 64 colourings
    3  2-D random geometric graph, n = 50 000, mean degree 10, ladder 2x4,
       k = 8, 32 colourings, enumeration capped at 10^6 rows per colouring
    4  Barabasi-Albert n = 200 000, m = 5; 256 queries of 5-10 vertices
       (random trees, cycles, partial 3-trees), 16 colourings each
    5  Chung-Lu n = 10^6, exponent 2.5, mean degree 10; a Poisson stream of
       queries drawn as in 4, 32 colourings each
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field
from typing import List, Tuple

import numpy as np

BASE_SEED = 0x190811248


@dataclass
class Graph:
    n: int
    row_ptr: np.ndarray
    col: np.ndarray
    name: str = ""

    @property
    def m(self) -> int:
        return int(self.col.size // 2)

    def degrees(self) -> np.ndarray:
        return np.diff(self.row_ptr)


@dataclass
class Pattern:
    n: int
    edges: List[Tuple[int, int]]
    name: str = ""
    family: str = ""

    def edge_array(self) -> np.ndarray:
        return np.asarray(self.edges, dtype=np.int32).reshape(-1, 2)


# ---------------------------------------------------------------------------
# CSR construction

def csr_from_edges(n: int, a: np.ndarray, b: np.ndarray, name: str = "") -> Graph:
    """Symmetric CSR with sorted rows; drops loops and duplicate edges."""
    a = np.asarray(a, dtype=np.int64)
    b = np.asarray(b, dtype=np.int64)
    keep = a != b
    a, b = a[keep], b[keep]
    lo = np.minimum(a, b)
    hi = np.maximum(a, b)
    key = np.unique(lo * n + hi)
    lo = key // n
    hi = key % n
    src = np.concatenate([lo, hi])
    dst = np.concatenate([hi, lo])
    order = np.lexsort((dst, src))
    src = src[order]
    dst = dst[order]
    counts = np.bincount(src, minlength=n)
    row_ptr = np.zeros(n + 1, dtype=np.int64)
    np.cumsum(counts, out=row_ptr[1:])
    return Graph(n, row_ptr, dst.astype(np.int32), name)


def disjoint_union(g1: Graph, g2: Graph) -> Graph:
    rp = np.concatenate([g1.row_ptr, g2.row_ptr[1:] + g1.row_ptr[-1]])
    col = np.concatenate([g1.col, g2.col + g1.n]).astype(np.int32)
    return Graph(g1.n + g2.n, rp, col, g1.name + "+" + g2.name)


def relabel(g: Graph, perm: np.ndarray) -> Graph:
    """Graph with vertex v renamed perm[v]."""
    src = np.repeat(np.arange(g.n, dtype=np.int64), np.diff(g.row_ptr))
    return csr_from_edges(g.n, perm[src], perm[g.col.astype(np.int64)], g.name + "~")


def edge_list(g: Graph) -> Tuple[np.ndarray, np.ndarray]:
    src = np.repeat(np.arange(g.n, dtype=np.int64), np.diff(g.row_ptr))
    dst = g.col.astype(np.int64)
    m = src < dst
    return src[m], dst[m]


# ---------------------------------------------------------------------------
# host graph models

def er_pairs(n: int, p: float, seed: int) -> Graph:
    """G(n, p): one Bernoulli(p) draw per pair i < j in lexicographic order."""
    rng = np.random.Generator(np.random.PCG64(seed))
    iu, ju = np.triu_indices(n, k=1)
    keep = rng.random(iu.size) < p
    return csr_from_edges(n, iu[keep], ju[keep], "ER(%d,%g)" % (n, p))


def er_skip(n: int, p: float, seed: int) -> Graph:
    """G(n, p) by geometric skipping over the lexicographic pair order."""
    rng = np.random.Generator(np.random.PCG64(seed))
    total = n * (n - 1) // 2
    pos = []
    cur = -1
    while True:
        need = int(max(1024, (total - cur) * p * 1.1 + 1024))
        skips = rng.geometric(p, size=need).astype(np.int64)
        cs = cur + np.cumsum(skips)
        pos.append(cs[cs < total])
        if cs[-1] >= total:
            break
        cur = int(cs[-1])
    t = np.concatenate(pos)
    # pair index t -> (i, j): row i starts at off(i) = i*n - i*(i+1)/2
    ii = np.arange(n, dtype=np.int64)
    off = ii * n - ii * (ii + 1) // 2
    i = np.searchsorted(off, t, side="right") - 1
    j = t - off[i] + i + 1
    return csr_from_edges(n, i, j, "ER(%d,%.3g)" % (n, p))


def rgg(n: int, mean_degree: float, seed: int) -> Graph:
    """2-D random geometric graph: n uniform points in the unit square (no
    torus), an edge for each pair closer than r = sqrt(d / (pi (n-1)))."""
    from scipy.spatial import cKDTree

    rng = np.random.Generator(np.random.PCG64(seed))
    pts = rng.random((n, 2))
    r = math.sqrt(mean_degree / (math.pi * (n - 1)))
    pairs = cKDTree(pts).query_pairs(r, output_type="ndarray")
    return csr_from_edges(n, pairs[:, 0], pairs[:, 1], "RGG(%d,%g)" % (n, mean_degree))


def barabasi_albert(n: int, m: int, seed: int) -> Graph:
    """Preferential attachment: start from K_{m+1}; every new vertex picks m
    distinct targets with probability proportional to degree (uniform draws
    from the list of edge endpoints, duplicates redrawn)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    m0 = m + 1
    ends = np.empty(2 * (m0 * (m0 - 1) // 2 + (n - m0) * m), dtype=np.int64)
    src_all = []
    dst_all = []
    ne = 0
    for i in range(m0):
        for j in range(i + 1, m0):
            src_all.append(i)
            dst_all.append(j)
            ends[ne] = i
            ends[ne + 1] = j
            ne += 2
    src = np.empty((n - m0) * m, dtype=np.int64)
    dst = np.empty((n - m0) * m, dtype=np.int64)
    w = 0
    buf = rng.integers(0, 1 << 62, size=1 << 16)
    bi = 0
    for v in range(m0, n):
        chosen = set()
        while len(chosen) < m:
            if bi == buf.size:
                buf = rng.integers(0, 1 << 62, size=1 << 16)
                bi = 0
            t = int(ends[buf[bi] % ne])
            bi += 1
            chosen.add(t)
        for t in sorted(chosen):
            src[w] = v
            dst[w] = t
            w += 1
            ends[ne] = v
            ends[ne + 1] = t
            ne += 2
    a = np.concatenate([np.asarray(src_all, dtype=np.int64), src[:w]])
    b = np.concatenate([np.asarray(dst_all, dtype=np.int64), dst[:w]])
    return csr_from_edges(n, a, b, "BA(%d,%d)" % (n, m))


def chung_lu_weights(n: int, beta: float, mean_degree: float) -> np.ndarray:
    """w_i = c (i + i0)^(-1/(beta-1)), c and i0 chosen so that the mean weight
    is mean_degree and the largest is sqrt(n * mean_degree) (structural
    cut-off, so w_i w_j / sum(w) <= 1)."""
    g = 1.0 / (beta - 1.0)
    wmax = math.sqrt(n * mean_degree)
    idx = np.arange(n, dtype=np.float64)

    def mean_for(i0):
        c = wmax * i0 ** g
        return float(np.mean(c * (idx + i0) ** (-g)))

    lo, hi = 1e-9, float(n) * 10
    for _ in range(200):
        mid = math.sqrt(lo * hi)
        if mean_for(mid) > mean_degree:
            hi = mid
        else:
            lo = mid
    i0 = math.sqrt(lo * hi)
    c = wmax * i0 ** g
    return c * (idx + i0) ** (-g)


def chung_lu(n: int, beta: float, mean_degree: float, seed: int) -> Graph:
    """Chung-Lu graph: edge {i, j} with probability min(1, w_i w_j / sum w),
    sampled in O(n + m) by geometric skipping over the weight-sorted partners
    of each vertex (all vertices advanced together, one skip per round)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    w = chung_lu_weights(n, beta, mean_degree)  # non-increasing
    S = float(w.sum())
    u = np.arange(n - 1, dtype=np.int64)
    v = u + 1
    p = np.minimum(w[u] * w[v] / S, 1.0)
    out_a = []
    out_b = []
    while u.size:
        r = rng.random(u.size)
        # skip r ~ Geometric(p) - 1 failures (p == 1: no skip)
        with np.errstate(divide="ignore", invalid="ignore"):
            skip = np.where(p >= 1.0, 0, np.floor(np.log(r) / np.log1p(-p)))
        skip = np.minimum(skip, n).astype(np.int64)
        v = v + skip
        alive = v < n
        u, v, p = u[alive], v[alive], p[alive]
        if not u.size:
            break
        q = np.minimum(w[u] * w[v] / S, 1.0)
        acc = rng.random(u.size) < q / p
        out_a.append(u[acc])
        out_b.append(v[acc])
        p = q
        v = v + 1
        alive = v < n
        u, v, p = u[alive], v[alive], p[alive]
    a = np.concatenate(out_a) if out_a else np.zeros(0, np.int64)
    b = np.concatenate(out_b) if out_b else np.zeros(0, np.int64)
    return csr_from_edges(n, a, b, "CL(%d,%g,%g)" % (n, beta, mean_degree))


# ---------------------------------------------------------------------------
# pattern graphs (the families of the paper's Table `prop` and Fig. `figpatt`)

def path(n: int) -> Pattern:
    return Pattern(n, [(i, i + 1) for i in range(n - 1)], "P%d" % n, "path")


def cycle(n: int) -> Pattern:
    return Pattern(n, [(i, (i + 1) % n) for i in range(n)], "C%d" % n, "cycle")


def star(n: int) -> Pattern:
    return Pattern(n, [(0, i) for i in range(1, n)], "S%d" % n, "star")


def complete(n: int) -> Pattern:
    return Pattern(n, [(i, j) for i in range(n) for j in range(i + 1, n)], "K%d" % n, "complete")


def grid(r: int, c: int) -> Pattern:
    e = []
    for i in range(r):
        for j in range(c):
            v = i * c + j
            if j + 1 < c:
                e.append((v, v + 1))
            if i + 1 < r:
                e.append((v, v + c))
    return Pattern(r * c, e, "G%d,%d" % (r, c), "grid")


def ladder(length: int = 4) -> Pattern:
    """2 x length ladder: top 0..L-1, bottom L..2L-1, rails and rungs."""
    L = length
    e = [(j, j + 1) for j in range(L - 1)] + [(L + j, L + j + 1) for j in range(L - 1)]
    e += [(j, L + j) for j in range(L)]
    return Pattern(2 * L, e, "L2x%d" % L, "ladder")


def pattern_A() -> Pattern:
    """Pattern A of Fig. `figpatt` (9 vertices, 8 edges, a tree)."""
    e = [(0, 1), (1, 2), (2, 3), (2, 4), (5, 4), (6, 4), (6, 7), (7, 8)]
    return Pattern(9, e, "A", "paper")


def pattern_B() -> Pattern:
    """Pattern B of Fig. `figpatt` (7 vertices, 7 edges, treewidth 2)."""
    e = [(0, 1), (1, 2), (0, 2), (1, 6), (1, 5), (2, 3), (3, 4)]
    return Pattern(7, e, "B", "paper")


def pattern_C() -> Pattern:
    """Pattern C of Fig. `figpatt` (9 vertices, 12 edges, treewidth 2)."""
    e = [(0, 3), (0, 4), (1, 3), (1, 5), (2, 4), (2, 5), (6, 1), (6, 2), (7, 0), (7, 2),
         (8, 0), (8, 1)]
    return Pattern(9, e, "C", "paper")


def pattern_D() -> Pattern:
    """Pattern D of Fig. `figpatt` (7 vertices, 6 edges, disconnected): an
    edge p1-p2 (ids 0, 1) and a 5-cycle on the figure's vertices 1..5 (ids 2..6)."""
    e = [(0, 1)] + [(1 + i, 2 + i) for i in range(1, 5)] + [(2, 6)]
    return Pattern(7, e, "D", "paper")


def random_tree(n: int, seed: int) -> Pattern:
    """Uniform labelled tree on n vertices from a uniform Pruefer sequence."""
    rng = np.random.Generator(np.random.PCG64(seed))
    if n == 1:
        return Pattern(1, [], "T1", "tree")
    if n == 2:
        return Pattern(2, [(0, 1)], "T2", "tree")
    seq = rng.integers(0, n, size=n - 2).tolist()
    degree = [1] * n
    for x in seq:
        degree[x] += 1
    edges = []
    for x in seq:
        for leaf in range(n):
            if degree[leaf] == 1:
                edges.append((min(leaf, x), max(leaf, x)))
                degree[leaf] -= 1
                degree[x] -= 1
                break
    rest = [v for v in range(n) if degree[v] == 1]
    edges.append((rest[0], rest[1]))
    return Pattern(n, sorted(edges), "T%d" % n, "tree")


def partial_3tree(n: int, seed: int) -> Pattern:
    """Random partial 3-tree: K4 on 0..3, every further vertex joined to a
    uniformly random triangle of the current 3-tree; then a BFS spanning tree
    from 0 is kept plus every other edge with probability 1/2.  Connected,
    treewidth <= 3."""
    assert n >= 4
    rng = np.random.Generator(np.random.PCG64(seed))
    edges = {(i, j) for i in range(4) for j in range(i + 1, 4)}
    tris = [(0, 1, 2), (0, 1, 3), (0, 2, 3), (1, 2, 3)]
    for v in range(4, n):
        a, b, c = tris[int(rng.integers(0, len(tris)))]
        for x in (a, b, c):
            edges.add((min(x, v), max(x, v)))
        tris += [(a, b, v), (a, c, v), (b, c, v)]
    adj = {v: set() for v in range(n)}
    for a, b in edges:
        adj[a].add(b)
        adj[b].add(a)
    seen = {0}
    order = [0]
    tree = set()
    for x in order:
        for y in sorted(adj[x]):
            if y not in seen:
                seen.add(y)
                order.append(y)
                tree.add((min(x, y), max(x, y)))
    keep = set(tree)
    for e in sorted(edges):
        if e not in tree and rng.random() < 0.5:
            keep.add(e)
    return Pattern(n, sorted(keep), "P3T%d" % n, "partial3tree")


def random_query(seed: int) -> Pattern:
    """A query of the batched/served workloads: size U{5..10}, family
    U{tree, cycle, partial 3-tree}."""
    rng = np.random.Generator(np.random.PCG64(seed))
    size = int(rng.integers(5, 11))
    fam = int(rng.integers(0, 3))
    sub = int(rng.integers(0, 1 << 62))
    if fam == 0:
        p = random_tree(size, sub)
    elif fam == 1:
        p = cycle(size)
    else:
        p = partial_3tree(size, sub)
    return p


def longest_induced_cycle(p: Pattern) -> int:
    """Length of the longest chordless (induced) cycle of F; 0 for a forest.
    Plain search over simple cycles (patterns have at most 16 vertices)."""
    adj = [set() for _ in range(p.n)]
    for a, b in p.edges:
        adj[a].add(b)
        adj[b].add(a)
    best = 0

    def grow(path, on):
        nonlocal best
        u = path[-1]
        for w in adj[u]:
            if w == path[0] and len(path) >= 3:
                L = len(path)
                if all(path[j] not in adj[path[i]] for i in range(L) for j in range(i + 2, L)
                       if not (i == 0 and j == L - 1)):
                    best = max(best, L)
            elif w > path[0] and w not in on:
                # a chord to an earlier path vertex (other than the previous
                # one) can never be removed: prune
                if any(w in adj[x] for x in path[1:-1]):
                    continue
                on.add(w)
                path.append(w)
                grow(path, on)
                path.pop()
                on.discard(w)

    for s in range(p.n):
        grow([s], {s})
    return best


# Work budget of the batched and served workloads: a query is redrawn when
# its pattern has a chordless cycle longer than this.  Such a cycle makes some
# DP table hold pairs of graph vertices joined by paths of about half its
# length with no edge between them to prune them, and on these heavy-tailed
# graphs the number of such pairs grows by the mean neighbour degree (about
# 30 on BA(200000, 5), 50 on CL(10^6, 2.5, 10)) per extra step.  Measured per
# colouring: C5 on BA(200000, 5) 4.4e8 entries in its largest table, C6
# 5.6e9; on CL(10^6) C5 3.7e9, and partial 3-trees with an induced 4-cycle
# above 4e8.  Everything else stays below about 5e8.
MAX_INDUCED_CYCLE = {4: 5, 5: 3}


def admissible(index: int, p: Pattern) -> bool:
    return longest_induced_cycle(p) <= MAX_INDUCED_CYCLE.get(index, 32)


def select_queries(index: int, count: int, fits=None, max_redraws: int = 200):
    """The query stream of a batched/served workload under the work budget.

    Query i starts from seed query_seeds(index, count)[i]; while the pattern
    is not admissible(index, .) (or fits(pattern, seed) is False, when a
    caller gives that extra test) the query is redrawn from seed + 1 (a fresh
    size and family draw).  Returns a list of (pattern, seed) and a dict of
    redraw counts keyed by (family, size) of the rejected draws."""
    out = []
    redraws = {}
    for s0 in query_seeds(index, count):
        s = s0
        for _ in range(max_redraws):
            p = random_query(s)
            if admissible(index, p) and (fits is None or fits(p, s)):
                break
            key = (p.family, p.n)
            redraws[key] = redraws.get(key, 0) + 1
            s += 1
        else:
            raise RuntimeError("no query within the budget after %d redraws" % max_redraws)
        out.append((p, s))
    return out, redraws


def colouring_seed(query_seed: int) -> int:
    """Seed of a query's colourings."""
    return query_seed ^ 0xC0


# ---------------------------------------------------------------------------
# the five standard workloads

@dataclass
class Workload:
    index: int
    name: str
    k: int
    colorings: int
    seed: int
    color_seed: int
    cap: int = 0  # enumeration cap per colouring; 0: no enumeration
    enumerate_all: bool = False
    extra: dict = field(default_factory=dict)


def workload(index: int) -> Workload:
    seed = BASE_SEED + index
    cseed = seed ^ 0xC0
    if index == 1:
        return Workload(1, "ER(200,0.05)/P5", 5, 1, seed, cseed, enumerate_all=True)
    if index == 2:
        return Workload(2, "ER(10000,d=8)/tree8", 8, 64, seed, cseed)
    if index == 3:
        return Workload(3, "RGG(50000,d=10)/ladder2x4", 8, 32, seed, cseed, cap=10**6)
    if index == 4:
        return Workload(4, "BA(200000,5)/256 queries", 0, 16, seed, cseed, extra={"queries": 256})
    if index == 5:
        return Workload(5, "CL(1e6,2.5,10)/stream", 0, 32, seed, cseed)
    raise ValueError(index)


def workload_graph(index: int) -> Graph:
    w = workload(index)
    if index == 1:
        return er_pairs(200, 0.05, w.seed)
    if index == 2:
        return er_skip(10000, 8.0 / 9999.0, w.seed)
    if index == 3:
        return rgg(50000, 10.0, w.seed)
    if index == 4:
        return barabasi_albert(200000, 5, w.seed)
    if index == 5:
        return chung_lu(1000000, 2.5, 10.0, w.seed)
    raise ValueError(index)


def workload_pattern(index: int) -> Pattern:
    w = workload(index)
    if index == 1:
        return path(5)
    if index == 2:
        return random_tree(8, w.seed ^ 0x7E)
    if index == 3:
        return ladder(4)
    raise ValueError("workload %d has a query stream, not one pattern" % index)


def query_seeds(index: int, count: int) -> List[int]:
    w = workload(index)
    rng = np.random.Generator(np.random.PCG64(w.seed ^ 0x51))
    return [int(x) for x in rng.integers(0, 1 << 62, size=count)]


# ---------------------------------------------------------------------------
# paper-shaped context workloads (Sec. 5.1, Sec. 5.4): synthetic stand-ins at
# the sizes the paper prints; no item of its data sets is reproduced

IMAGES_SIZE = (4838, 7067)    # Images: a segmented image's region graph (Sec. 5.1)
TRANS_SIZE = (45733, 44727)   # Trans: bank transfers (Sec. 5.1)


def images_standin(seed: int = BASE_SEED + 11) -> Graph:
    """Planar-like stand-in for Images: a 2-D random geometric graph on 4838
    points with the radius that gives 7067 edges in expectation."""
    n, m = IMAGES_SIZE
    g = rgg(n, 2.0 * m / n, seed)
    g.name = "RGG(4838,m~7067) [Images stand-in]"
    return g


def trans_standin(seed: int = BASE_SEED + 12) -> Graph:
    """Sparse heavy-tailed stand-in for Trans: Chung-Lu on 45733 vertices,
    exponent 2.5, mean degree 2 * 44727 / 45733."""
    n, m = TRANS_SIZE
    g = chung_lu(n, 2.5, 2.0 * m / n, seed)
    g.name = "CL(45733,2.5,m~44727) [Trans stand-in]"
    return g


def paper_patterns() -> List[Pattern]:
    """The pattern set of the paper's tables (Sec. 5.1, Table `prop`,
    Fig. `figpatt`): paths P5, P10, P15, star S5, cycles C5, C10, K4, the
    3 x 3 grid, and patterns A-D."""
    return [path(5), path(10), path(15), star(5), cycle(5), cycle(10), complete(4), grid(3, 3),
            pattern_A(), pattern_B(), pattern_C(), pattern_D()]


def er_sweep(p_target: float, p_pattern: float, seed: int):
    """One cell of the Erdos-Renyi setup of Sec. 5.4: target G(150, p_target),
    pattern G(10, p_pattern)."""
    g = er_pairs(150, p_target, seed)
    pg = er_pairs(10, p_pattern, seed ^ 0x5EED)
    src, dst = edge_list(pg)
    pat = Pattern(10, [(int(a), int(b)) for a, b in zip(src, dst)], "G(10,%.2f)" % p_pattern, "er")
    return g, pat
