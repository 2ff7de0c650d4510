"""Pure-Python brute force over all mappings -- TEST INFRASTRUCTURE ONLY.

The definition itself, for tiny inputs: a colourful copy of F in G is a
mapping Phi: V(F) -> V(G) that sends every edge of F to an edge of G (Sec. 1,
SubIso: an adjacency-preserving injective mapping) and gives the images
pairwise distinct colours (Sec. 2.1, colourful copy).  Automorphic images are
counted separately (the paper's default counting mode, Sec. 5.2).
"""
import itertools


def adjacency(g):
    adj = []
    for v in range(g.n):
        adj.append(set(int(x) for x in g.col[g.row_ptr[v]:g.row_ptr[v + 1]]))
    return adj


def all_mappings(g, pat, colors):
    """Every colourful mapping, in lexicographic order."""
    adj = adjacency(g)
    out = []
    for phi in itertools.product(range(g.n), repeat=pat.n):
        if len({int(colors[v]) for v in phi}) != pat.n:
            continue
        if all(phi[b] in adj[phi[a]] for a, b in pat.edges):
            out.append(phi)
    return out


def count(g, pat, colors):
    return len(all_mappings(g, pat, colors))


def injective_homomorphisms(g, pat):
    """Number of injective adjacency-preserving mappings (colours ignored)."""
    adj = adjacency(g)
    c = 0
    for phi in itertools.permutations(range(g.n), pat.n):
        if all(phi[b] in adj[phi[a]] for a, b in pat.edges):
            c += 1
    return c


def automorphisms(pat):
    """|Aut(F)| by trying every permutation of V(F)."""
    E = {frozenset(e) for e in pat.edges}
    c = 0
    for p in itertools.permutations(range(pat.n)):
        if all(frozenset((p[a], p[b])) in E for a, b in pat.edges):
            c += 1
    return c
