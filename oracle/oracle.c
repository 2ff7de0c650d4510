/*
 * oracle.c -- TEST INFRASTRUCTURE ONLY.
 *
 * A plain, slow, single-threaded CPU implementation of what the colour-coding
 * dynamic program of Malik, Suchy and Valla ("Efficient Implementation of Color
 * Coding Algorithm for Subgraph Isomorphism Problem", arXiv 1908.11248)
 * computes.  It is written from the paper, shares no code, header, table or
 * helper with the HIP library, and only the test-suite, the package smoke
 * check and the benchmark's CPU-baseline leg may load it.
 *
 * Contents (each function names the passage it follows):
 *   - splitmix64 and the stateless random colouring                (Sec. 2.1)
 *   - brute force over mappings: the definition of a colourful copy (Sec. 1,
 *     Sec. 2.1 Definition of colourful copy)
 *   - exact-width tree decomposition from elimination orderings     (Sec. 3)
 *     and its conversion to the paper's nice tree decomposition     (Sec. 1.2)
 *   - validation of a nice tree decomposition                       (Sec. 1.2)
 *   - the dynamic program over a nice TD                            (Sec. 3.1)
 *     with counts instead of existence bits (see below)
 *   - result reconstruction R(x, M)                                 (Sec. 4)
 *
 * Counting reading.  The paper's table holds D(x, phi, C) in {0,1}.  Here an
 * entry holds the NUMBER of colourful partial isomorphisms the definition of
 * D(x, phi, C) quantifies over, taken modulo 2^64: leaves give 1, introduce
 * carries the child's number, forget adds the numbers of the merged entries,
 * join multiplies the two children's numbers of each admissible colour-set
 * pair and adds over pairs.  An entry exists exactly when the paper's
 * D(x, phi, C) = 1, whatever its residue mod 2^64.  A sticky per-run flag is
 * raised when any sum or product exceeds 2^64 - 1 (the true value of some
 * entry then does not fit).
 *
 * Colours are 0-based: colour c is bit (1u << c) of a colour set.
 *
 * Graph input: CSR with int64 row pointers and int32 column ids, rows sorted
 * ascending, simple and symmetric (Sec. 1.2: graphs are undirected and simple).
 *
 * Tree decompositions are passed as plain int32 arrays:
 *     td[0] = number of nodes N, then per node i (5 ints):
 *     type (0 leaf, 1 introduce, 2 forget, 3 join), vertex u (-1 for a join),
 *     child0, child1 (-1 if absent), bag as a uint32 bitmask.
 * Nodes are in post-order (children before parents); the last node is the root.
 */
#define _GNU_SOURCE
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define ORC_MAXF 32
enum { T_LEAF = 0, T_INTRO = 1, T_FORGET = 2, T_JOIN = 3 };

/* error codes returned by the entry points */
#define ORC_OK 0
#define ORC_EINVAL -1
#define ORC_ERANGE -2
#define ORC_ENOMEM -3

/* ------------------------------------------------------------------------ */
/* Random colouring (Sec. 2.1: a uniformly random colouring of V(G) with the
 * colours of the pattern).  The paper does not name a generator; the oracle
 * uses the published splitmix64 generator (Steele, Lea, Flood 2014; Vigna's
 * public-domain reference): output = mix(state + 0x9E3779B97F4A7C15) with the
 * "variant 13" finaliser.  The colour of vertex v in colouring b under seed s
 * is floor(k * hi32(splitmix64(s XOR (b * 2^32 + v))) / 2^32).                */
uint64_t orc_splitmix64(uint64_t state) {
    uint64_t z = state + 0x9E3779B97F4A7C15ULL;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
    return z ^ (z >> 31);
}

int orc_color_of(uint64_t seed, int64_t b, int64_t v, int32_t k) {
    uint64_t h = orc_splitmix64(seed ^ (((uint64_t)b << 32) + (uint64_t)v));
    return (int)(((h >> 32) * (uint64_t)k) >> 32);
}

void orc_color_array(uint64_t seed, int64_t b, int32_t n, int32_t k, uint8_t *out) {
    for (int32_t v = 0; v < n; v++) out[v] = (uint8_t)orc_color_of(seed, b, v, k);
}

/* ------------------------------------------------------------------------ */
/* graph helpers                                                             */
typedef struct {
    int32_t n;
    const int64_t *rp;
    const int32_t *col;
} graph_t;

static int64_t gdeg(const graph_t *g, int32_t v) { return g->rp[v + 1] - g->rp[v]; }

/* {a, b} in E(G)?  Linear scan of a's row: plain on purpose. */
static int has_edge(const graph_t *g, int32_t a, int32_t b) {
    for (int64_t e = g->rp[a]; e < g->rp[a + 1]; e++)
        if (g->col[e] == b) return 1;
    return 0;
}

typedef struct {
    int32_t n;
    uint32_t adj[ORC_MAXF]; /* adj[u] = bitmask of N_F(u) */
} pattern_t;

static int popc(uint32_t x) { return __builtin_popcount(x); }

static int load_pattern(pattern_t *F, int32_t nF, int32_t mF, const int32_t *edges) {
    if (nF < 1 || nF > ORC_MAXF || mF < 0) return ORC_EINVAL;
    F->n = nF;
    memset(F->adj, 0, sizeof F->adj);
    for (int32_t i = 0; i < mF; i++) {
        int32_t a = edges[2 * i], b = edges[2 * i + 1];
        if (a < 0 || b < 0 || a >= nF || b >= nF || a == b) return ORC_EINVAL;
        F->adj[a] |= 1u << b;
        F->adj[b] |= 1u << a;
    }
    return ORC_OK;
}

/* ------------------------------------------------------------------------ */
/* Brute force: the definition.  Counts the mappings Phi: V(F) -> V(G) that
 * preserve adjacency (Sec. 1, SubIso) and whose images carry pairwise
 * distinct colours (Sec. 2.1, colourful copy); distinct colours force Phi to
 * be injective.  Pattern vertices are mapped in id order and candidates are
 * tried in ascending vertex order, so mappings are produced in lexicographic
 * order of (Phi(0), ..., Phi(nF-1)).                                         */
typedef struct {
    const graph_t *g;
    const pattern_t *F;
    const uint8_t *col;
    int32_t phi[ORC_MAXF];
    uint32_t used; /* colours used so far */
    uint64_t count;
    uint64_t cap;  /* stop after this many mappings (enumeration) */
    int32_t *rows; /* optional output */
    int stop;
} brute_t;

static void brute_rec(brute_t *s, int i) {
    if (s->stop) return;
    const pattern_t *F = s->F;
    if (i == F->n) {
        if (s->rows) memcpy(s->rows + (size_t)s->count * F->n, s->phi, sizeof(int32_t) * F->n);
        s->count++;
        if (s->count >= s->cap) s->stop = 1;
        return;
    }
    uint32_t earlier = F->adj[i] & ((1u << i) - 1u);
    if (i == 0 && s->phi[0] >= 0) { /* image of vertex 0 fixed by the caller */
        int32_t v = s->phi[0];
        uint32_t cb = 1u << s->col[v];
        s->used |= cb;
        brute_rec(s, 1);
        s->used &= ~cb;
        return;
    }
    int64_t lo, hi;
    const int32_t *cand = NULL;
    if (earlier) {
        int j = __builtin_ctz(earlier);
        int32_t w = s->phi[j];
        lo = s->g->rp[w];
        hi = s->g->rp[w + 1];
        cand = s->g->col;
    } else {
        lo = 0;
        hi = s->g->n;
    }
    for (int64_t t = lo; t < hi && !s->stop; t++) {
        int32_t v = cand ? cand[t] : (int32_t)t;
        uint32_t cb = 1u << s->col[v];
        if (s->used & cb) continue;
        int ok = 1;
        for (uint32_t m = earlier; m && ok; m &= m - 1) {
            int j = __builtin_ctz(m);
            if (!has_edge(s->g, s->phi[j], v)) ok = 0;
        }
        if (!ok) continue;
        s->phi[i] = v;
        s->used |= cb;
        brute_rec(s, i + 1);
        s->used &= ~cb;
    }
    s->phi[i] = -1;
}

/* Number of colourful mappings (fix0 >= 0 restricts Phi(0) = fix0). */
int orc_brute_count(int32_t n, const int64_t *rp, const int32_t *colidx, int32_t nF,
                    int32_t mF, const int32_t *edges, const uint8_t *colors, int32_t fix0,
                    uint64_t *count) {
    graph_t g = {n, rp, colidx};
    pattern_t F;
    int rc = load_pattern(&F, nF, mF, edges);
    if (rc) return rc;
    if (fix0 >= n) return ORC_EINVAL;
    brute_t s;
    memset(&s, 0, sizeof s);
    s.g = &g;
    s.F = &F;
    s.col = colors;
    s.cap = UINT64_MAX;
    for (int i = 0; i < ORC_MAXF; i++) s.phi[i] = -1;
    s.phi[0] = fix0;
    brute_rec(&s, 0);
    *count = s.count;
    return ORC_OK;
}

/* The lexicographically first min(count, cap) colourful mappings. */
int orc_brute_enum(int32_t n, const int64_t *rp, const int32_t *colidx, int32_t nF,
                   int32_t mF, const int32_t *edges, const uint8_t *colors, uint64_t cap,
                   int32_t *rows, uint64_t *n_rows) {
    graph_t g = {n, rp, colidx};
    pattern_t F;
    int rc = load_pattern(&F, nF, mF, edges);
    if (rc) return rc;
    brute_t s;
    memset(&s, 0, sizeof s);
    s.g = &g;
    s.F = &F;
    s.col = colors;
    s.cap = cap;
    s.rows = rows;
    for (int i = 0; i < ORC_MAXF; i++) s.phi[i] = -1;
    if (cap > 0) brute_rec(&s, 0);
    *n_rows = s.count;
    return ORC_OK;
}

/* ------------------------------------------------------------------------ */
/* Exact tree decomposition (Sec. 3: minimum width via triangulations and
 * elimination orderings, O(nF^2 2^nF)).  Written from the recurrence over
 * vertex subsets: with Q(S, v) = the vertices outside S u {v} reachable from v
 * by a path whose inner vertices all lie in S (v's neighbourhood in the filled
 * graph when the vertices of S are eliminated before v),
 *     TW(empty) = -1,  TW(S) = min_{v in S} max(TW(S \ {v}), |Q(S \ {v}, v)|).
 * Vertex 0 is eliminated last (the treewidth is unchanged: a chordal
 * completion has a perfect elimination ordering ending in any vertex), so the
 * root bag of its component is {0}.                                          */
static uint32_t q_set(const pattern_t *F, uint32_t S, int v) {
    uint32_t seen = 1u << v, frontier = 1u << v, out = 0;
    while (frontier) {
        int x = __builtin_ctz(frontier);
        frontier &= frontier - 1;
        uint32_t nb = F->adj[x] & ~seen;
        seen |= nb;
        out |= nb & ~S;
        frontier |= nb & S;
    }
    return out;
}

#define MAX_TD_NODES 4096
typedef struct {
    int n;
    int type[MAX_TD_NODES], u[MAX_TD_NODES], c0[MAX_TD_NODES], c1[MAX_TD_NODES];
    uint32_t bag[MAX_TD_NODES];
} nice_t;

static int add_node(nice_t *t, int type, int u, int c0, int c1, uint32_t bag) {
    if (t->n >= MAX_TD_NODES) return -1;
    int i = t->n++;
    t->type[i] = type;
    t->u[i] = u;
    t->c0[i] = c0;
    t->c1[i] = c1;
    t->bag[i] = bag;
    return i;
}

/* Introduce the vertices of `want` on top of node `top` (bag `have`), each
 * time preferring a vertex with a neighbour already in the bag. */
static int grow_to(nice_t *t, const pattern_t *F, int top, uint32_t have, uint32_t want) {
    uint32_t todo = want & ~have;
    while (todo) {
        int pick = -1;
        for (uint32_t m = todo; m; m &= m - 1) {
            int v = __builtin_ctz(m);
            if (F->adj[v] & have) { pick = v; break; }
        }
        if (pick < 0) pick = __builtin_ctz(todo);
        have |= 1u << pick;
        todo &= ~(1u << pick);
        top = add_node(t, T_INTRO, pick, top, -1, have);
        if (top < 0) return -1;
    }
    return top;
}

/* Builds the nice TD (Sec. 1.2 definition) below elimination-tree node v. */
static int nice_below(nice_t *t, const pattern_t *F, int v, const uint32_t *bag,
                      const int *parent, int nF) {
    int branches[ORC_MAXF], nb = 0;
    for (int c = 0; c < nF; c++) {
        if (c == v || parent[c] != v) continue;
        int top = nice_below(t, F, c, bag, parent, nF);
        if (top < 0) return -1;
        uint32_t have = bag[c];
        for (uint32_t m = have & ~bag[v]; m; m &= m - 1) { /* forget what v's bag lacks */
            int x = __builtin_ctz(m);
            have &= ~(1u << x);
            top = add_node(t, T_FORGET, x, top, -1, have);
            if (top < 0) return -1;
        }
        top = grow_to(t, F, top, have, bag[v]);
        if (top < 0) return -1;
        branches[nb++] = top;
    }
    if (nb == 0) {
        int top = add_node(t, T_LEAF, v, -1, -1, 1u << v);
        if (top < 0) return -1;
        return grow_to(t, F, top, 1u << v, bag[v]);
    }
    int top = branches[0];
    for (int i = 1; i < nb; i++) {
        top = add_node(t, T_JOIN, -1, top, branches[i], bag[v]);
        if (top < 0) return -1;
    }
    return top;
}

static int build_nice(const pattern_t *F, nice_t *t, int *width_out) {
    int nF = F->n;
    if (nF > 20) return ORC_ERANGE;
    uint32_t full = (nF == 32) ? 0xFFFFFFFFu : ((1u << nF) - 1u);
    uint32_t rest = full & ~1u; /* vertex 0 is eliminated last */
    size_t ns = (size_t)1 << nF;
    int8_t *tw = malloc(ns);
    int8_t *last = malloc(ns);
    if (!tw || !last) { free(tw); free(last); return ORC_ENOMEM; }
    for (size_t S = 0; S < ns; S++) { tw[S] = 127; last[S] = -1; }
    tw[0] = -1;
    /* subsets in increasing integer order: S \ {v} < S */
    for (size_t S = 1; S < ns; S++) {
        if (S & ~(size_t)rest) continue;
        for (uint32_t m = (uint32_t)S; m; m &= m - 1) {
            int v = __builtin_ctz(m);
            uint32_t Sv = (uint32_t)S & ~(1u << v);
            int q = popc(q_set(F, Sv, v));
            int w = tw[Sv] > q ? tw[Sv] : q;
            if (w < tw[S]) { tw[S] = (int8_t)w; last[S] = (int8_t)v; }
        }
    }
    int order[ORC_MAXF];
    uint32_t S = rest;
    for (int i = nF - 2; i >= 0; i--) {
        order[i] = last[S];
        S &= ~(1u << order[i]);
    }
    order[nF - 1] = 0;
    int width = tw[rest];
    int q0 = popc(q_set(F, rest, 0));
    if (q0 > width) width = q0;
    free(tw);
    free(last);
    /* bags of the elimination tree: bag(v) = {v} u Q(earlier, v); parent is
     * the earliest-eliminated vertex of Q(earlier, v). */
    uint32_t bag[ORC_MAXF];
    int parent[ORC_MAXF], pos[ORC_MAXF];
    for (int i = 0; i < nF; i++) pos[order[i]] = i;
    uint32_t earlier = 0;
    for (int i = 0; i < nF; i++) {
        int v = order[i];
        uint32_t q = q_set(F, earlier, v);
        bag[v] = q | (1u << v);
        parent[v] = -1;
        int best = nF;
        for (uint32_t m = q; m; m &= m - 1) {
            int w = __builtin_ctz(m);
            if (pos[w] < best) { best = pos[w]; parent[v] = w; }
        }
        earlier |= 1u << v;
    }
    /* roots of other components hang below vertex 0's node (their branch is
     * forgotten to the empty bag, then 0 is introduced with no neighbour) */
    for (int v = 1; v < nF; v++)
        if (parent[v] < 0) parent[v] = 0;
    t->n = 0;
    int top = nice_below(t, F, 0, bag, parent, nF);
    if (top < 0) return ORC_ERANGE;
    /* forget down to the empty root, vertex 0 last */
    uint32_t have = t->bag[top];
    for (uint32_t m = have & ~1u; m; m &= m - 1) {
        int x = __builtin_ctz(m);
        have &= ~(1u << x);
        top = add_node(t, T_FORGET, x, top, -1, have);
        if (top < 0) return ORC_ERANGE;
    }
    top = add_node(t, T_FORGET, 0, top, -1, 0);
    if (top < 0) return ORC_ERANGE;
    *width_out = width;
    return ORC_OK;
}

int orc_build_td(int32_t nF, int32_t mF, const int32_t *edges, int32_t *td, int32_t cap,
                 int32_t *len, int32_t *width) {
    pattern_t F;
    int rc = load_pattern(&F, nF, mF, edges);
    if (rc) return rc;
    nice_t *t = malloc(sizeof(nice_t));
    if (!t) return ORC_ENOMEM;
    int w = 0;
    rc = build_nice(&F, t, &w);
    if (rc) { free(t); return rc; }
    if (cap < 1 + 5 * t->n) { free(t); return ORC_ERANGE; }
    td[0] = t->n;
    for (int i = 0; i < t->n; i++) {
        td[1 + 5 * i + 0] = t->type[i];
        td[1 + 5 * i + 1] = t->u[i];
        td[1 + 5 * i + 2] = t->c0[i];
        td[1 + 5 * i + 3] = t->c1[i];
        td[1 + 5 * i + 4] = (int32_t)t->bag[i];
    }
    *len = 1 + 5 * t->n;
    *width = w;
    free(t);
    return ORC_OK;
}

/* The exact treewidth alone (same recurrence, over all of V(F)). */
int orc_treewidth(int32_t nF, int32_t mF, const int32_t *edges, int32_t *width) {
    pattern_t F;
    int rc = load_pattern(&F, nF, mF, edges);
    if (rc) return rc;
    if (nF > 20) return ORC_ERANGE;
    size_t ns = (size_t)1 << nF;
    int8_t *tw = malloc(ns);
    if (!tw) return ORC_ENOMEM;
    tw[0] = -1;
    for (size_t S = 1; S < ns; S++) {
        int best = 127;
        for (uint32_t m = (uint32_t)S; m; m &= m - 1) {
            int v = __builtin_ctz(m);
            uint32_t Sv = (uint32_t)S & ~(1u << v);
            int q = popc(q_set(&F, Sv, v));
            int w = tw[Sv] > q ? tw[Sv] : q;
            if (w < best) best = w;
        }
        tw[S] = (int8_t)best;
    }
    *width = tw[ns - 1];
    free(tw);
    return ORC_OK;
}

/* ------------------------------------------------------------------------ */
/* Validation of a nice tree decomposition: conditions (i)-(iii) of the tree
 * decomposition definition and the four node types, empty root of degree 1
 * (Sec. 1.2).  Returns 0 when valid, a positive code naming the failed rule. */
int orc_validate_td(int32_t nF, int32_t mF, const int32_t *edges, const int32_t *td,
                    int32_t len) {
    pattern_t F;
    if (load_pattern(&F, nF, mF, edges)) return 1;
    if (len < 1) return 2;
    int N = td[0];
    if (N < 1 || len != 1 + 5 * N) return 2;
    int *nparents = calloc(N, sizeof(int));
    if (!nparents) return 99;
    int bad = 0;
    uint32_t full = (nF == 32) ? 0xFFFFFFFFu : ((1u << nF) - 1u);
    uint32_t covered = 0;
    for (int i = 0; i < N && !bad; i++) {
        int type = td[1 + 5 * i], u = td[2 + 5 * i], c0 = td[3 + 5 * i], c1 = td[4 + 5 * i];
        uint32_t bag = (uint32_t)td[5 + 5 * i];
        if (bag & ~full) { bad = 3; break; }
        covered |= bag;
        int nch = (c0 >= 0) + (c1 >= 0);
        if ((c0 >= i) || (c1 >= i)) { bad = 4; break; } /* post-order */
        if (c0 >= 0) nparents[c0]++;
        if (c1 >= 0) nparents[c1]++;
        uint32_t b0 = c0 >= 0 ? (uint32_t)td[5 + 5 * c0] : 0;
        uint32_t b1 = c1 >= 0 ? (uint32_t)td[5 + 5 * c1] : 0;
        switch (type) {
        case T_LEAF:
            if (nch != 0 || u < 0 || u >= nF || bag != (1u << u)) bad = 5;
            break;
        case T_INTRO:
            if (nch != 1 || c0 < 0 || u < 0 || u >= nF || (b0 & (1u << u)) ||
                bag != (b0 | (1u << u)))
                bad = 6;
            break;
        case T_FORGET:
            if (nch != 1 || c0 < 0 || u < 0 || u >= nF || !(b0 & (1u << u)) ||
                bag != (b0 & ~(1u << u)))
                bad = 7;
            break;
        case T_JOIN:
            if (nch != 2 || bag != b0 || bag != b1) bad = 8;
            break;
        default:
            bad = 9;
        }
    }
    if (!bad) {
        for (int i = 0; i < N - 1; i++)
            if (nparents[i] != 1) { bad = 10; break; }
        if (!bad && nparents[N - 1] != 0) bad = 10;
    }
    if (!bad) {
        int rt = N - 1;
        int rc0 = td[3 + 5 * rt], rc1 = td[4 + 5 * rt];
        if (td[5 + 5 * rt] != 0 || rc0 < 0 || rc1 >= 0) bad = 11; /* empty root, degree 1 */
    }
    if (!bad && covered != full) bad = 12; /* (i) */
    if (!bad) { /* (ii) every edge inside some bag */
        for (int a = 0; a < nF && !bad; a++)
            for (uint32_t m = F.adj[a]; m; m &= m - 1) {
                int b = __builtin_ctz(m);
                int found = 0;
                for (int i = 0; i < N && !found; i++) {
                    uint32_t bag = (uint32_t)td[5 + 5 * i];
                    if ((bag >> a & 1) && (bag >> b & 1)) found = 1;
                }
                if (!found) { bad = 13; break; }
            }
    }
    if (!bad) { /* (iii) the nodes holding u form a connected subtree: exactly
                   one of them has a parent that does not hold u */
        int *par = malloc(sizeof(int) * N);
        for (int i = 0; i < N; i++) par[i] = -1;
        for (int i = 0; i < N; i++) {
            int c0 = td[3 + 5 * i], c1 = td[4 + 5 * i];
            if (c0 >= 0) par[c0] = i;
            if (c1 >= 0) par[c1] = i;
        }
        for (int u = 0; u < nF && !bad; u++) {
            int tops = 0;
            for (int i = 0; i < N; i++) {
                uint32_t bag = (uint32_t)td[5 + 5 * i];
                if (!(bag >> u & 1)) continue;
                if (par[i] < 0 || !((uint32_t)td[5 + 5 * par[i]] >> u & 1)) tops++;
            }
            if (tops != 1) bad = 14;
        }
        free(par);
    }
    free(nparents);
    return bad;
}

/* ------------------------------------------------------------------------ */
/* DP tables (Sec. 3.1 "Initial Algorithm Modification": one list D_x of the
 * nonzero configurations per node).  A mapping phi: V_x -> V(G) is the tuple
 * of images of the bag in ascending vertex-id order (the fixed bag order of
 * Sec. 3.2 "Representation of Mappings").                                    */
typedef struct {
    int b;
    int32_t bagv[ORC_MAXF];
    size_t n, cap;
    int32_t *phi; /* n * b */
    uint32_t *C;
    uint64_t *cnt;
} table_t;

static void tab_init(table_t *t, uint32_t bag) {
    memset(t, 0, sizeof *t);
    for (int v = 0; v < ORC_MAXF; v++)
        if (bag >> v & 1) t->bagv[t->b++] = v;
}

static void tab_free(table_t *t) {
    free(t->phi);
    free(t->C);
    free(t->cnt);
    t->phi = NULL;
    t->C = NULL;
    t->cnt = NULL;
    t->n = t->cap = 0;
}

static int tab_push(table_t *t, const int32_t *phi, uint32_t C, uint64_t cnt) {
    if (t->n == t->cap) {
        size_t nc = t->cap ? 2 * t->cap : 1024;
        int32_t *p = realloc(t->phi, sizeof(int32_t) * (t->b ? t->b : 1) * nc);
        uint32_t *c = realloc(t->C, sizeof(uint32_t) * nc);
        uint64_t *k = realloc(t->cnt, sizeof(uint64_t) * nc);
        if (p) t->phi = p;
        if (c) t->C = c;
        if (k) t->cnt = k;
        if (!p || !c || !k) return ORC_ENOMEM;
        t->cap = nc;
    }
    if (t->b) memcpy(t->phi + t->n * t->b, phi, sizeof(int32_t) * t->b);
    t->C[t->n] = C;
    t->cnt[t->n] = cnt;
    t->n++;
    return ORC_OK;
}

static int bag_pos(const table_t *t, int v) {
    for (int i = 0; i < t->b; i++)
        if (t->bagv[i] == v) return i;
    return -1;
}

/* sort by (phi, C) and add the counts of equal keys (mod 2^64). */
static _Thread_local const table_t *g_sort_tab; /* qsort context, one per thread */
static int cmp_entry(const void *pa, const void *pb) {
    size_t a = *(const size_t *)pa, b = *(const size_t *)pb;
    const table_t *t = g_sort_tab;
    for (int i = 0; i < t->b; i++) {
        int32_t x = t->phi[a * t->b + i], y = t->phi[b * t->b + i];
        if (x != y) return x < y ? -1 : 1;
    }
    if (t->C[a] != t->C[b]) return t->C[a] < t->C[b] ? -1 : 1;
    return 0;
}

static int sort_and_merge(table_t *t, int *ovf) {
    if (t->n == 0) return ORC_OK;
    size_t *idx = malloc(sizeof(size_t) * t->n);
    if (!idx) return ORC_ENOMEM;
    for (size_t i = 0; i < t->n; i++) idx[i] = i;
    g_sort_tab = t;
    qsort(idx, t->n, sizeof(size_t), cmp_entry);
    table_t o;
    tab_init(&o, 0);
    o.b = t->b;
    memcpy(o.bagv, t->bagv, sizeof o.bagv);
    for (size_t i = 0; i < t->n; i++) {
        size_t e = idx[i];
        if (o.n > 0) {
            size_t l = o.n - 1;
            int same = (o.C[l] == t->C[e]);
            for (int j = 0; j < t->b && same; j++)
                if (o.phi[l * t->b + j] != t->phi[e * t->b + j]) same = 0;
            if (same) {
                uint64_t s;
                if (__builtin_add_overflow(o.cnt[l], t->cnt[e], &s)) *ovf = 1;
                o.cnt[l] = s;
                continue;
            }
        }
        if (tab_push(&o, t->phi + e * t->b, t->C[e], t->cnt[e])) {
            free(idx);
            tab_free(&o);
            return ORC_ENOMEM;
        }
    }
    free(idx);
    tab_free(t);
    *t = o;
    return ORC_OK;
}

/* Options of a DP run (the `degmask` argument of the entry points):
 * bit 0: degree mask on (Sec. 3.2 "Masking Unprofitable Mappings");
 * bit 1: distance bound OFF (Sec. 3.2, last paragraphs of "Mapping Expansion
 * Optimizations": by default an introduced vertex with no bag neighbour only
 * takes images within distance dist_F(w, u) of phi(w) for the bag vertex w
 * nearest to u in F). */
#define ORC_DEGMASK 1
#define ORC_NO_DISTBOUND 2

typedef struct {
    const graph_t *g;
    const pattern_t *F;
    const uint8_t *col;
    int degmask;
    int ovf;
    int32_t lo0, hi0; /* images allowed for pattern vertex 0: [lo0, hi0) */
    int distbound;
} dpctx_t;

/* deg_G(v) >= deg_F(u) (Sec. 3.2 "Masking Unprofitable Mappings"), and for
 * pattern vertex 0 an image inside the requested range.  Restricting the
 * image of one pattern vertex keeps exactly the mappings with Phi(0) in the
 * range, so counts over disjoint ranges add up to the full count. */
static int deg_ok(const dpctx_t *c, int u, int32_t v) {
    if (u == 0 && (v < c->lo0 || v >= c->hi0)) return 0;
    return !(c->degmask & ORC_DEGMASK) || gdeg(c->g, v) >= popc(c->F->adj[u]);
}

/* distances in F from u (-1: another component) */
static void pattern_dist(const pattern_t *F, int u, int *dist) {
    int queue[ORC_MAXF], qh = 0, qt = 0;
    for (int v = 0; v < F->n; v++) dist[v] = -1;
    dist[u] = 0;
    queue[qt++] = u;
    while (qh < qt) {
        int x = queue[qh++];
        for (int y = 0; y < F->n; y++)
            if ((F->adj[x] >> y & 1) && dist[y] < 0) {
                dist[y] = dist[x] + 1;
                queue[qt++] = y;
            }
    }
}

/* The vertices of G within distance r of a, ascending (plain BFS; *out is
 * malloc'ed, *cnt its length). */
static int ball(const graph_t *g, int32_t a, int r, int32_t **out, int64_t *cnt) {
    int32_t *dist = malloc(sizeof(int32_t) * (size_t)g->n);
    int32_t *q = malloc(sizeof(int32_t) * (size_t)g->n);
    if (!dist || !q) {
        free(dist);
        free(q);
        return ORC_ENOMEM;
    }
    for (int32_t v = 0; v < g->n; v++) dist[v] = -1;
    int64_t qh = 0, qt = 0;
    dist[a] = 0;
    q[qt++] = a;
    while (qh < qt) {
        int32_t x = q[qh++];
        if (dist[x] == r) continue;
        for (int64_t e = g->rp[x]; e < g->rp[x + 1]; e++)
            if (dist[g->col[e]] < 0) {
                dist[g->col[e]] = dist[x] + 1;
                q[qt++] = g->col[e];
            }
    }
    int64_t m = 0;
    for (int32_t v = 0; v < g->n; v++)
        if (dist[v] >= 0) q[m++] = v;
    free(dist);
    *out = q;
    *cnt = m;
    return ORC_OK;
}

/* Leaf: u mapped to every vertex of G, colour set {zeta(v)} (Sec. 3.1). */
static int dp_leaf(dpctx_t *c, int u, table_t *out) {
    for (int32_t v = 0; v < c->g->n; v++) {
        if (!deg_ok(c, u, v)) continue;
        if (tab_push(out, &v, 1u << c->col[v], 1)) return ORC_ENOMEM;
    }
    return ORC_OK;
}

/* Introduce u over child y (Sec. 3.1): extend each (phi', C') by u -> v when
 * zeta(v) is not in C' and every edge {u, w} of F inside the bag is realised
 * by an edge {v, phi'(w)} of G.  Candidates come from the adjacency list of
 * the image of one bag neighbour of u; with no bag neighbour every vertex of
 * G is a candidate (Sec. 3.2 "Mapping Expansion Optimizations").            */
static int dp_intro(dpctx_t *c, int u, const table_t *y, table_t *out) {
    int pu = bag_pos(out, u);
    uint32_t nb_in_bag = 0; /* bag neighbours of u, as positions in y */
    int npos[ORC_MAXF], nn = 0;
    for (int i = 0; i < y->b; i++)
        if (c->F->adj[u] >> y->bagv[i] & 1) { npos[nn++] = i; nb_in_bag |= 1u << i; }
    /* no bag neighbour: the bag vertex nearest to u in F (smallest id on a
     * tie) bounds the candidates by its distance */
    int near = -1, rad = 0;
    if (!nn && c->distbound) {
        int dist[ORC_MAXF];
        pattern_dist(c->F, u, dist);
        for (int i = 0; i < y->b; i++) {
            int d = dist[y->bagv[i]];
            if (d > 0 && (near < 0 || d < rad)) {
                near = i;
                rad = d;
            }
        }
    }
    int32_t phi[ORC_MAXF];
    for (size_t e = 0; e < y->n; e++) {
        const int32_t *pp = y->phi + e * y->b;
        int64_t lo = 0, hi = c->g->n;
        const int32_t *cand = NULL;
        int32_t *ballv = NULL;
        if (nn) {
            int32_t w = pp[npos[0]];
            lo = c->g->rp[w];
            hi = c->g->rp[w + 1];
            cand = c->g->col;
        } else if (near >= 0) {
            int64_t m;
            if (ball(c->g, pp[near], rad, &ballv, &m)) return ORC_ENOMEM;
            lo = 0;
            hi = m;
            cand = ballv;
        }
        for (int64_t t = lo; t < hi; t++) {
            int32_t v = cand ? cand[t] : (int32_t)t;
            uint32_t cb = 1u << c->col[v];
            if (y->C[e] & cb) continue;
            int ok = deg_ok(c, u, v);
            for (int j = 0; j < nn && ok; j++)
                if (!has_edge(c->g, pp[npos[j]], v)) ok = 0;
            if (!ok) continue;
            for (int i = 0, k = 0; i < out->b; i++) phi[i] = (i == pu) ? v : pp[k++];
            if (tab_push(out, phi, y->C[e] | cb, y->cnt[e])) {
                free(ballv);
                return ORC_ENOMEM;
            }
        }
        free(ballv);
    }
    return ORC_OK;
}

/* Forget u (Sec. 3.1): restrict phi' to the smaller bag, keep the colour set
 * and merge entries that became equal (counts add). */
static int dp_forget(dpctx_t *c, int u, const table_t *y, table_t *out) {
    int pu = bag_pos(y, u);
    int32_t phi[ORC_MAXF];
    for (size_t e = 0; e < y->n; e++) {
        const int32_t *pp = y->phi + e * y->b;
        for (int i = 0, k = 0; i < y->b; i++)
            if (i != pu) phi[k++] = pp[i];
        if (tab_push(out, phi, y->C[e], y->cnt[e])) return ORC_ENOMEM;
    }
    return sort_and_merge(out, &c->ovf);
}

/* Join (Sec. 3.1): equal mappings of the two children combine their colour
 * sets C' u C'' when C' n C'' is exactly the colour set of the bag's image;
 * counts multiply, then equal (phi, C) add. */
static int dp_join(dpctx_t *c, const table_t *y, const table_t *z, table_t *out) {
    int b = out->b;
    size_t i = 0, j = 0;
    while (i < y->n && j < z->n) {
        int cmp = 0;
        for (int t = 0; t < b && !cmp; t++) {
            int32_t p = y->phi[i * b + t], q = z->phi[j * b + t];
            if (p != q) cmp = p < q ? -1 : 1;
        }
        if (cmp < 0) { i++; continue; }
        if (cmp > 0) { j++; continue; }
        size_t ie = i, je = j; /* extent of the two groups with this phi */
        while (ie < y->n && !memcmp(y->phi + ie * b, y->phi + i * b, sizeof(int32_t) * b)) ie++;
        while (je < z->n && !memcmp(z->phi + je * b, z->phi + j * b, sizeof(int32_t) * b)) je++;
        uint32_t bagcol = 0;
        for (int t = 0; t < b; t++) bagcol |= 1u << c->col[y->phi[i * b + t]];
        for (size_t a = i; a < ie; a++)
            for (size_t d = j; d < je; d++) {
                if ((y->C[a] & z->C[d]) != bagcol) continue;
                uint64_t p;
                if (__builtin_mul_overflow(y->cnt[a], z->cnt[d], &p)) c->ovf = 1;
                if (tab_push(out, y->phi + i * b, y->C[a] | z->C[d], p)) return ORC_ENOMEM;
            }
        i = ie;
        j = je;
    }
    return sort_and_merge(out, &c->ovf);
}

typedef struct {
    int N;
    const int32_t *td;
    table_t *tabs;
} run_t;

static int td_type(const int32_t *td, int i) { return td[1 + 5 * i]; }
static int td_u(const int32_t *td, int i) { return td[2 + 5 * i]; }
static int td_c0(const int32_t *td, int i) { return td[3 + 5 * i]; }
static int td_c1(const int32_t *td, int i) { return td[4 + 5 * i]; }
static uint32_t td_bag(const int32_t *td, int i) { return (uint32_t)td[5 + 5 * i]; }

/* Post-order evaluation (Sec. 3.1, last paragraph).  Node order in the array
 * is already a post-order. keep_all keeps every table for reconstruction. */
static int dp_run(dpctx_t *c, const int32_t *td, table_t *tabs, int keep_all,
                  int64_t *sizes) {
    int N = td[0];
    for (int i = 0; i < N; i++) {
        table_t *o = &tabs[i];
        tab_init(o, td_bag(td, i));
        int rc = ORC_OK;
        switch (td_type(td, i)) {
        case T_LEAF: rc = dp_leaf(c, td_u(td, i), o); break;
        case T_INTRO: rc = dp_intro(c, td_u(td, i), &tabs[td_c0(td, i)], o); break;
        case T_FORGET: rc = dp_forget(c, td_u(td, i), &tabs[td_c0(td, i)], o); break;
        case T_JOIN: rc = dp_join(c, &tabs[td_c0(td, i)], &tabs[td_c1(td, i)], o); break;
        }
        if (rc == ORC_OK) rc = sort_and_merge(o, &c->ovf); /* canonical order */
        if (rc) return rc;
        if (sizes) sizes[i] = (int64_t)o->n;
        if (!keep_all) {
            if (td_c0(td, i) >= 0) tab_free(&tabs[td_c0(td, i)]);
            if (td_c1(td, i) >= 0) tab_free(&tabs[td_c1(td, i)]);
        }
    }
    return ORC_OK;
}

static int check_inputs(int32_t n, int32_t nF, int32_t k, const uint8_t *colors) {
    if (n < 0 || nF < 1 || nF > ORC_MAXF || k < nF || k > 32) return ORC_ERANGE;
    for (int32_t v = 0; v < n; v++)
        if (colors[v] >= k) return ORC_EINVAL;
    return ORC_OK;
}

/* Count of colourful mappings = sum over the root list D_r of the empty
 * mapping's colour sets (Sec. 3.1: a solution exists iff D_r holds the empty
 * mapping with all colours; with k > nF every nF-subset may appear).
 * per_root_vertex (optional, length n): for the node just below the root
 * (bag {r0}), the sum of its entries grouped by the image of r0.
 * sizes (optional, length N): |D_x| per node. */
static int count_in_range(int32_t n, const int64_t *rp, const int32_t *colidx, int32_t nF,
                          int32_t mF, const int32_t *edges, int32_t k, const uint8_t *colors,
                          const int32_t *td, int32_t td_len, int32_t degmask, int32_t lo0,
                          int32_t hi0, uint64_t *count, uint8_t *overflow,
                          uint64_t *per_root_vertex, int64_t *sizes);

int orc_count(int32_t n, const int64_t *rp, const int32_t *colidx, int32_t nF, int32_t mF,
              const int32_t *edges, int32_t k, const uint8_t *colors, const int32_t *td,
              int32_t td_len, int32_t degmask, uint64_t *count, uint8_t *overflow,
              uint64_t *per_root_vertex, int64_t *sizes) {
    return count_in_range(n, rp, colidx, nF, mF, edges, k, colors, td, td_len, degmask, 0, n,
                          count, overflow, per_root_vertex, sizes);
}

/* The same count restricted to the mappings with Phi(0) in [lo0, hi0). */
int orc_count_range(int32_t n, const int64_t *rp, const int32_t *colidx, int32_t nF, int32_t mF,
                    const int32_t *edges, int32_t k, const uint8_t *colors, const int32_t *td,
                    int32_t td_len, int32_t degmask, int32_t lo0, int32_t hi0, uint64_t *count,
                    uint8_t *overflow, int64_t *sizes) {
    if (lo0 < 0 || hi0 < lo0 || hi0 > n) return ORC_EINVAL;
    return count_in_range(n, rp, colidx, nF, mF, edges, k, colors, td, td_len, degmask, lo0, hi0,
                          count, overflow, NULL, sizes);
}

static int count_in_range(int32_t n, const int64_t *rp, const int32_t *colidx, int32_t nF,
                          int32_t mF, const int32_t *edges, int32_t k, const uint8_t *colors,
                          const int32_t *td, int32_t td_len, int32_t degmask, int32_t lo0,
                          int32_t hi0, uint64_t *count, uint8_t *overflow,
                          uint64_t *per_root_vertex, int64_t *sizes) {
    int rc = check_inputs(n, nF, k, colors);
    if (rc) return rc;
    graph_t g = {n, rp, colidx};
    pattern_t F;
    if ((rc = load_pattern(&F, nF, mF, edges))) return rc;
    if (orc_validate_td(nF, mF, edges, td, td_len)) return ORC_EINVAL;
    int N = td[0];
    table_t *tabs = calloc(N, sizeof(table_t));
    if (!tabs) return ORC_ENOMEM;
    dpctx_t c = {&g, &F, colors, degmask, 0, lo0, hi0, !(degmask & ORC_NO_DISTBOUND)};
    /* keep the root's child when the per-vertex split is wanted */
    rc = dp_run(&c, td, tabs, per_root_vertex != NULL, sizes);
    if (rc == ORC_OK) {
        const table_t *r = &tabs[N - 1];
        uint64_t s = 0;
        for (size_t e = 0; e < r->n; e++)
            if (__builtin_add_overflow(s, r->cnt[e], &s)) c.ovf = 1;
        *count = s;
        if (per_root_vertex) {
            memset(per_root_vertex, 0, sizeof(uint64_t) * (size_t)n);
            const table_t *rc0 = &tabs[td_c0(td, N - 1)];
            for (size_t e = 0; e < rc0->n; e++) per_root_vertex[rc0->phi[e]] += rc0->cnt[e];
        }
        if (overflow) *overflow = (uint8_t)c.ovf;
    }
    for (int i = 0; i < N; i++) tab_free(&tabs[i]);
    free(tabs);
    return rc;
}

/* ------------------------------------------------------------------------ */
/* Result reconstruction R(x, M) (Sec. 4).  M is a set of (phi, C) pairs of
 * node x; the result L holds, for each pair, the list of mappings
 * Phi: V*_x -> V(G) that produced it.  A mapping is an int32 row of length nF
 * with -1 on vertices outside V*_x.                                          */
typedef struct {
    size_t n;
    int b;
    int32_t *phi;
    uint32_t *C;
} mset_t;

typedef struct {
    size_t nitems;
    size_t *start, *len; /* rows of item i: rows[start[i] .. start[i]+len[i]) */
    size_t nrows;
    int32_t *rows;
} llist_t;

static void ll_free(llist_t *l) {
    free(l->start);
    free(l->len);
    free(l->rows);
    memset(l, 0, sizeof *l);
}

static void ms_free(mset_t *m) {
    free(m->phi);
    free(m->C);
    memset(m, 0, sizeof *m);
}

/* binary search for (phi, C) in a sorted table; -1 if absent */
static int64_t tab_find(const table_t *t, const int32_t *phi, uint32_t C) {
    size_t lo = 0, hi = t->n;
    while (lo < hi) {
        size_t mid = (lo + hi) / 2;
        int cmp = 0;
        for (int i = 0; i < t->b && !cmp; i++) {
            int32_t x = t->phi[mid * t->b + i];
            if (x != phi[i]) cmp = x < phi[i] ? -1 : 1;
        }
        if (!cmp && t->C[mid] != C) cmp = t->C[mid] < C ? -1 : 1;
        if (!cmp) return (int64_t)mid;
        if (cmp < 0) lo = mid + 1; else hi = mid;
    }
    return -1;
}

/* first index whose phi is >= the given phi */
static size_t tab_lower_phi(const table_t *t, const int32_t *phi) {
    size_t lo = 0, hi = t->n;
    while (lo < hi) {
        size_t mid = (lo + hi) / 2;
        int cmp = 0;
        for (int i = 0; i < t->b && !cmp; i++) {
            int32_t x = t->phi[mid * t->b + i];
            if (x != phi[i]) cmp = x < phi[i] ? -1 : 1;
        }
        if (cmp < 0) lo = mid + 1; else hi = mid;
    }
    return lo;
}

typedef struct {
    const dpctx_t *c;
    const int32_t *td;
    const table_t *tabs;
    int nF;
} rec_t;

static int R(rec_t *s, int x, const mset_t *M, llist_t *L);

/* items of M given as table indices of a child: M-hat built from them */
static int ms_from_indices(const table_t *t, const size_t *idx, size_t n, mset_t *out) {
    out->n = n;
    out->b = t->b;
    out->phi = malloc(sizeof(int32_t) * (t->b ? t->b : 1) * (n ? n : 1));
    out->C = malloc(sizeof(uint32_t) * (n ? n : 1));
    if (!out->phi || !out->C) return ORC_ENOMEM;
    for (size_t i = 0; i < n; i++) {
        if (t->b) memcpy(out->phi + i * t->b, t->phi + idx[i] * t->b, sizeof(int32_t) * t->b);
        out->C[i] = t->C[idx[i]];
    }
    return ORC_OK;
}

static int cmp_size(const void *a, const void *b) {
    size_t x = *(const size_t *)a, y = *(const size_t *)b;
    return x < y ? -1 : x > y;
}

/* sorted, duplicate-free copy of a list of indices; map[i] = position of
 * in[i] in the copy */
static size_t uniq_indices(const size_t *in, size_t n, size_t *out, size_t *map) {
    memcpy(out, in, sizeof(size_t) * n);
    qsort(out, n, sizeof(size_t), cmp_size);
    size_t m = 0;
    for (size_t i = 0; i < n; i++)
        if (m == 0 || out[m - 1] != out[i]) out[m++] = out[i];
    for (size_t i = 0; i < n; i++) {
        size_t lo = 0, hi = m;
        while (lo < hi) {
            size_t mid = (lo + hi) / 2;
            if (out[mid] < in[i]) lo = mid + 1; else hi = mid;
        }
        map[i] = lo;
    }
    return m;
}

static int ll_alloc(llist_t *L, size_t nitems, size_t nrows, int nF) {
    L->nitems = nitems;
    L->nrows = nrows;
    L->start = calloc(nitems ? nitems : 1, sizeof(size_t));
    L->len = calloc(nitems ? nitems : 1, sizeof(size_t));
    L->rows = malloc(sizeof(int32_t) * (size_t)nF * (nrows ? nrows : 1));
    return (L->start && L->len && L->rows) ? ORC_OK : ORC_ENOMEM;
}

static int R(rec_t *s, int x, const mset_t *M, llist_t *L) {
    const int32_t *td = s->td;
    const table_t *tx = &s->tabs[x];
    int nF = s->nF, rc = ORC_OK;
    int type = td_type(td, x);
    if (type == T_LEAF) {
        /* one mapping per pair: Phi = phi */
        if ((rc = ll_alloc(L, M->n, M->n, nF))) return rc;
        int u = td_u(td, x);
        for (size_t i = 0; i < M->n; i++) {
            L->start[i] = i;
            L->len[i] = 1;
            for (int v = 0; v < nF; v++) L->rows[i * nF + v] = -1;
            L->rows[i * nF + u] = M->phi[i];
        }
        return ORC_OK;
    }
    if (type == T_INTRO) {
        /* M-hat: phi restricted to V_y, colour of phi(u) removed */
        int y = td_c0(td, x), u = td_u(td, x);
        const table_t *ty = &s->tabs[y];
        int pu = bag_pos(tx, u);
        size_t *idx = malloc(sizeof(size_t) * (M->n ? M->n : 1));
        size_t *uq = malloc(sizeof(size_t) * (M->n ? M->n : 1));
        size_t *map = malloc(sizeof(size_t) * (M->n ? M->n : 1));
        if (!idx || !uq || !map) { free(idx); free(uq); free(map); return ORC_ENOMEM; }
        int32_t ph[ORC_MAXF];
        for (size_t i = 0; i < M->n && !rc; i++) {
            const int32_t *p = M->phi + i * M->b;
            for (int a = 0, k = 0; a < M->b; a++)
                if (a != pu) ph[k++] = p[a];
            uint32_t Ch = M->C[i] & ~(1u << s->c->col[p[pu]]);
            int64_t f = tab_find(ty, ph, Ch);
            if (f < 0) rc = ORC_EINVAL; /* cannot happen for a pair of D_x */
            else idx[i] = (size_t)f;
        }
        mset_t Mh = {0};
        llist_t Lh = {0};
        size_t m = 0;
        if (!rc) m = uniq_indices(idx, M->n, uq, map);
        if (!rc) rc = ms_from_indices(ty, uq, m, &Mh);
        if (!rc) rc = R(s, y, &Mh, &Lh);
        if (!rc) {
            size_t total = 0;
            for (size_t i = 0; i < M->n; i++) total += Lh.len[map[i]];
            rc = ll_alloc(L, M->n, total, nF);
            size_t w = 0;
            for (size_t i = 0; i < M->n && !rc; i++) {
                size_t h = map[i];
                L->start[i] = w;
                L->len[i] = Lh.len[h];
                for (size_t r = 0; r < Lh.len[h]; r++, w++) {
                    memcpy(L->rows + w * nF, Lh.rows + (Lh.start[h] + r) * nF, sizeof(int32_t) * nF);
                    L->rows[w * nF + u] = M->phi[i * M->b + pu]; /* extend by phi(u) */
                }
            }
        }
        ms_free(&Mh);
        ll_free(&Lh);
        free(idx);
        free(uq);
        free(map);
        return rc;
    }
    if (type == T_FORGET) {
        /* M-hat: all (phi-hat, C) of D_y whose restriction to V_x is phi */
        int y = td_c0(td, x), u = td_u(td, x);
        const table_t *ty = &s->tabs[y];
        int pu = bag_pos(ty, u);
        /* per item, the matching child entries */
        size_t cap = 1024, nm = 0;
        size_t *cidx = malloc(sizeof(size_t) * cap);
        size_t *owner = malloc(sizeof(size_t) * cap);
        if (!cidx || !owner) { free(cidx); free(owner); return ORC_ENOMEM; }
        for (size_t i = 0; i < M->n && !rc; i++) {
            const int32_t *p = M->phi + i * M->b;
            for (size_t e = 0; e < ty->n; e++) { /* plain scan of D_y */
                if (ty->C[e] != M->C[i]) continue;
                const int32_t *q = ty->phi + e * ty->b;
                int same = 1;
                for (int a = 0, k = 0; a < ty->b && same; a++) {
                    if (a == pu) continue;
                    if (q[a] != p[k++]) same = 0;
                }
                if (!same) continue;
                if (nm == cap) {
                    cap *= 2;
                    size_t *a1 = realloc(cidx, sizeof(size_t) * cap);
                    size_t *a2 = realloc(owner, sizeof(size_t) * cap);
                    if (a1) cidx = a1;
                    if (a2) owner = a2;
                    if (!a1 || !a2) { rc = ORC_ENOMEM; break; }
                }
                cidx[nm] = e;
                owner[nm] = i;
                nm++;
            }
        }
        /* different items never share a child entry: cidx is duplicate-free */
        mset_t Mh = {0};
        llist_t Lh = {0};
        if (!rc) rc = ms_from_indices(ty, cidx, nm, &Mh);
        if (!rc) rc = R(s, y, &Mh, &Lh);
        if (!rc) {
            rc = ll_alloc(L, M->n, Lh.nrows, nF);
            size_t w = 0, h = 0;
            for (size_t i = 0; i < M->n && !rc; i++) { /* flatten per item */
                L->start[i] = w;
                for (; h < nm && owner[h] == i; h++) {
                    memcpy(L->rows + w * nF, Lh.rows + Lh.start[h] * nF,
                           sizeof(int32_t) * nF * Lh.len[h]);
                    w += Lh.len[h];
                }
                L->len[i] = w - L->start[i];
            }
        }
        ms_free(&Mh);
        ll_free(&Lh);
        free(cidx);
        free(owner);
        return rc;
    }
    /* join: for each (phi, C) all (phi, C') in D_y and (phi, C'') in D_z with
     * C' u C'' = C and C' n C'' = zeta(phi(V_x)) */
    int y = td_c0(td, x), z = td_c1(td, x);
    const table_t *ty = &s->tabs[y], *tz = &s->tabs[z];
    size_t cap = 1024, np = 0;
    size_t *py = malloc(sizeof(size_t) * cap), *pz = malloc(sizeof(size_t) * cap),
           *own = malloc(sizeof(size_t) * cap);
    if (!py || !pz || !own) { free(py); free(pz); free(own); return ORC_ENOMEM; }
    for (size_t i = 0; i < M->n && !rc; i++) {
        const int32_t *p = M->phi + i * M->b;
        uint32_t bagcol = 0;
        for (int a = 0; a < M->b; a++) bagcol |= 1u << s->c->col[p[a]];
        size_t a0 = tab_lower_phi(ty, p), d0 = tab_lower_phi(tz, p);
        for (size_t a = a0; a < ty->n && !memcmp(ty->phi + a * ty->b, p, sizeof(int32_t) * M->b); a++)
            for (size_t d = d0; d < tz->n && !memcmp(tz->phi + d * tz->b, p, sizeof(int32_t) * M->b); d++) {
                if ((ty->C[a] | tz->C[d]) != M->C[i] || (ty->C[a] & tz->C[d]) != bagcol) continue;
                if (np == cap) {
                    cap *= 2;
                    size_t *a1 = realloc(py, sizeof(size_t) * cap), *a2 = realloc(pz, sizeof(size_t) * cap),
                           *a3 = realloc(own, sizeof(size_t) * cap);
                    if (a1) py = a1;
                    if (a2) pz = a2;
                    if (a3) own = a3;
                    if (!a1 || !a2 || !a3) { rc = ORC_ENOMEM; break; }
                }
                py[np] = a;
                pz[np] = d;
                own[np] = i;
                np++;
            }
    }
    size_t *uy = malloc(sizeof(size_t) * (np ? np : 1)), *my = malloc(sizeof(size_t) * (np ? np : 1));
    size_t *uz = malloc(sizeof(size_t) * (np ? np : 1)), *mz = malloc(sizeof(size_t) * (np ? np : 1));
    mset_t M1 = {0}, M2 = {0};
    llist_t L1 = {0}, L2 = {0};
    if (!uy || !my || !uz || !mz) rc = ORC_ENOMEM;
    size_t ny = 0, nz = 0;
    if (!rc) {
        ny = uniq_indices(py, np, uy, my);
        nz = uniq_indices(pz, np, uz, mz);
        rc = ms_from_indices(ty, uy, ny, &M1);
    }
    if (!rc) rc = ms_from_indices(tz, uz, nz, &M2);
    if (!rc) rc = R(s, y, &M1, &L1);
    if (!rc) rc = R(s, z, &M2, &L2);
    if (!rc) {
        size_t total = 0;
        for (size_t h = 0; h < np; h++) total += L1.len[my[h]] * L2.len[mz[h]];
        rc = ll_alloc(L, M->n, total, nF);
        size_t w = 0, h = 0;
        for (size_t i = 0; i < M->n && !rc; i++) {
            L->start[i] = w;
            for (; h < np && own[h] == i; h++) { /* all combinations of the two lists */
                size_t A = my[h], B = mz[h];
                for (size_t r1 = 0; r1 < L1.len[A]; r1++)
                    for (size_t r2 = 0; r2 < L2.len[B]; r2++, w++) {
                        const int32_t *q1 = L1.rows + (L1.start[A] + r1) * nF;
                        const int32_t *q2 = L2.rows + (L2.start[B] + r2) * nF;
                        for (int v = 0; v < nF; v++) L->rows[w * nF + v] = q1[v] >= 0 ? q1[v] : q2[v];
                    }
            }
            L->len[i] = w - L->start[i];
        }
    }
    ms_free(&M1);
    ms_free(&M2);
    ll_free(&L1);
    ll_free(&L2);
    free(py); free(pz); free(own); free(uy); free(my); free(uz); free(mz);
    return rc;
}

static _Thread_local int g_nF_cmp;
static int cmp_row(const void *a, const void *b) {
    const int32_t *x = a, *y = b;
    for (int i = 0; i < g_nF_cmp; i++)
        if (x[i] != y[i]) return x[i] < y[i] ? -1 : 1;
    return 0;
}

/* All colourful mappings via R(r, D_r) on the root (Sec. 4), sorted
 * lexicographically, the first min(total, cap) copied to rows. */
int orc_enumerate(int32_t n, const int64_t *rp, const int32_t *colidx, int32_t nF, int32_t mF,
                  const int32_t *edges, int32_t k, const uint8_t *colors, const int32_t *td,
                  int32_t td_len, int32_t degmask, uint64_t cap, int32_t *rows,
                  uint64_t *n_rows, uint64_t *total) {
    int rc = check_inputs(n, nF, k, colors);
    if (rc) return rc;
    graph_t g = {n, rp, colidx};
    pattern_t F;
    if ((rc = load_pattern(&F, nF, mF, edges))) return rc;
    if (orc_validate_td(nF, mF, edges, td, td_len)) return ORC_EINVAL;
    int N = td[0];
    table_t *tabs = calloc(N, sizeof(table_t));
    if (!tabs) return ORC_ENOMEM;
    dpctx_t c = {&g, &F, colors, degmask, 0, 0, n, !(degmask & ORC_NO_DISTBOUND)};
    rc = dp_run(&c, td, tabs, 1, NULL);
    mset_t M = {0};
    llist_t L = {0};
    if (!rc) {
        const table_t *r = &tabs[N - 1];
        size_t *all = malloc(sizeof(size_t) * (r->n ? r->n : 1));
        if (!all) rc = ORC_ENOMEM;
        for (size_t i = 0; !rc && i < r->n; i++) all[i] = i;
        if (!rc) rc = ms_from_indices(r, all, r->n, &M);
        free(all);
    }
    rec_t s = {&c, td, tabs, nF};
    if (!rc) rc = R(&s, N - 1, &M, &L);
    if (!rc) {
        g_nF_cmp = nF;
        qsort(L.rows, L.nrows, sizeof(int32_t) * nF, cmp_row);
        uint64_t m = L.nrows < cap ? L.nrows : cap;
        if (rows && m) memcpy(rows, L.rows, sizeof(int32_t) * nF * m);
        *n_rows = m;
        *total = L.nrows;
    }
    ms_free(&M);
    ll_free(&L);
    for (int i = 0; i < N; i++) tab_free(&tabs[i]);
    free(tabs);
    return rc;
}
