/*
 * ccgpu.h -- C ABI of the MI355X (gfx950) colour-coding library.
 *
 * The library implements the colour-coding dynamic program for subgraph
 * isomorphism and enumeration of Malik, Suchy and Valla, "Efficient
 * Implementation of Color Coding Algorithm for Subgraph Isomorphism Problem"
 * (arXiv 1908.11248):
 *   - SubIso / SubEnum problem statement: Sec. 1 (adjacency-preserving
 *     injective mappings V(F) -> V(G), not necessarily induced);
 *   - random colouring and colourful copies: Sec. 2.1;
 *   - tree decomposition and nice tree decomposition: Sec. 1.2, Sec. 3;
 *   - the leaf / introduce / forget / join rules: Sec. 3.1;
 *   - degree mask and candidate limiting: Sec. 3.2;
 *   - result reconstruction: Sec. 4.
 *
 * Counting semantics.  count(G, F, zeta) is the number of mappings
 * Phi: V(F) -> V(G) that send every edge of F to an edge of G and give the
 * images pairwise distinct colours (hence Phi is injective).  Automorphic
 * images count separately: this is the paper's default counting mode
 * (Sec. 5.2, "the former version").  Counts are exact modulo 2^64; a per
 * colouring overflow flag is set when a DP entry's true value reaches 2^64
 * under the decomposition used (a clear flag means the count is exact).
 *
 * Conventions.
 *   - Every call returns a status (CC_OK = 0 or a negative CC_E* code) and
 *     records a message for cc_last_error() (thread-local).
 *   - Handles are opaque and owned by the library; *_free(NULL) is a no-op.
 *   - Input arrays are host arrays, copied by the call and still owned by
 *     the caller.  Output arrays are caller-allocated host arrays.
 *   - A context is used by one host thread at a time.  Calls that produce
 *     results synchronise the context's stream before they return.
 *   - Colours are 0-based: colour c of a k-colouring is c in [0, k).
 *   - Limits (CC_ERANGE when exceeded): a decomposition takes
 *     1 <= n_F <= 16 pattern vertices and treewidth <= 3; a colouring takes
 *     1 <= k <= 16 colours and at most 2^20 colourings; counting needs
 *     n_F <= k (colour sets are k-bit masks; the paper uses 32-bit masks for
 *     n_F <= 32, Sec. 3.2), enumeration and vertex sets k <= 12; n_G < 2^31;
 *     the packed table key (colouring index, bag images, colour set) must
 *     fit 128 bits.
 */
#ifndef CCGPU_H
#define CCGPU_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* status codes */
#define CC_OK 0
#define CC_EINVAL (-1)     /* malformed graph, pattern, decomposition or argument */
#define CC_ERANGE (-2)     /* a size limit above is exceeded */
#define CC_ENOMEM (-3)     /* device arena or host allocation failed */
#define CC_EDEVICE (-4)    /* a HIP runtime error */
#define CC_ECANCELLED (-5) /* request cancelled (serving) */

typedef struct cc_context cc_context;
typedef struct cc_graph cc_graph;
typedef struct cc_coloring cc_coloring;
typedef struct cc_decomp cc_decomp;

/* Message describing the last failing call on this thread ("" if none). */
const char *cc_last_error(void);

/* Creates a context on HIP device `device`.
 *   arena_dev    device memory of `device` that holds every DP table and the
 *                per-run scratch (e.g. a torch uint8 tensor's data pointer),
 *                256-byte aligned; the caller owns it and must keep it alive
 *                until cc_context_destroy returns.  NULL: the library
 *                allocates the arena itself.
 *   arena_bytes  size of the arena (>= 4096 with arena_dev; with NULL,
 *                0 means 3/4 of the device's free memory).
 *   hip_stream   hipStream_t to launch the single-query calls on (e.g. torch's
 *                current stream; NULL: the library creates one).  The caller
 *                keeps ownership of a stream it passes.
 * Errors: CC_EINVAL (misaligned or foreign arena), CC_EDEVICE (no such
 * device), CC_ENOMEM. */
int cc_context_create(int device, void *arena_dev, size_t arena_bytes, void *hip_stream,
                      cc_context **out);
int cc_context_destroy(cc_context *ctx);

/* Uploads host graph G (Sec. 1.2: simple and undirected) in CSR form:
 *   row_ptr[n + 1] (int64, row_ptr[0] = 0), col[row_ptr[n]] (int32).
 * Both directions of every edge must be present, rows strictly ascending,
 * no self-loops; violations return CC_EINVAL unless flags has
 * CC_GRAPH_CANONICALIZE, which sorts, symmetrises and removes loops and
 * duplicates instead.  The graph stays resident on the context's device. */
#define CC_GRAPH_CANONICALIZE 1u
int cc_load_graph(cc_context *ctx, int32_t n, const int64_t *row_ptr, const int32_t *col,
                  uint32_t flags, cc_graph **out);
void cc_graph_free(cc_graph *g);
int32_t cc_graph_num_vertices(const cc_graph *g);

/* Random colourings of G (Sec. 2.1).  Colouring b (0 <= b < num_colorings)
 * gives vertex v the colour
 *     floor(k * hi32(splitmix64(seed XOR (b * 2^32 + v))) / 2^32)
 * where splitmix64(s) is the first output of the published splitmix64
 * generator seeded with s.  Computed on the device. */
int cc_color(cc_context *ctx, const cc_graph *g, int32_t k, uint64_t seed,
             int32_t num_colorings, cc_coloring **out);
/* Explicit colourings: colors[b * n + v] in [0, k) (host array). */
int cc_color_explicit(cc_context *ctx, const cc_graph *g, int32_t k, int32_t num_colorings,
                      const uint8_t *colors, cc_coloring **out);
/* Copies colouring b to colors_out[n] (host). */
int cc_coloring_download(const cc_coloring *c, int32_t b, uint8_t *colors_out);
void cc_coloring_free(cc_coloring *c);

/* Nice tree decomposition of pattern F (Sec. 3): minimum width (exact, by
 * elimination orderings), then converted to the paper's nice form (Sec. 1.2:
 * single-vertex leaves, empty root of degree one).  Pattern vertex 0 is the
 * last vertex forgotten.  edges[2*i], edges[2*i+1] is the i-th edge of F.
 * Host-only; needs no context. */
int cc_build_decomposition(int32_t n_F, int32_t m_F, const int32_t *edges, uint32_t flags,
                           cc_decomp **out);
/* Exports the nice TD as int32 data: buf[0] = N nodes, then five ints per
 * node in post-order (root last): type (0 leaf, 1 introduce, 2 forget,
 * 3 join), vertex (-1 for a join), child0, child1 (-1 if absent), bag as a
 * uint32 bitmask.  *len receives 1 + 5N; CC_ERANGE if cap is smaller. */
int cc_decomp_export(const cc_decomp *d, int32_t *buf, size_t cap, size_t *len);
/* Imports a nice TD in the export format for pattern F; it is validated
 * against the definitions of Sec. 1.2 (CC_EINVAL if invalid). */
int cc_decomp_import(int32_t n_F, int32_t m_F, const int32_t *edges, const int32_t *buf,
                     size_t len, cc_decomp **out);
int32_t cc_decomp_width(const cc_decomp *d);
/* Human-readable device plan of the decomposition (one line per step: the
 * node rule, its variant, the table's column order).  *len receives the
 * length including the terminating NUL; CC_ERANGE if cap is smaller. */
int cc_decomp_describe(const cc_decomp *d, char *buf, size_t cap, size_t *len);
void cc_decomp_free(cc_decomp *d);

/* Runs the DP (Sec. 3.1) for every colouring of `c` in one batch and writes
 * counts[b] and (if not NULL) overflow[b] for b < num_colorings.
 * flags: CC_NO_DEGREE_MASK disables the degree mask of Sec. 3.2 (same
 * counts, bigger tables).  When every table of the plan has a one-vertex bag
 * (tree patterns) and the dense form fits the arena, tables are kept dense
 * over (colouring, bag image, colour set of the node's size); CC_SPARSE_TABLES
 * keeps them as sorted entry lists instead (same counts, table sizes and
 * overflow flags). */
#define CC_NO_DEGREE_MASK 1u
#define CC_SPARSE_TABLES 2u
/* Introduce nodes whose new vertex u has two or more neighbours in the bag
 * normally draw each entry's candidates from the adjacency list of the bag
 * neighbour whose image has the fewest neighbours (then re-sort); with
 * CC_CLASSIC_EXPAND they always use one fixed column's list (same counts). */
#define CC_CLASSIC_EXPAND 4u
int cc_count(cc_context *ctx, const cc_graph *g, const cc_coloring *c, const cc_decomp *d,
             uint32_t flags, uint64_t *counts, uint8_t *overflow);

/* cc_count restricted to the mappings with Phi(0) in [lo, hi) (0 <= lo <=
 * hi <= n_G).  Counts over disjoint ranges add up (mod 2^64) to cc_count's:
 * this is the unit of the anchor-range chunking below and of a split of one
 * colouring across devices.  Table sizes of nodes whose bag holds pattern
 * vertex 0 cover the range only; other nodes' tables are whole. */
int cc_count_range(cc_context *ctx, const cc_graph *g, const cc_coloring *c, const cc_decomp *d,
                   uint32_t flags, int32_t lo, int32_t hi, uint64_t *counts, uint8_t *overflow);

/* Anchor-range chunking.  When a table of cc_count / cc_count_range /
 * cc_count_batch / the server exceeds the per-table budget or the arena
 * (arenas of 256 MiB or more), the run is repeated in waves of half the
 * colourings, and a single colouring in two halves of the image range of
 * pattern vertex 0 (pattern vertex 0 stays in every bag above its
 * introduction, so each table of those nodes splits into disjoint parts),
 * recursively, at most 64 ranges per colouring.  Counts and flags equal the
 * unsplit run's (a carry in the final sum sets the flag).  This returns the
 * number of (colouring-wave, range) runs of the last single-query count on
 * ctx (1: not split). */
int32_t cc_last_chunk_count(const cc_context *ctx);

/* Estimated device memory of a count of pattern d with k colours and
 * num_colorings colourings on graph g: *peak_bytes the peak arena footprint,
 * *entries (optional) the sum of |D_x| over nodes and colourings.  A model
 * from the plan and g's degree statistics (mean neighbour degree, sampled
 * transitivity): introduce multiplies by the candidates of a bag neighbour's
 * adjacency list, the chance that the new colour is unused and that further
 * bag neighbours are adjacent; forget and join are capped by the number of
 * keys the bag can hold.  The serving loop admits queries by it.  Host only. */
int cc_estimate_memory(const cc_graph *g, const cc_decomp *d, int32_t k, int32_t num_colorings,
                       double *peak_bytes, double *entries);

/* cc_count for callers that cannot allocate memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): same
 * arguments, results and flags as cc_count, but the run makes no device or
 * pinned-host allocation (no hipMalloc, hipFree or allocating library call).
 * Its DP tables and scratch live in a fixed 64 MiB device array inside the
 * library (one per device, held until the process ends; its address is
 * taken when a context is created on the device); the results are read back
 * through a pinned buffer the context allocated at creation.  Inputs that
 * cannot fit (colourings x vertices x 16 bytes above 64 MiB, or tables that
 * outgrow the array during the run) fail with CC_ERANGE and a message
 * naming the limit.  All calls on one device share that array: calls that
 * overlap in time on the same device (from several threads or contexts)
 * race and must be serialised by the caller.  The per-table budget of
 * cc_set_table_budget does not apply. */
int cc_count_noalloc(cc_context *ctx, const cc_graph *g, const cc_coloring *c, const cc_decomp *d,
                     uint32_t flags, uint64_t *counts, uint8_t *overflow);

/* Same DP for one colouring index b; per_vertex[v] (n entries) receives the
 * number of colourful mappings with Phi(0) = v (the entries of the node
 * below the root, whose bag is {0}). */
int cc_count_by_vertex(cc_context *ctx, const cc_graph *g, const cc_coloring *c, int32_t b,
                       const cc_decomp *d, uint32_t flags, uint64_t *per_vertex,
                       uint64_t *count, uint8_t *overflow);

/* Enumeration (Sec. 4) for colouring index b: the first min(total, cap)
 * colourful mappings in ascending lexicographic order of
 * (Phi(0), ..., Phi(n_F - 1)), written row-major to rows[cap][n_F];
 * *n_rows = min(total, cap), *total = the count.  CC_ERANGE when the count
 * overflowed 64 bits. */
int cc_enumerate(cc_context *ctx, const cc_graph *g, const cc_coloring *c, int32_t b,
                 const cc_decomp *d, uint64_t cap, int32_t *rows, uint64_t *n_rows,
                 uint64_t *total);

/* Occurrences that differ in their vertex sets (Sec. 5.2: the method can
 * count every mapping, the default, or only occurrences with distinct vertex
 * sets).  For colouring b: *n_mappings = the colourful mappings (as
 * cc_count), *n_sets = the distinct sets {Phi(0), ..., Phi(n_F - 1)} among
 * them; sets (if not NULL, cap rows of n_F int32) receives those sets, each
 * sorted ascending, in lexicographic order.  CC_ERANGE when the mappings
 * exceed cap (every mapping is enumerated to find the sets). */
int cc_vertex_sets(cc_context *ctx, const cc_graph *g, const cc_coloring *c, int32_t b, const cc_decomp *d,
                   uint64_t cap, int32_t *sets, uint64_t *n_sets, uint64_t *n_mappings);

/* Repetition driver of the randomised algorithm (Sec. 2.1, Sec. 5.2):
 * colourings 0, 1, 2, ... of cc_color(k = n_F, seed) are run in batches of
 * `batch` until l = ceil(e^{n_F} ln(1/eps)) colourings are done (then a
 * fixed occurrence is missed with probability at most eps) or at least
 * max_solutions distinct solutions were found.  After each colouring with a
 * nonzero count its first max_solutions mappings (lexicographic) are added
 * to the set of solutions; solutions are mappings, or with
 * CC_SEARCH_DISTINCT_SETS their sorted vertex sets.  rows[max_solutions][n_F]
 * receives the lexicographically first min(found, max_solutions) solutions;
 * *colourings_run and *colourings_planned (= l) report the repetitions. */
#define CC_SEARCH_DISTINCT_SETS 1u
typedef struct {
    double eps;             /* error bound in (0, 1); the paper uses 1/e */
    uint64_t seed;          /* colouring seed */
    int32_t batch;          /* colourings per device batch (0: 16) */
    uint64_t max_solutions; /* stop once this many distinct solutions are found */
    uint32_t flags;         /* CC_SEARCH_DISTINCT_SETS */
} cc_search_opts;
int cc_search(cc_context *ctx, const cc_graph *g, const cc_decomp *d, const cc_search_opts *opts, int32_t *rows,
              uint64_t *n_rows, uint64_t *colourings_run, uint64_t *colourings_planned);

/* Per-node statistics of the last cc_count / cc_enumerate call on ctx:
 * entries[i] = sum over colourings of |D_x| for TD node i (export order),
 * up to cap nodes; *n_nodes receives the node count. */
int cc_last_table_sizes(const cc_context *ctx, int64_t *entries, size_t cap, size_t *n_nodes);

/* Per-kernel timing.  cc_profile_enable(ctx, 1) clears the statistics and
 * starts recording a HIP event pair around every kernel launch the library
 * makes on the context's stream; cc_profile_read copies up to cap records
 * (launches, total milliseconds, algorithmic bytes summed over launches:
 * the bytes the kernel's rule must read and write, not the bytes the
 * hardware moved).  Recording adds a little host overhead per launch. */
typedef struct {
    char name[32];
    uint64_t launches;
    double total_ms;
    double algo_bytes;
} cc_kernel_stat;
int cc_profile_enable(cc_context *ctx, int enable);
/* Restricts recording to the kernel of the given statistic name (as in
 * cc_kernel_stat.name), and to one launch in `every` of it (0 or 1: all), so
 * that event pairs add little to a timed run; NULL or "" records every
 * kernel again. */
int cc_profile_filter(cc_context *ctx, const char *name, uint32_t every);
int cc_profile_read(cc_context *ctx, cc_kernel_stat *stats, size_t cap, size_t *n);

/* Captured counts (HIP graphs).  cc_plan_create records the device work of
 * one count of pattern d with k colours and num_colorings colourings on g
 * (every kernel of the plan, which on dense one-column tables needs no host
 * round trip between steps) into a HIP graph; cc_plan_count colours with
 * cc_color(k, seed) numbering into the plan's own buffer and replays the
 * graph, writing counts[num_colorings] (and overflow) like cc_count.  The
 * plan owns its colour buffer and a slice of the context arena sized by one
 * eager run at creation, and its own stream.  CC_ERANGE for plans that do
 * not run on dense tables (tables with two or more bag vertices read their
 * sizes back between steps).  flags: CC_NO_DEGREE_MASK. */
typedef struct cc_plan cc_plan;
int cc_plan_create(cc_context *ctx, const cc_graph *g, const cc_decomp *d, int32_t k, int32_t num_colorings,
                   uint32_t flags, cc_plan **out);
int cc_plan_count(cc_plan *p, uint64_t seed, uint64_t *counts, uint8_t *overflow);
int cc_plan_destroy(cc_plan *p);

/* ---------------------------------------------------------------------- */
/* Batched queries: many (decomposition, colouring) pairs over one graph,
 * scheduled together.  counts_flat / overflow_flat receive, query after
 * query, num_colorings values each. */
typedef struct {
    const cc_decomp *decomp;
    const cc_coloring *coloring;
} cc_query;
int cc_count_batch(cc_context *ctx, const cc_graph *g, int32_t nq, const cc_query *q,
                   uint32_t flags, uint64_t *counts_flat, uint8_t *overflow_flat);
/* The queries run on `lanes` concurrent HIP streams of the context (0: the
 * tuned or default number), scheduled largest-plan first; a query that runs
 * out of arena memory while others hold it is re-run alone.  Results are
 * identical to one cc_count per query. */
int cc_set_batch_lanes(cc_context *ctx, int32_t lanes);
/* Schedule of a context: concurrent lanes of a batch; the introduce form
 * (entry-wise when it walks fewer than 1/entry_factor of the fixed column's
 * candidates); entry-wise introduces test adjacency once per group of
 * entries with equal bag images when the child has at least group_min
 * entries per such group (0: never); forget and join on sorted lists add up
 * by sorting when k > sort_above_k, else in dense 2^k LDS accumulators
 * (k <= 12 only).  Defaults: 4 lanes (0 = default), 3, 12, 2.  Every
 * schedule gives the same results. */
typedef struct {
    int32_t lanes;
    int32_t entry_factor;
    int32_t sort_above_k;
    int32_t group_min;
} cc_schedule;
int cc_get_schedule(const cc_context *ctx, cc_schedule *out);
int cc_set_schedule(cc_context *ctx, const cc_schedule *s);
/* Autotuner: times cc_count_batch on the given queries and keeps the
 * fastest schedule for the context, by coordinate descent: lanes 1, 2, 4, 8;
 * then entry_factor 1, 3, 8; then sort_above_k 12, 8, 0; then group_min 2,
 * 0, 4.  The counts of
 * every trial must agree (CC_EDEVICE otherwise).  *best receives the lanes. */
int cc_tune_batch(cc_context *ctx, const cc_graph *g, int32_t nq, const cc_query *q, uint32_t flags,
                  int32_t *best);
/* Work budget: with max_entries > 0 no DP table of one launch may hold more
 * entries.  A call whose tables would exceed it runs its colourings in waves
 * (halving recursively; results are unchanged) and fails with CC_ERANGE
 * only when a single colouring exceeds the budget. */
int cc_set_table_budget(cc_context *ctx, uint64_t max_entries);

/* ---------------------------------------------------------------------- */
/* Serving: a request loop over a resident graph (continuous batching).
 * Submitted queries wait in FIFO order and are admitted while a worker lane
 * is free and their estimated arena footprint fits the free part of the
 * memory budget.  The estimate is cc_estimate_memory's model of the query's
 * plan on the resident graph, scaled by a running correction (the geometric
 * mean of measured peak / model over completed queries, within [0.5, 4]);
 * a decomposition and colouring count seen before uses its measured peak
 * (+1/8) instead.  Admitted queries run concurrently on their own streams,
 * so their kernels overlap on the device; a query whose estimate exceeds the
 * budget still runs (alone when nothing else fits) and splits itself into
 * waves and anchor ranges when its tables do not fit.  With max_heavy > 0,
 * at most that many queries whose decomposition has width >= 2 are in
 * flight at once (0: no such limit).  A query that runs out of memory while
 * others hold it is re-queued to run alone.  Tail protection (tail_factor >
 * 0): while some running query has run longer than tail_factor times the
 * mean service time of the queries completed so far, no further query is
 * admitted, so a long query does not share the device with a stream of
 * newcomers (it then finishes about as fast as alone, which bounds the
 * latency tail).  Latency is measured from submission to completion. */
typedef struct {
    int32_t max_inflight;  /* worker lanes (concurrent queries), >= 1 */
    size_t mem_budget;     /* bytes of the arena the server may use (0: all) */
    uint64_t max_entries;  /* per-table budget of each query (0: none) */
    int32_t max_heavy;     /* width >= 2 queries in flight at once (0: no limit) */
    double tail_factor;    /* tail protection threshold (0: off) */
} cc_server_opts;
typedef struct {
    uint64_t submitted, completed, failed, requeued;
    double wall_s;   /* first submission to last completion */
    double qps;      /* completed / wall_s */
    double p50_ms, p99_ms, mean_ms, max_ms;
} cc_server_stats;
typedef struct cc_server cc_server;
int cc_server_start(cc_context *ctx, const cc_graph *g, const cc_server_opts *opts, cc_server **out);
/* Queues count(F, zeta_b) for b < num_colorings with colourings drawn as in
 * cc_color(k, seed); the decomposition must outlive the request. */
int cc_server_submit(cc_server *srv, const cc_decomp *d, int32_t k, uint64_t seed, int32_t num_colorings,
                     uint64_t *ticket);
/* (errors: CC_EINVAL for NULL arguments, CC_ERANGE when k or num_colorings
 * is outside the limits above, CC_ECANCELLED once the server is stopping) */
/* *state: 0 queued or running, 1 done (counts[num_colorings] and overflow
 * written), or a negative CC_E* code of a failed query. */
int cc_server_poll(cc_server *srv, uint64_t ticket, uint64_t *counts, uint8_t *overflow, int32_t *state);
/* Blocks until the ticket is done; same outputs as cc_server_poll. */
int cc_server_wait(cc_server *srv, uint64_t ticket, uint64_t *counts, uint8_t *overflow, int32_t *state);
/* Drains the queue, stops the workers and frees the server. */
int cc_server_stop(cc_server *srv, cc_server_stats *stats);

#ifdef __cplusplus
}
#endif

#endif /* CCGPU_H */
