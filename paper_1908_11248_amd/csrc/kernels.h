// Device kernels of the colour-coding DP and their host-side launchers.
//
// A DP table is a pair of arrays (keys, counts), sorted ascending by key and
// duplicate-free.  A key packs, from the most significant end:
//     colouring index (bb bits) | image of column 0 (vb bits) | ...
//     | image of column b-1 (vb bits) | colour set (kb bits)
// into a uint64 when bb + b*vb + kb <= 64 and into an unsigned __int128
// otherwise.  Counts are uint64 (mod 2^64).  Integer order of the packed keys
// is the lexicographic order of (colouring, images, colour set).
#pragma once

#include <hip/hip_runtime.h>

#include <vector>

#include <cstddef>
#include <cstdint>

namespace ccg {

typedef unsigned __int128 u128;

struct Lay {
    int b;   // columns
    int vb;  // bits per vertex image
    int kb;  // colour-set bits (= k)
    int bb;  // colouring-index bits
    int bits() const { return bb + b * vb + kb; }
    int kw() const { return bits() <= 64 ? 1 : 2; }
    size_t key_bytes() const { return kw() == 1 ? 8 : 16; }
};

struct DevGraph {
    int32_t n;
    int64_t m2;           // number of stored (directed) edges = 2 m
    const int64_t* rp;    // [n + 1]
    const int32_t* col;   // [2m], rows ascending
    const int32_t* esrc;  // [2m], source vertex of every stored edge
    const int32_t* heavy; // vertices of degree > kHeavyDegree, ascending
    int32_t nheavy;
    const uint64_t* eh;   // edge set: open addressing, linear probing, kEdgeEmpty in free cells
    uint64_t ehmask;      // cells - 1 (a power of two, at least 2 m: a load of at most one half)
    const uint8_t* deg8;  // [n] min(deg(v), 255): the degree masks read one byte
    // Images allowed for the vertex a step introduces: [vlo, vhi).  The whole
    // of V(G) except in the steps that introduce the anchor pattern vertex of
    // an anchor-range chunk (counts add over disjoint ranges of its image).
    int32_t vlo = 0, vhi = 0x7fffffff;
};

// edge-set key of {a, b} (a != b): smaller id in the high half
constexpr uint64_t kEdgeEmpty = ~uint64_t(0);
__host__ __device__ inline uint64_t edge_key(uint32_t a, uint32_t b) {
    return a < b ? (uint64_t(a) << 32) | b : (uint64_t(b) << 32) | a;
}
// cell of a key: the 64-bit finaliser of MurmurHash3 (Appleby)
__host__ __device__ inline uint64_t edge_cell(uint64_t key, uint64_t mask) {
    key ^= key >> 33;
    key *= 0xff51afd7ed558ccdull;
    key ^= key >> 33;
    key *= 0xc4ceb9fe1a85ec53ull;
    key ^= key >> 33;
    return key & mask;
}

constexpr int kHeavyDegree = 64;

struct DevTable {
    void* keys = nullptr;
    uint64_t* cnt = nullptr;
    uint64_t n = 0;
    Lay lay{};
};

// ---- launchers (all asynchronous on `s`) ----
// scan: out[i] = sum_{j<i} in[j] for i <= n (out has n + 1 slots)
void launch_scan_u32(const uint32_t* in, uint64_t* out, uint64_t n, uint64_t* tmp, hipStream_t s);
void launch_scan_u64(const uint64_t* in, uint64_t* out, uint64_t n, uint64_t* tmp, hipStream_t s);
size_t scan_tmp_bytes(uint64_t n);
void launch_fill_u64(uint64_t* p, uint64_t v, uint64_t n, hipStream_t s);
void launch_fill_u32(uint32_t* p, uint32_t v, uint64_t n, hipStream_t s);

void launch_color_hash(uint8_t* colors, int32_t n, int32_t B, int32_t k, uint64_t seed, hipStream_t s);
// colourings b0 .. b0 + B - 1 of the seed (written to colors[0 .. B n))
void launch_color_hash_from(uint8_t* colors, int32_t n, int32_t B, int32_t k, uint64_t seed, uint32_t b0,
                            hipStream_t s);

// runs of equal key >> shift in a sorted table: head_tiles(n) tiles; tsum[t]
// = number of runs starting in tile t; with toff = exclusive scan of tsum
// (toff[tiles] = G), starts[j] = first index of run j and starts[G] = n
uint64_t head_tiles(uint64_t n);
void launch_head_count(const void* keys, int kw, uint64_t n, int shift, uint64_t* tsum, hipStream_t s);
void launch_head_starts(const void* keys, int kw, uint64_t n, int shift, const uint64_t* toff, uint64_t* starts,
                        hipStream_t s);

// leaf
void launch_leaf_count(DevGraph g, int B, int degF, uint32_t* flags, hipStream_t s);
void launch_leaf_emit(DevGraph g, int B, int degF, const uint8_t* colors, const uint64_t* offs, Lay lo,
                      void* keys, uint64_t* cnt, hipStream_t s);

// introduce, push form
struct IntroArgs {
    int pos;       // output column of the new vertex
    int anchor;    // child column giving the candidates (-1: every vertex)
    int nchk;      // further child columns that must be adjacent
    int chk[4];
    int degF;
    // push form, per prefix group: the column, among the anchor and the
    // checked columns before pos, whose image has the fewest neighbours; its
    // adjacency list gives the candidates (the others are checked).  Written
    // by launch_push_work; null: the anchor.
    uint8_t* sel = nullptr;
    // push form, per segment (optional, n < 2^27): its candidate vertex v |
    // colour(v) << 27, written by launch_push_seglen and read by the expand
    // instead of walking group -> first key -> adjacency list -> colour again
    uint32_t* segv = nullptr;
    // entry-grouped form: the groups hold every child column (entries that
    // differ only in their colour sets), so every adjacency check is a
    // per-group one (push_work and push_seglen) and the expand only tests
    // colours
    bool grouped = false;
    // entry-wise form: two child columns whose pattern vertices are adjacent
    // in F (cn0 < 0: none).  Their images are adjacent in G, so the
    // candidates of an entry are the common neighbours of those images: the
    // list of that edge in the graph's common-neighbour index (cn_off /
    // cn_col, per stored edge); erow[e] keeps the list's start for entry e.
    int cn0 = -1, cn1 = -1;
    const uint64_t* cn_off = nullptr;
    const int32_t* cn_col = nullptr;
    int64_t* erow = nullptr;
    // entry-wise form: two child columns whose pattern vertices are not
    // adjacent (wd0 < 0: none); the candidates are the common neighbours of
    // their images, found in the graph's wedge index: a hash of vertex pairs
    // (wd_hk keys x << wd_vb | y, x < y; wd_hv their run) over the runs
    // wd_start[r] .. wd_start[r + 1] of middle vertices in wd_mid
    int wd0 = -1, wd1 = -1, wd_vb = 0;
    const uint64_t* wd_hk = nullptr;
    const uint32_t* wd_hv = nullptr;
    uint64_t wd_mask = 0;
    const uint64_t* wd_start = nullptr;
    const int32_t* wd_mid = nullptr;
};
void launch_push_work(const DevTable& in, const uint64_t* gstart, uint64_t G, DevGraph g,
                      const IntroArgs& a, uint32_t* wcount, hipStream_t s);
// load-balanced expand of introduce candidates (expand.hip): segment
// lengths, then count and emit over tiles of expand_tiles(T) items
void launch_push_seglen(const DevTable& in, const uint64_t* gstart, const uint64_t* woff, uint64_t G, uint64_t W,
                        DevGraph g, const uint8_t* colors, const IntroArgs& a, uint32_t* slen, hipStream_t s);
void launch_pull_seglen(const uint64_t* rstart, const uint64_t* rend, int B, DevGraph g, int degF, uint32_t* slen,
                        hipStream_t s);
uint64_t expand_tiles(uint64_t T);
// entry-wise form: one segment per child entry, candidates from the bag
// neighbour of u whose image has the fewest neighbours (src[e], a child
// column), every other bag neighbour an edge test; output in (entry,
// candidate) order with v at column pos (to be re-sorted on columns 0..pos)
// common-neighbour index of the stored edges: counts, then (off = their
// exclusive prefix sums) the lists
void launch_cn_count(DevGraph g, uint32_t* cnt, hipStream_t s);
// wedge index: per stored edge (w, x) at row position i, the d(w) - 1 - i
// pairs (x, y) of later neighbours y of w: counts, records (key x << vb | y,
// value w), then the hash of the sorted records' runs, and the values as int32
void launch_wedge_count(DevGraph g, uint32_t* cnt, hipStream_t s);
void launch_wedge_emit(DevGraph g, int vb, const uint64_t* off, uint64_t* keys, uint64_t* vals, hipStream_t s);
void launch_wedge_hash(const uint64_t* keys, const uint64_t* starts, uint64_t G, uint64_t* hk, uint32_t* hv,
                       uint64_t mask, hipStream_t s);
void launch_u64_to_i32(const uint64_t* in, int32_t* out, uint64_t n, hipStream_t s);
// count bounds of tree plans (slots.hip): hout[v] = sum of hin over N(v);
// out = a * b elementwise; *out = max(*out, max of h) (h >= 0, as bits)
void launch_hom_spmv(DevGraph g, const double* hin, double* hout, hipStream_t s);
void launch_hom_mul(const double* a, const double* b, double* out, uint64_t n, hipStream_t s);
void launch_hom_max(const double* h, uint64_t n, uint64_t* out, hipStream_t s);
void launch_cn_emit(DevGraph g, const uint64_t* off, int32_t* out, hipStream_t s);
// sums[0] += the anchor column's candidates, sums[1] += the entry-wise form's;
// stride > 1: over every stride-th entry only, writing no lengths
void launch_entry_seglen(const DevTable& in, DevGraph g, const IntroArgs& a, uint32_t* slen, uint8_t* src,
                         uint64_t* sums, uint64_t stride, hipStream_t s);
void launch_entry_count(const DevTable& in, const uint8_t* src, const uint64_t* soff, uint64_t T, DevGraph g,
                        const uint8_t* colors, const IntroArgs& a, uint32_t* tcount, uint16_t* pbits, hipStream_t s);
void launch_entry_emit(const DevTable& in, const uint8_t* src, const uint64_t* soff, uint64_t T, DevGraph g,
                       const uint8_t* colors, const IntroArgs& a, const uint64_t* toff, const uint16_t* pbits,
                       DevTable& out, hipStream_t s);
// distance-bounded form for an introduced vertex with no bag neighbour at
// distance 2 from the vertex of child column `col`: per entry, the ends of
// the walks of length 1 and 2 from that column's image (w2[v] = deg(v) + sum
// of its neighbours' degrees, nbpre[e] = degrees of the earlier neighbours
// in the row of stored edge e, from launch_nbdeg_prefix); the output holds
// duplicates and is in no order: sort it, then keep one entry per key
// (launch_take_runs over the run starts)
void launch_nbdeg_prefix(DevGraph g, uint64_t* nbpre, uint64_t* w2, hipStream_t s);
void launch_ball_seglen(const DevTable& in, int col, const uint64_t* w2, uint32_t* slen, hipStream_t s);
void launch_ball_count(const DevTable& in, int col, const uint64_t* nbpre, const uint64_t* soff, uint64_t T, DevGraph g,
                       const uint8_t* colors, const IntroArgs& a, uint32_t* tcount, uint16_t* pbits, hipStream_t s);
void launch_ball_emit(const DevTable& in, int col, const uint64_t* nbpre, const uint64_t* soff, uint64_t T, DevGraph g,
                      const uint8_t* colors, const IntroArgs& a, const uint64_t* toff, const uint16_t* pbits,
                      DevTable& out, hipStream_t s);
void launch_take_runs(const DevTable& in, const uint64_t* starts, uint64_t G, DevTable& out, hipStream_t s);
// forget by sorting: out (same n, layout with one column less) = in without
// its last column; after a sort of out and its run starts (shift 0),
// launch_reduce_runs sums every run into one entry (carry: ovf[colouring])
void launch_drop_last(const DevTable& in, DevTable& out, hipStream_t s);
// join by pairs: pcount[e] (out == nullptr) or the pairs at poff[e] (out)
// for entry e of y; the products are unreduced and unsorted
void launch_join_pairs(const DevTable& y, const DevTable& z, int32_t n, const uint8_t* colors, uint32_t* pcount,
                       const uint64_t* poff, DevTable* out, uint32_t* ovf, hipStream_t s);
void launch_reduce_runs(const DevTable& in, const uint64_t* starts, uint64_t G, DevTable& out, uint32_t* ovf,
                        hipStream_t s);
// survivor bits of the count pass and the tiles' segment and group bounds,
// both written by launch_expand_count and read back by the emit pass:
// expand_pass_words(T) words
uint64_t expand_pass_words(uint64_t T);
void launch_expand_count(bool pull, const DevTable& in, const uint64_t* gstart, const uint64_t* woff, uint64_t G,
                         const uint64_t* rstart, const uint64_t* soff, uint64_t S, uint64_t T, DevGraph g,
                         const uint8_t* colors, const IntroArgs& a, uint32_t* tcount, uint16_t* pbits, hipStream_t s);
void launch_expand_emit(bool pull, const DevTable& in, const uint64_t* gstart, const uint64_t* woff, uint64_t G,
                        const uint64_t* rstart, const uint64_t* soff, uint64_t S, uint64_t T, DevGraph g,
                        const uint8_t* colors, const IntroArgs& a, const uint64_t* toff, const uint16_t* pbits,
                        DevTable& out, uint64_t* osrc, hipStream_t s);

// introduce, pull form (child column 0 is the anchor).  launch_pull_index
// writes the (colouring, column 0) run index rstart/rend[b * n + v] of a
// table (slots must be zero beforehand); the join uses it too.
void launch_pull_index(const DevTable& in, int32_t n, uint64_t* rstart, uint64_t* rend, hipStream_t s);

// forget of the last column, reduced per group with a dense colour-set accumulator
void launch_forget_count(const DevTable& in, const uint64_t* gstart, uint64_t G, uint32_t* gcount,
                         hipStream_t s);
void launch_forget_emit(const DevTable& in, const uint64_t* gstart, uint64_t G, const uint64_t* goff,
                        DevTable& out, uint32_t* ovf, hipStream_t s);

// join of two tables with the same layout; zlo/zhi index the second child
// by (colouring, image of column 0) (launch_pull_index builds it)
void launch_join_count(const DevTable& y, const DevTable& z, const uint64_t* gstart, uint64_t G, int32_t n,
                       const uint8_t* colors, const uint64_t* zlo, const uint64_t* zhi, uint32_t* gcount,
                       hipStream_t s);
void launch_join_emit(const DevTable& y, const DevTable& z, const uint64_t* gstart, uint64_t G, int32_t n,
                      const uint8_t* colors, const uint64_t* zlo, const uint64_t* zhi, const uint64_t* goff,
                      DevTable& out, uint32_t* ovf, hipStream_t s);

// column permutation (out column j <- in column perm[j]) into tmp, then sort
// index_values: the values become the input positions instead of the counts
void launch_permute(const DevTable& in, const int* perm, DevTable& out, bool index_values, hipStream_t s);
// stable LSD radix sort of (keys, vals) on key bits [lo, bits), ping-ponging
// between the a- and b-buffers. Returns true when the result is in the
// b-buffers, which happens only with copy_back false; with copy_back true a
// result that the last pass wrote to the b-buffers is copied back into the
// a-buffers.
// With `from`, the first pass reads from->keys / from->vals (a table of n
// entries in layout from->lay, keys of the same width) with its columns
// reordered as by launch_permute into from->lay_out, and writes the a-buffers;
// with no bits to sort it only reorders into the a-buffers.
struct RadixSource {
    const void* keys;
    const uint64_t* vals;
    Lay lay, lay_out;
    int perm[4];
};
size_t radix_tmp_bytes(uint64_t n);
bool radix_sort(void* keys_a, uint64_t* vals_a, void* keys_b, uint64_t* vals_b, uint64_t n, int kw, int bits, int lo,
                void* tmp, hipStream_t s, bool copy_back = true, const RadixSource* from = nullptr);

// fused introduce (pull, one-column child) + forget of the child's column
// (fused.hip); in == nullptr means the child is a leaf synthesised from the
// colouring.  gcount: output entries per (b, v); icount: introduce entries.
void launch_edge_count(const DevTable* in, const uint64_t* rstart, const uint64_t* rend, int B, DevGraph g,
                       const uint8_t* colors, int degF_u, int degF_child, Lay LO, uint32_t* gcount, uint32_t* icount,
                       hipStream_t s);
void launch_edge_emit(const DevTable* in, const uint64_t* rstart, const uint64_t* rend, int B, DevGraph g,
                      const uint8_t* colors, int degF_u, int degF_child, const uint64_t* goff, DevTable& out,
                      uint32_t* ovf, hipStream_t s);
// Introduce u in pull form over a leaf child, neither table read (the leaf
// with mask degF_leaf is never stored): tiles of (colouring, directed edge)
// items; the count pass writes survivors per tile (leaf_pull_tiles of them),
// the emit pass the sorted output from the tiles' exclusive offsets.
uint64_t leaf_pull_tiles(const DevGraph& g, int B);
void launch_leaf_pull_count(DevGraph g, int B, int degF_u, int degF_leaf, const uint8_t* colors, Lay LO,
                            uint32_t* tcount, hipStream_t s);
void launch_leaf_pull_emit(DevGraph g, int B, int degF_u, int degF_leaf, const uint8_t* colors,
                           const uint64_t* toff, DevTable& out, hipStream_t s);
// The introduce after such a pull whose new vertex is adjacent in F to both
// of its vertices: the triangles (v, a, c), edge (v, a) in CSR order, c from
// the edge's common-neighbour list (cn_off, cn_col; total list positions),
// distinct colours, degree masks m0, m1, m2 per column; tri_tiles tiles.
uint64_t tri_tiles(uint64_t total, int B);
void launch_tri_count(DevGraph g, const uint64_t* cn_off, const int32_t* cn_col, uint64_t total, int B, int m0,
                      int m1, int m2, const uint8_t* colors, Lay LO, uint32_t* tcount, hipStream_t s);
void launch_tri_emit(DevGraph g, const uint64_t* cn_off, const int32_t* cn_col, uint64_t total, int B, int m0,
                     int m1, int m2, const uint8_t* colors, const uint64_t* toff, DevTable& out, hipStream_t s);

// enumeration support (enumerate.hip)
// forget: dst[e] = output position of child entry e
void launch_forget_dst(const DevTable& in, const uint64_t* gstart, uint64_t G, const uint64_t* goff, uint64_t* dst,
                       hipStream_t s);
// join: admissible pairs per group (count pass), then (dst, a, d) per pair
void launch_join_pairs_count(const DevTable& y, const DevTable& z, const uint64_t* gstart, uint64_t G, int32_t n,
                             const uint8_t* colors, uint32_t* pcount, hipStream_t s);
void launch_join_pairs_emit(const DevTable& y, const DevTable& z, const uint64_t* gstart, uint64_t G, int32_t n,
                            const uint8_t* colors, const uint64_t* goff, const uint64_t* poff, uint64_t* pdst,
                            uint64_t* pa, uint64_t* pd, hipStream_t s);
// segment starts of a sorted uint64 array: starts[key[j]] = first j
void launch_segment_starts(const uint64_t* keys, uint64_t n, uint64_t nseg, uint64_t* starts, hipStream_t s);
// gathers: out[j] = src[idx[j]]; out[j] = a[i[j]] * b[k[j]]
void launch_gather_u64(const uint64_t* src, const uint64_t* idx, uint64_t n, uint64_t* out, hipStream_t s);
void launch_iota(uint64_t* p, uint64_t n, hipStream_t s);
void launch_gather_product(const uint64_t* a, const uint64_t* ia, const uint64_t* b, const uint64_t* ib, uint64_t n,
                           uint64_t* out, hipStream_t s);

// one descriptor per plan step for the row decoder
enum EnumKind { EK_LEAF = 0, EK_INTRO = 1, EK_FORGET = 2, EK_JOIN = 3, EK_RESORT = 4 };
struct EnumStep {
    int kind;       // EnumKind
    int in0, in1;   // input steps
    int ucol;       // column of the step's vertex in its output (leaf / introduce), else -1
    int u;          // pattern vertex of that column
    Lay lay;
    const void* keys;
    const uint64_t* cnt;
    const uint64_t* src;     // introduce / resort: child entry of every output entry
    const uint64_t* seg;     // forget / join: contributor segment starts, per output entry (+1)
    const uint64_t* wcum;    // forget / join: exclusive prefix sums of contributor weights
    const uint64_t* ca;      // forget: contributing child entry; join: first-child entry
    const uint64_t* cb;      // join: second-child entry
};
// decodes rows r in [0, R): starting entry by prefix sums rcum over the
// first entries of the root's child table, then descends every step
void launch_unrank(const EnumStep* steps, int root_step, const uint64_t* rcum, uint64_t E, uint64_t R, int nF,
                   int vb, int rkw, void* rowkeys, uint32_t* err, hipStream_t s);

// root: counts[bid] += cnt for every entry of a one-column table; per-vertex optional
// Dense one-column tables (slots.hip).  Slot r of colour-set size s is the
// r-th mask of popcount s - 1 (increasing) over the k - 1 colours other than
// the bag vertex's; R(s) = C(k - 1, s - 1) slots per (colouring, vertex).
constexpr int kSlotBlock = 256;
constexpr int kSlotBits = 11;  // k - 1 <= 11
struct SlotGrid {
    int32_t n = 0;
    int B = 0, R = 1;
    int upb = 0;        // units (colouring, vertex) per block and thread row when R <= kSlotBlock, else 0
    int m = 1;          // vertices per thread (upb * m per block)
    int bpu = 0;        // blocks per unit when R > kSlotBlock
    uint32_t nbx = 0;   // blocks per colouring
    bool xcd = false;   // colourings dealt to XCDs in turn
    uint64_t blocks = 0;
};
SlotGrid slot_grid(int32_t n, int B, int R, int m_max);
// A slot table on the device: counts mod 2^64 as two planes of 32-bit words
// (low, high), presence bytes, each [B][n][R], and wide[b], set when some
// count of colouring b is 2^32 or more (then the high plane matters).  A
// table whose counts a bound keeps below 2^32 has no high plane (hi null),
// and one whose counts cannot wrap has no presence bytes (flag null: an
// entry is present iff its count is not 0).
struct SlotArrays {
    uint32_t* lo = nullptr;
    uint32_t* hi = nullptr;
    uint8_t* flag = nullptr;
    uint32_t* wide = nullptr;
    int R = 0;
};
// vertices per thread with which a join block stages its children's rows in LDS (0: none fit)
int slot_join_m(int R_out, int R_y, int R_z, int nsplit);
std::vector<uint16_t> slot_rank_tables();  // rank[2^11] then unrank[2^11], by popcount
int slot_unrank_offset(int popcount);
// Slot kernels store per-block partial entry counts (introduce entries,
// output entries) at part[2L], part[2L + 1]; launch_slot_sum adds those of
// `blocks` blocks into out[0], out[1].
void launch_slot_sum(const uint64_t* part, uint64_t blocks, uint64_t* out, hipStream_t s);
// the partials of up to kSlotSumSteps steps, each in its own segment of part
// (off[i] words from the start, blocks[i] blocks), added into nsz[2 step[i] ..]
constexpr int kSlotSumSteps = 96;
struct SlotSums {
    uint32_t n = 0;
    uint32_t step[kSlotSumSteps];
    uint64_t off[kSlotSumSteps];
    uint64_t blocks[kSlotSumSteps];
};
void launch_slot_sums(const uint64_t* part, const SlotSums& S, uint64_t* nsz, hipStream_t s);
void launch_slot_leaf(const SlotGrid& G, DevGraph g, int degF, SlotArrays out, uint64_t* part, hipStream_t s);
// Packed child slots of an edge step, for k <= kSlotPackK: the entry for
// output colour-set size p + 1, bag colour cv and output slot r (index
// slot_pack_offset(k, p) + cv C(k - 1, p) + r) holds in byte c, for every
// colour c of C - {cv}, 0x80 | the child's slot of C - {cv} (whose own bag
// colour is c); the other bytes are 0.
constexpr int kSlotPackK = 8;
std::vector<uint64_t> slot_pack_tables();
size_t slot_pack_offset(int k, int p);
// Pushed edge steps (k <= kSlotPushK; the list of one colour pair, at most
// C(8, 4) = 70 slots, and all k^2 lists fit a block's LDS): for child
// colour-set size p + 1, child
// bag colour cy and output bag colour cv != cy, entry (cy k + cv) W + w of
// the block at slot_push_offset(k, p), W = C(k - 2, p), holds the w-th child
// slot r whose set leaves cv out, | the output slot of that set plus cv << 16.
constexpr int kSlotPushK = 10;
std::vector<uint32_t> slot_push_tables();
size_t slot_push_offset(int k, int p);
// in.lo == nullptr: the child is a leaf (count 1 per vertex passing
// degF_child).  pack: the entries of (k, p) above, or null (ranks from the
// rank tables).  in_narrow: every count of the child is known to be below
// 2^32; in_exact: no count of the child can have wrapped.  out.wide must be cleared beforehand.
void launch_slot_edge(SlotArrays in, const SlotGrid& G, DevGraph g, const uint8_t* colors, int k, int degF_u,
                      int degF_child, const uint16_t* rank, const uint16_t* unrank, int uoff, const uint64_t* pack,
                      bool in_narrow, bool in_exact, SlotArrays out, uint64_t* part, uint32_t* ovf, hipStream_t s);
// Two introduce-over-a-leaf steps at one bag vertex and their join, with the
// children's tables never stored: out gets the join's table (colour sets of
// 3), part_a / part_c / part_j the per-block entry partials of the two
// children (introduce and forget) and of the join.  k >= 4.
void launch_slot_leaf_join(const SlotGrid& G, DevGraph g, const uint8_t* colors, int k, int degF_u, int degF_a,
                           int degF_c, const uint16_t* unrank, SlotArrays out, uint64_t* part_a, uint64_t* part_c,
                           uint64_t* part_j, hipStream_t s);
// Joins computed in the epilogue of the push form of an edge step (its
// child E), at the same bag vertex, with leaves hanging off that vertex (no
// neighbour degree mask; no count of the joins can wrap).  E's table is not
// stored.  chain = 0: one join of E with the fused join of two leaves (its
// counts 2 h1 h2 below 2^32).  chain = 1: E joined with one leaf; chain =
// 2: that result (not stored) joined with a second leaf.
struct PushJoin {
    int chain = 0;
    const uint32_t* splits = nullptr;  // the (last) join's split table (slot_split_tables)
    int nsplit = 0, sstride = 0;
    int lj_is_y = 0;                   // chain 0: the leaf join is the join's first child
    const uint16_t* unrank = nullptr;  // chain 0: colour pairs, unrank tables at slot_unrank_offset(2)
    // chain >= 1: the first join (E with a leaf): split table, slots of its
    // output, E (chain 2: that output) as the first child of each join
    const uint32_t* splits1 = nullptr;
    int nsplit1 = 0, sstride1 = 0, r1 = 0;
    int e_is_y1 = 0, e_is_y2 = 0;
    // set by the launcher: the epilogue's rows, its split rows, fit the
    // push kernel's chunk arrays
    int rows_static = 0, spl_static = 0;
    SlotArrays out;                    // the last join's table
    // per-block entry partials of E, the two leaves (chain 1: both the one
    // leaf), the leaf join (chain >= 1: the first join), the last join
    uint64_t* part_e = nullptr;
    uint64_t* part_a = nullptr;
    uint64_t* part_c = nullptr;
    uint64_t* part_lj = nullptr;
    uint64_t* part_j = nullptr;
};
// The same step pushed from the child's rows into LDS accumulators.  s_in:
// the child's colour-set size; push: the entries of (k, s_in - 1) above;
// wide: 64-bit accumulators (else every output count is below 2^32).  pj
// (optional, only where no count can wrap): the step's only reader is that
// join, computed instead of storing out (then out and part are unused).
// wrap: the step's counts may wrap (needs wide, no pj, out's presence bytes
// and the overflow flags ovf, which a wrapped sum raises); else no count of
// this or any table below can wrap (then every child table is exact).
void launch_slot_edge_push(SlotArrays in, int s_in, const SlotGrid& G, DevGraph g, const uint8_t* colors, int k,
                           int degF_u, const uint32_t* push, bool wide, SlotArrays out, uint64_t* part,
                           const PushJoin* pj, bool wrap, uint32_t* ovf, hipStream_t s);
// Dynamic LDS bytes of that launch (pj: its sizes chain, r1, nsplit1, nsplit
// and out.R are used); a launch needs at most kPushLdsMax (64 KiB per block
// less the kernel's static arrays).
size_t slot_push_lds(int k, int s_in, const SlotGrid& G, bool wide, const PushJoin* pj, bool wrap = false);
constexpr size_t kPushLdsMax = 54 * 1024;
constexpr size_t kSlotJoinLds = 48 << 10;  // LDS bytes a join block may stage its children's rows in
// split table rows of (p, q) (see slots.hip) start at slot_split_offset(p, q);
// row stride C(kSlotBits, p)
std::vector<uint32_t> slot_split_tables();
int slot_split_offset(int p, int q);
// nowrap: both children's counts are known to be below 2^32 and the output's
// below 2^64 (only honoured when the rows are staged); in_exact: no count of
// either child can have wrapped
void launch_slot_join(SlotArrays y, SlotArrays z, const uint32_t* splits, int nsplit, int sstride, bool nowrap,
                      bool in_exact, const SlotGrid& G, SlotArrays out, uint64_t* part, uint32_t* ovf, hipStream_t s);
// rpart: slot_root_partials(n, B) words of scratch
uint64_t slot_root_partials(int32_t n, int B);
// Also reduces the steps' entry partials listed in sums (as launch_slot_sums)
// in the same final launch.
void launch_slot_root(SlotArrays in, int s_in, int32_t n, int B, const uint8_t* colors, const uint16_t* unrank,
                      uint64_t* rpart, uint64_t* counts, uint32_t* ovf, uint64_t* per_vertex, uint32_t* csets,
                      int cwords, const uint64_t* part, const SlotSums& sums, uint64_t* nsz, hipStream_t s);

// root: per colouring the sum of the entries (counts), a sticky overflow flag,
// optionally the per-image sums of the bag vertex, and a bitmap of the colour
// sets present (cwords 32-bit words per colouring)
void launch_root(const DevTable& in, int32_t n, uint64_t* counts, uint32_t* ovf, uint64_t* per_vertex,
                 uint32_t* csets, int cwords, hipStream_t s);

}  // namespace ccg
