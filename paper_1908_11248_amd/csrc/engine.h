// Runtime objects behind the C ABI: context, device arena, resident graph,
// colourings, decompositions, and the DP executor.
#pragma once

#include <hip/hip_runtime.h>

#include <functional>
#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <unordered_map>
#include <vector>

#include "internal.h"
#include "kernels.h"

namespace ccg {

struct CcError {
    int code;
    std::string msg;
    bool budget = false;  // CC_ERANGE raised by the per-table work budget
};

[[noreturn]] void fail(int code, const std::string& msg);
void hip_check(hipError_t e, const char* what);

// First-fit allocator over one device buffer, shared by every lane of a
// context (calls are serialised by a mutex).  A lane releases a block only
// after the kernels of that lane that use it were enqueued; a block released
// by a lane is reused by the same lane in stream order, and by another lane
// only after the owner synchronised its stream (every run synchronises its
// stream before it returns its scratch and tables).
class Arena {
   public:
    void init(char* base, size_t size);
    void* alloc(size_t bytes);
    void release(void* p);
    size_t in_use() const { return in_use_; }
    size_t free_bytes() {
        std::lock_guard<std::mutex> g(mu_);
        return size_ - in_use_;
    }
    size_t peak() const { return peak_; }
    size_t size() const { return size_; }
    void reset_peak() { peak_ = in_use_; }

   private:
    std::mutex mu_;
    char* base_ = nullptr;
    size_t size_ = 0, in_use_ = 0, peak_ = 0;
    std::map<size_t, size_t> free_;            // offset -> bytes
    std::unordered_map<size_t, size_t> live_;  // offset -> bytes
};

// Per-kernel timing with HIP events on the context's stream (enabled on
// request; resolved after the stream synchronises at the end of a call).
struct KernelStat {
    std::string name;
    uint64_t launches = 0;
    double ms = 0;
    double bytes = 0;  // algorithmic bytes summed over launches
};

class Profiler {
   public:
    bool on = false;
    std::string only;     // record only kernels of this name (empty: all)
    uint32_t every = 1;   // of those, one launch in `every`
    uint32_t seen_ = 0;
    void reset();
    // returns a handle of the recorded launch (-1: not recorded) whose bytes
    // set_bytes may still change before resolve()
    int begin(hipStream_t s, const char* name, double bytes);
    void set_bytes(int handle, double bytes);
    void end(hipStream_t s);
    void resolve();  // call after the stream has synchronised
    const std::vector<KernelStat>& stats() const { return stats_; }
    ~Profiler();

   private:
    struct Pending {
        int stat;
        double bytes;
        hipEvent_t a, b;
    };
    std::vector<KernelStat> stats_;
    std::map<std::string, int> index_;
    std::vector<Pending> pending_;
    std::vector<hipEvent_t> pool_;
    bool armed_ = false;  // begin() recorded the pending launch's first event
    hipEvent_t take();
};

// One independent execution lane: a stream, a pinned staging word for the
// sizes read back between steps, and the lane's kernel timings.
struct Lane {
    hipStream_t stream = nullptr;
    bool own_stream = false;
    uint64_t* pinned = nullptr;
    // pinned host words a run reads its results back into (a copy to
    // pageable memory would go through a staging buffer and wait for it)
    uint64_t* results = nullptr;
    size_t results_words = 0;
    Profiler prof;
    void create(hipStream_t given);
    void destroy();
    uint64_t* result_words(size_t words);  // at least `words`, kept until destroy
};

}  // namespace ccg

// Device buffers of freed colourings, kept for the next colouring of the
// same size (a hipMalloc and hipFree per colouring would stall every step).
// Shared with the colourings, so a colouring freed after its context returns
// its buffer to the device instead.
struct ColorPool {
    std::mutex mu;
    bool alive = true;
    struct Idle {
        size_t bytes;
        uint8_t* buf;
        hipEvent_t ready;
    };
    std::vector<Idle> idle;
    static constexpr size_t kMax = 8;
};

struct cc_context {
    int device = 0;
    std::shared_ptr<ColorPool> color_pool = std::make_shared<ColorPool>();
    void* arena_mem = nullptr;
    ccg::Arena arena;
    ccg::Lane main;  // the lane of the single-query calls
    std::vector<std::unique_ptr<ccg::Lane>> workers;  // lanes of batched and served queries
    std::vector<int64_t> last_sizes;
    int32_t last_chunks = 1;  // anchor-range chunks of the last single-query count
    uint64_t max_entries = 0;  // per-table budget (0: none)
    int batch_lanes = 0;       // lanes for cc_count_batch (0: tuned on first use)
    // schedule choices (cc_tune_batch / cc_set_schedule):
    int entry_factor = 3;      // entry-wise introduce when it walks < 1/entry_factor of the fixed column's rows
    int sort_above_k = 12;     // sorted-list forget and join add up by sorting when k exceeds this (else dense LDS)
    int group_min = 2;         // entry-wise introduces group entries with equal bag images at this many per group
    uint16_t* slot_tables = nullptr;  // device: rank[2048] then unrank[2048] (slots.hip)
    uint32_t* slot_splits = nullptr;  // device: join split tables (slots.hip)
    uint64_t* slot_pack = nullptr;    // device: packed child slots of edge steps, k <= kSlotPackK
    uint32_t* slot_push = nullptr;    // device: (child slot, output slot) lists of pushed edge steps, k <= kSlotPackK
    ccg::Lane& worker(size_t i);
};

struct cc_graph {
    cc_context* ctx = nullptr;
    int32_t n = 0;
    int64_t m2 = 0;
    int64_t* rp = nullptr;
    int32_t* col = nullptr;
    int32_t* esrc = nullptr;
    int32_t* heavy = nullptr;
    int32_t nheavy = 0;
    uint64_t* ehash = nullptr;  // edge set (kernels.h edge_key / edge_cell)
    uint8_t* deg8 = nullptr;    // [n] min(degree, 255)
    uint64_t ehmask = 0;
    std::vector<int64_t> sorted_deg;  // host copy, ascending
    std::vector<int64_t> host_rp;     // host copy of the row pointers (degree prefix sums)
    std::vector<int64_t> deg_mass;    // deg_mass[i] = sum of sorted_deg[i..n)
    double nb_degree = 0;             // mean degree of an edge's endpoint: sum d^2 / sum d
    double transitivity = 0;          // closed wedges / wedges (sampled)
    // walk tables of the distance-bounded introduce, built on first use:
    // ball_pre[e] = degrees of the neighbours before stored edge e in its row,
    // ball_w2[v] = deg(v) + the degrees of v's neighbours
    std::mutex ball_mu;
    uint64_t* ball_pre = nullptr;
    uint64_t* ball_w2 = nullptr;
    // common-neighbour index (built when an introduce first needs it):
    // cn_off[e] .. cn_off[e + 1] in cn_col are the common neighbours of the
    // endpoints of stored edge e, ascending
    uint64_t* cn_off = nullptr;
    int32_t* cn_col = nullptr;
    uint64_t cn_total = 0;  // cn_off[2m]: the lists' total length
    // wedge index (built when an introduce first needs it and the graph has
    // at most 2^28 neighbour pairs): a hash of the vertex pairs x < y with a
    // common neighbour (keys x << wd_vb | y in wd_hk, their run in wd_hv) over
    // the runs wd_start[r] .. wd_start[r + 1] of common neighbours in wd_mid
    uint64_t* wd_hk = nullptr;
    uint32_t* wd_hv = nullptr;
    uint64_t wd_mask = 0;
    uint64_t* wd_start = nullptr;
    int32_t* wd_mid = nullptr;
    int wd_vb = 0;
    bool wd_tried = false;
    // log2 of the largest homomorphism count of a tree plan's subtrees by
    // their size (prefix maxima), keyed by the plan's step structure
    std::map<std::string, std::vector<double>> hom_bounds;
    // vertices with degree >= d
    int64_t count_deg_at_least(int64_t d) const;
    // fraction of edge endpoints whose vertex has degree >= d
    double nb_fraction_at_least(int64_t d) const;
    ccg::DevGraph dev() const { return ccg::DevGraph{n, m2, rp, col, esrc, heavy, nheavy, ehash, ehmask, deg8}; }
};

struct cc_coloring {
    cc_context* ctx = nullptr;
    int32_t n = 0, k = 0, B = 0;
    uint8_t* colors = nullptr;  // [B][n] on the device
    size_t bytes = 0;           // of the buffer
    hipEvent_t ready = nullptr;  // recorded once the colours are written
    std::shared_ptr<ColorPool> pool;
};

struct cc_decomp {
    ccg::Decomp d;
    ccg::Plan plan;
};

namespace ccg {

struct RunResult;
// A run recorded into a HIP graph: the host work that turns the read-back
// words into results, to call after each replay has synchronised.
struct SlotCapture {
    std::function<void(RunResult*, std::vector<uint64_t>*)> finish;
};

struct RunRequest {
    const cc_graph* g = nullptr;
    const uint8_t* colors = nullptr;  // device [B][n]
    int B = 0, k = 0;
    const cc_decomp* dec = nullptr;
    bool degree_mask = true;
    bool sparse_only = false;  // never use dense one-column tables
    bool per_vertex = false;  // also the per-image split of the node below the root
    bool keep_tables = false;
    bool links = false;  // record the contributor index the row decoder needs (implies keep_tables)
    uint64_t max_entries = 0;  // fail with CC_ERANGE when a table would exceed this (0: no limit)
    // anchor-range chunk: only mappings with Phi(anchor_vertex) in
    // [anchor_lo, anchor_hi) are counted (anchor_hi < 0: no restriction)
    int anchor_vertex = 0;
    int32_t anchor_lo = 0, anchor_hi = -1;
    int chunk_depth = 0;  // halvings of the anchor range so far
    Arena* arena = nullptr;    // device memory of the run's tables and scratch (nullptr: the context's)
    bool no_alloc = false;     // make no device or pinned-host allocation (fail with CC_ERANGE instead)
    bool classic_expand = false;  // never the entry-wise introduce (tests compare both)
    SlotCapture* capture = nullptr;  // record the device work only (dense-table plans; the stream is capturing)
    // dense plans: log2 bounds of the counts by colour-set size, from an
    // earlier run of the same plan on the same graph (a captured run cannot
    // compute them: that needs a read-back)
    const std::vector<double>* slot_lb_in = nullptr;
};

// contributor index of one step's table (enumeration)
struct StepLinks {
    uint64_t* src = nullptr;   // introduce / resort
    uint64_t* seg = nullptr;   // forget / join: [N_out + 1]
    uint64_t* wcum = nullptr;  // forget / join: [contributors + 1]
    uint64_t* ca = nullptr;
    uint64_t* cb = nullptr;
};

struct RunResult {
    std::vector<uint64_t> counts;      // [B]
    std::vector<uint8_t> overflow;     // [B]
    std::vector<uint64_t> per_vertex;  // [B * n] if requested
    std::vector<DevTable> tables;      // per plan step, when kept (arena-owned)
    std::vector<StepLinks> links;      // per plan step, when recorded (arena-owned)
    std::vector<int64_t> node_sizes;   // per TD node: sum over colourings of |D_x|
    std::vector<uint32_t> root_sets;   // [B][words]: bitmap of the colour sets at the root
    size_t peak_bytes = 0;             // largest arena footprint of the run
    int chunks = 1;                    // anchor-range chunks the result was computed in
    bool dense = false;                // ran on dense one-column tables
    std::vector<double> slot_lb;       // dense runs: log2 bounds of the counts by colour-set size
};

void run_dp(cc_context* ctx, Lane& lane, const RunRequest& rq, RunResult* out);

// Degree and wedge statistics of a host graph for the memory estimate
// (host CSR with sorted rows; fills the statistics fields of g).
void graph_statistics(cc_graph* g, const std::vector<int64_t>& rp, const std::vector<int32_t>& col);
// Estimated entries per colouring of every plan step's table, and the peak
// arena bytes of a run over B colourings (tables live at once plus the
// working buffers of the step that needs most), from the plan and the
// graph's degree statistics.  A model, not a bound: used to admit queries.
struct MemEstimate {
    std::vector<double> entries;  // per plan step, one colouring
    double peak_bytes = 0;        // B colourings
    double total_entries = 0;     // sum over steps, B colourings
};
MemEstimate estimate_memory(const cc_graph* g, const cc_decomp* d, int k, int B);
// run_dp, split while a table exceeds the per-table budget or the arena
// (CC_ENOMEM) into waves of colourings (halves, recursively; colourings are
// independent), and a single colouring into anchor-range chunks: disjoint
// ranges of the image of pattern vertex 0, whose counts add mod 2^64 (carry
// sets the overflow flag), whose tables of nodes holding vertex 0 partition
// the unsplit tables and whose other tables repeat.  Results equal one run;
// fails only when a range of one vertex still does not fit.
void run_dp_waves(cc_context* ctx, Lane& lane, const RunRequest& rq, RunResult* out);
void release_tables(cc_context* ctx, RunResult* r);
// the first min(total, cap) mappings of one colouring in lexicographic order
void run_enumerate(cc_context* ctx, Lane& lane, const cc_graph* g, const uint8_t* colors, int k, const cc_decomp* dec,
                   uint64_t cap, std::vector<int32_t>* rows, uint64_t* n_rows, uint64_t* total);
uint64_t read_u64(Lane& lane, const uint64_t* dev);
Lay table_layout(int b, int32_t n, int B, int k);

}  // namespace ccg
