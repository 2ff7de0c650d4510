// DP executor: runs a decomposition's plan (leaf / introduce / forget / join
// steps in post-order, Sec. 3.1) over a batch of colourings on one stream.
#include <algorithm>
#include <cmath>
#include <cstring>

#include "engine.h"

ccg::Lane& cc_context::worker(size_t i) {
    while (workers.size() <= i) {
        workers.emplace_back(new ccg::Lane());
        workers.back()->create(nullptr);
        workers.back()->prof.on = main.prof.on;  // lanes made while profiling take part in it
        workers.back()->prof.only = main.prof.only;
        workers.back()->prof.every = main.prof.every;
    }
    return *workers[i];
}

int64_t cc_graph::count_deg_at_least(int64_t d) const {
    return int64_t(sorted_deg.end() - std::lower_bound(sorted_deg.begin(), sorted_deg.end(), d));
}

double cc_graph::nb_fraction_at_least(int64_t d) const {
    if (sorted_deg.empty() || deg_mass.empty() || deg_mass[0] == 0) return 0;
    const size_t i = size_t(std::lower_bound(sorted_deg.begin(), sorted_deg.end(), d) - sorted_deg.begin());
    return i >= deg_mass.size() ? 0.0 : double(deg_mass[i]) / double(deg_mass[0]);
}

namespace ccg {

void fail(int code, const std::string& msg) { throw CcError{code, msg}; }

void hip_check(hipError_t e, const char* what) {
    if (e != hipSuccess) fail(CC_EDEVICE, std::string(what) + ": " + hipGetErrorString(e));
}

// ---------------------------------------------------------------------------
// arena

void Arena::init(char* base, size_t size) {
    base_ = base;
    size_ = size;
    free_.clear();
    live_.clear();
    in_use_ = peak_ = 0;
    if (size) free_[0] = size;
}

void* Arena::alloc(size_t bytes) {
    std::lock_guard<std::mutex> guard(mu_);
    bytes = std::max<size_t>(256, (bytes + 255) & ~size_t(255));
    for (auto it = free_.begin(); it != free_.end(); ++it) {
        if (it->second < bytes) continue;
        size_t off = it->first, len = it->second;
        free_.erase(it);
        if (len > bytes) free_[off + bytes] = len - bytes;
        live_[off] = bytes;
        in_use_ += bytes;
        peak_ = std::max(peak_, in_use_);
        return base_ + off;
    }
    fail(CC_ENOMEM, "device arena exhausted: " + std::to_string(bytes) + " bytes requested, " +
                        std::to_string(size_ - in_use_) + " free of " + std::to_string(size_));
}

void Arena::release(void* p) {
    if (!p) return;
    std::lock_guard<std::mutex> guard(mu_);
    size_t off = size_t((char*)p - base_);
    auto it = live_.find(off);
    if (it == live_.end()) return;
    size_t len = it->second;
    live_.erase(it);
    in_use_ -= len;
    auto nx = free_.lower_bound(off);
    if (nx != free_.end() && nx->first == off + len) {  // merge with the next block
        len += nx->second;
        free_.erase(nx);
    }
    auto pv = free_.lower_bound(off);
    if (pv != free_.begin()) {
        --pv;
        if (pv->first + pv->second == off) {  // merge with the previous block
            pv->second += len;
            return;
        }
    }
    free_[off] = len;
}

// ---------------------------------------------------------------------------
// profiler

hipEvent_t Profiler::take() {
    if (!pool_.empty()) {
        hipEvent_t e = pool_.back();
        pool_.pop_back();
        return e;
    }
    hipEvent_t e;
    hip_check(hipEventCreate(&e), "hipEventCreate");
    return e;
}

void Profiler::reset() {
    resolve();
    stats_.clear();
    index_.clear();
}

void Profiler::set_bytes(int handle, double bytes) {
    if (handle >= 0 && size_t(handle) < pending_.size()) pending_[size_t(handle)].bytes = bytes;
}

int Profiler::begin(hipStream_t s, const char* name, double bytes) {
    armed_ = false;
    if (!on || (!only.empty() && only != name)) return -1;
    if (every > 1 && (seen_++ % every) != 0) return -1;
    armed_ = true;
    auto it = index_.find(name);
    int id;
    if (it == index_.end()) {
        id = int(stats_.size());
        index_[name] = id;
        stats_.push_back(KernelStat{name, 0, 0, 0});
    } else {
        id = it->second;
    }
    Pending p{id, bytes, take(), take()};
    hip_check(hipEventRecord(p.a, s), "hipEventRecord");
    pending_.push_back(p);
    return int(pending_.size()) - 1;
}

void Profiler::end(hipStream_t s) {
    if (!on || !armed_ || pending_.empty()) return;
    armed_ = false;
    hip_check(hipEventRecord(pending_.back().b, s), "hipEventRecord");
}

void Profiler::resolve() {
    for (auto& p : pending_) {
        float ms = 0;
        if (hipEventSynchronize(p.b) == hipSuccess && hipEventElapsedTime(&ms, p.a, p.b) == hipSuccess) {
            stats_[p.stat].launches++;
            stats_[p.stat].ms += ms;
            stats_[p.stat].bytes += p.bytes;
        }
        pool_.push_back(p.a);
        pool_.push_back(p.b);
    }
    pending_.clear();
}

Profiler::~Profiler() {
    for (auto& p : pending_) {
        pool_.push_back(p.a);
        pool_.push_back(p.b);
    }
    for (hipEvent_t e : pool_) (void)hipEventDestroy(e);
}

// ---------------------------------------------------------------------------

static int bits_for(uint64_t count) {  // bits to hold values 0 .. count-1
    int b = 0;
    while (b < 63 && (uint64_t(1) << b) < count) b++;
    return b;
}

Lay table_layout(int b, int32_t n, int B, int k) {
    Lay L;
    L.b = b;
    L.vb = std::max(1, bits_for(uint64_t(n)));
    L.kb = k;
    L.bb = bits_for(uint64_t(B));
    return L;
}

uint64_t read_u64(Lane& lane, const uint64_t* dev) {
    hip_check(hipMemcpyAsync(lane.pinned, dev, 8, hipMemcpyDeviceToHost, lane.stream), "hipMemcpyAsync");
    hip_check(hipStreamSynchronize(lane.stream), "hipStreamSynchronize");
    return lane.pinned[0];
}

void Lane::create(hipStream_t given) {
    if (given) {
        stream = given;
    } else {
        hip_check(hipStreamCreateWithFlags(&stream, hipStreamNonBlocking), "hipStreamCreate");
        own_stream = true;
    }
    hip_check(hipHostMalloc((void**)&pinned, 64, hipHostMallocDefault), "hipHostMalloc");
}

uint64_t* Lane::result_words(size_t words) {
    if (words > results_words) {
        if (results) (void)hipHostFree(results);
        results = nullptr;
        results_words = 0;
        const size_t n = std::max<size_t>(words, 1024);
        hip_check(hipHostMalloc((void**)&results, n * 8, hipHostMallocDefault), "hipHostMalloc");
        results_words = n;
    }
    return results;
}

void Lane::destroy() {
    if (stream) (void)hipStreamSynchronize(stream);
    if (pinned) (void)hipHostFree(pinned);
    if (results) (void)hipHostFree(results);
    results = nullptr;
    results_words = 0;
    if (own_stream && stream) (void)hipStreamDestroy(stream);
    pinned = nullptr;
    stream = nullptr;
}

namespace {

// Algorithmic bytes of one DP table entry with a b-vertex bag, the per-entry
// unit of the roofline figures: b int32 images, a 16-bit colour set, a
// uint64 count and a 16-bit colouring index (the packed keys here are
// narrower; counters report the bytes actually moved).
inline double entry_bytes(int b) { return 4.0 * b + 12.0; }
// algorithmic bytes of an LSD radix sort of n entries of layout L on the key
// bits from lo up: every 8-bit pass reads and writes each key and count once
// (the cost the roofline model charges a sort: 2 passes (key + payload))
inline double sort_bytes(uint64_t n, const Lay& L, int lo) {
    const int passes = (L.bits() - lo + 7) / 8;
    return 2.0 * double(std::max(passes, 0)) * double(n) * (double(L.key_bytes()) + 8.0);
}

struct Exec {
    Lane& lane;
    hipStream_t s;
    Arena& A;
    uint64_t max_entries;
    std::unordered_map<void*, size_t> live;  // everything this run holds in the arena
    std::vector<void*> pending;              // released, returned to the arena at the next synchronisation
    size_t held = 0, peak = 0;               // bytes held by this run (released blocks leave at once)

    void* raw(size_t bytes) {
        void* p = A.alloc(bytes);
        live[p] = bytes;
        held += bytes;
        peak = std::max(peak, held);
        return p;
    }
    template <class T>
    T* alloc(uint64_t count) {
        return (T*)raw(std::max<uint64_t>(count, 1) * sizeof(T));
    }
    // Kernels already enqueued on this lane may still use p, and other lanes
    // share the arena: the block goes back only after this lane synchronises.
    void release(const void* p) {
        if (!p) return;
        auto it = live.find(const_cast<void*>(p));
        if (it != live.end()) {
            held -= it->second;
            live.erase(it);
        }
        pending.push_back(const_cast<void*>(p));
    }
    void synced() {  // call right after the lane's stream synchronised
        for (void* p : pending) A.release(p);
        pending.clear();
    }
    void release_all() {  // after a synchronisation, on failure
        synced();
        for (auto& kv : live) A.release(kv.first);
        live.clear();
    }
    uint64_t read(const uint64_t* dev) {
        uint64_t v = read_u64(lane, dev);
        synced();
        return v;
    }

    DevTable table(Lay lay, uint64_t n) {
        if (max_entries && n > max_entries)
            throw CcError{CC_ERANGE,
                          "a DP table of " + std::to_string(n) + " entries exceeds the per-table budget of " +
                              std::to_string(max_entries),
                          true};
        DevTable t;
        t.lay = lay;
        t.n = n;
        t.keys = raw(std::max<uint64_t>(n, 1) * lay.key_bytes());
        t.cnt = alloc<uint64_t>(n);
        return t;
    }
    void drop(DevTable& t) {
        release(t.keys);
        release(t.cnt);
        t.keys = nullptr;
        t.cnt = nullptr;
    }
    template <class F>
    int timed(const char* name, double bytes, F&& launch) {
        const int h = lane.prof.begin(s, name, bytes);
        launch();
        lane.prof.end(s);
        return h;
    }

    // exclusive scan of n counts; returns offsets[n + 1] and the total
    uint64_t scan(const uint32_t* in, uint64_t n, uint64_t** offs) {
        *offs = alloc<uint64_t>(n + 1);
        uint64_t* tmp = (uint64_t*)raw(scan_tmp_bytes(n));
        timed("scan", 4.0 * n + 8.0 * (n + 1), [&] { launch_scan_u32(in, *offs, n, tmp, s); });
        release(tmp);
        return read(*offs + n);
    }

    // runs of equal key >> shift; returns G and starts[G + 1]
    uint64_t groups(const DevTable& t, int shift, uint64_t** starts) {
        if (!t.n) {
            *starts = alloc<uint64_t>(1);
            launch_fill_u64(*starts, 0, 1, s);
            return 0;
        }
        const uint64_t nt = head_tiles(t.n);
        uint64_t* tsum = alloc<uint64_t>(nt);
        timed("heads", double(t.n) * t.lay.key_bytes() + 8.0 * nt,
              [&] { launch_head_count(t.keys, t.lay.kw(), t.n, shift, tsum, s); });
        uint64_t* toff = alloc<uint64_t>(nt + 1);
        uint64_t* tmp = (uint64_t*)raw(scan_tmp_bytes(nt));
        timed("scan", 16.0 * nt + 8.0, [&] { launch_scan_u64(tsum, toff, nt, tmp, s); });
        release(tmp);
        const uint64_t G = read(toff + nt);
        *starts = alloc<uint64_t>(G + 1);
        timed("group_starts", double(t.n) * t.lay.key_bytes() + 8.0 * (nt + G + 1),
              [&] { launch_head_starts(t.keys, t.lay.kw(), t.n, shift, toff, *starts, s); });
        release(tsum);
        release(toff);
        return G;
    }
};

// sorts (keys, vals) by keys < nkeys (stable)
void sort_pairs(Exec& X, uint64_t* keys, uint64_t* vals, uint64_t n, uint64_t nkeys) {
    if (n <= 1) return;
    int bits = 1;
    while (bits < 63 && (uint64_t(1) << bits) < nkeys) bits++;
    uint64_t* k2 = X.alloc<uint64_t>(n);
    uint64_t* v2 = X.alloc<uint64_t>(n);
    void* tmp = X.raw(radix_tmp_bytes(n));
    radix_sort(keys, vals, k2, v2, n, 1, bits, 0, tmp, X.s);
    X.release(tmp);
    X.release(v2);
    X.release(k2);
}

int binom(int a, int b) {
    if (b < 0 || b > a) return 0;
    int64_t c = 1;
    for (int i = 0; i < b; i++) c = c * (a - i) / (i + 1);
    return int(c);
}

// Colour-set size s of every step's output when every table of the plan has a
// one-vertex bag (leaves, fused introduce+forget pairs, one-vertex joins);
// false otherwise.
bool slot_plan(const Plan& plan, const std::vector<char>& fuse, std::vector<int>* sz) {
    const size_t S = plan.steps.size();
    sz->assign(S, 0);
    for (size_t i = 0; i < S; i++) {
        const Step& st = plan.steps[i];
        if (st.kind == S_LEAF) {
            (*sz)[i] = 1;
        } else if (fuse[i]) {
            (*sz)[i] = (*sz)[st.in0] + 1;
            (*sz)[i + 1] = (*sz)[i];
            i++;
        } else if (st.kind == S_JOIN && st.b_out == 1) {
            (*sz)[i] = (*sz)[st.in0] + (*sz)[st.in1] - 1;
        } else {
            return false;
        }
    }
    return plan.root_child >= 0 && plan.steps[plan.root_child].b_out == 1;
}

// Peak bytes of the dense tables of a slot plan, in step order.
uint64_t slot_peak_bytes(const Plan& plan, const std::vector<char>& fuse, const std::vector<char>& virt,
                         const std::vector<int>& sz, uint64_t units, int k) {
    const size_t S = plan.steps.size();
    std::vector<int> uses(S, 0);
    for (const Step& st : plan.steps) {
        if (st.in0 >= 0) uses[st.in0]++;
        if (st.in1 >= 0) uses[st.in1]++;
    }
    auto bytes = [&](size_t i) { return units * uint64_t(binom(k - 1, sz[i] - 1)) * 9u + 512; };
    uint64_t live = 0, peak = 0;
    for (size_t i = 0; i < S; i++) {
        const Step& st = plan.steps[i];
        if (virt[i]) continue;
        size_t o = fuse[i] ? i + 1 : i;
        live += bytes(o);
        peak = std::max(peak, live);
        for (int in : {st.in0, st.in1})
            if (in >= 0 && !virt[in] && --uses[in] == 0) live -= bytes(size_t(in));
        if (fuse[i]) i++;
    }
    return peak;
}

struct SlotTab {
    SlotArrays a;  // counts (two 32-bit planes), presence bytes, wide flags, R
    int s = 0;     // colour-set size
};

// Runs a slot plan on dense one-column tables (slots.hip): no count passes,
// scans or host round trips between steps.  Fills counts, flags and node
// sizes like the sparse path; the per-table budget is checked on the sizes
// afterwards (same outcome as the check before each sparse allocation).
void run_slots(cc_context* ctx, Exec& X, const RunRequest& rq, const std::vector<char>& fuse,
               const std::vector<char>& virt, const std::vector<int>& sz, RunResult* out) {
    const Plan& plan = rq.dec->plan;
    const Decomp& dec = rq.dec->d;
    const DevGraph g = rq.g->dev();
    const int B = rq.B, k = rq.k;
    hipStream_t s = X.s;
    const size_t S = plan.steps.size();
    const uint64_t units = uint64_t(B) * uint64_t(g.n);
    std::vector<int> uses(S, 0);
    for (const Step& st : plan.steps) {
        if (st.in0 >= 0) uses[st.in0]++;
        if (st.in1 >= 0) uses[st.in1]++;
    }
    std::vector<SlotTab> tab(S);
    // Every count of a table whose pattern subtree has s vertices is at most
    // dmax^(s - 1): an embedding maps the subtree's vertices other than the
    // bag vertex, parent before child, to neighbours of their parents'
    // images.  log2 of that bound decides which arithmetic is exact.
    const double ldmax = rq.g->sorted_deg.empty() ? 0.0 : std::log2(double(std::max<int64_t>(1, rq.g->sorted_deg.back())));
    // lb[s]: log2 of a bound on every count of a table of colour-set size s:
    // the smaller of that degree bound and the largest homomorphism count of
    // the plan's subtrees of at most s vertices (slots.hip, count bounds),
    // which needs one read-back (so a captured run takes an earlier run's)
    std::vector<double> lb(size_t(k) + 2);
    for (size_t s2 = 0; s2 < lb.size(); s2++) lb[s2] = double(std::max(int(s2) - 1, 0)) * ldmax;
    if (rq.slot_lb_in && rq.slot_lb_in->size() == lb.size()) {
        lb = *rq.slot_lb_in;
    } else if (!rq.capture && !rq.no_alloc && g.n > 0) {
        // the bounds depend on the graph and the plan's step structure only:
        // computed once per (graph, structure)
        std::string key;
        for (size_t i = 0; i < S; i++) {
            const Step& st = plan.steps[i];
            key += std::to_string(int(st.kind)) + ":" + std::to_string(st.in0) + ":" + std::to_string(st.in1) + ":" +
                   std::to_string(int(fuse[i])) + ":" + std::to_string(sz[i]) + ";";
        }
        cc_graph* gm = const_cast<cc_graph*>(rq.g);
        std::vector<double> pm_size;
        {
            std::lock_guard<std::mutex> lk(gm->ball_mu);
            auto it = gm->hom_bounds.find(key);
            if (it != gm->hom_bounds.end()) pm_size = it->second;
        }
        if (pm_size.empty()) {
            std::vector<double*> h(S, nullptr);
            uint64_t* hmax = nullptr;
            try {
                hmax = X.alloc<uint64_t>(S);
                launch_fill_u64(hmax, 0, S, s);
                for (size_t i = 0; i < S; i++) {
                    const Step& st = plan.steps[i];
                    size_t o = i;
                    if (st.kind == S_LEAF) {
                        h[i] = X.alloc<double>(uint64_t(g.n));
                        launch_fill_u64(reinterpret_cast<uint64_t*>(h[i]), 0x3FF0000000000000ull, uint64_t(g.n), s);  // 1.0
                    } else if (fuse[i]) {
                        o = i + 1;
                        h[o] = X.alloc<double>(uint64_t(g.n));
                        launch_hom_spmv(g, h[size_t(st.in0)], h[o], s);
                        i++;
                    } else if (st.kind == S_JOIN) {
                        h[i] = X.alloc<double>(uint64_t(g.n));
                        launch_hom_mul(h[size_t(st.in0)], h[size_t(st.in1)], h[i], uint64_t(g.n), s);
                    }
                    if (h[o]) launch_hom_max(h[o], uint64_t(g.n), hmax + o, s);
                }
                uint64_t* hb = X.lane.result_words(S);
                hip_check(hipMemcpyAsync(hb, hmax, 8 * S, hipMemcpyDeviceToHost, s), "copy bounds");
                hip_check(hipStreamSynchronize(s), "hipStreamSynchronize");
                std::vector<double> by_size(lb.size(), 0.0);
                for (size_t i = 0; i < S; i++) {
                    if (!h[i]) continue;
                    double m;
                    std::memcpy(&m, &hb[i], 8);
                    const double l = m > 1.0 ? std::log2(m) + 1e-6 : 0.0;  // margin for rounding
                    by_size[size_t(sz[i])] = std::max(by_size[size_t(sz[i])], l);
                }
                double pm = 0.0;
                for (size_t s2 = 0; s2 < by_size.size(); s2++) {
                    pm = std::max(pm, by_size[s2]);
                    by_size[s2] = pm;
                }
                pm_size = by_size;
                std::lock_guard<std::mutex> lk(gm->ball_mu);
                gm->hom_bounds[key] = pm_size;
            } catch (const CcError& e) {
                if (e.code != CC_ENOMEM) throw;  // no room: the degree bound stands
            }
            for (double* x : h)
                if (x) X.release(x);
            if (hmax) X.release(hmax);
        }
        for (size_t s2 = 0; s2 < lb.size() && s2 < pm_size.size(); s2++) lb[s2] = std::min(lb[s2], pm_size[s2]);
    }
    out->slot_lb = lb;
    auto below = [&](int set, int bits) { return lb[size_t(set)] < double(bits) - 1e-9; };
    // A join whose two inputs are introduce-over-a-leaf steps (at its bag
    // vertex, used by nothing else) runs as one kernel from neighbourhood
    // colour histograms; those inputs are deferred (never stored).
    const bool one_sum_plan = S <= size_t(kSlotSumSteps);
    std::vector<char> defer(S, 0), ljoin(S, 0);
    auto leaf_edge = [&](int t) {
        return t >= 1 && fuse[size_t(t - 1)] && virt[size_t(plan.steps[size_t(t - 1)].in0)] && uses[size_t(t)] == 1;
    };
    if (one_sum_plan && k >= 4 && k <= 12)
        for (size_t i = 0; i < S; i++) {
            const Step& st = plan.steps[i];
            if (st.kind != S_JOIN || st.in0 == st.in1 || !leaf_edge(st.in0) || !leaf_edge(st.in1)) continue;
            if (plan.steps[size_t(st.in0 - 1)].degF != plan.steps[size_t(st.in1 - 1)].degF) continue;
            ljoin[i] = 1;
            defer[size_t(st.in0)] = defer[size_t(st.in1)] = 1;
        }
    // A join of such a fused leaf join with an edge step in the push form (at
    // the same bag vertex, both read by nothing else) runs in the edge step's
    // kernel (PushJoin) when nothing can wrap, the leaves have no neighbour
    // degree mask and 2 dmax^2 < 2^32: neither child table is stored.
    // pskip: steps computed by such a kernel, at the join's place.
    std::vector<int> pedge(S, -1);  // join -> its edge step (the forget)
    std::vector<char> pskip(S, 0);
    auto leaf_mask = [&](int t) {  // the neighbour degree mask of leaf edge t
        return rq.degree_mask ? plan.steps[size_t(plan.steps[size_t(t - 1)].in0)].degF : 0;
    };
    // an edge step's push kernel (child set s_in, output s_e) fits a block's
    // LDS with the epilogue pj (null: none)
    auto push_fits = [&](int s_in, int s_e, const PushJoin* pj, bool wrap = false) {
        const SlotGrid G = slot_grid(g.n, B, binom(k - 1, s_e - 1), 8);
        return slot_push_lds(k, s_in, G, !below(s_e, 32), pj, wrap) <= kPushLdsMax;
    };
    if (k <= kSlotPushK && g.n < (1 << 24) && 1.0 + 2.0 * ldmax < 32.0 - 1e-9)
        for (size_t i = 0; i < S; i++) {
            const Step& st = plan.steps[i];
            if (st.kind != S_JOIN || st.in0 == st.in1 || !below(sz[i], 64)) continue;
            for (int side = 0; side < 2; side++) {
                const int l = side ? st.in1 : st.in0, e = side ? st.in0 : st.in1;
                if (!ljoin[size_t(l)] || uses[size_t(l)] != 1 || e < 1 || !fuse[size_t(e - 1)] || uses[size_t(e)] != 1)
                    continue;
                const Step& ie = plan.steps[size_t(e - 1)];
                if (virt[size_t(ie.in0)] || defer[size_t(e)] || !below(sz[size_t(e)], 64) ||
                    binom(k - 1, sz[size_t(e)] - 1) > kSlotBlock || binom(k - 1, sz[size_t(ie.in0)] - 1) > kSlotBlock)
                    continue;
                const Step& L = plan.steps[size_t(l)];
                if (leaf_mask(L.in0) > 1 || leaf_mask(L.in1) > 1 || plan.steps[size_t(L.in0 - 1)].degF != ie.degF)
                    continue;
                PushJoin shape;
                shape.nsplit = binom(sz[i] - 1, (st.in0 == l ? 3 : sz[size_t(e)]) - 1);
                shape.out.R = binom(k - 1, sz[i] - 1);
                if (!push_fits(sz[size_t(ie.in0)], sz[size_t(e)], &shape)) continue;
                pedge[i] = e;
                pskip[size_t(e)] = pskip[size_t(l)] = 1;
                break;
            }
        }
    // Likewise an edge step in the push form joined with one leaf edge at its
    // bag vertex, and that join (read by nothing else) with a second one:
    // chain[i] = (edge step, first leaf, second leaf or -1, first join or -1)
    // at the join that launches it.
    struct Chain {
        int e = -1, lx = -1, ly = -1, mid = -1;
    };
    std::vector<Chain> chain(S);
    std::vector<int> reader(S, -1);
    for (size_t i = 0; i < S; i++)
        for (int in : {plan.steps[i].in0, plan.steps[i].in1})
            if (in >= 0) reader[size_t(in)] = int(i);
    auto push_edge = [&](int e) {  // an edge step this fusion can take
        if (e < 1 || !fuse[size_t(e - 1)] || uses[size_t(e)] != 1 || defer[size_t(e)] || pskip[size_t(e)]) return false;
        const Step& ie = plan.steps[size_t(e - 1)];
        return !virt[size_t(ie.in0)] && below(sz[size_t(e)], 64) && binom(k - 1, sz[size_t(e)] - 1) <= kSlotBlock &&
               binom(k - 1, sz[size_t(ie.in0)] - 1) <= kSlotBlock;
    };
    auto push_leaf = [&](int t, int e) {  // a leaf edge at e's bag vertex without a neighbour mask
        return leaf_edge(t) && !defer[size_t(t)] && !pskip[size_t(t)] && leaf_mask(t) <= 1 &&
               plan.steps[size_t(t - 1)].degF == plan.steps[size_t(e - 1)].degF;
    };
    if (one_sum_plan && k <= kSlotPushK && g.n < (1 << 24))
        for (size_t i = 0; i < S; i++) {
            const Step& st = plan.steps[i];
            if (st.kind != S_JOIN || st.in0 == st.in1 || pedge[i] >= 0 || pskip[i] || !below(sz[i], 64)) continue;
            int e = -1, lx = -1;
            if (push_edge(st.in0) && push_leaf(st.in1, st.in0)) {
                e = st.in0;
                lx = st.in1;
            } else if (push_edge(st.in1) && push_leaf(st.in0, st.in1)) {
                e = st.in1;
                lx = st.in0;
            } else {
                continue;
            }
            Chain c;
            c.e = e;
            c.lx = lx;
            size_t at = i;
            const int s_in = sz[size_t(plan.steps[size_t(e - 1)].in0)];
            PushJoin shape;  // the first join's sizes (the launch uses the same)
            shape.chain = 1;
            shape.r1 = binom(k - 1, sz[i] - 1);
            shape.nsplit1 = binom(sz[i] - 1, (st.in0 == e ? sz[size_t(e)] : 2) - 1);
            shape.out.R = shape.r1;
            const int i2 = reader[i];
            if (uses[i] == 1 && i2 >= 0 && plan.steps[size_t(i2)].kind == S_JOIN && below(sz[size_t(i2)], 64)) {
                const Step& s2 = plan.steps[size_t(i2)];
                const int ly = s2.in0 == int(i) ? s2.in1 : s2.in0;
                PushJoin two = shape;
                two.chain = 2;
                two.nsplit = binom(sz[size_t(i2)] - 1, (s2.in0 == int(i) ? sz[i] : 2) - 1);
                two.out.R = binom(k - 1, sz[size_t(i2)] - 1);
                if (ly != int(i) && ly != lx && push_leaf(ly, e) && push_fits(s_in, sz[size_t(e)], &two)) {
                    c.ly = ly;
                    c.mid = int(i);
                    at = size_t(i2);
                    pskip[i] = pskip[size_t(ly)] = 1;
                }
            }
            if (c.mid < 0 && !push_fits(s_in, sz[size_t(e)], &shape)) continue;
            chain[at] = c;
            pskip[size_t(e)] = pskip[size_t(lx)] = 1;
        }
    // per step: introduce entries, output entries, added up from per-block
    // partials (one scratch buffer, reused step after step on the stream)
    // partials: one segment per step (summed by one launch at the end when
    // the plan has at most kSlotSumSteps steps), then the root's
    uint64_t nsz_words = 2 * S, part_words = 0, seg_max = 0;
    for (size_t i = 0; i < S; i++)
        if (sz[i] > 0) {
            const uint64_t w = 2 * slot_grid(g.n, B, binom(k - 1, sz[i] - 1), 1).blocks;
            part_words += w;
            seg_max = std::max(seg_max, w);
        }
    const bool one_sum = one_sum_plan;
    if (!one_sum) part_words = seg_max;
    for (size_t i = 0; i < S; i++) {  // the two extra segments of a fused leaf join
        if (ljoin[i]) part_words += 4 * slot_grid(g.n, B, binom(k - 1, 2), 1).blocks;
        // and the five of a join in a push kernel, on that kernel's grid
        if (pedge[i] >= 0) part_words += 10 * slot_grid(g.n, B, binom(k - 1, sz[size_t(pedge[i])] - 1), 8).blocks;
        if (chain[i].e >= 0) part_words += 10 * slot_grid(g.n, B, binom(k - 1, sz[size_t(chain[i].e)] - 1), 8).blocks;
    }
    const uint64_t root_off = part_words;
    part_words += slot_root_partials(g.n, B);
    // One block for everything the host reads back and every flag, cleared by
    // one fill and copied back by one copy: counts (B words, written by the
    // root), node sizes (nsz_words), then as 32-bit words the overflow flags
    // (B), the root's colour-set bitmaps (B cwords) and, not copied back, the
    // wide flags of every step's table (B each).
    const int cwords = k >= 5 ? 1 << (k - 5) : 1;
    const uint64_t res_words = B + nsz_words + (uint64_t(B) * (1 + cwords) + 1) / 2;
    uint64_t* res = X.alloc<uint64_t>(res_words + (uint64_t(S) * B + 1) / 2);
    launch_fill_u64(res, 0, res_words + (uint64_t(S) * B + 1) / 2, s);
    uint64_t* counts = res;
    uint64_t* nsz = res + B;
    uint32_t* ovf = reinterpret_cast<uint32_t*>(nsz + nsz_words);
    uint32_t* csets = ovf + B;
    uint32_t* wide = reinterpret_cast<uint32_t*>(res + res_words);
    uint64_t* part_base = X.alloc<uint64_t>(part_words);
    uint64_t* part = part_base;  // this step's segment
    SlotSums sums;
    // after step i's kernel: record (or reduce) its partials, move to the next segment
    auto partials_done = [&](size_t i, uint64_t blocks) {
        if (one_sum) {
            sums.step[sums.n] = uint32_t(i);
            sums.off[sums.n] = uint64_t(part - part_base);
            sums.blocks[sums.n] = blocks;
            sums.n++;
            part += 2 * blocks;
        } else {
            launch_slot_sum(part, blocks, nsz + 2 * i, s);
        }
    };
    const uint16_t* rank = ctx->slot_tables;
    const uint16_t* unrank = ctx->slot_tables + (1 << kSlotBits);
    const double csr = double(B) * (9.0 * g.n + 4.0 * g.m2);
    const double csr_alg = double(B) * (8.0 * g.n + 4.0 * g.m2 + g.n);  // row pointers, columns, colours
    // a high plane only where counts can reach 2^32, presence bytes only
    // where they can wrap
    auto make = [&](int set, size_t step) {
        SlotTab t;
        t.s = set;
        t.a.R = binom(k - 1, set - 1);
        t.a.wide = wide + step * B;
        const uint64_t n = units * t.a.R;
        t.a.lo = X.alloc<uint32_t>(below(set, 32) ? n : 2 * n);
        t.a.hi = below(set, 32) ? nullptr : t.a.lo + n;
        t.a.flag = below(set, 64) ? nullptr : X.alloc<uint8_t>(n);
        return t;
    };
    auto drop = [&](SlotTab& t) {
        X.release(t.a.lo);
        X.release(t.a.flag);
        t = SlotTab();
    };
    // Identical subtrees (same shape, same degree masks) give identical
    // tables: a step whose signature was seen reuses that table.  phys maps a
    // step to the step that holds its table, refs counts that table's
    // remaining readers.
    std::vector<std::string> sig(S);
    std::map<std::string, size_t> seen;
    std::vector<size_t> phys(S);
    std::vector<int> refs(S, 0);
    for (size_t i = 0; i < S; i++) phys[i] = i;
    refs[plan.root_child] = 1;  // the root reads it last
    auto done_with = [&](int in) {
        if (in < 0 || virt[in]) return;
        const size_t t = phys[in];
        if (--refs[t] == 0) drop(tab[t]);
    };
    // true when an earlier step's table, still held, can serve step i (and
    // records the alias); otherwise step i becomes the holder of its signature
    auto reuse = [&](size_t i) {
        auto it = seen.find(sig[i]);
        if (it == seen.end() || refs[phys[it->second]] == 0) {  // new, or already released
            seen[sig[i]] = i;
            refs[i] += uses[i];
            return false;
        }
        phys[i] = phys[it->second];
        refs[phys[i]] += uses[i] + (i == size_t(plan.root_child) ? 1 : 0);
        tab[i] = tab[phys[i]];
        return true;
    };
    std::vector<std::pair<int, int>> node_of;  // (TD node, nsz index)
    std::vector<int> budgeted;                 // nsz indices of tables under the budget
    // recorded launches whose algorithmic bytes follow from the table sizes
    // read back at the end: entries of the tables read and written, at
    // entry_bytes(1) each, plus the graph bytes
    struct SlotBytes {
        int h;
        int in0, in1, out;  // steps whose tables the launch reads / writes (-1: none)
        double extra;
    };
    std::vector<SlotBytes> slot_bytes;
    for (size_t i = 0; i < S; i++) {
        const Step& st = plan.steps[i];
        if (virt[i]) {
            sig[i] = "V" + std::to_string(rq.degree_mask ? st.degF : 0);
            if (st.node >= 0)
                out->node_sizes[st.node] = int64_t(B) * rq.g->count_deg_at_least(rq.degree_mask ? st.degF : 0);
            continue;
        }
        if (fuse[i]) {
            const Step& f = plan.steps[i + 1];
            sig[i + 1] = "E(" + sig[st.in0] + "," + std::to_string(rq.degree_mask ? st.degF : 0) + ")";
            if (defer[i + 1] || pskip[i + 1]) {  // computed with its join; its sizes come from that kernel
                if (st.node >= 0) node_of.push_back({st.node, int(2 * i)});
                if (f.node >= 0) node_of.push_back({f.node, int(2 * i + 1)});
                budgeted.push_back(int(2 * i + 1));
                i++;
                continue;
            }
            if (reuse(i + 1)) {
                const size_t t = phys[i + 1];  // its fused pair is steps t - 1, t
                if (st.node >= 0) node_of.push_back({st.node, int(2 * (t - 1))});
                if (f.node >= 0) node_of.push_back({f.node, int(2 * (t - 1) + 1)});
                done_with(st.in0);
                i++;
                continue;
            }
            const bool leafc = virt[st.in0] != 0;
            const SlotTab in = leafc ? SlotTab() : tab[st.in0];
            SlotTab o = make(sz[i + 1], i + 1);
            const int degF_u = rq.degree_mask ? st.degF : 0;
            const int degF_c = rq.degree_mask ? plan.steps[st.in0].degF : 0;
            const uint64_t* pack = !leafc && k <= kSlotPackK && g.n < (1 << 24) && o.a.R <= kSlotBlock
                                       ? ctx->slot_pack + slot_pack_offset(k, o.s - 1)
                                       : nullptr;
            // push from the child's rows (a wrapping push when the step's
            // counts may reach 2^64): a (neighbour, child slot) pair of the
            // push is always useful
            const bool wrap = !below(o.s, 64);
            const bool push = !leafc && k <= kSlotPushK && g.n < (1 << 24) && o.a.R <= kSlotBlock &&
                              in.a.R <= kSlotBlock && push_fits(in.s, o.s, nullptr, wrap);
            // vertices per thread (measured on workload 2): the gather's
            // latency wants more blocks, the push's LDS accumulators longer rows
            SlotGrid G = slot_grid(g.n, B, o.a.R, leafc ? 4 : push ? 8 : 2);
            const char* kname = push ? "slot_edge_push" : leafc ? "slot_edge_leaf" : "slot_edge";
            const int h_fe = X.timed(kname, double(units) * 9.0 * (in.a.R + o.a.R) + csr, [&] {
                if (push)
                    launch_slot_edge_push(in.a, in.s, G, g, rq.colors, k, degF_u,
                                          ctx->slot_push + slot_push_offset(k, in.s - 1), !below(o.s, 32), o.a, part, nullptr,
                                          wrap, ovf, s);
                else
                    launch_slot_edge(in.a, G, g, rq.colors, k, degF_u, degF_c, rank, unrank,
                                     slot_unrank_offset(o.s - 1), pack, !leafc && below(in.s, 32),
                                     !leafc && below(in.s, 64), o.a, part, ovf, s);
            });
            slot_bytes.push_back({h_fe, leafc ? -1 : st.in0, -1, int(i + 1), csr_alg});
            partials_done(i, G.blocks);
            tab[i + 1] = o;
            if (st.node >= 0) node_of.push_back({st.node, int(2 * i)});
            if (f.node >= 0) node_of.push_back({f.node, int(2 * i + 1)});
            budgeted.push_back(int(2 * i + 1));
            done_with(st.in0);
            i++;
            continue;
        }
        if (st.kind == S_LEAF)
            sig[i] = "L" + std::to_string(rq.degree_mask ? st.degF : 0);
        else
            sig[i] = "J(" + std::min(sig[st.in0], sig[st.in1]) + "," + std::max(sig[st.in0], sig[st.in1]) + ")";
        if (pskip[i]) {  // a leaf join computed in its reader's push kernel
            if (st.node >= 0) node_of.push_back({st.node, int(2 * i + 1)});
            budgeted.push_back(int(2 * i + 1));
            continue;
        }
        if (pedge[i] >= 0) {
            seen[sig[i]] = i;  // the holder of its signature, computed here
            refs[i] += uses[i];
            const int e = pedge[i], l = st.in0 == e ? st.in1 : st.in0;
            const Step& ie = plan.steps[size_t(e - 1)];
            const Step& L = plan.steps[size_t(l)];
            const SlotTab in = tab[ie.in0];
            const int s_e = sz[size_t(e)];
            SlotTab o = make(sz[i], i);
            const int p = o.s - 1, q = (st.in0 == l ? 3 : s_e) - 1;
            SlotGrid G = slot_grid(g.n, B, binom(k - 1, s_e - 1), 8);
            PushJoin pj;
            pj.splits = ctx->slot_splits + slot_split_offset(p, q);
            pj.nsplit = binom(p, q);
            pj.sstride = binom(kSlotBits, p);
            pj.lj_is_y = st.in0 == l;
            pj.unrank = unrank + slot_unrank_offset(2);
            pj.out = o.a;
            pj.part_e = part;
            partials_done(size_t(e - 1), G.blocks);
            pj.part_a = part;
            partials_done(size_t(L.in0 - 1), G.blocks);
            pj.part_c = part;
            partials_done(size_t(L.in1 - 1), G.blocks);
            pj.part_lj = part;
            partials_done(size_t(l), G.blocks);
            pj.part_j = part;
            partials_done(i, G.blocks);
            const int h_pe = X.timed("slot_edge_push", double(units) * 9.0 * (in.a.R + o.a.R) + csr, [&] {
                launch_slot_edge_push(in.a, in.s, G, g, rq.colors, k, rq.degree_mask ? ie.degF : 0,
                                      ctx->slot_push + slot_push_offset(k, in.s - 1), !below(s_e, 32), SlotArrays(),
                                      nullptr, &pj, false, nullptr, s);
            });
            slot_bytes.push_back({h_pe, ie.in0, -1, int(i), csr_alg});
            tab[i] = o;
            if (st.node >= 0) node_of.push_back({st.node, int(2 * i + 1)});
            budgeted.push_back(int(2 * i + 1));
            done_with(ie.in0);
            continue;
        }
        if (chain[i].e >= 0) {
            seen[sig[i]] = i;  // the holder of its signature, computed here
            refs[i] += uses[i];
            const Chain& c = chain[i];
            const Step& ie = plan.steps[size_t(c.e - 1)];
            const SlotTab in = tab[ie.in0];
            const int s_e = sz[size_t(c.e)];
            SlotTab o = make(sz[i], i);
            SlotGrid G = slot_grid(g.n, B, binom(k - 1, s_e - 1), 8);
            const size_t j1 = c.mid >= 0 ? size_t(c.mid) : i;  // the join of E with the first leaf
            const int p1 = sz[j1] - 1, q1 = (plan.steps[j1].in0 == c.e ? s_e : 2) - 1;
            PushJoin pj;
            pj.chain = c.mid >= 0 ? 2 : 1;
            pj.splits1 = ctx->slot_splits + slot_split_offset(p1, q1);
            pj.nsplit1 = binom(p1, q1);
            pj.sstride1 = binom(kSlotBits, p1);
            pj.r1 = binom(k - 1, sz[j1] - 1);
            pj.e_is_y1 = plan.steps[j1].in0 == c.e;
            if (c.mid >= 0) {
                const int p = o.s - 1, q = (st.in0 == c.mid ? sz[size_t(c.mid)] : 2) - 1;
                pj.splits = ctx->slot_splits + slot_split_offset(p, q);
                pj.nsplit = binom(p, q);
                pj.sstride = binom(kSlotBits, p);
                pj.e_is_y2 = st.in0 == c.mid;
            }
            pj.out = o.a;
            pj.part_e = part;
            partials_done(size_t(c.e - 1), G.blocks);
            pj.part_a = part;
            partials_done(size_t(c.lx - 1), G.blocks);
            pj.part_c = pj.part_a;
            if (c.ly >= 0) {
                pj.part_c = part;
                partials_done(size_t(c.ly - 1), G.blocks);
            }
            pj.part_lj = part;
            partials_done(j1, G.blocks);
            if (c.mid >= 0) {
                pj.part_j = part;
                partials_done(i, G.blocks);
            }
            const int h_pe = X.timed("slot_edge_push", double(units) * 9.0 * (in.a.R + o.a.R) + csr, [&] {
                launch_slot_edge_push(in.a, in.s, G, g, rq.colors, k, rq.degree_mask ? ie.degF : 0,
                                      ctx->slot_push + slot_push_offset(k, in.s - 1), !below(s_e, 32), SlotArrays(),
                                      nullptr, &pj, false, nullptr, s);
            });
            slot_bytes.push_back({h_pe, ie.in0, -1, int(i), csr_alg});
            tab[i] = o;
            if (st.node >= 0) node_of.push_back({st.node, int(2 * i + 1)});
            budgeted.push_back(int(2 * i + 1));
            done_with(ie.in0);
            continue;
        }
        if (ljoin[i]) {
            // the holder of its signature, computed here (no alias: the
            // deferred inputs' sizes are produced by this kernel only)
            seen[sig[i]] = i;
            refs[i] += uses[i];
            const Step& ia = plan.steps[size_t(st.in0 - 1)];
            const Step& ic = plan.steps[size_t(st.in1 - 1)];
            SlotTab o = make(3, i);
            SlotGrid G = slot_grid(g.n, B, o.a.R, 8);  // histograms amortised over more vertices per block
            uint64_t* pa = part;
            partials_done(size_t(st.in0 - 1), G.blocks);
            uint64_t* pc = part;
            partials_done(size_t(st.in1 - 1), G.blocks);
            uint64_t* pj = part;
            partials_done(i, G.blocks);
            const int h_lj = X.timed("slot_leaf_join", double(units) * 9.0 * (2.0 * (k - 1) + o.a.R) + csr, [&] {
                launch_slot_leaf_join(G, g, rq.colors, k, rq.degree_mask ? ia.degF : 0,
                                      rq.degree_mask ? plan.steps[size_t(ia.in0)].degF : 0,
                                      rq.degree_mask ? plan.steps[size_t(ic.in0)].degF : 0, unrank, o.a, pa, pc, pj,
                                      s);
            });
            slot_bytes.push_back({h_lj, -1, -1, int(i), csr_alg});
            tab[i] = o;
            if (st.node >= 0) node_of.push_back({st.node, int(2 * i + 1)});
            budgeted.push_back(int(2 * i + 1));
            continue;
        }
        if (reuse(i)) {
            if (st.node >= 0) node_of.push_back({st.node, int(2 * phys[i] + 1)});
            if (st.kind == S_JOIN) {
                done_with(st.in0);
                done_with(st.in1);
            }
            continue;
        }
        if (st.kind == S_LEAF) {
            SlotTab o = make(1, i);
            SlotGrid G = slot_grid(g.n, B, 1, 4);
            const int h_lf = X.timed("slot_leaf", double(units) * 9.0 + 8.0 * g.n,
                                     [&] { launch_slot_leaf(G, g, rq.degree_mask ? st.degF : 0, o.a, part, s); });
            slot_bytes.push_back({h_lf, -1, -1, int(i), 8.0 * g.n + double(units)});
            partials_done(i, G.blocks);
            tab[i] = o;
        } else {  // one-vertex join
            const SlotTab& y = tab[st.in0];
            const SlotTab& z = tab[st.in1];
            SlotTab o = make(y.s + z.s - 1, i);
            const int p = o.s - 1, q = y.s - 1;
            const int nsplit = binom(p, q);
            SlotGrid G = slot_grid(g.n, B, o.a.R, std::min(4, std::max(1, slot_join_m(o.a.R, y.a.R, z.a.R, nsplit))));
            const int h_j = X.timed("slot_join", double(units) * 9.0 * (y.a.R + z.a.R + o.a.R), [&] {
                launch_slot_join(y.a, z.a, ctx->slot_splits + slot_split_offset(p, q), nsplit, binom(kSlotBits, p),
                                 below(y.s, 32) && below(z.s, 32) && below(o.s, 64), below(y.s, 64) && below(z.s, 64),
                                 G, o.a, part, ovf, s);
            });
            slot_bytes.push_back({h_j, st.in0, st.in1, int(i), 0.0});
            partials_done(i, G.blocks);
            tab[i] = o;
            done_with(st.in0);
            done_with(st.in1);
        }
        if (st.node >= 0) node_of.push_back({st.node, int(2 * i + 1)});
        budgeted.push_back(int(2 * i + 1));
    }
    hip_check(hipGetLastError(), "kernel launch");

    const SlotTab& rc = tab[plan.root_child];
    uint64_t* pv = nullptr;
    if (rq.per_vertex) pv = X.alloc<uint64_t>(units);  // every entry is written
    const int h_root = X.timed("slot_root", double(units) * 9.0 * rc.a.R, [&] {
        // with the steps' entry partials (one_sum) reduced in its last launch
        launch_slot_root(rc.a, rc.s, g.n, B, rq.colors, unrank, part_base + root_off, counts, ovf, pv, csets, cwords,
                         part_base, sums, nsz, s);
    });
    if (rq.no_alloc && res_words > X.lane.results_words)
        fail(CC_ERANGE, "the run's results (" + std::to_string(res_words) +
                            " words) exceed the preallocated read-back buffer of " +
                            std::to_string(X.lane.results_words) + " words");
    uint64_t* host = X.lane.result_words(res_words);
    hip_check(hipMemcpyAsync(host, res, 8 * res_words, hipMemcpyDeviceToHost, s), "copy results");
    if (pv) {
        out->per_vertex.assign(units, 0);
        hip_check(hipMemcpyAsync(out->per_vertex.data(), pv, 8 * units, hipMemcpyDeviceToHost, s), "copy per-vertex");
    }
    // Host side, once the stream has run: counts, flags and node sizes from
    // the read-back words.  A captured run (HIP graph) keeps it to call after
    // each replay.
    const std::vector<int64_t> prefilled = out->node_sizes;
    const uint64_t max_entries = rq.max_entries;
    const size_t n_nodes = dec.nodes.size();
    auto finish = [host, B, nsz_words, cwords, budgeted, node_of, prefilled, max_entries,
                   n_nodes](RunResult* r, std::vector<uint64_t>* sizes_out) {
        r->node_sizes = prefilled;
        r->counts.assign(host, host + B);
        const std::vector<uint64_t> sizes(host + B, host + B + nsz_words);
        const uint32_t* of = reinterpret_cast<const uint32_t*>(host + B + nsz_words);
        const uint32_t* cs = of + B;
        for (int j : budgeted)
            if (max_entries && sizes[j] > max_entries)
                throw CcError{CC_ERANGE,
                              "a DP table of " + std::to_string(sizes[j]) + " entries exceeds the per-table budget of " +
                                  std::to_string(max_entries),
                              true};
        for (auto& nd : node_of) r->node_sizes[nd.first] = int64_t(sizes[nd.second]);
        r->overflow.assign(B, 0);
        for (int b = 0; b < B; b++) r->overflow[b] = of[b] ? 1 : 0;
        int64_t nzr = 0;
        for (uint64_t i = 0; i < uint64_t(B) * cwords; i++) nzr += __builtin_popcount(cs[i]);
        r->node_sizes[n_nodes - 1] = nzr;
        r->root_sets.assign(cs, cs + uint64_t(B) * cwords);
        if (sizes_out) *sizes_out = sizes;
    };
    if (rq.capture) {  // graph capture: nothing may wait for the stream
        rq.capture->finish = finish;
        return;
    }
    hip_check(hipStreamSynchronize(s), "hipStreamSynchronize");
    X.synced();
    std::vector<uint64_t> sizes;
    finish(out, &sizes);
    // entries of step t's table: its size word (a fused introduce + forget
    // pair keeps it with the introduce), through aliases of identical tables
    auto entries_of = [&](int t) -> double {
        if (t < 0) return 0.0;
        const size_t p = phys[size_t(t)];
        const size_t w = (p > 0 && fuse[p - 1]) ? 2 * (p - 1) + 1 : 2 * p + 1;
        return w < sizes.size() ? double(sizes[w]) : 0.0;
    };
    for (const SlotBytes& sb : slot_bytes)
        X.lane.prof.set_bytes(sb.h, (entries_of(sb.in0) + entries_of(sb.in1) + entries_of(sb.out)) * entry_bytes(1) +
                                        sb.extra);
    X.lane.prof.set_bytes(h_root, entries_of(plan.root_child) * entry_bytes(1));
    X.lane.prof.resolve();
    X.release(pv);
    X.release(part_base);
    X.release(res);
    drop(tab[plan.root_child]);
    X.synced();
    out->peak_bytes = X.peak;
}

}  // namespace

void release_tables(cc_context* ctx, RunResult* r) {
    for (auto& t : r->tables) {
        ctx->arena.release(t.keys);
        ctx->arena.release(t.cnt);
        t.keys = nullptr;
        t.cnt = nullptr;
    }
    for (auto& l : r->links) {
        for (void* p : {(void*)l.src, (void*)l.seg, (void*)l.wcum, (void*)l.ca, (void*)l.cb}) ctx->arena.release(p);
        l = StepLinks();
    }
    r->tables.clear();
    r->links.clear();
}

void run_dp(cc_context* ctx, Lane& lane, const RunRequest& rq, RunResult* out) {
    const Plan& plan = rq.dec->plan;
    const Decomp& dec = rq.dec->d;
    const DevGraph g_all = rq.g->dev();
    const DevGraph& g = g_all;  // every step but those introducing the chunk's anchor vertex
    const int B = rq.B, k = rq.k;
    if (k < dec.n || k > kMaxColours)
        fail(CC_ERANGE, "colours k must satisfy n_F <= k <= " + std::to_string(kMaxColours));
    if (k > kDenseColours && rq.links)
        fail(CC_ERANGE, "enumeration needs k <= " + std::to_string(kDenseColours));
    if (B < 1) fail(CC_EINVAL, "no colourings");
    for (int b = 1; b <= plan.max_bag; b++)
        if (table_layout(b, g.n, B, k).bits() > 128)
            fail(CC_ERANGE, "packed key (colouring, bag images, colour set) exceeds 128 bits");

    Arena& arena = rq.arena ? *rq.arena : ctx->arena;
    Exec X{lane, lane.stream, arena, rq.max_entries};
    hipStream_t s = lane.stream;
    // the graph's common-neighbour index, built the first time an introduce
    // can use it (not in calls that may not allocate)
    auto cn_ready = [&]() -> bool {
        cc_graph* gm = const_cast<cc_graph*>(rq.g);
        std::lock_guard<std::mutex> lk(gm->ball_mu);
        if (!gm->cn_off && !rq.no_alloc && g_all.m2 > 0) {
            const uint64_t m2 = uint64_t(g_all.m2);
            uint32_t* cnt = X.alloc<uint32_t>(m2);
            X.timed("cn_count", 12.0 * double(m2), [&] { launch_cn_count(g_all, cnt, s); });
            uint64_t* offs;
            const uint64_t total = X.scan(cnt, m2, &offs);
            X.release(cnt);
            uint64_t* off = nullptr;
            int32_t* lists = nullptr;
            hip_check(hipMalloc(&off, 8 * (size_t(m2) + 1)), "hipMalloc");
            if (hipMalloc(&lists, 4 * std::max<size_t>(total, 1)) != hipSuccess) {
                (void)hipFree(off);
                X.release(offs);
                fail(CC_ENOMEM, "common-neighbour index");
            }
            hip_check(hipMemcpyAsync(off, offs, 8 * (size_t(m2) + 1), hipMemcpyDeviceToDevice, s), "copy");
            X.timed("cn_emit", 12.0 * double(m2) + 4.0 * double(total), [&] { launch_cn_emit(g_all, off, lists, s); });
            hip_check(hipStreamSynchronize(s), "hipStreamSynchronize");
            X.release(offs);
            gm->cn_off = off;
            gm->cn_col = lists;
            gm->cn_total = total;
        }
        return gm->cn_off != nullptr;
    };
    // the graph's wedge index, built the first time an introduce can use it
    // (not in calls that may not allocate, nor past 2^28 neighbour pairs;
    // without room in the arena the introduce walks adjacency rows instead)
    auto wedge_ready = [&]() -> bool {
        cc_graph* gm = const_cast<cc_graph*>(rq.g);
        std::lock_guard<std::mutex> lk(gm->ball_mu);
        if (gm->wd_start) return true;
        if (gm->wd_tried || rq.no_alloc || g_all.m2 == 0) return false;
        double pairs = 0;
        for (int32_t v = 0; v < gm->n; v++) {
            const double d = double(gm->host_rp[size_t(v) + 1] - gm->host_rp[size_t(v)]);
            pairs += d * (d - 1) / 2;
        }
        if (pairs > double(uint64_t(1) << 28)) {
            gm->wd_tried = true;
            return false;
        }
        const int vb = std::max(1, bits_for(uint64_t(gm->n)));
        const uint64_t m2 = uint64_t(g_all.m2);
        std::vector<void*> temps;
        uint64_t* hk = nullptr;
        uint32_t* hv = nullptr;
        uint64_t* wstart = nullptr;
        int32_t* mid = nullptr;
        try {
            uint32_t* cnt = X.alloc<uint32_t>(m2);
            temps.push_back(cnt);
            X.timed("wedge_count", 12.0 * double(m2), [&] { launch_wedge_count(g_all, cnt, s); });
            uint64_t* off;
            const uint64_t R = X.scan(cnt, m2, &off);
            temps.push_back(off);
            uint64_t* keys = X.alloc<uint64_t>(std::max<uint64_t>(R, 1));
            uint64_t* vals = X.alloc<uint64_t>(std::max<uint64_t>(R, 1));
            temps.push_back(keys);
            temps.push_back(vals);
            X.timed("wedge_emit", 16.0 * double(R), [&] { launch_wedge_emit(g_all, vb, off, keys, vals, s); });
            if (R > 1) {
                void* kb2 = X.raw(R * 8);
                uint64_t* vb2 = X.alloc<uint64_t>(R);
                void* tmp = X.raw(radix_tmp_bytes(R));
                temps.push_back(kb2);
                temps.push_back(vb2);
                temps.push_back(tmp);
                bool in_b = false;
                X.timed("radix_sort", 2.0 * double((2 * vb + 7) / 8) * double(R) * 16.0,
                        [&] { in_b = radix_sort(keys, vals, kb2, vb2, R, 1, 2 * vb, 0, tmp, s, false); });
                if (in_b) {
                    keys = static_cast<uint64_t*>(kb2);
                    vals = vb2;
                }
            }
            DevTable t;
            t.keys = keys;
            t.cnt = vals;
            t.n = R;
            t.lay = Lay{2, vb, 0, 0};
            uint64_t* starts;
            const uint64_t G = X.groups(t, 0, &starts);
            temps.push_back(starts);
            uint64_t cells = 16;
            while (cells < 2 * std::max<uint64_t>(G, 1)) cells <<= 1;
            if (hipMalloc(&hk, 8 * cells) != hipSuccess || hipMalloc(&hv, 4 * cells) != hipSuccess ||
                hipMalloc(&wstart, 8 * (G + 1)) != hipSuccess ||
                hipMalloc(&mid, 4 * std::max<uint64_t>(R, 1)) != hipSuccess)
                fail(CC_ENOMEM, "wedge index");
            launch_fill_u64(hk, kEdgeEmpty, cells, s);
            X.timed("wedge_hash", 28.0 * double(G), [&] { launch_wedge_hash(keys, starts, G, hk, hv, cells - 1, s); });
            hip_check(hipMemcpyAsync(wstart, starts, 8 * (G + 1), hipMemcpyDeviceToDevice, s), "copy");
            launch_u64_to_i32(vals, mid, R, s);
            hip_check(hipStreamSynchronize(s), "hipStreamSynchronize");
            for (void* p : temps) X.release(p);
            gm->wd_hk = hk;
            gm->wd_hv = hv;
            gm->wd_mask = cells - 1;
            gm->wd_start = wstart;
            gm->wd_mid = mid;
            gm->wd_vb = vb;
            return true;
        } catch (const CcError& e) {
            (void)hipStreamSynchronize(s);
            for (void* p : temps) X.release(p);
            for (void* p : {(void*)hk, (void*)hv, (void*)wstart, (void*)mid})
                if (p) (void)hipFree(p);
            gm->wd_tried = true;
            if (e.code != CC_ENOMEM) throw;
            return false;
        }
    };
    const size_t S = plan.steps.size();
    std::vector<DevTable> tab(S);
    std::vector<StepLinks> lk(S);
    const bool links = rq.links;
    const bool keep = rq.keep_tables || rq.links;
    std::vector<int> uses(S, 0);
    for (const Step& st : plan.steps) {
        if (st.in0 >= 0) uses[st.in0]++;
        if (st.in1 >= 0) uses[st.in1]++;
    }
    // Fusions (not when the contributor index is recorded): an introduce in
    // pull form over a one-column child followed by the forget of that column
    // runs as one gather (fused.hip); a leaf consumed only by such a step is
    // never materialised.  Nor is a leaf whose only reader is an introduce in
    // pull form with no edge test (lpull: its entries come from the edges).
    std::vector<char> fuse(S, 0), virt(S, 0), lpull(S, 0);
    if (!keep) {
        for (size_t i = 0; i + 1 < S; i++) {
            const Step& a = plan.steps[i];
            const Step& f = plan.steps[i + 1];
            if (a.kind == S_INTRO_PULL && a.b_in == 1 && a.nchk == 0 && f.kind == S_FORGET_LAST && f.in0 == int(i) &&
                uses[i] == 1 && k <= 12) {
                fuse[i] = 1;
                if (plan.steps[a.in0].kind == S_LEAF && uses[a.in0] == 1) virt[a.in0] = 1;
            }
        }
        for (size_t i = 0; i < S; i++) {
            const Step& a = plan.steps[i];
            if (fuse[i] || (i > 0 && fuse[i - 1]) || a.kind != S_INTRO_PULL || a.b_in != 1 || a.nchk != 0 ||
                rq.classic_expand || a.in0 < 0)
                continue;
            const Step& l = plan.steps[size_t(a.in0)];
            // (an anchor-range chunk restricting the leaf's image keeps the table)
            if (l.kind != S_LEAF || uses[size_t(a.in0)] != 1 || (rq.anchor_hi >= 0 && l.u == rq.anchor_vertex))
                continue;
            lpull[i] = 1;
            virt[size_t(a.in0)] = 1;
        }
    }
    // An introduce in push form over such a pull (its only reader), whose new
    // vertex is adjacent in F to both of the pull's vertices, at position 1
    // or 2: its entries are triangles of G, emitted from the common-neighbour
    // lists of the pull's edges (tri[j] = the pull; the pull's pairs are only
    // counted, for its node size).
    std::vector<int> tri(S, -1);
    std::vector<char> tskip(S, 0);
    if (!keep && rq.anchor_hi < 0 && g_all.n <= (1 << 27))
        for (size_t j = 0; j < S; j++) {
            const Step& st = plan.steps[j];
            if (st.kind != S_INTRO_PUSH || st.in0 < 0 || !lpull[size_t(st.in0)] || uses[size_t(st.in0)] != 1 ||
                st.b_in != 2 || (st.pos != 1 && st.pos != 2) || st.nchk != 1 || st.anchor < 0)
                continue;
            const int c0 = st.anchor, c1 = st.chk[0];
            if (!((c0 == 0 && c1 == 1) || (c0 == 1 && c1 == 0)) || !cn_ready()) continue;
            tri[j] = st.in0;
            tskip[size_t(st.in0)] = 1;
        }
    out->node_sizes.assign(dec.nodes.size(), 0);

    // dense one-column tables when the plan allows them and they fit a
    // quarter of the arena (an anchor-range chunk runs on sorted lists)
    const bool chunked = rq.anchor_hi >= 0;
    if (rq.capture && (rq.per_vertex || keep || chunked))
        fail(CC_EINVAL, "only plain counts can be captured into a graph");
    std::vector<int> sz;
    if (!keep && !rq.sparse_only && !chunked && k <= kDenseColours && slot_plan(plan, fuse, &sz)) {
        const uint64_t units = uint64_t(B) * uint64_t(g.n);
        // a quarter of the shared arena; all of a captured plan's own slice
        const uint64_t room = rq.capture ? arena.size() : arena.size() / 4;
        bool fits = slot_peak_bytes(plan, fuse, virt, sz, units, k) <= room;
        // 32-bit block indices; slot offsets within one colouring's table below
        // 2^28 (they share a staged word with a colour)
        bool shape_ok = true;
        for (size_t i = 0; i < S && shape_ok; i++)
            if (sz[i] > 0 && (slot_grid(g.n, B, binom(k - 1, sz[i] - 1), 1).blocks >= (uint64_t(1) << 32) ||
                              uint64_t(g.n) * binom(k - 1, sz[i] - 1) >= (uint64_t(1) << 28)))
                shape_ok = false;
        // too many colourings for dense tables, but one fits: waves of
        // colourings on dense tables beat one launch on sorted lists
        if (shape_ok && !fits && B > 1 && !rq.no_alloc && !rq.capture &&
            slot_peak_bytes(plan, fuse, virt, sz, uint64_t(g.n), k) <= room)
            throw CcError{CC_ERANGE, "dense tables of " + std::to_string(B) + " colourings exceed a quarter of the arena",
                          true};
        fits = fits && shape_ok;
        if (fits) {
            out->dense = true;
            try {
                run_slots(ctx, X, rq, fuse, virt, sz, out);
            } catch (...) {
                (void)hipStreamSynchronize(s);
                X.release_all();
                throw;
            }
            return;
        }
    }

    if (rq.capture)
        fail(CC_ERANGE, "only plans whose tables all fit as dense one-column tables (trees) can be captured");
    uint32_t* ovf = X.alloc<uint32_t>(B);
    launch_fill_u32(ovf, 0, B, s);
    try {
        for (size_t i = 0; i < S; i++) {
            const Step& st = plan.steps[i];
            // an anchor-range chunk restricts the image of the anchor vertex
            // where a step introduces it (a leaf, or an introduce possibly fused)
            DevGraph g = g_all;
            if (chunked && st.u == rq.anchor_vertex &&
                (st.kind == S_LEAF || st.kind == S_INTRO_PUSH || st.kind == S_INTRO_PULL)) {
                g.vlo = rq.anchor_lo;
                g.vhi = rq.anchor_hi;
            }
            if (virt[i]) {  // consumed by a fused edge step
                if (st.node >= 0)
                    out->node_sizes[st.node] = int64_t(B) * rq.g->count_deg_at_least(rq.degree_mask ? st.degF : 0);
                continue;
            }
            if (fuse[i]) {
                const Step& f = plan.steps[i + 1];
                Lay lo = table_layout(f.b_out, g.n, B, k);
                const bool leafc = virt[st.in0] != 0;
                const DevTable* in = leafc ? nullptr : &tab[st.in0];
                const int degF_u = rq.degree_mask ? st.degF : 0;
                const int degF_c = rq.degree_mask ? plan.steps[st.in0].degF : 0;
                uint64_t slots = uint64_t(B) * g.n;
                uint64_t *rstart = nullptr, *rend = nullptr;
                if (!leafc) {
                    rstart = X.alloc<uint64_t>(slots);
                    rend = X.alloc<uint64_t>(slots);
                    launch_fill_u64(rstart, 0, slots, s);
                    launch_fill_u64(rend, 0, slots, s);
                    X.timed("pull_index", double(in->n) * in->lay.key_bytes(),
                            [&] { launch_pull_index(*in, g.n, rstart, rend, s); });
                }
                uint32_t* gcount = X.alloc<uint32_t>(slots);
                uint32_t* icount = X.alloc<uint32_t>(slots);
                double in_bytes = leafc ? double(slots) : double(in->n) * (in->lay.key_bytes() + 8);
                X.timed("edge_count", in_bytes + 16.0 * slots + 8.0 * g.m2,
                        [&] { launch_edge_count(in, rstart, rend, B, g, rq.colors, degF_u, degF_c, lo, gcount, icount, s); });
                uint64_t* ioff;
                uint64_t NI = X.scan(icount, slots, &ioff);
                X.release(ioff);
                X.release(icount);
                uint64_t* goff;
                uint64_t N = X.scan(gcount, slots, &goff);
                X.release(gcount);
                DevTable& o = tab[i + 1];
                o = X.table(lo, N);
                if (N)
                    X.timed("edge_emit",
                            (leafc ? 0.0 : double(in->n) * entry_bytes(1)) + double(N) * entry_bytes(1) +
                                double(B) * (8.0 * g.n + 4.0 * g.m2 + g.n),
                            [&] { launch_edge_emit(in, rstart, rend, B, g, rq.colors, degF_u, degF_c, goff, o, ovf, s); });
                X.release(goff);
                X.release(rstart);
                X.release(rend);
                if (st.node >= 0) out->node_sizes[st.node] = int64_t(NI);
                if (f.node >= 0) out->node_sizes[f.node] = int64_t(N);
                if (!leafc && --uses[st.in0] == 0) X.drop(tab[st.in0]);
                i++;  // the forget step is done
                continue;
            }
            Lay lo = table_layout(st.b_out, g.n, B, k);
            IntroArgs ia;
            ia.pos = st.pos;
            ia.anchor = st.anchor;
            ia.nchk = st.nchk;
            for (int j = 0; j < 4; j++) ia.chk[j] = st.chk[j];
            ia.degF = rq.degree_mask ? st.degF : 0;
            DevTable& o = tab[i];
            if (tskip[i] || tri[i] >= 0) {
                const Step& pl = plan.steps[size_t(tskip[i] ? int(i) : tri[i])];  // the pull
                const int m_pull = rq.degree_mask ? pl.degF : 0;
                const int m_leaf = rq.degree_mask ? plan.steps[size_t(pl.in0)].degF : 0;
                int64_t node_n = 0;
                if (tskip[i]) {  // the pull's pairs: counted only
                    const uint64_t tiles = leaf_pull_tiles(g, B);
                    if (tiles) {
                        uint32_t* tcount = X.alloc<uint32_t>(tiles);
                        X.timed("leaf_pull_count", 10.0 * double(B) * double(g.m2),
                                [&] { launch_leaf_pull_count(g, B, m_pull, m_leaf, rq.colors, lo, tcount, s); });
                        uint64_t* toff;
                        node_n = int64_t(X.scan(tcount, tiles, &toff));
                        X.release(toff);
                        X.release(tcount);
                    }
                    // the per-table budget holds for this table too, as if it were stored
                    if (X.max_entries && uint64_t(node_n) > X.max_entries)
                        throw CcError{CC_ERANGE,
                                      "a DP table of " + std::to_string(node_n) +
                                          " entries exceeds the per-table budget of " + std::to_string(X.max_entries),
                                      true};
                } else {
                    // output columns: the pull's u, then (pos 1) u and the
                    // leaf vertex, or (pos 2) the leaf vertex and u
                    const int m_u = ia.degF;
                    const int m1 = st.pos == 1 ? m_u : m_leaf, m2 = st.pos == 1 ? m_leaf : m_u;
                    const cc_graph* gm = rq.g;
                    const uint64_t tiles = tri_tiles(gm->cn_total, B);
                    uint64_t N = 0;
                    uint64_t* toff = nullptr;
                    if (tiles) {
                        uint32_t* tcount = X.alloc<uint32_t>(tiles);
                        X.timed("tri_count", double(B) * (13.0 * double(g.m2) + 4.0 * double(gm->cn_total)), [&] {
                            launch_tri_count(g, gm->cn_off, gm->cn_col, gm->cn_total, B, m_pull, m1, m2, rq.colors, lo,
                                             tcount, s);
                        });
                        N = X.scan(tcount, tiles, &toff);
                        X.release(tcount);
                    }
                    o = X.table(lo, N);
                    if (N)
                        X.timed("tri_emit", double(B) * (13.0 * double(g.m2) + 4.0 * double(gm->cn_total)) +
                                                double(N) * entry_bytes(lo.b), [&] {
                            launch_tri_emit(g, gm->cn_off, gm->cn_col, gm->cn_total, B, m_pull, m1, m2, rq.colors, toff,
                                            o, s);
                        });
                    if (toff) X.release(toff);
                    node_n = int64_t(o.n);
                }
                if (st.node >= 0) out->node_sizes[st.node] = node_n;
                if (!keep) {
                    for (int in : {st.in0, st.in1})
                        if (in >= 0 && --uses[in] == 0) X.drop(tab[in]);
                }
                continue;
            }
            // Introduce by entries: candidates from the bag neighbour of u
            // whose image has the fewest neighbours, per child entry; used
            // when u has a further bag neighbour that the push or pull form
            // would test per item anyway (so those forms cannot prune by it
            // before walking a possibly huge row); the output is re-sorted
            // on (colouring, columns 0..pos).
            // It walks fewer candidates, but each one costs more (its own
            // degree, colour and edge tests instead of per-group ones): it is
            // taken when it walks under a third of the anchor column's rows.
            const bool entry_eligible =
                !links && !rq.classic_expand && tab[st.in0].n > 0 &&
                ((st.kind == S_INTRO_PULL && st.nchk >= 1) ||
                 (st.kind == S_INTRO_PUSH && std::any_of(st.chk, st.chk + st.nchk, [&](int c) { return c >= st.pos; })));
            // Distance-bounded introduce (u has no bag neighbour, but a bag
            // vertex at distance 2 in F): candidates within two steps of
            // that vertex's image instead of all of V(G).
            int ball_col = -1;
            if (st.kind == S_INTRO_PUSH && st.anchor < 0 && !links && !rq.classic_expand && tab[st.in0].n > 0 &&
                g.m2 < (int64_t(1) << 32)) {
                int dist[32];
                for (int v = 0; v < 32; v++) dist[v] = -1;
                int queue[32], qh = 0, qt = 0;
                dist[st.u] = 0;
                queue[qt++] = st.u;
                while (qh < qt) {
                    const int x = queue[qh++];
                    for (uint32_t m = dec.adj[x]; m; m &= m - 1) {
                        const int y = __builtin_ctz(m);
                        if (dist[y] < 0) {
                            dist[y] = dist[x] + 1;
                            queue[qt++] = y;
                        }
                    }
                }
                // the bag vertex nearest to u (smallest id on a tie); its
                // distance bounds the candidates (a ball of radius 2 here;
                // farther ones scan V(G))
                const Step& ch = plan.steps[size_t(st.in0)];
                int best_d = 1 << 20, best_v = 1 << 20;
                for (int j = 0; j < ch.b_out; j++) {
                    const int w = ch.cols[j];
                    if (w < 0 || dist[w] <= 0) continue;
                    if (dist[w] < best_d || (dist[w] == best_d && w < best_v)) {
                        best_d = dist[w];
                        best_v = w;
                        ball_col = j;
                    }
                }
                if (best_d != 2) ball_col = -1;
            }
            if (ball_col >= 0) {
                const DevTable& in = tab[st.in0];
                cc_graph* gm = const_cast<cc_graph*>(rq.g);
                {
                    std::lock_guard<std::mutex> lk(gm->ball_mu);
                    if (!gm->ball_pre) {
                        uint64_t *pre = nullptr, *w2 = nullptr;
                        hip_check(hipMalloc(&pre, 8 * size_t(std::max<int64_t>(g.m2, 1))), "hipMalloc");
                        if (hipMalloc(&w2, 8 * size_t(std::max<int32_t>(g.n, 1))) != hipSuccess) {
                            (void)hipFree(pre);
                            fail(CC_ENOMEM, "walk tables of the distance-bounded introduce");
                        }
                        launch_nbdeg_prefix(g_all, pre, w2, s);
                        hip_check(hipStreamSynchronize(s), "hipStreamSynchronize");
                        gm->ball_pre = pre;
                        gm->ball_w2 = w2;
                    }
                }
                uint32_t* slen = X.alloc<uint32_t>(in.n);
                X.timed("ball_seglen", double(in.n) * entry_bytes(in.lay.b),
                        [&] { launch_ball_seglen(in, ball_col, gm->ball_w2, slen, s); });
                uint64_t* soff;
                const uint64_t T = X.scan(slen, in.n, &soff);
                X.release(slen);
                const uint64_t tiles = expand_tiles(T);
                uint32_t* tcount = X.alloc<uint32_t>(tiles);
                uint16_t* pbits = X.alloc<uint16_t>(expand_pass_words(T));
                X.timed("ball_count", double(in.n) * entry_bytes(in.lay.b) + 5.0 * T,
                        [&] { launch_ball_count(in, ball_col, gm->ball_pre, soff, T, g, rq.colors, ia, tcount, pbits, s); });
                uint64_t* toff;
                const uint64_t Nd = X.scan(tcount, tiles, &toff);
                X.release(tcount);
                DevTable dup = X.table(lo, Nd);
                if (Nd)
                    X.timed("ball_emit", double(in.n) * entry_bytes(in.lay.b) + double(Nd) * entry_bytes(lo.b), [&] {
                        launch_ball_emit(in, ball_col, gm->ball_pre, soff, T, g, rq.colors, ia, toff, pbits, dup, s);
                    });
                X.release(pbits);
                X.release(toff);
                X.release(soff);
                if (Nd > 1) {
                    void* kb2 = X.raw(Nd * lo.key_bytes());
                    uint64_t* vb2 = X.alloc<uint64_t>(Nd);
                    void* tmp = X.raw(radix_tmp_bytes(Nd));
                    bool in_b = false;
                    X.timed("radix_sort", sort_bytes(Nd, lo, 0), [&] {
                        in_b = radix_sort(dup.keys, dup.cnt, kb2, vb2, Nd, lo.kw(), lo.bits(), 0, tmp, s, false);
                    });
                    if (in_b) {
                        std::swap(dup.keys, kb2);
                        std::swap(dup.cnt, vb2);
                    }
                    X.release(tmp);
                    X.release(vb2);
                    X.release(kb2);
                }
                uint64_t* starts;
                const uint64_t Gu = X.groups(dup, 0, &starts);
                o = X.table(lo, Gu);
                X.timed("take_runs", double(Gu) * entry_bytes(lo.b) * 2, [&] { launch_take_runs(dup, starts, Gu, o, s); });
                X.release(starts);
                X.drop(dup);
                if (st.node >= 0) out->node_sizes[st.node] = int64_t(o.n);
                if (!keep) {
                    for (int in2 : {st.in0, st.in1})
                        if (in2 >= 0 && --uses[in2] == 0) X.drop(tab[in2]);
                }
                continue;
            }
            bool entry_form = false;
            uint32_t* e_slen = nullptr;
            uint8_t* e_src = nullptr;
            uint64_t* e_soff = nullptr;
            uint64_t e_T = 0;
            IntroArgs ea = ia;
            if (entry_eligible) {
                const DevTable& in = tab[st.in0];
                ea.sel = nullptr;
                ea.segv = nullptr;
                // two bag neighbours of u adjacent to each other in F: the
                // candidates are the common neighbours of their images
                {
                    const Step& ch = plan.steps[size_t(st.in0)];
                    int cand[5], nc = 0;
                    cand[nc++] = st.anchor;
                    for (int j = 0; j < st.nchk; j++) cand[nc++] = st.chk[j];
                    for (int p = 0; p < nc && ea.cn0 < 0; p++)
                        for (int q = p + 1; q < nc && ea.cn0 < 0; q++)
                            if ((dec.adj[ch.cols[cand[p]]] >> ch.cols[cand[q]]) & 1u) {
                                ea.cn0 = cand[p];
                                ea.cn1 = cand[q];
                            }
                }
                if (ea.cn0 >= 0) {
                    if (cn_ready()) {
                        ea.cn_off = rq.g->cn_off;
                        ea.cn_col = rq.g->cn_col;
                    } else {
                        ea.cn0 = ea.cn1 = -1;
                    }
                } else if (st.nchk >= 1 && wedge_ready()) {
                    // two bag neighbours not adjacent in F: the common
                    // neighbours of their images, from the wedge index
                    ea.wd0 = st.anchor;
                    ea.wd1 = st.chk[0];
                    ea.wd_vb = rq.g->wd_vb;
                    ea.wd_hk = rq.g->wd_hk;
                    ea.wd_hv = rq.g->wd_hv;
                    ea.wd_mask = rq.g->wd_mask;
                    ea.wd_start = rq.g->wd_start;
                    ea.wd_mid = rq.g->wd_mid;
                }
                // sums[0]: candidates of the fixed-column forms (the anchor's
                // degree per entry), sums[1]: of the entry-wise form; a large
                // table decides on a sample of about 2^16 entries first,
                // unless the candidates are common neighbours (then the
                // entry-wise form nearly always walks far fewer)
                uint64_t* sums = X.alloc<uint64_t>(2);
                launch_fill_u64(sums, 0, 2, s);
                const uint64_t factor = uint64_t(std::max(1, ctx->entry_factor));
                const uint64_t stride = ea.cn0 < 0 && ea.wd0 < 0 && in.n >= (uint64_t(1) << 20) ? in.n >> 16 : 1;
                bool decided = false;
                if (stride > 1) {
                    X.timed("entry_sample", double(in.n / stride) * (entry_bytes(in.lay.b) + 8.0),
                            [&] { launch_entry_seglen(in, g, ea, nullptr, nullptr, sums, stride, s); });
                    const uint64_t cls = read_u64(X.lane, sums), ent = read_u64(X.lane, sums + 1);
                    entry_form = factor * ent < cls;
                    decided = true;
                }
                if (!decided || entry_form) {
                    if (ea.cn0 >= 0 || ea.wd0 >= 0) ea.erow = X.alloc<int64_t>(in.n);
                    e_slen = X.alloc<uint32_t>(in.n);
                    e_src = X.alloc<uint8_t>(in.n);
                    launch_fill_u64(sums, 0, 2, s);
                    X.timed("entry_seglen", double(in.n) * entry_bytes(in.lay.b) + 8.0 * in.n,
                            [&] { launch_entry_seglen(in, g, ea, e_slen, e_src, sums, 1, s); });
                    e_T = X.scan(e_slen, in.n, &e_soff);  // synchronises: the sums are final
                    X.release(e_slen);
                    if (!decided) entry_form = factor * e_T < read_u64(X.lane, sums);
                    if (!entry_form) {
                        X.release(e_soff);
                        X.release(e_src);
                        if (ea.erow) X.release(ea.erow);
                        ea.erow = nullptr;
                    }
                }
                X.release(sums);
            }
            if (entry_form) {
                const DevTable& in = tab[st.in0];
                // Entries that differ only in their colour sets share every
                // adjacency test: when they come at least two to a group, the
                // tests run once per (group, candidate) with the push-form
                // kernels over groups of whole bags, and the expand then only
                // tests colours.  Output order (group, candidate, colour set)
                // is key order when u is the last column; else the same
                // re-sort follows.
                uint64_t* fgs = nullptr;
                const uint64_t Gf = X.groups(in, in.lay.kb, &fgs);
                if (ea.cn0 < 0 && ea.wd0 < 0 && g.n <= (1 << 27) && ctx->group_min > 0 &&
                    uint64_t(ctx->group_min) * Gf <= in.n) {
                    X.release(e_soff);
                    X.release(e_src);
                    IntroArgs ga = ea;
                    ga.grouped = true;
                    uint32_t* wcount = X.alloc<uint32_t>(Gf);
                    uint8_t* gsel = X.alloc<uint8_t>(Gf);
                    ga.sel = gsel;
                    X.timed("group_work", double(Gf) * (in.lay.key_bytes() + 13.0),
                            [&] { launch_push_work(in, fgs, Gf, g, ga, wcount, s); });
                    uint64_t* woff;
                    const uint64_t W = X.scan(wcount, Gf, &woff);
                    X.release(wcount);
                    uint32_t* slen = X.alloc<uint32_t>(W);
                    ga.segv = X.alloc<uint32_t>(W);
                    X.timed("group_seglen", 28.0 * W,
                            [&] { launch_push_seglen(in, fgs, woff, Gf, W, g, rq.colors, ga, slen, s); });
                    uint64_t* soff;
                    const uint64_t T = X.scan(slen, W, &soff);
                    X.release(slen);
                    const uint64_t tiles = expand_tiles(T);
                    uint32_t* tcount = X.alloc<uint32_t>(tiles);
                    uint16_t* pbits = X.alloc<uint16_t>(expand_pass_words(T));
                    X.timed("group_count", double(T) * in.lay.key_bytes(), [&] {
                        launch_expand_count(false, in, fgs, woff, Gf, nullptr, soff, W, T, g, rq.colors, ga, tcount, pbits,
                                            s);
                    });
                    uint64_t* toff;
                    const uint64_t N = X.scan(tcount, tiles, &toff);
                    X.release(tcount);
                    o = X.table(lo, N);
                    if (N)
                        X.timed("group_emit", double(in.n) * entry_bytes(in.lay.b) + double(N) * entry_bytes(lo.b), [&] {
                            launch_expand_emit(false, in, fgs, woff, Gf, nullptr, soff, W, T, g, rq.colors, ga, toff, pbits,
                                               o, nullptr, s);
                        });
                    X.release(pbits);
                    X.release(toff);
                    X.release(soff);
                    X.release(ga.segv);
                    X.release(woff);
                    X.release(gsel);
                    X.release(fgs);
                    if (N > 1 && st.pos != lo.b - 1) {
                        // stable sort on (colouring, columns 0..pos)
                        const int sort_lo = lo.kb + (lo.b - 1 - st.pos) * lo.vb;
                        void* kb2 = X.raw(N * lo.key_bytes());
                        uint64_t* vb2 = X.alloc<uint64_t>(N);
                        void* tmp = X.raw(radix_tmp_bytes(N));
                        bool in_b = false;
                        X.timed("radix_sort", sort_bytes(N, lo, sort_lo), [&] {
                            in_b = radix_sort(o.keys, o.cnt, kb2, vb2, N, lo.kw(), lo.bits(), sort_lo, tmp, s, false);
                        });
                        if (in_b) {
                            std::swap(o.keys, kb2);
                            std::swap(o.cnt, vb2);
                        }
                        X.release(tmp);
                        X.release(vb2);
                        X.release(kb2);
                    }
                } else {
                    X.release(fgs);
                    uint8_t* src = e_src;
                    uint64_t* soff = e_soff;
                    const uint64_t T = e_T;
                    const uint64_t tiles = expand_tiles(T);
                    uint32_t* tcount = X.alloc<uint32_t>(tiles);
                    uint16_t* pbits = X.alloc<uint16_t>(expand_pass_words(T));
                    X.timed("entry_count", double(in.n) * entry_bytes(in.lay.b) + 5.0 * T,
                            [&] { launch_entry_count(in, src, soff, T, g, rq.colors, ea, tcount, pbits, s); });
                    uint64_t* toff;
                    const uint64_t N = X.scan(tcount, tiles, &toff);
                    X.release(tcount);
                    o = X.table(lo, N);
                    if (N) {
                        X.timed("entry_emit", double(in.n) * entry_bytes(in.lay.b) + double(N) * entry_bytes(lo.b), [&] {
                            launch_entry_emit(in, src, soff, T, g, rq.colors, ea, toff, pbits, o, s);
                        });
                    }
                    X.release(pbits);
                    X.release(toff);
                    X.release(soff);
                    X.release(src);
                    if (ea.erow) X.release(ea.erow);
                    if (N > 1) {
                        // stable sort on (colouring, columns 0..pos)
                        const int sort_lo = lo.kb + (lo.b - 1 - st.pos) * lo.vb;
                        void* kb2 = X.raw(N * lo.key_bytes());
                        uint64_t* vb2 = X.alloc<uint64_t>(N);
                        void* tmp = X.raw(radix_tmp_bytes(N));
                        bool in_b = false;
                        X.timed("radix_sort", sort_bytes(N, lo, sort_lo), [&] {
                            in_b = radix_sort(o.keys, o.cnt, kb2, vb2, N, lo.kw(), lo.bits(), sort_lo, tmp, s, false);
                        });
                        if (in_b) {
                            std::swap(o.keys, kb2);
                            std::swap(o.cnt, vb2);
                        }
                        X.release(tmp);
                        X.release(vb2);
                        X.release(kb2);
                    }
                }
                if (st.node >= 0) out->node_sizes[st.node] = int64_t(o.n);
                if (!keep) {
                    for (int in2 : {st.in0, st.in1})
                        if (in2 >= 0 && --uses[in2] == 0) X.drop(tab[in2]);
                }
                continue;
            }
            switch (st.kind) {
                case S_LEAF: {
                    uint64_t total = uint64_t(g.n) * B;
                    uint32_t* flags = X.alloc<uint32_t>(total);
                    X.timed("leaf_count", 4.0 * total + 8.0 * g.n, [&] { launch_leaf_count(g, B, ia.degF, flags, s); });
                    uint64_t* offs;
                    uint64_t N = X.scan(flags, total, &offs);
                    X.release(flags);
                    o = X.table(lo, N);
                    X.timed("leaf_emit", 8.0 * g.n + double(total) + double(N) * entry_bytes(1),
                            [&] { launch_leaf_emit(g, B, ia.degF, rq.colors, offs, lo, o.keys, o.cnt, s); });
                    X.release(offs);
                    break;
                }
                case S_INTRO_PUSH: {
                    const DevTable& in = tab[st.in0];
                    if (in.n == 0) {
                        o = X.table(lo, 0);
                        break;
                    }
                    int shift = in.lay.kb + (in.lay.b - st.pos) * in.lay.vb;
                    uint64_t* gstart;
                    uint64_t G = X.groups(in, shift, &gstart);
                    uint32_t* wcount = X.alloc<uint32_t>(G);
                    uint8_t* gsel = X.alloc<uint8_t>(G);
                    ia.sel = gsel;
                    // two bag neighbours of u before pos adjacent to each other
                    // in F: a group's candidates are the common neighbours of
                    // their images
                    if (st.anchor >= 0 && !links && g.n <= (1 << 27)) {
                        const Step& ch = plan.steps[size_t(st.in0)];
                        int cand[5], nc = 0;
                        cand[nc++] = st.anchor;
                        for (int j = 0; j < st.nchk; j++)
                            if (st.chk[j] < st.pos) cand[nc++] = st.chk[j];
                        for (int p = 0; p < nc && ia.cn0 < 0; p++)
                            for (int q = p + 1; q < nc && ia.cn0 < 0; q++)
                                if ((dec.adj[ch.cols[cand[p]]] >> ch.cols[cand[q]]) & 1u) {
                                    ia.cn0 = cand[p];
                                    ia.cn1 = cand[q];
                                }
                        if (ia.cn0 >= 0 && cn_ready()) {
                            ia.cn_off = rq.g->cn_off;
                            ia.cn_col = rq.g->cn_col;
                            ia.erow = X.alloc<int64_t>(G);
                        } else {
                            ia.cn0 = ia.cn1 = -1;
                        }
                    }
                    X.timed("push_work", 20.0 * G, [&] { launch_push_work(in, gstart, G, g, ia, wcount, s); });
                    uint64_t* woff;
                    uint64_t W = X.scan(wcount, G, &woff);
                    X.release(wcount);
                    uint32_t* slen = X.alloc<uint32_t>(W);
                    // each segment's candidate and its colour, for the expand passes
                    ia.segv = g.n <= (1 << 27) ? X.alloc<uint32_t>(W) : nullptr;
                    X.timed("push_seglen", 28.0 * W,
                            [&] { launch_push_seglen(in, gstart, woff, G, W, g, rq.colors, ia, slen, s); });
                    uint64_t* soff;
                    uint64_t T = X.scan(slen, W, &soff);
                    X.release(slen);
                    uint64_t tiles = expand_tiles(T);
                    uint32_t* tcount = X.alloc<uint32_t>(tiles);
                    uint16_t* pbits = X.alloc<uint16_t>(expand_pass_words(T));
                    X.timed("push_count", double(T) * in.lay.key_bytes(), [&] {
                        launch_expand_count(false, in, gstart, woff, G, nullptr, soff, W, T, g, rq.colors, ia, tcount, pbits, s);
                    });
                    uint64_t* toff;
                    uint64_t N = X.scan(tcount, tiles, &toff);
                    X.release(tcount);
                    o = X.table(lo, N);
                    if (links) lk[i].src = X.alloc<uint64_t>(N);
                    if (N)
                        X.timed("push_emit", double(in.n) * entry_bytes(in.lay.b) + double(N) * entry_bytes(lo.b) + 5.0 * W, [&] {
                            launch_expand_emit(false, in, gstart, woff, G, nullptr, soff, W, T, g, rq.colors, ia, toff, pbits, o,
                                               lk[i].src, s);
                        });
                    X.release(pbits);
                    X.release(toff);
                    X.release(soff);
                    X.release(woff);
                    X.release(ia.segv);
                    ia.segv = nullptr;
                    if (ia.erow) X.release(ia.erow);
                    ia.erow = nullptr;
                    ia.cn0 = ia.cn1 = -1;
                    X.release(gsel);
                    X.release(gstart);
                    break;
                }
                case S_INTRO_PULL: {
                    if (lpull[i]) {
                        const int degF_l = rq.degree_mask ? plan.steps[size_t(st.in0)].degF : 0;
                        const uint64_t tiles = leaf_pull_tiles(g, B);
                        if (!tiles) {  // no edges
                            o = X.table(lo, 0);
                            break;
                        }
                        uint32_t* tcount = X.alloc<uint32_t>(tiles);
                        const double edges = double(B) * double(g.m2);
                        X.timed("leaf_pull_count", 8.0 * double(g.m2) + 2.0 * edges + 4.0 * double(tiles), [&] {
                            launch_leaf_pull_count(g, B, ia.degF, degF_l, rq.colors, lo, tcount, s);
                        });
                        uint64_t* toff;
                        const uint64_t N = X.scan(tcount, tiles, &toff);
                        X.release(tcount);
                        o = X.table(lo, N);
                        if (N)
                            X.timed("leaf_pull_emit", 8.0 * double(g.m2) + 2.0 * edges + double(N) * entry_bytes(lo.b), [&] {
                                launch_leaf_pull_emit(g, B, ia.degF, degF_l, rq.colors, toff, o, s);
                            });
                        X.release(toff);
                        break;
                    }
                    const DevTable& in = tab[st.in0];
                    if (in.n == 0) {
                        o = X.table(lo, 0);
                        break;
                    }
                    uint64_t slots = uint64_t(B) * g.n;
                    uint64_t* rstart = X.alloc<uint64_t>(slots);
                    uint64_t* rend = X.alloc<uint64_t>(slots);
                    launch_fill_u64(rstart, 0, slots, s);
                    launch_fill_u64(rend, 0, slots, s);
                    X.timed("pull_index", double(in.n) * in.lay.key_bytes(), [&] { launch_pull_index(in, g.n, rstart, rend, s); });
                    uint64_t S = uint64_t(B) * uint64_t(g.m2);
                    uint32_t* slen = X.alloc<uint32_t>(S);
                    X.timed("pull_seglen", 32.0 * S, [&] { launch_pull_seglen(rstart, rend, B, g, ia.degF, slen, s); });
                    uint64_t* soff;
                    uint64_t T = X.scan(slen, S, &soff);
                    X.release(slen);
                    uint64_t tiles = expand_tiles(T);
                    uint32_t* tcount = X.alloc<uint32_t>(tiles);
                    uint16_t* pbits = X.alloc<uint16_t>(expand_pass_words(T));
                    X.timed("pull_count", double(T) * in.lay.key_bytes(), [&] {
                        launch_expand_count(true, in, nullptr, nullptr, 0, rstart, soff, S, T, g, rq.colors, ia, tcount, pbits, s);
                    });
                    uint64_t* toff;
                    uint64_t N = X.scan(tcount, tiles, &toff);
                    X.release(tcount);
                    o = X.table(lo, N);
                    if (links) lk[i].src = X.alloc<uint64_t>(N);
                    if (N)
                        X.timed("pull_emit", double(in.n) * entry_bytes(in.lay.b) + double(N) * entry_bytes(lo.b) + 5.0 * S, [&] {
                            launch_expand_emit(true, in, nullptr, nullptr, 0, rstart, soff, S, T, g, rq.colors, ia, toff, pbits, o,
                                               lk[i].src, s);
                        });
                    X.release(pbits);
                    X.release(toff);
                    X.release(soff);
                    X.release(rstart);
                    X.release(rend);
                    break;
                }
                case S_FORGET_LAST: {
                    const DevTable& in = tab[st.in0];
                    if (in.n == 0) {
                        o = X.table(lo, 0);
                        break;
                    }
                    if (k > kDenseColours || (!links && k > ctx->sort_above_k)) {
                        // colour sets too wide for the dense accumulators (or
                        // the schedule prefers sorting): drop
                        // the column, sort, add up runs of equal keys
                        DevTable d = X.table(lo, in.n);
                        hip_check(hipMemcpyAsync(d.cnt, in.cnt, 8 * in.n, hipMemcpyDeviceToDevice, s), "copy counts");
                        X.timed("drop_last", double(in.n) * (entry_bytes(in.lay.b) + entry_bytes(lo.b)),
                                [&] { launch_drop_last(in, d, s); });
                        if (in.n > 1) {
                            void* kb2 = X.raw(in.n * lo.key_bytes());
                            uint64_t* vb2 = X.alloc<uint64_t>(in.n);
                            void* tmp = X.raw(radix_tmp_bytes(in.n));
                            bool in_b = false;
                            X.timed("radix_sort", sort_bytes(in.n, lo, 0), [&] {
                                in_b = radix_sort(d.keys, d.cnt, kb2, vb2, in.n, lo.kw(), lo.bits(), 0, tmp, s, false);
                            });
                            if (in_b) {
                                std::swap(d.keys, kb2);
                                std::swap(d.cnt, vb2);
                            }
                            X.release(tmp);
                            X.release(vb2);
                            X.release(kb2);
                        }
                        uint64_t* starts;
                        const uint64_t Gr = X.groups(d, 0, &starts);
                        o = X.table(lo, Gr);
                        X.timed("reduce_runs", double(in.n) * entry_bytes(lo.b) + double(Gr) * entry_bytes(lo.b),
                                [&] { launch_reduce_runs(d, starts, Gr, o, ovf, s); });
                        X.release(starts);
                        X.drop(d);
                        break;
                    }
                    uint64_t* gstart;
                    uint64_t G = X.groups(in, in.lay.kb + in.lay.vb, &gstart);
                    uint32_t* gcount = X.alloc<uint32_t>(G);
                    X.timed("forget_count", double(in.n) * in.lay.key_bytes() + 4.0 * G,
                            [&] { launch_forget_count(in, gstart, G, gcount, s); });
                    uint64_t* goff;
                    uint64_t N = X.scan(gcount, G, &goff);
                    X.release(gcount);
                    o = X.table(lo, N);
                    X.timed("forget_emit", double(in.n) * entry_bytes(in.lay.b) + double(N) * entry_bytes(lo.b),
                            [&] { launch_forget_emit(in, gstart, G, goff, o, ovf, s); });
                    if (links) {
                        // contributors of every output entry: child entries sorted by output position
                        uint64_t* dst = X.alloc<uint64_t>(in.n);
                        launch_forget_dst(in, gstart, G, goff, dst, s);
                        uint64_t* ca = X.alloc<uint64_t>(in.n);
                        launch_iota(ca, in.n, s);
                        sort_pairs(X, dst, ca, in.n, N);
                        StepLinks& L = lk[i];
                        L.ca = ca;
                        L.seg = X.alloc<uint64_t>(N + 1);
                        launch_segment_starts(dst, in.n, N, L.seg, s);
                        uint64_t* w = X.alloc<uint64_t>(in.n);
                        launch_gather_u64(in.cnt, ca, in.n, w, s);
                        L.wcum = X.alloc<uint64_t>(in.n + 1);
                        uint64_t* tmp = (uint64_t*)X.raw(scan_tmp_bytes(in.n));
                        launch_scan_u64(w, L.wcum, in.n, tmp, s);
                        X.release(tmp);
                        X.release(w);
                        X.release(dst);
                    }
                    X.release(goff);
                    X.release(gstart);
                    break;
                }
                case S_JOIN: {
                    const DevTable& y = tab[st.in0];
                    const DevTable& z = tab[st.in1];
                    if (y.n == 0 || z.n == 0) {
                        o = X.table(lo, 0);
                        break;
                    }
                    if (k > kDenseColours || (!links && k > ctx->sort_above_k)) {
                        // colour sets too wide for the dense accumulators (or
                        // the schedule prefers sorting): all admissible
                        // pairs, then sort and add up runs
                        uint32_t* pc = X.alloc<uint32_t>(y.n);
                        X.timed("join_pairs_count", double(y.n + z.n) * entry_bytes(y.lay.b),
                                [&] { launch_join_pairs(y, z, g.n, rq.colors, pc, nullptr, nullptr, ovf, s); });
                        uint64_t* poff;
                        const uint64_t P = X.scan(pc, y.n, &poff);
                        X.release(pc);
                        DevTable pr = X.table(lo, P);
                        if (P)
                            X.timed("join_pairs_emit", double(y.n + z.n) * entry_bytes(y.lay.b) + double(P) * entry_bytes(lo.b),
                                    [&] { launch_join_pairs(y, z, g.n, rq.colors, nullptr, poff, &pr, ovf, s); });
                        X.release(poff);
                        if (P > 1) {
                            void* kb2 = X.raw(P * lo.key_bytes());
                            uint64_t* vb2 = X.alloc<uint64_t>(P);
                            void* tmp = X.raw(radix_tmp_bytes(P));
                            bool in_b = false;
                            X.timed("radix_sort", sort_bytes(P, lo, 0), [&] {
                                in_b = radix_sort(pr.keys, pr.cnt, kb2, vb2, P, lo.kw(), lo.bits(), 0, tmp, s, false);
                            });
                            if (in_b) {
                                std::swap(pr.keys, kb2);
                                std::swap(pr.cnt, vb2);
                            }
                            X.release(tmp);
                            X.release(vb2);
                            X.release(kb2);
                        }
                        uint64_t* starts;
                        const uint64_t Gr = X.groups(pr, 0, &starts);
                        o = X.table(lo, Gr);
                        X.timed("reduce_runs", double(P) * entry_bytes(lo.b) + double(Gr) * entry_bytes(lo.b),
                                [&] { launch_reduce_runs(pr, starts, Gr, o, ovf, s); });
                        X.release(starts);
                        X.drop(pr);
                        break;
                    }
                    uint64_t* gstart;
                    uint64_t G = X.groups(y, y.lay.kb, &gstart);
                    uint64_t slots = uint64_t(B) * g.n;
                    uint64_t* zlo = X.alloc<uint64_t>(slots);
                    uint64_t* zhi = X.alloc<uint64_t>(slots);
                    launch_fill_u64(zlo, 0, slots, s);
                    launch_fill_u64(zhi, 0, slots, s);
                    X.timed("join_index", double(z.n) * z.lay.key_bytes(), [&] { launch_pull_index(z, g.n, zlo, zhi, s); });
                    uint32_t* gcount = X.alloc<uint32_t>(G);
                    X.timed("join_count", double(y.n + z.n) * y.lay.key_bytes() + 4.0 * G,
                            [&] { launch_join_count(y, z, gstart, G, g.n, rq.colors, zlo, zhi, gcount, s); });
                    uint64_t* goff;
                    uint64_t N = X.scan(gcount, G, &goff);
                    X.release(gcount);
                    o = X.table(lo, N);
                    if (N)
                        X.timed("join_emit", double(y.n + z.n) * entry_bytes(y.lay.b) + double(N) * entry_bytes(lo.b),
                                [&] { launch_join_emit(y, z, gstart, G, g.n, rq.colors, zlo, zhi, goff, o, ovf, s); });
                    X.release(zlo);
                    X.release(zhi);
                    if (links && N) {
                        uint32_t* pc = X.alloc<uint32_t>(G);
                        launch_join_pairs_count(y, z, gstart, G, g.n, rq.colors, pc, s);
                        uint64_t* poff;
                        uint64_t P = X.scan(pc, G, &poff);
                        X.release(pc);
                        uint64_t* pdst = X.alloc<uint64_t>(P);
                        uint64_t* pa = X.alloc<uint64_t>(P);
                        uint64_t* pd = X.alloc<uint64_t>(P);
                        launch_join_pairs_emit(y, z, gstart, G, g.n, rq.colors, goff, poff, pdst, pa, pd, s);
                        X.release(poff);
                        uint64_t* perm = X.alloc<uint64_t>(P);
                        launch_iota(perm, P, s);
                        sort_pairs(X, pdst, perm, P, N);
                        StepLinks& L = lk[i];
                        L.ca = X.alloc<uint64_t>(P);
                        L.cb = X.alloc<uint64_t>(P);
                        launch_gather_u64(pa, perm, P, L.ca, s);
                        launch_gather_u64(pd, perm, P, L.cb, s);
                        L.seg = X.alloc<uint64_t>(N + 1);
                        launch_segment_starts(pdst, P, N, L.seg, s);
                        uint64_t* w = X.alloc<uint64_t>(P);
                        launch_gather_product(y.cnt, L.ca, z.cnt, L.cb, P, w, s);
                        L.wcum = X.alloc<uint64_t>(P + 1);
                        uint64_t* tmp = (uint64_t*)X.raw(scan_tmp_bytes(P));
                        launch_scan_u64(w, L.wcum, P, tmp, s);
                        X.release(tmp);
                        X.release(w);
                        X.release(perm);
                        X.release(pa);
                        X.release(pd);
                        X.release(pdst);
                    }
                    X.release(goff);
                    X.release(gstart);
                    break;
                }
                case S_RESORT: {
                    const DevTable& in = tab[st.in0];
                    o = X.table(lo, in.n);
                    // The input (introduce at the last column) is sorted by
                    // (colouring, its columns, colour set).  When only that last
                    // column moves, to output position p, a stable sort on the
                    // key bits of (colouring, columns 0..p) gives the order.
                    int sort_lo = 0;
                    {
                        int p = -1;
                        bool moved_only = true;
                        for (int j = 0, prev = -1; j < lo.b; j++) {
                            if (st.perm[j] == lo.b - 1) {
                                p = j;
                            } else {
                                moved_only &= st.perm[j] > prev;
                                prev = st.perm[j];
                            }
                        }
                        if (p >= 0 && moved_only) sort_lo = lo.kb + (lo.b - 1 - p) * lo.vb;
                    }
                    if (in.n && links) {
                        // sort (key, input position), then gather the counts
                        uint64_t* idx = X.alloc<uint64_t>(in.n);
                        DevTable t2 = o;
                        t2.cnt = idx;
                        launch_permute(in, st.perm, t2, true, s);
                        void* kb2 = X.raw(in.n * lo.key_bytes());
                        uint64_t* vb2 = X.alloc<uint64_t>(in.n);
                        void* tmp = X.raw(radix_tmp_bytes(in.n));
                        if (radix_sort(o.keys, idx, kb2, vb2, in.n, lo.kw(), lo.bits(), sort_lo, tmp, s, false)) {
                            std::swap(o.keys, kb2);  // the sorted data is in the second buffers: keep those
                            std::swap(idx, vb2);
                        }
                        X.release(tmp);
                        X.release(vb2);
                        X.release(kb2);
                        launch_gather_u64(in.cnt, idx, in.n, o.cnt, s);
                        lk[i].src = idx;
                    } else if (in.n) {
                        // same key width: the sort's first pass reads the input and
                        // reorders its columns on the way
                        const bool fold = in.lay.kw() == lo.kw();
                        if (!fold)
                            X.timed("permute", double(in.n) * (in.lay.key_bytes() + lo.key_bytes() + 16),
                                    [&] { launch_permute(in, st.perm, o, false, s); });
                        void* kb2 = X.raw(in.n * lo.key_bytes());
                        uint64_t* vb2 = X.alloc<uint64_t>(in.n);
                        void* tmp = X.raw(radix_tmp_bytes(in.n));
                        RadixSource from{in.keys, in.cnt, in.lay, lo, {st.perm[0], st.perm[1], st.perm[2], st.perm[3]}};
                        bool in_b = false;
                        X.timed("radix_sort", sort_bytes(in.n, lo, sort_lo), [&] {
                            in_b = radix_sort(o.keys, o.cnt, kb2, vb2, in.n, lo.kw(), lo.bits(), sort_lo, tmp, s, false,
                                              fold ? &from : nullptr);
                        });
                        if (in_b) {  // the sorted data is in the second buffers: keep those
                            std::swap(o.keys, kb2);
                            std::swap(o.cnt, vb2);
                        }
                        X.release(tmp);
                        X.release(vb2);
                        X.release(kb2);
                    }
                    break;
                }
            }
            if (st.node >= 0) out->node_sizes[st.node] = int64_t(o.n);
            if (!keep) {
                for (int in : {st.in0, st.in1})
                    if (in >= 0 && --uses[in] == 0) X.drop(tab[in]);
            }
        }
        hip_check(hipGetLastError(), "kernel launch");

        // root: counts and overflow flags per colouring
        const DevTable& rc = tab[plan.root_child];
        uint64_t* counts = X.alloc<uint64_t>(B);
        launch_fill_u64(counts, 0, B, s);
        uint64_t* pv = nullptr;
        if (rq.per_vertex) {
            pv = X.alloc<uint64_t>(uint64_t(B) * g.n);
            launch_fill_u64(pv, 0, uint64_t(B) * g.n, s);
        }
        const int cwords = k >= 5 ? 1 << (k - 5) : 1;
        uint32_t* csets = X.alloc<uint32_t>(uint64_t(B) * cwords);
        launch_fill_u32(csets, 0, uint64_t(B) * cwords, s);
        X.timed("root", double(rc.n) * entry_bytes(1),
                [&] { launch_root(rc, g.n, counts, ovf, pv, csets, cwords, s); });
        std::vector<uint32_t> cs(uint64_t(B) * cwords);
        hip_check(hipMemcpyAsync(cs.data(), csets, 4 * cs.size(), hipMemcpyDeviceToHost, s), "copy colour sets");
        out->counts.assign(B, 0);
        std::vector<uint32_t> of(B, 0);
        hip_check(hipMemcpyAsync(out->counts.data(), counts, 8 * size_t(B), hipMemcpyDeviceToHost, s), "copy counts");
        hip_check(hipMemcpyAsync(of.data(), ovf, 4 * size_t(B), hipMemcpyDeviceToHost, s), "copy flags");
        if (pv) {
            out->per_vertex.assign(uint64_t(B) * g.n, 0);
            hip_check(hipMemcpyAsync(out->per_vertex.data(), pv, 8 * uint64_t(B) * g.n, hipMemcpyDeviceToHost, s),
                      "copy per-vertex");
        }
        hip_check(hipStreamSynchronize(s), "hipStreamSynchronize");
        X.synced();
        lane.prof.resolve();
        out->overflow.assign(B, 0);
        for (int b = 0; b < B; b++) out->overflow[b] = of[b] ? 1 : 0;
        int root_node = int(dec.nodes.size()) - 1;
        int64_t nz = 0;
        for (uint32_t w : cs) nz += __builtin_popcount(w);
        out->node_sizes[root_node] = nz;
        out->root_sets = cs;
        X.release(csets);
        X.release(counts);
        X.release(pv);
        X.release(ovf);
        if (keep) {
            out->tables = tab;
            out->links = lk;
        } else {
            X.drop(tab[plan.root_child]);
        }
        X.synced();  // the stream is idle: everything released goes back
        out->peak_bytes = X.peak;
    } catch (...) {
        (void)hipStreamSynchronize(s);
        X.release_all();
        throw;
    }
}

}  // namespace ccg

namespace ccg {

// At most 2^6 anchor-range chunks per colouring, and none in an arena below
// 256 MiB (there the tables are not what exhausts it).
constexpr int kMaxChunkDepth = 6;

static bool splittable(cc_context* ctx, const CcError& e, const RunRequest& rq) {
    if (rq.keep_tables || rq.links || rq.no_alloc) return false;
    const Arena& A = rq.arena ? *rq.arena : ctx->arena;
    return e.budget || (e.code == CC_ENOMEM && A.size() >= (size_t(256) << 20));
}

void run_dp_waves(cc_context* ctx, Lane& lane, const RunRequest& rq, RunResult* out) {
    try {
        run_dp(ctx, lane, rq, out);
        return;
    } catch (const CcError& e) {
        if (!splittable(ctx, e, rq)) throw;
        const int32_t lo = rq.anchor_hi >= 0 ? rq.anchor_lo : 0;
        const int32_t hi = rq.anchor_hi >= 0 ? rq.anchor_hi : rq.g->n;
        if (rq.B <= 1 && (hi - lo <= 1 || rq.chunk_depth >= kMaxChunkDepth)) throw;
    }
    RunResult ra, rb;
    if (rq.B > 1) {  // waves of colourings
        const int B1 = rq.B / 2;
        RunRequest a = rq, b = rq;
        a.B = B1;
        b.B = rq.B - B1;
        b.colors = rq.colors + size_t(B1) * size_t(rq.g->n);
        run_dp_waves(ctx, lane, a, &ra);
        run_dp_waves(ctx, lane, b, &rb);
        out->counts = ra.counts;
        out->counts.insert(out->counts.end(), rb.counts.begin(), rb.counts.end());
        out->overflow = ra.overflow;
        out->overflow.insert(out->overflow.end(), rb.overflow.begin(), rb.overflow.end());
        if (rq.per_vertex) {
            out->per_vertex = ra.per_vertex;
            out->per_vertex.insert(out->per_vertex.end(), rb.per_vertex.begin(), rb.per_vertex.end());
        }
        out->node_sizes = ra.node_sizes;
        for (size_t i = 0; i < out->node_sizes.size() && i < rb.node_sizes.size(); i++)
            out->node_sizes[i] += rb.node_sizes[i];
        out->root_sets = ra.root_sets;
        out->root_sets.insert(out->root_sets.end(), rb.root_sets.begin(), rb.root_sets.end());
        out->peak_bytes = std::max(ra.peak_bytes, rb.peak_bytes);
        out->chunks = ra.chunks + rb.chunks;
        return;
    }
    // one colouring: two anchor ranges of equal degree mass (the entries an
    // anchor image carries grow with its degree; on heavy-tailed graphs equal
    // vertex counts would leave the hubs' range as large as the whole)
    const int32_t lo = rq.anchor_hi >= 0 ? rq.anchor_lo : 0;
    const int32_t hi = rq.anchor_hi >= 0 ? rq.anchor_hi : rq.g->n;
    int32_t mid = lo + (hi - lo) / 2;
    {
        const std::vector<int64_t>& rp = rq.g->host_rp;
        const int64_t half = rp[size_t(lo)] + (rp[size_t(hi)] - rp[size_t(lo)] + 1) / 2;
        const int32_t m = int32_t(std::lower_bound(rp.begin() + lo, rp.begin() + hi + 1, half) - rp.begin());
        if (rp[size_t(hi)] > rp[size_t(lo)]) mid = std::min(std::max(m, lo + 1), hi - 1);
    }
    RunRequest a = rq, b = rq;
    a.anchor_lo = lo;
    a.anchor_hi = mid;
    b.anchor_lo = mid;
    b.anchor_hi = hi;
    a.chunk_depth = b.chunk_depth = rq.chunk_depth + 1;
    run_dp_waves(ctx, lane, a, &ra);
    run_dp_waves(ctx, lane, b, &rb);
    out->counts.assign(1, ra.counts[0] + rb.counts[0]);
    const bool carry = ra.counts[0] + rb.counts[0] < ra.counts[0];
    out->overflow.assign(1, uint8_t(ra.overflow[0] || rb.overflow[0] || carry));
    if (rq.per_vertex) {  // the ranges are disjoint: each vertex has one nonzero part
        out->per_vertex = ra.per_vertex;
        for (size_t v = 0; v < out->per_vertex.size(); v++) out->per_vertex[v] += rb.per_vertex[v];
    }
    const Decomp& dec = rq.dec->d;
    out->node_sizes = ra.node_sizes;
    for (size_t i = 0; i + 1 < dec.nodes.size() && i < rb.node_sizes.size(); i++)
        if (dec.nodes[i].bag >> rq.anchor_vertex & 1u) out->node_sizes[i] += rb.node_sizes[i];
    out->root_sets = ra.root_sets;
    for (size_t w = 0; w < out->root_sets.size() && w < rb.root_sets.size(); w++) out->root_sets[w] |= rb.root_sets[w];
    int64_t nz = 0;
    for (uint32_t w : out->root_sets) nz += __builtin_popcount(w);
    out->node_sizes[dec.nodes.size() - 1] = nz;
    out->peak_bytes = std::max(ra.peak_bytes, rb.peak_bytes);
    out->chunks = ra.chunks + rb.chunks;
}

// Enumeration (Sec. 4) of one colouring: forward DP keeping every table and
// its contributor index, lexicographic cut on the image of vertex 0 (the
// node below the root holds bag {0}, sorted by that image), row decoding on
// the device, a radix sort of the packed rows and truncation to `cap`.
void run_enumerate(cc_context* ctx, Lane& lane, const cc_graph* g, const uint8_t* colors, int k, const cc_decomp* dec,
                   uint64_t cap, std::vector<int32_t>* rows, uint64_t* n_rows, uint64_t* total) {
    const Plan& plan = dec->plan;
    const int nF = dec->d.n;
    const TdNode& below_root = dec->d.nodes[dec->d.nodes[dec->d.nodes.size() - 1].c0];
    if (below_root.bag != 1u) fail(CC_EINVAL, "enumeration needs pattern vertex 0 forgotten last");
    const int vb = table_layout(1, g->n, 1, k).vb;
    if (nF * vb > 128) fail(CC_ERANGE, "packed rows (n_F x vertex bits) exceed 128 bits");
    RunRequest rq;
    rq.g = g;
    rq.colors = colors;
    rq.B = 1;
    rq.k = k;
    rq.dec = dec;
    rq.links = true;
    rq.max_entries = ctx->max_entries;
    RunResult r;
    run_dp(ctx, lane, rq, &r);
    hipStream_t s = lane.stream;
    Arena& A = ctx->arena;
    std::vector<void*> extra;
    auto alloc = [&](size_t bytes) {
        void* p = A.alloc(bytes);
        extra.push_back(p);
        return p;
    };
    try {
        ctx->last_sizes = r.node_sizes;
        if (r.overflow[0]) fail(CC_ERANGE, "the count overflowed 64 bits; rows cannot be decoded");
        *total = r.counts[0];
        rows->clear();
        *n_rows = 0;
        const DevTable& rc = r.tables[plan.root_child];
        if (cap == 0 || r.counts[0] == 0 || rc.n == 0) {
            release_tables(ctx, &r);
            return;
        }
        // lexicographic cut: keep the entries with Phi(0) <= t for the least t
        // whose rows reach cap (all entries when the count is at most cap)
        std::vector<uint64_t> hk(rc.n * (rc.lay.kw() == 1 ? 1 : 2)), hc(rc.n);
        hip_check(hipMemcpyAsync(hk.data(), rc.keys, rc.n * rc.lay.key_bytes(), hipMemcpyDeviceToHost, s), "copy");
        hip_check(hipMemcpyAsync(hc.data(), rc.cnt, rc.n * 8, hipMemcpyDeviceToHost, s), "copy");
        hip_check(hipStreamSynchronize(s), "sync");
        auto v0_of = [&](uint64_t e) -> uint64_t {
            u128 key = rc.lay.kw() == 1 ? u128(hk[e]) : ((u128(hk[2 * e + 1]) << 64) | hk[2 * e]);
            return uint64_t(key >> rc.lay.kb) & ((uint64_t(1) << rc.lay.vb) - 1);
        };
        std::vector<uint64_t> rcum(rc.n + 1, 0);
        for (uint64_t e = 0; e < rc.n; e++) rcum[e + 1] = rcum[e] + hc[e];
        uint64_t E = rc.n;
        if (r.counts[0] > cap) {
            uint64_t e = 0;
            while (rcum[e + 1] < cap) e++;  // entry where the cap is reached
            uint64_t t = v0_of(e);
            E = e + 1;
            while (E < rc.n && v0_of(E) == t) E++;
        }
        const uint64_t R = rcum[E];
        uint64_t* d_rcum = (uint64_t*)alloc(8 * (E + 1));
        hip_check(hipMemcpyAsync(d_rcum, rcum.data(), 8 * (E + 1), hipMemcpyHostToDevice, s), "copy");
        // step descriptors
        std::vector<EnumStep> es(plan.steps.size());
        for (size_t i = 0; i < plan.steps.size(); i++) {
            const Step& st = plan.steps[i];
            EnumStep& d = es[i];
            d.in0 = st.in0;
            d.in1 = st.in1;
            d.ucol = -1;
            d.u = st.u;
            d.lay = r.tables[i].lay;
            d.keys = r.tables[i].keys;
            d.cnt = r.tables[i].cnt;
            d.src = r.links[i].src;
            d.seg = r.links[i].seg;
            d.wcum = r.links[i].wcum;
            d.ca = r.links[i].ca;
            d.cb = r.links[i].cb;
            switch (st.kind) {
                case S_LEAF: d.kind = EK_LEAF; d.ucol = 0; break;
                case S_INTRO_PUSH:
                case S_INTRO_PULL: d.kind = EK_INTRO; d.ucol = st.pos; break;
                case S_FORGET_LAST: d.kind = EK_FORGET; break;
                case S_JOIN: d.kind = EK_JOIN; break;
                case S_RESORT: d.kind = EK_RESORT; break;
            }
        }
        EnumStep* d_steps = (EnumStep*)alloc(sizeof(EnumStep) * es.size());
        hip_check(hipMemcpyAsync(d_steps, es.data(), sizeof(EnumStep) * es.size(), hipMemcpyHostToDevice, s), "copy");
        uint32_t* err = (uint32_t*)alloc(4);
        launch_fill_u32(err, 0, 1, s);
        const int rbits = nF * vb;
        const int rkw = rbits <= 64 ? 1 : 2;
        const size_t rkb = rkw == 1 ? 8 : 16;
        void* keys = alloc(std::max<uint64_t>(R, 1) * rkb);
        lane.prof.begin(s, "unrank", double(R) * rkb);
        launch_unrank(d_steps, plan.root_child, d_rcum, E, R, nF, vb, rkw, keys, err, s);
        lane.prof.end(s);
        uint64_t* vals = (uint64_t*)alloc(std::max<uint64_t>(R, 1) * 8);
        launch_fill_u64(vals, 0, R, s);
        void* k2 = alloc(std::max<uint64_t>(R, 1) * rkb);
        uint64_t* v2 = (uint64_t*)alloc(std::max<uint64_t>(R, 1) * 8);
        void* tmp = alloc(radix_tmp_bytes(R));
        lane.prof.begin(s, "row_sort", double(R) * (rkb + 8) * 2);
        radix_sort(keys, vals, k2, v2, R, rkw, rbits, 0, tmp, s);
        lane.prof.end(s);
        const uint64_t m = std::min(R, cap);
        std::vector<uint64_t> hrows(m * (rkw == 1 ? 1 : 2));
        uint32_t herr = 0;
        hip_check(hipMemcpyAsync(hrows.data(), keys, m * rkb, hipMemcpyDeviceToHost, s), "copy rows");
        hip_check(hipMemcpyAsync(&herr, err, 4, hipMemcpyDeviceToHost, s), "copy err");
        hip_check(hipStreamSynchronize(s), "sync");
        lane.prof.resolve();
        if (herr) fail(CC_EDEVICE, "row decoder reported an inconsistent index");
        rows->resize(m * size_t(nF));
        const uint64_t vmask = (uint64_t(1) << vb) - 1;
        for (uint64_t i = 0; i < m; i++) {
            u128 key = rkw == 1 ? u128(hrows[i]) : ((u128(hrows[2 * i + 1]) << 64) | hrows[2 * i]);
            for (int j = nF - 1; j >= 0; j--) {
                (*rows)[i * nF + j] = int32_t(uint64_t(key) & vmask);
                key >>= vb;
            }
        }
        *n_rows = m;
    } catch (...) {
        (void)hipStreamSynchronize(s);
        for (void* p : extra) A.release(p);
        release_tables(ctx, &r);
        throw;
    }
    for (void* p : extra) A.release(p);
    release_tables(ctx, &r);
}

}  // namespace ccg
