// C ABI of the colour-coding library (declarations and semantics in
// include/ccgpu.h).  Every entry point converts internal exceptions into a
// status code and a thread-local message.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>
#include <numeric>
#include <vector>

#include "engine.h"

using namespace ccg;

// edge-set cells per stored (directed) edge, rounded up to a power of two
static constexpr uint64_t kEdgeCellFactor = 2;

// Device scratch of cc_count_noalloc: a fixed array in the code object, so
// that call allocates nothing.  Every device the library runs on holds its
// own copy until the process ends.  In host code `scratch` is only a
// stand-in for the symbol: kernels get the device address that
// hipGetSymbolAddress returned for the current device (g_scratch_ptr).
#define CC_NOALLOC_SCRATCH_BYTES (size_t(64) << 20)
static __device__ __align__(256) char scratch[CC_NOALLOC_SCRATCH_BYTES];

namespace {
constexpr int kMaxDevices = 64;
constexpr size_t kResultWordsAtInit = size_t(1) << 15;  // pinned read-back words of the main lane
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};  // per device, set while that device is current
hipError_t g_scratch_err[kMaxDevices] = {};
ccg::Arena g_scratch_arena[kMaxDevices];

// Looks up this device's scratch address once (the device must be current).
// A failure is kept and reported by cc_count_noalloc; the other entry points
// do not use the array.
void lookup_scratch(int device) {
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (g_scratch_ptr[device]) return;
    void* p = nullptr;
    hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    g_scratch_err[device] = e;
    g_scratch_ptr[device] = e == hipSuccess ? p : nullptr;
    if (e != hipSuccess) (void)hipGetLastError();  // not sticky for the other calls
}

thread_local std::string g_last_error;

template <class F>
int guarded(F&& f) {
    try {
        f();
        g_last_error.clear();
        return CC_OK;
    } catch (const CcError& e) {
        g_last_error = e.msg;
        return e.code;
    } catch (const std::bad_alloc&) {
        g_last_error = "host allocation failed";
        return CC_ENOMEM;
    } catch (const std::exception& e) {
        g_last_error = e.what();
        return CC_EINVAL;
    }
}

void need(bool ok, int code, const std::string& msg) {
    if (!ok) fail(code, msg);
}
}  // namespace

namespace ccg {
void set_error(const std::string& msg) { g_last_error = msg; }
}  // namespace ccg

extern "C" {

const char* cc_last_error(void) { return g_last_error.c_str(); }

int cc_context_create(int device, void* arena_dev, size_t arena_bytes, void* hip_stream, cc_context** out) {
    return guarded([&] {
        need(out != nullptr, CC_EINVAL, "out is NULL");
        need(!arena_dev || arena_bytes >= 4096, CC_EINVAL, "a caller arena needs arena_bytes >= 4096");
        need((uintptr_t(arena_dev) & 255) == 0, CC_EINVAL, "a caller arena must be 256-byte aligned");
        int ndev = 0;
        hip_check(hipGetDeviceCount(&ndev), "hipGetDeviceCount");
        need(device >= 0 && device < ndev && device < kMaxDevices, CC_EDEVICE, "no such HIP device");
        hip_check(hipSetDevice(device), "hipSetDevice");
        lookup_scratch(device);  // once per device, with that device current
        auto* c = new cc_context();
        c->device = device;
        try {
            c->main.create((hipStream_t)hip_stream);
            (void)c->main.result_words(kResultWordsAtInit);
            if (arena_dev) {
                // caller-owned device memory (a torch tensor, say): used, never freed
                hipPointerAttribute_t at;
                hip_check(hipPointerGetAttributes(&at, arena_dev), "arena pointer attributes");
                need(at.type == hipMemoryTypeDevice && at.device == device, CC_EINVAL,
                     "the caller arena is not device memory of this device");
                c->arena.init((char*)arena_dev, arena_bytes);
            } else {
                if (arena_bytes == 0) {
                    size_t freeb = 0, total = 0;
                    hip_check(hipMemGetInfo(&freeb, &total), "hipMemGetInfo");
                    arena_bytes = freeb / 4 * 3;
                }
                hip_check(hipMalloc(&c->arena_mem, arena_bytes), "arena hipMalloc");
                c->arena.init((char*)c->arena_mem, arena_bytes);
            }
            std::vector<uint16_t> st = slot_rank_tables();
            hip_check(hipMalloc(&c->slot_tables, st.size() * 2), "hipMalloc");
            hip_check(hipMemcpy(c->slot_tables, st.data(), st.size() * 2, hipMemcpyHostToDevice), "hipMemcpy");
            std::vector<uint32_t> sp = slot_split_tables();
            hip_check(hipMalloc(&c->slot_splits, sp.size() * 4), "hipMalloc");
            hip_check(hipMemcpy(c->slot_splits, sp.data(), sp.size() * 4, hipMemcpyHostToDevice), "hipMemcpy");
            std::vector<uint64_t> pk = slot_pack_tables();
            hip_check(hipMalloc(&c->slot_pack, pk.size() * 8), "hipMalloc");
            hip_check(hipMemcpy(c->slot_pack, pk.data(), pk.size() * 8, hipMemcpyHostToDevice), "hipMemcpy");
            std::vector<uint32_t> pu = slot_push_tables();
            hip_check(hipMalloc(&c->slot_push, pu.size() * 4), "hipMalloc");
            hip_check(hipMemcpy(c->slot_push, pu.data(), pu.size() * 4, hipMemcpyHostToDevice), "hipMemcpy");
        } catch (...) {
            if (c->slot_push) (void)hipFree(c->slot_push);
            if (c->slot_tables) (void)hipFree(c->slot_tables);
            if (c->slot_splits) (void)hipFree(c->slot_splits);
            if (c->slot_pack) (void)hipFree(c->slot_pack);
            if (c->arena_mem) (void)hipFree(c->arena_mem);
            c->main.destroy();
            delete c;
            throw;
        }
        *out = c;
    });
}

int cc_context_destroy(cc_context* ctx) {
    if (!ctx) return CC_OK;
    return guarded([&] {
        (void)hipSetDevice(ctx->device);
        for (auto& w : ctx->workers) w->destroy();
        ctx->main.destroy();
        {
            std::lock_guard<std::mutex> lk(ctx->color_pool->mu);
            ctx->color_pool->alive = false;
            for (auto& b : ctx->color_pool->idle) {
                (void)hipFree(b.buf);
                if (b.ready) (void)hipEventDestroy(b.ready);
            }
            ctx->color_pool->idle.clear();
        }
        if (ctx->slot_tables) (void)hipFree(ctx->slot_tables);
        if (ctx->slot_splits) (void)hipFree(ctx->slot_splits);
        if (ctx->slot_pack) (void)hipFree(ctx->slot_pack);
        if (ctx->slot_push) (void)hipFree(ctx->slot_push);
        if (ctx->arena_mem) (void)hipFree(ctx->arena_mem);
        delete ctx;
    });
}

int cc_load_graph(cc_context* ctx, int32_t n, const int64_t* row_ptr, const int32_t* col, uint32_t flags,
                  cc_graph** out) {
    return guarded([&] {
        need(ctx && out && n >= 0 && (n == 0 || row_ptr), CC_EINVAL, "bad arguments");
        need(n < INT32_MAX, CC_ERANGE, "n_G must be below 2^31");
        std::vector<int64_t> rp(row_ptr, row_ptr + n + 1);
        need(rp[0] == 0, CC_EINVAL, "row_ptr[0] must be 0");
        for (int32_t v = 0; v < n; v++) need(rp[v + 1] >= rp[v], CC_EINVAL, "row_ptr must be non-decreasing");
        int64_t m2 = rp[n];
        std::vector<int32_t> cl(col, col + m2);
        for (int64_t e = 0; e < m2; e++) need(cl[e] >= 0 && cl[e] < n, CC_EINVAL, "column id out of range");
        auto canonical = [&]() {
            for (int32_t v = 0; v < n; v++)
                for (int64_t e = rp[v]; e < rp[v + 1]; e++) {
                    if (cl[e] == v) return false;                            // loop
                    if (e > rp[v] && cl[e] <= cl[e - 1]) return false;       // unsorted / duplicate
                }
            // symmetry: every (v, w) has (w, v)
            for (int32_t v = 0; v < n; v++)
                for (int64_t e = rp[v]; e < rp[v + 1]; e++) {
                    int32_t w = cl[e];
                    if (!std::binary_search(cl.begin() + rp[w], cl.begin() + rp[w + 1], v)) return false;
                }
            return true;
        };
        if (!canonical()) {
            need(flags & CC_GRAPH_CANONICALIZE, CC_EINVAL,
                 "graph is not simple, symmetric and row-sorted (pass CC_GRAPH_CANONICALIZE to fix it)");
            std::vector<std::pair<int32_t, int32_t>> es;
            for (int32_t v = 0; v < n; v++)
                for (int64_t e = rp[v]; e < rp[v + 1]; e++)
                    if (cl[e] != v) {
                        es.push_back({v, cl[e]});
                        es.push_back({cl[e], v});
                    }
            std::sort(es.begin(), es.end());
            es.erase(std::unique(es.begin(), es.end()), es.end());
            std::fill(rp.begin(), rp.end(), 0);
            cl.resize(es.size());
            for (size_t i = 0; i < es.size(); i++) {
                rp[es[i].first + 1]++;
                cl[i] = es[i].second;
            }
            for (int32_t v = 0; v < n; v++) rp[v + 1] += rp[v];
            m2 = int64_t(es.size());
        }
        std::vector<int32_t> src(m2);
        for (int32_t v = 0; v < n; v++)
            for (int64_t e = rp[v]; e < rp[v + 1]; e++) src[e] = v;
        // edge set for adjacency tests: 2m cells or more, a power of two (a
        // load of at most one half; the kernels read a chain a 64-byte group
        // of eight cells at a time, and at this load it rarely leaves its home
        // group, while the table stays small enough for the last-level cache
        // on graphs of 10^7 edges)
        uint64_t cells = 16;
        while (cells < uint64_t(std::max<int64_t>(m2, 1)) * kEdgeCellFactor) cells <<= 1;
        std::vector<uint64_t> eh(cells, kEdgeEmpty);
        for (int32_t v = 0; v < n; v++)
            for (int64_t e = rp[v]; e < rp[v + 1]; e++) {
                const uint32_t w = uint32_t(cl[e]);
                if (w <= uint32_t(v)) continue;  // each edge once
                const uint64_t key = edge_key(uint32_t(v), w);
                uint64_t h = edge_cell(key, cells - 1);
                while (eh[h] != kEdgeEmpty) h = (h + 1) & (cells - 1);
                eh[h] = key;
            }
        std::vector<int32_t> heavy;
        for (int32_t v = 0; v < n; v++)
            if (rp[v + 1] - rp[v] > kHeavyDegree) heavy.push_back(v);
        hip_check(hipSetDevice(ctx->device), "hipSetDevice");
        auto* g = new cc_graph();
        g->ctx = ctx;
        g->n = n;
        g->m2 = m2;
        g->host_rp = rp;
        g->sorted_deg.resize(n);
        for (int32_t v = 0; v < n; v++) g->sorted_deg[v] = rp[v + 1] - rp[v];
        std::sort(g->sorted_deg.begin(), g->sorted_deg.end());
        graph_statistics(g, rp, cl);
        try {
            hip_check(hipMalloc(&g->rp, 8 * size_t(n + 1)), "hipMalloc");
            hip_check(hipMalloc(&g->col, 4 * size_t(std::max<int64_t>(m2, 1))), "hipMalloc");
            hip_check(hipMalloc(&g->esrc, 4 * size_t(std::max<int64_t>(m2, 1))), "hipMalloc");
            hip_check(hipMalloc(&g->ehash, 8 * cells), "hipMalloc");
            {
                std::vector<uint8_t> d8(std::max<int32_t>(n, 1), 0);
                for (int32_t v = 0; v < n; v++) d8[v] = uint8_t(std::min<int64_t>(rp[v + 1] - rp[v], 255));
                hip_check(hipMalloc(&g->deg8, d8.size()), "hipMalloc");
                hip_check(hipMemcpy(g->deg8, d8.data(), d8.size(), hipMemcpyHostToDevice), "hipMemcpy");
            }
            hip_check(hipMemcpy(g->ehash, eh.data(), 8 * cells, hipMemcpyHostToDevice), "hipMemcpy");
            g->ehmask = cells - 1;
            hip_check(hipMalloc(&g->heavy, 4 * std::max<size_t>(heavy.size(), 1)), "hipMalloc");
            g->nheavy = int32_t(heavy.size());
            if (!heavy.empty())
                hip_check(hipMemcpy(g->heavy, heavy.data(), 4 * heavy.size(), hipMemcpyHostToDevice), "hipMemcpy");
            hip_check(hipMemcpy(g->rp, rp.data(), 8 * size_t(n + 1), hipMemcpyHostToDevice), "hipMemcpy");
            if (m2) {
                hip_check(hipMemcpy(g->col, cl.data(), 4 * size_t(m2), hipMemcpyHostToDevice), "hipMemcpy");
                hip_check(hipMemcpy(g->esrc, src.data(), 4 * size_t(m2), hipMemcpyHostToDevice), "hipMemcpy");
            }
        } catch (...) {
            cc_graph_free(g);
            throw;
        }
        *out = g;
    });
}

void cc_graph_free(cc_graph* g) {
    if (!g) return;
    if (g->rp) (void)hipFree(g->rp);
    if (g->col) (void)hipFree(g->col);
    if (g->esrc) (void)hipFree(g->esrc);
    if (g->heavy) (void)hipFree(g->heavy);
    if (g->ehash) (void)hipFree(g->ehash);
    if (g->deg8) (void)hipFree(g->deg8);
    if (g->ball_pre) (void)hipFree(g->ball_pre);
    if (g->ball_w2) (void)hipFree(g->ball_w2);
    if (g->cn_off) (void)hipFree(g->cn_off);
    if (g->cn_col) (void)hipFree(g->cn_col);
    if (g->wd_hk) (void)hipFree(g->wd_hk);
    if (g->wd_hv) (void)hipFree(g->wd_hv);
    if (g->wd_start) (void)hipFree(g->wd_start);
    if (g->wd_mid) (void)hipFree(g->wd_mid);
    delete g;
}

int32_t cc_graph_num_vertices(const cc_graph* g) { return g ? g->n : -1; }

// a device buffer of `bytes` for a colouring and its ready event: an idle
// pair of that size, else new ones
static void color_buffer(cc_context* ctx, cc_coloring* c, size_t bytes) {
    c->pool = ctx->color_pool;
    c->bytes = bytes;
    {
        std::lock_guard<std::mutex> lk(c->pool->mu);
        auto& idle = c->pool->idle;
        for (size_t i = 0; i < idle.size(); i++)
            if (idle[i].bytes == bytes) {
                c->colors = idle[i].buf;
                c->ready = idle[i].ready;
                idle.erase(idle.begin() + i);
                return;
            }
    }
    hip_check(hipMalloc(&c->colors, bytes), "hipMalloc colours");
    hipError_t e = hipEventCreateWithFlags(&c->ready, hipEventDisableTiming);
    if (e != hipSuccess) {
        (void)hipFree(c->colors);
        c->colors = nullptr;
        c->ready = nullptr;
        hip_check(e, "hipEventCreate");
    }
}

// a stream that reads colouring c waits until its colours are written
static void wait_colors(const cc_coloring* c, hipStream_t s) {
    if (c->ready) hip_check(hipStreamWaitEvent(s, c->ready, 0), "hipStreamWaitEvent");
}

int cc_color(cc_context* ctx, const cc_graph* g, int32_t k, uint64_t seed, int32_t num_colorings,
             cc_coloring** out) {
    return guarded([&] {
        need(ctx && g && out, CC_EINVAL, "bad arguments");
        need(k >= 1 && k <= kMaxColours, CC_ERANGE, "k must be in [1, " + std::to_string(kMaxColours) + "]");
        need(num_colorings >= 1 && num_colorings <= (1 << 20), CC_ERANGE, "num_colorings out of range");
        hip_check(hipSetDevice(ctx->device), "hipSetDevice");
        auto* c = new cc_coloring();
        c->ctx = ctx;
        c->n = g->n;
        c->k = k;
        c->B = num_colorings;
        try {
            color_buffer(ctx, c, std::max<size_t>(1, size_t(g->n) * num_colorings));
        } catch (...) {
            delete c;
            throw;
        }
        launch_color_hash(c->colors, g->n, num_colorings, k, seed, ctx->main.stream);
        // no wait here: readers on other streams wait for this event
        hipError_t e = hipEventRecord(c->ready, ctx->main.stream);
        if (e != hipSuccess) {
            cc_coloring_free(c);
            hip_check(e, "hipEventRecord");
        }
        *out = c;
    });
}

int cc_color_explicit(cc_context* ctx, const cc_graph* g, int32_t k, int32_t num_colorings, const uint8_t* colors,
                      cc_coloring** out) {
    return guarded([&] {
        need(ctx && g && out && colors, CC_EINVAL, "bad arguments");
        need(k >= 1 && k <= kMaxColours, CC_ERANGE, "k must be in [1, " + std::to_string(kMaxColours) + "]");
        need(num_colorings >= 1 && num_colorings <= (1 << 20), CC_ERANGE, "num_colorings out of range");
        size_t total = size_t(g->n) * num_colorings;
        for (size_t i = 0; i < total; i++) need(colors[i] < k, CC_EINVAL, "colour out of range");
        hip_check(hipSetDevice(ctx->device), "hipSetDevice");
        auto* c = new cc_coloring();
        c->ctx = ctx;
        c->n = g->n;
        c->k = k;
        c->B = num_colorings;
        try {
            color_buffer(ctx, c, std::max<size_t>(total, 1));
        } catch (...) {
            delete c;
            throw;
        }
        if (total) {
            hipError_t e = hipMemcpy(c->colors, colors, total, hipMemcpyHostToDevice);
            if (e != hipSuccess) {
                cc_coloring_free(c);
                hip_check(e, "hipMemcpy colours");
            }
        }
        *out = c;
    });
}

int cc_coloring_download(const cc_coloring* c, int32_t b, uint8_t* colors_out) {
    return guarded([&] {
        need(c && colors_out && b >= 0 && b < c->B, CC_EINVAL, "bad arguments");
        hip_check(hipSetDevice(c->ctx->device), "hipSetDevice");
        if (c->ready) hip_check(hipEventSynchronize(c->ready), "hipEventSynchronize");
        if (c->n)
            hip_check(hipMemcpy(colors_out, c->colors + size_t(b) * c->n, size_t(c->n), hipMemcpyDeviceToHost),
                      "hipMemcpy");
    });
}

void cc_coloring_free(cc_coloring* c) {
    if (!c) return;
    if (c->colors) {
        bool kept = false;
        if (c->pool) {
            std::lock_guard<std::mutex> lk(c->pool->mu);
            if (c->pool->alive && c->pool->idle.size() < ColorPool::kMax) {
                c->pool->idle.push_back({c->bytes, c->colors, c->ready});
                kept = true;
            }
        }
        if (!kept) {
            (void)hipFree(c->colors);
            if (c->ready) (void)hipEventDestroy(c->ready);
        }
    }
    delete c;
}

static std::vector<std::pair<int, int>> edge_vec(int32_t m_F, const int32_t* edges) {
    std::vector<std::pair<int, int>> e;
    for (int32_t i = 0; i < m_F; i++) e.push_back({edges[2 * i], edges[2 * i + 1]});
    return e;
}

int cc_build_decomposition(int32_t n_F, int32_t m_F, const int32_t* edges, uint32_t flags, cc_decomp** out) {
    (void)flags;
    return guarded([&] {
        need(out && m_F >= 0 && (m_F == 0 || edges), CC_EINVAL, "bad arguments");
        auto* d = new cc_decomp();
        std::string err;
        int rc = build_decomposition(n_F, edge_vec(m_F, edges), &d->d, &err);
        if (rc == CC_OK) rc = make_plan(d->d, &d->plan, &err);
        if (rc != CC_OK) {
            delete d;
            fail(rc, err);
        }
        *out = d;
    });
}

int cc_decomp_export(const cc_decomp* d, int32_t* buf, size_t cap, size_t* len) {
    return guarded([&] {
        need(d && len, CC_EINVAL, "bad arguments");
        size_t N = d->d.nodes.size();
        *len = 1 + 5 * N;
        need(buf && cap >= *len, CC_ERANGE, "buffer too small");
        buf[0] = int32_t(N);
        for (size_t i = 0; i < N; i++) {
            const TdNode& x = d->d.nodes[i];
            buf[1 + 5 * i] = x.type;
            buf[2 + 5 * i] = x.u;
            buf[3 + 5 * i] = x.c0;
            buf[4 + 5 * i] = x.c1;
            buf[5 + 5 * i] = int32_t(x.bag);
        }
    });
}

int cc_decomp_import(int32_t n_F, int32_t m_F, const int32_t* edges, const int32_t* buf, size_t len,
                     cc_decomp** out) {
    return guarded([&] {
        need(out && buf && len >= 1 && (m_F == 0 || edges), CC_EINVAL, "bad arguments");
        need(n_F >= 1 && n_F <= kMaxPattern, CC_ERANGE, "pattern size must be in [1, 16]");
        int32_t N = buf[0];
        need(N >= 1 && len == size_t(1 + 5 * N), CC_EINVAL, "length does not match the node count");
        auto* d = new cc_decomp();
        d->d.n = n_F;
        for (auto& e : edge_vec(m_F, edges)) {
            if (e.first < 0 || e.second < 0 || e.first >= n_F || e.second >= n_F || e.first == e.second) {
                delete d;
                fail(CC_EINVAL, "pattern edge out of range or a loop");
            }
            d->d.adj[e.first] |= 1u << e.second;
            d->d.adj[e.second] |= 1u << e.first;
        }
        for (int a = 0; a < n_F; a++)
            for (uint32_t m = d->d.adj[a]; m; m &= m - 1) {
                int b = __builtin_ctz(m);
                if (a < b) d->d.edges.push_back({a, b});
            }
        int width = 0;
        for (int32_t i = 0; i < N; i++) {
            TdNode x{buf[1 + 5 * i], buf[2 + 5 * i], buf[3 + 5 * i], buf[4 + 5 * i], uint32_t(buf[5 + 5 * i])};
            d->d.nodes.push_back(x);
            width = std::max(width, __builtin_popcount(x.bag) - 1);
        }
        d->d.width = width;
        std::string err;
        int rc = validate_decomposition(d->d, &err);
        if (rc == CC_OK) rc = make_plan(d->d, &d->plan, &err);
        if (rc != CC_OK) {
            delete d;
            fail(rc, err);
        }
        *out = d;
    });
}

int32_t cc_decomp_width(const cc_decomp* d) { return d ? d->d.width : -1; }

int cc_decomp_describe(const cc_decomp* d, char* buf, size_t cap, size_t* len) {
    return guarded([&] {
        need(d && len, CC_EINVAL, "bad arguments");
        std::string out = describe_plan(d->d, d->plan);
        *len = out.size() + 1;
        need(buf && cap >= *len, CC_ERANGE, "buffer too small");
        std::memcpy(buf, out.c_str(), out.size() + 1);
    });
}

void cc_decomp_free(cc_decomp* d) { delete d; }

static void check_run_args(cc_context* ctx, const cc_graph* g, const cc_coloring* c, const cc_decomp* d) {
    need(ctx && g && c && d, CC_EINVAL, "bad arguments");
    need(g->ctx == ctx && c->ctx == ctx, CC_EINVAL, "graph or colouring belongs to another context");
    need(c->n == g->n, CC_EINVAL, "colouring and graph sizes differ");
    need(c->k >= d->d.n, CC_ERANGE, "fewer colours than pattern vertices");
}

int cc_count(cc_context* ctx, const cc_graph* g, const cc_coloring* c, const cc_decomp* d, uint32_t flags,
             uint64_t* counts, uint8_t* overflow) {
    return guarded([&] {
        check_run_args(ctx, g, c, d);
        need(counts != nullptr, CC_EINVAL, "counts is NULL");
        hip_check(hipSetDevice(ctx->device), "hipSetDevice");
        RunRequest rq;
        rq.g = g;
        rq.colors = c->colors;
        rq.B = c->B;
        rq.k = c->k;
        rq.dec = d;
        rq.degree_mask = !(flags & CC_NO_DEGREE_MASK);
        rq.sparse_only = (flags & CC_SPARSE_TABLES) != 0;
        rq.classic_expand = (flags & CC_CLASSIC_EXPAND) != 0;
        rq.max_entries = ctx->max_entries;
        RunResult r;
        wait_colors(c, ctx->main.stream);
        run_dp_waves(ctx, ctx->main, rq, &r);
        std::copy(r.counts.begin(), r.counts.end(), counts);
        if (overflow) std::copy(r.overflow.begin(), r.overflow.end(), overflow);
        ctx->last_sizes = r.node_sizes;
        ctx->last_chunks = r.chunks;
    });
}

int cc_count_range(cc_context* ctx, const cc_graph* g, const cc_coloring* c, const cc_decomp* d, uint32_t flags,
                   int32_t lo, int32_t hi, uint64_t* counts, uint8_t* overflow) {
    return guarded([&] {
        check_run_args(ctx, g, c, d);
        need(counts != nullptr, CC_EINVAL, "counts is NULL");
        need(lo >= 0 && lo <= hi && hi <= g->n, CC_EINVAL, "need 0 <= lo <= hi <= n_G");
        hip_check(hipSetDevice(ctx->device), "hipSetDevice");
        RunRequest rq;
        rq.g = g;
        rq.colors = c->colors;
        rq.B = c->B;
        rq.k = c->k;
        rq.dec = d;
        rq.degree_mask = !(flags & CC_NO_DEGREE_MASK);
        rq.sparse_only = (flags & CC_SPARSE_TABLES) != 0;
        rq.classic_expand = (flags & CC_CLASSIC_EXPAND) != 0;
        rq.max_entries = ctx->max_entries;
        rq.anchor_lo = lo;
        rq.anchor_hi = hi;
        RunResult r;
        wait_colors(c, ctx->main.stream);
        run_dp_waves(ctx, ctx->main, rq, &r);
        std::copy(r.counts.begin(), r.counts.end(), counts);
        if (overflow) std::copy(r.overflow.begin(), r.overflow.end(), overflow);
        ctx->last_sizes = r.node_sizes;
        ctx->last_chunks = r.chunks;
    });
}

int32_t cc_last_chunk_count(const cc_context* ctx) { return ctx ? ctx->last_chunks : -1; }

int cc_estimate_memory(const cc_graph* g, const cc_decomp* d, int32_t k, int32_t num_colorings, double* peak_bytes,
                       double* entries) {
    return guarded([&] {
        need(g && d && peak_bytes && num_colorings >= 1, CC_EINVAL, "bad arguments");
        need(k >= d->d.n && k <= kMaxColours, CC_ERANGE, "colours k must satisfy n_F <= k <= " + std::to_string(kMaxColours));
        MemEstimate e = estimate_memory(g, d, k, num_colorings);
        *peak_bytes = e.peak_bytes;
        if (entries) *entries = e.total_entries;
    });
}

int cc_count_noalloc(cc_context* ctx, const cc_graph* g, const cc_coloring* c, const cc_decomp* d, uint32_t flags,
                     uint64_t* counts, uint8_t* overflow) {
    return guarded([&] {
        check_run_args(ctx, g, c, d);
        need(counts != nullptr, CC_EINVAL, "counts is NULL");
        // every run holds at least its first leaf table: B x n entries of 16 bytes
        const uint64_t least = uint64_t(c->B) * uint64_t(std::max(g->n, 1)) * 16u;
        need(least <= CC_NOALLOC_SCRATCH_BYTES, CC_ERANGE,
             "colourings x vertices = " + std::to_string(uint64_t(c->B) * uint64_t(g->n)) +
                 " is too large for the " + std::to_string(CC_NOALLOC_SCRATCH_BYTES >> 20) +
                 " MiB static scratch of cc_count_noalloc");
        hip_check(hipSetDevice(ctx->device), "hipSetDevice");
        void* base = nullptr;
        {
            std::lock_guard<std::mutex> lk(g_scratch_mu);
            base = g_scratch_ptr[ctx->device];  // looked up when the context was created
            if (!base)
                fail(CC_EDEVICE, std::string("hipGetSymbolAddress(scratch) failed: ") +
                                     hipGetErrorString(g_scratch_err[ctx->device]));
        }
        Arena& A = g_scratch_arena[ctx->device];
        A.init((char*)base, CC_NOALLOC_SCRATCH_BYTES);  // the last call's contents are dead
        RunRequest rq;
        rq.g = g;
        rq.colors = c->colors;
        rq.B = c->B;
        rq.k = c->k;
        rq.dec = d;
        rq.degree_mask = !(flags & CC_NO_DEGREE_MASK);
        rq.sparse_only = (flags & CC_SPARSE_TABLES) != 0;
        rq.classic_expand = (flags & CC_CLASSIC_EXPAND) != 0;
        rq.arena = &A;
        rq.no_alloc = true;
        RunResult r;
        wait_colors(c, ctx->main.stream);
        try {
            run_dp(ctx, ctx->main, rq, &r);
        } catch (const CcError& e) {
            if (e.code == CC_ENOMEM)
                fail(CC_ERANGE, "the DP tables exceed the " + std::to_string(CC_NOALLOC_SCRATCH_BYTES >> 20) +
                                    " MiB static scratch of cc_count_noalloc (" + e.msg + ")");
            throw;
        }
        std::copy(r.counts.begin(), r.counts.end(), counts);
        if (overflow) std::copy(r.overflow.begin(), r.overflow.end(), overflow);
        ctx->last_sizes = r.node_sizes;
    });
}

int cc_count_by_vertex(cc_context* ctx, const cc_graph* g, const cc_coloring* c, int32_t b, const cc_decomp* d,
                       uint32_t flags, uint64_t* per_vertex, uint64_t* count, uint8_t* overflow) {
    return guarded([&] {
        check_run_args(ctx, g, c, d);
        need(b >= 0 && b < c->B, CC_EINVAL, "colouring index out of range");
        need(per_vertex != nullptr, CC_EINVAL, "per_vertex is NULL");
        const TdNode& rc = d->d.nodes[d->d.nodes[d->d.nodes.size() - 1].c0];
        need(rc.bag == 1u, CC_EINVAL, "the node below the root must hold pattern vertex 0 only");
        hip_check(hipSetDevice(ctx->device), "hipSetDevice");
        RunRequest rq;
        rq.g = g;
        rq.colors = c->colors + size_t(b) * g->n;
        rq.B = 1;
        rq.k = c->k;
        rq.dec = d;
        rq.degree_mask = !(flags & CC_NO_DEGREE_MASK);
        rq.sparse_only = (flags & CC_SPARSE_TABLES) != 0;
        rq.classic_expand = (flags & CC_CLASSIC_EXPAND) != 0;
        rq.per_vertex = true;
        rq.max_entries = ctx->max_entries;
        RunResult r;
        wait_colors(c, ctx->main.stream);
        run_dp(ctx, ctx->main, rq, &r);
        std::copy(r.per_vertex.begin(), r.per_vertex.end(), per_vertex);
        if (count) *count = r.counts[0];
        if (overflow) *overflow = r.overflow[0];
        ctx->last_sizes = r.node_sizes;
    });
}

int cc_last_table_sizes(const cc_context* ctx, int64_t* entries, size_t cap, size_t* n_nodes) {
    return guarded([&] {
        need(ctx && n_nodes, CC_EINVAL, "bad arguments");
        *n_nodes = ctx->last_sizes.size();
        for (size_t i = 0; i < std::min(cap, ctx->last_sizes.size()); i++) entries[i] = ctx->last_sizes[i];
    });
}

int cc_profile_enable(cc_context* ctx, int enable) {
    return guarded([&] {
        need(ctx != nullptr, CC_EINVAL, "ctx is NULL");
        ctx->main.prof.reset();
        ctx->main.prof.on = enable != 0;
        for (auto& w : ctx->workers) {
            w->prof.reset();
            w->prof.on = enable != 0;
        }
    });
}

int cc_profile_filter(cc_context* ctx, const char* name, uint32_t every) {
    return guarded([&] {
        need(ctx != nullptr, CC_EINVAL, "ctx is NULL");
        std::string n = name ? name : "";
        need(n.size() < 32, CC_EINVAL, "kernel names are shorter than 32 characters");
        for (ccg::Lane* l : {&ctx->main}) {
            l->prof.only = n;
            l->prof.every = every ? every : 1;
            l->prof.seen_ = 0;
        }
        for (auto& w : ctx->workers) {
            w->prof.only = n;
            w->prof.every = every ? every : 1;
            w->prof.seen_ = 0;
        }
    });
}

int cc_profile_read(cc_context* ctx, cc_kernel_stat* stats, size_t cap, size_t* n) {
    return guarded([&] {
        need(ctx && n, CC_EINVAL, "bad arguments");
        // statistics of every lane, merged by kernel name
        std::vector<KernelStat> st;
        auto merge = [&](Profiler& p) {
            p.resolve();
            for (const auto& k : p.stats()) {
                auto it = std::find_if(st.begin(), st.end(), [&](const KernelStat& x) { return x.name == k.name; });
                if (it == st.end()) {
                    st.push_back(k);
                } else {
                    it->launches += k.launches;
                    it->ms += k.ms;
                    it->bytes += k.bytes;
                }
            }
        };
        merge(ctx->main.prof);
        for (auto& w : ctx->workers) merge(w->prof);
        *n = st.size();
        for (size_t i = 0; i < std::min(cap, st.size()); i++) {
            std::memset(stats[i].name, 0, sizeof stats[i].name);
            std::strncpy(stats[i].name, st[i].name.c_str(), sizeof stats[i].name - 1);
            stats[i].launches = st[i].launches;
            stats[i].total_ms = st[i].ms;
            stats[i].algo_bytes = st[i].bytes;
        }
    });
}

int cc_enumerate(cc_context* ctx, const cc_graph* g, const cc_coloring* c, int32_t b, const cc_decomp* d,
                 uint64_t cap, int32_t* rows, uint64_t* n_rows, uint64_t* total) {
    return guarded([&] {
        check_run_args(ctx, g, c, d);
        need(b >= 0 && b < c->B, CC_EINVAL, "colouring index out of range");
        need(n_rows && total && (cap == 0 || rows), CC_EINVAL, "bad arguments");
        hip_check(hipSetDevice(ctx->device), "hipSetDevice");
        std::vector<int32_t> out;
        wait_colors(c, ctx->main.stream);
        run_enumerate(ctx, ctx->main, g, c->colors + size_t(b) * g->n, c->k, d, cap, &out, n_rows, total);
        if (!out.empty()) std::memcpy(rows, out.data(), out.size() * sizeof(int32_t));
    });
}

}  // extern "C"
