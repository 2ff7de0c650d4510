// Captured counts: the device work of one count (a tree plan on dense
// tables: every kernel, no host round trip between them) recorded once into
// a HIP graph and replayed for each new batch of colourings.  The plan owns
// its colour buffer and a private slice of the context arena, so the
// addresses baked into the graph stay valid and unshared.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>

#include "engine.h"

using namespace ccg;

struct cc_plan {
    cc_context* ctx = nullptr;
    const cc_graph* g = nullptr;
    const cc_decomp* d = nullptr;
    int k = 0, B = 0;
    uint32_t flags = 0;
    Lane lane;
    Arena arena;
    void* arena_mem = nullptr;
    uint8_t* colors = nullptr;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    SlotCapture cap;
};

namespace {
template <class F>
int guarded_plan(F&& f) {
    try {
        f();
        set_error("");
        return CC_OK;
    } catch (const CcError& e) {
        set_error(e.msg);
        return e.code;
    } catch (const std::bad_alloc&) {
        set_error("host allocation failed");
        return CC_ENOMEM;
    }
}

void plan_free(cc_plan* p) {
    if (!p) return;
    if (p->lane.stream) (void)hipStreamSynchronize(p->lane.stream);
    if (p->exec) (void)hipGraphExecDestroy(p->exec);
    if (p->graph) (void)hipGraphDestroy(p->graph);
    if (p->arena_mem) p->ctx->arena.release(p->arena_mem);
    if (p->colors) p->ctx->arena.release(p->colors);
    p->lane.destroy();
    delete p;
}
}  // namespace

extern "C" {

int cc_plan_create(cc_context* ctx, const cc_graph* g, const cc_decomp* d, int32_t k, int32_t num_colorings,
                   uint32_t flags, cc_plan** out) {
    return guarded_plan([&] {
        if (!ctx || !g || !d || !out || g->ctx != ctx || num_colorings < 1) fail(CC_EINVAL, "bad arguments");
        if (k < d->d.n || k > kMaxColours || num_colorings > (1 << 20))
            fail(CC_ERANGE, "colours k must satisfy n_F <= k <= " + std::to_string(kMaxColours));
        hip_check(hipSetDevice(ctx->device), "hipSetDevice");
        auto* p = new cc_plan();
        p->ctx = ctx;
        p->g = g;
        p->d = d;
        p->k = k;
        p->B = num_colorings;
        p->flags = flags;
        try {
            p->lane.create(nullptr);
            p->lane.result_words(size_t(1) << 15);
            p->colors = (uint8_t*)ctx->arena.alloc(std::max<size_t>(1, size_t(g->n) * size_t(num_colorings)));
            launch_color_hash(p->colors, g->n, num_colorings, k, 0, p->lane.stream);
            RunRequest rq;
            rq.g = g;
            rq.colors = p->colors;
            rq.B = num_colorings;
            rq.k = k;
            rq.dec = d;
            rq.degree_mask = !(flags & CC_NO_DEGREE_MASK);
            // an eager run sizes the plan's memory and checks the dense form
            RunResult sizing;
            run_dp(ctx, p->lane, rq, &sizing);
            if (!sizing.dense)
                fail(CC_ERANGE, "only plans whose tables all fit as dense one-column tables (trees) can be captured");
            // the measured peak, with room for the dense-table estimate the
            // executor checks before it takes the dense form
            const size_t bytes = 3 * sizing.peak_bytes + (size_t(1) << 20);
            p->arena_mem = ctx->arena.alloc(bytes);
            p->arena.init((char*)p->arena_mem, bytes);
            rq.arena = &p->arena;
            rq.capture = &p->cap;
            rq.slot_lb_in = &sizing.slot_lb;
            hip_check(hipStreamBeginCapture(p->lane.stream, hipStreamCaptureModeRelaxed), "hipStreamBeginCapture");
            RunResult rec;
            try {
                run_dp(ctx, p->lane, rq, &rec);
            } catch (...) {
                hipGraph_t dead = nullptr;
                (void)hipStreamEndCapture(p->lane.stream, &dead);
                if (dead) (void)hipGraphDestroy(dead);
                throw;
            }
            hip_check(hipStreamEndCapture(p->lane.stream, &p->graph), "hipStreamEndCapture");
            hip_check(hipGraphInstantiate(&p->exec, p->graph, nullptr, nullptr, 0), "hipGraphInstantiate");
        } catch (...) {
            plan_free(p);
            throw;
        }
        *out = p;
    });
}

int cc_plan_count(cc_plan* p, uint64_t seed, uint64_t* counts, uint8_t* overflow) {
    return guarded_plan([&] {
        if (!p || !counts) fail(CC_EINVAL, "bad arguments");
        hip_check(hipSetDevice(p->ctx->device), "hipSetDevice");
        launch_color_hash(p->colors, p->g->n, p->B, p->k, seed, p->lane.stream);
        hip_check(hipGraphLaunch(p->exec, p->lane.stream), "hipGraphLaunch");
        hip_check(hipStreamSynchronize(p->lane.stream), "hipStreamSynchronize");
        RunResult r;
        p->cap.finish(&r, nullptr);
        std::copy(r.counts.begin(), r.counts.end(), counts);
        if (overflow) std::copy(r.overflow.begin(), r.overflow.end(), overflow);
        p->ctx->last_sizes = r.node_sizes;
    });
}

int cc_plan_destroy(cc_plan* p) {
    if (!p) return CC_OK;
    return guarded_plan([&] {
        (void)hipSetDevice(p->ctx->device);
        plan_free(p);
    });
}

}  // extern "C"
