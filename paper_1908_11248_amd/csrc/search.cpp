// Around the counting DP: occurrences that differ in their vertex sets
// (Sec. 5.2 remark: the implementation can count all mappings, or only
// occurrences with distinct vertex sets), and the repetition driver of the
// randomised algorithm (Sec. 2.1: a fixed occurrence is colourful with
// probability n_F!/n_F^{n_F} >= e^{-n_F}, so after l runs with fresh random
// colourings it is missed with probability at most (1 - e^{-n_F})^l <=
// exp(-l e^{-n_F}); l = ceil(e^{n_F} ln(1/eps)) runs bound that by eps; the
// paper's experiments use eps = 1/e and stop at the first 100 000 solutions,
// Sec. 5.2).  Rows come from the device enumeration (Sec. 4); the
// de-duplication across colourings is host work on the rows returned.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <set>
#include <vector>

#include "engine.h"

using namespace ccg;

namespace {

template <class F>
int guarded_search(F&& f) {
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

// rows (n_F ints each) -> their vertex sets, sorted within the row
void to_sets(std::vector<int32_t>* rows, int nF) {
    for (size_t i = 0; i + size_t(nF) <= rows->size(); i += size_t(nF))
        std::sort(rows->begin() + i, rows->begin() + i + nF);
}

}  // namespace

extern "C" {

int cc_vertex_sets(cc_context* ctx, const cc_graph* g, const cc_coloring* c, int32_t b, const cc_decomp* d, uint64_t cap,
                   int32_t* sets, uint64_t* n_sets, uint64_t* n_mappings) {
    return guarded_search([&] {
        if (!ctx || !g || !c || !d || !n_sets || !n_mappings || b < 0 || b >= c->B || g->ctx != ctx || c->ctx != ctx ||
            c->n != g->n)
            fail(CC_EINVAL, "bad arguments");
        if (c->k < d->d.n) fail(CC_ERANGE, "fewer colours than pattern vertices");
        hip_check(hipSetDevice(ctx->device), "hipSetDevice");
        const int nF = d->d.n;
        std::vector<int32_t> rows;
        uint64_t nr = 0, total = 0;
        if (c->ready) hip_check(hipStreamWaitEvent(ctx->main.stream, c->ready, 0), "hipStreamWaitEvent");
        run_enumerate(ctx, ctx->main, g, c->colors + size_t(b) * g->n, c->k, d, cap, &rows, &nr, &total);
        *n_mappings = total;
        if (total > cap) fail(CC_ERANGE, "the mappings (" + std::to_string(total) + ") exceed cap");
        to_sets(&rows, nF);
        // distinct sorted rows, in lexicographic order
        std::vector<size_t> idx(nr);
        for (size_t i = 0; i < nr; i++) idx[i] = i;
        auto row = [&](size_t i) { return rows.data() + i * size_t(nF); };
        std::sort(idx.begin(), idx.end(), [&](size_t x, size_t y) {
            return std::lexicographical_compare(row(x), row(x) + nF, row(y), row(y) + nF);
        });
        uint64_t m = 0;
        for (size_t j = 0; j < idx.size(); j++) {
            if (j > 0 && std::equal(row(idx[j]), row(idx[j]) + nF, row(idx[j - 1]))) continue;
            if (sets) std::memcpy(sets + m * size_t(nF), row(idx[j]), sizeof(int32_t) * size_t(nF));
            m++;
        }
        *n_sets = m;
    });
}

int cc_search(cc_context* ctx, const cc_graph* g, const cc_decomp* d, const cc_search_opts* opts, int32_t* rows_out,
              uint64_t* n_rows, uint64_t* colourings_run, uint64_t* colourings_planned) {
    return guarded_search([&] {
        if (!ctx || !g || !d || !opts || !n_rows || !colourings_run || !colourings_planned || g->ctx != ctx)
            fail(CC_EINVAL, "bad arguments");
        if (!(opts->eps > 0.0 && opts->eps < 1.0)) fail(CC_EINVAL, "eps must lie in (0, 1)");
        if (opts->max_solutions == 0 || !rows_out) fail(CC_EINVAL, "need max_solutions >= 1 and a rows buffer");
        const int nF = d->d.n;
        const int k = nF;  // the paper colours with exactly n_F colours
        if (k > kMaxColours) fail(CC_ERANGE, "n_F above the colour limit");
        hip_check(hipSetDevice(ctx->device), "hipSetDevice");
        const double l = std::ceil(std::exp(double(nF)) * std::log(1.0 / opts->eps));
        const uint64_t planned = l > 1e15 ? uint64_t(1e15) : uint64_t(l);
        *colourings_planned = planned;
        const int batch = std::max(1, std::min<int>(opts->batch > 0 ? opts->batch : 16, 1 << 12));
        const bool by_set = (opts->flags & CC_SEARCH_DISTINCT_SETS) != 0;
        std::set<std::vector<int32_t>> found;
        uint64_t run = 0;
        Lane& lane = ctx->main;
        uint8_t* colors = nullptr;
        try {
            colors = (uint8_t*)ctx->arena.alloc(size_t(g->n) * size_t(batch));
            while (run < planned && found.size() < opts->max_solutions) {
                const int B = int(std::min<uint64_t>(uint64_t(batch), planned - run));
                // colourings run .. run + B - 1 of the seed, as cc_color(k, seed) numbers them
                launch_color_hash_from(colors, g->n, B, k, opts->seed, uint32_t(run), lane.stream);
                RunRequest rq;
                rq.g = g;
                rq.colors = colors;
                rq.B = B;
                rq.k = k;
                rq.dec = d;
                rq.max_entries = ctx->max_entries;
                RunResult r;
                run_dp_waves(ctx, lane, rq, &r);
                for (int b = 0; b < B && found.size() < opts->max_solutions; b++) {
                    run++;
                    if (r.counts[size_t(b)] == 0 && !r.overflow[size_t(b)]) continue;
                    std::vector<int32_t> rows;
                    uint64_t nr = 0, total = 0;
                    run_enumerate(ctx, lane, g, colors + size_t(b) * g->n, k, d, opts->max_solutions, &rows, &nr, &total);
                    if (by_set) to_sets(&rows, nF);
                    for (uint64_t i = 0; i < nr; i++)
                        found.insert(std::vector<int32_t>(rows.begin() + i * nF, rows.begin() + (i + 1) * nF));
                }
                if (found.size() >= opts->max_solutions) break;
            }
        } catch (...) {
            (void)hipStreamSynchronize(lane.stream);
            if (colors) ctx->arena.release(colors);
            throw;
        }
        (void)hipStreamSynchronize(lane.stream);
        ctx->arena.release(colors);
        *colourings_run = run;
        uint64_t m = 0;
        for (const auto& r : found) {
            if (m == opts->max_solutions) break;
            std::memcpy(rows_out + m * size_t(nF), r.data(), sizeof(int32_t) * size_t(nF));
            m++;
        }
        *n_rows = m;
    });
}

}  // extern "C"
