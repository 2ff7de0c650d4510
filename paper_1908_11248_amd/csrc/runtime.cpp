// Multi-query runtime: concurrent batches over worker lanes, the lane-count
// autotuner, and the serving loop (continuous batching with memory-gated
// admission).  Every query is one run of the DP executor on one lane; lanes
// are independent HIP streams sharing the context's arena, so the kernels of
// concurrent queries overlap on the device.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <cmath>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <mutex>
#include <set>
#include <thread>
#include <unordered_map>
#include <vector>

#include "engine.h"

using namespace ccg;

namespace {

using Clock = std::chrono::steady_clock;

struct QueryRun {
    const cc_decomp* d;
    const uint8_t* colors;
    int B, k;
};

// one query on one lane; returns CC_OK or the error code (message in *err)
int run_one(cc_context* ctx, Lane& lane, const cc_graph* g, const QueryRun& q, uint32_t flags, uint64_t max_entries,
            RunResult* r, std::string* err) {
    try {
        RunRequest rq;
        rq.g = g;
        rq.colors = q.colors;
        rq.B = q.B;
        rq.k = q.k;
        rq.dec = q.d;
        rq.degree_mask = !(flags & CC_NO_DEGREE_MASK);
        rq.sparse_only = (flags & CC_SPARSE_TABLES) != 0;
        rq.classic_expand = (flags & CC_CLASSIC_EXPAND) != 0;
        rq.max_entries = max_entries;
        run_dp_waves(ctx, lane, rq, r);
        return CC_OK;
    } catch (const CcError& e) {
        *err = e.msg;
        return e.code;
    } catch (const std::bad_alloc&) {
        *err = "host allocation failed";
        return CC_ENOMEM;
    }
}

// plan size proxy for scheduling: more and wider bags first
double plan_weight(const cc_decomp* d, int B) {
    double w = 0;
    for (const Step& s : d->plan.steps) w += double(1 << (2 * s.b_out));
    return w * B;
}

int batch_run(cc_context* ctx, const cc_graph* g, int32_t nq, const cc_query* q, uint32_t flags, uint64_t* counts,
              uint8_t* ovf, int lanes, std::string* err) {
    std::vector<size_t> off(nq + 1, 0);
    for (int32_t i = 0; i < nq; i++) off[i + 1] = off[i] + size_t(q[i].coloring->B);
    std::vector<int32_t> order(nq);
    for (int32_t i = 0; i < nq; i++) order[i] = i;
    std::stable_sort(order.begin(), order.end(), [&](int32_t a, int32_t b) {
        return plan_weight(q[a].decomp, q[a].coloring->B) > plan_weight(q[b].decomp, q[b].coloring->B);
    });
    lanes = std::max(1, std::min(lanes, int(nq)));
    for (int l = 0; l < lanes; l++) ctx->worker(l);
    std::atomic<int32_t> next{0};
    std::mutex mu;
    int first_rc = CC_OK;
    std::string first_err;
    std::vector<int32_t> retry;
    int64_t sizes_total = 0;
    std::vector<int64_t> sizes_sum;
    auto worker = [&](int l) {
        (void)hipSetDevice(ctx->device);
        Lane& lane = ctx->worker(l);
        for (;;) {
            int32_t t = next.fetch_add(1);
            if (t >= nq) break;
            int32_t i = order[t];
            QueryRun qr{q[i].decomp, q[i].coloring->colors, q[i].coloring->B, q[i].coloring->k};
            RunResult r;
            std::string e;
            int rc = CC_OK;
            if (q[i].coloring->ready && hipStreamWaitEvent(lane.stream, q[i].coloring->ready, 0) != hipSuccess) {
                rc = CC_EDEVICE;
                e = "hipStreamWaitEvent failed";
            }
            if (rc == CC_OK) rc = run_one(ctx, lane, g, qr, flags, ctx->max_entries, &r, &e);
            std::lock_guard<std::mutex> guard(mu);
            if (rc == CC_ENOMEM && lanes > 1) {
                retry.push_back(i);  // memory was held by concurrent queries
            } else if (rc != CC_OK) {
                if (first_rc == CC_OK) {
                    first_rc = rc;
                    first_err = "query " + std::to_string(i) + ": " + e;
                }
            } else {
                std::copy(r.counts.begin(), r.counts.end(), counts + off[i]);
                if (ovf) std::copy(r.overflow.begin(), r.overflow.end(), ovf + off[i]);
                for (int64_t x : r.node_sizes) sizes_total += x;
            }
        }
    };
    std::vector<std::thread> th;
    for (int l = 1; l < lanes; l++) th.emplace_back(worker, l);
    worker(0);
    for (auto& t : th) t.join();
    std::sort(retry.begin(), retry.end());
    for (int32_t i : retry) {  // alone now
        if (first_rc != CC_OK) break;
        QueryRun qr{q[i].decomp, q[i].coloring->colors, q[i].coloring->B, q[i].coloring->k};
        RunResult r;
        std::string e;
        if (q[i].coloring->ready) (void)hipStreamWaitEvent(ctx->main.stream, q[i].coloring->ready, 0);
        int rc = run_one(ctx, ctx->main, g, qr, flags, ctx->max_entries, &r, &e);
        if (rc != CC_OK) {
            first_rc = rc;
            first_err = "query " + std::to_string(i) + ": " + e;
            break;
        }
        std::copy(r.counts.begin(), r.counts.end(), counts + off[i]);
        if (ovf) std::copy(r.overflow.begin(), r.overflow.end(), ovf + off[i]);
        for (int64_t x : r.node_sizes) sizes_total += x;
    }
    ctx->last_sizes.assign(1, sizes_total);  // batches report the total over all nodes and queries
    if (first_rc != CC_OK) *err = first_err;
    return first_rc;
}

double percentile(std::vector<double> v, double p) {
    if (v.empty()) return 0;
    std::sort(v.begin(), v.end());
    double idx = p * double(v.size() - 1);
    size_t lo = size_t(idx), hi = std::min(v.size() - 1, lo + 1);
    return v[lo] + (v[hi] - v[lo]) * (idx - double(lo));
}

}  // namespace

// ---------------------------------------------------------------------------
// serving

struct cc_server {
    struct Req {
        uint64_t id;
        const cc_decomp* d;
        int32_t k;
        uint64_t seed;
        int32_t B;
        size_t est = 0;
        double model = 0;  // estimate_memory's peak bytes
        Clock::time_point arrival, started, done_at;
        int state = 0;  // 0 waiting/running, 1 done, < 0 error
        bool alone = false;
        std::vector<uint64_t> counts;
        std::vector<uint8_t> ovf;
    };
    cc_context* ctx;
    const cc_graph* g;
    cc_server_opts opts;
    size_t budget = 0, reserved = 0;
    int running = 0, running_alone = 0, running_heavy = 0;
    std::mutex mu;
    std::condition_variable cv_work, cv_done;
    std::deque<uint64_t> queue;
    std::unordered_map<uint64_t, Req> reqs;
    std::map<std::pair<const cc_decomp*, int32_t>, size_t> peak_seen;
    double correction = 1.0;  // running geometric mean of measured peak / model, clamped
    uint64_t next_id = 1;
    bool stopping = false;
    std::vector<std::thread> workers;
    uint64_t submitted = 0, completed = 0, failed = 0, requeued = 0;
    std::vector<double> latencies_ms;
    double service_sum_ms = 0;  // of the completed queries (tail protection)
    std::set<uint64_t> in_flight;
    bool have_first = false;
    Clock::time_point first_arrival, last_done;

    // Admission size of a request: the measured peak of an earlier run of
    // the same decomposition and colouring count, else the memory model of
    // the plan on this graph (estimate_memory) scaled by the running
    // correction, plus the colouring buffer; never above the whole budget
    // (a larger query runs alone and splits itself into waves and ranges).
    size_t estimate(const Req& r) {
        auto it = peak_seen.find({r.d, r.B});
        double e;
        if (it != peak_seen.end())
            e = double(it->second) * 1.125;
        else
            e = r.model * correction + double(g->n) * double(r.B);
        return size_t(std::min(e, double(budget)));
    }

    // a running query is far past the mean service time: admit nothing new
    bool tail_hold() {
        if (opts.tail_factor <= 0 || completed < 4 || in_flight.empty()) return false;
        const double limit = opts.tail_factor * service_sum_ms / double(completed);
        const Clock::time_point now = Clock::now();
        for (uint64_t id : in_flight)
            if (std::chrono::duration<double, std::milli>(now - reqs[id].started).count() > limit) return true;
        return false;
    }

    // oldest admissible request (lock held); 0 if none
    uint64_t pick() {
        if (running_alone || tail_hold()) return 0;
        for (size_t i = 0; i < queue.size(); i++) {
            Req& r = reqs[queue[i]];
            if (r.alone) {
                if (running == 0 && i == 0) return queue[i];
                if (i == 0) return 0;  // waits for the device to drain
                continue;
            }
            if (opts.max_heavy > 0 && heavy(r) && running_heavy >= opts.max_heavy) continue;
            if (reserved + r.est <= budget || running == 0) return queue[i];
        }
        return 0;
    }

    static bool heavy(const Req& r) { return r.d->d.width >= 2; }

    void work(int lane_index) {
        (void)hipSetDevice(ctx->device);
        Lane& lane = ctx->worker(size_t(lane_index));
        std::unique_lock<std::mutex> lk(mu);
        for (;;) {
            uint64_t id = 0;
            cv_work.wait(lk, [&] { return (id = pick()) != 0 || (stopping && queue.empty()); });
            if (id == 0) return;
            queue.erase(std::find(queue.begin(), queue.end(), id));
            Req& r = reqs[id];
            r.started = Clock::now();
            in_flight.insert(id);
            r.est = estimate(r);
            size_t hold = r.alone ? budget : r.est;
            reserved += hold;
            running++;
            if (r.alone) running_alone++;
            const bool hv = heavy(r);
            if (hv) running_heavy++;
            const cc_decomp* d = r.d;
            int32_t k = r.k, B = r.B;
            uint64_t seed = r.seed;
            lk.unlock();

            RunResult res;
            std::string err;
            int rc = CC_OK;
            uint8_t* colors = nullptr;
            try {
                colors = (uint8_t*)ctx->arena.alloc(size_t(g->n) * size_t(B));
                launch_color_hash(colors, g->n, B, k, seed, lane.stream);
            } catch (const CcError& e) {
                rc = e.code;
                err = e.msg;
            }
            if (rc == CC_OK) {
                QueryRun qr{d, colors, B, k};
                rc = run_one(ctx, lane, g, qr, 0, opts.max_entries, &res, &err);
            }
            (void)hipStreamSynchronize(lane.stream);
            if (colors) ctx->arena.release(colors);

            lk.lock();
            in_flight.erase(id);
            reserved -= hold;
            running--;
            if (r.alone) running_alone--;
            if (hv) running_heavy--;
            Req& rr = reqs[id];
            if (rc == CC_ENOMEM && !rr.alone) {
                rr.alone = true;  // run again when nothing else holds memory
                queue.push_front(id);
                requeued++;
            } else {
                rr.done_at = Clock::now();
                if (rc == CC_OK) {
                    rr.state = 1;
                    rr.counts = res.counts;
                    rr.ovf = res.overflow;
                    peak_seen[{d, B}] = std::max(peak_seen[{d, B}], res.peak_bytes + size_t(g->n) * size_t(B));
                    if (rr.model > 0 && res.peak_bytes > 0 && res.chunks == 1) {
                        const double ratio = std::min(4.0, std::max(0.25, double(res.peak_bytes) / rr.model));
                        correction = std::exp(0.8 * std::log(correction) + 0.2 * std::log(ratio));
                        correction = std::min(4.0, std::max(0.5, correction));
                    }
                    completed++;
                    service_sum_ms += std::chrono::duration<double, std::milli>(rr.done_at - rr.started).count();
                    latencies_ms.push_back(std::chrono::duration<double, std::milli>(rr.done_at - rr.arrival).count());
                    last_done = rr.done_at;
                } else {
                    rr.state = rc;
                    failed++;
                }
                cv_done.notify_all();
            }
            cv_work.notify_all();
        }
    }
};

extern "C" {

int cc_set_batch_lanes(cc_context* ctx, int32_t lanes) {
    if (!ctx || lanes < 0 || lanes > 64) return CC_EINVAL;
    ctx->batch_lanes = lanes;
    return CC_OK;
}

int cc_set_table_budget(cc_context* ctx, uint64_t max_entries) {
    if (!ctx) return CC_EINVAL;
    ctx->max_entries = max_entries;
    return CC_OK;
}

int cc_count_batch(cc_context* ctx, const cc_graph* g, int32_t nq, const cc_query* q, uint32_t flags,
                   uint64_t* counts_flat, uint8_t* overflow_flat) {
    if (!ctx || !g || nq < 0 || (nq && !q) || !counts_flat) {
        set_error("bad arguments");
        return CC_EINVAL;
    }
    for (int32_t i = 0; i < nq; i++) {
        if (!q[i].decomp || !q[i].coloring || q[i].coloring->ctx != ctx || q[i].coloring->n != g->n) {
            set_error("query " + std::to_string(i) + ": bad decomposition or colouring");
            return CC_EINVAL;
        }
        if (q[i].coloring->k < q[i].decomp->d.n) {
            set_error("query " + std::to_string(i) + ": fewer colours than pattern vertices");
            return CC_ERANGE;
        }
    }
    if (hipSetDevice(ctx->device) != hipSuccess) {
        set_error("hipSetDevice failed");
        return CC_EDEVICE;
    }
    std::string err;
    int lanes = ctx->batch_lanes > 0 ? ctx->batch_lanes : 4;
    int rc = batch_run(ctx, g, nq, q, flags, counts_flat, overflow_flat, lanes, &err);
    set_error(rc == CC_OK ? "" : err);
    return rc;
}

int cc_tune_batch(cc_context* ctx, const cc_graph* g, int32_t nq, const cc_query* q, uint32_t flags, int32_t* best) {
    if (!ctx || !g || !best || nq <= 0 || !q) {
        set_error("bad arguments");
        return CC_EINVAL;
    }
    size_t total = 0;
    for (int32_t i = 0; i < nq; i++) total += size_t(q[i].coloring->B);
    std::vector<uint64_t> counts(total), first(total);
    bool have_first = false;
    // one timed batch under the current schedule; every schedule must give
    // the same counts
    auto timed = [&](double* dt) {
        auto t0 = Clock::now();
        int rc = cc_count_batch(ctx, g, nq, q, flags, counts.data(), nullptr);
        *dt = std::chrono::duration<double>(Clock::now() - t0).count();
        if (rc != CC_OK) return rc;
        if (!have_first) {
            first = counts;
            have_first = true;
        } else if (counts != first) {
            set_error("schedules gave different counts");
            return CC_EDEVICE;
        }
        return CC_OK;
    };
    // coordinate descent: lanes, then the introduce form threshold, then
    // dense LDS accumulators against sorting in forget and join
    double best_t = 1e300;
    int best_l = 1;
    for (int l : {1, 2, 4, 8}) {
        ctx->batch_lanes = l;
        double dt;
        if (int rc = timed(&dt)) return rc;
        if (dt < best_t) {
            best_t = dt;
            best_l = l;
        }
    }
    ctx->batch_lanes = best_l;
    const int f0 = ctx->entry_factor;
    int best_f = f0;
    for (int f : {1, 8}) {
        ctx->entry_factor = f;
        double dt;
        if (int rc = timed(&dt)) {
            ctx->entry_factor = f0;
            return rc;
        }
        if (dt < best_t) {
            best_t = dt;
            best_f = f;
        }
    }
    ctx->entry_factor = best_f;
    const int s0 = ctx->sort_above_k;
    int best_s = s0;
    for (int sk : {8, 0}) {
        ctx->sort_above_k = sk;
        double dt;
        if (int rc = timed(&dt)) {
            ctx->sort_above_k = s0;
            return rc;
        }
        if (dt < best_t) {
            best_t = dt;
            best_s = sk;
        }
    }
    ctx->sort_above_k = best_s;
    const int m0 = ctx->group_min;
    int best_m = m0;
    for (int gm : {0, 4}) {
        ctx->group_min = gm;
        double dt;
        if (int rc = timed(&dt)) {
            ctx->group_min = m0;
            return rc;
        }
        if (dt < best_t) {
            best_t = dt;
            best_m = gm;
        }
    }
    ctx->group_min = best_m;
    *best = best_l;
    return CC_OK;
}

int cc_get_schedule(const cc_context* ctx, cc_schedule* out) {
    if (!ctx || !out) return CC_EINVAL;
    out->lanes = ctx->batch_lanes;
    out->entry_factor = ctx->entry_factor;
    out->sort_above_k = ctx->sort_above_k;
    out->group_min = ctx->group_min;
    return CC_OK;
}

int cc_set_schedule(cc_context* ctx, const cc_schedule* s) {
    if (!ctx || !s || s->lanes < 0 || s->lanes > 64 || s->entry_factor < 1 || s->sort_above_k < 0 || s->group_min < 0) {
        set_error("bad arguments");
        return CC_EINVAL;
    }
    ctx->batch_lanes = s->lanes;
    ctx->entry_factor = s->entry_factor;
    ctx->sort_above_k = s->sort_above_k;
    ctx->group_min = s->group_min;
    return CC_OK;
}

int cc_server_start(cc_context* ctx, const cc_graph* g, const cc_server_opts* opts, cc_server** out) {
    if (!ctx || !g || !opts || !out || opts->max_inflight < 1 || opts->max_inflight > 64) {
        set_error("bad arguments");
        return CC_EINVAL;
    }
    if (hipSetDevice(ctx->device) != hipSuccess) {
        set_error("hipSetDevice failed");
        return CC_EDEVICE;
    }
    auto* s = new cc_server();
    s->ctx = ctx;
    s->g = g;
    s->opts = *opts;
    s->budget = opts->mem_budget ? std::min(opts->mem_budget, ctx->arena.size()) : ctx->arena.size();
    try {
        for (int l = 0; l < opts->max_inflight; l++) ctx->worker(size_t(l));
    } catch (const CcError& e) {
        set_error(e.msg);
        delete s;
        return e.code;
    }
    for (int l = 0; l < opts->max_inflight; l++) s->workers.emplace_back([s, l] { s->work(l); });
    *out = s;
    return CC_OK;
}

int cc_server_submit(cc_server* srv, const cc_decomp* d, int32_t k, uint64_t seed, int32_t num_colorings,
                     uint64_t* ticket) {
    if (!srv || !d || !ticket || num_colorings < 1) {
        set_error("bad arguments");
        return CC_EINVAL;
    }
    if (k < d->d.n || k > kMaxColours || num_colorings > (1 << 20)) {
        set_error("colours k must satisfy n_F <= k <= " + std::to_string(kMaxColours) +
                  " and num_colorings <= 2^20");
        return CC_ERANGE;
    }
    std::lock_guard<std::mutex> guard(srv->mu);
    if (srv->stopping) {
        set_error("server is stopping");
        return CC_ECANCELLED;
    }
    cc_server::Req r;
    r.id = srv->next_id++;
    r.d = d;
    r.k = k;
    r.seed = seed;
    r.B = num_colorings;
    r.arrival = Clock::now();
    r.model = estimate_memory(srv->g, d, k, num_colorings).peak_bytes;
    r.est = srv->estimate(r);
    if (!srv->have_first) {
        srv->have_first = true;
        srv->first_arrival = r.arrival;
    }
    srv->reqs[r.id] = r;
    srv->queue.push_back(r.id);
    srv->submitted++;
    *ticket = r.id;
    srv->cv_work.notify_all();
    return CC_OK;
}

static int copy_result(cc_server::Req& r, uint64_t* counts, uint8_t* overflow, int32_t* state) {
    *state = r.state;
    if (r.state == 1) {
        if (counts) std::copy(r.counts.begin(), r.counts.end(), counts);
        if (overflow) std::copy(r.ovf.begin(), r.ovf.end(), overflow);
    }
    return CC_OK;
}

int cc_server_poll(cc_server* srv, uint64_t ticket, uint64_t* counts, uint8_t* overflow, int32_t* state) {
    if (!srv || !state) return CC_EINVAL;
    std::lock_guard<std::mutex> guard(srv->mu);
    auto it = srv->reqs.find(ticket);
    if (it == srv->reqs.end()) {
        set_error("unknown ticket");
        return CC_EINVAL;
    }
    return copy_result(it->second, counts, overflow, state);
}

int cc_server_wait(cc_server* srv, uint64_t ticket, uint64_t* counts, uint8_t* overflow, int32_t* state) {
    if (!srv || !state) return CC_EINVAL;
    std::unique_lock<std::mutex> lk(srv->mu);
    auto it = srv->reqs.find(ticket);
    if (it == srv->reqs.end()) {
        set_error("unknown ticket");
        return CC_EINVAL;
    }
    srv->cv_done.wait(lk, [&] { return it->second.state != 0; });
    return copy_result(it->second, counts, overflow, state);
}

int cc_server_stop(cc_server* srv, cc_server_stats* stats) {
    if (!srv) return CC_OK;
    {
        std::lock_guard<std::mutex> guard(srv->mu);
        srv->stopping = true;
        srv->cv_work.notify_all();
    }
    for (auto& t : srv->workers) t.join();
    if (stats) {
        std::memset(stats, 0, sizeof *stats);
        stats->submitted = srv->submitted;
        stats->completed = srv->completed;
        stats->failed = srv->failed;
        stats->requeued = srv->requeued;
        if (srv->completed) {
            stats->wall_s = std::chrono::duration<double>(srv->last_done - srv->first_arrival).count();
            stats->qps = stats->wall_s > 0 ? double(srv->completed) / stats->wall_s : 0;
            stats->p50_ms = percentile(srv->latencies_ms, 0.50);
            stats->p99_ms = percentile(srv->latencies_ms, 0.99);
            double sum = 0, mx = 0;
            for (double x : srv->latencies_ms) {
                sum += x;
                mx = std::max(mx, x);
            }
            stats->mean_ms = sum / double(srv->latencies_ms.size());
            stats->max_ms = mx;
        }
    }
    delete srv;
    return CC_OK;
}

}  // extern "C"
