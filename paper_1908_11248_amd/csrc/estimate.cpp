// Table-memory estimate of a query: the serving loop admits queries by it
// (a query starts when its estimated peak fits the free memory budget).
//
// The model follows the sizes the DP rules of Sec. 3.1 produce, per
// colouring, from degree statistics of G (the paper's memory bound,
// O(n_G^{tw+1} tw n_F 2^{n_F}), Sec. 1, is far too loose to admit by):
//   leaf u        the vertices passing the degree mask;
//   introduce u   child entries x candidates x P(colour of the candidate not
//                 yet used) x P(every further bag neighbour adjacent);
//                 candidates come from a bag neighbour's adjacency list (the
//                 mean degree of an edge's endpoint, restricted to endpoints
//                 passing the degree mask), or all of V(G) without one;
//   forget u      the child's entries, capped by the number of distinct
//                 (bag images, colour set) keys the smaller bag can hold;
//   join          the larger child, under the same cap;
// where the cap for a bag of b vertices and colour sets of size s is
// n_G * dbar^(b-1) * C(k - b, s - b) (connected b-tuples times the colour
// sets containing the bag's colours), dbar the mean neighbour degree.
#include <algorithm>
#include <cmath>
#include <cstdint>
#include <vector>

#include "engine.h"

namespace ccg {

void graph_statistics(cc_graph* g, const std::vector<int64_t>& rp, const std::vector<int32_t>& col) {
    const int32_t n = g->n;
    g->deg_mass.assign(size_t(n) + 1, 0);
    for (int32_t i = n - 1; i >= 0; i--) g->deg_mass[size_t(i)] = g->deg_mass[size_t(i) + 1] + g->sorted_deg[size_t(i)];
    double s1 = 0, s2 = 0, wedges = 0;
    for (int32_t v = 0; v < n; v++) {
        const double d = double(rp[size_t(v) + 1] - rp[size_t(v)]);
        s1 += d;
        s2 += d * d;
        wedges += d * (d - 1) / 2;
    }
    g->nb_degree = s1 > 0 ? s2 / s1 : 0;
    // transitivity from 2^14 wedges drawn with probability proportional to
    // their centre's wedge count (a fixed splitmix64 stream: deterministic)
    g->transitivity = 0;
    if (wedges <= 0) return;
    std::vector<double> cum(size_t(n) + 1, 0);
    for (int32_t v = 0; v < n; v++) {
        const double d = double(rp[size_t(v) + 1] - rp[size_t(v)]);
        cum[size_t(v) + 1] = cum[size_t(v)] + d * (d - 1) / 2;
    }
    uint64_t state = 0x5eedULL;
    auto next = [&]() {
        uint64_t z = (state += 0x9E3779B97F4A7C15ULL);
        z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
        z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
        return z ^ (z >> 31);
    };
    const int samples = 1 << 14;
    int closed = 0;
    for (int t = 0; t < samples; t++) {
        const double x = double(next() >> 11) * (1.0 / 9007199254740992.0) * cum[size_t(n)];
        int32_t v = int32_t(std::upper_bound(cum.begin(), cum.end(), x) - cum.begin()) - 1;
        v = std::min(std::max(v, 0), n - 1);
        const int64_t d = rp[size_t(v) + 1] - rp[size_t(v)];
        if (d < 2) continue;
        const int64_t i = int64_t(next() % uint64_t(d));
        int64_t j = int64_t(next() % uint64_t(d - 1));
        if (j >= i) j++;
        const int32_t a = col[size_t(rp[size_t(v)] + i)], b = col[size_t(rp[size_t(v)] + j)];
        if (std::binary_search(col.begin() + rp[size_t(a)], col.begin() + rp[size_t(a) + 1], b)) closed++;
    }
    g->transitivity = double(closed) / samples;
}

namespace {
double binom_d(int a, int b) {
    if (b < 0 || b > a) return 0;
    double c = 1;
    for (int i = 0; i < b; i++) c = c * double(a - i) / double(i + 1);
    return c;
}
}  // namespace

MemEstimate estimate_memory(const cc_graph* g, const cc_decomp* d, int k, int B) {
    const Plan& plan = d->plan;
    const size_t S = plan.steps.size();
    MemEstimate est;
    est.entries.assign(S, 0);
    std::vector<int> s(S, 0);  // colour-set size = pattern vertices below
    const double n = double(std::max(g->n, 1));
    const double dbar = std::max(1.0, g->nb_degree);
    const double T = std::min(1.0, std::max(g->transitivity, 1.0 / n));
    auto cap = [&](int b, int sz) {
        if (b <= 0) return binom_d(k, sz);
        return n * std::pow(dbar, b - 1) * binom_d(k - b, sz - b);
    };
    for (size_t i = 0; i < S; i++) {
        const Step& st = plan.steps[i];
        const double in0 = st.in0 >= 0 ? est.entries[size_t(st.in0)] : 0;
        const int s0 = st.in0 >= 0 ? s[size_t(st.in0)] : 0;
        double out = 0;
        switch (st.kind) {
            case S_LEAF:
                s[i] = 1;
                out = double(g->count_deg_at_least(st.degF));
                break;
            case S_INTRO_PUSH:
            case S_INTRO_PULL: {
                s[i] = s0 + 1;
                const double free_colour = double(std::max(0, k - s0)) / double(k);
                const double cand = st.anchor >= 0 ? dbar * g->nb_fraction_at_least(st.degF)
                                                   : double(g->count_deg_at_least(st.degF));
                out = in0 * cand * free_colour * std::pow(T, st.nchk);
                out = std::min(out, cap(st.b_out, s[i]));
                break;
            }
            case S_FORGET_LAST:
                s[i] = s0;
                out = std::min(in0, cap(st.b_out, s[i]));
                break;
            case S_JOIN: {
                const double in1 = est.entries[size_t(st.in1)];
                s[i] = s0 + s[size_t(st.in1)] - st.b_out;
                out = std::min(std::max(in0, in1), cap(st.b_out, s[i]));
                break;
            }
            case S_RESORT:
                s[i] = s0;
                out = in0;
                break;
        }
        est.entries[i] = out;
        est.total_entries += out * B;
    }
    // peak: tables live between their producer and last consumer, plus the
    // step's working buffers (count arrays and offsets ~ its output, a
    // radix sort's second buffers = its table, run starts ~ its input)
    std::vector<int> uses(S, 0);
    for (const Step& st : plan.steps) {
        if (st.in0 >= 0) uses[size_t(st.in0)]++;
        if (st.in1 >= 0) uses[size_t(st.in1)]++;
    }
    auto bytes = [&](size_t i) {
        const int b = plan.steps[i].b_out;
        const double bits = std::ceil(std::log2(double(std::max(B, 1)))) + b * std::ceil(std::log2(n)) + k;
        const double key = bits > 64 ? 16 : 8;
        return est.entries[i] * B * (key + 8);
    };
    // an introduce by pull over a one-column child followed by the forget of
    // that column runs as one gather: its own table is never stored
    std::vector<char> fused(S, 0);
    for (size_t i = 0; i + 1 < S; i++) {
        const Step& a = plan.steps[i];
        const Step& f = plan.steps[i + 1];
        if (a.kind == S_INTRO_PULL && a.b_in == 1 && a.nchk == 0 && f.kind == S_FORGET_LAST && f.in0 == int(i) &&
            uses[i] == 1)
            fused[i] = 1;
    }
    double live = 0, peak = 0;
    for (size_t i = 0; i < S; i++) {
        const Step& st = plan.steps[i];
        if (fused[i]) continue;  // no table; its forget reads the child directly
        const double out = bytes(i);
        double work = out;  // counts, offsets, survivor bits
        if (st.kind == S_RESORT) work = 2 * out;
        if (st.kind == S_FORGET_LAST || st.kind == S_JOIN) {
            int in = st.in0;
            if (in >= 0 && fused[size_t(in)]) in = plan.steps[size_t(in)].in0;  // the gather reads the child
            work = in >= 0 ? bytes(size_t(in)) : 0;
        }
        live += out;
        peak = std::max(peak, live + work);
        for (int in : {st.in0, st.in1}) {
            if (in < 0) continue;
            if (fused[size_t(in)]) {  // the fused introduce's child is this step's real input
                const int c = plan.steps[size_t(in)].in0;
                if (c >= 0 && --uses[size_t(c)] == 0) live -= bytes(size_t(c));
                continue;
            }
            if (--uses[size_t(in)] == 0) live -= bytes(size_t(in));
        }
    }
    // plans of one-vertex bags (trees) may run on dense tables instead:
    // n_G x B x C(k-1, s-1) slots of at most 9 bytes per table
    if (plan.max_bag <= 2) {
        std::vector<int> u2(S, 0);
        for (const Step& st : plan.steps) {
            if (st.in0 >= 0) u2[size_t(st.in0)]++;
            if (st.in1 >= 0) u2[size_t(st.in1)]++;
        }
        auto dense = [&](size_t i) {
            return plan.steps[i].b_out == 1 ? n * B * binom_d(k - 1, s[i] - 1) * 9.0 : 0.0;
        };
        double dl = 0, dp = 0;
        for (size_t i = 0; i < S; i++) {
            const Step& st = plan.steps[i];
            dl += dense(i);
            dp = std::max(dp, dl);
            for (int in : {st.in0, st.in1})
                if (in >= 0 && --u2[size_t(in)] == 0) dl -= dense(size_t(in));
        }
        peak = std::max(peak, dp);
    }
    // colourings and the per-(colouring, vertex) index arrays of pull steps
    est.peak_bytes = peak + double(B) * n * (1 + 16);
    return est;
}

}  // namespace ccg
