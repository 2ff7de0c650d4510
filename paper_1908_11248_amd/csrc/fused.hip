// Fused introduce + forget for one-column tables (tree edges of the pattern).
//
// With a child table keyed (colouring, image y of a, C) and pattern edge
// {u, a}, the plan's steps
//     introduce u (pull form: output keyed (b, v, y, C | {zeta(v)}))
//     forget a    (drop y, add equal (b, v, C))
// compose into one per-(b, v) gather: for every neighbour y of v, the run of
// child entries with image y whose colour set misses zeta(v) is added into a
// dense colour-set accumulator of (b, v).  The introduce table (the larger of
// the two) is never written.  When the child is a leaf (Sec. 3.1 leaf rule)
// its entries ({zeta(y)}, 1) are synthesised from the colouring instead of
// read.  Units are (b, v) in key order, so the output is sorted.
#include <hip/hip_runtime.h>

#include "device.h"
#include "kernels.h"

namespace ccg {

template <class KI, class KO, bool EMIT, bool LEAFCHILD>
__global__ void __launch_bounds__(64)
k_edge(const KI* __restrict__ keys, const uint64_t* __restrict__ cnt, Lay L, const uint64_t* __restrict__ rstart,
       const uint64_t* __restrict__ rend, int B, DevGraph g, const uint8_t* __restrict__ colors, int degF_u,
       int degF_child, uint32_t* gcount, uint32_t* icount, const uint64_t* __restrict__ goff, KO* okeys,
       uint64_t* ocnt, Lay LO, uint32_t* ovf) {
    Acc acc = acc_bind(LO.kb, EMIT);
    __shared__ uint64_t pre[65];
    __shared__ uint64_t r0s[64];
    __shared__ uint32_t ys[64];
    const uint64_t units = uint64_t(B) * uint64_t(g.n);
    const int lane = threadIdx.x;
    for (uint64_t w = blockIdx.x; w < units; w += gridDim.x) {
        const uint32_t bid = uint32_t(w / uint64_t(g.n));
        const uint32_t v = uint32_t(w % uint64_t(g.n));
        const int64_t rb = g.rp[v], re = g.rp[v + 1];
        if (re - rb < degF_u) {
            if (!EMIT && lane == 0) {
                gcount[w] = 0;
                icount[w] = 0;
            }
            continue;
        }
        const uint8_t* col_b = colors + uint64_t(bid) * g.n;
        const uint32_t cb = 1u << col_b[v];
        acc_clear(acc, EMIT);
        bool over = false;
        uint32_t passed = 0;
        for (int64_t nb0 = rb; nb0 < re; nb0 += 64) {
            __syncthreads();
            int64_t e = nb0 + lane;
            uint64_t len = 0, r0 = 0;
            uint32_t y = 0;
            if (e < re) {
                y = uint32_t(g.col[e]);
                if (LEAFCHILD) {
                    len = (g.rp[y + 1] - g.rp[y] >= degF_child) ? 1 : 0;
                } else {
                    uint64_t slot = uint64_t(bid) * uint64_t(g.n) + y;
                    r0 = rstart[slot];
                    len = rend[slot] - r0;
                }
            }
            uint64_t inc = wave_incl_scan(len);
            pre[lane] = inc - len;
            r0s[lane] = r0;
            ys[lane] = y;
            if (lane == 63) pre[64] = inc;
            __syncthreads();
            const uint64_t T = pre[64];
            for (uint64_t t = lane; t < T; t += 64) {
                // neighbour j with pre[j] <= t < pre[j + 1]
                int lo = 0, hi = 64;
                while (hi - lo > 1) {
                    int mid = (lo + hi) >> 1;
                    if (pre[mid] <= t) lo = mid;
                    else hi = mid;
                }
                uint32_t C;
                uint64_t c;
                if (LEAFCHILD) {
                    C = 1u << col_b[ys[lo]];
                    c = 1;
                } else {
                    uint64_t i = r0s[lo] + (t - pre[lo]);
                    C = kset(keys[i], L);
                    c = cnt[i];
                }
                if (C & cb) continue;
                C |= cb;
                passed++;
                atomicOr(&acc.bits[C >> 5], 1u << (C & 31));
                if (EMIT) {
                    uint64_t old = atomicAdd((unsigned long long*)&acc.val[C], (unsigned long long)c);
                    over |= (old + c < old);
                }
            }
        }
        __syncthreads();
        if (EMIT) {
            if (__ballot(over) && lane == 0) atomicOr(&ovf[bid], 1u);
            uint32_t cols[1] = {v};
            KO prefix = kpack<KO>(bid, cols, 1, 0u, LO);
            acc_emit<KO>(acc, prefix, goff[w], okeys, ocnt);
        } else {
            uint32_t c = acc_count(acc);
            uint32_t p = uint32_t(wave_sum(passed));
            if (lane == 0) {
                gcount[w] = c;
                icount[w] = p;
            }
        }
        __syncthreads();
    }
}

template <bool EMIT, bool LEAFCHILD>
static void edge_launch(const DevTable* in, const uint64_t* rstart, const uint64_t* rend, int B, DevGraph g,
                        const uint8_t* colors, int degF_u, int degF_child, uint32_t* gcount, uint32_t* icount,
                        const uint64_t* goff, DevTable* out, Lay LO, uint32_t* ovf, hipStream_t s) {
    uint64_t units = uint64_t(B) * uint64_t(g.n);
    if (!units) return;
    unsigned grid = unsigned(units < (1u << 20) ? units : (1u << 20));
    size_t lds = acc_bytes(LO.kb, EMIT);
    const void* ik = in ? in->keys : nullptr;
    const uint64_t* ic = in ? in->cnt : nullptr;
    Lay LI = in ? in->lay : LO;
    void* ok = out ? out->keys : nullptr;
    uint64_t* oc = out ? out->cnt : nullptr;
    int ki = LI.kw(), ko = LO.kw();
    if (ki == 1 && ko == 1)
        k_edge<uint64_t, uint64_t, EMIT, LEAFCHILD><<<grid, 64, lds, s>>>(
            (const uint64_t*)ik, ic, LI, rstart, rend, B, g, colors, degF_u, degF_child, gcount, icount, goff,
            (uint64_t*)ok, oc, LO, ovf);
    else if (ki == 1)
        k_edge<uint64_t, u128, EMIT, LEAFCHILD><<<grid, 64, lds, s>>>(
            (const uint64_t*)ik, ic, LI, rstart, rend, B, g, colors, degF_u, degF_child, gcount, icount, goff,
            (u128*)ok, oc, LO, ovf);
    else if (ko == 1)
        k_edge<u128, uint64_t, EMIT, LEAFCHILD><<<grid, 64, lds, s>>>(
            (const u128*)ik, ic, LI, rstart, rend, B, g, colors, degF_u, degF_child, gcount, icount, goff,
            (uint64_t*)ok, oc, LO, ovf);
    else
        k_edge<u128, u128, EMIT, LEAFCHILD><<<grid, 64, lds, s>>>((const u128*)ik, ic, LI, rstart, rend, B, g, colors,
                                                                  degF_u, degF_child, gcount, icount, goff, (u128*)ok,
                                                                  oc, LO, ovf);
}

void launch_edge_count(const DevTable* in, const uint64_t* rstart, const uint64_t* rend, int B, DevGraph g,
                       const uint8_t* colors, int degF_u, int degF_child, Lay LO, uint32_t* gcount, uint32_t* icount,
                       hipStream_t s) {
    if (in)
        edge_launch<false, false>(in, rstart, rend, B, g, colors, degF_u, degF_child, gcount, icount, nullptr, nullptr,
                                  LO, nullptr, s);
    else
        edge_launch<false, true>(nullptr, nullptr, nullptr, B, g, colors, degF_u, degF_child, gcount, icount, nullptr,
                                 nullptr, LO, nullptr, s);
}

void launch_edge_emit(const DevTable* in, const uint64_t* rstart, const uint64_t* rend, int B, DevGraph g,
                      const uint8_t* colors, int degF_u, int degF_child, const uint64_t* goff, DevTable& out,
                      uint32_t* ovf, hipStream_t s) {
    if (in)
        edge_launch<true, false>(in, rstart, rend, B, g, colors, degF_u, degF_child, nullptr, nullptr, goff, &out,
                                 out.lay, ovf, s);
    else
        edge_launch<true, true>(nullptr, nullptr, nullptr, B, g, colors, degF_u, degF_child, nullptr, nullptr, goff,
                                &out, out.lay, ovf, s);
}

}  // namespace ccg
