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
// read, and counted per neighbour colour (the outputs are {zeta(v), c}).
// Units are (b, v) in key order, so the output is sorted.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "device.h"
#include "kernels.h"

namespace ccg {

// U units per 64-lane workgroup, 64 / U lanes each: the dependent loads of
// U units are in flight together.  Loop trip counts are made uniform across
// the wave (maxima over the U units), so the workgroup barriers stay legal.
template <class KI, class KO, bool EMIT, bool LEAFCHILD, int U>
__global__ void __launch_bounds__(64)
k_edge(const KI* __restrict__ keys, const uint64_t* __restrict__ cnt, Lay L, const uint64_t* __restrict__ rstart,
       const uint64_t* __restrict__ rend, int B, DevGraph g, const uint8_t* __restrict__ colors, int degF_u,
       int degF_child, uint32_t* gcount, uint32_t* icount, const uint64_t* __restrict__ goff, KO* okeys,
       uint64_t* ocnt, Lay LO, uint32_t* ovf, bool heavy_only, int skip_above) {
    // heavy_only: the units are (b, heavy vertex); otherwise (b, v) for all v,
    // skipping (no writes at all) vertices of degree > skip_above when > 0
    constexpr int LN = 64 / U;  // lanes per unit
    extern __shared__ uint64_t smem[];
    const int slots = 1 << LO.kb;
    const int words = LO.kb >= 5 ? (1 << (LO.kb - 5)) : 1;
    const int lane = threadIdx.x, sub = lane / LN, sl = lane % LN;
    uint64_t* val = EMIT ? smem + size_t(sub) * slots : nullptr;
    uint32_t* bits = reinterpret_cast<uint32_t*>(smem + (EMIT ? size_t(U) * slots : 0)) + sub * words;
    __shared__ uint64_t pre[U][LN + 1];
    __shared__ uint64_t r0s[U][LN];
    __shared__ uint32_t ys[U][LN];
    const uint64_t nv = heavy_only ? uint64_t(g.nheavy) : uint64_t(g.n);
    const uint64_t units = uint64_t(B) * nv;
    const uint64_t subgroup_mask = (LN == 64) ? ~0ull : ((1ull << LN) - 1ull);
    for (uint64_t w0 = uint64_t(blockIdx.x) * U; w0 < units; w0 += uint64_t(gridDim.x) * U) {
        bool mine = w0 + sub < units;  // this launch owns the unit (writes its results)
        bool active = mine;
        uint32_t bid = 0, v = 0, cb = 0;
        int64_t rb = 0, re = 0;
        if (active) {
            bid = uint32_t((w0 + sub) / nv);
            uint64_t j = (w0 + sub) % nv;
            v = heavy_only ? uint32_t(g.heavy[j]) : uint32_t(j);
            rb = g.rp[v];
            re = g.rp[v + 1];
            if (skip_above > 0 && re - rb > skip_above) mine = active = false;
            if (re - rb < degF_u || int32_t(v) < g.vlo || int32_t(v) >= g.vhi) active = false;
        }
        const uint64_t w = uint64_t(bid) * uint64_t(g.n) + v;  // the unit's output slot
        if (!active) re = rb;
        const uint8_t* col_b = colors + uint64_t(bid) * g.n;
        if (active) cb = 1u << col_b[v];
        if constexpr (LEAFCHILD) {
            // The leaf's entries are ({zeta(y)}, 1), so the output sets are
            // {zeta(v), c}: a count per neighbour colour c replaces the 2^k
            // accumulator, and increasing c is increasing set order.
            uint32_t* hc = reinterpret_cast<uint32_t*>(smem) + sub * 32;
            for (int i = sl; i < 32; i += LN) hc[i] = 0;
            __syncthreads();
            uint32_t passed = 0;
            for (int64_t e = rb + sl; e < re; e += LN) {
                const uint32_t y = uint32_t(g.col[e]);
                const uint32_t cy = col_b[y];
                if (g.rp[y + 1] - g.rp[y] >= degF_child && !((1u << cy) & cb)) {
                    atomicAdd(&hc[cy], 1u);
                    passed++;
                }
            }
            __syncthreads();
            // lane sl takes colour sl (LN >= k); hc[zeta(v)] stays 0
            const uint32_t h = active && sl < LO.kb ? hc[sl] : 0u;
            const uint64_t m = (__ballot(h != 0) >> (sub * LN)) & subgroup_mask;
            if (EMIT) {
                if (h) {
                    uint32_t colv[1] = {v};
                    const KO prefix = kpack<KO>(bid, colv, 1, 0u, LO);
                    const uint64_t o = goff[w] + uint64_t(__popcll(m & ((1ull << sl) - 1ull)));
                    okeys[o] = prefix | KO(cb | (1u << sl));
                    ocnt[o] = h;
                }
            } else {
                uint64_t p = passed;
                for (int d = LN / 2; d >= 1; d >>= 1) p += __shfl_xor(p, d, LN);
                if (mine && sl == 0) {
                    gcount[w] = active ? uint32_t(__popcll(m)) : 0u;
                    icount[w] = active ? uint32_t(p) : 0u;
                }
            }
            __syncthreads();
            continue;
        }
        for (int i = sl; i < slots && EMIT; i += LN) val[i] = 0;
        for (int i = sl; i < words; i += LN) bits[i] = 0;
        bool over = false;
        uint32_t passed = 0;
        // neighbour chunks of LN: the wave runs the largest count over its units
        int64_t nch = (re - rb + LN - 1) / LN;
        for (int d = 32; d >= 1; d >>= 1) nch = max(nch, (int64_t)__shfl_xor(nch, d, 64));
        for (int64_t c = 0; c < nch; c++) {
            __syncthreads();
            int64_t e = rb + c * LN + sl;
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
            uint64_t inc = len;
            for (int d = 1; d < LN; d <<= 1) {
                uint64_t t = __shfl_up(inc, d, LN);
                if (sl >= d) inc += t;
            }
            pre[sub][sl] = inc - len;
            r0s[sub][sl] = r0;
            ys[sub][sl] = y;
            if (sl == LN - 1) pre[sub][LN] = inc;
            __syncthreads();
            const uint64_t T = pre[sub][LN];
            uint64_t Tmax = T;
            for (int d = 32; d >= 1; d >>= 1) Tmax = max(Tmax, (uint64_t)__shfl_xor(Tmax, d, 64));
            // NB items per lane and round: their searches and loads are all
            // issued before the first accumulator update, so one round costs
            // about one memory latency instead of NB
            constexpr int NB = 4;
            for (uint64_t t0 = 0; t0 < Tmax; t0 += NB * LN) {
                uint32_t Cs[NB];
                uint64_t cvs[NB];
                uint32_t okm = 0;
#pragma unroll
                for (int j = 0; j < NB; j++) {
                    const uint64_t t = t0 + uint64_t(j * LN + sl);
                    const bool ok = t < T;
                    okm |= uint32_t(ok) << j;
                    int lo = 0, hi = LN;
                    while (hi - lo > 1) {
                        int mid = (lo + hi) >> 1;
                        if (pre[sub][mid] <= t) lo = mid;
                        else hi = mid;
                    }
                    if (LEAFCHILD) {
                        Cs[j] = 1u << col_b[ys[sub][lo]];
                        cvs[j] = 1;
                    } else {
                        // rows outside this unit's items read entry 0 (the table is
                        // not empty whenever some unit of the wave has items)
                        const uint64_t i = ok ? r0s[sub][lo] + (t - pre[sub][lo]) : 0;
                        const uint32_t C = kset(keys[i], L);
                        Cs[j] = C;
                        cvs[j] = EMIT ? cnt[i] : 0;
                    }
                }
#pragma unroll
                for (int j = 0; j < NB; j++) {
                    uint32_t C = Cs[j];
                    if (!((okm >> j) & 1u) || (C & cb)) continue;
                    C |= cb;
                    passed++;
                    atomicOr(&bits[C >> 5], 1u << (C & 31));
                    if (EMIT) {
                        const uint64_t cv = cvs[j];
                        uint64_t old = atomicAdd((unsigned long long*)&val[C], (unsigned long long)cv);
                        over |= (old + cv < old);
                    }
                }
            }
        }
        __syncthreads();
        if (EMIT) {
            uint64_t ob = __ballot(over);
            if (((ob >> (sub * LN)) & subgroup_mask) && sl == 0) atomicOr(&ovf[bid], 1u);
            uint32_t colv[1] = {v};
            KO prefix = kpack<KO>(bid, colv, 1, 0u, LO);
            uint64_t run = active ? goff[w] : 0;
            for (int c0 = 0; c0 < slots; c0 += LN) {
                int C = c0 + sl;
                bool present = active && C < slots && ((bits[C >> 5] >> (C & 31)) & 1u);
                uint64_t m = (__ballot(present) >> (sub * LN)) & subgroup_mask;
                if (present) {
                    uint64_t o = run + __popcll(m & ((1ull << sl) - 1ull));
                    okeys[o] = prefix | KO(C);
                    ocnt[o] = val[C];
                }
                run += __popcll(m);
            }
        } else {
            uint64_t c = 0;
            for (int i = sl; i < words; i += LN) c += __popc(bits[i]);
            uint64_t p = passed;
            for (int d = LN / 2; d >= 1; d >>= 1) {
                c += __shfl_xor(c, d, LN);
                p += __shfl_xor(p, d, LN);
            }
            if (mine && sl == 0) {
                gcount[w] = active ? uint32_t(c) : 0u;
                icount[w] = active ? uint32_t(p) : 0u;
            }
        }
        __syncthreads();
    }
}

template <bool EMIT, bool LEAFCHILD, int U>
static void edge_launch_u(const DevTable* in, const uint64_t* rstart, const uint64_t* rend, int B, DevGraph g,
                          const uint8_t* colors, int degF_u, int degF_child, uint32_t* gcount, uint32_t* icount,
                          const uint64_t* goff, DevTable* out, Lay LO, uint32_t* ovf, bool heavy_only, int skip_above,
                          hipStream_t s) {
    uint64_t units = uint64_t(B) * uint64_t(heavy_only ? g.nheavy : g.n);
    if (!units) return;
    uint64_t blocks = (units + U - 1) / U;
    unsigned grid = unsigned(blocks < (1u << 20) ? blocks : (1u << 20));
    size_t words = LO.kb >= 5 ? (size_t(1) << (LO.kb - 5)) : 1;
    // a leaf child needs 32 colour counters per unit, else the 2^k accumulator
    size_t lds = LEAFCHILD ? size_t(U) * 32 * 4 : (EMIT ? size_t(U) * (size_t(8) << LO.kb) : 0) + size_t(U) * 4 * words;
    const void* ik = in ? in->keys : nullptr;
    const uint64_t* ic = in ? in->cnt : nullptr;
    Lay LI = in ? in->lay : LO;
    void* ok = out ? out->keys : nullptr;
    uint64_t* oc = out ? out->cnt : nullptr;
    int ki = LI.kw(), ko = LO.kw();
    if (ki == 1 && ko == 1)
        k_edge<uint64_t, uint64_t, EMIT, LEAFCHILD, U><<<grid, 64, lds, s>>>(
            (const uint64_t*)ik, ic, LI, rstart, rend, B, g, colors, degF_u, degF_child, gcount, icount, goff,
            (uint64_t*)ok, oc, LO, ovf, heavy_only, skip_above);
    else if (ki == 1)
        k_edge<uint64_t, u128, EMIT, LEAFCHILD, U><<<grid, 64, lds, s>>>(
            (const uint64_t*)ik, ic, LI, rstart, rend, B, g, colors, degF_u, degF_child, gcount, icount, goff,
            (u128*)ok, oc, LO, ovf, heavy_only, skip_above);
    else if (ko == 1)
        k_edge<u128, uint64_t, EMIT, LEAFCHILD, U><<<grid, 64, lds, s>>>(
            (const u128*)ik, ic, LI, rstart, rend, B, g, colors, degF_u, degF_child, gcount, icount, goff,
            (uint64_t*)ok, oc, LO, ovf, heavy_only, skip_above);
    else
        k_edge<u128, u128, EMIT, LEAFCHILD, U><<<grid, 64, lds, s>>>((const u128*)ik, ic, LI, rstart, rend, B, g, colors,
                                                                     degF_u, degF_child, gcount, icount, goff,
                                                                     (u128*)ok, oc, LO, ovf, heavy_only, skip_above);
}

// Units per workgroup: as many as the LDS accumulators allow.  Vertices of
// degree > kHeavyDegree would stall the other units of their workgroup; they
// run in a second launch with one unit per workgroup.
static int edge_units(int kb) { return kb <= 9 ? 4 : (kb <= 11 ? 2 : 1); }

template <bool EMIT, bool LEAFCHILD>
static void edge_launch(const DevTable* in, const uint64_t* rstart, const uint64_t* rend, int B, DevGraph g,
                        const uint8_t* colors, int degF_u, int degF_child, uint32_t* gcount, uint32_t* icount,
                        const uint64_t* goff, DevTable* out, Lay LO, uint32_t* ovf, hipStream_t s) {
    if (!(uint64_t(B) * uint64_t(g.n))) return;
    int u = edge_units(LO.kb);
    int skip = (u > 1 && g.nheavy > 0) ? kHeavyDegree : 0;
    switch (u) {
        case 4:
            edge_launch_u<EMIT, LEAFCHILD, 4>(in, rstart, rend, B, g, colors, degF_u, degF_child, gcount, icount, goff,
                                              out, LO, ovf, false, skip, s);
            break;
        case 2:
            edge_launch_u<EMIT, LEAFCHILD, 2>(in, rstart, rend, B, g, colors, degF_u, degF_child, gcount, icount, goff,
                                              out, LO, ovf, false, skip, s);
            break;
        default:
            edge_launch_u<EMIT, LEAFCHILD, 1>(in, rstart, rend, B, g, colors, degF_u, degF_child, gcount, icount, goff,
                                              out, LO, ovf, false, 0, s);
    }
    if (skip)
        edge_launch_u<EMIT, LEAFCHILD, 1>(in, rstart, rend, B, g, colors, degF_u, degF_child, gcount, icount, goff, out,
                                          LO, ovf, true, 0, s);
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


// Introduce u in pull form over a leaf (Sec. 3.1 leaf and introduce rules;
// degree masks of Sec. 3.2).  The leaf's table holds ((b, y), {zeta(y)}, 1)
// for every y passing its mask, so the introduce's entries are the adjacent
// pairs (v, y) with v passing u's mask and range, y the leaf's mask, and
// zeta(v) != zeta(y): key (b, v, y, {zeta(v), zeta(y)}), count 1.  Neither
// table is read: the items are the (colouring, directed edge) pairs, in
// colouring-major CSR order, which is key order, so the output is sorted.
// A tile is kLeafPullItems rounds of kBlock consecutive edges of one
// colouring; the count pass stores a tile's survivors, the emit pass ranks
// each round's survivors across the block (a ballot per wave), so a round's
// outputs are one contiguous run.
constexpr int kLeafPullItems = 16;
constexpr uint64_t kLeafPullTile = uint64_t(kBlock) * kLeafPullItems;

uint64_t leaf_pull_tiles(const DevGraph& g, int B) {
    return uint64_t(B) * ((uint64_t(g.m2) + kLeafPullTile - 1) / kLeafPullTile);
}

template <class KO, bool EMIT>
__global__ void __launch_bounds__(kBlock)
k_leaf_pull(DevGraph g, int B, int degF_u, int degF_leaf, const uint8_t* __restrict__ colors, uint64_t tpb,
            uint32_t* tcount, const uint64_t* __restrict__ toff, Lay LO, KO* okeys, uint64_t* ocnt) {
    __shared__ uint32_t s_w[kBlock / 64];
    const uint64_t tiles = tpb * uint64_t(B), m2 = uint64_t(g.m2);
    const uint32_t wv = threadIdx.x >> 6, ln = threadIdx.x & 63u;
    for (uint64_t tile = blockIdx.x; tile < tiles; tile += gridDim.x) {
        const uint32_t b = uint32_t(tile / tpb);
        const uint64_t e0 = (tile - uint64_t(b) * tpb) * kLeafPullTile;
        const uint8_t* cb = colors + uint64_t(b) * uint32_t(g.n);
        uint64_t o = EMIT ? toff[tile] : 0;
        uint32_t mine = 0;
        for (int j = 0; j < kLeafPullItems; j++) {
            const uint64_t e = e0 + uint64_t(j) * kBlock + threadIdx.x;
            bool ok = false;
            uint32_t v = 0, y = 0, cv = 0, cy = 0;
            if (e < m2) {
                v = uint32_t(g.esrc[e]);
                y = uint32_t(g.col[e]);
                cv = cb[v];
                cy = cb[y];
                ok = cv != cy && intro_ok(g, v, degF_u) && int(g.deg8[y]) >= degF_leaf;
            }
            if (!EMIT) {
                mine += ok;
                continue;
            }
            const uint64_t bal = __ballot(ok);
            if (ln == 0) s_w[wv] = uint32_t(__popcll(bal));
            __syncthreads();
            uint32_t before = 0, round = 0;
#pragma unroll
            for (int w = 0; w < kBlock / 64; w++) {
                const uint32_t c = s_w[w];
                before += w < int(wv) ? c : 0u;
                round += c;
            }
            __syncthreads();
            if (ok) {
                const uint64_t p = o + before + uint32_t(__popcll(bal & ((1ull << ln) - 1ull)));
                const uint32_t cols[2] = {v, y};
                okeys[p] = kpack<KO>(b, cols, 2, (1u << cv) | (1u << cy), LO);
                ocnt[p] = 1;
            }
            o += round;
        }
        if (!EMIT) {
            const uint32_t w = uint32_t(wave_sum(mine));
            if (ln == 0) s_w[wv] = w;
            __syncthreads();
            if (threadIdx.x == 0) {
                uint32_t t = 0;
                for (int i = 0; i < kBlock / 64; i++) t += s_w[i];
                tcount[tile] = t;
            }
            __syncthreads();
        }
    }
}

template <bool EMIT>
static void leaf_pull_launch(DevGraph g, int B, int degF_u, int degF_leaf, const uint8_t* colors, uint32_t* tcount,
                             const uint64_t* toff, Lay LO, void* okeys, uint64_t* ocnt, hipStream_t s) {
    const uint64_t tiles = leaf_pull_tiles(g, B);
    if (!tiles) return;
    const uint64_t tpb = tiles / uint64_t(B);
    const unsigned grid = unsigned(std::min<uint64_t>(tiles, 1u << 16));
    if (LO.kw() == 1)
        k_leaf_pull<uint64_t, EMIT><<<grid, kBlock, 0, s>>>(g, B, degF_u, degF_leaf, colors, tpb, tcount, toff, LO,
                                                            (uint64_t*)okeys, ocnt);
    else
        k_leaf_pull<u128, EMIT><<<grid, kBlock, 0, s>>>(g, B, degF_u, degF_leaf, colors, tpb, tcount, toff, LO,
                                                        (u128*)okeys, ocnt);
}

void launch_leaf_pull_count(DevGraph g, int B, int degF_u, int degF_leaf, const uint8_t* colors, Lay LO,
                            uint32_t* tcount, hipStream_t s) {
    leaf_pull_launch<false>(g, B, degF_u, degF_leaf, colors, tcount, nullptr, LO, nullptr, nullptr, s);
}

void launch_leaf_pull_emit(DevGraph g, int B, int degF_u, int degF_leaf, const uint8_t* colors,
                           const uint64_t* toff, DevTable& out, hipStream_t s) {
    leaf_pull_launch<true>(g, B, degF_u, degF_leaf, colors, nullptr, toff, out.lay, out.keys, out.cnt, s);
}

// The introduce that follows such a pull, when its new vertex is adjacent in
// F to both of the pull's vertices, whose images are adjacent in G: its
// candidates are the common neighbours of that edge (Sec. 3.2), so its
// entries are the triangles (v, a, c) of G, a edge (v, a) in CSR order and c
// from the edge's common-neighbour list (ascending), with three distinct
// colours and each vertex passing its column's degree mask (m0, m1, m2), each
// of count 1.  Items are the positions of the lists, colouring-major, in key
// order, so the output is sorted; neither the pull's table nor the
// introduce's candidates are materialised.  A thread takes kTriItems
// consecutive items (one search for its first edge, then it walks on).
constexpr int kTriItems = 16;
constexpr uint64_t kTriTile = uint64_t(kBlock) * kTriItems;

uint64_t tri_tiles(uint64_t total, int B) { return uint64_t(B) * ((total + kTriTile - 1) / kTriTile); }

template <class KO, bool EMIT>
__global__ void __launch_bounds__(kBlock)
k_tri(DevGraph g, const uint64_t* __restrict__ cn_off, const int32_t* __restrict__ cn_col, uint64_t total, int B,
      int m0, int m1, int m2, const uint8_t* __restrict__ colors, uint64_t tpb, uint32_t* tcount,
      const uint64_t* __restrict__ toff, Lay LO, KO* okeys, uint64_t* ocnt) {
    const uint64_t tiles = tpb * uint64_t(B), E = uint64_t(g.m2);
    for (uint64_t tile = blockIdx.x; tile < tiles; tile += gridDim.x) {
        const uint32_t b = uint32_t(tile / tpb);
        const uint64_t t0 = (tile - uint64_t(b) * tpb) * kTriTile + uint64_t(threadIdx.x) * kTriItems;
        const uint64_t t1 = t0 + kTriItems < total ? t0 + kTriItems : total;
        const uint8_t* cb = colors + uint64_t(b) * uint32_t(g.n);
        // the edge of item t0: cn_off[e] <= t0 < cn_off[e + 1]
        uint64_t e = t0 < t1 ? upper_bound_u64(cn_off, 0, E + 1, t0) - 1 : 0;
        uint32_t pass = 0, n_pass = 0;
        for (uint64_t t = t0; t < t1; t++) {
            while (cn_off[e + 1] <= t) e++;
            const uint32_t v = uint32_t(g.esrc[e]), a = uint32_t(g.col[e]), c = uint32_t(cn_col[t]);
            const uint32_t cv = cb[v], ca = cb[a], cc = cb[c];
            const bool ok = cv != ca && cv != cc && ca != cc && int(g.deg8[v]) >= m0 && int(g.deg8[a]) >= m1 &&
                            int(g.deg8[c]) >= m2;
            pass |= uint32_t(ok) << (t - t0);
            n_pass += ok;
        }
        uint64_t sum;
        const uint64_t my = block_excl_scan(n_pass, &sum);
        if (!EMIT) {
            if (threadIdx.x == 0) tcount[tile] = uint32_t(sum);
            continue;
        }
        uint64_t o = toff[tile] + my;
        e = t0 < t1 ? upper_bound_u64(cn_off, 0, E + 1, t0) - 1 : 0;
        for (uint64_t t = t0; t < t1 && pass; t++) {
            while (cn_off[e + 1] <= t) e++;
            if (!((pass >> (t - t0)) & 1u)) continue;
            const uint32_t cols[3] = {uint32_t(g.esrc[e]), uint32_t(g.col[e]), uint32_t(cn_col[t])};
            okeys[o] = kpack<KO>(b, cols, 3, (1u << cb[cols[0]]) | (1u << cb[cols[1]]) | (1u << cb[cols[2]]), LO);
            ocnt[o] = 1;
            o++;
        }
    }
}

template <bool EMIT>
static void tri_launch(DevGraph g, const uint64_t* cn_off, const int32_t* cn_col, uint64_t total, int B, int m0,
                       int m1, int m2, const uint8_t* colors, uint32_t* tcount, const uint64_t* toff, Lay LO,
                       void* okeys, uint64_t* ocnt, hipStream_t s) {
    const uint64_t tiles = tri_tiles(total, B);
    if (!tiles) return;
    const uint64_t tpb = tiles / uint64_t(B);
    const unsigned grid = unsigned(std::min<uint64_t>(tiles, 1u << 16));
    if (LO.kw() == 1)
        k_tri<uint64_t, EMIT><<<grid, kBlock, 0, s>>>(g, cn_off, cn_col, total, B, m0, m1, m2, colors, tpb, tcount,
                                                      toff, LO, (uint64_t*)okeys, ocnt);
    else
        k_tri<u128, EMIT><<<grid, kBlock, 0, s>>>(g, cn_off, cn_col, total, B, m0, m1, m2, colors, tpb, tcount, toff,
                                                  LO, (u128*)okeys, ocnt);
}

void launch_tri_count(DevGraph g, const uint64_t* cn_off, const int32_t* cn_col, uint64_t total, int B, int m0,
                      int m1, int m2, const uint8_t* colors, Lay LO, uint32_t* tcount, hipStream_t s) {
    tri_launch<false>(g, cn_off, cn_col, total, B, m0, m1, m2, colors, tcount, nullptr, LO, nullptr, nullptr, s);
}

void launch_tri_emit(DevGraph g, const uint64_t* cn_off, const int32_t* cn_col, uint64_t total, int B, int m0,
                     int m1, int m2, const uint8_t* colors, const uint64_t* toff, DevTable& out, hipStream_t s) {
    tri_launch<true>(g, cn_off, cn_col, total, B, m0, m1, m2, colors, nullptr, toff, out.lay, out.keys, out.cnt, s);
}

}  // namespace ccg
