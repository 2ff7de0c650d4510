// Dense one-column tables ("slot tables") for patterns whose decomposition
// only ever holds one bag vertex per table: trees, after the introduce of a
// parent is fused with the forget of its child (Sec. 3, introduce and forget
// nodes) and joins happen on a one-vertex bag (Sec. 3, join nodes).
//
// A table at node x keeps, for colouring b and bag image v, every colour set
// C of size s = |V_x| that contains colour(v).  C minus colour(v), squeezed to
// k - 1 bits, has s - 1 bits; its rank among the masks of that popcount in
// increasing numeric order is the slot.  Slot order is therefore key order,
// and a table is two dense arrays over (b, v, slot): the count (mod 2^64) and
// a presence byte (the entry exists in the paper's sense iff some partial
// embedding reaches it; a count can wrap to 0 while the entry exists).
//
// Every kernel is output-stationary: one thread per output slot gathers what
// flows into it, so no accumulator, count pass, scan or sort is needed and
// every output is written exactly once, in order.  A block covers a run of
// consecutive vertices of one colouring; what its threads share (the
// neighbour lists and colours, the children's rows of a join, the rank table)
// is staged in LDS once per block.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <stdexcept>
#include <type_traits>

#include "device.h"
#include "kernels.h"

namespace ccg {

namespace {

constexpr int kEdgeChunk = 2048;  // neighbours staged per round
constexpr int kPushChunk = 1024;  // neighbour entries staged per round by the push form

__host__ __device__ __forceinline__ uint32_t bit_open(uint32_t m, uint32_t c) {  // insert a 0 at bit c
    return ((m >> c) << (c + 1)) | (m & ((1u << c) - 1u));
}
__host__ __device__ __forceinline__ uint32_t bit_close(uint32_t m, uint32_t c) {  // delete bit c
    return ((m >> (c + 1)) << c) | (m & ((1u << c) - 1u));
}

__device__ __forceinline__ uint32_t block_index() { return blockIdx.y * gridDim.x + blockIdx.x; }

// block -> (colouring, vertices [v0, v1), place j within the colouring).
// With xcd set, consecutive blocks (which the dispatcher deals round-robin to
// the eight XCDs) take eight different colourings, so each XCD's L2 holds
// the rows of the colouring it works on.  An empty range marks a block past
// the end.
__device__ __forceinline__ void block_range_at(const SlotGrid& G, uint32_t L, uint32_t* b, uint32_t* v0,
                                               uint32_t* v1, uint32_t* jb) {
    *b = 0;
    *v0 = *v1 = 0;
    *jb = 0;
    if (L >= G.blocks) return;
    uint32_t bb, j;
    if (G.xcd) {
        const uint32_t q = L >> 3;
        bb = (L & 7u) + 8u * (q / G.nbx);
        j = q % G.nbx;
    } else {
        bb = L / G.nbx;
        j = L % G.nbx;
    }
    if (bb >= uint32_t(G.B)) return;
    *b = bb;
    *jb = j;
    if (G.upb > 0) {
        *v0 = j * uint32_t(G.upb * G.m);
        *v1 = min(*v0 + uint32_t(G.upb * G.m), uint32_t(G.n));
    } else {
        *v0 = j / uint32_t(G.bpu);
        *v1 = *v0 + 1;
    }
}

__device__ __forceinline__ void block_range(const SlotGrid& G, uint32_t* b, uint32_t* v0, uint32_t* v1,
                                            uint32_t* jb) {
    block_range_at(G, block_index(), b, v0, v1, jb);
}

// this thread's slot r and first vertex; its i-th vertex is v + i * upb
__device__ __forceinline__ void slot_of(const SlotGrid& G, uint32_t v0, uint32_t jb, uint32_t* v, uint32_t* r,
                                        bool* lane_ok) {
    if (G.upb > 0) {
        const uint32_t u = threadIdx.x / uint32_t(G.R);
        *v = v0 + u;
        *r = threadIdx.x - u * uint32_t(G.R);
        *lane_ok = u < uint32_t(G.upb);
    } else {
        *v = v0;
        *r = (jb % uint32_t(G.bpu)) * kSlotBlock + threadIdx.x;
        *lane_ok = *r < uint32_t(G.R);
    }
}

// Entry counts of a block: (extra, present) summed over its threads and
// stored at part[2L], part[2L + 1] (L = block index); k_slot_sum adds them
// up.  Plain stores: no address is shared between blocks.  Ends with a
// barrier, so the next call may reuse the per-wave slots.
__device__ __forceinline__ void count_entries_at(uint32_t present, uint64_t extra, uint64_t* part, uint64_t blocks,
                                                 uint32_t L) {
    __shared__ uint64_t s_p[2][kSlotBlock / 64];
    const uint64_t pr = wave_sum(present);
    const uint64_t ex = wave_sum(extra);
    if (__lane_id() == 0) {
        s_p[0][threadIdx.x >> 6] = ex;
        s_p[1][threadIdx.x >> 6] = pr;
    }
    __syncthreads();
    if (threadIdx.x < 2 && L < blocks) {
        uint64_t t = 0;
        for (int i = 0; i < kSlotBlock / 64; i++) t += s_p[threadIdx.x][i];
        part[2 * uint64_t(L) + threadIdx.x] = t;
    }
    __syncthreads();
}

// count_entries for N tables at once (one barrier pair): part[j] gets
// (extra[j], present[j]).
template <int N>
__device__ __forceinline__ void count_entries_n(const uint32_t (&present)[N], const uint64_t (&extra)[N],
                                                uint64_t* const (&part)[N], uint64_t blocks) {
    __shared__ uint64_t s_q[2 * N][kSlotBlock / 64];
    const uint32_t L = block_index();
#pragma unroll
    for (int j = 0; j < N; j++) {
        const uint64_t ex = wave_sum(extra[j]);
        const uint64_t pr = wave_sum(present[j]);
        if (__lane_id() == 0) {
            s_q[2 * j][threadIdx.x >> 6] = ex;
            s_q[2 * j + 1][threadIdx.x >> 6] = pr;
        }
    }
    __syncthreads();
    if (threadIdx.x < 2 * N && L < blocks) {
        uint64_t t = 0;
        for (int i = 0; i < kSlotBlock / 64; i++) t += s_q[threadIdx.x][i];
        part[threadIdx.x / 2][2 * uint64_t(L) + (threadIdx.x & 1)] = t;
    }
    __syncthreads();
}

__device__ __forceinline__ void count_entries(uint32_t present, uint64_t extra, uint64_t* part, uint64_t blocks) {
    count_entries_at(present, extra, part, blocks, block_index());
}

// (sum, wrapped) over a block, sums mod 2^64: every lane of a butterfly sums
// all 64 values, and a total of 2^64 or more wraps in every lane's tree
__device__ __forceinline__ void block_sum_wrap(uint64_t* sum, bool* over) {
    __shared__ uint64_t s_s[kSlotBlock / 64];
    __shared__ uint32_t s_o[kSlotBlock / 64];
    uint64_t v = *sum;
    bool o = *over;
    for (int d = 32; d >= 1; d >>= 1) {
        const uint64_t x = __shfl_xor(v, d, 64);
        const uint64_t t = v + x;
        o |= t < v;
        v = t;
    }
    const bool wo = __ballot(o) != 0;
    if (__lane_id() == 0) {
        s_s[threadIdx.x >> 6] = v;
        s_o[threadIdx.x >> 6] = wo;
    }
    __syncthreads();
    v = 0;
    o = false;
    for (int i = 0; i < int(blockDim.x >> 6); i++) {
        const uint64_t t = v + s_s[i];
        o |= (t < v) || s_o[i];
        v = t;
    }
    *sum = v;
    *over = o;
}

__device__ __forceinline__ void stage_rank(uint16_t* s_rank, const uint16_t* __restrict__ rank, int k) {
    for (int i = threadIdx.x; i < (1 << (k - 1)); i += kSlotBlock) s_rank[i] = rank[i];
}

// dst[i] = src[i] for i < n by the block, four loads per thread in flight
template <class T>
__device__ __forceinline__ void stage_copy(T* dst, const T* __restrict__ src, uint32_t n, T* ored = nullptr) {
    T acc = 0;
    for (uint32_t i0 = 0; i0 < n; i0 += 4 * kSlotBlock) {
        T v[4];
#pragma unroll
        for (int j = 0; j < 4; j++) {
            const uint32_t i = i0 + j * kSlotBlock + threadIdx.x;
            v[j] = i < n ? src[i] : T(0);
        }
#pragma unroll
        for (int j = 0; j < 4; j++) {
            const uint32_t i = i0 + j * kSlotBlock + threadIdx.x;
            if (i < n) dst[i] = v[j];
            acc |= v[j];
        }
    }
    if (ored) *ored |= acc;  // the OR of this thread's values
}

// the two copies of stage_copy by the block at once: eight loads per
// thread in flight, four from each source
template <class T>
__device__ __forceinline__ void stage_copy2(T* d0, const T* __restrict__ s0, uint32_t n0, T* d1,
                                            const T* __restrict__ s1, uint32_t n1) {
    for (uint32_t i0 = 0; i0 < max(n0, n1); i0 += 4 * kSlotBlock) {
        T v0[4], v1[4];
#pragma unroll
        for (int j = 0; j < 4; j++) {
            const uint32_t i = i0 + j * kSlotBlock + threadIdx.x;
            v0[j] = i < n0 ? s0[i] : T(0);
            v1[j] = i < n1 ? s1[i] : T(0);
        }
#pragma unroll
        for (int j = 0; j < 4; j++) {
            const uint32_t i = i0 + j * kSlotBlock + threadIdx.x;
            if (i < n0) d0[i] = v0[j];
            if (i < n1) d1[i] = v1[j];
        }
    }
}

// dst[i] = lo[i] | hi[i] << 32 for i < n by the block (no high plane: 0)
__device__ __forceinline__ void stage_pair(uint64_t* dst, const uint32_t* __restrict__ lo,
                                           const uint32_t* __restrict__ hi, uint32_t n) {
    for (uint32_t i0 = 0; i0 < n; i0 += 2 * kSlotBlock) {
        uint32_t l[2], h[2];
#pragma unroll
        for (int j = 0; j < 2; j++) {
            const uint32_t i = i0 + j * kSlotBlock + threadIdx.x;
            l[j] = i < n ? lo[i] : 0u;
            h[j] = i < n && hi ? hi[i] : 0u;
        }
#pragma unroll
        for (int j = 0; j < 2; j++) {
            const uint32_t i = i0 + j * kSlotBlock + threadIdx.x;
            if (i < n) dst[i] = uint64_t(l[j]) | (uint64_t(h[j]) << 32);
        }
    }
}

// stores a count into the planes and its presence byte, the high plane and
// the bytes only where the table has them (streaming: the output is not read
// again by the kernel that writes it)
__device__ __forceinline__ void store_slot(const SlotArrays& o, uint64_t i, uint64_t c, bool present) {
    __builtin_nontemporal_store(uint32_t(c), &o.lo[i]);
    if (o.hi) __builtin_nontemporal_store(uint32_t(c >> 32), &o.hi[i]);
    if (o.flag) __builtin_nontemporal_store(uint8_t(present), &o.flag[i]);
}

// Four staged neighbours of one vertex with packed child slots: entry e =
// y | 8 colour(y) << 24 selects byte colour(y) of P, which holds 0x80 | the
// child's slot when colour(y) is in the child's colour set (else 0).  Every
// load is issued (a masked neighbour reads slot 0 of its own row, or of
// vertex 0 for the zero padding past a range) and the value is dropped by
// ok.  lo/hi/fl: colouring b's part of the child's planes.  NARROW: every
// count of the child's colouring is below 2^32, so the low plane suffices and
// no sum can wrap (fewer than 2^32 terms).  EXACT: no count of the colouring
// has wrapped, so an entry is present iff its count is not 0.
template <bool NARROW, bool EXACT, bool CHECK>
__device__ __forceinline__ void pack_step(const uint32_t* __restrict__ lo, const uint32_t* __restrict__ hi,
                                          const uint8_t* __restrict__ fl, const uint32_t* s_nb, int i, int z,
                                          uint64_t P, uint32_t R_in, uint64_t& sum, uint32_t& cnt, uint32_t& over) {
    uint32_t idx[4];
    bool ok[4];
#pragma unroll
    for (int j = 0; j < 4; j++) {
        const uint32_t e = s_nb[i + j];
        const uint32_t f = uint32_t(P >> (e >> 24));
        ok[j] = (f & 0x80u) != 0 && (!CHECK || i + j < z);
        idx[j] = __umul24(e, R_in) + (f & 0x7fu);  // < n R_in < 2^28
    }
    if (NARROW) {
        uint32_t cv[4];
#pragma unroll
        for (int j = 0; j < 4; j++) cv[j] = lo[idx[j]];
#pragma unroll
        for (int j = 0; j < 4; j++) cv[j] = ok[j] ? cv[j] : 0u;
#pragma unroll
        for (int j = 0; j < 4; j++) cnt += EXACT ? uint32_t(cv[j] != 0) : uint32_t(ok[j] && fl[idx[j]] != 0);
        sum += (uint64_t(cv[0]) + cv[1]) + (uint64_t(cv[2]) + cv[3]);
    } else {
        uint32_t l[4], h[4];
#pragma unroll
        for (int j = 0; j < 4; j++) {
            l[j] = lo[idx[j]];
            h[j] = hi[idx[j]];
        }
        uint64_t cv[4];
#pragma unroll
        for (int j = 0; j < 4; j++) cv[j] = ok[j] ? uint64_t(l[j]) | (uint64_t(h[j]) << 32) : 0u;
#pragma unroll
        for (int j = 0; j < 4; j++) cnt += EXACT ? uint32_t(cv[j] != 0) : uint32_t(ok[j] && fl[idx[j]] != 0);
#pragma unroll
        for (int j = 0; j < 4; j++) over |= uint32_t(__builtin_add_overflow(sum, cv[j], &sum));
    }
}

// neighbours [a, z) of the staged chunk: groups of four, the last one masked
template <bool NARROW, bool EXACT>
__device__ __forceinline__ void pack_gather(const uint32_t* __restrict__ lo, const uint32_t* __restrict__ hi,
                                            const uint8_t* __restrict__ fl, const uint32_t* s_nb, int a, int z,
                                            uint64_t P, uint32_t R_in, uint64_t& sum, uint32_t& cnt, uint32_t& over) {
    int i = a;
    for (; i + 4 <= z; i += 4) pack_step<NARROW, EXACT, false>(lo, hi, fl, s_nb, i, z, P, R_in, sum, cnt, over);
    if (i < z) pack_step<NARROW, EXACT, true>(lo, hi, fl, s_nb, i, z, P, R_in, sum, cnt, over);
}

// sets flag[b] when some lane's value has a nonzero high word (one atomic per wave)
__device__ __forceinline__ void flag_wide(uint32_t hi, uint32_t* flag) {
    if (__ballot(hi != 0) != 0 && __lane_id() == 0) atomicOr(flag, 1u);
}

}  // namespace

// Leaf (Sec. 3.1, leaf nodes; degree mask of Sec. 3.2): one slot per (b, v).
template <int M>
__global__ void __launch_bounds__(kSlotBlock) k_slot_leaf(SlotGrid G, DevGraph g, int degF, SlotArrays out,
                                                          uint64_t* part) {
    uint32_t b, v0, v1, jb, v, r;
    bool lane_ok;
    block_range(G, &b, &v0, &v1, &jb);
    slot_of(G, v0, jb, &v, &r, &lane_ok);
    uint32_t npres = 0;
#pragma unroll
    for (int i = 0; i < M; i++) {
        const uint32_t vi = v + uint32_t(i * G.upb);
        if (lane_ok && vi < v1) {
            const bool pres = g.rp[vi + 1] - g.rp[vi] >= degF;
            store_slot(out, uint64_t(b) * uint32_t(g.n) + vi, pres ? 1 : 0, pres);
            npres += pres;
        }
    }
    count_entries(npres, 0, part, G.blocks);
}

// Introduce u (image v) over a leaf child, followed by the forget of the
// leaf's vertex (Sec. 3): the child table holds one entry, of count 1, per
// vertex that passes the child's degree mask, so output slot (b, v,
// {colour(v), c}) counts the neighbours of v of colour c that pass it.  The
// block builds the colour histograms of its vertices' neighbourhoods in LDS
// from its CSR range, split evenly over the threads (a hub costs no more than
// its share), then every thread reads its slots from them.
template <int M>
__global__ void __launch_bounds__(kSlotBlock)
k_slot_edge_leaf(SlotGrid G, DevGraph g, const uint8_t* __restrict__ colors, int k, int degF_u, int degF_child,
                 SlotArrays out, uint64_t* part) {
    // [upb M + 1] CSR offsets relative to the block's first vertex, then
    // [upb M][k] neighbour counts by colour
    extern __shared__ uint32_t s_leaf[];
    uint32_t b, v0, v1, jb, v, r;
    bool lane_ok;
    block_range(G, &b, &v0, &v1, &jb);
    slot_of(G, v0, jb, &v, &r, &lane_ok);
    const uint32_t nv = v1 - v0;
    const uint8_t* cb = colors + uint64_t(b) * uint32_t(g.n);
    uint32_t* s_off = s_leaf;
    uint32_t* s_hist = s_leaf + G.upb * M + 1;
    const int64_t e_lo = nv ? g.rp[v0] : 0;
    for (uint32_t i = threadIdx.x; nv && i <= nv; i += kSlotBlock) s_off[i] = uint32_t(g.rp[v0 + i] - e_lo);
    for (uint32_t i = threadIdx.x; i < nv * uint32_t(k); i += kSlotBlock) s_hist[i] = 0;
    __syncthreads();
    const uint32_t E = nv ? s_off[nv] : 0;
    const uint32_t per = (E + kSlotBlock - 1) / kSlotBlock;
    uint32_t e = min(E, threadIdx.x * per);
    const uint32_t e_end = min(E, e + per);
    if (e < e_end) {
        // the vertex whose range holds entry e: s_off[lo] <= e < s_off[hi]
        uint32_t lo = 0, hi = nv;
        while (hi - lo > 1) {
            const uint32_t mid = (lo + hi) >> 1;
            if (s_off[mid] <= e)
                lo = mid;
            else
                hi = mid;
        }
        uint32_t lv = lo;
        for (; e < e_end; e += 4) {
            // four neighbours in flight: ids, then colours (and degrees)
            uint32_t y[4], c[4];
            bool pass[4];
#pragma unroll
            for (int j = 0; j < 4; j++) y[j] = e + j < e_end ? uint32_t(g.col[e_lo + e + j]) : 0u;
#pragma unroll
            for (int j = 0; j < 4; j++) {
                c[j] = cb[y[j]];
                pass[j] = e + j < e_end && (degF_child <= 1 || g.rp[y[j] + 1] - g.rp[y[j]] >= degF_child);
            }
#pragma unroll
            for (int j = 0; j < 4; j++) {
                if (e + j >= e_end) break;
                while (e + j >= s_off[lv + 1]) lv++;
                if (pass[j]) atomicAdd(&s_hist[lv * uint32_t(k) + c[j]], 1u);
            }
        }
    }
    __syncthreads();
    uint32_t npres = 0;
    uint64_t nin = 0;
#pragma unroll
    for (int i = 0; i < M; i++) {
        const uint32_t vi = v + uint32_t(i * G.upb);
        if (lane_ok && vi < v1) {
            const uint32_t lv = vi - v0;
            const uint32_t cv = cb[vi];
            // slot r of set size 2 is the r-th colour other than colour(v)
            const uint32_t h =
                s_off[lv + 1] - s_off[lv] >= uint32_t(degF_u) ? s_hist[lv * uint32_t(k) + r + (r >= cv)] : 0u;
            store_slot(out, (uint64_t(b) * uint32_t(g.n) + vi) * uint32_t(G.R) + r, h, h != 0);
            npres += h != 0;
            nin += h;
        }
    }
    count_entries(npres, nin, part, G.blocks);
}

// Two introduce-over-a-leaf steps at the same bag vertex u and the join of
// their tables (Sec. 3): the children's tables are the neighbourhood colour
// histograms h_a, h_c of v (neighbours passing the two leaves' degree masks),
// so output slot (b, v, {colour(v), c1, c2}) is h_a[c1] h_c[c2] + h_a[c2]
// h_c[c1] (below 2^63: each factor is at most the largest degree, below
// 2^31).  The children's tables are never stored; their entry counts (the
// introduce and forget nodes of each) go to part_a and part_c, the join's to
// part_j.  Needs R = C(k - 1, 2) >= k - 1 (k >= 4): the threads of slots
// r < k - 1 also count the children's entries of colour r (skipping
// colour(v)).
template <int M>
__global__ void __launch_bounds__(kSlotBlock)
k_slot_leaf_join(SlotGrid G, DevGraph g, const uint8_t* __restrict__ colors, int k, int degF_u, int degF_a,
                 int degF_c, const uint16_t* __restrict__ unrank, int uoff2, SlotArrays out, uint64_t* part_a,
                 uint64_t* part_c, uint64_t* part_j) {
    // [upb M + 1] CSR offsets relative to the block's first vertex, then the
    // [upb M][k] histograms h_a and h_c
    extern __shared__ uint32_t s_leaf[];
    uint32_t b, v0, v1, jb, v, r;
    bool lane_ok;
    block_range(G, &b, &v0, &v1, &jb);
    slot_of(G, v0, jb, &v, &r, &lane_ok);
    const uint32_t nv = v1 - v0, cap = uint32_t(G.upb * M);
    const uint8_t* cb = colors + uint64_t(b) * uint32_t(g.n);
    uint32_t* s_off = s_leaf;
    uint32_t* h_a = s_leaf + cap + 1;
    uint32_t* h_c = h_a + cap * uint32_t(k);
    const int64_t e_lo = nv ? g.rp[v0] : 0;
    for (uint32_t i = threadIdx.x; nv && i <= nv; i += kSlotBlock) s_off[i] = uint32_t(g.rp[v0 + i] - e_lo);
    for (uint32_t i = threadIdx.x; i < nv * uint32_t(k); i += kSlotBlock) h_a[i] = h_c[i] = 0;
    __syncthreads();
    const uint32_t E = nv ? s_off[nv] : 0;
    const uint32_t per = (E + kSlotBlock - 1) / kSlotBlock;
    uint32_t e = min(E, threadIdx.x * per);
    const uint32_t e_end = min(E, e + per);
    if (e < e_end) {
        // the vertex whose range holds entry e: s_off[lo] <= e < s_off[hi]
        uint32_t lo = 0, hi = nv;
        while (hi - lo > 1) {
            const uint32_t mid = (lo + hi) >> 1;
            if (s_off[mid] <= e)
                lo = mid;
            else
                hi = mid;
        }
        uint32_t lv = lo;
        for (; e < e_end; e += 4) {
            uint32_t y[4], c[4];
            int64_t d[4];
#pragma unroll
            for (int j = 0; j < 4; j++) y[j] = e + j < e_end ? uint32_t(g.col[e_lo + e + j]) : 0u;
#pragma unroll
            for (int j = 0; j < 4; j++) {
                c[j] = cb[y[j]];
                d[j] = degF_a > 1 || degF_c > 1 ? g.rp[y[j] + 1] - g.rp[y[j]] : 1;
            }
#pragma unroll
            for (int j = 0; j < 4; j++) {
                if (e + j >= e_end) break;
                while (e + j >= s_off[lv + 1]) lv++;
                if (d[j] >= degF_a) atomicAdd(&h_a[lv * uint32_t(k) + c[j]], 1u);
                if (d[j] >= degF_c) atomicAdd(&h_c[lv * uint32_t(k) + c[j]], 1u);
            }
        }
    }
    __syncthreads();
    uint32_t pr_a = 0, pr_c = 0, pr_j = 0, hi = 0;
    uint64_t in_a = 0, in_c = 0;
    const uint32_t m = lane_ok ? unrank[uoff2 + r] : 3u;  // two of the k - 1 other colours
    const uint32_t p1 = __ffs(m) - 1, p2 = 31 - __clz(m);
#pragma unroll
    for (int i = 0; i < M; i++) {
        const uint32_t vi = v + uint32_t(i * G.upb);
        if (!(lane_ok && vi < v1)) continue;
        const uint32_t lv = vi - v0;
        const uint32_t cv = cb[vi];
        const bool pass = s_off[lv + 1] - s_off[lv] >= uint32_t(degF_u);
        const uint32_t* ha = h_a + lv * uint32_t(k);
        const uint32_t* hc = h_c + lv * uint32_t(k);
        const uint32_t c1 = p1 + (p1 >= cv), c2 = p2 + (p2 >= cv);
        const uint64_t cnt = pass ? uint64_t(ha[c1]) * hc[c2] + uint64_t(ha[c2]) * hc[c1] : 0;
        store_slot(out, (uint64_t(b) * uint32_t(g.n) + vi) * uint32_t(G.R) + r, cnt, cnt != 0);
        pr_j += cnt != 0;
        hi |= uint32_t(cnt >> 32);
        if (pass && r < uint32_t(k - 1)) {  // colour slot r of the children's tables
            const uint32_t c = r + (r >= cv);
            in_a += ha[c];
            pr_a += ha[c] != 0;
            in_c += hc[c];
            pr_c += hc[c] != 0;
        }
    }
    flag_wide(hi, &out.wide[b]);
    count_entries(pr_a, in_a, part_a, G.blocks);
    count_entries(pr_c, in_c, part_c, G.blocks);
    count_entries(pr_j, 0, part_j, G.blocks);
}

// Introduce u (image v, every neighbour y of v is a candidate for the child's
// bag vertex) followed by the forget of the child's vertex: output slot
// (b, v, C) sums the child entries (b, y, C - colour(v)) over neighbours y,
// which requires colour(y) in C - colour(v).  The block partials count the
// introduce entries (child entries that pass) and the output entries.
// The neighbour lists of the block's vertices are one CSR range; it is
// staged in rounds of kEdgeChunk.  A thread serves the same slot of M
// vertices.  PACK (k <= kSlotPackK): the child slot of every neighbour colour
// comes from one packed word per vertex (slot_pack_tables) instead of a rank
// lookup.
template <int M, bool PACK>
__global__ void __launch_bounds__(kSlotBlock)
k_slot_edge(SlotArrays in, SlotGrid G, DevGraph g, const uint8_t* __restrict__ colors, int k, int degF_u,
            const uint16_t* __restrict__ rank, const uint16_t* __restrict__ unrank, int uoff,
            const uint64_t* __restrict__ pack, bool in_narrow, bool in_exact, SlotArrays out, uint64_t* part,
            uint32_t* ovf) {
    extern __shared__ uint16_t s_rank[];  // rank of every mask over k - 1 bits
    // staged neighbours: PACK: y | 8 colour << 24; otherwise the neighbour's
    // row offset y R_in (< 2^28) | colour << 28.  Four entries of padding let
    // a batch read past the end of a range.
    __shared__ uint32_t s_nb[kEdgeChunk + 4];
    uint32_t b, v0, v1, jb, v, r;
    bool lane_ok;
    block_range(G, &b, &v0, &v1, &jb);
    slot_of(G, v0, jb, &v, &r, &lane_ok);
    const uint32_t n = uint32_t(g.n);
    const uint32_t R_in = uint32_t(in.R);
    const uint64_t row0 = uint64_t(b) * n;
    // colouring b's part of the child table (n * R_in < 2^28 slots)
    const uint32_t* ilo = in.lo + row0 * R_in;
    const uint32_t* ihi = in.hi ? in.hi + row0 * R_in : nullptr;
    const uint8_t* ifl = in.flag ? in.flag + row0 * R_in : nullptr;
    if (!PACK) stage_rank(s_rank, rank, k);
    const uint8_t* cb = colors + row0;
    int64_t rb[M], re[M];
    uint32_t Cx[M];
    uint64_t P[M];
    uint64_t sum[M];
    uint32_t cnt[M];  // child entries gathered per vertex: the introduce entries; > 0 iff present
    uint32_t over = 0;
    const uint32_t mr = lane_ok && !PACK ? unrank[uoff + r] : 0;
#pragma unroll
    for (int i = 0; i < M; i++) {
        const uint32_t vi = v + uint32_t(i * G.upb);
        rb[i] = re[i] = 0;
        Cx[i] = 0;
        P[i] = 0;
        sum[i] = 0;
        cnt[i] = 0;
        if (lane_ok && vi < v1) {
            const int64_t a = g.rp[vi], z = g.rp[vi + 1];
            if (z - a >= degF_u) {
                rb[i] = a;
                re[i] = z;
                if (PACK)
                    P[i] = pack[uint32_t(cb[vi]) * uint32_t(G.R) + r];
                else  // the output set without colour(v), as a k-bit mask: the child's set
                    Cx[i] = bit_open(mr, cb[vi]);
            }
        }
    }
    // the child table of colouring b is exact (no count wrapped while it was
    // built) when a bound says so or b's overflow flag is still clear; then
    // presence is count != 0 (and the child has presence bytes otherwise)
    const bool exact = in_exact || (v1 > v0 && ovf[b] == 0);
    const bool narrow = in_narrow || !ihi || in.wide[b] == 0;
    const uint32_t rmask = (1u << (k - 1)) - 1u;  // keeps rank reads of masked-out lanes in the table
    const int64_t e_lo = v1 > v0 ? g.rp[v0] : 0, e_hi = v1 > v0 ? g.rp[v1] : 0;
    for (int64_t c0 = e_lo; c0 < e_hi; c0 += kEdgeChunk) {
        const int cn = int(min(int64_t(kEdgeChunk), e_hi - c0));
        __syncthreads();
        for (int i0 = 0; i0 < cn; i0 += 4 * kSlotBlock) {
            // four neighbours per thread: their loads are in flight together
            uint32_t y[4], c[4];
#pragma unroll
            for (int j = 0; j < 4; j++) {
                const int i = i0 + j * kSlotBlock + int(threadIdx.x);
                y[j] = i < cn ? uint32_t(g.col[c0 + i]) : 0u;
            }
#pragma unroll
            for (int j = 0; j < 4; j++) c[j] = cb[y[j]];
#pragma unroll
            for (int j = 0; j < 4; j++) {
                const int i = i0 + j * kSlotBlock + int(threadIdx.x);
                if (i < cn) s_nb[i] = PACK ? y[j] | (c[j] << 27) : y[j] * R_in | (c[j] << 28);
            }
        }
        if (threadIdx.x < 4) s_nb[cn + threadIdx.x] = 0;  // padding: vertex 0, colour 0
        __syncthreads();
#pragma unroll
        for (int u = 0; u < M; u++) {
            const int a = int(max(rb[u], c0) - c0), z = int(min(re[u], c0 + cn) - c0);
            if (PACK) {
                if (narrow && exact)
                    pack_gather<true, true>(ilo, ihi, ifl, s_nb, a, z, P[u], R_in, sum[u], cnt[u], over);
                else if (exact)
                    pack_gather<false, true>(ilo, ihi, ifl, s_nb, a, z, P[u], R_in, sum[u], cnt[u], over);
                else
                    pack_gather<false, false>(ilo, ihi, ifl, s_nb, a, z, P[u], R_in, sum[u], cnt[u], over);
                continue;
            }
            // four neighbours per round: their slot loads are in flight together.
            // Absent child entries read as 0, so every loaded count is added.
            constexpr int NB = 4;
            for (int i = a; i < z; i += NB) {
                uint32_t idx[NB];
                uint64_t cv[NB];
                bool ok[NB];
#pragma unroll
                for (int j = 0; j < NB; j++) {
                    const uint32_t e = s_nb[i + j];  // past z: padding or other vertices, masked by ok
                    const uint32_t cy = e >> 28;
                    ok[j] = (i + j < z) && ((Cx[u] >> cy) & 1u);
                    // slot within colouring b's table (< 2^28)
                    idx[j] = (e & 0x0fffffffu) + s_rank[bit_close(Cx[u], cy) & rmask];
                }
#pragma unroll
                for (int j = 0; j < NB; j++)
                    cv[j] = ok[j] ? (narrow ? uint64_t(ilo[idx[j]]) : uint64_t(ilo[idx[j]]) | (uint64_t(ihi[idx[j]]) << 32))
                                  : 0;
                if (exact) {
                    // no count of this colouring has wrapped: present entries hold >= 1
#pragma unroll
                    for (int j = 0; j < NB; j++) cnt[u] += cv[j] != 0;
                } else {
#pragma unroll
                    for (int j = 0; j < NB; j++) cnt[u] += ok[j] && ifl[idx[j]] != 0;
                }
#pragma unroll
                for (int j = 0; j < NB; j++) over |= uint32_t(__builtin_add_overflow(sum[u], cv[j], &sum[u]));
            }
        }
    }
    uint32_t npres = 0;
    uint64_t nin = 0;
#pragma unroll
    for (int i = 0; i < M; i++) {
        nin += cnt[i];
        npres += cnt[i] != 0;
    }
#pragma unroll
    for (int i = 0; i < M; i++) {
        const uint32_t vi = v + uint32_t(i * G.upb);
        if (lane_ok && vi < v1) store_slot(out, (row0 + vi) * uint32_t(G.R) + r, sum[i], cnt[i] != 0);
    }
    if (over) atomicOr(&ovf[b], 1u);
    uint32_t hi = 0;
#pragma unroll
    for (int i = 0; i < M; i++) hi |= uint32_t(sum[i] >> 32);
    flag_wide(hi, &out.wide[b]);
    count_entries(npres, nin, part, G.blocks);
}

// The join rows of push_join_epilogue: thread (slot r, first vertex) sums
// four vertices' splits at a time; Y, Z are the join's children (the leaf
// join rows in LDS as 32-bit words, E's accumulators).
template <class TY, class TZ>
__device__ __forceinline__ void push_join_rows(const TY* ys, uint32_t Ry, const TZ* zs, uint32_t Rz,
                                               const uint32_t* s_sp, int nsplit, uint32_t nv, SlotArrays out,
                                               uint64_t u0, uint32_t* pr, uint32_t* hi) {
    const uint32_t R_j = uint32_t(out.R), up = kSlotBlock / R_j;
    const uint32_t r = threadIdx.x % R_j, first = threadIdx.x / R_j;
    if (first >= up) return;
    for (uint32_t lv0 = first; lv0 < nv; lv0 += 4 * up) {
        uint64_t sum[4] = {0, 0, 0, 0};
        uint32_t by[4], bz[4];
#pragma unroll
        for (int j = 0; j < 4; j++) {
            const uint32_t lv = min(lv0 + uint32_t(j) * up, nv - 1);  // rows past nv are read, then dropped
            by[j] = lv * Ry;
            bz[j] = lv * Rz;
        }
        for (int t = 0; t < nsplit; t++) {
            const uint32_t sp = s_sp[uint32_t(t) * R_j + r];
            const uint32_t ry = sp & 0xffffu, rz = sp >> 16;
#pragma unroll
            for (int j = 0; j < 4; j++) sum[j] += uint64_t(ys[by[j] + ry]) * uint64_t(zs[bz[j] + rz]);
        }
#pragma unroll
        for (int j = 0; j < 4; j++) {
            const uint32_t lv = lv0 + uint32_t(j) * up;
            if (lv >= nv) break;
            store_slot(out, (u0 + lv) * R_j + r, sum[j], sum[j] != 0);
            *pr += sum[j] != 0;
            *hi |= uint32_t(sum[j] >> 32);
        }
    }
}

// A join of LDS rows X (stride Rx) with a leaf's table at the same vertex
// (slot q of vertex lv: h[colour q, skipping colour(v)]), thread (slot r,
// first vertex) summing four vertices at a time; the rows go to LDS (to,
// stride R_o) or, when to is null, to out.
template <class TX>
__device__ __forceinline__ void push_leaf_rows(const TX* xs, uint32_t Rx, bool x_is_y, const uint32_t* s_h,
                                               const uint8_t* s_cv, int k, const uint32_t* s_sp, int nsplit,
                                               uint32_t nv, uint32_t R_o, uint64_t* to, SlotArrays out, uint64_t u0,
                                               uint32_t* pr, uint32_t* hi) {
    const uint32_t up = kSlotBlock / R_o;
    const uint32_t r = threadIdx.x % R_o, first = threadIdx.x / R_o;
    if (first >= up) return;
    for (uint32_t lv0 = first; lv0 < nv; lv0 += 4 * up) {
        uint64_t sum[4] = {0, 0, 0, 0};
        uint32_t lvs[4], cv[4];
#pragma unroll
        for (int j = 0; j < 4; j++) {
            lvs[j] = min(lv0 + uint32_t(j) * up, nv - 1);  // rows past nv are read, then dropped
            cv[j] = s_cv[lvs[j]];
        }
        for (int t = 0; t < nsplit; t++) {
            const uint32_t sp = s_sp[uint32_t(t) * R_o + r];
            const uint32_t rx = x_is_y ? sp & 0xffffu : sp >> 16, rl = x_is_y ? sp >> 16 : sp & 0xffffu;
#pragma unroll
            for (int j = 0; j < 4; j++)
                sum[j] += uint64_t(xs[lvs[j] * Rx + rx]) * s_h[lvs[j] * uint32_t(k) + rl + (rl >= cv[j])];
        }
#pragma unroll
        for (int j = 0; j < 4; j++) {
            const uint32_t lv = lv0 + uint32_t(j) * up;
            if (lv >= nv) break;
            if (to)
                to[lv * R_o + r] = sum[j];
            else
                store_slot(out, (u0 + lv) * R_o + r, sum[j], sum[j] != 0);
            *pr += sum[j] != 0;
            *hi |= uint32_t(sum[j] >> 32);
        }
    }
}

// Epilogue of k_slot_edge_push<.., true>: after the push, with E's rows in
// acc and every vertex's neighbour counts by colour in s_h (vertices
// 0 .. nv - 1 of the block, first unit u0), the leaf join rows, the join
// and the entry partials of E, the two leaves, the leaf join and the join.
template <class Acc>
__device__ void push_join_epilogue(const Acc* acc, const uint32_t* s_off, const uint8_t* s_cv, const uint32_t* s_h,
                                   uint32_t* s_lj, uint32_t* s_sp, uint32_t nv, uint32_t R, int k, int degF_u,
                                   uint64_t u0, uint32_t b, uint32_t nin, const PushJoin& pj, uint64_t blocks) {
    const uint32_t R_lj = uint32_t((k - 1) * (k - 2) / 2), R_j = uint32_t(pj.out.R);
    // E: present slots (exact: present iff not 0)
    uint32_t pr_e = 0;
    for (uint32_t i = threadIdx.x; i < nv * R; i += kSlotBlock) pr_e += acc[i] != 0;
    if (pj.chain) {
        // E joined with one leaf (then the result with a second one): the
        // leaves' tables, and the first join's rows in LDS (s_lj, as 64-bit
        // words) when there are two
        uint32_t pr_l = 0;
        uint64_t in_l = 0;
        for (uint32_t i = threadIdx.x; i < nv * uint32_t(k - 1); i += kSlotBlock) {
            const uint32_t lv = i / uint32_t(k - 1), q = i - lv * uint32_t(k - 1);
            if (s_off[lv + 1] - s_off[lv] < uint32_t(degF_u)) continue;
            const uint32_t hq = s_h[lv * uint32_t(k) + q + (q >= s_cv[lv])];
            pr_l += hq != 0;
            in_l += hq;
        }
        const uint32_t R_1 = uint32_t(pj.r1);
        uint32_t* sp1 = s_sp;
        uint32_t* sp2 = s_sp + pj.nsplit1 * R_1;
        for (uint32_t i = threadIdx.x; i < uint32_t(pj.nsplit1) * R_1; i += kSlotBlock) {
            const uint32_t t = i / R_1;
            sp1[i] = pj.splits1[size_t(t) * pj.sstride1 + (i - t * R_1)];
        }
        if (pj.chain == 2)
            for (uint32_t i = threadIdx.x; i < uint32_t(pj.nsplit) * R_j; i += kSlotBlock) {
                const uint32_t t = i / R_j;
                sp2[i] = pj.splits[size_t(t) * pj.sstride + (i - t * R_j)];
            }
        __syncthreads();
        uint32_t pr_1 = 0, pr_j = 0, hi = 0;
        uint64_t* s_t1 = reinterpret_cast<uint64_t*>(s_lj);
        if (nv) {
            if (pj.chain == 2) {
                uint32_t hi1 = 0;
                push_leaf_rows(acc, R, pj.e_is_y1, s_h, s_cv, k, sp1, pj.nsplit1, nv, R_1, s_t1, pj.out, u0, &pr_1,
                               &hi1);
            } else {
                push_leaf_rows(acc, R, pj.e_is_y1, s_h, s_cv, k, sp1, pj.nsplit1, nv, R_1, nullptr, pj.out, u0, &pr_j,
                               &hi);
            }
        }
        if (pj.chain == 2) {
            __syncthreads();
            if (nv)
                push_leaf_rows(s_t1, R_1, pj.e_is_y2, s_h, s_cv, k, sp2, pj.nsplit, nv, R_j, nullptr, pj.out, u0, &pr_j,
                               &hi);
        }
        flag_wide(hi, &pj.out.wide[b]);
        if (pj.chain == 2) {
            const uint32_t prs[5] = {pr_e, pr_l, pr_l, pr_1, pr_j};
            const uint64_t exs[5] = {nin, in_l, in_l, 0, 0};
            uint64_t* const parts[5] = {pj.part_e, pj.part_a, pj.part_c, pj.part_lj, pj.part_j};
            count_entries_n<5>(prs, exs, parts, blocks);
        } else {  // one leaf: part_c is part_a
            const uint32_t prs[3] = {pr_e, pr_l, pr_j};
            const uint64_t exs[3] = {nin, in_l, 0};
            uint64_t* const parts[3] = {pj.part_e, pj.part_a, pj.part_lj};
            count_entries_n<3>(prs, exs, parts, blocks);
        }
        return;
    }
    // the leaf join, slot q = a pair {c1, c2} of the other colours: 2 h[c1]
    // h[c2]; the threads of slots q < k - 1 also count the leaves' colour
    // slot q (colour q, skipping colour(v)), h[colour], for both leaves
    uint32_t pr_l = 0, pr_lj = 0;
    uint64_t in_l = 0;
    {
        const uint32_t up = kSlotBlock / R_lj, q = threadIdx.x % R_lj, first = threadIdx.x / R_lj;
        if (first < up) {
            const uint32_t m = pj.unrank[q];
            const uint32_t p1 = __ffs(m) - 1, p2 = 31 - __clz(m);
            for (uint32_t lv = first; lv < nv; lv += up) {
                const uint32_t cv = s_cv[lv];
                const uint32_t* h = s_h + lv * uint32_t(k);
                uint32_t x = 0;
                if (s_off[lv + 1] - s_off[lv] >= uint32_t(degF_u)) {
                    x = 2u * h[p1 + (p1 >= cv)] * h[p2 + (p2 >= cv)];
                    if (q < uint32_t(k - 1)) {
                        const uint32_t hq = h[q + (q >= cv)];
                        pr_l += hq != 0;
                        in_l += hq;
                    }
                }
                s_lj[lv * R_lj + q] = x;
                pr_lj += x != 0;
            }
        }
    }
    for (uint32_t i = threadIdx.x; i < uint32_t(pj.nsplit) * R_j; i += kSlotBlock) {
        const uint32_t t = i / R_j;
        s_sp[i] = pj.splits[size_t(t) * pj.sstride + (i - t * R_j)];
    }
    __syncthreads();
    // the join: exact sums of exact products (no count of it can wrap)
    uint32_t pr_j = 0, hi = 0;
    if (nv) {
        if (pj.lj_is_y)
            push_join_rows(s_lj, R_lj, acc, R, s_sp, pj.nsplit, nv, pj.out, u0, &pr_j, &hi);
        else
            push_join_rows(acc, R, s_lj, R_lj, s_sp, pj.nsplit, nv, pj.out, u0, &pr_j, &hi);
    }
    flag_wide(hi, &pj.out.wide[b]);
    const uint32_t prs[5] = {pr_e, pr_l, pr_l, pr_lj, pr_j};
    const uint64_t exs[5] = {nin, in_l, in_l, 0, 0};
    uint64_t* const parts[5] = {pj.part_e, pj.part_a, pj.part_c, pj.part_lj, pj.part_j};
    count_entries_n<5>(prs, exs, parts, blocks);
}

// The same step pushed from the child's rows: for a neighbour entry (v, y)
// with colour(y) != colour(v), the child slots of y whose set C_y leaves out
// colour(v) are the same C(k-2, s_in-1) = W slots for every such pair of
// colours (slot_push_tables lists them with the output slot of C_y +
// colour(v)); W threads take one each and add the child's count into v's
// output row, kept in LDS.  Every thread's work is useful, where the gather
// spends most of its (output slot, neighbour) pairs on sets that do not
// contain colour(y).  Without WRAP no count of this or any lower table can
// wrap (a count bound), so every child table is exact and a sum is present
// iff it is not 0.  WIDE: 64-bit accumulators, else every output count is
// below 2^32.
//
// WRAP (with WIDE, not EPI): the bound allows counts of 2^64 or more, so sums
// wrap mod 2^64 and the output has presence bytes.  The child is exact when
// it has no presence bytes or colouring b's overflow flag is clear (its
// producers raise it before this launch), and then an entry is present iff
// its count is not 0; else its presence byte says.  An output slot is present
// iff its sum is not 0 or it took a present 0 or its sum wrapped (a bit per
// slot in LDS, set in those rare cases); a wrapped sum raises ovf[b].
//
// EPI: the step's table E is not stored.  Its only reader, a join at the
// same bag vertex with the fused leaf join of two leaves hanging off that
// vertex (Sec. 3, join nodes; leaves without a neighbour degree mask), is
// computed here instead (PushJoin): the block counts its vertices'
// neighbours by colour while it stages them, which gives the leaf tables
// h[c] and the leaf join 2 h[c1] h[c2] (below 2^32 by a bound), and the join
// output follows from the split table with E's rows still in LDS.  The
// partials of all five tables are written.
template <bool WIDE, bool EPI, bool WRAP, bool SEARCH>
__global__ void __launch_bounds__(kSlotBlock)
k_slot_edge_push(SlotArrays in, SlotGrid G, DevGraph g, const uint8_t* __restrict__ colors, int k, int degF_u,
                 const uint32_t* __restrict__ cmap, int W, SlotArrays out, uint64_t* part, PushJoin pj,
                 uint32_t* ovf) {
    static_assert(!WRAP || (WIDE && !EPI), "a wrapping push has 64-bit sums and no epilogue");
    using Acc = typename std::conditional<WIDE, unsigned long long, uint32_t>::type;
    // [upb M][R] accumulators, [upb M + 1] CSR offsets, the k k W (child
    // slot, output slot) pairs of cmap, [upb M] colours; EPI: then (4-byte
    // aligned) [upb M][k] neighbour counts by colour, then the epilogue's
    // rows and split rows (PushJoin) unless they fit s_stat; WRAP: then the
    // [upb M][R] bits of the slots whose presence is not their sum's
    extern __shared__ uint64_t s_dyn[];
    // the staged neighbour entries of a chunk, free again after the push:
    // s_y: neighbour | colour << 24; s_lv: its vertex within the block |
    // (colour(y) k + colour(v)) << 16, or 0xffffffff when v is masked or the
    // colours are equal
    __shared__ uint64_t s_stat[kPushChunk];
    uint32_t* s_y = reinterpret_cast<uint32_t*>(s_stat);
    uint32_t* s_lv = s_y + kPushChunk;
    uint32_t b, v0, v1, jb, v, r;
    bool lane_ok;
    block_range(G, &b, &v0, &v1, &jb);
    slot_of(G, v0, jb, &v, &r, &lane_ok);
    const uint32_t nv = v1 - v0, cap = uint32_t(G.upb * G.m), R = uint32_t(G.R), R_in = uint32_t(in.R);
    Acc* acc = reinterpret_cast<Acc*>(s_dyn);
    uint32_t* s_off = reinterpret_cast<uint32_t*>(acc + cap * R);
    uint32_t* s_cm = s_off + cap + 1;
    uint8_t* s_cv = reinterpret_cast<uint8_t*>(s_cm + k * k * W);
    uint32_t* s_h = reinterpret_cast<uint32_t*>(s_cm + k * k * W + (cap + 3) / 4);
    const uint32_t R_lj = uint32_t((k - 1) * (k - 2) / 2);
    // the epilogue's rows (8-byte aligned: a chain keeps 64-bit rows), then
    // its split rows, each in the chunk arrays when the launcher found room
    const uint32_t epi_rows = pj.chain == 2 ? 2u * cap * uint32_t(pj.r1) : pj.chain ? 0u : cap * R_lj;
    uint32_t* s_next = s_h + cap * uint32_t(k);
    s_next += (reinterpret_cast<uintptr_t>(s_next) >> 2) & 1u;
    uint32_t* s_st = reinterpret_cast<uint32_t*>(s_stat);
    uint32_t* s_lj = pj.rows_static ? s_st : s_next;
    if (!pj.rows_static) s_next += epi_rows;
    uint32_t* s_sp = pj.spl_static ? s_st + (pj.rows_static ? epi_rows : 0u) : s_next;
    const uint64_t row0 = uint64_t(b) * uint32_t(g.n);
    const uint8_t* cb = colors + row0;
    const uint32_t* ilo = in.lo + row0 * R_in;
    // the child's high plane only for a colouring in which some child count
    // reached 2^32 (its producer's flag); else every high word is 0
    const uint32_t* ihi = in.hi && (!in.wide || in.wide[b]) ? in.hi + row0 * R_in : nullptr;
    const uint8_t* ifl = WRAP && in.flag && ovf[b] != 0 ? in.flag + row0 * R_in : nullptr;
    uint32_t* s_cb = s_h;
    uint32_t carry = 0;
    const int64_t e_lo = nv ? g.rp[v0] : 0;
    for (uint32_t i = threadIdx.x; i < nv * R; i += kSlotBlock) acc[i] = 0;
    if (WRAP)
        for (uint32_t i = threadIdx.x; i < (nv * R + 31) / 32; i += kSlotBlock) s_cb[i] = 0;
    if (EPI)
        for (uint32_t i = threadIdx.x; i < nv * uint32_t(k); i += kSlotBlock) s_h[i] = 0;
    for (uint32_t i = threadIdx.x; nv && i <= nv; i += kSlotBlock) s_off[i] = uint32_t(g.rp[v0 + i] - e_lo);
    for (uint32_t i = threadIdx.x; i < nv; i += kSlotBlock) s_cv[i] = cb[v0 + i];
    for (uint32_t i = threadIdx.x; i < uint32_t(k * k * W); i += kSlotBlock) s_cm[i] = cmap[i];
    __syncthreads();
    const uint32_t E = nv ? s_off[nv] : 0;
    const uint32_t rows = kSlotBlock / uint32_t(W);  // neighbour entries per pass, W threads each
    const uint32_t te = threadIdx.x / uint32_t(W), tr = threadIdx.x - te * uint32_t(W);
    // largest power of two below nv: the first step of the search for an
    // entry's vertex
    const uint32_t top = nv > 1 ? 1u << (31 - __clz(nv - 1)) : 0u;
    // SEARCH (a graph with vertices of degree > kHeavyDegree): each staged
    // entry finds its vertex by a search, since a hub would keep one walking
    // thread busy for whole chunks; otherwise one thread per vertex walks its
    // few entries, which costs fewer LDS reads
    uint32_t nin = 0;
    for (uint32_t c0 = 0; c0 < E; c0 += kPushChunk) {
        const uint32_t cn = min(uint32_t(kPushChunk), E - c0);
        // one thread per staged entry: its neighbour, the neighbour's colour
        // and (search) its vertex within the block, the last lv whose row
        // starts at or before it
        for (uint32_t i0 = 0; i0 < cn; i0 += 4 * kSlotBlock) {
            uint32_t y[4];
#pragma unroll
            for (int j = 0; j < 4; j++) {
                const uint32_t i = i0 + j * kSlotBlock + threadIdx.x;
                y[j] = i < cn ? uint32_t(g.col[e_lo + c0 + i]) : 0u;
            }
#pragma unroll
            for (int j = 0; j < 4; j++) {
                const uint32_t i = i0 + j * kSlotBlock + threadIdx.x;
                const uint32_t c = cb[y[j]];
                if (i < cn && SEARCH) {
                    const uint32_t e = c0 + i;
                    uint32_t lv = 0;
                    for (uint32_t st = top; st; st >>= 1)
                        if (lv + st < nv && s_off[lv + st] <= e) lv += st;
                    const bool pass = s_off[lv + 1] - s_off[lv] >= uint32_t(degF_u);
                    const uint32_t cv = s_cv[lv];
                    s_y[i] = y[j] | (c << 24);
                    s_lv[i] = pass && c != cv ? lv | ((c * uint32_t(k) + cv) << 16) : 0xffffffffu;
                    if (EPI) atomicAdd(&s_h[lv * uint32_t(k) + c], 1u);
                } else if (i < cn) {
                    s_y[i] = y[j] | (c << 24);
                }
            }
        }
        __syncthreads();
        if (!SEARCH) {
            for (uint32_t lv = threadIdx.x; lv < nv; lv += kSlotBlock) {
                const uint32_t a = max(s_off[lv], c0), z = min(s_off[lv + 1], c0 + cn);
                const bool pass = s_off[lv + 1] - s_off[lv] >= uint32_t(degF_u);
                const uint32_t cv = s_cv[lv];
                for (uint32_t e = a; e < z; e++) {
                    const uint32_t cy = s_y[e - c0] >> 24;
                    s_lv[e - c0] = pass && cy != cv ? lv | ((cy * uint32_t(k) + cv) << 16) : 0xffffffffu;
                    if (EPI) s_h[lv * uint32_t(k) + cy]++;  // row lv is this thread's alone
                }
            }
            __syncthreads();
        }
        if (te < rows) {
            // eight neighbour entries per thread and round: their row loads are
            // in flight together
            constexpr int NE = 8;
            for (uint32_t e0 = te; e0 < cn; e0 += NE * rows) {
                uint32_t lv[NE], cm[NE], lo[NE], hi[NE];
                uint8_t fl[NE];
#pragma unroll
                for (int j = 0; j < NE; j++) {
                    const uint32_t e = e0 + j * rows;
                    const uint32_t ec = e < cn ? e : e0;  // past the chunk: a valid entry, masked
                    const uint32_t ye = s_y[ec];
                    const uint32_t m = e < cn ? s_lv[ec] : 0xffffffffu;
                    lv[j] = m == 0xffffffffu ? 0xffffu : m & 0xffffu;
                    cm[j] = m == 0xffffffffu ? 0u : s_cm[(m >> 16) * uint32_t(W) + tr];
                    const uint32_t idx = (ye & 0xffffffu) * R_in + (cm[j] & 0xffffu);  // < n R_in < 2^28
                    lo[j] = ilo[idx];
                    hi[j] = WIDE && ihi ? ihi[idx] : 0u;
                    fl[j] = WRAP && ifl ? ifl[idx] : uint8_t(1);
                }
#pragma unroll
                for (int j = 0; j < NE; j++) {
                    if (lv[j] == 0xffffu) continue;
                    const Acc val = WIDE ? (Acc(hi[j]) << 32) | lo[j] : Acc(lo[j]);
                    const uint32_t slot = lv[j] * R + (cm[j] >> 16);
                    if (WRAP) {
                        if (ifl ? fl[j] == 0 : val == 0) continue;  // absent
                        nin++;
                        bool mark = val == 0;
                        if (!mark) {
                            const Acc old = atomicAdd(&acc[slot], val);
                            mark = old + val < old;
                            carry |= uint32_t(mark);
                        }
                        if (mark) atomicOr(&s_cb[slot >> 5], 1u << (slot & 31u));
                        continue;
                    }
                    if (val == 0) continue;
                    nin++;
                    atomicAdd(&acc[slot], val);
                }
            }
        }
        __syncthreads();
    }
    if (EPI) {
        push_join_epilogue<Acc>(acc, s_off, s_cv, s_h, s_lj, s_sp, nv, R, k, degF_u, row0 + v0, b, nin, pj, G.blocks);
        return;
    }
    uint32_t npres = 0, hi = 0;
#pragma unroll 4
    for (int i = 0; i < G.m; i++) {
        const uint32_t vi = v + uint32_t(i * G.upb);
        if (lane_ok && vi < v1) {
            const uint32_t slot = (vi - v0) * R + r;
            const uint64_t c = acc[slot];
            const bool p = c != 0 || (WRAP && ((s_cb[slot >> 5] >> (slot & 31u)) & 1u));
            store_slot(out, (row0 + vi) * R + r, c, p);
            npres += p;
            hi |= uint32_t(c >> 32);
        }
    }
    flag_wide(hi, &out.wide[b]);
    if (WRAP && __ballot(carry != 0) != 0 && __lane_id() == 0) atomicOr(&ovf[b], 1u);
    count_entries(npres, nin, part, G.blocks);
}

// Join on a one-vertex bag (Sec. 3, join nodes): output slot (b, v, C) sums
// y(C_y) * z(C_z) over the splits of C - colour(v) into disjoint parts of the
// children's sizes.  The splits of slot r are the same for every vertex and
// colouring: row t of the split table holds (rank of C_y, rank of C_z) for
// every r (slot_split_tables), so a thread walks the rows once for its M
// vertices.  With STAGE the children's rows of the block's vertices
// (contiguous in both tables) and the split table are staged in LDS: only
// the low planes when both children's counts of the colouring are below
// 2^32 (then products are exact in 64 bits), else both planes combined.
// Presence bytes are read only for a colouring whose counts have wrapped.
// nowrap (from a bound on the counts, see run_slots): both children are
// narrow and no output sum can reach 2^64, so no wrap is tracked at all.
template <bool STAGE, int M>
__global__ void __launch_bounds__(kSlotBlock)
k_slot_join(SlotArrays y, SlotArrays z, const uint32_t* __restrict__ splits, int nsplit, int sstride, bool nowrap,
            bool in_exact, SlotGrid G, SlotArrays out, uint64_t* part, uint32_t* ovf) {
    extern __shared__ uint64_t s_mem[];
    uint32_t b, v0, v1, jb, v, r;
    bool lane_ok;
    block_range(G, &b, &v0, &v1, &jb);
    slot_of(G, v0, jb, &v, &r, &lane_ok);
    const uint32_t nu = v1 - v0;
    const uint64_t base = uint64_t(b) * uint32_t(G.n) + v0;  // first unit of the block
    // both children exact (by a bound, or no wrap yet in colouring b): an
    // entry is present iff its count is not 0; otherwise a child without
    // presence bytes is exact by its bound
    const bool exact = in_exact || (v1 > v0 && ovf[b] == 0);
    const bool narrow = nowrap || (y.wide[b] == 0 && z.wide[b] == 0);
    const int R = G.R, R_y = y.R, R_z = z.R;
    // layout: [y counts][z counts][split rows][y flags][z flags]; narrow
    // rows are 32-bit words at the start of the count regions.  nowrap:
    // [y words][z words][split rows] (exact, so no flags)
    const size_t cap = STAGE ? size_t(G.upb) * M : 0;
    uint64_t* s_yc = s_mem;
    uint64_t* s_zc = s_yc + cap * R_y;
    uint32_t* s_y32 = reinterpret_cast<uint32_t*>(s_yc);
    uint32_t* s_z32 = nowrap ? s_y32 + cap * R_y : reinterpret_cast<uint32_t*>(s_zc);
    uint32_t* s_sp = nowrap ? s_z32 + cap * R_z : reinterpret_cast<uint32_t*>(s_zc + cap * R_z);
    uint8_t* s_yf = reinterpret_cast<uint8_t*>(s_sp + (STAGE ? size_t(nsplit) * R : 0));
    uint8_t* s_zf = s_yf + cap * R_y;
    if (STAGE) {
        const uint32_t ny = nu * uint32_t(R_y), nz = nu * uint32_t(R_z);
        if (narrow) {
            stage_copy2(s_y32, y.lo + base * uint32_t(R_y), ny, s_z32, z.lo + base * uint32_t(R_z), nz);
        } else {
            stage_pair(s_yc, y.lo + base * uint32_t(R_y), y.hi ? y.hi + base * uint32_t(R_y) : nullptr, ny);
            stage_pair(s_zc, z.lo + base * uint32_t(R_z), z.hi ? z.hi + base * uint32_t(R_z) : nullptr, nz);
        }
        for (uint32_t i = threadIdx.x; i < uint32_t(nsplit * R); i += kSlotBlock) {
            const uint32_t t = i / uint32_t(R);
            s_sp[i] = splits[size_t(t) * sstride + (i - t * uint32_t(R))];
        }
        if (!exact && y.flag) stage_copy(s_yf, y.flag + base * uint32_t(R_y), ny);
        if (!exact && z.flag) stage_copy(s_zf, z.flag + base * uint32_t(R_z), nz);
        __syncthreads();
    }
    uint64_t sum[M];
    uint32_t pres = 0;
    bool over = false;
    using Idx = typename std::conditional<STAGE, uint32_t, uint64_t>::type;  // LDS or global row offsets
    Idx by[M], bz[M];
#pragma unroll
    for (int i = 0; i < M; i++) {
        sum[i] = 0;
        const uint64_t u = uint64_t(v - v0) + uint64_t(i) * G.upb;  // place within the block
        by[i] = Idx(STAGE ? u * uint32_t(R_y) : (base + u) * uint32_t(R_y));
        bz[i] = Idx(STAGE ? u * uint32_t(R_z) : (base + u) * uint32_t(R_z));
    }
    bool live[M];
#pragma unroll
    for (int i = 0; i < M; i++) live[i] = lane_ok && v + uint32_t(i * G.upb) < v1;
    if (STAGE && exact && lane_ok) {
        // Branch-free: every staged vertex row is read (rows past the block's
        // vertices hold stale LDS and are dropped by `live` at the end).  An
        // absent entry holds 0, so products of absent entries add nothing;
        // wrap and presence are kept per vertex.
        uint32_t wrap[M], seen[M];
#pragma unroll
        for (int i = 0; i < M; i++) {
            wrap[i] = 0;
            seen[i] = 0;
        }
        if (nowrap) {
            // exact sums of exact products: an entry is present iff its sum is not 0
            for (int t = 0; t < nsplit; t++) {
                const uint32_t e = s_sp[t * R + r];
                const uint32_t ry = e & 0xffffu, rz = e >> 16;
                uint32_t a[M], c[M];
#pragma unroll
                for (int i = 0; i < M; i++) {
                    a[i] = s_y32[by[i] + ry];
                    c[i] = s_z32[bz[i] + rz];
                }
#pragma unroll
                for (int i = 0; i < M; i++) sum[i] += uint64_t(a[i]) * c[i];
            }
#pragma unroll
            for (int i = 0; i < M; i++) seen[i] = sum[i] != 0;
        } else if (narrow) {
            // products of 32-bit factors are exact and nonzero iff both factors
            // are, so the OR of the products tells presence; wraps are counted
            uint64_t orp[M];
#pragma unroll
            for (int i = 0; i < M; i++) orp[i] = 0;
            for (int t = 0; t < nsplit; t++) {
                const uint32_t e = s_sp[t * R + r];
                const uint32_t ry = e & 0xffffu, rz = e >> 16;
                uint32_t a[M], c[M];
#pragma unroll
                for (int i = 0; i < M; i++) {
                    a[i] = s_y32[by[i] + ry];
                    c[i] = s_z32[bz[i] + rz];
                }
#pragma unroll
                for (int i = 0; i < M; i++) {
                    const uint64_t pr = uint64_t(a[i]) * c[i];
                    const uint64_t t2 = sum[i] + pr;
                    wrap[i] += t2 < pr;
                    sum[i] = t2;
                    orp[i] |= pr;
                }
            }
#pragma unroll
            for (int i = 0; i < M; i++) seen[i] = orp[i] != 0;
        } else {
            for (int t = 0; t < nsplit; t++) {
                const uint32_t e = s_sp[t * R + r];
                const uint32_t ry = e & 0xffffu, rz = e >> 16;
#pragma unroll
                for (int i = 0; i < M; i++) {
                    const uint64_t a = s_yc[by[i] + ry], c = s_zc[bz[i] + rz];
                    const uint64_t pr = a * c;
                    wrap[i] |= __umul64hi(a, c) != 0;
                    wrap[i] |= uint32_t(__builtin_add_overflow(sum[i], pr, &sum[i]));
                    seen[i] |= uint32_t(a != 0) & uint32_t(c != 0);
                }
            }
        }
#pragma unroll
        for (int i = 0; i < M; i++) {
            if (!live[i]) continue;
            over |= wrap[i] != 0;
            pres |= seen[i] << i;
        }
    } else if (live[0]) {
        for (int t = 0; t < nsplit; t++) {
            const uint32_t e = STAGE ? s_sp[t * R + r] : splits[size_t(t) * sstride + r];
            const uint32_t ry = e & 0xffffu, rz = e >> 16;
#pragma unroll
            for (int i = 0; i < M; i++) {
                if (!live[i]) continue;
                const uint64_t iy = by[i] + ry, iz = bz[i] + rz;
                uint64_t a, c;
                if (STAGE) {
                    a = narrow ? s_y32[iy] : s_yc[iy];
                    c = narrow ? s_z32[iz] : s_zc[iz];
                } else {
                    a = uint64_t(y.lo[iy]) | (y.hi ? uint64_t(y.hi[iy]) << 32 : 0);
                    c = uint64_t(z.lo[iz]) | (z.hi ? uint64_t(z.hi[iz]) << 32 : 0);
                }
                const bool fy = exact || !y.flag ? a != 0 : (STAGE ? s_yf[iy] : y.flag[iy]) != 0;
                const bool fz = exact || !z.flag ? c != 0 : (STAGE ? s_zf[iz] : z.flag[iz]) != 0;
                const bool f = fy && fz;
                if (!f) continue;
                uint64_t pr;
                if (((a | c) >> 32) == 0) {
                    pr = uint64_t(uint32_t(a)) * uint32_t(c);  // no wrap possible
                } else {
                    pr = a * c;
                    over |= __umul64hi(a, c) != 0;
                }
                sum[i] += pr;
                over |= sum[i] < pr;
                pres |= 1u << i;
            }
        }
    }
    uint32_t hi = 0;
#pragma unroll
    for (int i = 0; i < M; i++) {
        if (!live[i]) continue;
        store_slot(out, (base + uint64_t(v - v0) + uint64_t(i) * G.upb) * uint32_t(R) + r, sum[i], (pres >> i) & 1u);
        hi |= uint32_t(sum[i] >> 32);
    }
    if (over) atomicOr(&ovf[b], 1u);
    flag_wide(hi, &out.wide[b]);
    count_entries(__popc(pres), 0, part, G.blocks);
}

// The no-wrap join (k_slot_join with STAGE and nowrap) as persistent blocks:
// a block takes the virtual blocks L, L + stride, ... and loads the next
// one's child words into registers while it computes the current one from
// LDS, so the loads' latency overlaps the multiply-adds.  The split rows are
// staged once.  stride is a multiple of 8 (or the whole grid), so every
// virtual block of a block keeps the XCD of the one-shot mapping.
constexpr int kPipeWords = 8;  // staged child words per thread and virtual block
template <int M>
__global__ void __launch_bounds__(kSlotBlock)
k_slot_join_pipe(SlotArrays y, SlotArrays z, const uint32_t* __restrict__ splits, int nsplit, int sstride,
                 SlotGrid G, uint32_t stride, SlotArrays out, uint64_t* part) {
    extern __shared__ uint32_t s_w[];  // [upb M][R_y] y words, [upb M][R_z] z words, [nsplit][R] split rows
    const int R = G.R, R_y = y.R, R_z = z.R;
    const uint32_t cap = uint32_t(G.upb) * M;
    uint32_t* s_y32 = s_w;
    uint32_t* s_z32 = s_w + cap * R_y;
    uint32_t* s_sp = s_z32 + cap * R_z;
    for (uint32_t i = threadIdx.x; i < uint32_t(nsplit * R); i += kSlotBlock) {
        const uint32_t t = i / uint32_t(R);
        s_sp[i] = splits[size_t(t) * sstride + (i - t * uint32_t(R))];
    }
    uint32_t w[kPipeWords];
    // the child words of virtual block L: y's rows, then z's
    auto fetch = [&](uint32_t L) {
        uint32_t b, v0, v1, jb;
        block_range_at(G, L, &b, &v0, &v1, &jb);
        const uint64_t base = uint64_t(b) * uint32_t(G.n) + v0;
        const uint32_t ny = (v1 - v0) * uint32_t(R_y), nz = (v1 - v0) * uint32_t(R_z);
        const uint32_t* ys = y.lo + base * uint32_t(R_y);
        const uint32_t* zs = z.lo + base * uint32_t(R_z);
#pragma unroll
        for (int j = 0; j < kPipeWords; j++) {
            const uint32_t i = threadIdx.x + j * kSlotBlock;
            w[j] = i < ny ? ys[i] : i < ny + nz ? zs[i - ny] : 0u;
        }
    };
    uint32_t L = block_index();
    if (L < G.blocks) fetch(L);
    for (; L < G.blocks; L += stride) {
        uint32_t b, v0, v1, jb, v, r;
        bool lane_ok;
        block_range_at(G, L, &b, &v0, &v1, &jb);
        slot_of(G, v0, jb, &v, &r, &lane_ok);
        const uint32_t ny = (v1 - v0) * uint32_t(R_y), nz = (v1 - v0) * uint32_t(R_z);
#pragma unroll
        for (int j = 0; j < kPipeWords; j++) {
            const uint32_t i = threadIdx.x + j * kSlotBlock;
            if (i < ny)
                s_y32[i] = w[j];
            else if (i < ny + nz)
                s_z32[i - ny] = w[j];
        }
        __syncthreads();
        if (L + stride < G.blocks) fetch(L + stride);  // in flight during the sums below
        uint64_t sum[M];
        uint32_t by[M], bz[M];
#pragma unroll
        for (int i = 0; i < M; i++) {
            sum[i] = 0;
            const uint32_t u = (v - v0) + uint32_t(i * G.upb);
            by[i] = u * uint32_t(R_y);
            bz[i] = u * uint32_t(R_z);
        }
        if (lane_ok) {
            for (int t = 0; t < nsplit; t++) {
                const uint32_t e = s_sp[t * R + r];
                const uint32_t ry = e & 0xffffu, rz = e >> 16;
                uint32_t a[M], c[M];
#pragma unroll
                for (int i = 0; i < M; i++) {
                    a[i] = s_y32[by[i] + ry];
                    c[i] = s_z32[bz[i] + rz];
                }
#pragma unroll
                for (int i = 0; i < M; i++) sum[i] += uint64_t(a[i]) * c[i];
            }
        }
        uint32_t npres = 0, hi = 0;
#pragma unroll
        for (int i = 0; i < M; i++) {
            const uint32_t vi = v + uint32_t(i * G.upb);
            if (!(lane_ok && vi < v1)) continue;
            store_slot(out, (uint64_t(b) * uint32_t(G.n) + vi) * uint32_t(R) + r, sum[i], sum[i] != 0);
            npres += sum[i] != 0;
            hi |= uint32_t(sum[i] >> 32);
        }
        flag_wide(hi, &out.wide[b]);
        count_entries_at(npres, 0, part, G.blocks, L);  // its barrier also frees the staged rows
    }
}

// Root (Sec. 3, the root's value): per colouring, the sum of every entry of
// the one-column table below the root.  Each block stores its (sum, wrapped)
// at rpart[2 (b nbx + j)] (j = the block's place within colouring b) and
// k_slot_root_sum adds them; per_vertex (optional) gets the sum per image of
// the bag vertex, and csets a bitmap of the colour sets present (the entries
// of the root's own table), gathered per block in LDS.  One slot per vertex,
// M vertices per thread.
template <int M>
__global__ void __launch_bounds__(kSlotBlock)
k_slot_root(SlotArrays in, const uint8_t* __restrict__ colors, const uint16_t* __restrict__ unrank, int uoff, SlotGrid G,
            uint64_t* rpart, uint64_t* per_vertex, uint32_t* csets, int cwords) {
    extern __shared__ uint32_t s_cs[];
    uint32_t b, v0, v1, jb, v, r;
    bool lane_ok;
    block_range(G, &b, &v0, &v1, &jb);
    slot_of(G, v0, jb, &v, &r, &lane_ok);
    for (int i = threadIdx.x; i < cwords; i += kSlotBlock) s_cs[i] = 0;
    __syncthreads();
    uint64_t sum = 0;
    bool over = false;
#pragma unroll
    for (int i = 0; i < M; i++) {
        const uint32_t vi = v + uint32_t(i * G.upb);
        if (!(lane_ok && vi < v1)) continue;
        const uint64_t unit = uint64_t(b) * uint32_t(G.n) + vi;
        const int R_in = in.R;
        const uint32_t* pl = in.lo + unit * uint32_t(R_in);
        const uint32_t* ph = in.hi ? in.hi + unit * uint32_t(R_in) : nullptr;
        const uint8_t* f = in.flag ? in.flag + unit * uint32_t(R_in) : nullptr;
        const uint32_t cv = colors[unit];
        uint64_t us = 0;
        for (int j = 0; j < R_in; j++) {
            const uint64_t c = uint64_t(pl[j]) | (ph ? uint64_t(ph[j]) << 32 : 0);
            us += c;
            over |= us < c;
            if (f ? f[j] != 0 : c != 0) {  // no presence bytes: exact by a bound
                const uint32_t C = bit_open(unrank[uoff + j], cv) | (1u << cv);
                atomicOr(&s_cs[C >> 5], 1u << (C & 31));
            }
        }
        if (per_vertex) per_vertex[unit] = us;
        sum += us;
        over |= sum < us;
    }
    block_sum_wrap(&sum, &over);
    if (v1 > v0) {
        if (threadIdx.x == 0) {
            rpart[2 * (uint64_t(b) * G.nbx + jb)] = sum;
            rpart[2 * (uint64_t(b) * G.nbx + jb) + 1] = over;
        }
        for (int i = threadIdx.x; i < cwords; i += kSlotBlock)
            if (s_cs[i]) atomicOr(&csets[uint64_t(b) * cwords + i], s_cs[i]);
    }
}

// the partials of several steps: block x of step st adds every 16th
// segment of its partials into nsz[2 step], nsz[2 step + 1]
__device__ __forceinline__ void slot_sums_block(const uint64_t* __restrict__ part, const SlotSums& S, uint64_t* nsz,
                                                int st, uint32_t x) {
    const uint64_t* p = part + S.off[st];
    const uint64_t blocks = S.blocks[st];
    __shared__ uint64_t s_p[2][kSlotBlock / 64];
    uint64_t a = 0, c = 0;
    for (uint64_t i = uint64_t(x) * kSlotBlock + threadIdx.x; i < blocks; i += 16 * kSlotBlock) {
        a += p[2 * i];
        c += p[2 * i + 1];
    }
    a = wave_sum(a);
    c = wave_sum(c);
    if (__lane_id() == 0) {
        s_p[0][threadIdx.x >> 6] = a;
        s_p[1][threadIdx.x >> 6] = c;
    }
    __syncthreads();
    if (threadIdx.x < 2) {
        uint64_t t = 0;
        for (int i = 0; i < kSlotBlock / 64; i++) t += s_p[threadIdx.x][i];
        if (t) atomicAdd((unsigned long long*)&nsz[2 * S.step[st] + threadIdx.x], (unsigned long long)t);
    }
}

// counts[b] = the sum of colouring b's block partials; ovf[b] set if any
// wrapped.  Blocks B and above reduce the steps' entry partials (as
// k_slot_sums, 16 blocks per step), so both final reductions take one launch.
__global__ void __launch_bounds__(kSlotBlock)
k_slot_root_sum(const uint64_t* __restrict__ rpart, uint32_t nbx, int B, uint64_t* counts, uint32_t* ovf,
                const uint64_t* __restrict__ part, SlotSums S, uint64_t* nsz) {
    if (int(blockIdx.x) >= B) {
        const uint32_t j = blockIdx.x - uint32_t(B);
        slot_sums_block(part, S, nsz, int(j / 16), j % 16);
        return;
    }
    const uint32_t b = blockIdx.x;
    uint64_t sum = 0;
    bool over = false;
    for (uint32_t j = threadIdx.x; j < nbx; j += kSlotBlock) {
        const uint64_t c = rpart[2 * (uint64_t(b) * nbx + j)];
        sum += c;
        over |= (sum < c) || rpart[2 * (uint64_t(b) * nbx + j) + 1] != 0;
    }
    block_sum_wrap(&sum, &over);
    if (threadIdx.x == 0) {
        counts[b] = sum;
        if (over) ovf[b] = 1u;
    }
}

// out[0..1] += the (extra, present) partials of `blocks` blocks
__global__ void __launch_bounds__(kSlotBlock) k_slot_sum(const uint64_t* __restrict__ part, uint64_t blocks, uint64_t* out) {
    __shared__ uint64_t s_p[2][kSlotBlock / 64];
    uint64_t a = 0, c = 0;
    for (uint64_t i = uint64_t(blockIdx.x) * kSlotBlock + threadIdx.x; i < blocks; i += uint64_t(gridDim.x) * kSlotBlock) {
        a += part[2 * i];
        c += part[2 * i + 1];
    }
    a = wave_sum(a);
    c = wave_sum(c);
    if (__lane_id() == 0) {
        s_p[0][threadIdx.x >> 6] = a;
        s_p[1][threadIdx.x >> 6] = c;
    }
    __syncthreads();
    if (threadIdx.x < 2) {
        uint64_t t = 0;
        for (int i = 0; i < kSlotBlock / 64; i++) t += s_p[threadIdx.x][i];
        if (t) atomicAdd((unsigned long long*)&out[threadIdx.x], (unsigned long long)t);
    }
}

// the partials of several steps in one launch: blockIdx.y = step
__global__ void __launch_bounds__(kSlotBlock) k_slot_sums(const uint64_t* __restrict__ part, SlotSums S, uint64_t* nsz) {
    slot_sums_block(part, S, nsz, int(blockIdx.y), blockIdx.x);
}

void launch_slot_sums(const uint64_t* part, const SlotSums& S, uint64_t* nsz, hipStream_t s) {
    if (S.n) k_slot_sums<<<dim3(16, unsigned(S.n)), kSlotBlock, 0, s>>>(part, S, nsz);
}

void launch_slot_sum(const uint64_t* part, uint64_t blocks, uint64_t* out, hipStream_t s) {
    if (!blocks) return;
    const uint64_t g = std::min<uint64_t>(256, (blocks + kSlotBlock - 1) / kSlotBlock);
    k_slot_sum<<<unsigned(g), kSlotBlock, 0, s>>>(part, blocks, out);
}

std::vector<uint16_t> slot_rank_tables() {
    const int M = 1 << kSlotBits;
    std::vector<uint16_t> t(2 * M);
    int cursor[kSlotBits + 1] = {0};
    for (int m = 0; m < M; m++) {
        const int p = __builtin_popcount(unsigned(m));
        t[m] = uint16_t(cursor[p]);
        t[M + slot_unrank_offset(p) + cursor[p]] = uint16_t(m);
        cursor[p]++;
    }
    return t;
}

int slot_unrank_offset(int popcount) {  // masks of smaller popcount over kSlotBits bits
    int off = 0, c = 1;                   // c = C(kSlotBits, q)
    for (int q = 0; q < popcount; q++) {
        off += c;
        c = c * (kSlotBits - q) / (q + 1);
    }
    return off;
}

static dim3 slot_dims(uint64_t blocks) {  // x a multiple of 8, so the XCD of a block is its linear index mod 8
    const uint64_t X = 1u << 16;
    return blocks <= X ? dim3(unsigned(blocks)) : dim3(unsigned(X), unsigned((blocks + X - 1) / X));
}

SlotGrid slot_grid(int32_t n, int B, int R, int m_max) {
    SlotGrid G;
    G.n = n;
    G.B = B;
    G.R = R;
    G.xcd = B >= 8;
    // vertices per thread: as many as m_max allows while the grid keeps some
    // 2048 blocks to spread over the chip
    for (int m = (R <= kSlotBlock ? m_max : 1); m >= 1; m >>= 1) {
        int64_t nbx;
        G.m = m;
        if (R <= kSlotBlock) {
            G.upb = kSlotBlock / R;
            G.bpu = 0;
            nbx = (int64_t(n) + int64_t(G.upb) * m - 1) / (int64_t(G.upb) * m);
        } else {
            G.upb = 0;
            G.bpu = (R + kSlotBlock - 1) / kSlotBlock;
            nbx = int64_t(n) * G.bpu;
        }
        if (nbx >= (int64_t(1) << 32)) {  // beyond a 32-bit block index: callers take the sparse path
            G.nbx = 0;
            G.blocks = ~uint64_t(0);
            return G;
        }
        G.nbx = uint32_t(nbx);
        G.blocks = G.xcd ? uint64_t(nbx) * 8u * uint64_t((B + 7) / 8) : uint64_t(nbx) * uint64_t(B);
        if (G.blocks >= 2048 || m == 1) break;
    }
    return G;
}

// Split tables: for colour-set masks of p bits (slot r = rank among them) and
// every q-subset A of the mask (row t, Gosper order over bit positions):
// rank(A) | rank(mask - A) << 16.  Rows of (p, q) have stride C(kSlotBits, p)
// and start at slot_split_offset(p, q).
static int binom11(int p) {
    int c = 1;
    for (int i = 0; i < p; i++) c = c * (kSlotBits - i) / (i + 1);
    return c;
}
static int binom_pq(int p, int q) {
    if (q < 0 || q > p) return 0;
    int c = 1;
    for (int i = 0; i < q; i++) c = c * (p - i) / (i + 1);
    return c;
}

int slot_split_offset(int p, int q) {
    int off = 0;
    for (int pp = 0; pp <= kSlotBits; pp++)
        for (int qq = 0; qq <= pp; qq++) {
            if (pp == p && qq == q) return off;
            off += binom_pq(pp, qq) * binom11(pp);
        }
    return off;
}

std::vector<uint32_t> slot_split_tables() {
    std::vector<uint16_t> rt = slot_rank_tables();
    const int M = 1 << kSlotBits;
    std::vector<uint32_t> t(size_t(slot_split_offset(kSlotBits + 1, 0)));
    for (int p = 0; p <= kSlotBits; p++) {
        const int R = binom11(p);
        for (int q = 0; q <= p; q++) {
            const size_t off = size_t(slot_split_offset(p, q));
            for (int r = 0; r < R; r++) {
                const uint32_t m = rt[M + slot_unrank_offset(p) + r];
                int pos[kSlotBits], np = 0;
                for (int b = 0; b < kSlotBits; b++)
                    if ((m >> b) & 1u) pos[np++] = b;
                int row = 0;
                for (uint32_t x = 0; x < (1u << p); x++) {  // q-subsets of the positions, increasing
                    if (__builtin_popcount(x) != q) continue;
                    uint32_t A = 0;
                    for (int j = 0; j < p; j++)
                        if ((x >> j) & 1u) A |= 1u << pos[j];
                    t[off + size_t(row) * R + r] = uint32_t(rt[A]) | (uint32_t(rt[m ^ A]) << 16);
                    row++;
                }
            }
        }
    }
    return t;
}

size_t slot_pack_offset(int k, int p) {
    size_t off = 0;
    for (int kk = 2; kk <= kSlotPackK; kk++)
        for (int pp = 1; pp < kk; pp++) {
            if (kk == k && pp == p) return off;
            off += size_t(kk) * binom_pq(kk - 1, pp);
        }
    return off;  // past the last: the total
}

std::vector<uint64_t> slot_pack_tables() {
    std::vector<uint16_t> rt = slot_rank_tables();
    const int M = 1 << kSlotBits;
    std::vector<uint64_t> t(slot_pack_offset(kSlotPackK + 1, 1));
    for (int k = 2; k <= kSlotPackK; k++)
        for (int p = 1; p < k; p++) {
            const int R = binom_pq(k - 1, p);
            const size_t off = slot_pack_offset(k, p);
            for (int cv = 0; cv < k; cv++)
                for (int r = 0; r < R; r++) {
                    // the child's colour set: output slot r's set without cv, over k bits
                    const uint32_t C = bit_open(rt[M + slot_unrank_offset(p) + r], uint32_t(cv));
                    uint64_t w = 0;
                    for (int c = 0; c < k; c++)
                        if ((C >> c) & 1u) w |= uint64_t(0x80u | rt[bit_close(C, uint32_t(c))]) << (8 * c);
                    t[off + size_t(cv) * R + r] = w;
                }
        }
    return t;
}

// W(k, p) = C(k - 2, p): child slots of set size p + 1 that leave out a
// given colour other than the child's own
size_t slot_push_offset(int k, int p) {
    size_t off = 0;
    for (int kk = 2; kk <= kSlotPushK; kk++)
        for (int pp = 0; pp < kk - 1; pp++) {
            if (kk == k && pp == p) return off;
            off += size_t(kk) * kk * binom_pq(kk - 2, pp);
        }
    return off;  // past the last: the total
}

std::vector<uint32_t> slot_push_tables() {
    std::vector<uint16_t> rt = slot_rank_tables();
    const int M = 1 << kSlotBits;
    std::vector<uint32_t> t(slot_push_offset(kSlotPushK + 1, 0), 0xffffffffu);
    for (int k = 2; k <= kSlotPushK; k++)
        for (int p = 0; p < k - 1; p++) {
            const int R = binom_pq(k - 1, p), W = binom_pq(k - 2, p);
            const size_t off = slot_push_offset(k, p);
            for (int cy = 0; cy < k; cy++)
                for (int cv = 0; cv < k; cv++) {
                    if (cv == cy) continue;  // no child set leaves its own colour out
                    int w = 0;
                    for (int r = 0; r < R; r++) {
                        // the child's set over k bits, its own colour included
                        const uint32_t C = bit_open(rt[M + slot_unrank_offset(p) + r], uint32_t(cy)) | (1u << cy);
                        if ((C >> cv) & 1u) continue;
                        t[off + (size_t(cy) * k + cv) * W + w] = uint32_t(r) | (uint32_t(rt[bit_close(C, uint32_t(cv))]) << 16);
                        w++;
                    }
                }
        }
    return t;
}

// vertices per thread with which a join block stages its children's rows and
// split rows in kSlotJoinLds (0: none fit)
int slot_join_m(int R_out, int R_y, int R_z, int nsplit) {
    if (R_out > kSlotBlock) return 0;
    const size_t upb = size_t(kSlotBlock / R_out), spl = size_t(nsplit) * R_out * 4;
    for (int m = 8; m >= 1; m >>= 1)
        if (upb * m * size_t(R_y + R_z) * 9 + spl <= kSlotJoinLds) return m;
    return 0;
}

#define SLOT_BY_M(MACRO) \
    switch (G.m) {       \
        case 8: MACRO(8); break; \
        case 4: MACRO(4); break; \
        case 2: MACRO(2); break; \
        default: MACRO(1); break; \
    }

void launch_slot_leaf(const SlotGrid& G, DevGraph g, int degF, SlotArrays out, uint64_t* part, hipStream_t s) {
    if (!G.blocks) return;
#define LEAF_M(M) k_slot_leaf<M><<<slot_dims(G.blocks), kSlotBlock, 0, s>>>(G, g, degF, out, part)
    SLOT_BY_M(LEAF_M)
#undef LEAF_M
}

void launch_slot_leaf_join(const SlotGrid& G, DevGraph g, const uint8_t* colors, int k, int degF_u, int degF_a,
                           int degF_c, const uint16_t* unrank, SlotArrays out, uint64_t* part_a, uint64_t* part_c,
                           uint64_t* part_j, hipStream_t s) {
    if (!G.blocks) return;
    if (k < 4 || G.upb == 0 || G.R != (k - 1) * (k - 2) / 2)
        throw std::runtime_error("launch_slot_leaf_join: needs k >= 4 and R = C(k - 1, 2)");
    const size_t lds = 4 * (size_t(G.upb) * G.m * (2 * k + 1) + 1);
#define LEAF_JOIN_M(M)                                                                                              \
    k_slot_leaf_join<M><<<slot_dims(G.blocks), kSlotBlock, lds, s>>>(G, g, colors, k, degF_u, degF_a, degF_c, unrank, \
                                                                      slot_unrank_offset(2), out, part_a, part_c,   \
                                                                      part_j)
    SLOT_BY_M(LEAF_JOIN_M)
#undef LEAF_JOIN_M
}

void launch_slot_edge(SlotArrays in, const SlotGrid& G, DevGraph g, const uint8_t* colors, int k, int degF_u,
                      int degF_child, const uint16_t* rank, const uint16_t* unrank, int uoff, const uint64_t* pack,
                      bool in_narrow, bool in_exact, SlotArrays out, uint64_t* part, uint32_t* ovf, hipStream_t s) {
    if (!G.blocks) return;
    if (!in.lo) {  // leaf child: output set size 2, R = k - 1
        if (G.R != k - 1 || G.upb == 0) throw std::runtime_error("launch_slot_edge: a leaf child needs R = k - 1");
        const size_t lds = 4 * (size_t(G.upb) * G.m * (k + 1) + 1);
#define LEAF_EDGE_M(M) \
    k_slot_edge_leaf<M><<<slot_dims(G.blocks), kSlotBlock, lds, s>>>(G, g, colors, k, degF_u, degF_child, out, part)
        SLOT_BY_M(LEAF_EDGE_M)
#undef LEAF_EDGE_M
        return;
    }
    if (pack && (k > kSlotPackK || g.n >= (1 << 24) || G.upb == 0))
        throw std::runtime_error("launch_slot_edge: packed slots need k <= 8, n < 2^24 and R <= 256");
    const size_t lds = pack ? 0 : size_t(2) << (k - 1);
#define EDGE_ARGS in, G, g, colors, k, degF_u, rank, unrank, uoff, pack, in_narrow, in_exact, out, part, ovf
#define EDGE_M(M)                                                                     \
    if (pack)                                                                         \
        k_slot_edge<M, true><<<slot_dims(G.blocks), kSlotBlock, lds, s>>>(EDGE_ARGS); \
    else                                                                              \
        k_slot_edge<M, false><<<slot_dims(G.blocks), kSlotBlock, lds, s>>>(EDGE_ARGS)
    SLOT_BY_M(EDGE_M)
#undef EDGE_M
#undef EDGE_ARGS
}

// Dynamic LDS of k_slot_edge_push for grid G, child set size s_in and the
// epilogue pj (null: none); sets pj's rows_static and spl_static.
static size_t push_lds(int k, int s_in, const SlotGrid& G, bool wide, PushJoin* pj, bool wrap) {
    const int W = binom_pq(k - 2, s_in - 1);
    const size_t cap = size_t(G.upb) * G.m;
    size_t lds = cap * G.R * (wide ? 8 : 4) + 4 * (cap + 1) + 4 * size_t(k) * k * W + 4 * ((cap + 3) / 4);
    if (wrap) lds += 4 * ((cap * G.R + 31) / 32);
    if (pj) {
        // the epilogue's rows and split rows (32-bit words), in the chunk
        // arrays (kPushChunk 64-bit words) when they fit
        const size_t rows = pj->chain == 2 ? 2 * cap * size_t(pj->r1)
                            : pj->chain    ? 0
                                           : cap * size_t((k - 1) * (k - 2) / 2);
        const size_t spl = pj->chain ? size_t(pj->nsplit1) * pj->r1 + (pj->chain == 2 ? size_t(pj->nsplit) * pj->out.R : 0)
                                     : size_t(pj->nsplit) * pj->out.R;
        pj->rows_static = rows <= 2 * size_t(kPushChunk);
        pj->spl_static = (pj->rows_static ? rows : 0) + spl <= 2 * size_t(kPushChunk);
        lds += 4 * cap * size_t(k) + 4 + 4 * ((pj->rows_static ? 0 : rows) + (pj->spl_static ? 0 : spl));
    }
    return lds;
}

size_t slot_push_lds(int k, int s_in, const SlotGrid& G, bool wide, const PushJoin* pj, bool wrap) {
    PushJoin p = pj ? *pj : PushJoin();
    return push_lds(k, s_in, G, wide, pj ? &p : nullptr, wrap);
}

void launch_slot_edge_push(SlotArrays in, int s_in, const SlotGrid& G, DevGraph g, const uint8_t* colors, int k,
                           int degF_u, const uint32_t* push, bool wide, SlotArrays out, uint64_t* part,
                           const PushJoin* pj, bool wrap, uint32_t* ovf, hipStream_t s) {
    if (!G.blocks) return;
    if (wrap && (pj || !wide || !ovf || !out.flag))
        throw std::runtime_error("launch_slot_edge_push: a wrapping push needs 64-bit sums, presence bytes and the "
                                 "overflow flags, and no epilogue");
    if (k > kSlotPushK || g.n >= (1 << 24) || G.upb == 0 || s_in < 1 || s_in > k - 1)
        throw std::runtime_error("launch_slot_edge_push: needs k <= 10, n < 2^24, R <= 256 and a child set below k");
    if (pj && !pj->chain && k < 4) throw std::runtime_error("launch_slot_edge_push: a fused leaf join needs k >= 4");
    const int W = binom_pq(k - 2, s_in - 1);
    PushJoin none{};
    PushJoin pjl = pj ? *pj : none;
    const size_t lds = push_lds(k, s_in, G, wide, pj ? &pjl : nullptr, wrap);
    if (lds > kPushLdsMax) throw std::runtime_error("launch_slot_edge_push: dynamic LDS beyond kPushLdsMax");
#define PUSH_LAUNCH(WIDE, EPI, WRAP)                                                                                \
    do {                                                                                                             \
        if (g.nheavy > 0)                                                                                            \
            k_slot_edge_push<WIDE, EPI, WRAP, true><<<slot_dims(G.blocks), kSlotBlock, lds, s>>>(                    \
                in, G, g, colors, k, degF_u, push, W, out, part, pj ? pjl : none, ovf);                              \
        else                                                                                                         \
            k_slot_edge_push<WIDE, EPI, WRAP, false><<<slot_dims(G.blocks), kSlotBlock, lds, s>>>(                   \
                in, G, g, colors, k, degF_u, push, W, out, part, pj ? pjl : none, ovf);                              \
    } while (0)
    if (pj) {
        if (wide)
            PUSH_LAUNCH(true, true, false);
        else
            PUSH_LAUNCH(false, true, false);
    } else if (wrap) {
        PUSH_LAUNCH(true, false, true);
    } else {
        if (wide)
            PUSH_LAUNCH(true, false, false);
        else
            PUSH_LAUNCH(false, false, false);
    }
#undef PUSH_LAUNCH
}

void launch_slot_join(SlotArrays y, SlotArrays z, const uint32_t* splits, int nsplit, int sstride, bool nowrap,
                      bool in_exact, const SlotGrid& G, SlotArrays out, uint64_t* part, uint32_t* ovf, hipStream_t s) {
    if (!G.blocks) return;
    const bool stage = G.upb > 0 && slot_join_m(G.R, y.R, z.R, nsplit) >= G.m;
    const size_t cap = size_t(G.upb) * G.m;
    if (stage && nowrap && cap * (y.R + z.R) <= size_t(kPipeWords) * kSlotBlock && G.blocks < (uint64_t(1) << 32)) {
        const uint64_t grid = std::min<uint64_t>(G.blocks, 2048);  // a multiple of 8 when smaller than the grid
        const size_t lds = 4 * (cap * (y.R + z.R) + size_t(nsplit) * G.R);
#define PIPE_M(M)                                                                                                   \
    k_slot_join_pipe<M><<<unsigned(grid), kSlotBlock, lds, s>>>(y, z, splits, nsplit, sstride, G, uint32_t(grid), out, \
                                                                 part)
        SLOT_BY_M(PIPE_M)
#undef PIPE_M
        return;
    }
    const size_t lds = !stage   ? 0
                       : nowrap ? size_t(G.upb) * G.m * size_t(y.R + z.R) * 4 + size_t(nsplit) * G.R * 4
                                : size_t(G.upb) * G.m * size_t(y.R + z.R) * 9 + size_t(nsplit) * G.R * 4;
#define JOIN_M(M)                                                                                                      \
    if (stage)                                                                                                         \
        k_slot_join<true, M><<<slot_dims(G.blocks), kSlotBlock, lds, s>>>(y, z, splits, nsplit, sstride, nowrap,      \
                                                                           in_exact, G, out, part, ovf);               \
    else                                                                                                               \
        k_slot_join<false, M><<<slot_dims(G.blocks), kSlotBlock, 0, s>>>(y, z, splits, nsplit, sstride, false,         \
                                                                          in_exact, G, out, part, ovf)
    SLOT_BY_M(JOIN_M)
#undef JOIN_M
}

void launch_slot_root(SlotArrays in, int s_in, int32_t n, int B, const uint8_t* colors, const uint16_t* unrank,
                      uint64_t* rpart, uint64_t* counts, uint32_t* ovf, uint64_t* per_vertex, uint32_t* csets,
                      int cwords, const uint64_t* part, const SlotSums& sums, uint64_t* nsz, hipStream_t s) {
    SlotGrid G = slot_grid(n, B, 1, 8);
    if (!G.blocks) {
        launch_fill_u64(counts, 0, uint64_t(B), s);
        launch_slot_sums(part, sums, nsz, s);
        return;
    }
#define ROOT_M(M)                                                                                                 \
    k_slot_root<M><<<slot_dims(G.blocks), kSlotBlock, size_t(4) * cwords, s>>>(                                   \
        in, colors, unrank, slot_unrank_offset(s_in - 1), G, rpart, per_vertex, csets, cwords)
    SLOT_BY_M(ROOT_M)
#undef ROOT_M
    k_slot_root_sum<<<unsigned(B) + 16u * sums.n, kSlotBlock, 0, s>>>(rpart, G.nbx, B, counts, ovf, part, sums, nsz);
}

uint64_t slot_root_partials(int32_t n, int B) { return 2 * uint64_t(slot_grid(n, B, 1, 8).nbx) * uint64_t(B); }

// ---- count bounds of tree plans ---------------------------------------------
//
// Every count of a dense table (colouring b, image v, colour set C) is at most
// the number of homomorphisms of the table's pattern subtree into G that map
// its bag vertex to v: a leaf gives 1, an edge step sums its child's bound
// over N(v), a join multiplies its children's bounds.  These are real
// numbers here (doubles; only their maximum over v is used, with a margin),
// and the executor keeps a table narrow (no high plane) or exact (no presence
// bytes) when the maximum is below 2^32 or 2^64.  The bound is far below
// deg_max^(s - 1) on heavy-tailed graphs, where a few hubs set deg_max.

__global__ void k_hom_spmv(DevGraph g, const double* __restrict__ hin, double* __restrict__ hout) {
    for (uint64_t v = uint64_t(blockIdx.x) * blockDim.x + threadIdx.x; v < uint64_t(g.n);
         v += uint64_t(gridDim.x) * blockDim.x) {
        double acc = 0.0;
        for (int64_t e = g.rp[v]; e < g.rp[v + 1]; e++) acc += hin[g.col[e]];
        hout[v] = acc;
    }
}

__global__ void k_hom_mul(const double* __restrict__ a, const double* __restrict__ b, double* __restrict__ out,
                          uint64_t n) {
    for (uint64_t v = uint64_t(blockIdx.x) * blockDim.x + threadIdx.x; v < n; v += uint64_t(gridDim.x) * blockDim.x)
        out[v] = a[v] * b[v];
}

// maximum of non-negative doubles: their bit patterns order like the values
__global__ void k_hom_max(const double* __restrict__ h, uint64_t n, unsigned long long* out) {
    __shared__ unsigned long long w[kBlock / 64];
    unsigned long long m = 0;
    for (uint64_t v = uint64_t(blockIdx.x) * blockDim.x + threadIdx.x; v < n; v += uint64_t(gridDim.x) * blockDim.x) {
        const unsigned long long x = static_cast<unsigned long long>(__double_as_longlong(h[v]));
        m = x > m ? x : m;
    }
    for (int o = 32; o > 0; o >>= 1) {
        const unsigned long long y = __shfl_xor(m, o, 64);
        m = y > m ? y : m;
    }
    if ((threadIdx.x & 63) == 0) w[threadIdx.x >> 6] = m;
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int i = 1; i < kBlock / 64; i++) m = w[i] > m ? w[i] : m;
        atomicMax(out, m);
    }
}

void launch_hom_spmv(DevGraph g, const double* hin, double* hout, hipStream_t s) {
    if (g.n) k_hom_spmv<<<grid_for(uint64_t(g.n)), kBlock, 0, s>>>(g, hin, hout);
}

void launch_hom_mul(const double* a, const double* b, double* out, uint64_t n, hipStream_t s) {
    if (n) k_hom_mul<<<grid_for(n), kBlock, 0, s>>>(a, b, out, n);
}

void launch_hom_max(const double* h, uint64_t n, uint64_t* out, hipStream_t s) {
    if (n) k_hom_max<<<grid_for(n), kBlock, 0, s>>>(h, n, reinterpret_cast<unsigned long long*>(out));
}

}  // namespace ccg
