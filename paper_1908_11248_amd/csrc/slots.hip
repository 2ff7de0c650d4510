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

#include "device.h"
#include "kernels.h"

namespace ccg {

namespace {

constexpr int kEdgeChunk = 1024;  // neighbours staged per round

__device__ __forceinline__ uint32_t bit_open(uint32_t m, uint32_t c) {  // insert a 0 at bit c
    return ((m >> c) << (c + 1)) | (m & ((1u << c) - 1u));
}
__device__ __forceinline__ uint32_t bit_close(uint32_t m, uint32_t c) {  // delete bit c
    return ((m >> (c + 1)) << c) | (m & ((1u << c) - 1u));
}

__device__ __forceinline__ uint32_t block_index() { return blockIdx.y * gridDim.x + blockIdx.x; }

// block -> (colouring, vertices [v0, v1)).  With xcd set, consecutive blocks
// (which the dispatcher deals round-robin to the eight XCDs) take eight
// different colourings, so each XCD's L2 holds the rows of the colouring it
// works on.  An empty range marks a block past the end.
__device__ __forceinline__ void block_range(const SlotGrid& G, uint32_t* b, uint32_t* v0, uint32_t* v1) {
    *b = 0;
    *v0 = *v1 = 0;
    const uint32_t L = block_index();
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
    if (G.upb > 0) {
        *v0 = j * uint32_t(G.upb);
        *v1 = min(*v0 + uint32_t(G.upb), uint32_t(G.n));
    } else {
        *v0 = j / uint32_t(G.bpu);
        *v1 = *v0 + 1;
    }
}

// this thread's (vertex, slot) inside the block's range; false if none
__device__ __forceinline__ bool slot_in(const SlotGrid& G, uint32_t v0, uint32_t v1, uint32_t* v, uint32_t* r) {
    uint32_t vv, rr;
    if (G.upb > 0) {
        const uint32_t u = threadIdx.x / uint32_t(G.R);
        vv = v0 + u;
        rr = threadIdx.x - u * uint32_t(G.R);
    } else {
        vv = v0;
        rr = ((block_index() >> (G.xcd ? 3 : 0)) % G.nbx % uint32_t(G.bpu)) * kSlotBlock + threadIdx.x;
    }
    *v = vv;
    *r = rr;
    return vv < v1 && rr < uint32_t(G.R);
}

// Entry counters of a step: kSlotCounters pairs (extra, present), each in
// its own 128-byte line; a wave adds into the pair of its block, so no
// single address takes every wave's atomic.
__device__ __forceinline__ void count_entries(bool present, uint64_t extra, unsigned long long* nsz) {
    const uint64_t pm = __ballot(present);
    const uint64_t ex = wave_sum(extra);
    if (__lane_id() == 0) {
        unsigned long long* c = nsz + uint64_t(block_index() % kSlotCounters) * kSlotCounterStride;
        if (pm) atomicAdd(&c[1], (unsigned long long)__popcll(pm));
        if (ex) atomicAdd(&c[0], (unsigned long long)ex);
    }
}

__device__ __forceinline__ void stage_rank(uint16_t* s_rank, const uint16_t* __restrict__ rank, int k) {
    for (int i = threadIdx.x; i < (1 << (k - 1)); i += kSlotBlock) s_rank[i] = rank[i];
}

}  // namespace

// Leaf (Sec. 3, leaf nodes; degree mask of Sec. 4): one slot per (b, v).
__global__ void __launch_bounds__(kSlotBlock)
k_slot_leaf(SlotGrid G, DevGraph g, int degF, uint64_t* ocnt, uint8_t* oflag, unsigned long long* nsz) {
    uint32_t b, v0, v1, v, r;
    block_range(G, &b, &v0, &v1);
    const bool valid = slot_in(G, v0, v1, &v, &r);
    bool pres = false;
    if (valid) {
        pres = g.rp[v + 1] - g.rp[v] >= degF;
        const uint64_t o = uint64_t(b) * uint32_t(g.n) + v;
        ocnt[o] = pres ? 1 : 0;
        oflag[o] = pres;
    }
    count_entries(pres, 0, nsz);
}

// Introduce u (image v, every neighbour y of v is a candidate for the child's
// bag vertex) followed by the forget of the child's vertex: output slot
// (b, v, C) sums the child entries (b, y, C - colour(v)) over neighbours y,
// which requires colour(y) in C - colour(v).  nsz[0] receives the number of
// introduce entries (child entries that pass), nsz[1] the output entries.
// The neighbour lists of the block's vertices are one CSR range; it is
// staged in rounds of kEdgeChunk (ids, and colours with the leaf child's
// degree test in bit 7).
template <bool LEAFCHILD>
__global__ void __launch_bounds__(kSlotBlock)
k_slot_edge(const uint64_t* __restrict__ icnt, const uint8_t* __restrict__ iflag, int R_in, SlotGrid G, DevGraph g,
            const uint8_t* __restrict__ colors, int k, int degF_u, int degF_child, const uint16_t* __restrict__ rank,
            const uint16_t* __restrict__ unrank, int uoff, uint64_t* ocnt, uint8_t* oflag, unsigned long long* nsz,
            uint32_t* ovf) {
    extern __shared__ uint16_t s_rank[];  // rank of every mask over k - 1 bits
    __shared__ uint32_t s_y[kEdgeChunk];
    __shared__ uint8_t s_c[kEdgeChunk];
    uint32_t b, v0, v1, v, r;
    block_range(G, &b, &v0, &v1);
    const bool valid = slot_in(G, v0, v1, &v, &r);
    stage_rank(s_rank, rank, k);
    const uint32_t n = uint32_t(g.n);
    const uint8_t* cb = colors + uint64_t(b) * n;
    const uint64_t row0 = uint64_t(b) * n;
    int64_t rb = 0, re = 0;
    uint32_t Cx = 0;
    bool act = false;
    if (valid) {
        rb = g.rp[v];
        re = g.rp[v + 1];
        act = re - rb >= degF_u;
        // the output set without colour(v), as a k-bit mask: the child's set
        if (act) Cx = bit_open(unrank[uoff + r], cb[v]);
    }
    uint64_t sum = 0, nin = 0;
    bool pres = false, over = false;
    // the child table of colouring b is exact (no count wrapped while it was
    // built) when b's overflow flag is still clear; then presence is count != 0
    const bool exact = LEAFCHILD || (v1 > v0 && ovf[b] == 0);
    const int64_t e_lo = v1 > v0 ? g.rp[v0] : 0, e_hi = v1 > v0 ? g.rp[v1] : 0;
    for (int64_t c0 = e_lo; c0 < e_hi; c0 += kEdgeChunk) {
        const int cn = int(min(int64_t(kEdgeChunk), e_hi - c0));
        __syncthreads();
        for (int i = threadIdx.x; i < cn; i += kSlotBlock) {
            const uint32_t y = uint32_t(g.col[c0 + i]);
            uint32_t c = cb[y];
            if (LEAFCHILD && g.rp[y + 1] - g.rp[y] >= degF_child) c |= 0x80u;
            s_y[i] = y;
            s_c[i] = uint8_t(c);
        }
        __syncthreads();
        if (!act) continue;
        const int a = int(max(rb, c0) - c0), z = int(min(re, c0 + cn) - c0);
        if (LEAFCHILD) {
            for (int i = a; i < z; i++) {
                const uint32_t c = s_c[i];
                if (((Cx >> (c & 0x7fu)) & 1u) && (c & 0x80u)) {
                    sum += 1;
                    nin++;
                    pres = true;
                }
            }
            continue;
        }
        // four neighbours per round: their slot loads are in flight together
        for (int i = a; i < z; i += 4) {
            uint64_t idx[4], cv[4];
            uint32_t ok = 0, fl = 0;
#pragma unroll
            for (int j = 0; j < 4; j++) {
                const int ii = min(i + j, z - 1);
                const uint32_t cy = s_c[ii] & 0x7fu;
                ok |= uint32_t((i + j < z) && ((Cx >> cy) & 1u)) << j;
                idx[j] = (row0 + s_y[ii]) * uint32_t(R_in) + s_rank[bit_close(Cx, cy)];
            }
#pragma unroll
            for (int j = 0; j < 4; j++) cv[j] = ((ok >> j) & 1u) ? icnt[idx[j]] : 0;
            if (exact) {
                // no count of this colouring has wrapped: present entries hold >= 1
#pragma unroll
                for (int j = 0; j < 4; j++) fl |= uint32_t(cv[j] != 0) << j;
            } else {
#pragma unroll
                for (int j = 0; j < 4; j++) fl |= uint32_t(((ok >> j) & 1u) && iflag[idx[j]]) << j;
            }
#pragma unroll
            for (int j = 0; j < 4; j++) {
                if ((fl >> j) & 1u) {
                    sum += cv[j];
                    over |= sum < cv[j];
                    nin++;
                    pres = true;
                }
            }
        }
    }
    if (valid) {
        const uint64_t o = (row0 + v) * uint32_t(G.R) + r;
        ocnt[o] = sum;
        oflag[o] = pres;
        if (over) atomicOr(&ovf[b], 1u);
    }
    count_entries(pres, nin, nsz);
}

// Join on a one-vertex bag (Sec. 3, join nodes): output slot (b, v, C) sums
// y(C_y) * z(C_z) over the splits of C - colour(v) into disjoint parts of the
// children's sizes (q of its p bits for the first child).  The splits are the
// q-subsets of bit positions, the same for every thread (Gosper's successor
// on a wave-uniform index), deposited into each thread's own mask.  With
// STAGE the children's rows of the block's vertices (contiguous in both
// tables) are staged in LDS; presence bytes are read only for a colouring
// whose counts have wrapped.
template <bool STAGE>
__global__ void __launch_bounds__(kSlotBlock)
k_slot_join(const uint64_t* __restrict__ ycnt, const uint8_t* __restrict__ yflag, int R_y,
            const uint64_t* __restrict__ zcnt, const uint8_t* __restrict__ zflag, int R_z, int q, int p, int k,
            SlotGrid G, const uint16_t* __restrict__ rank, const uint16_t* __restrict__ unrank, int uoff,
            uint64_t* ocnt, uint8_t* oflag, unsigned long long* nsz, uint32_t* ovf) {
    extern __shared__ uint64_t s_mem[];
    uint32_t b, v0, v1, v, r;
    block_range(G, &b, &v0, &v1);
    const bool valid = slot_in(G, v0, v1, &v, &r);
    const uint32_t nu = v1 - v0;
    const uint64_t base = uint64_t(b) * uint32_t(G.n) + v0;  // first unit of the block
    const bool exact = v1 > v0 && ovf[b] == 0;
    // layout: [y counts][z counts][rank table][y flags][z flags]
    const size_t cap = size_t(G.upb > 0 ? G.upb : 1);
    uint64_t* s_yc = s_mem;
    uint64_t* s_zc = s_yc + (STAGE ? cap * R_y : 0);
    uint16_t* s_rank = reinterpret_cast<uint16_t*>(s_zc + (STAGE ? cap * R_z : 0));
    uint8_t* s_yf = reinterpret_cast<uint8_t*>(s_rank + (1 << (k - 1)));
    uint8_t* s_zf = s_yf + (STAGE ? cap * R_y : 0);
    stage_rank(s_rank, rank, k);
    if (STAGE) {
        const uint32_t ny = nu * uint32_t(R_y), nz = nu * uint32_t(R_z);
        for (uint32_t i = threadIdx.x; i < ny; i += kSlotBlock) s_yc[i] = ycnt[base * uint32_t(R_y) + i];
        for (uint32_t i = threadIdx.x; i < nz; i += kSlotBlock) s_zc[i] = zcnt[base * uint32_t(R_z) + i];
        if (!exact) {
            for (uint32_t i = threadIdx.x; i < ny; i += kSlotBlock) s_yf[i] = yflag[base * uint32_t(R_y) + i];
            for (uint32_t i = threadIdx.x; i < nz; i += kSlotBlock) s_zf[i] = zflag[base * uint32_t(R_z) + i];
        }
    }
    __syncthreads();
    uint64_t sum = 0;
    bool pres = false, over = false;
    if (valid) {
        const uint32_t m = unrank[uoff + r];
        const uint64_t u = v - v0;
        const uint64_t by = STAGE ? u * uint32_t(R_y) : (base + u) * uint32_t(R_y);
        const uint64_t bz = STAGE ? u * uint32_t(R_z) : (base + u) * uint32_t(R_z);
        uint32_t bitpos[kSlotBits];  // one-hot j-th set bit of m
        {
            uint32_t mm = m;
#pragma unroll
            for (int j = 0; j < kSlotBits; j++) {
                bitpos[j] = mm & (0u - mm);
                mm &= mm - 1u;
            }
        }
        const uint32_t lim = 1u << p;
        uint32_t x = (1u << q) - 1u;
        bool more = true;
        while (more) {
            // up to four q-subsets x of the p positions (wave-uniform)
            uint32_t xs[4];
            int nx = 0;
#pragma unroll
            for (int j = 0; j < 4; j++) {
                if (more) {
                    xs[j] = x;
                    nx = j + 1;
                    if (x == 0) {
                        more = false;  // q = 0: the empty set only
                    } else {
                        const uint32_t c = x & (0u - x), rr = x + c;
                        x = (((rr ^ x) >> 2) >> (__ffs(c) - 1)) | rr;
                        more = x < lim;
                    }
                } else {
                    xs[j] = 0;
                }
            }
            uint64_t iy[4], iz[4], ya[4], zc[4];
#pragma unroll
            for (int j = 0; j < 4; j++) {
                uint32_t A = 0;
#pragma unroll
                for (int t = 0; t < kSlotBits; t++)
                    if ((xs[j] >> t) & 1u) A |= bitpos[t];
                iy[j] = by + s_rank[A];
                iz[j] = bz + s_rank[m ^ A];
            }
#pragma unroll
            for (int j = 0; j < 4; j++) {
                ya[j] = j < nx ? (STAGE ? s_yc[iy[j]] : ycnt[iy[j]]) : 0;
                zc[j] = j < nx ? (STAGE ? s_zc[iz[j]] : zcnt[iz[j]]) : 0;
            }
#pragma unroll
            for (int j = 0; j < 4; j++) {
                if (j >= nx) break;
                const bool f = exact ? (ya[j] != 0 && zc[j] != 0)
                                     : (STAGE ? (s_yf[iy[j]] && s_zf[iz[j]]) : (yflag[iy[j]] && zflag[iz[j]]));
                if (f) {
                    const uint64_t pr = ya[j] * zc[j];
                    over |= __umul64hi(ya[j], zc[j]) != 0;
                    sum += pr;
                    over |= sum < pr;
                    pres = true;
                }
            }
        }
        const uint64_t o = (base + u) * uint32_t(G.R) + r;
        ocnt[o] = sum;
        oflag[o] = pres;
        if (over) atomicOr(&ovf[b], 1u);
    }
    count_entries(pres, 0, nsz);
}

// Root (Sec. 3, the root's value): per colouring, the sum of every entry of
// the one-column table below the root; per_vertex (optional) gets the sum per
// image of that bag vertex, and csets a bitmap of the colour sets present
// (the entries of the root's own table), gathered per block in LDS.  One
// thread per (b, v).
__global__ void __launch_bounds__(kSlotBlock)
k_slot_root(const uint64_t* __restrict__ icnt, const uint8_t* __restrict__ iflag, int R_in,
            const uint8_t* __restrict__ colors, const uint16_t* __restrict__ unrank, int uoff, SlotGrid G,
            uint64_t* counts, uint32_t* ovf, uint64_t* per_vertex, uint32_t* csets, int cwords) {
    extern __shared__ uint32_t s_cs[];
    uint32_t b, v0, v1, v, r;
    block_range(G, &b, &v0, &v1);
    const bool valid = slot_in(G, v0, v1, &v, &r);
    for (int i = threadIdx.x; i < cwords; i += kSlotBlock) s_cs[i] = 0;
    __syncthreads();
    uint64_t sum = 0;
    bool over = false;
    if (valid) {
        const uint64_t unit = uint64_t(b) * uint32_t(G.n) + v;
        const uint64_t* p = icnt + unit * uint32_t(R_in);
        const uint8_t* f = iflag + unit * uint32_t(R_in);
        const uint32_t cv = colors[unit];
        for (int j = 0; j < R_in; j++) {
            const uint64_t c = p[j];
            sum += c;
            over |= sum < c;
            if (f[j]) {
                const uint32_t C = bit_open(unrank[uoff + j], cv) | (1u << cv);
                atomicOr(&s_cs[C >> 5], 1u << (C & 31));
            }
        }
        if (per_vertex) per_vertex[unit] = sum;
    }
    // every lane of the butterfly sums all 64 values, and a total of 2^64 or
    // more wraps in every lane's tree
    for (int d = 32; d >= 1; d >>= 1) {
        const uint64_t o = __shfl_xor(sum, d, 64);
        const uint64_t t = sum + o;
        over |= t < sum;
        sum = t;
    }
    const bool wave_over = __ballot(over) != 0;
    if (__lane_id() == 0 && __ballot(valid)) {
        const uint64_t old = atomicAdd((unsigned long long*)&counts[b], (unsigned long long)sum);
        if (wave_over || old + sum < old) atomicOr(&ovf[b], 1u);
    }
    __syncthreads();
    if (v1 > v0)
        for (int i = threadIdx.x; i < cwords; i += kSlotBlock)
            if (s_cs[i]) atomicOr(&csets[uint64_t(b) * cwords + i], s_cs[i]);
}

// nsz[j] = sum of the kSlotCounters spread counters j of each step
__global__ void k_slot_counters(const unsigned long long* spread, uint64_t* nsz) {
    const unsigned long long* c = spread + uint64_t(blockIdx.x >> 1) * kSlotCounters * kSlotCounterStride;
    const int j = blockIdx.x & 1;
    uint64_t v = 0;
    for (int i = threadIdx.x; i < kSlotCounters; i += 64) v += c[uint64_t(i) * kSlotCounterStride + j];
    v = wave_sum(v);
    if (threadIdx.x == 0) nsz[blockIdx.x] = v;
}

void launch_slot_counters(const unsigned long long* spread, int steps, uint64_t* nsz, hipStream_t s) {
    if (steps) k_slot_counters<<<2 * steps, 64, 0, s>>>(spread, nsz);
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

SlotGrid slot_grid(int32_t n, int B, int R) {
    SlotGrid G;
    G.n = n;
    G.B = B;
    G.R = R;
    int64_t nbx;
    if (R <= kSlotBlock) {
        G.upb = kSlotBlock / R;
        G.bpu = 0;
        nbx = (int64_t(n) + G.upb - 1) / G.upb;
    } else {
        G.upb = 0;
        G.bpu = (R + kSlotBlock - 1) / kSlotBlock;
        nbx = int64_t(n) * G.bpu;
    }
    G.xcd = B >= 8;
    if (nbx >= (int64_t(1) << 32)) {  // beyond a 32-bit block index: callers take the sparse path
        G.nbx = 0;
        G.blocks = ~uint64_t(0);
        return G;
    }
    G.nbx = uint32_t(nbx);
    G.blocks = G.xcd ? uint64_t(nbx) * 8u * uint64_t((B + 7) / 8) : uint64_t(nbx) * uint64_t(B);
    return G;
}

void launch_slot_leaf(const SlotGrid& G, DevGraph g, int degF, uint64_t* ocnt, uint8_t* oflag,
                      unsigned long long* nsz, hipStream_t s) {
    if (G.blocks) k_slot_leaf<<<slot_dims(G.blocks), kSlotBlock, 0, s>>>(G, g, degF, ocnt, oflag, nsz);
}

void launch_slot_edge(const uint64_t* icnt, const uint8_t* iflag, int R_in, const SlotGrid& G, DevGraph g,
                      const uint8_t* colors, int k, int degF_u, int degF_child, const uint16_t* rank,
                      const uint16_t* unrank, int uoff, uint64_t* ocnt, uint8_t* oflag, unsigned long long* nsz,
                      uint32_t* ovf, hipStream_t s) {
    if (!G.blocks) return;
    const size_t lds = size_t(2) << (k - 1);
    if (icnt)
        k_slot_edge<false><<<slot_dims(G.blocks), kSlotBlock, lds, s>>>(
            icnt, iflag, R_in, G, g, colors, k, degF_u, degF_child, rank, unrank, uoff, ocnt, oflag, nsz, ovf);
    else
        k_slot_edge<true><<<slot_dims(G.blocks), kSlotBlock, lds, s>>>(
            icnt, iflag, R_in, G, g, colors, k, degF_u, degF_child, rank, unrank, uoff, ocnt, oflag, nsz, ovf);
}

void launch_slot_join(const uint64_t* ycnt, const uint8_t* yflag, int R_y, const uint64_t* zcnt,
                      const uint8_t* zflag, int R_z, int q, int p, int k, const SlotGrid& G, const uint16_t* rank,
                      const uint16_t* unrank, int uoff, uint64_t* ocnt, uint8_t* oflag, unsigned long long* nsz,
                      uint32_t* ovf, hipStream_t s) {
    if (!G.blocks) return;
    const size_t units = size_t(G.upb > 0 ? G.upb : 1);
    const size_t staged = units * size_t(R_y + R_z) * 9;
    const size_t ranks = size_t(2) << (k - 1);
    if (staged + ranks <= kSlotJoinLds)
        k_slot_join<true><<<slot_dims(G.blocks), kSlotBlock, staged + ranks, s>>>(
            ycnt, yflag, R_y, zcnt, zflag, R_z, q, p, k, G, rank, unrank, uoff, ocnt, oflag, nsz, ovf);
    else
        k_slot_join<false><<<slot_dims(G.blocks), kSlotBlock, ranks, s>>>(
            ycnt, yflag, R_y, zcnt, zflag, R_z, q, p, k, G, rank, unrank, uoff, ocnt, oflag, nsz, ovf);
}

void launch_slot_root(const uint64_t* icnt, const uint8_t* iflag, int R_in, int s_in, int32_t n, int B,
                      const uint8_t* colors, const uint16_t* unrank, uint64_t* counts, uint32_t* ovf,
                      uint64_t* per_vertex, uint32_t* csets, int cwords, hipStream_t s) {
    SlotGrid G = slot_grid(n, B, 1);
    if (G.blocks)
        k_slot_root<<<slot_dims(G.blocks), kSlotBlock, size_t(4) * cwords, s>>>(
            icnt, iflag, R_in, colors, unrank, slot_unrank_offset(s_in - 1), G, counts, ovf, per_vertex, csets,
            cwords);
}

}  // namespace ccg
