// Device-side helpers shared by the kernel files: packed key fields, CSR
// edge tests, wave/block scans and the dense colour-set accumulator.
#pragma once

#include <hip/hip_runtime.h>

#include "kernels.h"

namespace ccg {

namespace dev {

constexpr int kBlock = 256;
constexpr int kScanItems = 8;
constexpr int kScanTile = kBlock * kScanItems;

inline unsigned grid_for(uint64_t items, int per_block = kBlock, unsigned cap = 1u << 20) {
    uint64_t b = (items + per_block - 1) / per_block;
    if (b < 1) b = 1;
    if (b > cap) b = cap;
    return unsigned(b);
}

// ---- packed key fields ----
template <class K>
__device__ __forceinline__ uint32_t kcol(K key, const Lay& L, int j) {
    return uint32_t(key >> (L.kb + (L.b - 1 - j) * L.vb)) & ((1u << L.vb) - 1u);
}
template <class K>
__device__ __forceinline__ uint32_t kset(K key, const Lay& L) {
    return uint32_t(key) & ((1u << L.kb) - 1u);
}
template <class K>
__device__ __forceinline__ uint32_t kbid(K key, const Lay& L) {
    int sh = L.kb + L.b * L.vb;
    return sh >= int(8 * sizeof(K)) ? 0u : uint32_t(key >> sh);
}
template <class K>
__device__ __forceinline__ K kpack(uint32_t bid, const uint32_t* cols, int b, uint32_t C, const Lay& L) {
    K k = K(bid);
    for (int j = 0; j < b; j++) k = (k << L.vb) | K(cols[j]);
    return (k << L.kb) | K(C);
}
template <class K>
__device__ __forceinline__ K shr(K key, int sh) {
    return sh >= int(8 * sizeof(K)) ? K(0) : (key >> sh);
}

__device__ __forceinline__ int64_t gdeg(const DevGraph& g, uint32_t v) { return g.rp[v + 1] - g.rp[v]; }
// v passes the degree mask of the introduced vertex (deg_G(v) >= deg_F(u),
// Sec. 3.2) and lies in the step's image range
// (deg_F(u) <= 15 < 255, so the clamped byte decides it)
__device__ __forceinline__ bool intro_ok(const DevGraph& g, uint32_t v, int degF) {
    return int(g.deg8[v]) >= degF && int32_t(v) >= g.vlo && int32_t(v) < g.vhi;
}

// The edge set is probed a group of kEdgeGroup cells at a time (aligned, one
// vector load per two cells; the table is a power of two of at least 16
// cells, so groups never wrap).  A key sits at or after its home cell, before
// the first empty cell from there on: in the home group, cells before the
// home cell can hold the key (a hit all the same) but their empty cells do
// not end the search.  Returns 1: present, 0: absent, -1: look on in the
// next group.
constexpr int kEdgeGroup = 2;
__device__ __forceinline__ int edge_group(const uint64_t* __restrict__ eh, uint64_t grp, int first, uint64_t key) {
    uint64_t c[kEdgeGroup];
    if (kEdgeGroup == 1) {
        c[0] = eh[grp];
    } else {
        const ulonglong2* p = reinterpret_cast<const ulonglong2*>(eh + grp);
#pragma unroll
        for (int j = 0; j < kEdgeGroup / 2; j++) {
            const ulonglong2 x = p[j];
            c[2 * j] = x.x;
            c[2 * j + 1] = x.y;
        }
    }
    bool hit = false, empty = false;
#pragma unroll
    for (int j = 0; j < kEdgeGroup; j++) {
        hit |= c[j] == key;
        empty |= j >= first && c[j] == kEdgeEmpty;
    }
    return hit ? 1 : (empty ? 0 : -1);
}

// presence of an edge-set key: the home group, then the following ones
__device__ __forceinline__ bool edge_present(const DevGraph& g, uint64_t key) {
    const uint64_t h = edge_cell(key, g.ehmask);
    uint64_t grp = h & ~uint64_t(kEdgeGroup - 1);
    int r = edge_group(g.eh, grp, int(h & (kEdgeGroup - 1)), key);
    while (r < 0) {
        grp = (grp + kEdgeGroup) & g.ehmask;
        r = edge_group(g.eh, grp, 0, key);
    }
    return r > 0;
}

// index in col of the stored edge between x and y (x != y), searched in the
// shorter of the two rows; -1 when they are not adjacent
__device__ __forceinline__ int64_t edge_index(const DevGraph& g, uint32_t x, uint32_t y) {
    int64_t lo = g.rp[x], end = g.rp[x + 1];
    const int64_t lo_y = g.rp[y], end_y = g.rp[y + 1];
    uint32_t key = y;
    if (end_y - lo_y < end - lo) {
        lo = lo_y;
        end = end_y;
        key = x;
    }
    int64_t hi = end;
    while (lo < hi) {
        const int64_t mid = (lo + hi) >> 1;
        if (uint32_t(g.col[mid]) < key)
            lo = mid + 1;
        else
            hi = mid;
    }
    return (lo < end && uint32_t(g.col[lo]) == key) ? lo : -1;
}

// {a, b} in E(G)
__device__ __forceinline__ bool has_edge(const DevGraph& g, uint32_t a, uint32_t b) {
    if (a == b) return false;
    return edge_present(g, edge_key(a, b));
}

// four keys at once: the home groups' loads are in flight together
// (bit j of want: probe key j; returns the bits of the present ones)
__device__ __forceinline__ uint32_t edges_present4(const DevGraph& g, const uint64_t key[4], uint32_t want) {
    int r[4];
    uint64_t grp[4];
#pragma unroll
    for (int j = 0; j < 4; j++) {
        const uint64_t h = edge_cell(key[j], g.ehmask);
        grp[j] = h & ~uint64_t(kEdgeGroup - 1);
        r[j] = ((want >> j) & 1u) ? edge_group(g.eh, grp[j], int(h & (kEdgeGroup - 1)), key[j]) : 0;
    }
    uint32_t out = 0;
#pragma unroll
    for (int j = 0; j < 4; j++) {
        while (r[j] < 0) {  // rare: the chain runs past the home group
            grp[j] = (grp[j] + kEdgeGroup) & g.ehmask;
            r[j] = edge_group(g.eh, grp[j], 0, key[j]);
        }
        out |= uint32_t(r[j] > 0) << j;
    }
    return out;
}

__device__ __forceinline__ uint64_t lanemask_lt() {
    unsigned lane = __lane_id();
    return lane ? ((~0ull) >> (64 - lane)) : 0ull;
}

__device__ __forceinline__ uint64_t wave_incl_scan(uint64_t v) {
    int lane = __lane_id();
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
        uint64_t t = __shfl_up(v, d, 64);
        if (lane >= d) v += t;
    }
    return v;
}

__device__ __forceinline__ uint64_t wave_sum(uint64_t v) {
#pragma unroll
    for (int d = 32; d >= 1; d >>= 1) v += __shfl_xor(v, d, 64);
    return v;
}

// exclusive scan across a 256-thread block; *total = block sum
__device__ __forceinline__ uint64_t block_excl_scan(uint64_t v, uint64_t* total) {
    __shared__ uint64_t wsum[kBlock / 64];
    int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    uint64_t inc = wave_incl_scan(v);
    if (lane == 63) wsum[w] = inc;
    __syncthreads();
    uint64_t off = 0, tot = 0;
#pragma unroll
    for (int i = 0; i < kBlock / 64; i++) {
        if (i < w) off += wsum[i];
        tot += wsum[i];
    }
    __syncthreads();
    *total = tot;
    return off + inc - v;
}

// first index in [lo, hi) of a non-decreasing array with a[i] > x
__device__ __forceinline__ uint64_t upper_bound_u64(const uint64_t* a, uint64_t lo, uint64_t hi, uint64_t x) {
    while (lo < hi) {
        uint64_t mid = (lo + hi) >> 1;
        if (a[mid] <= x) lo = mid + 1;
        else hi = mid;
    }
    return lo;
}

}  // namespace dev

using namespace dev;

// ---------------------------------------------------------------------------
// Dense colour-set accumulator, one 64-lane workgroup per group: 2^k uint64
// counters plus a 2^k-bit presence mask in LDS.  Presence is tracked apart
// from the counters because a count may be 0 modulo 2^64 while the entry
// exists (the paper's nonzero configuration).

struct Acc {
    uint64_t* val;   // [1 << kb]
    uint32_t* bits;  // [max(1, (1 << kb) / 32)]
    int kb;
    __device__ int slots() const { return 1 << kb; }
    __device__ int words() const { return kb >= 5 ? (1 << (kb - 5)) : 1; }
};

// with values == false only the presence mask is allocated (count passes)
__device__ __forceinline__ Acc acc_bind(int kb, bool values) {
    extern __shared__ uint64_t smem[];
    Acc a;
    a.kb = kb;
    a.val = values ? smem : nullptr;
    a.bits = reinterpret_cast<uint32_t*>(values ? smem + (1 << kb) : smem);
    return a;
}

inline size_t acc_bytes(int kb, bool values) {
    size_t words = kb >= 5 ? (size_t(1) << (kb - 5)) : 1;
    return (values ? (size_t(8) << kb) : 0) + 4 * words;
}

__device__ __forceinline__ void acc_clear(Acc& a, bool values) {
    int lane = threadIdx.x;
    if (values)
        for (int i = lane; i < a.slots(); i += 64) a.val[i] = 0;
    for (int i = lane; i < a.words(); i += 64) a.bits[i] = 0;
}

__device__ __forceinline__ uint32_t acc_count(const Acc& a) {
    uint64_t c = 0;
    for (int i = threadIdx.x; i < a.words(); i += 64) c += __popc(a.bits[i]);
    return uint32_t(wave_sum(c));
}

// writes the present slots in increasing colour-set order
template <class KO>
__device__ __forceinline__ void acc_emit(const Acc& a, KO prefix, uint64_t base, KO* okeys, uint64_t* ocnt) {
    uint64_t run = 0;
    int lane = threadIdx.x;
    for (int c0 = 0; c0 < a.slots(); c0 += 64) {
        int C = c0 + lane;
        bool present = C < a.slots() && ((a.bits[C >> 5] >> (C & 31)) & 1u);
        uint64_t m = __ballot(present);
        if (present) {
            uint64_t o = base + run + __popcll(m & lanemask_lt());
            okeys[o] = prefix | KO(C);
            ocnt[o] = a.val[C];
        }
        run += __popcll(m);
    }
}


}  // namespace ccg
