// HIP kernels for gfx950 (CDNA4, wave64) implementing the node rules of the
// colour-coding dynamic program (Sec. 3.1) on sorted, packed-key tables.
//
// Work decomposition.  Every rule whose output size is data-dependent runs
// as count -> exclusive scan -> emit: a first kernel writes the number of
// entries each work unit produces, a scan turns them into write offsets, and
// the second kernel writes each unit's entries at its offset.  Units are
// processed in key order and each unit writes its entries in key order, so
// the output is sorted without a sort and is identical from run to run.
#include <hip/hip_runtime.h>

#include "device.h"
#include "kernels.h"

namespace ccg {


// ---------------------------------------------------------------------------
// scan (reduce, scan of block sums, down-sweep)

template <class T>
__global__ void __launch_bounds__(kBlock) k_scan_reduce(const T* __restrict__ in, uint64_t n, uint64_t* bsum) {
    uint64_t base = uint64_t(blockIdx.x) * kScanTile;
    uint64_t s = 0;
    for (int i = 0; i < kScanItems; i++) {
        uint64_t idx = base + uint64_t(i) * kBlock + threadIdx.x;
        if (idx < n) s += uint64_t(in[idx]);
    }
    uint64_t tot;
    block_excl_scan(s, &tot);
    if (threadIdx.x == 0) bsum[blockIdx.x] = tot;
}

template <class T>
__global__ void __launch_bounds__(kBlock) k_scan_down(const T* __restrict__ in, uint64_t n,
                                                      const uint64_t* __restrict__ boff, uint64_t* out) {
    uint64_t base = uint64_t(blockIdx.x) * kScanTile + uint64_t(threadIdx.x) * kScanItems;
    uint64_t vals[kScanItems];
    uint64_t s = 0;
#pragma unroll
    for (int i = 0; i < kScanItems; i++) {
        uint64_t idx = base + i;
        vals[i] = idx < n ? uint64_t(in[idx]) : 0;
        s += vals[i];
    }
    uint64_t tot;
    uint64_t off = block_excl_scan(s, &tot) + (boff ? boff[blockIdx.x] : 0);
#pragma unroll
    for (int i = 0; i < kScanItems; i++) {
        uint64_t idx = base + i;
        if (idx < n) out[idx] = off;
        off += vals[i];
    }
    if (blockIdx.x == gridDim.x - 1 && threadIdx.x == kBlock - 1) out[n] = off;
}

static size_t scan_tmp_rec(uint64_t n) {
    uint64_t nb = (n + kScanTile - 1) / kScanTile;
    if (nb <= 1) return 0;
    return (2 * (nb + 1)) * sizeof(uint64_t) + scan_tmp_rec(nb);
}

size_t scan_tmp_bytes(uint64_t n) { return scan_tmp_rec(n) + 256; }

template <class T>
static void scan_rec(const T* in, uint64_t* out, uint64_t n, uint64_t* tmp, hipStream_t s) {
    uint64_t nb = (n + kScanTile - 1) / kScanTile;
    if (nb <= 1) {
        k_scan_down<T><<<1, kBlock, 0, s>>>(in, n, nullptr, out);
        return;
    }
    uint64_t* bsum = tmp;
    uint64_t* boff = tmp + (nb + 1);
    k_scan_reduce<T><<<unsigned(nb), kBlock, 0, s>>>(in, n, bsum);
    scan_rec<uint64_t>(bsum, boff, nb, tmp + 2 * (nb + 1), s);
    k_scan_down<T><<<unsigned(nb), kBlock, 0, s>>>(in, n, boff, out);
}

void launch_scan_u32(const uint32_t* in, uint64_t* out, uint64_t n, uint64_t* tmp, hipStream_t s) {
    scan_rec<uint32_t>(in, out, n, tmp, s);
}

void launch_scan_u64(const uint64_t* in, uint64_t* out, uint64_t n, uint64_t* tmp, hipStream_t s) {
    scan_rec<uint64_t>(in, out, n, tmp, s);
}

__global__ void k_fill_u64(uint64_t* p, uint64_t v, uint64_t n) {
    for (uint64_t i = uint64_t(blockIdx.x) * blockDim.x + threadIdx.x; i < n; i += uint64_t(gridDim.x) * blockDim.x)
        p[i] = v;
}
__global__ void k_fill_u32(uint32_t* p, uint32_t v, uint64_t n) {
    for (uint64_t i = uint64_t(blockIdx.x) * blockDim.x + threadIdx.x; i < n; i += uint64_t(gridDim.x) * blockDim.x)
        p[i] = v;
}
void launch_fill_u64(uint64_t* p, uint64_t v, uint64_t n, hipStream_t s) {
    if (n) k_fill_u64<<<grid_for(n), kBlock, 0, s>>>(p, v, n);
}
void launch_fill_u32(uint32_t* p, uint32_t v, uint64_t n, hipStream_t s) {
    if (n) k_fill_u32<<<grid_for(n), kBlock, 0, s>>>(p, v, n);
}

// ---------------------------------------------------------------------------
// random colouring: splitmix64 of (seed XOR (b * 2^32 + v)), high word scaled to [0, k)

__device__ __forceinline__ uint64_t splitmix64(uint64_t x) {
    uint64_t z = x + 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

__global__ void k_color_hash(uint8_t* colors, int32_t n, int32_t B, int32_t k, uint64_t seed, uint32_t b0) {
    uint64_t total = uint64_t(n) * uint64_t(B);
    for (uint64_t i = uint64_t(blockIdx.x) * blockDim.x + threadIdx.x; i < total;
         i += uint64_t(gridDim.x) * blockDim.x) {
        uint64_t b = b0 + i / uint64_t(n), v = i % uint64_t(n);
        uint64_t h = splitmix64(seed ^ ((b << 32) + v));
        colors[i] = uint8_t(((h >> 32) * uint64_t(k)) >> 32);
    }
}

void launch_color_hash(uint8_t* colors, int32_t n, int32_t B, int32_t k, uint64_t seed, hipStream_t s) {
    launch_color_hash_from(colors, n, B, k, seed, 0, s);
}

void launch_color_hash_from(uint8_t* colors, int32_t n, int32_t B, int32_t k, uint64_t seed, uint32_t b0,
                            hipStream_t s) {
    uint64_t total = uint64_t(n) * uint64_t(B);
    if (total) k_color_hash<<<grid_for(total), kBlock, 0, s>>>(colors, n, B, k, seed, b0);
}

// ---------------------------------------------------------------------------
// run heads and run starts: runs of equal key >> shift in a sorted table, in
// two passes over the keys (per-tile head counts, then, after a scan of those,
// every run's first index written at its rank)

constexpr int kHeadItems = 16;
constexpr uint64_t kHeadTile = uint64_t(kBlock) * kHeadItems;

uint64_t head_tiles(uint64_t n) { return (n + kHeadTile - 1) / kHeadTile; }

// bit r: item base + r * kBlock + threadIdx.x starts a run
template <class K>
__device__ __forceinline__ uint32_t head_bits(const K* __restrict__ keys, uint64_t n, int shift, uint64_t base) {
    uint32_t hb = 0;
#pragma unroll
    for (int r = 0; r < kHeadItems; r++) {
        const uint64_t i = base + uint64_t(r) * kBlock + threadIdx.x;
        if (i < n && (i == 0 || shr(keys[i], shift) != shr(keys[i - 1], shift))) hb |= 1u << r;
    }
    return hb;
}

template <class K>
__global__ void __launch_bounds__(kBlock) k_head_count(const K* __restrict__ keys, uint64_t n, int shift,
                                                       uint64_t* tsum) {
    const uint32_t hb = head_bits(keys, n, shift, uint64_t(blockIdx.x) * kHeadTile);
    uint64_t tot;
    block_excl_scan(uint64_t(__popc(hb)), &tot);
    if (threadIdx.x == 0) tsum[blockIdx.x] = tot;
}

template <class K>
__global__ void __launch_bounds__(kBlock) k_head_starts(const K* __restrict__ keys, uint64_t n, int shift,
                                                        const uint64_t* __restrict__ toff, uint64_t* starts) {
    __shared__ uint32_t s_w[kBlock / 64];
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const uint64_t base = uint64_t(blockIdx.x) * kHeadTile;
    const uint32_t hb = head_bits(keys, n, shift, base);
    uint64_t at = toff[blockIdx.x];
    // round r: heads in (wave, lane) order, which is index order
    for (int r = 0; r < kHeadItems; r++) {
        const bool h = (hb >> r) & 1u;
        const uint64_t m = __ballot(h);
        if (lane == 0) s_w[w] = uint32_t(__popcll(m));
        __syncthreads();
        uint64_t before = 0, tot = 0;
#pragma unroll
        for (int q = 0; q < kBlock / 64; q++) {
            const uint32_t c = s_w[q];
            if (q < w) before += c;
            tot += c;
        }
        if (h) starts[at + before + __popcll(m & lanemask_lt())] = base + uint64_t(r) * kBlock + threadIdx.x;
        at += tot;
        __syncthreads();
    }
    if (blockIdx.x == gridDim.x - 1 && threadIdx.x == 0) starts[toff[gridDim.x]] = n;
}

void launch_head_count(const void* keys, int kw, uint64_t n, int shift, uint64_t* tsum, hipStream_t s) {
    const uint64_t nb = head_tiles(n);
    if (!nb) return;
    if (kw == 1)
        k_head_count<uint64_t><<<unsigned(nb), kBlock, 0, s>>>((const uint64_t*)keys, n, shift, tsum);
    else
        k_head_count<u128><<<unsigned(nb), kBlock, 0, s>>>((const u128*)keys, n, shift, tsum);
}

void launch_head_starts(const void* keys, int kw, uint64_t n, int shift, const uint64_t* toff, uint64_t* starts,
                        hipStream_t s) {
    const uint64_t nb = head_tiles(n);
    if (!nb) return;
    if (kw == 1)
        k_head_starts<uint64_t><<<unsigned(nb), kBlock, 0, s>>>((const uint64_t*)keys, n, shift, toff, starts);
    else
        k_head_starts<u128><<<unsigned(nb), kBlock, 0, s>>>((const u128*)keys, n, shift, toff, starts);
}

// ---------------------------------------------------------------------------
// leaf (Sec. 3.1): u -> v for every v with deg_G(v) >= deg_F(u) (Sec. 3.2)

__global__ void k_leaf_count(DevGraph g, int B, int degF, uint32_t* flags) {
    uint64_t total = uint64_t(g.n) * B;
    for (uint64_t i = uint64_t(blockIdx.x) * blockDim.x + threadIdx.x; i < total; i += uint64_t(gridDim.x) * blockDim.x) {
        uint32_t v = uint32_t(i % uint64_t(g.n));
        flags[i] = intro_ok(g, v, degF);
    }
}

template <class K>
__global__ void k_leaf_emit(DevGraph g, int B, int degF, const uint8_t* __restrict__ colors,
                            const uint64_t* __restrict__ offs, Lay lo, K* keys, uint64_t* cnt) {
    uint64_t total = uint64_t(g.n) * B;
    for (uint64_t i = uint64_t(blockIdx.x) * blockDim.x + threadIdx.x; i < total; i += uint64_t(gridDim.x) * blockDim.x) {
        uint32_t v = uint32_t(i % uint64_t(g.n));
        uint32_t bid = uint32_t(i / uint64_t(g.n));
        if (!intro_ok(g, v, degF)) continue;
        uint64_t o = offs[i];
        keys[o] = kpack<K>(bid, &v, 1, 1u << colors[i], lo);
        cnt[o] = 1;
    }
}

void launch_leaf_count(DevGraph g, int B, int degF, uint32_t* flags, hipStream_t s) {
    uint64_t total = uint64_t(g.n) * B;
    if (total) k_leaf_count<<<grid_for(total), kBlock, 0, s>>>(g, B, degF, flags);
}

void launch_leaf_emit(DevGraph g, int B, int degF, const uint8_t* colors, const uint64_t* offs, Lay lo,
                      void* keys, uint64_t* cnt, hipStream_t s) {
    uint64_t total = uint64_t(g.n) * B;
    if (!total) return;
    if (lo.kw() == 1)
        k_leaf_emit<uint64_t><<<grid_for(total), kBlock, 0, s>>>(g, B, degF, colors, offs, lo, (uint64_t*)keys, cnt);
    else
        k_leaf_emit<u128><<<grid_for(total), kBlock, 0, s>>>(g, B, degF, colors, offs, lo, (u128*)keys, cnt);
}

// ---------------------------------------------------------------------------
// introduce, push form: candidates per prefix group (the child entries that
// share the images of the columns before the insertion point) come from the
// adjacency list of a mapped bag neighbour (Sec. 3.2); expand.hip does the
// rest.

template <class K>
__global__ void k_push_work(const K* __restrict__ keys, Lay L, const uint64_t* __restrict__ gstart, uint64_t G,
                            DevGraph g, IntroArgs a, uint32_t* wcount) {
    for (uint64_t i = uint64_t(blockIdx.x) * blockDim.x + threadIdx.x; i < G; i += uint64_t(gridDim.x) * blockDim.x) {
        if (a.anchor < 0) {
            wcount[i] = uint32_t(g.n);
        } else if (a.cn0 >= 0) {  // the common neighbours of two adjacent bag images
            const K k0 = keys[gstart[i]];
            const int64_t ei = edge_index(g, kcol(k0, L, a.cn0), kcol(k0, L, a.cn1));
            const uint64_t c0 = ei >= 0 ? a.cn_off[ei] : 0, c1 = ei >= 0 ? a.cn_off[ei + 1] : 0;
            wcount[i] = uint32_t(c1 - c0);
            a.erow[i] = int64_t(c0);
        } else {
            // candidates: neighbours of the image with the fewest of them
            // (Sec. 3.2: every bag neighbour's image must be adjacent)
            const K k0 = keys[gstart[i]];
            int best = a.anchor;
            int64_t bd = gdeg(g, kcol(k0, L, a.anchor));
            for (int c = 0; c < a.nchk; c++) {
                if (!a.grouped && a.chk[c] >= a.pos) continue;
                const int64_t d = gdeg(g, kcol(k0, L, a.chk[c]));
                if (d < bd) {
                    bd = d;
                    best = a.chk[c];
                }
            }
            wcount[i] = uint32_t(bd);
            if (a.sel) a.sel[i] = uint8_t(best);
        }
    }
}

void launch_push_work(const DevTable& in, const uint64_t* gstart, uint64_t G, DevGraph g, const IntroArgs& a,
                      uint32_t* wcount, hipStream_t s) {
    if (!G) return;
    if (in.lay.kw() == 1)
        k_push_work<uint64_t><<<grid_for(G), kBlock, 0, s>>>((const uint64_t*)in.keys, in.lay, gstart, G, g, a, wcount);
    else
        k_push_work<u128><<<grid_for(G), kBlock, 0, s>>>((const u128*)in.keys, in.lay, gstart, G, g, a, wcount);
}

// ---------------------------------------------------------------------------
// introduce, pull form: u inserted as column 0.  For every colouring b and
// every stored edge (v, y) of G (rows ascending), the child's run of entries
// with column 0 = y is extended by u -> v (expand.hip); output order
// (b, v, y, rest, C).  The run index below locates those runs.

template <class K>
__global__ void k_pull_index(const K* __restrict__ keys, uint64_t N, Lay L, int32_t n, uint64_t* rstart,
                             uint64_t* rend) {
    int sh = L.kb + (L.b - 1) * L.vb;
    for (uint64_t i = uint64_t(blockIdx.x) * blockDim.x + threadIdx.x; i < N; i += uint64_t(gridDim.x) * blockDim.x) {
        K k = keys[i];
        K p = shr(k, sh);
        uint64_t slot = uint64_t(kbid(k, L)) * uint64_t(n) + kcol(k, L, 0);
        if (i == 0 || shr(keys[i - 1], sh) != p) rstart[slot] = i;
        if (i + 1 == N || shr(keys[i + 1], sh) != p) rend[slot] = i + 1;
    }
}

void launch_pull_index(const DevTable& in, int32_t n, uint64_t* rstart, uint64_t* rend, hipStream_t s) {
    if (!in.n) return;
    if (in.lay.kw() == 1)
        k_pull_index<uint64_t><<<grid_for(in.n), kBlock, 0, s>>>((const uint64_t*)in.keys, in.n, in.lay, n, rstart, rend);
    else
        k_pull_index<u128><<<grid_for(in.n), kBlock, 0, s>>>((const u128*)in.keys, in.n, in.lay, n, rstart, rend);
}

// ---------------------------------------------------------------------------
// forget of the last column (Sec. 3.1 forget rule): per run of equal
// (colouring, first b-1 images), add the counts of equal colour sets.
// Runs longer than kForgetSmall go through a dense LDS accumulator, one run
// per 64-lane workgroup; shorter ones through k_forget_small.
constexpr int kForgetSmall = 16;

// lane 0's value of x, word by word
template <class T>
__device__ __forceinline__ T from_lane0(T x) {
    uint32_t w[sizeof(T) / 4];
    __builtin_memcpy(w, &x, sizeof(T));
#pragma unroll
    for (int i = 0; i < int(sizeof(T) / 4); i++) w[i] = __builtin_amdgcn_readlane(w[i], 0);
    __builtin_memcpy(&x, w, sizeof(T));
    return x;
}

template <class KI, class KO, bool EMIT>
__global__ void __launch_bounds__(64)
k_forget(const KI* __restrict__ keys, const uint64_t* __restrict__ cnt, Lay L, const uint64_t* __restrict__ gstart,
         uint64_t G, uint32_t* gcount, const uint64_t* __restrict__ goff, KO* okeys, uint64_t* ocnt, uint32_t* ovf) {
    Acc acc = acc_bind(L.kb, EMIT);
    const int sh = L.kb + L.vb;  // drop the colour set and the last column
    const int lane = threadIdx.x;
    // 64 groups per visit: each lane reads one group's bounds, the block then
    // takes the longer ones in turn (the others are k_forget_small's), with
    // the first 64 entries of the next one loading while it works on one
    for (uint64_t g0 = uint64_t(blockIdx.x) * 64; g0 < G; g0 += uint64_t(gridDim.x) * 64) {
        const uint64_t gl = g0 + lane;
        uint64_t s0 = 0, s1 = 0, so = 0;
        if (gl < G) {
            s0 = gstart[gl];
            s1 = gstart[gl + 1];
            if (EMIT) so = goff[gl];
        }
        uint64_t todo = __ballot(s1 - s0 > uint64_t(kForgetSmall));
        // bounds of group g0 + j, from lane j
        auto bounds = [&](int j, uint64_t& e0, uint64_t& e1) {
            e0 = uint64_t(__builtin_amdgcn_readlane(uint32_t(s0), j)) |
                 (uint64_t(__builtin_amdgcn_readlane(uint32_t(s0 >> 32), j)) << 32);
            e1 = uint64_t(__builtin_amdgcn_readlane(uint32_t(s1), j)) |
                 (uint64_t(__builtin_amdgcn_readlane(uint32_t(s1 >> 32), j)) << 32);
        };
        int nj = 0;
        uint64_t n0 = 0, n1 = 0;
        KI nk = KI(0);
        uint64_t nc = 0;
        if (todo) {
            nj = __ffsll((unsigned long long)todo) - 1;
            bounds(nj, n0, n1);
            if (n0 + lane < n1) {
                nk = keys[n0 + lane];
                if (EMIT) nc = cnt[n0 + lane];
            }
        }
        while (todo) {
            const uint64_t grp = g0 + uint64_t(nj);
            const uint64_t e0 = n0, e1 = n1;
            const KI k0 = nk;
            const uint64_t c0 = nc;
            todo &= todo - 1;
            if (todo) {
                nj = __ffsll((unsigned long long)todo) - 1;
                bounds(nj, n0, n1);
                if (n0 + lane < n1) {
                    nk = keys[n0 + lane];
                    if (EMIT) nc = cnt[n0 + lane];
                }
            }
            acc_clear(acc, EMIT);
            __syncthreads();
            bool over = false;
            // every group here has more than 16 entries, so lane 0's is one
            if (e0 + lane < e1) {
                const uint32_t C = kset(k0, L);
                atomicOr(&acc.bits[C >> 5], 1u << (C & 31));
                if (EMIT) {
                    uint64_t old = atomicAdd((unsigned long long*)&acc.val[C], (unsigned long long)c0);
                    over |= (old + c0 < old);
                }
            }
            for (uint64_t e = e0 + 64 + lane; e < e1; e += 64) {
                uint32_t C = kset(keys[e], L);
                atomicOr(&acc.bits[C >> 5], 1u << (C & 31));
                if (EMIT) {
                    uint64_t c = cnt[e];
                    uint64_t old = atomicAdd((unsigned long long*)&acc.val[C], (unsigned long long)c);
                    over |= (old + c < old);
                }
            }
            __syncthreads();
            if (EMIT) {
                const KI kf = from_lane0(k0);
                if (__ballot(over) && lane == 0) atomicOr(&ovf[kbid(kf, L)], 1u);
                KO prefix = KO(shr(kf, sh)) << L.kb;
                const int j = int(grp - g0);  // the group's output offset, from lane j
                const uint64_t ob = uint64_t(__builtin_amdgcn_readlane(uint32_t(so), j)) |
                                    (uint64_t(__builtin_amdgcn_readlane(uint32_t(so >> 32), j)) << 32);
                acc_emit<KO>(acc, prefix, ob, okeys, ocnt);
            } else {
                uint32_t c = acc_count(acc);
                if (lane == 0) gcount[grp] = c;
            }
            __syncthreads();
        }
    }
}

// Runs of at most kForgetSmall entries, one per 16-lane row of a wave (one
// entry per lane): equal colour sets are found by comparing all pairs, each
// lane's values reaching the rest of its row by a DPP row broadcast, and a
// set's place in the output is the number of distinct smaller sets, so the
// output stays sorted without an accumulator.
static_assert(kForgetSmall == 16, "one run per 16-lane DPP row");

// lane I of every 16-lane row, to all lanes of that row (DPP row_newbcast);
// every lane of the wave must be active
template <int I>
__device__ __forceinline__ uint32_t row_bcast(uint32_t x) {
    return uint32_t(__builtin_amdgcn_update_dpp(0, int(x), 0x150 + I, 0xF, 0xF, false));
}

// lane I's entry against this lane's: equal sets add, and a lane is the first
// of its set when no lower lane holds it.  NW: counts are 64-bit (else every
// count of the wave is below 2^28, so sixteen of them add in 32 bits)
template <int I, bool EMIT, bool NW>
__device__ __forceinline__ void small_pairs(uint32_t mm, int sl, bool valid, uint32_t C, uint64_t c, bool& first,
                                            uint64_t& sum, bool& over) {
    if (uint32_t(I) >= mm) return;
    const uint32_t Ci = row_bcast<I>(C);
    const bool eq = valid && Ci == C;
    first = first && !(eq && I < sl);
    if (EMIT && NW) {
        const uint64_t ci = uint64_t(row_bcast<I>(uint32_t(c))) | (uint64_t(row_bcast<I>(uint32_t(c >> 32))) << 32);
        const uint64_t add = eq ? ci : 0;
        sum += add;
        over |= sum < add;
    } else if (EMIT) {
        const uint32_t ci = row_bcast<I>(uint32_t(c));
        sum = uint32_t(sum) + (eq ? ci : 0u);
    }
    if constexpr (I + 1 < kForgetSmall) small_pairs<I + 1, EMIT, NW>(mm, sl, valid, C, c, first, sum, over);
}

// number of first lanes (distinct sets) below C; F is C on first lanes and
// all ones elsewhere
template <int I>
__device__ __forceinline__ void small_rank(uint32_t mm, uint32_t F, uint32_t C, uint32_t& rank) {
    if (uint32_t(I) >= mm) return;
    rank += row_bcast<I>(F) < C ? 1u : 0u;
    if constexpr (I + 1 < kForgetSmall) small_rank<I + 1>(mm, F, C, rank);
}

// Each 16-lane row takes kForgetSmallU runs per pass and issues all their
// loads before it compares, which keeps more bytes in flight per wave.
constexpr int kForgetSmallU = 4;
template <class KI, class KO, bool EMIT>
__global__ void __launch_bounds__(kBlock)
k_forget_small(const KI* __restrict__ keys, const uint64_t* __restrict__ cnt, Lay L,
               const uint64_t* __restrict__ gstart, uint64_t G, uint32_t* gcount, const uint64_t* __restrict__ goff,
               KO* okeys, uint64_t* ocnt, uint32_t* ovf) {
    constexpr int LN = kForgetSmall, U = kForgetSmallU;
    const int sh = L.kb + L.vb;  // drop the colour set and the last column
    const int sl = threadIdx.x % LN;
    const uint64_t rows = kBlock / LN;  // runs per block and pass
    // the loop bound is uniform over the block, so every lane reaches the
    // row broadcasts
    for (uint64_t base = uint64_t(blockIdx.x) * rows * U; base < G; base += uint64_t(gridDim.x) * rows * U) {
        uint64_t e0[U], m[U], o0[U];
#pragma unroll
        for (int u = 0; u < U; u++) {
            const uint64_t grp = base + u * rows + threadIdx.x / LN;
            e0[u] = 0;
            m[u] = 0;
            o0[u] = 0;
            if (grp < G) {
                e0[u] = gstart[grp];
                m[u] = gstart[grp + 1] - e0[u];
                if (EMIT) o0[u] = goff[grp];
                if (m[u] > uint64_t(LN)) m[u] = 0;  // k_forget's run
            }
        }
        KI k[U];
        uint64_t c[U];
#pragma unroll
        for (int u = 0; u < U; u++) {
            const bool valid = uint64_t(sl) < m[u];
            k[u] = valid ? keys[e0[u] + sl] : KI(0);
            c[u] = (valid && EMIT) ? cnt[e0[u] + sl] : 0;
        }
#pragma unroll
        for (int u = 0; u < U; u++) {
            const uint64_t grp = base + u * rows + threadIdx.x / LN;
            const bool valid = uint64_t(sl) < m[u];
            const uint32_t C = valid ? kset(k[u], L) : ~0u;
            // the wave runs the longest of its four runs (m is equal on a row)
            const uint32_t m32 = uint32_t(m[u]);
            const uint32_t mm = max(max(__builtin_amdgcn_readlane(m32, 0), __builtin_amdgcn_readlane(m32, 16)),
                                    max(__builtin_amdgcn_readlane(m32, 32), __builtin_amdgcn_readlane(m32, 48)));
            bool first = valid, over = false;
            uint64_t sum = 0;
            if (!EMIT || __ballot(c[u] >> 28) == 0)
                small_pairs<0, EMIT, false>(mm, sl, valid, C, c[u], first, sum, over);
            else
                small_pairs<0, EMIT, true>(mm, sl, valid, C, c[u], first, sum, over);
            if (EMIT) {
                uint32_t rank = 0;
                small_rank<0>(mm, first ? C : ~0u, C, rank);
                if (first) {
                    const uint64_t o = o0[u] + rank;
                    okeys[o] = (KO(shr(k[u], sh)) << L.kb) | KO(C);
                    ocnt[o] = sum;
                }
                if (over) atomicOr(&ovf[kbid(k[u], L)], 1u);
            } else {
                const uint64_t fb = __ballot(first);
                if (sl == 0 && grp < G && m[u] > 0) {
                    const int base_l = int(threadIdx.x % 64) / LN * LN;
                    gcount[grp] = uint32_t(__popcll((fb >> base_l) & ((1ull << LN) - 1ull)));
                }
            }
        }
    }
}

template <bool EMIT>
static void forget_dispatch(const DevTable& in, const uint64_t* gstart, uint64_t G, uint32_t* gcount,
                            const uint64_t* goff, DevTable* out, uint32_t* ovf, hipStream_t s) {
    if (!G) return;
    Lay LO{in.lay.b - 1, in.lay.vb, in.lay.kb, in.lay.bb};
    const uint64_t visits = (G + 63) / 64;
    unsigned grid = unsigned(visits < (1u << 16) ? visits : (1u << 16));
    size_t lds = acc_bytes(in.lay.kb, EMIT);
    int ki = in.lay.kw(), ko = LO.kw();
    void* okk = out ? out->keys : nullptr;
    uint64_t* oc = out ? out->cnt : nullptr;
    // runs of 1-16 entries one per 16-lane row, longer ones k_forget
    {
        const uint64_t per = uint64_t(kBlock / kForgetSmall) * kForgetSmallU;
        const uint64_t sblocks = (G + per - 1) / per;
        const unsigned sgrid = unsigned(sblocks < (1u << 20) ? sblocks : (1u << 20));
#define FORGET_SMALL(KIT, KOT)                                                                                       \
    k_forget_small<KIT, KOT, EMIT><<<sgrid, kBlock, 0, s>>>((const KIT*)in.keys, in.cnt, in.lay, gstart, \
                                                                        G, gcount, goff, (KOT*)okk, oc, ovf)
        if (ki == 1) {
            FORGET_SMALL(uint64_t, uint64_t);
        } else if (ko == 1) {
            FORGET_SMALL(u128, uint64_t);
        } else {
            FORGET_SMALL(u128, u128);
        }
#undef FORGET_SMALL
    }
    if (ki == 1)
        k_forget<uint64_t, uint64_t, EMIT><<<grid, 64, lds, s>>>((const uint64_t*)in.keys, in.cnt, in.lay, gstart, G, gcount,
                                                                 goff, (uint64_t*)okk, oc, ovf);
    else if (ko == 1)
        k_forget<u128, uint64_t, EMIT><<<grid, 64, lds, s>>>((const u128*)in.keys, in.cnt, in.lay, gstart, G, gcount, goff,
                                                             (uint64_t*)okk, oc, ovf);
    else
        k_forget<u128, u128, EMIT><<<grid, 64, lds, s>>>((const u128*)in.keys, in.cnt, in.lay, gstart, G, gcount, goff,
                                                         (u128*)okk, oc, ovf);
}

void launch_forget_count(const DevTable& in, const uint64_t* gstart, uint64_t G, uint32_t* gcount, hipStream_t s) {
    forget_dispatch<false>(in, gstart, G, gcount, nullptr, nullptr, nullptr, s);
}
void launch_forget_emit(const DevTable& in, const uint64_t* gstart, uint64_t G, const uint64_t* goff, DevTable& out,
                        uint32_t* ovf, hipStream_t s) {
    forget_dispatch<true>(in, gstart, G, nullptr, goff, &out, ovf, s);
}

// ---------------------------------------------------------------------------
// join (Sec. 3.1 join rule): for equal (colouring, images) in both children,
// every pair with C' n C'' equal to the colour set of the bag's images gives
// C' u C'' with count c' c''; equal results add.  One 64-lane workgroup per
// run of the first child.  The matching run of the second child is found
// through a dense index over (colouring, image of column 0), narrowed by a
// binary search only when the bag has more than one column.  Colour sets and
// counts of both runs are staged in LDS in chunks and the |Y| x |Z| pair loop
// is spread over all lanes.

constexpr int kJoinChunk = 256;

template <class K>
__device__ __forceinline__ uint64_t lower_bound_prefix(const K* keys, uint64_t lo, uint64_t hi, K p, int sh, bool strict) {
    while (lo < hi) {
        uint64_t mid = (lo + hi) >> 1;
        K q = shr(keys[mid], sh);
        if (q < p || (strict && q == p)) lo = mid + 1;
        else hi = mid;
    }
    return lo;
}

template <class K, bool EMIT, int U>
__global__ void __launch_bounds__(64)
k_join(const K* __restrict__ yk, const uint64_t* __restrict__ yc, const K* __restrict__ zk,
       const uint64_t* __restrict__ zc, Lay L, const uint64_t* __restrict__ gstart, uint64_t G, int32_t n,
       const uint8_t* __restrict__ colors, const uint64_t* __restrict__ zlo, const uint64_t* __restrict__ zhi,
       uint32_t* gcount, const uint64_t* __restrict__ goff, K* okeys, uint64_t* ocnt, uint32_t* ovf) {
    // U runs per 64-lane workgroup, LN lanes each; trip counts are wave-uniform
    constexpr int LN = 64 / U;
    constexpr int CH = kJoinChunk / U;  // staged entries per run and side
    extern __shared__ uint64_t smem[];
    const int slots = 1 << L.kb;
    const int words = L.kb >= 5 ? (1 << (L.kb - 5)) : 1;
    const int lane = threadIdx.x, sub = lane / LN, sl = lane % LN;
    uint64_t* val = EMIT ? smem + size_t(sub) * slots : nullptr;
    uint32_t* bits = reinterpret_cast<uint32_t*>(smem + (EMIT ? size_t(U) * slots : 0)) + sub * words;
    __shared__ uint32_t ys[U][CH], zs[U][CH];
    __shared__ uint64_t yv[U][EMIT ? CH : 1], zv[U][EMIT ? CH : 1];
    const uint64_t subgroup_mask = (LN == 64) ? ~0ull : ((1ull << LN) - 1ull);
    const int sh = L.kb;
    for (uint64_t g0 = uint64_t(blockIdx.x) * U; g0 < G; g0 += uint64_t(gridDim.x) * U) {
        const uint64_t grp = g0 + sub;
        bool active = grp < G;
        uint64_t e0 = 0, e1 = 0, z0 = 0, z1 = 0;
        uint32_t bid = 0, bagcol = 0;
        K p = 0;
        if (active) {
            e0 = gstart[grp];
            e1 = gstart[grp + 1];
            K k0 = yk[e0];
            p = shr(k0, sh);
            bid = kbid(k0, L);
            uint64_t slot = uint64_t(bid) * uint64_t(n) + kcol(k0, L, 0);
            z0 = zlo[slot];
            z1 = zhi[slot];
            if (L.b > 1 && z0 < z1) {
                uint64_t a0 = lower_bound_prefix(zk, z0, z1, p, sh, false);
                z1 = lower_bound_prefix(zk, a0, z1, p, sh, true);
                z0 = a0;
            }
            if (z0 == z1) active = false;
            for (int j = 0; j < L.b && active; j++) bagcol |= 1u << colors[uint64_t(bid) * n + kcol(k0, L, j)];
        }
        if (!active) {
            e1 = e0;
            z1 = z0;
        }
        for (int i = sl; i < slots && EMIT; i += LN) val[i] = 0;
        for (int i = sl; i < words; i += LN) bits[i] = 0;
        bool over = false;
        // chunk loops, wave-uniform: the largest chunk counts over the U runs
        uint64_t ncy = (e1 - e0 + CH - 1) / CH, ncz = (z1 - z0 + CH - 1) / CH;
        for (int d = 32; d >= 1; d >>= 1) {
            ncy = max(ncy, (uint64_t)__shfl_xor(ncy, d, 64));
            ncz = max(ncz, (uint64_t)__shfl_xor(ncz, d, 64));
        }
        for (uint64_t cy = 0; cy < ncy; cy++) {
            uint64_t ya = e0 + cy * CH;
            uint32_t ny = ya < e1 ? uint32_t(e1 - ya < CH ? e1 - ya : CH) : 0u;
            for (uint64_t cz = 0; cz < ncz; cz++) {
                uint64_t za = z0 + cz * CH;
                uint32_t nz = za < z1 ? uint32_t(z1 - za < CH ? z1 - za : CH) : 0u;
                __syncthreads();
                for (uint32_t i = sl; i < ny; i += LN) {
                    ys[sub][i] = kset(yk[ya + i], L);
                    if (EMIT) yv[sub][i] = yc[ya + i];
                }
                for (uint32_t i = sl; i < nz; i += LN) {
                    zs[sub][i] = kset(zk[za + i], L);
                    if (EMIT) zv[sub][i] = zc[za + i];
                }
                __syncthreads();
                uint32_t P = ny * nz;
                uint32_t Pmax = P;
                for (int d = 32; d >= 1; d >>= 1) Pmax = max(Pmax, (uint32_t)__shfl_xor(Pmax, d, 64));
                // q / nz as a multiply by ceil(2^32 / nz): exact while q * nz < 2^32,
                // which holds for q < CH^2 and nz <= CH
                const uint64_t rz = nz ? ((uint64_t(1) << 32) + nz - 1) / nz : 0;
                for (uint32_t q0 = 0; q0 < Pmax; q0 += LN) {
                    uint32_t q = q0 + sl;
                    if (q >= P) continue;
                    uint32_t a = uint32_t((uint64_t(q) * rz) >> 32), d = q - a * nz;
                    uint32_t Cy = ys[sub][a], Cz = zs[sub][d];
                    if ((Cy & Cz) != bagcol) continue;
                    uint32_t C = Cy | Cz;
                    atomicOr(&bits[C >> 5], 1u << (C & 31));
                    if (EMIT) {
                        uint64_t cyv = yv[sub][a], czv = zv[sub][d];
                        uint64_t prod = cyv * czv;
                        over |= __umul64hi(cyv, czv) != 0;
                        uint64_t old = atomicAdd((unsigned long long*)&val[C], (unsigned long long)prod);
                        over |= (old + prod < old);
                    }
                }
            }
        }
        __syncthreads();
        if (EMIT) {
            uint64_t ob = __ballot(over);
            if (((ob >> (sub * LN)) & subgroup_mask) && sl == 0) atomicOr(&ovf[bid], 1u);
            uint64_t run = active ? goff[grp] : 0;
            K prefix = p << L.kb;
            for (int c0 = 0; c0 < slots; c0 += LN) {
                int C = c0 + sl;
                bool present = active && C < slots && ((bits[C >> 5] >> (C & 31)) & 1u);
                uint64_t m = (__ballot(present) >> (sub * LN)) & subgroup_mask;
                if (present) {
                    uint64_t o = run + __popcll(m & ((1ull << sl) - 1ull));
                    okeys[o] = prefix | K(C);
                    ocnt[o] = val[C];
                }
                run += __popcll(m);
            }
        } else {
            uint64_t c = 0;
            for (int i = sl; i < words; i += LN) c += __popc(bits[i]);
            for (int d = LN / 2; d >= 1; d >>= 1) c += __shfl_xor(c, d, LN);
            if (grp < G && sl == 0) gcount[grp] = active ? uint32_t(c) : 0u;
        }
        __syncthreads();
    }
}

template <bool EMIT, int U>
static void join_launch_u(const DevTable& y, const DevTable& z, const uint64_t* gstart, uint64_t G, int32_t n,
                          const uint8_t* colors, const uint64_t* zlo, const uint64_t* zhi, uint32_t* gcount,
                          const uint64_t* goff, DevTable* out, uint32_t* ovf, hipStream_t s) {
    uint64_t blocks = (G + U - 1) / U;
    unsigned grid = unsigned(blocks < (1u << 20) ? blocks : (1u << 20));
    size_t words = y.lay.kb >= 5 ? (size_t(1) << (y.lay.kb - 5)) : 1;
    size_t lds = (EMIT ? size_t(U) * (size_t(8) << y.lay.kb) : 0) + size_t(U) * 4 * words;
    void* okk = out ? out->keys : nullptr;
    uint64_t* oc = out ? out->cnt : nullptr;
    if (y.lay.kw() == 1)
        k_join<uint64_t, EMIT, U><<<grid, 64, lds, s>>>((const uint64_t*)y.keys, y.cnt, (const uint64_t*)z.keys, z.cnt,
                                                        y.lay, gstart, G, n, colors, zlo, zhi, gcount, goff,
                                                        (uint64_t*)okk, oc, ovf);
    else
        k_join<u128, EMIT, U><<<grid, 64, lds, s>>>((const u128*)y.keys, y.cnt, (const u128*)z.keys, z.cnt, y.lay, gstart,
                                                    G, n, colors, zlo, zhi, gcount, goff, (u128*)okk, oc, ovf);
}

template <bool EMIT>
static void join_dispatch(const DevTable& y, const DevTable& z, const uint64_t* gstart, uint64_t G, int32_t n,
                          const uint8_t* colors, const uint64_t* zlo, const uint64_t* zhi, uint32_t* gcount,
                          const uint64_t* goff, DevTable* out, uint32_t* ovf, hipStream_t s) {
    if (!G) return;
    // runs per workgroup from the average run length of both children
    double avg = double(y.n + z.n) / double(G);
    int kb = y.lay.kb;
    if (kb <= 9 && avg <= 96)
        join_launch_u<EMIT, 4>(y, z, gstart, G, n, colors, zlo, zhi, gcount, goff, out, ovf, s);
    else if (kb <= 11 && avg <= 256)
        join_launch_u<EMIT, 2>(y, z, gstart, G, n, colors, zlo, zhi, gcount, goff, out, ovf, s);
    else
        join_launch_u<EMIT, 1>(y, z, gstart, G, n, colors, zlo, zhi, gcount, goff, out, ovf, s);
}

void launch_join_count(const DevTable& y, const DevTable& z, const uint64_t* gstart, uint64_t G, int32_t n,
                       const uint8_t* colors, const uint64_t* zlo, const uint64_t* zhi, uint32_t* gcount, hipStream_t s) {
    join_dispatch<false>(y, z, gstart, G, n, colors, zlo, zhi, gcount, nullptr, nullptr, nullptr, s);
}
void launch_join_emit(const DevTable& y, const DevTable& z, const uint64_t* gstart, uint64_t G, int32_t n,
                      const uint8_t* colors, const uint64_t* zlo, const uint64_t* zhi, const uint64_t* goff,
                      DevTable& out, uint32_t* ovf, hipStream_t s) {
    join_dispatch<true>(y, z, gstart, G, n, colors, zlo, zhi, nullptr, goff, &out, ovf, s);
}

// ---------------------------------------------------------------------------
// column permutation + LSD radix sort (stable, 8-bit digits)

struct Perm {
    int p[4];
};

// k with its columns reordered: column j of the result is column pm.p[j] of k
template <class KI, class KO>
__device__ __forceinline__ KO permute_key(KI k, const Lay& L, const Perm& pm, const Lay& LO) {
    uint32_t cols[4];
    for (int j = 0; j < LO.b; j++) cols[j] = kcol(k, L, pm.p[j]);
    return kpack<KO>(kbid(k, L), cols, LO.b, kset(k, L), LO);
}

template <class KI, class KO>
__global__ void k_permute(const KI* __restrict__ keys, const uint64_t* __restrict__ cnt, uint64_t N, Lay L, Perm pm,
                          Lay LO, KO* okeys, uint64_t* ocnt, bool index_values) {
    for (uint64_t i = uint64_t(blockIdx.x) * blockDim.x + threadIdx.x; i < N; i += uint64_t(gridDim.x) * blockDim.x) {
        okeys[i] = permute_key<KI, KO>(keys[i], L, pm, LO);
        ocnt[i] = index_values ? i : cnt[i];
    }
}

void launch_permute(const DevTable& in, const int* perm, DevTable& out, bool index_values, hipStream_t s) {
    if (!in.n) return;
    Perm pm{{perm[0], perm[1], perm[2], perm[3]}};
    unsigned grid = grid_for(in.n);
    int ki = in.lay.kw(), ko = out.lay.kw();
    if (ki == 1 && ko == 1)
        k_permute<uint64_t, uint64_t><<<grid, kBlock, 0, s>>>((const uint64_t*)in.keys, in.cnt, in.n, in.lay, pm, out.lay,
                                                              (uint64_t*)out.keys, out.cnt, index_values);
    else if (ki == 2 && ko == 2)
        k_permute<u128, u128><<<grid, kBlock, 0, s>>>((const u128*)in.keys, in.cnt, in.n, in.lay, pm, out.lay,
                                                      (u128*)out.keys, out.cnt, index_values);
    else if (ki == 1)
        k_permute<uint64_t, u128><<<grid, kBlock, 0, s>>>((const uint64_t*)in.keys, in.cnt, in.n, in.lay, pm, out.lay,
                                                          (u128*)out.keys, out.cnt, index_values);
    else
        k_permute<u128, uint64_t><<<grid, kBlock, 0, s>>>((const u128*)in.keys, in.cnt, in.n, in.lay, pm, out.lay,
                                                          (uint64_t*)out.keys, out.cnt, index_values);
}

constexpr int kRadixItems = 16;
constexpr int kRadixTile = kBlock * kRadixItems;

// PERM: the keys are those of the table before its columns are reordered
// (L -> LO by pm), and the pass works on the reordered keys
template <class K, bool PERM>
__global__ void __launch_bounds__(kBlock) k_radix_hist(const K* __restrict__ keys, uint64_t n, int shift, uint32_t* hist,
                                                       uint64_t nblk, Lay L, Perm pm, Lay LO) {
    __shared__ uint32_t h[256];
    h[threadIdx.x] = 0;
    __syncthreads();
    uint64_t base = uint64_t(blockIdx.x) * kRadixTile;
    // all loads first, then the digits
    K k[kRadixItems];
#pragma unroll
    for (int r = 0; r < kRadixItems; r++) {
        const uint64_t i = base + uint64_t(r) * kBlock + threadIdx.x;
        k[r] = i < n ? keys[i] : K(0);
    }
#pragma unroll
    for (int r = 0; r < kRadixItems; r++) {
        const uint64_t i = base + uint64_t(r) * kBlock + threadIdx.x;
        if (i < n) {
            const K kr = PERM ? permute_key<K, K>(k[r], L, pm, LO) : k[r];
            atomicAdd(&h[uint32_t(kr >> shift) & 255u], 1u);
        }
    }
    __syncthreads();
    hist[uint64_t(threadIdx.x) * nblk + blockIdx.x] = h[threadIdx.x];
}

// Stable scatter of one tile: items are ranked in (round, wave, lane) order,
// which is their order in the input, and placed in LDS in digit order; the
// tile then leaves in that order, so the writes of one digit's run are
// contiguous (keys first, then values, through the same LDS buffer).
template <class K, bool PERM>
__global__ void __launch_bounds__(kBlock) k_radix_scatter(const K* __restrict__ keys, const uint64_t* __restrict__ vals,
                                                          uint64_t n, int shift, const uint32_t* __restrict__ hist,
                                                          const uint64_t* __restrict__ offs, uint64_t nblk, K* okeys,
                                                          uint64_t* ovals, Lay L, Perm pm, Lay LO) {
    __shared__ K s_key[kRadixTile];                 // keys, then (as 64-bit words) values, in digit order
    __shared__ uint8_t s_dig[kRadixTile];           // digit of every position
    __shared__ uint32_t s_start[256];               // tile-local start of every digit
    __shared__ uint64_t s_goff[256];                // where that digit's run goes
    __shared__ uint32_t run[256];
    __shared__ uint32_t wcnt[kBlock / 64][256];
    __shared__ uint32_t s_wtot[kBlock / 64];
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const uint64_t base = uint64_t(blockIdx.x) * kRadixTile;
    const uint32_t cnt = uint32_t(n - base < uint64_t(kRadixTile) ? n - base : uint64_t(kRadixTile));
    // exclusive scan of the tile's digit counts, one digit per thread
    const uint32_t hd = hist[uint64_t(threadIdx.x) * nblk + blockIdx.x];
    uint32_t x = hd;
    for (int o = 1; o < 64; o <<= 1) {
        const uint32_t y = __shfl_up(x, o, 64);
        if (lane >= o) x += y;
    }
    if (lane == 63) s_wtot[w] = x;
    for (int i = lane; i < 256; i += 64) wcnt[w][i] = 0;
    __syncthreads();
    uint32_t excl = x - hd;
    for (int q = 0; q < w; q++) excl += s_wtot[q];
    s_start[threadIdx.x] = excl;
    run[threadIdx.x] = excl;
    s_goff[threadIdx.x] = offs[uint64_t(threadIdx.x) * nblk + blockIdx.x];
    // every item of the thread in flight at once
    K k[kRadixItems];
    uint64_t v[kRadixItems];
#pragma unroll
    for (int r = 0; r < kRadixItems; r++) {
        const uint32_t i = uint32_t(r) * kBlock + threadIdx.x;
        k[r] = i < cnt ? keys[base + i] : K(0);
        v[r] = i < cnt ? vals[base + i] : 0;
    }
    if (PERM) {  // after all loads are issued
#pragma unroll
        for (int r = 0; r < kRadixItems; r++)
            if (uint32_t(r) * kBlock + threadIdx.x < cnt) k[r] = permute_key<K, K>(k[r], L, pm, LO);
    }
    __syncthreads();
    uint32_t pos[kRadixItems];
#pragma unroll
    for (int r = 0; r < kRadixItems; r++) {
        const bool valid = uint32_t(r) * kBlock + threadIdx.x < cnt;
        const uint32_t d = valid ? (uint32_t(k[r] >> shift) & 255u) : 0u;
        uint64_t same = __ballot(valid);
#pragma unroll
        for (int bit = 0; bit < 8; bit++) {
            const bool on = (d >> bit) & 1u;
            const uint64_t m = __ballot(on);
            same &= on ? m : ~m;
        }
        const uint32_t rank_in_wave = __popcll(same & lanemask_lt());
        if (valid && rank_in_wave == 0) wcnt[w][d] = __popcll(same);
        __syncthreads();
        pos[r] = run[d] + rank_in_wave;
        for (int q = 0; q < w; q++) pos[r] += wcnt[q][d];
        if (!valid) pos[r] = ~0u;
        __syncthreads();
        {
            uint32_t t = 0;
            for (int q = 0; q < kBlock / 64; q++) {
                t += wcnt[q][threadIdx.x];
                wcnt[q][threadIdx.x] = 0;
            }
            run[threadIdx.x] += t;
        }
        __syncthreads();  // the counters are cleared before the next round's leaders write them
    }
#pragma unroll
    for (int r = 0; r < kRadixItems; r++)
        if (pos[r] != ~0u) {
            s_key[pos[r]] = k[r];
            s_dig[pos[r]] = uint8_t(uint32_t(k[r] >> shift) & 255u);
        }
    __syncthreads();
    for (uint32_t j = threadIdx.x; j < cnt; j += kBlock) {
        const uint32_t d = s_dig[j];
        okeys[s_goff[d] + (j - s_start[d])] = s_key[j];
    }
    __syncthreads();
    uint64_t* s_val = reinterpret_cast<uint64_t*>(s_key);
#pragma unroll
    for (int r = 0; r < kRadixItems; r++)
        if (pos[r] != ~0u) s_val[pos[r]] = v[r];
    __syncthreads();
    for (uint32_t j = threadIdx.x; j < cnt; j += kBlock) {
        const uint32_t d = s_dig[j];
        ovals[s_goff[d] + (j - s_start[d])] = s_val[j];
    }
}

size_t radix_tmp_bytes(uint64_t n) {
    uint64_t nblk = (n + kRadixTile - 1) / kRadixTile;
    uint64_t h = 256 * nblk;
    return h * 4 + (h + 1) * 8 + scan_tmp_bytes(h) + 256;
}

template <class K>
static void radix_pass(bool perm, const void* src_k, const uint64_t* src_v, void* dst_k, uint64_t* dst_v, uint64_t n,
                       int shift, uint32_t* hist, uint64_t* offs, uint64_t* stmp, const Lay& L, const Perm& pm,
                       const Lay& LO, hipStream_t s) {
    const uint64_t nblk = (n + kRadixTile - 1) / kRadixTile;
    const K* sk = (const K*)src_k;
    if (perm)
        k_radix_hist<K, true><<<unsigned(nblk), kBlock, 0, s>>>(sk, n, shift, hist, nblk, L, pm, LO);
    else
        k_radix_hist<K, false><<<unsigned(nblk), kBlock, 0, s>>>(sk, n, shift, hist, nblk, L, pm, LO);
    launch_scan_u32(hist, offs, 256 * nblk, stmp, s);
    if (perm)
        k_radix_scatter<K, true><<<unsigned(nblk), kBlock, 0, s>>>(sk, src_v, n, shift, hist, offs, nblk, (K*)dst_k, dst_v,
                                                                   L, pm, LO);
    else
        k_radix_scatter<K, false><<<unsigned(nblk), kBlock, 0, s>>>(sk, src_v, n, shift, hist, offs, nblk, (K*)dst_k,
                                                                    dst_v, L, pm, LO);
}

bool radix_sort(void* keys_a, uint64_t* vals_a, void* keys_b, uint64_t* vals_b, uint64_t n, int kw, int bits, int lo,
                void* tmp, hipStream_t s, bool copy_back, const RadixSource* from) {
    const int passes = (n <= 1 || bits <= lo) ? 0 : (bits - lo + 7) / 8;
    if (from && passes == 0) {  // nothing to sort: only the reordering
        DevTable in{const_cast<void*>(from->keys), const_cast<uint64_t*>(from->vals), n, from->lay};
        DevTable out{keys_a, vals_a, n, from->lay_out};
        launch_permute(in, from->perm, out, false, s);
        return false;
    }
    if (passes == 0) return false;
    uint64_t nblk = (n + kRadixTile - 1) / kRadixTile;
    uint64_t h = 256 * nblk;
    uint32_t* hist = (uint32_t*)tmp;
    uint64_t* offs = (uint64_t*)((char*)tmp + ((h * 4 + 255) / 256) * 256);
    uint64_t* stmp = offs + h + 1;
    const Lay L = from ? from->lay : Lay{};
    const Lay LO = from ? from->lay_out : Lay{};
    const Perm pm = from ? Perm{{from->perm[0], from->perm[1], from->perm[2], from->perm[3]}} : Perm{{0, 1, 2, 3}};
    // without a source table the passes go a -> b -> a ...; with one, the
    // first reads it and writes a
    const void* src_k = from ? from->keys : keys_a;
    const uint64_t* src_v = from ? from->vals : vals_a;
    void* dst_k = from ? keys_a : keys_b;
    uint64_t* dst_v = from ? vals_a : vals_b;
    for (int p = 0; p < passes; p++) {
        const int shift = lo + 8 * p;
        const bool perm = from && p == 0;
        if (kw == 1)
            radix_pass<uint64_t>(perm, src_k, src_v, dst_k, dst_v, n, shift, hist, offs, stmp, L, pm, LO, s);
        else
            radix_pass<u128>(perm, src_k, src_v, dst_k, dst_v, n, shift, hist, offs, stmp, L, pm, LO, s);
        // the next pass reads what this one wrote and writes the other buffer
        const bool wrote_a = dst_k == keys_a;
        src_k = dst_k;
        src_v = dst_v;
        dst_k = wrote_a ? keys_b : keys_a;
        dst_v = wrote_a ? vals_b : vals_a;
    }
    if (src_k == keys_a) return false;
    if (!copy_back) return true;
    (void)hipMemcpyAsync(keys_a, src_k, n * (kw == 1 ? 8 : 16), hipMemcpyDeviceToDevice, s);
    (void)hipMemcpyAsync(vals_a, src_v, n * 8, hipMemcpyDeviceToDevice, s);
    return false;
}

// ---------------------------------------------------------------------------
// root (Sec. 3.1, last paragraph): the count of colouring b is the sum of the
// entries of the node below the root (bag {r0}) for that colouring.

template <class K>
__global__ void k_root(const K* __restrict__ keys, const uint64_t* __restrict__ cnt, uint64_t N, Lay L, int32_t n,
                       uint64_t* counts, uint32_t* ovf, uint64_t* per_vertex, uint32_t* csets, int cwords) {
    // csets: per colouring, a bitmap over colour sets of the root's entries
    // entries are sorted by colouring: every thread sums a contiguous chunk
    // and flushes one atomic per colouring it sees
    constexpr uint64_t kChunk = 32;
    uint64_t chunks = (N + kChunk - 1) / kChunk;
    for (uint64_t c = uint64_t(blockIdx.x) * blockDim.x + threadIdx.x; c < chunks; c += uint64_t(gridDim.x) * blockDim.x) {
        uint64_t i0 = c * kChunk, i1 = i0 + kChunk < N ? i0 + kChunk : N;
        uint32_t cur = kbid(keys[i0], L);
        uint64_t sum = 0;
        bool over = false;
        for (uint64_t i = i0; i < i1; i++) {
            K k = keys[i];
            uint32_t bid = kbid(k, L);
            uint64_t v = cnt[i];
            if (bid != cur) {
                uint64_t old = atomicAdd((unsigned long long*)&counts[cur], (unsigned long long)sum);
                if (over || old + sum < old) atomicOr(&ovf[cur], 1u);
                cur = bid;
                sum = 0;
                over = false;
            }
            over |= (sum + v < sum);
            sum += v;
            const uint32_t C = kset(k, L);
            uint32_t* w = &csets[uint64_t(bid) * cwords + (C >> 5)];
            if (!(__atomic_load_n(w, __ATOMIC_RELAXED) & (1u << (C & 31)))) atomicOr(w, 1u << (C & 31));
            if (per_vertex) atomicAdd((unsigned long long*)&per_vertex[uint64_t(bid) * n + kcol(k, L, 0)], (unsigned long long)v);
        }
        uint64_t old = atomicAdd((unsigned long long*)&counts[cur], (unsigned long long)sum);
        if (over || old + sum < old) atomicOr(&ovf[cur], 1u);
    }
}

void launch_root(const DevTable& in, int32_t n, uint64_t* counts, uint32_t* ovf, uint64_t* per_vertex,
                 uint32_t* csets, int cwords, hipStream_t s) {
    if (!in.n) return;
    if (in.lay.kw() == 1)
        k_root<uint64_t><<<grid_for((in.n + 31) / 32), kBlock, 0, s>>>((const uint64_t*)in.keys, in.cnt, in.n, in.lay, n,
                                                                       counts, ovf, per_vertex, csets, cwords);
    else
        k_root<u128><<<grid_for((in.n + 31) / 32), kBlock, 0, s>>>((const u128*)in.keys, in.cnt, in.n, in.lay, n, counts,
                                                                   ovf, per_vertex, csets, cwords);
}

}  // namespace ccg
