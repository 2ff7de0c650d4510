// Introduce (Sec. 3.1 introduce rule) as a load-balanced expand.
//
// The candidate pairs of an introduce node form segments: in the push form a
// segment is (prefix group of the child, one candidate image v of the new
// vertex taken from the adjacency list of the anchor's image); in the pull
// form it is (colouring b, stored edge (v, y) of G), the run of child entries
// whose column 0 is y.  An item is (segment, child entry).  A first kernel
// writes every segment's length (0 when v fails the degree mask, Sec. 3.2,
// or an adjacency check that does not depend on the entry), a scan gives the
// item offsets, and the expand kernels walk fixed tiles of 4096 items, 16
// consecutive items per thread, so a hub's long run is spread over many
// threads and blocks.  Items are tested for the colour of v (not in C) and
// the remaining adjacency checks; survivors are compacted in item order,
// which is the key order of the output.
#include <hip/hip_runtime.h>

#include "device.h"
#include "kernels.h"

namespace ccg {

constexpr int kExpItems = 16;
constexpr int kExpTile = kBlock * kExpItems;

// ---- segment lengths -------------------------------------------------------

// Tiles of kSegTile consecutive segments, kSegItems per thread: the block
// finds the tile's group range once, each thread searches only that range for
// its first segment's group and walks on from there, so consecutive segments
// of one group share its first key and anchor row.
constexpr int kSegItems = 4;
constexpr uint64_t kSegTile = uint64_t(kBlock) * kSegItems;

template <class K>
__global__ void __launch_bounds__(kBlock)
k_push_seglen(const K* __restrict__ keys, Lay L, const uint64_t* __restrict__ gstart,
              const uint64_t* __restrict__ woff, uint64_t G, uint64_t W, DevGraph g,
              const uint8_t* __restrict__ colors, IntroArgs a, uint32_t* slen) {
    __shared__ uint64_t gb[2];
    const uint64_t tiles = (W + kSegTile - 1) / kSegTile;
    for (uint64_t tile = blockIdx.x; tile < tiles; tile += gridDim.x) {
        const uint64_t s_lo = tile * kSegTile;
        const uint64_t s_hi = s_lo + kSegTile < W ? s_lo + kSegTile : W;
        if (threadIdx.x == 0) {
            gb[0] = upper_bound_u64(woff, 0, G + 1, s_lo) - 1;              // group of the first segment
            gb[1] = upper_bound_u64(woff, gb[0], G + 1, s_hi - 1);          // one past the last one's
        }
        __syncthreads();
        const uint64_t g_lo = gb[0], g_end = gb[1];
        __syncthreads();
        const uint64_t s0 = s_lo + uint64_t(threadIdx.x) * kSegItems;
        if (s0 >= s_hi) continue;
        uint64_t grp = upper_bound_u64(woff, g_lo, g_end + 1, s0) - 1;
        // the group's state: first key, candidate source column (-2: the
        // common neighbours of columns cn0 and cn1) and its list
        K k0;
        int src;
        int64_t row;
        const int32_t* cand = g.col;
        uint32_t glen;
        auto load_group = [&]() {
            const uint64_t e0 = gstart[grp];
            k0 = keys[e0];
            if (a.cn0 >= 0) {
                src = -2;
                row = a.erow[grp];
                cand = a.cn_col;
            } else {
                src = a.anchor >= 0 && a.sel ? int(a.sel[grp]) : a.anchor;
                row = src >= 0 ? g.rp[kcol(k0, L, src)] : 0;
                cand = g.col;
            }
            glen = uint32_t(gstart[grp + 1] - e0);
        };
        auto tested = [&](int c) { return c != src && c != a.cn0 && c != a.cn1; };
        load_group();
        for (int j = 0; j < kSegItems; j++) {
            const uint64_t s = s0 + uint64_t(j);
            if (s >= s_hi) break;
            if (woff[grp + 1] <= s) {
                do grp++;
                while (woff[grp + 1] <= s);
                load_group();
            }
            const uint64_t t = s - woff[grp];
            const uint32_t v = src != -1 ? uint32_t(cand[row + int64_t(t)]) : uint32_t(t);
            bool ok = intro_ok(g, v, a.degF);
            // the bag neighbours before pos other than those the candidates came from
            if (ok && tested(a.anchor)) ok = has_edge(g, kcol(k0, L, a.anchor), v);
            for (int c = 0; c < a.nchk && ok; c++)
                if ((a.grouped || a.chk[c] < a.pos) && tested(a.chk[c])) ok = has_edge(g, kcol(k0, L, a.chk[c]), v);
            slen[s] = ok ? glen : 0u;
            if (a.segv) a.segv[s] = v | uint32_t(colors[uint64_t(kbid(k0, L)) * uint32_t(g.n) + v]) << 27;
        }
    }
}

__global__ void k_pull_seglen(const uint64_t* __restrict__ rstart, const uint64_t* __restrict__ rend, int B, DevGraph g,
                              int degF, uint32_t* slen) {
    uint64_t W = uint64_t(B) * uint64_t(g.m2);
    for (uint64_t s = uint64_t(blockIdx.x) * blockDim.x + threadIdx.x; s < W; s += uint64_t(gridDim.x) * blockDim.x) {
        uint32_t bid = uint32_t(s / uint64_t(g.m2));
        uint64_t e = s % uint64_t(g.m2);
        uint32_t v = uint32_t(g.esrc[e]);
        uint64_t slot = uint64_t(bid) * uint64_t(g.n) + uint32_t(g.col[e]);
        slen[s] = intro_ok(g, v, degF) ? uint32_t(rend[slot] - rstart[slot]) : 0u;
    }
}

// ---- the expand ----------------------------------------------------------

struct SegState {
    uint32_t bid, v, cb;
    uint64_t base;  // child index of the segment's first item
};

// state of segment s; in the push form *grp is the segment's prefix group,
// advanced linearly from its previous value (segments and groups are both
// in increasing order)
template <class K, bool PULL>
__device__ __forceinline__ SegState seg_state(uint64_t s, uint64_t* grp, const K* keys, const Lay& L,
                                              const uint64_t* gstart, const uint64_t* woff, const uint64_t* rstart,
                                              const DevGraph& g, const uint8_t* colors, const IntroArgs& a) {
    SegState st;
    if (PULL) {
        st.bid = uint32_t(s / uint64_t(g.m2));
        uint64_t e = s % uint64_t(g.m2);
        st.v = uint32_t(g.esrc[e]);
        st.base = rstart[uint64_t(st.bid) * uint64_t(g.n) + uint32_t(g.col[e])];
    } else {
        while (woff[*grp + 1] <= s) (*grp)++;
        st.base = gstart[*grp];
        if (a.segv) {  // v and its colour from the seglen pass
            const uint32_t sv = a.segv[s];
            st.v = sv & ((1u << 27) - 1u);
            st.cb = 1u << (sv >> 27);
            st.bid = 0;  // not needed: an item's colouring is in its own key
            return st;
        }
        uint64_t t = s - woff[*grp];
        K k0 = keys[st.base];
        st.bid = kbid(k0, L);
        const int src = a.anchor >= 0 && a.sel ? int(a.sel[*grp]) : a.anchor;
        st.v = src >= 0 ? uint32_t(g.col[g.rp[kcol(k0, L, src)] + int64_t(t)]) : uint32_t(t);
    }
    st.cb = 1u << colors[uint64_t(st.bid) * g.n + st.v];
    return st;
}

// per tile: the first segment, one past the last, and (push form) the same
// for prefix groups; one tile per thread, so the searches run side by side
__global__ void k_expand_bounds(const uint64_t* __restrict__ soff, uint64_t S, const uint64_t* __restrict__ woff,
                                uint64_t G, uint64_t T, bool pull, uint64_t* tb) {
    const uint64_t tiles = (T + kExpTile - 1) / kExpTile;
    for (uint64_t tile = uint64_t(blockIdx.x) * blockDim.x + threadIdx.x; tile < tiles;
         tile += uint64_t(gridDim.x) * blockDim.x) {
        const uint64_t tile0 = tile * kExpTile;
        const uint64_t tile1 = tile0 + kExpTile < T ? tile0 + kExpTile : T;
        const uint64_t s_lo = upper_bound_u64(soff, 0, S + 1, tile0) - 1;
        const uint64_t s_hi = upper_bound_u64(soff, s_lo, S + 1, tile1 - 1);
        uint64_t g_lo = 0, g_hi = 0;
        if (!pull) {
            g_lo = upper_bound_u64(woff, 0, G + 1, s_lo) - 1;
            g_hi = upper_bound_u64(woff, g_lo, G + 1, s_hi - 1);
        }
        tb[4 * tile] = s_lo;
        tb[4 * tile + 1] = s_hi;
        tb[4 * tile + 2] = g_lo;
        tb[4 * tile + 3] = g_hi;
    }
}

template <class KI, class KO, bool EMIT, bool PULL>
__global__ void __launch_bounds__(kBlock)
k_expand(const KI* __restrict__ keys, const uint64_t* __restrict__ cnt, Lay L, const uint64_t* __restrict__ gstart,
         const uint64_t* __restrict__ woff, uint64_t G, const uint64_t* __restrict__ rstart,
         const uint64_t* __restrict__ soff, uint64_t S, uint64_t T, DevGraph g, const uint8_t* __restrict__ colors,
         IntroArgs a, uint32_t* tcount, const uint64_t* __restrict__ toff, KO* okeys, uint64_t* ocnt, Lay LO,
         uint64_t* osrc, uint16_t* pbits) {
    // pbits: the count pass stores every thread's survivor bits, the emit pass
    // reads them; after them, k_expand_bounds's four words per tile
    const uint64_t tiles = (T + kExpTile - 1) / kExpTile;
    const uint64_t* tbounds = reinterpret_cast<const uint64_t*>(pbits + tiles * kBlock);
    for (uint64_t tile = blockIdx.x; tile < tiles; tile += gridDim.x) {
        const uint64_t tile0 = tile * kExpTile;
        const uint64_t tile1 = tile0 + kExpTile < T ? tile0 + kExpTile : T;
        const uint64_t s_lo = tbounds[4 * tile], s_hi = tbounds[4 * tile + 1];
        const uint64_t g_lo = PULL ? 0 : tbounds[4 * tile + 2], g_hi = PULL ? 0 : tbounds[4 * tile + 3];
        const uint64_t t0 = tile0 + uint64_t(threadIdx.x) * kExpItems;
        const uint64_t t1 = t0 + kExpItems < tile1 ? t0 + kExpItems : tile1;
        uint32_t pass = 0;  // bit j: item t0 + j survives
        uint32_t n_pass = 0;
        uint64_t seg0 = 0, grp0 = g_lo;
        if (t0 < tile1 && EMIT) {
            seg0 = upper_bound_u64(soff, s_lo, s_hi + 1, t0) - 1;
            if (!PULL) grp0 = upper_bound_u64(woff, g_lo, g_hi + 1, seg0) - 1;
            pass = pbits[tile * kBlock + threadIdx.x];
            n_pass = __popc(pass);
        } else if (t0 < tile1) {
            seg0 = upper_bound_u64(soff, s_lo, s_hi + 1, t0) - 1;
            if (!PULL) grp0 = upper_bound_u64(woff, g_lo, g_hi + 1, seg0) - 1;
            uint64_t seg = seg0, grp = grp0;
            SegState st = seg_state<KI, PULL>(seg, &grp, keys, L, gstart, woff, rstart, g, colors, a);
            grp0 = grp;
            // four items per round: their key loads and edge-set probes are in
            // flight together
            for (uint64_t tb = t0; tb < t1; tb += 4) {
                uint64_t idx[4];
                uint32_t vv[4], cb4[4], ok = 0;
#pragma unroll
                for (int j = 0; j < 4; j++) {
                    const uint64_t t = tb + j;
                    idx[j] = st.base;
                    vv[j] = st.v;
                    cb4[j] = ~0u;
                    if (t < t1) {
                        if (soff[seg + 1] <= t) {
                            do seg++;
                            while (soff[seg + 1] <= t);
                            st = seg_state<KI, PULL>(seg, &grp, keys, L, gstart, woff, rstart, g, colors, a);
                        }
                        idx[j] = st.base + (t - soff[seg]);
                        vv[j] = st.v;
                        cb4[j] = st.cb;
                    }
                }
                KI kk[4];
#pragma unroll
                for (int j = 0; j < 4; j++) kk[j] = keys[idx[j]];
#pragma unroll
                for (int j = 0; j < 4; j++) ok |= uint32_t(!(kset(kk[j], L) & cb4[j])) << j;
                for (int c = 0; c < a.nchk; c++) {
                    if (!(PULL || (!a.grouped && a.chk[c] >= a.pos))) continue;
                    uint64_t key[4];
#pragma unroll
                    for (int j = 0; j < 4; j++) {
                        const uint32_t u = kcol(kk[j], L, a.chk[c]);
                        key[j] = edge_key(u, vv[j]);
                        if (u == vv[j]) ok &= ~(1u << j);
                    }
                    ok &= edges_present4(g, key, ok);
                }
                pass |= ok << (tb - t0);
                n_pass += __popc(ok);
            }
            pbits[tile * kBlock + threadIdx.x] = uint16_t(pass);
        }
        uint64_t total;
        uint64_t my = block_excl_scan(n_pass, &total);
        if (!EMIT) {
            if (threadIdx.x == 0) tcount[tile] = uint32_t(total);
            continue;
        }
        if (!pass) continue;
        uint64_t o = toff[tile] + my;
        uint64_t seg = seg0, grp = grp0;
        SegState st = seg_state<KI, PULL>(seg, &grp, keys, L, gstart, woff, rstart, g, colors, a);
        // four surviving items per round: their loads are in flight together
        uint32_t rest = pass;
        while (rest) {
            uint64_t idx[4];
            uint32_t vv[4], cb4[4];
            int nb = 0;
#pragma unroll
            for (int j = 0; j < 4; j++) {
                idx[j] = st.base;
                vv[j] = st.v;
                cb4[j] = st.cb;
                if (rest) {
                    const uint64_t t = t0 + uint64_t(__ffs(rest) - 1);
                    rest &= rest - 1u;
                    if (soff[seg + 1] <= t) {
                        do seg++;
                        while (soff[seg + 1] <= t);
                        st = seg_state<KI, PULL>(seg, &grp, keys, L, gstart, woff, rstart, g, colors, a);
                    }
                    idx[j] = st.base + (t - soff[seg]);
                    vv[j] = st.v;
                    cb4[j] = st.cb;
                    nb = j + 1;
                }
            }
            KI kk[4];
            uint64_t cv[4];
#pragma unroll
            for (int j = 0; j < 4; j++) {
                kk[j] = keys[idx[j]];
                cv[j] = cnt[idx[j]];
            }
#pragma unroll
            for (int j = 0; j < 4; j++) {
                if (j >= nb) break;
                uint32_t cols[5];
                if (PULL) {
                    cols[0] = vv[j];
                    for (int c = 1; c < LO.b; c++) cols[c] = kcol(kk[j], L, c - 1);
                } else {
                    for (int c = 0, s2 = 0; c < LO.b; c++) cols[c] = (c == a.pos) ? vv[j] : kcol(kk[j], L, s2++);
                }
                okeys[o] = kpack<KO>(kbid(kk[j], L), cols, LO.b, kset(kk[j], L) | cb4[j], LO);
                ocnt[o] = cv[j];
                if (osrc) osrc[o] = idx[j];
                o++;
            }
        }
    }
}

// the run of the pair (x, y), x < y, in the wedge index; -1: no common neighbour
__device__ __forceinline__ int64_t wedge_run(const IntroArgs& a, uint32_t x, uint32_t y) {
    const uint64_t key = (uint64_t(x) << a.wd_vb) | uint64_t(y);
    uint64_t h = edge_cell(key, a.wd_mask);
    for (;;) {
        const uint64_t k = a.wd_hk[h];
        if (k == key) return int64_t(a.wd_hv[h]);
        if (k == kEdgeEmpty) return -1;
        h = (h + 1) & a.wd_mask;
    }
}

// ---- entry-wise expand -----------------------------------------------------
//
// A segment is one child entry; its candidates for the new vertex are the
// adjacency list of the image of whichever bag neighbour of u has the fewest
// neighbours for that entry, and each other bag neighbour is an edge test.
// The push and pull forms above draw candidates from one fixed column, which
// on heavy-tailed graphs walks a hub's whole row for every entry holding the
// hub even when another bag neighbour of u maps to a vertex of degree 5.
// Items come out in (entry, candidate) order with v at column pos; the
// caller restores key order with a stable sort on (colouring, columns
// 0..pos): entries are in key order and within one entry the candidates
// ascend, so equal (colouring, columns 0..pos) keep (later columns, colour
// set) order.

// also adds up, into *anchor_items, the candidates the fixed-column forms
// would walk (the anchor's degree per entry), so the caller can pick a form
template <class K>
__global__ void __launch_bounds__(kBlock)
k_entry_seglen(const K* __restrict__ keys, Lay L, uint64_t N, uint64_t stride, DevGraph g, IntroArgs a, uint32_t* slen,
               uint8_t* src, unsigned long long* sums) {
    // stride > 1: a sample (every stride-th entry), sums only
    uint64_t mine = 0, items = 0;
    const uint64_t M = (N + stride - 1) / stride;
    for (uint64_t j = uint64_t(blockIdx.x) * blockDim.x + threadIdx.x; j < M; j += uint64_t(gridDim.x) * blockDim.x) {
        const uint64_t e = j * stride;
        const K k = keys[e];
        int best = a.anchor;
        int64_t bd = gdeg(g, kcol(k, L, a.anchor));
        mine += uint64_t(bd);
        if (a.cn0 >= 0) {  // the common neighbours of two adjacent bag images
            const int64_t ei = edge_index(g, kcol(k, L, a.cn0), kcol(k, L, a.cn1));
            const uint64_t c0 = ei >= 0 ? a.cn_off[ei] : 0, c1 = ei >= 0 ? a.cn_off[ei + 1] : 0;
            items += c1 - c0;
            if (stride == 1) {
                slen[e] = uint32_t(c1 - c0);
                src[e] = uint8_t(0x80 | (a.cn0 << 3) | a.cn1);
                a.erow[e] = int64_t(c0);
            }
            continue;
        }
        if (a.wd0 >= 0) {  // the common neighbours of two non-adjacent bag images
            uint32_t x = kcol(k, L, a.wd0), y = kcol(k, L, a.wd1);
            if (x > y) {
                const uint32_t t = x;
                x = y;
                y = t;
            }
            const int64_t r = wedge_run(a, x, y);
            const uint64_t c0 = r >= 0 ? a.wd_start[r] : 0, c1 = r >= 0 ? a.wd_start[r + 1] : 0;
            items += c1 - c0;
            if (stride == 1) {
                slen[e] = uint32_t(c1 - c0);
                src[e] = uint8_t(0xC0 | (a.wd0 << 3) | a.wd1);
                a.erow[e] = int64_t(c0);
            }
            continue;
        }
        for (int c = 0; c < a.nchk; c++) {
            const int64_t d = gdeg(g, kcol(k, L, a.chk[c]));
            if (d < bd) {
                bd = d;
                best = a.chk[c];
            }
        }
        items += uint64_t(bd);
        if (stride == 1) {
            slen[e] = uint32_t(bd);
            src[e] = uint8_t(best);
        }
    }
    uint64_t total;
    (void)block_excl_scan(mine, &total);
    if (threadIdx.x == 0 && total) atomicAdd(&sums[0], (unsigned long long)total);
    (void)block_excl_scan(items, &total);
    if (threadIdx.x == 0 && total) atomicAdd(&sums[1], (unsigned long long)total);
}

template <class KI, class KO, bool EMIT>
__global__ void __launch_bounds__(kBlock)
k_expand_entry(const KI* __restrict__ keys, const uint64_t* __restrict__ cnt, Lay L, const uint8_t* __restrict__ src,
               const uint64_t* __restrict__ soff, uint64_t S, uint64_t T, DevGraph g,
               const uint8_t* __restrict__ colors, IntroArgs a, uint32_t* tcount, const uint64_t* __restrict__ toff,
               KO* okeys, uint64_t* ocnt, Lay LO, uint16_t* pbits) {
    const uint64_t tiles = (T + kExpTile - 1) / kExpTile;
    const uint64_t* tbounds = reinterpret_cast<const uint64_t*>(pbits + tiles * kBlock);
    // the bag neighbours of u (child columns): the anchor, then the checks
    int nb[5];
    int nnb = 0;
    nb[nnb++] = a.anchor;
    for (int c = 0; c < a.nchk; c++) nb[nnb++] = a.chk[c];
    for (uint64_t tile = blockIdx.x; tile < tiles; tile += gridDim.x) {
        const uint64_t tile0 = tile * kExpTile;
        const uint64_t tile1 = tile0 + kExpTile < T ? tile0 + kExpTile : T;
        const uint64_t s_lo = tbounds[4 * tile], s_hi = tbounds[4 * tile + 1];
        const uint64_t t0 = tile0 + uint64_t(threadIdx.x) * kExpItems;
        const uint64_t t1 = t0 + kExpItems < tile1 ? t0 + kExpItems : tile1;
        uint32_t pass = 0;
        uint32_t n_pass = 0;
        uint64_t seg0 = 0;
        if (t0 < tile1) seg0 = upper_bound_u64(soff, s_lo, s_hi + 1, t0) - 1;
        // the segment's entry: key, candidate list, colouring, colour set;
        // source byte sc: the column whose adjacency list gives the
        // candidates, or 0x80 | c0 << 3 | c1 for the common neighbours of
        // columns c0 and c1 (with 0x40: from the wedge index, the columns'
        // vertices not adjacent in F)
        uint64_t seg = seg0;
        KI key{};
        int64_t row = 0;
        const int32_t* cand = g.col;
        uint32_t sc = 0;
        auto load_seg = [&]() {
            key = keys[seg];
            sc = src[seg];
            if (sc & 0x80u) {
                row = a.erow[seg];
                cand = (sc & 0x40u) ? a.wd_mid : a.cn_col;
            } else {
                row = g.rp[kcol(key, L, int(sc))];
                cand = g.col;
            }
        };
        // bag neighbour column nb needs no edge test: it gave the candidates
        auto is_source = [](uint32_t s_, int nbc) {
            return (s_ & 0x80u) ? (uint32_t(nbc) == ((s_ >> 3) & 7u) || uint32_t(nbc) == (s_ & 7u)) : uint32_t(nbc) == s_;
        };
        if (t0 < tile1) load_seg();
        if (EMIT) {
            if (t0 < tile1) {
                pass = pbits[tile * kBlock + threadIdx.x];
                n_pass = __popc(pass);
            }
        } else if (t0 < tile1) {
            for (uint64_t tb = t0; tb < t1; tb += 4) {
                uint32_t vv[4], scj[4], ok = 0;
                KI kk[4];
#pragma unroll
                for (int j = 0; j < 4; j++) {
                    const uint64_t t = tb + j;
                    vv[j] = 0;
                    kk[j] = key;
                    scj[j] = sc;
                    if (t < t1) {
                        if (soff[seg + 1] <= t) {
                            do seg++;
                            while (soff[seg + 1] <= t);
                            load_seg();
                        }
                        vv[j] = uint32_t(cand[row + int64_t(t - soff[seg])]);
                        kk[j] = key;
                        scj[j] = sc;
                        ok |= 1u << j;
                    }
                }
                // the colour of v not yet used, the degree mask and the image range
#pragma unroll
                for (int j = 0; j < 4; j++) {
                    if (!((ok >> j) & 1u)) continue;
                    const uint32_t cb = 1u << colors[uint64_t(kbid(kk[j], L)) * uint32_t(g.n) + vv[j]];
                    if ((kset(kk[j], L) & cb) || !intro_ok(g, vv[j], a.degF)) ok &= ~(1u << j);
                }
                // every bag neighbour other than the candidates' source is
                // adjacent (the source is, by construction)
                for (int c = 0; c < nnb; c++) {
                    uint64_t ek[4];
                    uint32_t probe = 0;
#pragma unroll
                    for (int j = 0; j < 4; j++) {
                        const uint32_t w = kcol(kk[j], L, nb[c]);
                        ek[j] = edge_key(w, vv[j]);
                        if (w == vv[j]) ok &= ~(1u << j);
                        if (((ok >> j) & 1u) && !is_source(scj[j], nb[c])) probe |= 1u << j;
                    }
                    ok &= ~probe | edges_present4(g, ek, probe);
                }
                pass |= ok << (tb - t0);
                n_pass += __popc(ok);
            }
            pbits[tile * kBlock + threadIdx.x] = uint16_t(pass);
        }
        uint64_t total;
        uint64_t my = block_excl_scan(n_pass, &total);
        if (!EMIT) {
            if (threadIdx.x == 0) tcount[tile] = uint32_t(total);
            continue;
        }
        if (!pass) continue;
        uint64_t o = toff[tile] + my;
        seg = seg0;
        load_seg();
        uint32_t rest = pass;
        while (rest) {
            const uint64_t t = t0 + uint64_t(__ffs(rest) - 1);
            rest &= rest - 1u;
            if (soff[seg + 1] <= t) {
                do seg++;
                while (soff[seg + 1] <= t);
                load_seg();
            }
            const uint32_t v = uint32_t(cand[row + int64_t(t - soff[seg])]);
            const uint32_t bid = kbid(key, L);
            uint32_t cols[5];
            for (int c = 0, s2 = 0; c < LO.b; c++) cols[c] = (c == a.pos) ? v : kcol(key, L, s2++);
            okeys[o] = kpack<KO>(bid, cols, LO.b, kset(key, L) | (1u << colors[uint64_t(bid) * uint32_t(g.n) + v]), LO);
            ocnt[o] = cnt[seg];
            o++;
        }
    }
}

// ---- common-neighbour index ---------------------------------------------------
//
// For every stored edge e = (a, b): the common neighbours of a and b in
// increasing order, found by walking the shorter row and searching each of
// its vertices in the longer one from the last position found (both rows
// ascend).  An introduced vertex adjacent in F to two bag vertices that are
// adjacent to each other has exactly these candidates (Sec. 3.2: every bag
// neighbour's image must be adjacent to the candidate).

template <bool EMIT>
__global__ void k_cn(DevGraph g, uint32_t* cnt, const uint64_t* __restrict__ off, int32_t* out) {
    for (uint64_t e = uint64_t(blockIdx.x) * blockDim.x + threadIdx.x; e < uint64_t(g.m2);
         e += uint64_t(gridDim.x) * blockDim.x) {
        const uint32_t a = uint32_t(g.esrc[e]), b = uint32_t(g.col[e]);
        int64_t ia = g.rp[a], ea = g.rp[a + 1], ib = g.rp[b], eb = g.rp[b + 1];
        if (ea - ia > eb - ib) {
            const int64_t t0 = ia, t1 = ea;
            ia = ib;
            ea = eb;
            ib = t0;
            eb = t1;
        }
        uint32_t c = 0;
        const uint64_t o = EMIT ? off[e] : 0;
        int64_t p = ib;
        for (int64_t i = ia; i < ea && p < eb; i++) {
            const uint32_t x = uint32_t(g.col[i]);
            int64_t hi = eb;
            while (p < hi) {
                const int64_t mid = (p + hi) >> 1;
                if (uint32_t(g.col[mid]) < x)
                    p = mid + 1;
                else
                    hi = mid;
            }
            if (p < eb && uint32_t(g.col[p]) == x) {
                if (EMIT) out[o + c] = int32_t(x);
                c++;
                p++;
            }
        }
        if (!EMIT) cnt[e] = c;
    }
}

// ---- wedge index ---------------------------------------------------------------
//
// Two bag neighbours a, b of an introduced vertex u that are not adjacent in
// F: u's candidates are the common neighbours of phi(a) and phi(b), vertices
// at distance 2 or less of each other in G.  For every vertex w and every
// pair x < y of its neighbours (rows ascend, so a stored edge (w, x) at row
// position i pairs with the positions after i) a record (x << vb | y, w);
// sorted, one pair's records are its common neighbours; an open-addressing
// hash of the pairs gives a pair's run.

__global__ void k_wedge_count(DevGraph g, uint32_t* cnt) {
    for (uint64_t e = uint64_t(blockIdx.x) * blockDim.x + threadIdx.x; e < uint64_t(g.m2);
         e += uint64_t(gridDim.x) * blockDim.x) {
        const uint32_t w = uint32_t(g.esrc[e]);
        const int64_t r0 = g.rp[w], d = g.rp[w + 1] - r0, i = int64_t(e) - r0;
        cnt[e] = uint32_t(d - 1 - i);
    }
}

__global__ void k_wedge_emit(DevGraph g, int vb, const uint64_t* __restrict__ off, uint64_t* keys, uint64_t* vals) {
    for (uint64_t e = uint64_t(blockIdx.x) * blockDim.x + threadIdx.x; e < uint64_t(g.m2);
         e += uint64_t(gridDim.x) * blockDim.x) {
        const uint32_t w = uint32_t(g.esrc[e]);
        const int64_t r1 = g.rp[w + 1];
        const uint64_t x = uint64_t(uint32_t(g.col[e]));
        uint64_t o = off[e];
        for (int64_t j = int64_t(e) + 1; j < r1; j++, o++) {
            keys[o] = (x << vb) | uint64_t(uint32_t(g.col[j]));
            vals[o] = w;
        }
    }
}

__global__ void k_wedge_hash(const uint64_t* __restrict__ keys, const uint64_t* __restrict__ starts, uint64_t G,
                             unsigned long long* hk, uint32_t* hv, uint64_t mask) {
    for (uint64_t r = uint64_t(blockIdx.x) * blockDim.x + threadIdx.x; r < G; r += uint64_t(gridDim.x) * blockDim.x) {
        const uint64_t key = keys[starts[r]];
        uint64_t h = edge_cell(key, mask);
        // the keys are distinct and the table has at least twice as many
        // cells: every insertion finds a free cell
        for (;;) {
            const unsigned long long old = atomicCAS(&hk[h], (unsigned long long)kEdgeEmpty, (unsigned long long)key);
            if (old == (unsigned long long)kEdgeEmpty) {
                hv[h] = uint32_t(r);
                break;
            }
            h = (h + 1) & mask;
        }
    }
}

__global__ void k_u64_to_i32(const uint64_t* __restrict__ in, int32_t* out, uint64_t n) {
    for (uint64_t i = uint64_t(blockIdx.x) * blockDim.x + threadIdx.x; i < n; i += uint64_t(gridDim.x) * blockDim.x)
        out[i] = int32_t(in[i]);
}

void launch_wedge_count(DevGraph g, uint32_t* cnt, hipStream_t s) {
    if (g.m2) k_wedge_count<<<grid_for(uint64_t(g.m2)), kBlock, 0, s>>>(g, cnt);
}

void launch_wedge_emit(DevGraph g, int vb, const uint64_t* off, uint64_t* keys, uint64_t* vals, hipStream_t s) {
    if (g.m2) k_wedge_emit<<<grid_for(uint64_t(g.m2)), kBlock, 0, s>>>(g, vb, off, keys, vals);
}

void launch_wedge_hash(const uint64_t* keys, const uint64_t* starts, uint64_t G, uint64_t* hk, uint32_t* hv,
                       uint64_t mask, hipStream_t s) {
    if (G)
        k_wedge_hash<<<grid_for(G), kBlock, 0, s>>>(keys, starts, G, reinterpret_cast<unsigned long long*>(hk), hv,
                                                     mask);
}

void launch_u64_to_i32(const uint64_t* in, int32_t* out, uint64_t n, hipStream_t s) {
    if (n) k_u64_to_i32<<<grid_for(n), kBlock, 0, s>>>(in, out, n);
}

void launch_cn_count(DevGraph g, uint32_t* cnt, hipStream_t s) {
    if (g.m2) k_cn<false><<<grid_for(uint64_t(g.m2)), kBlock, 0, s>>>(g, cnt, nullptr, nullptr);
}

void launch_cn_emit(DevGraph g, const uint64_t* off, int32_t* out, hipStream_t s) {
    if (g.m2) k_cn<true><<<grid_for(uint64_t(g.m2)), kBlock, 0, s>>>(g, nullptr, off, out);
}

// ---- distance-bounded introduce (no bag neighbour) ----------------------------
//
// Sec. 3.2, last paragraphs of "Mapping Expansion Optimizations": a vertex u
// with no neighbour in the bag, at distance r = dist_F(w, u) from a bag
// vertex w, can only map to a vertex within distance r of phi(w) in G.  For
// r = 2 the candidates of an entry are the ends of the walks of length 1 and
// 2 from a = phi(w): deg(a) + sum over x in N(a) of deg(x) items, the
// second level addressed through per-edge prefix sums of the neighbours'
// degrees (nbpre[e] for stored edge e = (a, col[e]): the degrees of the
// earlier neighbours in a's row).  A vertex reached by several walks is
// emitted several times: the caller sorts the output and keeps one entry of
// each key (equal keys come from the same child entry and carry its count).

__global__ void k_nbdeg_prefix(DevGraph g, uint64_t* nbpre, uint64_t* w2) {
    for (uint64_t v = uint64_t(blockIdx.x) * blockDim.x + threadIdx.x; v < uint64_t(g.n);
         v += uint64_t(gridDim.x) * blockDim.x) {
        uint64_t acc = 0;
        for (int64_t e = g.rp[v]; e < g.rp[v + 1]; e++) {
            nbpre[e] = acc;
            acc += uint64_t(gdeg(g, uint32_t(g.col[e])));
        }
        w2[v] = uint64_t(gdeg(g, uint32_t(v))) + acc;
    }
}

void launch_nbdeg_prefix(DevGraph g, uint64_t* nbpre, uint64_t* w2, hipStream_t s) {
    if (g.n) k_nbdeg_prefix<<<grid_for(uint64_t(g.n)), kBlock, 0, s>>>(g, nbpre, w2);
}

template <class K>
__global__ void k_ball_seglen(const K* __restrict__ keys, Lay L, uint64_t N, int col, const uint64_t* __restrict__ w2,
                              uint32_t* slen) {
    for (uint64_t e = uint64_t(blockIdx.x) * blockDim.x + threadIdx.x; e < N; e += uint64_t(gridDim.x) * blockDim.x) {
        const uint64_t len = w2[kcol(keys[e], L, col)];
        slen[e] = uint32_t(len < 0xffffffffull ? len : 0xffffffffull);
    }
}

// the walk end of item t (< deg(a) + sum deg) from a
__device__ __forceinline__ uint32_t ball_vertex(const DevGraph& g, const uint64_t* nbpre, uint32_t a, uint64_t t) {
    const int64_t r0 = g.rp[a], r1 = g.rp[a + 1];
    const uint64_t d = uint64_t(r1 - r0);
    if (t < d) return uint32_t(g.col[r0 + int64_t(t)]);
    const uint64_t u = t - d;
    // last neighbour x of a (row position i) with nbpre[r0 + i] <= u
    int64_t lo = r0, hi = r1;
    while (hi - lo > 1) {
        const int64_t mid = (lo + hi) >> 1;
        if (nbpre[mid] <= u) lo = mid;
        else hi = mid;
    }
    const uint32_t x = uint32_t(g.col[lo]);
    return uint32_t(g.col[g.rp[x] + int64_t(u - nbpre[lo])]);
}

template <class KI, class KO, bool EMIT>
__global__ void __launch_bounds__(kBlock)
k_expand_ball(const KI* __restrict__ keys, const uint64_t* __restrict__ cnt, Lay L, int col,
              const uint64_t* __restrict__ nbpre, const uint64_t* __restrict__ soff, uint64_t T, DevGraph g,
              const uint8_t* __restrict__ colors, IntroArgs a, uint32_t* tcount, const uint64_t* __restrict__ toff,
              KO* okeys, uint64_t* ocnt, Lay LO, uint16_t* pbits) {
    const uint64_t tiles = (T + kExpTile - 1) / kExpTile;
    const uint64_t* tbounds = reinterpret_cast<const uint64_t*>(pbits + tiles * kBlock);
    for (uint64_t tile = blockIdx.x; tile < tiles; tile += gridDim.x) {
        const uint64_t tile0 = tile * kExpTile;
        const uint64_t tile1 = tile0 + kExpTile < T ? tile0 + kExpTile : T;
        const uint64_t s_lo = tbounds[4 * tile], s_hi = tbounds[4 * tile + 1];
        const uint64_t t0 = tile0 + uint64_t(threadIdx.x) * kExpItems;
        const uint64_t t1 = t0 + kExpItems < tile1 ? t0 + kExpItems : tile1;
        uint32_t pass = 0, n_pass = 0;
        uint64_t seg = 0;
        if (t0 < tile1) seg = upper_bound_u64(soff, s_lo, s_hi + 1, t0) - 1;
        const uint64_t seg0 = seg;
        KI key{};
        uint32_t img = 0;
        if (t0 < tile1) {
            key = keys[seg];
            img = kcol(key, L, col);
        }
        if (EMIT) {
            if (t0 < tile1) {
                pass = pbits[tile * kBlock + threadIdx.x];
                n_pass = __popc(pass);
            }
        } else {
            for (uint64_t t = t0; t < t1; t++) {
                if (soff[seg + 1] <= t) {
                    do seg++;
                    while (soff[seg + 1] <= t);
                    key = keys[seg];
                    img = kcol(key, L, col);
                }
                const uint32_t v = ball_vertex(g, nbpre, img, t - soff[seg]);
                const uint32_t cb = 1u << colors[uint64_t(kbid(key, L)) * uint32_t(g.n) + v];
                if (!(kset(key, L) & cb) && intro_ok(g, v, a.degF)) {
                    pass |= 1u << (t - t0);
                    n_pass++;
                }
            }
            if (t0 < tile1) pbits[tile * kBlock + threadIdx.x] = uint16_t(pass);
        }
        uint64_t total;
        const uint64_t my = block_excl_scan(n_pass, &total);
        if (!EMIT) {
            if (threadIdx.x == 0) tcount[tile] = uint32_t(total);
            continue;
        }
        if (!pass) continue;
        uint64_t o = toff[tile] + my;
        seg = seg0;
        key = keys[seg];
        img = kcol(key, L, col);
        uint32_t rest = pass;
        while (rest) {
            const uint64_t t = t0 + uint64_t(__ffs(rest) - 1);
            rest &= rest - 1u;
            if (soff[seg + 1] <= t) {
                do seg++;
                while (soff[seg + 1] <= t);
                key = keys[seg];
                img = kcol(key, L, col);
            }
            const uint32_t v = ball_vertex(g, nbpre, img, t - soff[seg]);
            const uint32_t bid = kbid(key, L);
            uint32_t cols[5];
            for (int c = 0, s2 = 0; c < LO.b; c++) cols[c] = (c == a.pos) ? v : kcol(key, L, s2++);
            okeys[o] = kpack<KO>(bid, cols, LO.b, kset(key, L) | (1u << colors[uint64_t(bid) * uint32_t(g.n) + v]), LO);
            ocnt[o] = cnt[seg];
            o++;
        }
    }
}

// keeps the first entry of every run of equal keys (starts[G + 1] from the
// run-start pass with shift 0)
template <class K>
__global__ void k_take_runs(const K* __restrict__ keys, const uint64_t* __restrict__ cnt,
                            const uint64_t* __restrict__ starts, uint64_t G, K* okeys, uint64_t* ocnt) {
    for (uint64_t i = uint64_t(blockIdx.x) * blockDim.x + threadIdx.x; i < G; i += uint64_t(gridDim.x) * blockDim.x) {
        okeys[i] = keys[starts[i]];
        ocnt[i] = cnt[starts[i]];
    }
}

void launch_ball_seglen(const DevTable& in, int col, const uint64_t* w2, uint32_t* slen, hipStream_t s) {
    if (!in.n) return;
    if (in.lay.kw() == 1)
        k_ball_seglen<uint64_t><<<grid_for(in.n), kBlock, 0, s>>>((const uint64_t*)in.keys, in.lay, in.n, col, w2, slen);
    else
        k_ball_seglen<u128><<<grid_for(in.n), kBlock, 0, s>>>((const u128*)in.keys, in.lay, in.n, col, w2, slen);
}

template <bool EMIT>
static void ball_dispatch(const DevTable& in, int col, const uint64_t* nbpre, const uint64_t* soff, uint64_t T,
                          DevGraph g, const uint8_t* colors, const IntroArgs& a, uint32_t* tcount,
                          const uint64_t* toff, DevTable* out, uint16_t* pbits, hipStream_t s) {
    const uint64_t tiles = expand_tiles(T);
    if (!tiles) return;
    const unsigned grid = unsigned(tiles < (1u << 20) ? tiles : (1u << 20));
    Lay LO = out ? out->lay : Lay{in.lay.b + 1, in.lay.vb, in.lay.kb, in.lay.bb};
    void* ok = out ? out->keys : nullptr;
    uint64_t* oc = out ? out->cnt : nullptr;
    const int ki = in.lay.kw(), ko = LO.kw();
    if (ki == 1 && ko == 1)
        k_expand_ball<uint64_t, uint64_t, EMIT><<<grid, kBlock, 0, s>>>((const uint64_t*)in.keys, in.cnt, in.lay, col,
                                                                        nbpre, soff, T, g, colors, a, tcount, toff,
                                                                        (uint64_t*)ok, oc, LO, pbits);
    else if (ki == 1)
        k_expand_ball<uint64_t, u128, EMIT><<<grid, kBlock, 0, s>>>((const uint64_t*)in.keys, in.cnt, in.lay, col, nbpre,
                                                                    soff, T, g, colors, a, tcount, toff, (u128*)ok, oc,
                                                                    LO, pbits);
    else
        k_expand_ball<u128, u128, EMIT><<<grid, kBlock, 0, s>>>((const u128*)in.keys, in.cnt, in.lay, col, nbpre, soff, T,
                                                                g, colors, a, tcount, toff, (u128*)ok, oc, LO, pbits);
}

void launch_ball_count(const DevTable& in, int col, const uint64_t* nbpre, const uint64_t* soff, uint64_t T, DevGraph g,
                       const uint8_t* colors, const IntroArgs& a, uint32_t* tcount, uint16_t* pbits, hipStream_t s) {
    const uint64_t tiles = expand_tiles(T);
    if (!tiles) return;
    k_expand_bounds<<<grid_for(tiles), kBlock, 0, s>>>(soff, in.n, nullptr, 0, T, true,
                                                      reinterpret_cast<uint64_t*>(pbits + tiles * kBlock));
    ball_dispatch<false>(in, col, nbpre, soff, T, g, colors, a, tcount, nullptr, nullptr, pbits, s);
}

void launch_ball_emit(const DevTable& in, int col, const uint64_t* nbpre, const uint64_t* soff, uint64_t T, DevGraph g,
                      const uint8_t* colors, const IntroArgs& a, const uint64_t* toff, const uint16_t* pbits,
                      DevTable& out, hipStream_t s) {
    ball_dispatch<true>(in, col, nbpre, soff, T, g, colors, a, nullptr, toff, &out, const_cast<uint16_t*>(pbits), s);
}

void launch_take_runs(const DevTable& in, const uint64_t* starts, uint64_t G, DevTable& out, hipStream_t s) {
    if (!G) return;
    if (in.lay.kw() == 1)
        k_take_runs<uint64_t><<<grid_for(G), kBlock, 0, s>>>((const uint64_t*)in.keys, in.cnt, starts, G,
                                                             (uint64_t*)out.keys, out.cnt);
    else
        k_take_runs<u128><<<grid_for(G), kBlock, 0, s>>>((const u128*)in.keys, in.cnt, starts, G, (u128*)out.keys,
                                                         out.cnt);
}

// ---- forget by sorting (colour sets wider than the dense accumulators) ------
//
// Forget u (Sec. 3.1) without a 2^k accumulator: every entry's key loses its
// last column, the keys are sorted (stable radix), and each run of equal keys
// becomes one entry whose count is the run's sum mod 2^64; a carry sets the
// colouring's overflow flag.

template <class KI, class KO>
__global__ void k_drop_last(const KI* __restrict__ keys, uint64_t N, Lay L, Lay LO, KO* okeys) {
    for (uint64_t i = uint64_t(blockIdx.x) * blockDim.x + threadIdx.x; i < N; i += uint64_t(gridDim.x) * blockDim.x) {
        const KI k = keys[i];
        uint32_t cols[4];
        for (int c = 0; c < LO.b; c++) cols[c] = kcol(k, L, c);
        okeys[i] = kpack<KO>(kbid(k, L), cols, LO.b, kset(k, L), LO);
    }
}

template <class K>
__global__ void k_reduce_runs(const K* __restrict__ keys, const uint64_t* __restrict__ cnt,
                              const uint64_t* __restrict__ starts, uint64_t G, Lay L, K* okeys, uint64_t* ocnt,
                              uint32_t* ovf) {
    for (uint64_t i = uint64_t(blockIdx.x) * blockDim.x + threadIdx.x; i < G; i += uint64_t(gridDim.x) * blockDim.x) {
        const uint64_t a = starts[i], b = starts[i + 1];
        uint64_t sum = 0;
        bool over = false;
        for (uint64_t j = a; j < b; j++) {
            const uint64_t v = cnt[j];
            over |= sum + v < sum;
            sum += v;
        }
        okeys[i] = keys[a];
        ocnt[i] = sum;
        if (over) atomicOr(&ovf[kbid(keys[a], L)], 1u);
    }
}

// Join (Sec. 3.1) without a 2^k accumulator: one thread per entry of y finds
// the run of z with the same (colouring, bag images) by binary search and
// pairs its colour set with every colour set there whose intersection is
// exactly the colours of the bag's images; the products (mod 2^64, a carry
// beyond 64 bits sets the colouring's flag) are emitted unreduced, in no
// order: the caller sorts them and adds up runs of equal keys.
template <class K>
__device__ __forceinline__ uint64_t key_lower_bound(const K* keys, uint64_t n, K prefix, int sh) {
    uint64_t lo = 0, hi = n;
    while (lo < hi) {
        const uint64_t mid = (lo + hi) >> 1;
        if (shr(keys[mid], sh) < prefix) lo = mid + 1;
        else hi = mid;
    }
    return lo;
}

template <class K, bool EMIT>
__global__ void k_join_pairs(const K* __restrict__ ykeys, const uint64_t* __restrict__ ycnt, uint64_t ny,
                             const K* __restrict__ zkeys, const uint64_t* __restrict__ zcnt, uint64_t nz, Lay L,
                             int32_t n, const uint8_t* __restrict__ colors, uint32_t* pcount,
                             const uint64_t* __restrict__ poff, K* okeys, uint64_t* ocnt, uint32_t* ovf) {
    const int sh = L.kb;
    const K cmask = (K(1) << L.kb) - K(1);
    for (uint64_t e = uint64_t(blockIdx.x) * blockDim.x + threadIdx.x; e < ny; e += uint64_t(gridDim.x) * blockDim.x) {
        const K ky = ykeys[e];
        const K prefix = shr(ky, sh);
        const uint32_t bid = kbid(ky, L);
        uint32_t bag = 0;
        for (int c = 0; c < L.b; c++) bag |= 1u << colors[uint64_t(bid) * uint32_t(n) + kcol(ky, L, c)];
        const uint32_t cy = kset(ky, L);
        uint64_t j = key_lower_bound(zkeys, nz, prefix, sh);
        uint32_t m = 0;
        uint64_t o = EMIT ? poff[e] : 0;
        bool over = false;
        for (; j < nz; j++) {
            const K kz = zkeys[j];
            if (shr(kz, sh) != prefix) break;
            const uint32_t cz = kset(kz, L);
            if ((cy & cz) != bag) continue;
            if (EMIT) {
                const uint64_t a = ycnt[e], b = zcnt[j];
                over |= __umul64hi(a, b) != 0;
                okeys[o] = (ky & ~cmask) | K(cy | cz);
                ocnt[o] = a * b;
                o++;
            } else {
                m++;
            }
        }
        if (!EMIT) pcount[e] = m;
        if (EMIT && over) atomicOr(&ovf[bid], 1u);
    }
}

void launch_join_pairs(const DevTable& y, const DevTable& z, int32_t n, const uint8_t* colors, uint32_t* pcount,
                       const uint64_t* poff, DevTable* out, uint32_t* ovf, hipStream_t s) {
    if (!y.n || !z.n) return;
    const unsigned grid = grid_for(y.n);
    if (y.lay.kw() == 1) {
        if (out)
            k_join_pairs<uint64_t, true><<<grid, kBlock, 0, s>>>((const uint64_t*)y.keys, y.cnt, y.n,
                                                                 (const uint64_t*)z.keys, z.cnt, z.n, y.lay, n, colors,
                                                                 nullptr, poff, (uint64_t*)out->keys, out->cnt, ovf);
        else
            k_join_pairs<uint64_t, false><<<grid, kBlock, 0, s>>>((const uint64_t*)y.keys, y.cnt, y.n,
                                                                  (const uint64_t*)z.keys, z.cnt, z.n, y.lay, n, colors,
                                                                  pcount, nullptr, nullptr, nullptr, nullptr);
    } else {
        if (out)
            k_join_pairs<u128, true><<<grid, kBlock, 0, s>>>((const u128*)y.keys, y.cnt, y.n, (const u128*)z.keys, z.cnt,
                                                             z.n, y.lay, n, colors, nullptr, poff, (u128*)out->keys,
                                                             out->cnt, ovf);
        else
            k_join_pairs<u128, false><<<grid, kBlock, 0, s>>>((const u128*)y.keys, y.cnt, y.n, (const u128*)z.keys,
                                                              z.cnt, z.n, y.lay, n, colors, pcount, nullptr, nullptr,
                                                              nullptr, nullptr);
    }
}

void launch_drop_last(const DevTable& in, DevTable& out, hipStream_t s) {
    if (!in.n) return;
    const int ki = in.lay.kw(), ko = out.lay.kw();
    if (ki == 1)
        k_drop_last<uint64_t, uint64_t><<<grid_for(in.n), kBlock, 0, s>>>((const uint64_t*)in.keys, in.n, in.lay, out.lay,
                                                                          (uint64_t*)out.keys);
    else if (ko == 1)
        k_drop_last<u128, uint64_t><<<grid_for(in.n), kBlock, 0, s>>>((const u128*)in.keys, in.n, in.lay, out.lay,
                                                                      (uint64_t*)out.keys);
    else
        k_drop_last<u128, u128><<<grid_for(in.n), kBlock, 0, s>>>((const u128*)in.keys, in.n, in.lay, out.lay,
                                                                  (u128*)out.keys);
}

void launch_reduce_runs(const DevTable& in, const uint64_t* starts, uint64_t G, DevTable& out, uint32_t* ovf,
                        hipStream_t s) {
    if (!G) return;
    if (in.lay.kw() == 1)
        k_reduce_runs<uint64_t><<<grid_for(G), kBlock, 0, s>>>((const uint64_t*)in.keys, in.cnt, starts, G, in.lay,
                                                               (uint64_t*)out.keys, out.cnt, ovf);
    else
        k_reduce_runs<u128><<<grid_for(G), kBlock, 0, s>>>((const u128*)in.keys, in.cnt, starts, G, in.lay,
                                                           (u128*)out.keys, out.cnt, ovf);
}

// ---- launchers -------------------------------------------------------------

void launch_entry_seglen(const DevTable& in, DevGraph g, const IntroArgs& a, uint32_t* slen, uint8_t* src,
                         uint64_t* sums, uint64_t stride, hipStream_t s) {
    if (!in.n) return;
    auto* ai = reinterpret_cast<unsigned long long*>(sums);
    const uint64_t M = (in.n + stride - 1) / stride;
    // a bounded grid: each block adds its sums with two atomics
    const unsigned grid = grid_for(M, kBlock, 4096);
    if (in.lay.kw() == 1)
        k_entry_seglen<uint64_t><<<grid, kBlock, 0, s>>>((const uint64_t*)in.keys, in.lay, in.n, stride, g, a, slen, src,
                                                         ai);
    else
        k_entry_seglen<u128><<<grid, kBlock, 0, s>>>((const u128*)in.keys, in.lay, in.n, stride, g, a, slen, src, ai);
}

template <bool EMIT>
static void entry_dispatch(const DevTable& in, const uint8_t* src, const uint64_t* soff, uint64_t T, DevGraph g,
                           const uint8_t* colors, const IntroArgs& a, uint32_t* tcount, const uint64_t* toff,
                           DevTable* out, uint16_t* pbits, hipStream_t s) {
    const uint64_t tiles = expand_tiles(T);
    if (!tiles) return;
    const unsigned grid = unsigned(tiles < (1u << 20) ? tiles : (1u << 20));
    Lay LO = out ? out->lay : Lay{in.lay.b + 1, in.lay.vb, in.lay.kb, in.lay.bb};
    void* ok = out ? out->keys : nullptr;
    uint64_t* oc = out ? out->cnt : nullptr;
    const int ki = in.lay.kw(), ko = LO.kw();
    if (ki == 1 && ko == 1)
        k_expand_entry<uint64_t, uint64_t, EMIT><<<grid, kBlock, 0, s>>>((const uint64_t*)in.keys, in.cnt, in.lay, src,
                                                                         soff, in.n, T, g, colors, a, tcount, toff,
                                                                         (uint64_t*)ok, oc, LO, pbits);
    else if (ki == 1)
        k_expand_entry<uint64_t, u128, EMIT><<<grid, kBlock, 0, s>>>((const uint64_t*)in.keys, in.cnt, in.lay, src, soff,
                                                                     in.n, T, g, colors, a, tcount, toff, (u128*)ok, oc,
                                                                     LO, pbits);
    else
        k_expand_entry<u128, u128, EMIT><<<grid, kBlock, 0, s>>>((const u128*)in.keys, in.cnt, in.lay, src, soff, in.n,
                                                                 T, g, colors, a, tcount, toff, (u128*)ok, oc, LO,
                                                                 pbits);
}

void launch_entry_count(const DevTable& in, const uint8_t* src, const uint64_t* soff, uint64_t T, DevGraph g,
                        const uint8_t* colors, const IntroArgs& a, uint32_t* tcount, uint16_t* pbits, hipStream_t s) {
    const uint64_t tiles = expand_tiles(T);
    if (!tiles) return;
    k_expand_bounds<<<grid_for(tiles), kBlock, 0, s>>>(soff, in.n, nullptr, 0, T, true,
                                                      reinterpret_cast<uint64_t*>(pbits + tiles * kBlock));
    entry_dispatch<false>(in, src, soff, T, g, colors, a, tcount, nullptr, nullptr, pbits, s);
}

void launch_entry_emit(const DevTable& in, const uint8_t* src, const uint64_t* soff, uint64_t T, DevGraph g,
                       const uint8_t* colors, const IntroArgs& a, const uint64_t* toff, const uint16_t* pbits,
                       DevTable& out, hipStream_t s) {
    entry_dispatch<true>(in, src, soff, T, g, colors, a, nullptr, toff, &out, const_cast<uint16_t*>(pbits), s);
}

void launch_push_seglen(const DevTable& in, const uint64_t* gstart, const uint64_t* woff, uint64_t G, uint64_t W,
                        DevGraph g, const uint8_t* colors, const IntroArgs& a, uint32_t* slen, hipStream_t s) {
    if (!W) return;
    if (a.segv && g.n > (1 << 27)) throw std::runtime_error("launch_push_seglen: packed segment vertices need n <= 2^27");
    const uint64_t tiles = (W + kSegTile - 1) / kSegTile;
    const unsigned grid = unsigned(tiles < (1u << 20) ? tiles : (1u << 20));
    if (in.lay.kw() == 1)
        k_push_seglen<uint64_t><<<grid, kBlock, 0, s>>>((const uint64_t*)in.keys, in.lay, gstart, woff, G, W, g, colors,
                                                        a, slen);
    else
        k_push_seglen<u128><<<grid, kBlock, 0, s>>>((const u128*)in.keys, in.lay, gstart, woff, G, W, g, colors, a,
                                                    slen);
}

void launch_pull_seglen(const uint64_t* rstart, const uint64_t* rend, int B, DevGraph g, int degF, uint32_t* slen,
                        hipStream_t s) {
    uint64_t W = uint64_t(B) * uint64_t(g.m2);
    if (W) k_pull_seglen<<<grid_for(W), kBlock, 0, s>>>(rstart, rend, B, g, degF, slen);
}

uint64_t expand_tiles(uint64_t T) { return (T + kExpTile - 1) / kExpTile; }

template <bool EMIT, bool PULL>
static void expand_dispatch(const DevTable& in, const uint64_t* gstart, const uint64_t* woff, uint64_t G,
                            const uint64_t* rstart, const uint64_t* soff, uint64_t S, uint64_t T, DevGraph g,
                            const uint8_t* colors, const IntroArgs& a, uint32_t* tcount, const uint64_t* toff,
                            DevTable* out, uint64_t* osrc, uint16_t* pbits, hipStream_t s) {
    uint64_t tiles = expand_tiles(T);
    if (!tiles) return;
    unsigned grid = unsigned(tiles < (1u << 20) ? tiles : (1u << 20));
    Lay LO = out ? out->lay : Lay{in.lay.b + 1, in.lay.vb, in.lay.kb, in.lay.bb};
    void* ok = out ? out->keys : nullptr;
    uint64_t* oc = out ? out->cnt : nullptr;
    int ki = in.lay.kw(), ko = LO.kw();
    if (ki == 1 && ko == 1)
        k_expand<uint64_t, uint64_t, EMIT, PULL><<<grid, kBlock, 0, s>>>(
            (const uint64_t*)in.keys, in.cnt, in.lay, gstart, woff, G, rstart, soff, S, T, g, colors, a, tcount, toff,
            (uint64_t*)ok, oc, LO, osrc, pbits);
    else if (ki == 1)
        k_expand<uint64_t, u128, EMIT, PULL><<<grid, kBlock, 0, s>>>((const uint64_t*)in.keys, in.cnt, in.lay, gstart, woff,
                                                                      G, rstart, soff, S, T, g, colors, a, tcount, toff,
                                                                      (u128*)ok, oc, LO, osrc, pbits);
    else
        k_expand<u128, u128, EMIT, PULL><<<grid, kBlock, 0, s>>>((const u128*)in.keys, in.cnt, in.lay, gstart, woff, G,
                                                                  rstart, soff, S, T, g, colors, a, tcount, toff,
                                                                  (u128*)ok, oc, LO, osrc, pbits);
}

// survivor bits (one 16-bit word per thread and tile), then four 64-bit tile
// bounds per tile
uint64_t expand_pass_words(uint64_t T) { return expand_tiles(T) * (kBlock + 16); }

void launch_expand_count(bool pull, const DevTable& in, const uint64_t* gstart, const uint64_t* woff, uint64_t G,
                         const uint64_t* rstart, const uint64_t* soff, uint64_t S, uint64_t T, DevGraph g,
                         const uint8_t* colors, const IntroArgs& a, uint32_t* tcount, uint16_t* pbits, hipStream_t s) {
    const uint64_t tiles = expand_tiles(T);
    if (!tiles) return;
    k_expand_bounds<<<grid_for(tiles), kBlock, 0, s>>>(soff, S, woff, G, T, pull,
                                                      reinterpret_cast<uint64_t*>(pbits + tiles * kBlock));
    if (pull)
        expand_dispatch<false, true>(in, gstart, woff, G, rstart, soff, S, T, g, colors, a, tcount, nullptr, nullptr,
                                     nullptr, pbits, s);
    else
        expand_dispatch<false, false>(in, gstart, woff, G, rstart, soff, S, T, g, colors, a, tcount, nullptr, nullptr,
                                      nullptr, pbits, s);
}

void launch_expand_emit(bool pull, const DevTable& in, const uint64_t* gstart, const uint64_t* woff, uint64_t G,
                        const uint64_t* rstart, const uint64_t* soff, uint64_t S, uint64_t T, DevGraph g,
                        const uint8_t* colors, const IntroArgs& a, const uint64_t* toff, const uint16_t* pbits,
                        DevTable& out, uint64_t* osrc, hipStream_t s) {
    uint16_t* pb = const_cast<uint16_t*>(pbits);  // read only in the emit pass
    if (pull)
        expand_dispatch<true, true>(in, gstart, woff, G, rstart, soff, S, T, g, colors, a, nullptr, toff, &out, osrc, pb,
                                    s);
    else
        expand_dispatch<true, false>(in, gstart, woff, G, rstart, soff, S, T, g, colors, a, nullptr, toff, &out, osrc,
                                     pb, s);
}

}  // namespace ccg
