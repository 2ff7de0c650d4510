// Kernels of the enumeration path (Sec. 4, result reconstruction).
//
// The paper rebuilds the mappings top-down with sets M of (phi, C) pairs and
// glues lists bottom-up.  Here every table entry instead carries an index of
// the entries it was built from (one child entry for introduce, the merged
// child entries for forget, the admissible colour-set pairs for join) with
// exclusive prefix sums of their counts.  A row number r in [0, count) then
// decodes to one mapping by descending from the root: at a forget node the
// prefix sums pick the contributing child entry, at a join node the pair and
// the mixed-radix split of the remaining rank between the two children.
// Every row is decoded independently, one thread per row.
#include <hip/hip_runtime.h>

#include "device.h"
#include "kernels.h"

namespace ccg {

// forget: output position of every child entry = group offset + rank of its
// colour set among the group's present colour sets
template <class K>
__global__ void __launch_bounds__(64)
k_forget_dst(const K* __restrict__ keys, Lay L, const uint64_t* __restrict__ gstart, uint64_t G,
             const uint64_t* __restrict__ goff, uint64_t* dst) {
    Acc acc = acc_bind(L.kb, false);
    __shared__ uint32_t wpre[1 << 7];  // prefix popcounts of the mask words (kb <= 12)
    for (uint64_t grp = blockIdx.x; grp < G; grp += gridDim.x) {
        uint64_t e0 = gstart[grp], e1 = gstart[grp + 1];
        acc_clear(acc, false);
        __syncthreads();
        for (uint64_t e = e0 + threadIdx.x; e < e1; e += 64) {
            uint32_t C = kset(keys[e], L);
            atomicOr(&acc.bits[C >> 5], 1u << (C & 31));
        }
        __syncthreads();
        if (threadIdx.x == 0) {
            uint32_t run = 0;
            for (int i = 0; i < acc.words(); i++) {
                wpre[i] = run;
                run += __popc(acc.bits[i]);
            }
        }
        __syncthreads();
        for (uint64_t e = e0 + threadIdx.x; e < e1; e += 64) {
            uint32_t C = kset(keys[e], L);
            uint32_t below = acc.bits[C >> 5] & ((1u << (C & 31)) - 1u);
            dst[e] = goff[grp] + wpre[C >> 5] + __popc(below);
        }
        __syncthreads();
    }
}

void launch_forget_dst(const DevTable& in, const uint64_t* gstart, uint64_t G, const uint64_t* goff, uint64_t* dst,
                       hipStream_t s) {
    if (!G) return;
    unsigned grid = unsigned(G < (1u << 20) ? G : (1u << 20));
    size_t lds = acc_bytes(in.lay.kb, false);
    if (in.lay.kw() == 1)
        k_forget_dst<uint64_t><<<grid, 64, lds, s>>>((const uint64_t*)in.keys, in.lay, gstart, G, goff, dst);
    else
        k_forget_dst<u128><<<grid, 64, lds, s>>>((const u128*)in.keys, in.lay, gstart, G, goff, dst);
}

// join: for every Y group, the admissible (a, d) pairs in (a, d) order with
// the output position of their union colour set
template <class K>
__device__ __forceinline__ uint64_t lb_prefix(const K* keys, uint64_t n, K p, int sh, bool strict) {
    uint64_t lo = 0, hi = n;
    while (lo < hi) {
        uint64_t mid = (lo + hi) >> 1;
        K q = shr(keys[mid], sh);
        if (q < p || (strict && q == p)) lo = mid + 1;
        else hi = mid;
    }
    return lo;
}

template <class K, bool EMIT>
__global__ void __launch_bounds__(64)
k_join_pairs(const K* __restrict__ yk, const K* __restrict__ zk, uint64_t nz, Lay L,
             const uint64_t* __restrict__ gstart, uint64_t G, int32_t n, const uint8_t* __restrict__ colors,
             uint32_t* pcount, const uint64_t* __restrict__ goff, const uint64_t* __restrict__ poff, uint64_t* pdst,
             uint64_t* pa, uint64_t* pd) {
    Acc acc = acc_bind(L.kb, false);
    __shared__ uint32_t wpre[1 << 7];
    const int sh = L.kb;
    for (uint64_t grp = blockIdx.x; grp < G; grp += gridDim.x) {
        uint64_t e0 = gstart[grp], e1 = gstart[grp + 1];
        K k0 = yk[e0];
        K p = shr(k0, sh);
        uint64_t z0 = lb_prefix(zk, nz, p, sh, false);
        uint64_t z1 = lb_prefix(zk, nz, p, sh, true);
        uint32_t bid = kbid(k0, L);
        uint32_t bagcol = 0;
        for (int j = 0; j < L.b; j++) bagcol |= 1u << colors[uint64_t(bid) * n + kcol(k0, L, j)];
        uint64_t ny = e1 - e0, nzg = z1 - z0;
        if (EMIT) {
            acc_clear(acc, false);
            __syncthreads();
            for (uint64_t a = 0; a < ny; a++) {
                uint32_t Cy = kset(yk[e0 + a], L);
                for (uint64_t d = threadIdx.x; d < nzg; d += 64) {
                    uint32_t Cz = kset(zk[z0 + d], L);
                    if ((Cy & Cz) != bagcol) continue;
                    uint32_t C = Cy | Cz;
                    atomicOr(&acc.bits[C >> 5], 1u << (C & 31));
                }
            }
            __syncthreads();
            if (threadIdx.x == 0) {
                uint32_t run = 0;
                for (int i = 0; i < acc.words(); i++) {
                    wpre[i] = run;
                    run += __popc(acc.bits[i]);
                }
            }
            __syncthreads();
        }
        uint64_t written = 0;
        uint32_t found = 0;
        for (uint64_t a = 0; a < ny; a++) {
            uint32_t Cy = kset(yk[e0 + a], L);
            for (uint64_t d0 = 0; d0 < nzg; d0 += 64) {
                uint64_t d = d0 + threadIdx.x;
                bool ok = false;
                uint32_t Cz = 0;
                if (d < nzg) {
                    Cz = kset(zk[z0 + d], L);
                    ok = (Cy & Cz) == bagcol;
                }
                uint64_t m = __ballot(ok);
                if (EMIT && ok) {
                    uint32_t C = Cy | Cz;
                    uint32_t below = acc.bits[C >> 5] & ((1u << (C & 31)) - 1u);
                    uint64_t o = poff[grp] + written + __popcll(m & lanemask_lt());
                    pdst[o] = goff[grp] + wpre[C >> 5] + __popc(below);
                    pa[o] = e0 + a;
                    pd[o] = z0 + d;
                }
                written += __popcll(m);
                found += uint32_t(__popcll(m));
            }
        }
        if (!EMIT && threadIdx.x == 0) pcount[grp] = found;
        __syncthreads();
    }
}

void launch_join_pairs_count(const DevTable& y, const DevTable& z, const uint64_t* gstart, uint64_t G, int32_t n,
                             const uint8_t* colors, uint32_t* pcount, hipStream_t s) {
    if (!G) return;
    unsigned grid = unsigned(G < (1u << 20) ? G : (1u << 20));
    size_t lds = acc_bytes(y.lay.kb, false);
    if (y.lay.kw() == 1)
        k_join_pairs<uint64_t, false><<<grid, 64, lds, s>>>((const uint64_t*)y.keys, (const uint64_t*)z.keys, z.n, y.lay,
                                                            gstart, G, n, colors, pcount, nullptr, nullptr, nullptr,
                                                            nullptr, nullptr);
    else
        k_join_pairs<u128, false><<<grid, 64, lds, s>>>((const u128*)y.keys, (const u128*)z.keys, z.n, y.lay, gstart, G, n,
                                                        colors, pcount, nullptr, nullptr, nullptr, nullptr, nullptr);
}

void launch_join_pairs_emit(const DevTable& y, const DevTable& z, const uint64_t* gstart, uint64_t G, int32_t n,
                            const uint8_t* colors, const uint64_t* goff, const uint64_t* poff, uint64_t* pdst,
                            uint64_t* pa, uint64_t* pd, hipStream_t s) {
    if (!G) return;
    unsigned grid = unsigned(G < (1u << 20) ? G : (1u << 20));
    size_t lds = acc_bytes(y.lay.kb, false);
    if (y.lay.kw() == 1)
        k_join_pairs<uint64_t, true><<<grid, 64, lds, s>>>((const uint64_t*)y.keys, (const uint64_t*)z.keys, z.n, y.lay,
                                                           gstart, G, n, colors, nullptr, goff, poff, pdst, pa, pd);
    else
        k_join_pairs<u128, true><<<grid, 64, lds, s>>>((const u128*)y.keys, (const u128*)z.keys, z.n, y.lay, gstart, G, n,
                                                       colors, nullptr, goff, poff, pdst, pa, pd);
}

__global__ void k_segment_starts(const uint64_t* __restrict__ keys, uint64_t n, uint64_t nseg, uint64_t* starts) {
    for (uint64_t j = uint64_t(blockIdx.x) * blockDim.x + threadIdx.x; j < n; j += uint64_t(gridDim.x) * blockDim.x)
        if (j == 0 || keys[j] != keys[j - 1]) starts[keys[j]] = j;
    if (blockIdx.x == 0 && threadIdx.x == 0) starts[nseg] = n;
}

void launch_segment_starts(const uint64_t* keys, uint64_t n, uint64_t nseg, uint64_t* starts, hipStream_t s) {
    k_segment_starts<<<grid_for(n), kBlock, 0, s>>>(keys, n, nseg, starts);
}

__global__ void k_gather(const uint64_t* __restrict__ src, const uint64_t* __restrict__ idx, uint64_t n, uint64_t* out) {
    for (uint64_t j = uint64_t(blockIdx.x) * blockDim.x + threadIdx.x; j < n; j += uint64_t(gridDim.x) * blockDim.x)
        out[j] = src[idx[j]];
}

void launch_gather_u64(const uint64_t* src, const uint64_t* idx, uint64_t n, uint64_t* out, hipStream_t s) {
    if (n) k_gather<<<grid_for(n), kBlock, 0, s>>>(src, idx, n, out);
}

__global__ void k_iota(uint64_t* p, uint64_t n) {
    for (uint64_t j = uint64_t(blockIdx.x) * blockDim.x + threadIdx.x; j < n; j += uint64_t(gridDim.x) * blockDim.x)
        p[j] = j;
}

void launch_iota(uint64_t* p, uint64_t n, hipStream_t s) {
    if (n) k_iota<<<grid_for(n), kBlock, 0, s>>>(p, n);
}

__global__ void k_gather_product(const uint64_t* __restrict__ a, const uint64_t* __restrict__ ia,
                                 const uint64_t* __restrict__ b, const uint64_t* __restrict__ ib, uint64_t n,
                                 uint64_t* out) {
    for (uint64_t j = uint64_t(blockIdx.x) * blockDim.x + threadIdx.x; j < n; j += uint64_t(gridDim.x) * blockDim.x)
        out[j] = a[ia[j]] * b[ib[j]];
}

void launch_gather_product(const uint64_t* a, const uint64_t* ia, const uint64_t* b, const uint64_t* ib, uint64_t n,
                           uint64_t* out, hipStream_t s) {
    if (n) k_gather_product<<<grid_for(n), kBlock, 0, s>>>(a, ia, b, ib, n, out);
}

// ---------------------------------------------------------------------------
// row decoder

__device__ __forceinline__ uint32_t step_col(const EnumStep& S, uint64_t e, int j) {
    const Lay& L = S.lay;
    if (L.bb + L.b * L.vb + L.kb <= 64) return kcol(((const uint64_t*)S.keys)[e], L, j);
    return kcol(((const u128*)S.keys)[e], L, j);
}

// largest j in [s0, s1) with wcum[j] - wcum[s0] <= q (differences are exact
// modulo 2^64 because every segment's total is an exact count)
__device__ __forceinline__ uint64_t pick(const uint64_t* wcum, uint64_t s0, uint64_t s1, uint64_t q) {
    uint64_t base = wcum[s0], lo = s0, hi = s1;
    while (hi - lo > 1) {
        uint64_t mid = (lo + hi) >> 1;
        if (wcum[mid] - base <= q) lo = mid;
        else hi = mid;
    }
    return lo;
}

template <class RK>
__global__ void k_unrank(const EnumStep* __restrict__ steps, int root_step, const uint64_t* __restrict__ rcum, uint64_t E,
                         uint64_t R, int nF, int vb, RK* rowkeys, uint32_t* err) {
    constexpr int kStack = 40;
    for (uint64_t r = uint64_t(blockIdx.x) * blockDim.x + threadIdx.x; r < R; r += uint64_t(gridDim.x) * blockDim.x) {
        uint32_t phi[16];
        for (int i = 0; i < 16; i++) phi[i] = 0;
        int st_step[kStack];
        uint64_t st_e[kStack], st_q[kStack];
        int sp = 0;
        uint64_t o = upper_bound_u64(rcum, 0, E + 1, r) - 1;
        st_step[0] = root_step;
        st_e[0] = o;
        st_q[0] = r - rcum[o];
        sp = 1;
        while (sp > 0) {
            sp--;
            const EnumStep& S = steps[st_step[sp]];
            uint64_t e = st_e[sp], q = st_q[sp];
            int push_n = 0;
            int ns[2];
            uint64_t ne[2], nq[2];
            switch (S.kind) {
                case EK_LEAF:
                    phi[S.u] = step_col(S, e, S.ucol);
                    break;
                case EK_INTRO:
                    phi[S.u] = step_col(S, e, S.ucol);
                    ns[0] = S.in0; ne[0] = S.src[e]; nq[0] = q; push_n = 1;
                    break;
                case EK_RESORT:
                    ns[0] = S.in0; ne[0] = S.src[e]; nq[0] = q; push_n = 1;
                    break;
                case EK_FORGET: {
                    uint64_t j = pick(S.wcum, S.seg[e], S.seg[e + 1], q);
                    ns[0] = S.in0; ne[0] = S.ca[j]; nq[0] = q - (S.wcum[j] - S.wcum[S.seg[e]]); push_n = 1;
                    break;
                }
                case EK_JOIN: {
                    uint64_t j = pick(S.wcum, S.seg[e], S.seg[e + 1], q);
                    uint64_t rest = q - (S.wcum[j] - S.wcum[S.seg[e]]);
                    uint64_t nzc = steps[S.in1].cnt[S.cb[j]];
                    ns[0] = S.in0; ne[0] = S.ca[j]; nq[0] = rest / nzc;
                    ns[1] = S.in1; ne[1] = S.cb[j]; nq[1] = rest % nzc;
                    push_n = 2;
                    break;
                }
                default:
                    atomicOr(err, 2u);
            }
            for (int t = 0; t < push_n; t++) {
                if (sp >= kStack) {
                    atomicOr(err, 1u);
                    break;
                }
                st_step[sp] = ns[t];
                st_e[sp] = ne[t];
                st_q[sp] = nq[t];
                sp++;
            }
        }
        RK key = 0;
        for (int i = 0; i < nF; i++) key = (key << vb) | RK(phi[i]);
        rowkeys[r] = key;
    }
}

void launch_unrank(const EnumStep* steps, int root_step, const uint64_t* rcum, uint64_t E, uint64_t R, int nF, int vb,
                   int rkw, void* rowkeys, uint32_t* err, hipStream_t s) {
    if (!R) return;
    if (rkw == 1)
        k_unrank<uint64_t><<<grid_for(R), kBlock, 0, s>>>(steps, root_step, rcum, E, R, nF, vb, (uint64_t*)rowkeys, err);
    else
        k_unrank<u128><<<grid_for(R), kBlock, 0, s>>>(steps, root_step, rcum, E, R, nF, vb, (u128*)rowkeys, err);
}

}  // namespace ccg
