// Initial bisection, gains, swap refinement and balancing (Algorithms 3-5).
//
// Gains (Algorithm 4) are computed in transpose.hpp: a hyperedge pass finds
// what a pin on each side gains from the hyperedge (+w(e) when it is alone on
// its side, -w(e) when the hyperedge is uncut), a node pass sums that over the
// node's hyperedges.
//
// Every "pick the r best nodes in (gain desc, id asc) order" step - the
// ceil(sqrt n) moves of Algorithm 3, the two sorted lists of Algorithm 5 and
// the balance step - is a segmented radix select on the unique 64-bit key
// (gain, id): eight 8-bit digit passes of per-list histograms find the key of
// the r-th element of each list (a list is one side of one segment), then a
// node is chosen iff its key is <= that threshold.  No full sort is needed
// and the chosen set is exactly the sorted prefix.
#pragma once
#include "level.hpp"

namespace bp {

// selection mode bits per segment
constexpr uint8_t kList0 = 1, kList1 = 2, kGainNonNeg = 4, kMinPair = 8;

// ---- segmented radix select ---------------------------------------------------

constexpr int kSelNodesPerBlock = 1024;
constexpr int kSelLdsLists = 4;

__device__ __forceinline__ bool sel_eligible(int64_t v, const int32_t *gain, const uint8_t *side,
                                             const int32_t *nseg, const uint8_t *mode,
                                             int32_t *list, uint64_t *key)
{
    int32_t s = nseg[v];
    uint8_t md = mode[s];
    int32_t sd = side[v];
    if (!((md >> sd) & 1)) return false;
    int32_t g = gain[v];
    if ((md & kGainNonNeg) && g < 0) return false;
    *list = 2 * s + sd;
    *key = gain_order_key(g, (uint32_t)v);
    return true;
}

__global__ __launch_bounds__(kBlock) void k_sel_hist(int32_t N, int pass, const int32_t *gain,
                                                     const uint8_t *side, const int32_t *nseg,
                                                     const uint8_t *mode, const uint64_t *prefix,
                                                     const uint8_t *ldone, uint32_t *hist)
{
    __shared__ uint32_t h[kSelLdsLists * 256];
    int64_t v0 = (int64_t)blockIdx.x * kSelNodesPerBlock;
    if (v0 >= N) return;
    int64_t v1 = v0 + kSelNodesPerBlock < N ? v0 + kSelNodesPerBlock : N;
    int32_t cbase = 2 * nseg[v0];
    bool use_lds = 2 * nseg[v1 - 1] + 1 - cbase < kSelLdsLists;
    if (use_lds) {
        for (int i = threadIdx.x; i < kSelLdsLists * 256; i += blockDim.x) h[i] = 0;
        __syncthreads();
    }
    int shift = 56 - 8 * pass;
    for (int64_t v = v0 + threadIdx.x; v < v1; v += blockDim.x) {
        int32_t c;
        uint64_t k;
        if (!sel_eligible(v, gain, side, nseg, mode, &c, &k)) continue;
        // pass 0 sees every eligible node; its pick resets the per-list state
        if (pass > 0 && (ldone[c] || ((k ^ prefix[c]) >> (shift + 8)) != 0)) continue;
        int dig = (int)((k >> shift) & 0xff);
        if (use_lds) atomicAdd(&h[(c - cbase) * 256 + dig], 1u);
        else atomicAdd(&hist[(int64_t)c * 256 + dig], 1u);
    }
    if (use_lds) {
        __syncthreads();
        for (int i = threadIdx.x; i < kSelLdsLists * 256; i += blockDim.x) {
            uint32_t x = h[i];
            if (x) atomicAdd(&hist[(int64_t)(cbase + i / 256) * 256 + (i & 255)], x);
        }
    }
}

// One wavefront per list: choose the digit holding the r-th element.
__global__ __launch_bounds__(kBlock) void k_sel_pick(int32_t nlists, int pass, const uint8_t *mode,
                                                     const int32_t *m, uint32_t *hist,
                                                     uint64_t *prefix, int32_t *rem, int32_t *rsel,
                                                     uint8_t *ldone, uint64_t *thr)
{
    int64_t c = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
    int lane = threadIdx.x & 63;
    if (c >= nlists) return;
    uint32_t *hc = hist + c * 256;
    uint32_t x[4];
#pragma unroll
    for (int j = 0; j < 4; j++) x[j] = hc[lane * 4 + j];
    int shift = 56 - 8 * pass;
    int32_t r;
    if (pass == 0) {
        int32_t s = (int32_t)(c >> 1), sd = (int32_t)(c & 1);
        uint8_t md = mode[s];
        int64_t tot = wave_sum((int64_t)x[0] + x[1] + x[2] + x[3]);
        int64_t r0 = 0;
        if ((md >> sd) & 1) {
            if (md & kMinPair) {
                uint32_t *ho = hist + (c ^ 1) * 256;
                int64_t o = wave_sum((int64_t)ho[lane * 4] + ho[lane * 4 + 1] + ho[lane * 4 + 2] +
                                     ho[lane * 4 + 3]);
                r0 = tot < o ? tot : o;
            } else {
                r0 = tot < (int64_t)m[s] ? tot : (int64_t)m[s];
            }
        }
        if (lane == 0) {
            rsel[c] = (int32_t)r0;
            rem[c] = (int32_t)r0;
            prefix[c] = 0;
            ldone[c] = r0 == 0;
            thr[c] = 0;
        }
        if (r0 == 0) return;
        r = (int32_t)r0;
    } else {
        if (ldone[c]) return;
        r = rem[c];
    }
    // Pass-0 histograms are cleared by k_sel_clear after every list has read
    // them (a MinPair list also reads its partner's); later passes clear their
    // own below.
    uint32_t s4 = x[0] + x[1] + x[2] + x[3];
    uint32_t incl = wave_incl_scan(s4);
    uint32_t before = incl - s4;
    // lane holding the digit: before < r <= incl
    unsigned long long bal = __ballot((int64_t)before < r && r <= (int64_t)incl);
    int owner = __ffsll((long long)bal) - 1;
    int32_t digit = 0, below = 0, inbin = 0;
    if (lane == owner) {
        uint32_t acc = before;
#pragma unroll
        for (int j = 0; j < 4; j++) {
            if ((int64_t)acc + x[j] >= r) {
                digit = lane * 4 + j;
                below = (int32_t)acc;
                inbin = (int32_t)x[j];
                break;
            }
            acc += x[j];
        }
    }
    digit = __shfl(digit, owner, 64);
    below = __shfl(below, owner, 64);
    inbin = __shfl(inbin, owner, 64);
    if (lane == 0) {
        uint64_t p = prefix[c] | ((uint64_t)digit << shift);
        int32_t left = r - below;
        prefix[c] = p;
        rem[c] = left;
        if (left == inbin || pass == 7) {
            uint64_t low = shift ? ((1ull << shift) - 1) : 0ull;
            thr[c] = p | low;
            ldone[c] = 1;
        }
    }
    if (pass > 0) {
#pragma unroll
        for (int j = 0; j < 4; j++) hc[lane * 4 + j] = 0;
    }
}

// Clears pass-0 histograms that were kept for MinPair partners.
__global__ void k_sel_clear(int64_t n, uint32_t *hist)
{
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x)
        hist[i] = 0;
}

__device__ __forceinline__ bool sel_chosen(int64_t v, const int32_t *gain, const uint8_t *side,
                                           const int32_t *nseg, const uint8_t *mode,
                                           const int32_t *rsel, const uint64_t *thr)
{
    int32_t c;
    uint64_t k;
    if (!sel_eligible(v, gain, side, nseg, mode, &c, &k)) return false;
    return rsel[c] > 0 && k <= thr[c];
}

// Flip chosen nodes; side weights of each segment updated with one atomic per
// workgroup when the workgroup lies in one segment.
__global__ __launch_bounds__(kBlock) void k_apply_flip(int32_t N, const int32_t *gain,
                                                       uint8_t *side, const int32_t *nseg,
                                                       const uint8_t *mode, const int32_t *rsel,
                                                       const uint64_t *thr, const int32_t *nw,
                                                       unsigned long long *segw)
{
    __shared__ int64_t lds[16];
    int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    int64_t vl = (int64_t)blockIdx.x * blockDim.x + blockDim.x - 1;
    if (vl >= N) vl = N - 1;
    int64_t vf = (int64_t)blockIdx.x * blockDim.x;
    bool one_seg = nseg[vf] == nseg[vl];
    int64_t d01 = 0;  // weight moved 0 -> 1 minus weight moved 1 -> 0
    if (v < N && sel_chosen(v, gain, side, nseg, mode, rsel, thr)) {
        int32_t sd = side[v];
        int64_t w = nw[v];
        side[v] = (uint8_t)(1 - sd);
        if (one_seg) {
            d01 += sd ? -w : w;
        } else {
            int32_t s = nseg[v];
            atomicAdd(&segw[2 * s + sd], (unsigned long long)(-w));
            atomicAdd(&segw[2 * s + 1 - sd], (unsigned long long)w);
        }
    }
    if (one_seg) {
        d01 = block_sum(d01, lds);
        if (threadIdx.x == 0 && d01 != 0) {
            int32_t s = nseg[vf];
            atomicAdd(&segw[2 * s], (unsigned long long)(-d01));
            atomicAdd(&segw[2 * s + 1], (unsigned long long)d01);
        }
    }
}

// ---- per-level setup ------------------------------------------------------------

// side of level j: projected from level j+1 for segments coarsened past j,
// all-ones start of Algorithm 3 for segments whose coarsest level is j.
__global__ __launch_bounds__(kBlock) void k_project(int32_t N, int32_t j, const int32_t *nseg,
                                                    const int32_t *coarsest,
                                                    const int32_t *parent,
                                                    const uint8_t *side_coarse, uint8_t *side)
{
    int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (v >= N) return;
    int32_t c = coarsest[nseg[v]];
    if (c > j) side[v] = side_coarse[parent[v]];
    else if (c == j) side[v] = 1;
}

// Side weights of every segment (block-aggregated atomics).
__global__ __launch_bounds__(kBlock) void k_side_weights(int32_t N, const int32_t *nseg,
                                                         const uint8_t *side, const int32_t *nw,
                                                         unsigned long long *segw)
{
    __shared__ int64_t lds[16];
    int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    int64_t vf = (int64_t)blockIdx.x * blockDim.x;
    int64_t vl = vf + blockDim.x - 1 < N ? vf + blockDim.x - 1 : N - 1;
    bool one_seg = nseg[vf] == nseg[vl];
    int64_t w0 = 0, w1 = 0;
    if (v < N) {
        int64_t w = nw[v];
        if (one_seg) {
            if (side[v]) w1 = w;
            else w0 = w;
        } else {
            atomicAdd(&segw[2 * nseg[v] + side[v]], (unsigned long long)w);
        }
    }
    if (one_seg) {
        w0 = block_sum(w0, lds);
        w1 = block_sum(w1, lds);
        if (threadIdx.x == 0) {
            int32_t s = nseg[vf];
            if (w0) atomicAdd(&segw[2 * s], (unsigned long long)w0);
            if (w1) atomicAdd(&segw[2 * s + 1], (unsigned long long)w1);
        }
    }
}

// Per-segment modes.  One thread per segment.
// Algorithm 3 loop test: P0 below its share and P1 non-empty.
__global__ void k_mode_initial(int32_t S, int32_t j, const int32_t *nbase, const int32_t *coarsest,
                               const int32_t *k0, const int32_t *k1, const int64_t *W,
                               const unsigned long long *segw, int32_t *cnt1, const int32_t *rsel,
                               int first, uint8_t *mode, uint8_t *gmask, int32_t *m,
                               LevelInfo *info)
{
    int32_t s = blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= S) return;
    uint8_t md = 0;
    if (coarsest[s] == j) {
        int32_t n = nbase[s + 1] - nbase[s];
        if (first) cnt1[s] = n;
        else cnt1[s] -= rsel[2 * s + 1];
        int64_t ks = (int64_t)k0[s] + k1[s];
        bool go = (int64_t)segw[2 * s] * ks < W[s] * (int64_t)k0[s] && cnt1[s] > 0;
        if (go) {
            md = kList1;
            m[s] = (int32_t)ceil_sqrt_i64(n);
            atomicAdd(&info->flag, 1);
        }
    }
    mode[s] = md;
    gmask[s] = md ? 1 : 0;
}

__global__ void k_mode_refine(int32_t S, int32_t j, const int32_t *coarsest, uint8_t *mode,
                              uint8_t *gmask, uint8_t *done)
{
    int32_t s = blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= S) return;
    bool present = coarsest[s] >= j;
    mode[s] = present ? (kList0 | kList1 | kGainNonNeg | kMinPair) : 0;
    gmask[s] = present ? 1 : 0;
    done[s] = present ? 0 : 1;
}

// Balance step test: the side over its bound, how much must leave, how much
// the other side can take.
__global__ void k_mode_balance(int32_t S, const int32_t *nbase, const unsigned long long *segw,
                               const int64_t *max0, const int64_t *max1, uint8_t *done,
                               uint8_t *mode, uint8_t *gmask, int32_t *m, int64_t *need,
                               int64_t *room, int32_t *ccount, LevelInfo *info)
{
    int32_t s = blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= S) return;
    uint8_t md = 0;
    ccount[s] = 0;
    if (!done[s]) {
        int64_t w0 = (int64_t)segw[2 * s], w1 = (int64_t)segw[2 * s + 1];
        int h = -1;
        if (w0 > max0[s]) h = 0;
        else if (w1 > max1[s]) h = 1;
        if (h < 0) {
            done[s] = 1;
        } else {
            md = h ? kList1 : kList0;
            need[s] = h ? w1 - max1[s] : w0 - max0[s];
            room[s] = h ? max0[s] - w0 : max1[s] - w1;
            m[s] = (int32_t)ceil_sqrt_i64(nbase[s + 1] - nbase[s]);
            atomicAdd(&info->flag, 1);
        }
    }
    mode[s] = md;
    gmask[s] = md ? 1 : 0;
}

__global__ __launch_bounds__(kBlock) void k_bal_gather(int32_t N, const int32_t *gain,
                                                       const uint8_t *side, const int32_t *nseg,
                                                       const uint8_t *mode, const int32_t *rsel,
                                                       const uint64_t *thr, int32_t *ccount,
                                                       uint64_t *cand, int32_t stride)
{
    int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (v >= N) return;
    int32_t c;
    uint64_t k;
    if (!sel_eligible(v, gain, side, nseg, mode, &c, &k)) return;
    if (rsel[c] <= 0 || k > thr[c]) return;
    int32_t s = c >> 1;
    int32_t at = atomicAdd(&ccount[s], 1);
    cand[(int64_t)s * stride + at] = k;
}

// One workgroup per balancing segment: sort its candidates, take the shortest
// prefix covering the excess, cut back to what the other side can take, move.
__global__ __launch_bounds__(1024) void k_bal_finish(int32_t S, const uint8_t *mode,
                                                     const int32_t *ccount, uint64_t *cand,
                                                     int32_t stride, int32_t lds_cap,
                                                     const int32_t *nw,
                                                     const int64_t *need, const int64_t *room,
                                                     uint8_t *side, unsigned long long *segw,
                                                     uint8_t *done, int32_t *stuck)
{
    extern __shared__ uint64_t keys_lds[];
    __shared__ int64_t lds64[16];
    __shared__ int64_t carry;
    __shared__ int32_t p1s, ps;
    int32_t s = blockIdx.x;
    uint8_t md = mode[s];
    if (!md) return;
    int h = (md & kList1) ? 1 : 0;
    int32_t cnt = ccount[s];
    int n2 = next_pow2(cnt > 0 ? cnt : 1);
    // sort in LDS when the launch reserved room for it, else in place
    uint64_t *a = n2 <= lds_cap ? keys_lds : cand + (int64_t)s * stride;
    for (int i = threadIdx.x; i < n2; i += blockDim.x)
        a[i] = i < cnt ? cand[(int64_t)s * stride + i] : kNoKey;
    __syncthreads();
    block_bitonic_sort(a, n2);
    int64_t nd = need[s], rm = room[s];
    if (threadIdx.x == 0) {
        carry = 0;
        p1s = cnt;
        ps = 0;
    }
    __syncthreads();
    // prefix weights in sorted order, chunk by chunk
    for (int base = 0; base < cnt; base += blockDim.x) {
        int i = base + threadIdx.x;
        int64_t w = i < cnt ? (int64_t)nw[(uint32_t)(a[i] & 0xffffffffu)] : 0;
        int64_t tot;
        int64_t incl = block_excl_scan(w, lds64, &tot) + w + carry;
        // prefix length i+1 reaches the excess
        if (i < cnt && incl >= nd) atomicMin(&p1s, i + 1);
        __syncthreads();
        if (threadIdx.x == 0) carry += tot;
        __syncthreads();
    }
    int32_t p1 = p1s;
    if (threadIdx.x == 0) carry = 0;
    __syncthreads();
    for (int base = 0; base < p1; base += blockDim.x) {
        int i = base + threadIdx.x;
        int64_t w = i < p1 ? (int64_t)nw[(uint32_t)(a[i] & 0xffffffffu)] : 0;
        int64_t tot;
        int64_t incl = block_excl_scan(w, lds64, &tot) + w + carry;
        if (i < p1 && incl <= rm) atomicMax(&ps, i + 1);
        __syncthreads();
        if (threadIdx.x == 0) carry += tot;
        __syncthreads();
    }
    int32_t p = ps;
    int64_t moved = 0;
    for (int i = threadIdx.x; i < p; i += blockDim.x) {
        uint32_t v = (uint32_t)(a[i] & 0xffffffffu);
        side[v] = (uint8_t)(1 - h);
        moved += nw[v];
    }
    moved = block_sum(moved, lds64);
    if (threadIdx.x == 0) {
        if (p == 0) {
            stuck[s] = 1;
            done[s] = 1;
        } else {
            atomicAdd(&segw[2 * s + h], (unsigned long long)(-moved));
            atomicAdd(&segw[2 * s + 1 - h], (unsigned long long)moved);
        }
    }
}

// Sum of (prefix weights <= room) is monotone, so "largest prefix within
// room" is the count of prefixes within room; the atomicMax above computes it.

}  // namespace bp
