// Per-level pieces of uncoarsening (Algorithms 3 and 5): projection of the
// coarser level's bisection, side weights per segment, and the final step of
// each balance round (sort the <= ceil(sqrt n) candidates of a segment, take
// the shortest prefix that removes the excess, cut back to what the other
// side can take).  Gains and the selections live in uncoarsen.hpp.
#pragma once
#include "level.hpp"

namespace bp {

// selection mode bits per segment
constexpr uint8_t kList0 = 1, kList1 = 2, kGainNonNeg = 4, kMinPair = 8;

// ---- per-level setup ------------------------------------------------------------

// side of level j: projected from level j+1 for segments coarsened past j,
// all-ones start of Algorithm 3 for segments whose coarsest level is j.
// Also zeroes zero[0, nzero) (block 0), for the side weights that follow.
__global__ __launch_bounds__(kBlock) void k_project(int32_t N, int32_t j, const int32_t *nseg,
                                                    const int32_t *coarsest,
                                                    const int32_t *parent,
                                                    const uint8_t *side_coarse, uint8_t *side,
                                                    unsigned long long *zero, int32_t nzero)
{
    if (blockIdx.x == 0)
        for (int32_t i = threadIdx.x; i < nzero; i += blockDim.x) zero[i] = 0ull;
    int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (v >= N) return;
    int32_t c = coarsest[nseg[v]];
    if (c > j) side[v] = side_coarse[parent[v]];
    else if (c == j) side[v] = 1;
}

// Side weights of every segment (chunked; per-segment sums in LDS).
__global__ __launch_bounds__(kBlock) void k_side_weights(int32_t N, const int32_t *nseg,
                                                         const uint8_t *side, const int32_t *nw,
                                                         unsigned long long *segw)
{
    __shared__ unsigned long long acc[kAggLists];
    int64_t lo, hi;
    reduce_chunk(N, gridDim.x, blockIdx.x, lo, hi);
    if (lo >= hi) return;
    int32_t c0 = 2 * nseg[lo], nl = 2 * nseg[hi - 1] + 2 - c0;
    bool local = nl <= kAggLists;
    for (int i = threadIdx.x; i < kAggLists; i += blockDim.x) acc[i] = 0;
    __syncthreads();
    for (int64_t v = lo + threadIdx.x; v < hi; v += blockDim.x) {
        int32_t c = 2 * nseg[v] + side[v];
        unsigned long long w = (unsigned long long)nw[v];
        if (!w) continue;
        if (local) atomicAdd(&acc[c - c0], w);
        else atomicAdd(&segw[c], w);
    }
    __syncthreads();
    if (local)
        for (int i = threadIdx.x; i < nl; i += blockDim.x)
            if (acc[i]) atomicAdd(&segw[c0 + i], acc[i]);
}

constexpr int kLogChunk = 64;  // incidences of a moved node per logged chunk

// What a balance round moved, for the next round's gain update: every moved
// node's incidence range, logged in chunks of 64 (node, first incidence) so
// that the next step is evenly parallel.
struct MoveLog {
    const int32_t *noff;
    int32_t *cnode, *cbeg;
    int32_t *count;  // [0] logged chunks, [1] listed small hyperedges, [2] listed big ones
};

// Logs the moves of the first p keys' nodes (one workgroup).
__device__ __forceinline__ void log_moves(int32_t p, const uint64_t *a, const MoveLog &ml, int64_t *lds64)
{
    __shared__ int32_t base_s;
    for (int32_t base = 0; base < p; base += blockDim.x) {
        int32_t i = base + threadIdx.x;
        int32_t v = 0, b = 0, c = 0;
        if (i < p) {
            v = (int32_t)(uint32_t)(a[i] & 0xffffffffu);
            b = ml.noff[v];
            c = (int32_t)ceil_div(ml.noff[v + 1] - b, kLogChunk);
        }
        int64_t tot;
        int64_t ex = block_excl_scan((int64_t)c, lds64, &tot);
        if (threadIdx.x == 0) base_s = tot ? atomicAdd(&ml.count[0], (int32_t)tot) : 0;
        __syncthreads();
        int32_t o = base_s + (int32_t)ex;
        for (int32_t j = 0; j < c; j++) {
            ml.cnode[o + j] = v;
            ml.cbeg[o + j] = b + j * kLogChunk;
        }
        __syncthreads();
    }
}

// What the balance step of a segment needs besides its sorted candidates.
struct BalFinish {
    const uint8_t *mode;
    const int32_t *nw;
    const int64_t *need, *room;
    uint8_t *side;
    unsigned long long *segw;
    uint8_t *done;
    int32_t *stuck;
    MoveLog ml;
    int32_t *go;          // go[3]: most further rounds a segment is estimated to need
    int64_t *bal_moved;   // [2S] weight moved and rounds run this level
    const int32_t *rsel;  // [2S] nodes each list chose (multi-workgroup rounds; else null)
};

// Balance step of segment s given its candidates a[0..cnt) in ascending
// (gain desc, id asc) order: take the shortest prefix covering the excess,
// cut back to what the other side can take, move it.  One workgroup.
__device__ __forceinline__ void bal_take_prefix(int32_t s, const uint64_t *a, int32_t cnt, const BalFinish &bf, int64_t *lds64)
{
    __shared__ int64_t carry;
    __shared__ int32_t p1s, ps;
    int h = (bf.mode[s] & kList1) ? 1 : 0;
    int64_t nd = bf.need[s], rm = bf.room[s];
    if (threadIdx.x == 0) {
        carry = 0;
        p1s = cnt;
        ps = 0;
    }
    __syncthreads();
    // prefix weights in sorted order, chunk by chunk
    for (int base = 0; base < cnt; base += blockDim.x) {
        int i = base + threadIdx.x;
        int64_t w = i < cnt ? (int64_t)bf.nw[(uint32_t)(a[i] & 0xffffffffu)] : 0;
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
        int64_t w = i < p1 ? (int64_t)bf.nw[(uint32_t)(a[i] & 0xffffffffu)] : 0;
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
        bf.side[v] = (uint8_t)(1 - h);
        moved += bf.nw[v];
    }
    moved = block_sum(moved, lds64);
    if (bf.ml.cnode) log_moves(p, a, bf.ml, lds64);
    if (threadIdx.x == 0) {
        if (p == 0) {
            bf.stuck[s] = 1;
            bf.done[s] = 1;
        } else {
            atomicAdd(&bf.segw[2 * s + h], (unsigned long long)(-moved));
            atomicAdd(&bf.segw[2 * s + 1 - h], (unsigned long long)moved);
            // rounds still needed if later rounds move what the level's
            // rounds moved on average
            int64_t mw = bf.bal_moved[2 * s] + moved, mr = bf.bal_moved[2 * s + 1] + 1;
            bf.bal_moved[2 * s] = mw;
            bf.bal_moved[2 * s + 1] = mr;
            int64_t rest = nd - moved;
            if (rest > 0) {
                int64_t est = mw > 0 ? (rest * mr + mw - 1) / mw : 1;
                atomicMax(&bf.go[3], (int32_t)(est < (1 << 20) ? est : (1 << 20)));
            }
        }
    }
}

// The chosen nodes' weights and incidence ranges (noff[v], noff[v + 1]) in
// their order, gathered by the caller while it ranked them; null: gathered
// by the finish.
struct BalPre {
    const int32_t *w = nullptr, *nb = nullptr, *ne = nullptr;
};

// The balance prefix (Algorithm 5) over the first take keys of a (ascending
// order keys, take <= the workgroup's threads), by the whole workgroup: the
// shortest prefix reaching the excess, cut to what fits the room, moved and
// logged.  h, nd, rm: the segment's over-weight side, excess and room; bm0,
// bm1 (thread 0): its moved weight and rounds so far - loaded by the caller
// ahead of its own work, as pre may be.
__device__ __forceinline__ void bal_finish_block(int32_t s, const uint64_t *a, int32_t take, const BalFinish &bf,
                                                 int h, int64_t nd, int64_t rm, int64_t bm0, int64_t bm1,
                                                 BalPre pre = BalPre{})
{
    __shared__ int64_t lds64[16];
    __shared__ int32_t cnt_scan[16], p1s, fits, logbase;
    __shared__ int64_t movedw;
    const int32_t tid = threadIdx.x;
    if (tid == 0) {
        p1s = take;
        fits = 0;
        movedw = 0;
    }
    // the shortest prefix reaching the excess, cut to what fits the room
    // (weights are non-negative: prefix weights ascend, so each wavefront's
    // first reaching lane and its fitting lanes come from two ballots).  One
    // chosen node a thread: its weight and, for the move log, its incidence
    // range are gathered together after the ranking, and the log's chunk
    // counts are scanned with the weights (the logged nodes are a prefix of
    // the chosen ones, so their offsets are the same prefix sums)
    const bool logm = bf.ml.cnode != nullptr;
    int32_t v = 0, nb = 0, nc = 0;
    int64_t w = 0;
    if (tid < take) {
        v = (int32_t)(uint32_t)(a[tid] & 0xffffffffu);
        if (pre.w) {
            w = pre.w[tid];
            if (logm) {
                nb = pre.nb[tid];
                nc = (int32_t)ceil_div(pre.ne[tid] - nb, kLogChunk);
            }
        } else {
            w = bf.nw[v];
            if (logm) {
                nb = bf.ml.noff[v];
                nc = (int32_t)ceil_div(bf.ml.noff[v + 1] - nb, kLogChunk);
            }
        }
    }
    int64_t incl = wave_incl_scan(w);
    int32_t cincl = wave_incl_scan(nc);
    if ((tid & 63) == 63) {
        lds64[tid >> 6] = incl;
        cnt_scan[tid >> 6] = cincl;
    }
    __syncthreads();
    for (int q = 0; q < (tid >> 6); q++) {
        incl += lds64[q];
        cincl += cnt_scan[q];
    }
    unsigned long long reach = __ballot(tid < take && incl >= nd), fit = __ballot(tid < take && incl <= rm);
    if ((tid & 63) == 0) {
        if (reach) atomicMin(&p1s, (tid & ~63) + __ffsll((long long)reach));
        if (fit) atomicAdd(&fits, __popcll(fit));
    }
    __syncthreads();
    int32_t p = min(p1s, fits);
    if (tid < p) bf.side[v] = (uint8_t)(1 - h);
    if (p > 0 && tid == p - 1) {
        movedw = incl;
        if (logm) logbase = cincl ? atomicAdd(&bf.ml.count[0], cincl) : 0;
    }
    __syncthreads();
    if (logm && tid < p) {
        int32_t o = logbase + cincl - nc;
        for (int32_t j = 0; j < nc; j++) {
            bf.ml.cnode[o + j] = v;
            bf.ml.cbeg[o + j] = nb + j * kLogChunk;
        }
    }
    if (tid == 0) {
        int64_t moved = movedw;
        if (p == 0) {
            bf.stuck[s] = 1;
            bf.done[s] = 1;
        } else {
            atomicAdd(&bf.segw[2 * s + h], (unsigned long long)(-moved));
            atomicAdd(&bf.segw[2 * s + 1 - h], (unsigned long long)moved);
            int64_t mw = bm0 + moved, mr = bm1 + 1;
            bf.bal_moved[2 * s] = mw;
            bf.bal_moved[2 * s + 1] = mr;
            int64_t rest = nd - moved;
            if (rest > 0) {
                int64_t est = mw > 0 ? (rest * mr + mw - 1) / mw : 1;
                atomicMax(&bf.go[3], (int32_t)(est < (1 << 20) ? est : (1 << 20)));
            }
        }
    }
}

constexpr int32_t kRankSortMax = 1024;  // candidates ordered by counting up to this many
constexpr int32_t kBalGather = 512;     // balance candidates a segment may gather, at least

// One workgroup per balancing segment: sort its gathered candidates, then
// the prefix step.  The launch reserves lds_cap keys of LDS (lds_cap may be
// 0): short lists are ordered by counting from one LDS copy into a second
// one behind it and finished by one wavefront, longer ones sorted by a
// bitonic network in LDS, or in place when they do not fit.
__global__ __launch_bounds__(1024) void k_bal_finish(int32_t S, const int32_t *ccount, uint64_t *cand,
                                                     int32_t stride, int32_t lds_cap, BalFinish bf)
{
    extern __shared__ uint64_t keys_lds[];
    __shared__ int64_t lds64[16];
    int32_t s = blockIdx.x;
    const uint8_t md = bf.mode[s];
    if (!md) return;
    int32_t cnt = ccount[s];
    // the segment's balance state, loaded ahead of the candidates' ordering
    const int h = (md & kList1) ? 1 : 0;
    const int64_t nd = bf.need[s], rm = bf.room[s];
    int64_t bm0 = 0, bm1 = 0;
    if (threadIdx.x == 0) {
        bm0 = bf.bal_moved[2 * s];
        bm1 = bf.bal_moved[2 * s + 1];
    }
    // a selection that stopped at a whole bin gathered more nodes than the
    // list chose: the chosen ones are the first rsel in order
    int32_t take = cnt;
    if (bf.rsel) {
        int32_t r = bf.rsel[2 * s + ((bf.mode[s] & kList1) ? 1 : 0)];
        take = r < cnt ? r : cnt;
    }
    const uint64_t *src = cand + (int64_t)s * stride;
    if (cnt <= kRankSortMax && 2 * cnt <= lds_cap) {
        for (int i = threadIdx.x; i < cnt; i += blockDim.x) keys_lds[i] = src[i];
        __syncthreads();
        block_rank_sort(keys_lds, keys_lds + cnt, cnt);
        bal_finish_block(s, keys_lds + cnt, take, bf, h, nd, rm, bm0, bm1);
        return;
    }
    int n2 = next_pow2(cnt > 0 ? cnt : 1);
    uint64_t *a = n2 <= lds_cap ? keys_lds : cand + (int64_t)s * stride;
    for (int i = threadIdx.x; i < n2; i += blockDim.x)
        a[i] = i < cnt ? src[i] : kNoKey;
    __syncthreads();
    block_bitonic_sort(a, n2);
    __syncthreads();
    if (take <= (int32_t)blockDim.x) bal_finish_block(s, a, take, bf, h, nd, rm, bm0, bm1);
    else bal_take_prefix(s, a, take, bf, lds64);
}

}  // namespace bp
