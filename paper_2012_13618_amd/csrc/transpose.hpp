// Node-major incidence of a level: for every node, the ascending list of its
// hyperedges (the bipartite graph of Section 1.1 read from the node side).
//
// Built by a stable LSD radix sort of (node id, hyperedge id) pairs taken in
// pin order, 8-bit digits: per-tile digit histograms, one prefix scan of the
// (digit, tile) counts, and a stable scatter whose in-tile ranks come from
// wavefront ballots and which writes each tile out in digit order.  Node offsets are binary searches into the sorted keys.
//
// With it, the per-node steps - the 64-bit minimum of Algorithm 1 and the gain
// sum of Algorithm 4 (uncoarsen.hpp) - are gathers over a node's own
// hyperedges with no atomics, so a node contained in very many hyperedges (a
// heavy coarse node) is reduced by one workgroup instead of receiving that
// many atomic updates.
#pragma once
#include "level.hpp"
#include "scan.hpp"

namespace bp {

constexpr int kRsItems = 16;
constexpr int kRsTile = kBlock * kRsItems;   // 4096 pairs per tile
constexpr int kNodeSmallMax = 32;            // node degree: one thread
constexpr int kNodeMidMax = 2048;            // one wavefront; above: chunks
constexpr int kNodeChunk = 4096;             // incidences per workgroup for big nodes

__global__ __launch_bounds__(kBlock) void k_rs_hist(const uint32_t *keys, int64_t n, int shift,
                                                    uint32_t *counts, int64_t ntiles)
{
    __shared__ uint32_t h[256];
    h[threadIdx.x] = 0;
    __syncthreads();
    int64_t base = (int64_t)blockIdx.x * kRsTile;
#pragma unroll 4
    for (int r = 0; r < kRsItems; r++) {
        int64_t i = base + r * kBlock + threadIdx.x;
        if (i < n) atomicAdd(&h[(keys[i] >> shift) & 255u], 1u);
    }
    __syncthreads();
    counts[(int64_t)threadIdx.x * ntiles + blockIdx.x] = h[threadIdx.x];
}

// Stable scatter of one tile.  Each wavefront ranks its own 1024 consecutive
// items (64 a step, in order) against a digit counter row of its own, so no
// workgroup barrier separates the steps; one scan over the digits then gives
// every item its place in the tile's digit order, the tile is staged in that
// order in LDS, and it is written out from there: consecutive threads write
// consecutive addresses of a digit's run.
static_assert(kBlock == 256, "one digit per thread");
__global__ __launch_bounds__(kBlock) void k_rs_scatter(const uint32_t *kin, const int32_t *vin,
                                                       int64_t n, int shift,
                                                       const uint32_t *offs, int64_t ntiles,
                                                       uint32_t *kout, int32_t *vout)
{
    __shared__ uint32_t base[256], tstart[256];
    __shared__ uint32_t wrun[kBlock / 64][256];
    __shared__ uint32_t lk[kRsTile];
    __shared__ int32_t lv[kRsTile];
    __shared__ uint32_t lds[16];
    const int t = threadIdx.x, w = t >> 6, lane = t & 63;
    const unsigned long long below = (1ull << lane) - 1;
    const int64_t tile = (int64_t)blockIdx.x * kRsTile, wb = tile + (int64_t)w * (kRsItems * 64);
    base[t] = offs[(int64_t)t * ntiles + blockIdx.x];
    // this wavefront's items in registers first: their loads in flight together
    uint32_t keys[kRsItems], rk[kRsItems];
    int32_t vals[kRsItems];
#pragma unroll
    for (int r = 0; r < kRsItems; r++) {
        int64_t i = wb + r * 64 + lane;
        keys[r] = i < n ? kin[i] : 0u;
        vals[r] = i < n ? vin[i] : 0;
    }
    for (int d = lane; d < 256; d += 64) wrun[w][d] = 0;
    // rank of each item among the earlier items of its wavefront with its digit
    // (the row is this wavefront's alone; its LDS accesses execute in order)
#pragma unroll
    for (int r = 0; r < kRsItems; r++) {
        bool valid = wb + r * 64 + lane < n;
        uint32_t dig = (keys[r] >> shift) & 255u;
        unsigned long long same = __ballot(valid);
#pragma unroll
        for (int b = 0; b < 8; b++) {
            unsigned long long m = __ballot((dig >> b) & 1u);
            same &= ((dig >> b) & 1u) ? m : ~m;
        }
        int rank = __popcll(same & below);
        uint32_t before = wrun[w][dig];
        rk[r] = before + (uint32_t)rank;
        if (valid && rank == 0) wrun[w][dig] = before + (uint32_t)__popcll(same);
    }
    __syncthreads();
    // per digit (thread t): the earlier wavefronts' counts, and the digit's start
    // in the tile's order
    uint32_t c[kBlock / 64], tot = 0;
#pragma unroll
    for (int x = 0; x < kBlock / 64; x++) {
        c[x] = wrun[x][t];
        tot += c[x];
    }
    uint32_t all;
    uint32_t st = block_excl_scan(tot, lds, &all);
    tstart[t] = st;
    uint32_t acc = st;
#pragma unroll
    for (int x = 0; x < kBlock / 64; x++) {
        wrun[x][t] = acc;
        acc += c[x];
    }
    __syncthreads();
#pragma unroll
    for (int r = 0; r < kRsItems; r++) {
        if (wb + r * 64 + lane >= n) continue;
        uint32_t dig = (keys[r] >> shift) & 255u;
        uint32_t lp = wrun[w][dig] + rk[r];
        lk[lp] = keys[r];
        lv[lp] = vals[r];
    }
    __syncthreads();
    const int32_t tn = (int32_t)min<int64_t>(kRsTile, n - tile);
#pragma unroll 4
    for (int32_t j = t; j < tn; j += kBlock) {
        uint32_t key = lk[j];
        uint32_t dig = (key >> shift) & 255u;
        uint32_t pos = base[dig] + ((uint32_t)j - tstart[dig]);
        kout[pos] = key;
        vout[pos] = lv[j];
    }
}

// pins -> (node, hyperedge) pairs in pin order: the nodes are the pins
// themselves, so only each pin's hyperedge is written
struct ExpandPairsOp {
    const int32_t *off;
    int32_t *vals;
    template <int S> __device__ __forceinline__ void run(int64_t vb, int32_t count, const int32_t *list) const;
};

template <int S>
__device__ __forceinline__ void ExpandPairsOp::run(int64_t vb, int32_t count, const int32_t *list) const
{
    int lane, stride;
    int32_t e = sched_hedge_at<S>(vb, count, list, lane, stride);
    if (e < 0) return;
    int32_t b = off[e], d = off[e + 1] - b;
    if (!thread_split<S>(d)) return;
    for (int i = lane; i < d; i += stride) vals[b + i] = e;
}

// noff[v] = first position of node v in the sorted keys (lower bound)
__global__ __launch_bounds__(kBlock) void k_node_offsets(const uint32_t *keys, int64_t P,
                                                         int32_t N, int32_t *noff)
{
    int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (v > N) return;
    int64_t lo = 0, hi = P;
    while (lo < hi) {
        int64_t mid = (lo + hi) >> 1;
        if ((int64_t)keys[mid] < v) lo = mid + 1;
        else hi = mid;
    }
    noff[v] = (int32_t)lo;
}

// Node buckets, staged per workgroup like the hyperedge lists.
constexpr int kClsNodes = 2048;

__global__ __launch_bounds__(kBlock) void k_classify_nodes(int32_t N, const int32_t *noff,
                                                           int32_t *lmid, int32_t *lbig,
                                                           int32_t *counters)
{
    __shared__ int32_t items[2][kClsNodes];
    __shared__ int32_t cnt[2], base[2];
    int64_t first = (int64_t)blockIdx.x * kClsNodes;
    if (first >= N) return;
    if (threadIdx.x < 2) cnt[threadIdx.x] = 0;
    __syncthreads();
    for (int r = 0; r < kClsNodes / kBlock; r++) {
        int64_t v = first + r * kBlock + threadIdx.x;
        int32_t d = v < N ? noff[v + 1] - noff[v] : 0;
        lds_append(d > kNodeSmallMax && d <= kNodeMidMax, (int32_t)v, items[0], &cnt[0]);
        lds_append(d > kNodeMidMax, (int32_t)v, items[1], &cnt[1]);
    }
    __syncthreads();
    if (threadIdx.x < 2) base[threadIdx.x] = cnt[threadIdx.x] ? atomicAdd(&counters[threadIdx.x], cnt[threadIdx.x]) : 0;
    __syncthreads();
    for (int i = threadIdx.x; i < cnt[0]; i += blockDim.x) lmid[base[0] + i] = items[0][i];
    for (int i = threadIdx.x; i < cnt[1]; i += blockDim.x) lbig[base[1] + i] = items[1][i];
}

// Chunk table of the big nodes: one workgroup walks them in tiles of 256 and
// places each node's chunks after a prefix sum of the chunk counts.
__global__ __launch_bounds__(kBlock) void k_big_chunks(const int32_t *lnbig, const int32_t *noff,
                                                       int32_t *ncount, int32_t *chunk_node,
                                                       int32_t *chunk_beg, int32_t *chunk_big,
                                                       int32_t *big_chunks, int32_t *bigslot)
{
    __shared__ int32_t lds[16];
    int32_t cb = ncount[1], q0 = 0;
    for (int32_t t = 0; t < cb; t += kBlock) {
        int32_t i = t + threadIdx.x;
        int32_t v = 0, b = 0, n = 0;
        if (i < cb) {
            v = lnbig[i];
            b = noff[v];
            n = (int32_t)ceil_div(noff[v + 1] - b, kNodeChunk);
            big_chunks[i] = n;
            bigslot[v] = i;
        }
        int32_t tot;
        int32_t q = q0 + block_excl_scan(n, lds, &tot);
        for (int32_t j = 0; j < n; j++) {
            chunk_node[q + j] = v;
            chunk_beg[q + j] = b + j * kNodeChunk;
            chunk_big[q + j] = i;
        }
        q0 += tot;
    }
    if (threadIdx.x == 0) ncount[2] = q0;
}

// Largest node degree and largest hyperedge weight of a level (the gain span
// bound of the selection), for up to kBoundLevels levels in one launch (grid y
// = level): out[2 j], out[2 j + 1] for level y of the launch.
constexpr int kBoundLevels = 32;
struct LevelBoundArgs {
    const int32_t *noff[kBoundLevels];
    const int32_t *hw[kBoundLevels];
    int32_t N[kBoundLevels], E[kBoundLevels];
};

__global__ __launch_bounds__(kBlock) void k_level_bound(LevelBoundArgs a, unsigned long long *outs)
{
    int j = blockIdx.y;
    int32_t N = a.N[j], E = a.E[j];
    const int32_t *noff = a.noff[j], *hw = a.hw[j];
    unsigned long long *out = outs + 2 * j;
    int64_t n = N > E ? N : E, lo, hi;
    reduce_chunk(n, gridDim.x, blockIdx.x, lo, hi);
    unsigned long long d = 0, w = 0;
    for (int64_t i = lo + threadIdx.x; i < hi; i += blockDim.x) {
        if (i < N) {
            unsigned long long x = (unsigned long long)(noff[i + 1] - noff[i]);
            d = x > d ? x : d;
        }
        if (i < E) {
            unsigned long long x = (unsigned long long)hw[i];
            w = x > w ? x : w;
        }
    }
    __shared__ unsigned long long ld[16], lw[16];
    d = wave_max(d);
    w = wave_max(w);
    if ((threadIdx.x & 63) == 0) {
        ld[threadIdx.x >> 6] = d;
        lw[threadIdx.x >> 6] = w;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int i = 1; i < (int)(blockDim.x >> 6); i++) {
            d = ld[i] > d ? ld[i] : d;
            w = lw[i] > w ? lw[i] : w;
        }
        if (d) atomicMax(&out[0], d);
        if (w) atomicMax(&out[1], w);
    }
}

// ---- Algorithm 1, node side ------------------------------------------------------

// Big nodes: each workgroup takes one chunk and folds its minimum in with a
// 64-bit atomicMin (key[] starts at the no-hyperedge value).
__global__ __launch_bounds__(kBlock) void k_match_chunks(const int32_t *ncount, const int32_t *chunk_node,
                                                         const int32_t *chunk_beg, const int32_t *noff,
                                                         const int32_t *inc, const int32_t *nseg,
                                                         const uint8_t *sact, const uint64_t *hkey,
                                                         unsigned long long *key)
{
    __shared__ unsigned long long lds[16];
    int32_t q = blockIdx.x;
    if (q >= ncount[2]) return;
    int32_t v = chunk_node[q];
    if (!sact[nseg[v]]) return;
    int32_t b = chunk_beg[q], e = min(b + kNodeChunk, noff[v + 1]);
    unsigned long long m = kNoKey;
    for (int32_t i = b + threadIdx.x; i < e; i += blockDim.x) {
        unsigned long long k = hkey[inc[i]];
        m = k < m ? k : m;
    }
    m = block_min(m, lds);
    if (threadIdx.x == 0 && m != kNoKey) atomicMin(&key[v], m);
}

__global__ __launch_bounds__(kBlock) void k_hedge_keys(int32_t E, const int32_t *off,
                                                       const int32_t *hw, const int32_t *hseg,
                                                       const int32_t *hbase, const uint8_t *sact,
                                                       int policy, uint64_t *hkey)
{
    int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= E) return;
    int32_t s = hseg[e];
    hkey[e] = sact[s] ? hedge_key(policy, (uint32_t)(e - hbase[s]), off[e + 1] - off[e], hw[e]) : kNoKey;
}

// Node schedule: SMALL = every node of degree <= 32 by one thread, WAVE/BLOCK
// = listed nodes, their count read on the device (the grid is an upper bound).
template <int S>
__device__ __forceinline__ int32_t sched_node(int64_t vb, int32_t count, const int32_t *dcount,
                                              const int32_t *list, int &lane, int &stride)
{
    return sched_hedge_at<S>(vb, S == SMALL ? count : *dcount, list, lane, stride);
}

// Block vb of schedule S of Algorithm 1's per-node minimum.
template <int S>
__device__ __forceinline__ void match_nodes(int64_t vb, int32_t count, const int32_t *dcount, const int32_t *list,
                                            const int32_t *noff, const int32_t *inc, const int32_t *nseg,
                                            const uint8_t *sact, const uint64_t *hkey, uint64_t *key)
{
    __shared__ unsigned long long lds[16];
    int lane, stride;
    int32_t v = sched_node<S>(vb, count, dcount, list, lane, stride);
    if (v < 0) return;
    int32_t b = noff[v], d = noff[v + 1] - b;
    if (S == SMALL && d > kNodeSmallMax) {
        if (d > kNodeMidMax) key[v] = kNoKey;  // start value of the chunked minimum
        return;
    }
    unsigned long long m = kNoKey;
    if (sact[nseg[v]])
        for (int i = lane; i < d; i += stride) {
            unsigned long long k = hkey[inc[b + i]];
            m = k < m ? k : m;
        }
    m = group_min<S>(m, lds);
    if (lane == 0) key[v] = m;
}

// Nodes of degree <= 32 one per thread (blocks [0, ceil(N / kBlock))) and the
// listed mid nodes one per wavefront (the other blocks; their count is read
// on the device, the grid is an upper bound), in one launch.
__global__ __launch_bounds__(kBlock) void k_match_sw(int32_t N, const int32_t *dcount, const int32_t *lnmid,
                                                     const int32_t *noff, const int32_t *inc, const int32_t *nseg,
                                                     const uint8_t *sact, const uint64_t *hkey, uint64_t *key)
{
    int64_t b = blockIdx.x, ns = ceil_div(N, kBlock);
    if (b < ns) match_nodes<SMALL>(b, N, dcount, nullptr, noff, inc, nseg, sact, hkey, key);
    else match_nodes<WAVE>(b - ns, N, dcount, lnmid, noff, inc, nseg, sact, hkey, key);
}

}  // namespace bp
