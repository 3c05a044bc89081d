// One coarsening step over all active segments of a level (Algorithms 1, 2).
//
//  match     Algorithm 1: every node takes the 64-bit minimum of
//            (priority << 32 | hash(local id + 1)) over its hyperedges (a
//            per-node reduction over the node-major incidence); the hash is a
//            bijection, so the winning hyperedge is decoded from the key.
//  group     Algorithm 2, first loop: |S(e)| and the weight of S(e) by
//            integer atomics; sets of two or more are merged.
//  attach    Algorithm 2, second loop: a singleton joins the lightest merged
//            set among its hyperedge's pins (ties: smaller node id) as a
//            64-bit min of (set weight << 32 | node id).
//  ids       coarse node ids by prefix scan over group leaders (smallest
//            member), weights summed with atomics.
//  hedges    Algorithm 2, third loop: sorted distinct parents per hyperedge
//            (registers / wave LDS / workgroup LDS / global by degree),
//            kept when at least two.
//  dedup     identical pin sets merged: fingerprint hash table with atomicMin
//            of the source id, then an exact pin-by-pin check; weights added
//            into the surviving (smallest) source; compaction by scan.
#pragma once
#include "level.hpp"
#include "scan.hpp"

namespace bp {

constexpr uint64_t kEmptySlot = ~0ull;

struct CoarsenBufs {
    uint64_t *key;     // [N]
    int32_t *match;    // [N]
    int32_t *grp;      // [N]
    int32_t *cid;      // [N]
    uint64_t *cg;      // [E] nodes matched to the hyperedge << 32 | their weight
    int32_t *lead;     // [E]
    int32_t *qpins;    // [P]
    int32_t *qlen;     // [E]
    uint64_t *fp;      // [E]
    int32_t *hslot;    // [E]
    int32_t *rep;      // [E]
    int32_t *wsum;     // [E]
    int32_t *hdst;     // [E]
    int32_t *hb_tmp;   // [S]
    uint64_t *tkeys;   // [T]
    int32_t *tmin;     // [T]
    int32_t tmask;
    int32_t *counters; // [8]: unresolved, nmid, nbig, nhuge
    int32_t *totN;     // scan total
    uint64_t *totEP;   // scan total
    int32_t *huge_scratch;
};

// Also Algorithm 1's hyperedge keys (what k_hedge_keys computes): hkey[e].
struct HedgeKeyArgs {
    const int32_t *off, *hw, *hseg, *hbase;
    const uint8_t *sact;
    int policy;
    uint64_t *hkey;
};

__global__ void k_coarsen_init(int32_t N, int32_t E, int64_t T, uint64_t *key, int32_t *grp,
                               int32_t *cnw, uint64_t *cg, int32_t *lead,
                               int32_t *wsum, uint64_t *tkeys, int32_t *tmin, int32_t *counters,
                               HedgeKeyArgs hk)
{
    int64_t n = N > E ? N : E;
    if (T > n) n = T;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x) {
        if (i < N) {
            key[i] = kNoKey;
            grp[i] = -1;
            cnw[i] = 0;
        }
        if (i < E) {
            cg[i] = 0;
            lead[i] = INT32_MAX;
            wsum[i] = 0;
            int32_t s = hk.hseg[i];
            hk.hkey[i] = hk.sact[s] ? hedge_key(hk.policy, (uint32_t)(i - hk.hbase[s]), hk.off[i + 1] - hk.off[i],
                                                hk.hw[i])
                                    : kNoKey;
        }
        if (i < T) {
            tkeys[i] = kEmptySlot;
            tmin[i] = INT32_MAX;
        }
        if (i < 8) counters[i] = 0;
    }
}

__global__ __launch_bounds__(kBlock) void k_decode(int32_t N, const uint64_t *key,
                                                   const int32_t *nseg, const int32_t *hbase,
                                                   const uint8_t *sact, const int32_t *nw,
                                                   int32_t *match, uint64_t *cg)
{
    int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (v >= N) return;
    int32_t s = nseg[v];
    uint64_t k = key[v];
    if (!sact[s] || k == kNoKey) {
        match[v] = -1;
        return;
    }
    int32_t e = hbase[s] + (int32_t)(fmix32_inv((uint32_t)k) - 1u);
    match[v] = e;
    // count and weight in one atomic: a weight sum stays below 2^31, so the
    // low half never carries into the count
    atomicAdd((unsigned long long *)&cg[e], (1ull << 32) | (uint32_t)nw[v]);
}

struct AttachOp {
    const int32_t *off, *pins, *hseg;
    const uint8_t *sact;
    const int32_t *match;
    const uint64_t *cg;
    int32_t *grp;
    template <int S> __device__ __forceinline__ void run(int64_t vb, int32_t count, const int32_t *list) const;
};

template <int S>
__device__ __forceinline__ void AttachOp::run(int64_t vb, int32_t count, const int32_t *list) const
{
    __shared__ unsigned long long lds[16];
    int lane, stride;
    int32_t e = sched_hedge_at<S>(vb, count, list, lane, stride);
    if (e < 0) return;
    int32_t b = off[e], d = off[e + 1] - b;
    if (!thread_split<S>(d)) return;
    if ((cg[e] >> 32) != 1 || !sact[hseg[e]]) return;
    unsigned long long best = kNoKey, uu = kNoKey;
    for (int i = lane; i < d; i += stride) {
        int32_t v = pins[b + i];
        int32_t m = match[v];
        if (m == e) {
            uu = (unsigned long long)v;
        } else {
            uint64_t x = cg[m];
            if ((x >> 32) >= 2) {
                unsigned long long c = (x << 32) | (uint32_t)v;
                best = c < best ? c : best;
            }
        }
    }
    best = group_min<S>(best, lds);
    uu = group_min<S>(uu, lds);
    if (lane == 0 && best != kNoKey) grp[(int32_t)uu] = match[(int32_t)(best & 0xffffffffu)];
}

__global__ __launch_bounds__(kBlock) void k_lead(int32_t N, const int32_t *nseg,
                                                 const uint8_t *sact, const int32_t *match,
                                                 const uint64_t *cg, int32_t *grp, int32_t *lead)
{
    int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (v >= N || !sact[nseg[v]]) return;
    int32_t m = match[v];
    int32_t g = (m >= 0 && (cg[m] >> 32) >= 2) ? m : grp[v];
    grp[v] = g;
    if (g >= 0) atomicMin(&lead[g], (int32_t)v);
}

__global__ __launch_bounds__(kBlock) void k_parent(int32_t N, const int32_t *nseg,
                                                   const uint8_t *sact, const int32_t *grp,
                                                   const int32_t *lead, const int32_t *cid,
                                                   const int32_t *nw, int32_t *parent,
                                                   int32_t *cnw, int32_t *cnseg)
{
    int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (v >= N) return;
    int32_t s = nseg[v];
    if (!sact[s]) return;
    int32_t g = grp[v];
    int32_t l = g < 0 ? (int32_t)v : lead[g];
    int32_t c = cid[l];
    parent[v] = c;
    atomicAdd(&cnw[c], nw[v]);
    if (l == v) cnseg[c] = s;
}

__device__ __forceinline__ uint64_t fp_finish(uint64_t sum, int32_t len)
{
    uint64_t f = sum + (uint64_t)len * 0x9E3779B97F4A7C15ull;
    return f == kEmptySlot ? f - 1 : f;
}
__device__ __forceinline__ uint64_t fp_term(int32_t q, uint64_t salt)
{
    return mix64((uint64_t)(uint32_t)q + salt);
}

// Parents of a hyperedge of up to N pins (N a power of two) sorted by one thread
// in registers by a bitonic network (padding INT32_MAX sorts last), then the
// distinct ones written in order with their fingerprint.
template <int N>
__device__ __forceinline__ void qbuild_regs(int64_t e, int32_t b, int32_t d, const int32_t *pins,
                                            const int32_t *parent, int32_t *qpins, int32_t *qlen, uint64_t *fp)
{
    int32_t q[N];
#pragma unroll
    for (int i = 0; i < N; i++) q[i] = i < d ? parent[pins[b + i]] : INT32_MAX;
#pragma unroll
    for (int k = 2; k <= N; k <<= 1)
#pragma unroll
        for (int j = k >> 1; j > 0; j >>= 1)
#pragma unroll
            for (int i = 0; i < N; i++) {
                int p = i ^ j;
                if (p > i) {
                    bool up = (i & k) == 0;
                    int32_t x = q[i], y = q[p];
                    bool sw = (x > y) == up;
                    q[i] = sw ? y : x;
                    q[p] = sw ? x : y;
                }
            }
    int32_t len = 0;
    uint64_t sum = 0;
#pragma unroll
    for (int i = 0; i < N; i++) {
        bool first = i < d && (i == 0 || q[i] != q[i - 1]);
        if (first) {
            qpins[b + len] = q[i];
            sum += fp_term(q[i], 0);
            len++;
        }
    }
    qlen[e] = len >= 2 ? len : 0;
    fp[e] = fp_finish(sum, len);
}

// Third loop of Algorithm 2 for hyperedges of degree <= 8: parents sorted in
// registers by an odd-even transposition network; 9..16 pins by the bitonic
// network above (a wavefront's shuffles would cost more per hyperedge; a
// 32-key network would take registers the common small case needs for
// occupancy).  Block vb of the one-thread-per-hyperedge sweep.
constexpr int32_t kQbuildThreadMax = 16;
__device__ __forceinline__ void qbuild_small(int64_t vb, int32_t E, const int32_t *off, const int32_t *pins,
                                             const int32_t *hseg, const uint8_t *sact, const int32_t *parent,
                                             int32_t *qpins, int32_t *qlen, uint64_t *fp)
{
    int64_t e = vb * blockDim.x + threadIdx.x;
    if (e >= E) return;
    int32_t b = off[e], d = off[e + 1] - b;
    if (d > kQbuildThreadMax) return;
    if (!sact[hseg[e]]) {
        qlen[e] = 0;
        return;
    }
    if (d > kSmallMax) {
        qbuild_regs<kQbuildThreadMax>(e, b, d, pins, parent, qpins, qlen, fp);
        return;
    }
    int32_t q[kSmallMax];
#pragma unroll
    for (int i = 0; i < kSmallMax; i++) q[i] = i < d ? parent[pins[b + i]] : INT32_MAX;
#pragma unroll
    for (int r = 0; r < kSmallMax; r++) {
#pragma unroll
        for (int i = r & 1; i + 1 < kSmallMax; i += 2) {
            int32_t x = q[i], y = q[i + 1];
            q[i] = x < y ? x : y;
            q[i + 1] = x < y ? y : x;
        }
    }
    int32_t len = 0;
    uint64_t sum = 0;
#pragma unroll
    for (int i = 0; i < kSmallMax; i++) {
        bool first = i < d && (i == 0 || q[i] != q[i - 1]);
        if (first) {
            qpins[b + len] = q[i];
            sum += fp_term(q[i], 0);
            len++;
        }
    }
    qlen[e] = len >= 2 ? len : 0;
    fp[e] = fp_finish(sum, len);
}

// Ascending bitonic sort of 64*R keys held R per lane (key i = lane*R + t),
// entirely in registers: steps across lanes use shuffles, steps inside a lane
// are plain compare-exchanges.
template <int R> __device__ __forceinline__ void wave_sort_regs(int32_t (&x)[R])
{
    const int lane = threadIdx.x & 63;
#pragma unroll
    for (int k = 2; k <= 64 * R; k <<= 1) {
#pragma unroll
        for (int j = k >> 1; j > 0; j >>= 1) {
            if (j >= R) {
                int lj = j / R;
#pragma unroll
                for (int t = 0; t < R; t++) {
                    int i = lane * R + t;
                    int32_t y = __shfl_xor(x[t], lj, 64);
                    bool up = (i & k) == 0, lower = (i & j) == 0;
                    int32_t mn = x[t] < y ? x[t] : y, mx = x[t] < y ? y : x[t];
                    x[t] = (lower == up) ? mn : mx;
                }
            } else {
#pragma unroll
                for (int t = 0; t < R; t++) {
                    int p = t ^ j;
                    if (p > t) {
                        int i = lane * R + t;
                        bool up = (i & k) == 0;
                        int32_t a = x[t], b = x[p];
                        bool sw = (a > b) == up;
                        x[t] = sw ? b : a;
                        x[p] = sw ? a : b;
                    }
                }
            }
        }
    }
}

// Distinct keys of a sorted register tile (first d keys valid) written to
// dst in order; returns the count and the fingerprint sum.
template <int R>
__device__ __forceinline__ int32_t wave_unique_emit(const int32_t (&x)[R], int32_t d, int32_t *dst,
                                                    uint64_t *sum_out)
{
    const int lane = threadIdx.x & 63;
    int32_t prev_last = __shfl_up(x[R - 1], 1, 64);
    int flags = 0, cnt = 0;
    uint64_t sum = 0;
#pragma unroll
    for (int t = 0; t < R; t++) {
        int i = lane * R + t;
        int32_t before = t == 0 ? prev_last : x[t > 0 ? t - 1 : 0];
        bool first = i < d && (i == 0 || x[t] != before);
        if (first) {
            flags |= 1 << t;
            cnt++;
            sum += fp_term(x[t], 0);
        }
    }
    int32_t incl = wave_incl_scan(cnt);
    int32_t len = __shfl(incl, 63, 64);
    int32_t pos = incl - cnt;
#pragma unroll
    for (int t = 0; t < R; t++)
        if (flags & (1 << t)) dst[pos++] = x[t];
    *sum_out = wave_sum(sum);
    return len;
}

// Degree 17..256: one wavefront per hyperedge, parents sorted in registers
// (block vb of that sweep).
__device__ __forceinline__ void qbuild_wave(int64_t vb, int32_t count, const int32_t *list, const int32_t *off,
                                            const int32_t *pins, const int32_t *hseg, const uint8_t *sact,
                                            const int32_t *parent, int32_t *qpins, int32_t *qlen, uint64_t *fp)
{
    int lane = threadIdx.x & 63;
    int64_t w = (vb * blockDim.x + threadIdx.x) >> 6;
    if (w >= count) return;
    int32_t e = list[w];
    int32_t b = off[e], d = off[e + 1] - b;
    if (d <= kQbuildThreadMax) return;  // the one-thread sweep took it
    if (!sact[hseg[e]]) {
        if (lane == 0) qlen[e] = 0;
        return;
    }
    int32_t len;
    uint64_t sum;
    if (d <= 64) {
        int32_t x[1];
        x[0] = lane < d ? parent[pins[b + lane]] : INT32_MAX;
        wave_sort_regs<1>(x);
        len = wave_unique_emit<1>(x, d, qpins + b, &sum);
    } else {
        int32_t x[4];
#pragma unroll
        for (int t = 0; t < 4; t++) {
            int i = lane * 4 + t;
            x[t] = i < d ? parent[pins[b + i]] : INT32_MAX;
        }
        wave_sort_regs<4>(x);
        len = wave_unique_emit<4>(x, d, qpins + b, &sum);
    }
    if (lane == 0) {
        qlen[e] = len >= 2 ? len : 0;
        fp[e] = fp_finish(sum, len);
    }
}

// Both sweeps in one launch: blocks [0, ceil(E / kBlock)) one thread per
// hyperedge, the rest one wavefront per listed mid hyperedge.
__global__ __launch_bounds__(kBlock) void k_qbuild_sw(int32_t E, int32_t nmid, const int32_t *lmid,
                                                      const int32_t *off, const int32_t *pins,
                                                      const int32_t *hseg, const uint8_t *sact,
                                                      const int32_t *parent, int32_t *qpins, int32_t *qlen,
                                                      uint64_t *fp)
{
    int64_t b = blockIdx.x, ns = ceil_div(E, kBlock);
    if (b < ns) qbuild_small(b, E, off, pins, hseg, sact, parent, qpins, qlen, fp);
    else qbuild_wave(b - ns, nmid, lmid, off, pins, hseg, sact, parent, qpins, qlen, fp);
}

// Sorted distinct parents of one hyperedge by a whole workgroup: a is a
// power-of-two buffer (LDS for degree <= 8192, else global scratch), sorted,
// its first d entries the hyperedge's parents.  Each wavefront walks its own
// contiguous part of a, 64 entries a step: a first sweep counts the distinct
// values by ballots, one pass over the wavefronts' counts gives each its
// start, and a second sweep writes them - two barriers for the whole list.
__device__ void block_unique_emit(const int32_t *a, int n2, int32_t d, int32_t b, int32_t *qpins,
                                  int32_t *len_out, uint64_t *sum_out)
{
    __shared__ int32_t wtot[16];
    __shared__ uint64_t ldsu[16];
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6, nw = blockDim.x >> 6;
    const int per = n2 / nw;  // a multiple of 64: n2 >= 64 * the wavefronts
    const int i0 = w * per;
    const unsigned long long below = (1ull << lane) - 1;
    int32_t c = 0;
    for (int st = 0; st < per && i0 + st < d; st += 64) {
        int i = i0 + st + lane;
        bool first = i < d && (i == 0 || a[i] != a[i - 1]);
        c += __popcll(__ballot(first));
    }
    if (lane == 0) wtot[w] = c;
    __syncthreads();
    int32_t at = 0, tot = 0;
    for (int x = 0; x < nw; x++) {
        int32_t v = wtot[x];
        if (x < w) at += v;
        tot += v;
    }
    uint64_t sum = 0;
    for (int st = 0; st < per && i0 + st < d; st += 64) {
        int i = i0 + st + lane;
        int32_t x = a[i];
        bool first = i < d && (i == 0 || x != a[i - 1]);
        unsigned long long bm = __ballot(first);
        if (first) {
            qpins[b + at + __popcll(bm & below)] = x;
            sum += fp_term(x, 0);
        }
        at += __popcll(bm);
    }
    sum = block_sum(sum, ldsu);
    *len_out = tot;
    *sum_out = sum;
}

// Big hyperedges (the listed ones above 256 pins), in two launches: up to
// kQWaveMax pins a wavefront each, the parents sorted in registers (8 or 16 a
// lane), four at once in a workgroup and without barriers
// (k_qbuild_big_waves, workgroup b takes list entries 4b .. 4b+3); the larger
// ones (up to kBigMax) a workgroup each, sorted in LDS (k_qbuild_block).
constexpr int32_t kQWaveMax = 1024;

template <int R>
__device__ __forceinline__ void qbuild_wave_regs(int32_t e, int32_t b, int32_t d, const int32_t *pins,
                                                 const int32_t *parent, int32_t *qpins, int32_t *qlen, uint64_t *fp)
{
    const int lane = threadIdx.x & 63;
    int32_t x[R];
#pragma unroll
    for (int t = 0; t < R; t++) {
        int i = lane * R + t;
        x[t] = i < d ? parent[pins[b + i]] : INT32_MAX;
    }
    wave_sort_regs<R>(x);
    uint64_t sum;
    int32_t len = wave_unique_emit<R>(x, d, qpins + b, &sum);
    if (lane == 0) {
        qlen[e] = len >= 2 ? len : 0;
        fp[e] = fp_finish(sum, len);
    }
}

__global__ __launch_bounds__(kBlock) void k_qbuild_big_waves(int32_t count, const int32_t *list,
                                                             const int32_t *off, const int32_t *pins,
                                                             const int32_t *hseg, const uint8_t *sact,
                                                             const int32_t *parent, int32_t *qpins,
                                                             int32_t *qlen, uint64_t *fp)
{
    const int lane = threadIdx.x & 63;
    int64_t i = (int64_t)blockIdx.x * (kBlock / 64) + (threadIdx.x >> 6);
    if (i >= count) return;
    int32_t e = list[i];
    int32_t b = off[e], d = off[e + 1] - b;
    if (d > kQWaveMax) return;  // k_qbuild_block's
    if (!sact[hseg[e]]) {
        if (lane == 0) qlen[e] = 0;
    } else if (d <= 512) {
        qbuild_wave_regs<8>(e, b, d, pins, parent, qpins, qlen, fp);
    } else {
        qbuild_wave_regs<16>(e, b, d, pins, parent, qpins, qlen, fp);
    }
}

__global__ __launch_bounds__(kBlock) void k_qbuild_block(int32_t count, const int32_t *list,
                                                         const int32_t *off, const int32_t *pins,
                                                         const int32_t *hseg,
                                                         const uint8_t *sact,
                                                         const int32_t *parent, int32_t *qpins,
                                                         int32_t *qlen, uint64_t *fp)
{
    extern __shared__ int32_t dyn[];
    int32_t e = list[blockIdx.x];
    int32_t b = off[e], d = off[e + 1] - b;
    if (d <= kQWaveMax || d > kBigMax) return;  // a wavefront's, or k_qbuild_huge's
    if (!sact[hseg[e]]) {
        if (threadIdx.x == 0) qlen[e] = 0;
        return;
    }
    int n2 = next_pow2(d);
    for (int i = threadIdx.x; i < n2; i += blockDim.x) dyn[i] = i < d ? parent[pins[b + i]] : INT32_MAX;
    __syncthreads();
    block_bitonic_sort(dyn, n2);
    int32_t len;
    uint64_t sum;
    block_unique_emit(dyn, n2, d, b, qpins, &len, &sum);
    if (threadIdx.x == 0) {
        qlen[e] = len >= 2 ? len : 0;
        fp[e] = fp_finish(sum, len);
    }
}

// Hyperedges above the LDS capacity: one launch each, sorted in global scratch.
__global__ __launch_bounds__(1024) void k_qbuild_huge(const int32_t *lhuge, int32_t idx,
                                                      const int32_t *off, const int32_t *pins,
                                                      const int32_t *hseg, const uint8_t *sact,
                                                      const int32_t *parent, int32_t *scratch,
                                                      int32_t *qpins, int32_t *qlen, uint64_t *fp)
{
    int32_t e = lhuge[idx];
    int32_t b = off[e], d = off[e + 1] - b;
    if (!sact[hseg[e]]) {
        if (threadIdx.x == 0) qlen[e] = 0;
        return;
    }
    int n2 = next_pow2(d);
    for (int i = threadIdx.x; i < n2; i += blockDim.x) scratch[i] = i < d ? parent[pins[b + i]] : INT32_MAX;
    __syncthreads();
    block_bitonic_sort(scratch, n2);
    int32_t len;
    uint64_t sum;
    block_unique_emit(scratch, n2, d, b, qpins, &len, &sum);
    if (threadIdx.x == 0) {
        qlen[e] = len >= 2 ? len : 0;
        fp[e] = fp_finish(sum, len);
    }
}

// Re-fingerprint with a new salt (only after a fingerprint collision between
// different pin sets left hyperedges unresolved; practically never).
__global__ void k_refingerprint(int32_t E, const int32_t *off, const int32_t *qpins,
                                const int32_t *qlen, const int32_t *rep, uint64_t salt,
                                uint64_t *fp)
{
    int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= E || rep[e] != -2) return;
    uint64_t sum = 0;
    int32_t len = qlen[e];
    for (int i = 0; i < len; i++) sum += fp_term(qpins[off[e] + i], salt);
    fp[e] = fp_finish(sum, len);
}

// Slot of fingerprint f in the open-addressing table (inserted if new), with
// hyperedge e offered as its smallest id.
__device__ __forceinline__ int32_t dd_slot(unsigned long long f, int32_t e, unsigned long long *tkeys,
                                           int32_t *tmin, int32_t tmask)
{
    uint32_t h = (uint32_t)(f ^ (f >> 32)) & (uint32_t)tmask;
    for (;;) {
        unsigned long long prev = atomicCAS(&tkeys[h], kEmptySlot, f);
        if (prev == kEmptySlot || prev == f) break;
        h = (h + 1) & (uint32_t)tmask;
    }
    atomicMin(&tmin[h], e);
    return (int32_t)h;
}

__device__ __forceinline__ unsigned long long readlane_u64(unsigned long long v, int src)
{
    uint32_t lo = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)v, src);
    uint32_t hi = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(v >> 32), src);
    return ((unsigned long long)hi << 32) | lo;
}

// Duplicates share a fingerprint and so one slot, where per-hyperedge atomics
// serialize on coarse levels (many hyperedges over the same few nodes): the
// lanes sharing the first active lane's fingerprint (twice over) insert once,
// with the first lane's id - the smallest, ids ascend with the lane.
__global__ __launch_bounds__(kBlock) void k_dd_insert(int32_t E, const int32_t *qlen,
                                                      const uint64_t *fp, const int32_t *rep,
                                                      int only_unresolved,
                                                      unsigned long long *tkeys, int32_t *tmin,
                                                      int32_t tmask, int32_t *hslot)
{
    int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    bool act = e < E && qlen[e] >= 2 && !(only_unresolved && rep[e] != -2);
    unsigned long long f = act ? fp[e] : 0ull;
    int lane = threadIdx.x & 63;
    unsigned long long am = __ballot(act);
#pragma unroll
    for (int k = 0; k < 2; k++) {
        if (!am) break;
        int leader = __ffsll((long long)am) - 1;
        unsigned long long lf = readlane_u64(f, leader);
        unsigned long long eq = __ballot(act && f == lf);
        int32_t h = 0;
        if (lane == leader) h = dd_slot(f, (int32_t)e, tkeys, tmin, tmask);
        h = __builtin_amdgcn_readlane(h, leader);
        if ((eq >> lane) & 1) {
            hslot[e] = h;
            act = false;
        }
        am &= ~eq;
    }
    if (act) hslot[e] = dd_slot(f, (int32_t)e, tkeys, tmin, tmask);
}

// Representative of each hyperedge (the smallest id with the same pin set) and
// the weight sums.  Lanes adding to the first adding lane's representative
// (twice over) add with one atomic.
__global__ __launch_bounds__(kBlock) void k_dd_resolve(int32_t E, const int32_t *off,
                                                       const int32_t *qpins, const int32_t *qlen,
                                                       const int32_t *hw, const int32_t *hslot,
                                                       const int32_t *tmin, int only_unresolved,
                                                       int32_t *rep, int32_t *wsum,
                                                       int32_t *unresolved)
{
    int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    bool act = e < E;
    int32_t len = act ? qlen[e] : 0;
    if (act) {
        if (only_unresolved) {
            act = rep[e] == -2;
        } else if (len < 2) {
            rep[e] = -1;
            act = false;
        }
    }
    int32_t r = 0;
    bool add = false;
    if (act) {
        r = tmin[hslot[e]];
        bool same = true;
        if (r != e) {
            same = qlen[r] == len;
            const int32_t *a = qpins + off[e], *c = qpins + off[r];
            for (int i = 0; same && i < len; i++) same = a[i] == c[i];
        }
        if (same) {
            rep[e] = r;
            add = true;
        } else {
            rep[e] = -2;
            atomicAdd(unresolved, 1);
        }
    }
    int32_t w = add ? hw[e] : 0;
    int lane = threadIdx.x & 63;
    unsigned long long am = __ballot(add);
#pragma unroll
    for (int k = 0; k < 2; k++) {
        if (!am) break;
        int leader = __ffsll((long long)am) - 1;
        int32_t lr = __builtin_amdgcn_readlane(r, leader);
        unsigned long long eq = __ballot(add && r == lr);
        int32_t sum = wave_sum(((eq >> lane) & 1) ? w : 0);
        if (lane == leader) atomicAdd(&wsum[lr], sum);
        if ((eq >> lane) & 1) add = false;
        am &= ~eq;
    }
    if (add) atomicAdd(&wsum[r], w);
}


struct CopyPinsOp {
    const int32_t *off, *rep, *qlen, *qpins, *hdst;
    int32_t *cpins;
    template <int S> __device__ __forceinline__ void run(int64_t vb, int32_t count, const int32_t *list) const;
};

template <int S>
__device__ __forceinline__ void CopyPinsOp::run(int64_t vb, int32_t count, const int32_t *list) const
{
    int lane, stride;
    int32_t e = sched_hedge_at<S>(vb, count, list, lane, stride);
    if (e < 0) return;
    int32_t b = off[e];
    if (!thread_split<S>(off[e + 1] - b)) return;
    if (rep[e] != e) return;
    int32_t len = qlen[e], dst = hdst[e];
    for (int i = lane; i < len; i += stride) cpins[dst + i] = qpins[b + i];
}

// Sizes of the coarse level, its segment tables and which segments continue.
// One workgroup (kFixupThreads); each thread owns a contiguous run of
// segments.  A segment with no hyperedges starts its coarse hyperedges where
// the next segment that had some starts (suffix minimum of the starts).
constexpr int kFixupThreads = 1024;

__global__ __launch_bounds__(kFixupThreads) void k_level_fixup(
    int32_t S, int32_t N, int32_t E, const int32_t *nbase, const int32_t *hbase, const int32_t *cid,
    const int32_t *hb_tmp, const int32_t *totN, const uint64_t *totEP, int32_t level_next, int32_t max_levels,
    int32_t min_nodes, const uint8_t *sact, uint8_t *sact_next, int32_t *coarsest, int32_t *c_nbase,
    int32_t *c_hbase, int32_t *c_off, const int32_t *counters, LevelInfo *info)
{
    __shared__ int32_t rmin[kFixupThreads / 64];
    __shared__ int32_t red[kFixupThreads / 64][4];
    const int tid = threadIdx.x;
    int32_t Nc = *totN;
    int32_t Ec = (int32_t)(*totEP >> 32), Pc = (int32_t)(*totEP & 0xffffffffu);
    int32_t q = (S + kFixupThreads - 1) / kFixupThreads;
    int32_t s0 = min(S, tid * q), s1 = min(S, s0 + q);
    // own run: suffix minimum of the starts of segments that had hyperedges
    int32_t m = INT32_MAX;
    for (int32_t s = s1 - 1; s >= s0; s--) {
        if (hbase[s] != hbase[s + 1]) m = min(m, hb_tmp[s]);
        c_hbase[s] = m;
    }
    for (int32_t s = s0; s < s1; s++) c_nbase[s] = nbase[s] < N ? cid[nbase[s]] : Nc;
    if (tid == 0) {
        c_off[Ec] = Pc;
        c_hbase[S] = Ec;
        c_nbase[S] = Nc;
    }
    // the runs after this one: suffix minimum over the threads (wavefront
    // shuffles, then the wavefronts after this one)
    int lane = tid & 63, wv = tid >> 6;
    int32_t incl = m;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        int32_t y = __shfl_down(incl, o, 64);
        if (lane + o < 64) incl = min(incl, y);
    }
    int32_t after = __shfl_down(incl, 1, 64);
    if (lane == 63) after = INT32_MAX;
    if (lane == 0) rmin[wv] = incl;
    __syncthreads();
    after = min(after, Ec);
    for (int w = wv + 1; w < kFixupThreads / 64; w++) after = min(after, rmin[w]);
    for (int32_t s = s0; s < s1; s++) c_hbase[s] = min(c_hbase[s], after);
    __syncthreads();
    int32_t active = 0, maxn = 0, maxp = 0, maxe = 0;
    for (int32_t s = s0; s < s1; s++) {
        int32_t ns = c_nbase[s + 1] - c_nbase[s], es = c_hbase[s + 1] - c_hbase[s];
        int32_t ps = c_off[c_hbase[s + 1]] - c_off[c_hbase[s]];
        maxn = max(maxn, ns);
        maxp = max(maxp, ps);
        maxe = max(maxe, es);
        bool go = false;
        if (sact[s]) {
            coarsest[s] = level_next;
            go = level_next < max_levels && es > 0 && ns > min_nodes;
            active += go ? 1 : 0;
        }
        sact_next[s] = go ? 1 : 0;
    }
    active = wave_sum(active);
    maxn = wave_max(maxn);
    maxp = wave_max(maxp);
    maxe = wave_max(maxe);
    if ((tid & 63) == 0) {
        red[tid >> 6][0] = active;
        red[tid >> 6][1] = maxn;
        red[tid >> 6][2] = maxp;
        red[tid >> 6][3] = maxe;
    }
    __syncthreads();
    if (tid == 0) {
        for (int w = 1; w < kFixupThreads / 64; w++) {
            active += red[w][0];
            maxn = max(maxn, red[w][1]);
            maxp = max(maxp, red[w][2]);
            maxe = max(maxe, red[w][3]);
        }
        info->N = Nc;
        info->E = Ec;
        info->P = Pc;
        info->nmid = counters[1];
        info->nbig = counters[2];
        info->nhuge = counters[3];
        info->unresolved = counters[0];
        info->active = active;
        info->maxseg_nodes = maxn;
        info->maxseg_pins = maxp;
        info->maxseg_hedges = maxe;
    }
}

}  // namespace bp
