// Input normalisation, nested k-way subgraph extraction (Algorithm 6), the
// connectivity-1 cut (problem statement) and device-side input validation.
#pragma once
#include "level.hpp"
#include "scan.hpp"

namespace bp {

// ---- validation -----------------------------------------------------------------

struct ValidateOut {
    int32_t bad_offsets;
    int32_t bad_pins;
    int32_t bad_weights;
    int32_t pad;
    unsigned long long sum_nw, sum_hw;
};

__global__ __launch_bounds__(kBlock) void k_validate(int32_t N, int32_t E, const int32_t *off,
                                                     const int32_t *pins, const int32_t *nw,
                                                     const int32_t *hw, ValidateOut *out)
{
    __shared__ int64_t lds[16];
    int64_t tid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    int64_t stride = (int64_t)gridDim.x * blockDim.x;
    int64_t P = off[E];
    int64_t snw = 0, shw = 0;
    int bo = 0, bp_ = 0, bw = 0;
    for (int64_t e = tid; e < E; e += stride) {
        if (off[e + 1] < off[e]) bo = 1;
        if (hw) {
            if (hw[e] < 0) bw = 1;
            shw += hw[e];
        }
    }
    if (tid == 0 && (off[0] != 0 || P < 0)) bo = 1;
    for (int64_t i = tid; i < P && !bo; i += stride) {
        int32_t v = pins[i];
        if (v < 0 || v >= N) bp_ = 1;
    }
    for (int64_t v = tid; v < N; v += stride) {
        if (nw) {
            if (nw[v] < 0) bw = 1;
            snw += nw[v];
        }
    }
    snw = block_sum(snw, lds);
    shw = block_sum(shw, lds);
    if (bo) atomicOr(&out->bad_offsets, 1);
    if (bp_) atomicOr(&out->bad_pins, 1);
    if (bw) atomicOr(&out->bad_weights, 1);
    if (threadIdx.x == 0) {
        atomicAdd(&out->sum_nw, (unsigned long long)snw);
        atomicAdd(&out->sum_hw, (unsigned long long)shw);
    }
}

// ---- level 0: drop hyperedges that cannot be cut --------------------------------

// copy the kept hyperedges' pins (degree >= 2) to their compacted place
constexpr int kNormShort = 16;

__global__ __launch_bounds__(kBlock) void k_norm_copy(int32_t E, const int32_t *off,
                                                      const int32_t *pins, const int32_t *dst,
                                                      int32_t *cpins)
{
    // a thread per hyperedge of at most kNormShort pins (its loads all in
    // flight before the stores); longer ones are copied by the whole
    // wavefront, one after another, 8 loads a lane in flight.  Every lane
    // reaches the ballot: lanes past E carry an empty hyperedge.
    const int lane = threadIdx.x & 63;
    int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    int32_t b = 0, d = 0, o = 0;
    if (e < E) {
        b = off[e];
        d = off[e + 1] - b;
        if (d >= 2) o = dst[e];
        else d = 0;
    }
    if (d <= kNormShort) {
        int32_t v[kNormShort];
#pragma unroll
        for (int i = 0; i < kNormShort; i++)
            if (i < d) v[i] = pins[b + i];
#pragma unroll
        for (int i = 0; i < kNormShort; i++)
            if (i < d) cpins[o + i] = v[i];
    }
    unsigned long long lm = __ballot(d > kNormShort);
    while (lm) {
        int l = __ffsll((long long)lm) - 1;
        lm &= lm - 1;
        int32_t lb = __shfl(b, l, 64), ld = __shfl(d, l, 64), lo = __shfl(o, l, 64);
        for (int32_t i0 = 0; i0 < ld; i0 += 8 * 64) {
            int32_t v[8];
#pragma unroll
            for (int u = 0; u < 8; u++) {
                int32_t i = i0 + u * 64 + lane;
                v[u] = i < ld ? pins[lb + i] : 0;
            }
#pragma unroll
            for (int u = 0; u < 8; u++) {
                int32_t i = i0 + u * 64 + lane;
                if (i < ld) cpins[lo + i] = v[u];
            }
        }
    }
}

__global__ void k_iota(int64_t n, int32_t *p)
{
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x)
        p[i] = (int32_t)i;
}

__global__ void k_copy_weights(int64_t n, const int32_t *src, int32_t *dst)
{
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x)
        dst[i] = src ? src[i] : 1;
}

// Schedule lists of a freshly built level: each workgroup stages the
// hyperedges of its kClsItems ids in LDS and reserves room in each list with
// one atomic (same-address atomics from many workgroups serialise).  With
// tot (a level just compacted) the count and the pin total come from the
// device: E is then only a bound.  List order is arbitrary; every consumer
// treats its items independently.
constexpr int kClsItems = 2048;

// Block vb of the classification.
__device__ __forceinline__ void classify_block(int64_t vb, int32_t E, const int32_t *off, const uint64_t *tot,
                                               int32_t *lmid, int32_t *lbig, int32_t *lhuge, int32_t *counters)
{
    __shared__ int32_t items[3][kClsItems];
    __shared__ int32_t cnt[3], base[3];
    int32_t P = 0;
    if (tot) {
        E = (int32_t)(*tot >> 32);
        P = (int32_t)(*tot & 0xffffffffu);
    }
    int64_t first = vb * kClsItems;
    if (first >= E) return;
    if (!tot) P = off[E];
    if (threadIdx.x < 3) cnt[threadIdx.x] = 0;
    __syncthreads();
    for (int r = 0; r < kClsItems / kBlock; r++) {
        int64_t e = first + r * kBlock + threadIdx.x;
        int32_t d = 0;
        if (e < E) d = (e + 1 < E ? off[e + 1] : P) - off[e];
        lds_append(d > kSmallMax && d <= kMidMax, (int32_t)e, items[0], &cnt[0]);
        lds_append(d > kMidMax, (int32_t)e, items[1], &cnt[1]);
        lds_append(d > kBigMax, (int32_t)e, items[2], &cnt[2]);
    }
    __syncthreads();
    if (threadIdx.x < 3) base[threadIdx.x] = cnt[threadIdx.x] ? atomicAdd(&counters[1 + threadIdx.x], cnt[threadIdx.x]) : 0;
    __syncthreads();
    for (int i = threadIdx.x; i < cnt[0]; i += blockDim.x) lmid[base[0] + i] = items[0][i];
    for (int i = threadIdx.x; i < cnt[1]; i += blockDim.x) lbig[base[1] + i] = items[1][i];
    for (int i = threadIdx.x; i < cnt[2]; i += blockDim.x) lhuge[base[2] + i] = items[2][i];
}

__global__ __launch_bounds__(kBlock) void k_classify(int32_t E, const int32_t *off, const uint64_t *tot,
                                                     int32_t *lmid, int32_t *lbig, int32_t *lhuge,
                                                     int32_t *counters)
{
    classify_block(blockIdx.x, E, off, tot, lmid, lbig, lhuge, counters);
}

template <int S>
__global__ __launch_bounds__(kBlock) void k_count_side1(int32_t count, const int32_t *list,
                                                        const int32_t *off, const int32_t *pins,
                                                        const uint8_t *side, int32_t *n1out)
{
    __shared__ int32_t lds[16];
    int lane, stride;
    int32_t e = sched_hedge<S>(count, list, lane, stride);
    if (e < 0) return;
    int32_t b = off[e], d = off[e + 1] - b;
    if (!thread_split<S>(d)) return;
    int32_t n1 = 0;
    for (int i = lane; i < d; i += stride) n1 += side[pins[b + i]];
    n1 = group_sum<S>(n1, lds);
    if (lane == 0) n1out[e] = n1;
}

// Child table: child (s, side) continues when it still has >= 2 parts.
struct ChildTable {
    int32_t *idx;     // [2S] child segment index or -1 (final part)
    int32_t *nbase;   // [C+1]
    int32_t *hbase;   // [C+1]
    int32_t *pbase;   // [C+1]
    int32_t *k;       // [C] parts of each child
    int32_t *lo;      // [C]
    uint64_t *F;      // [C] per-bisection factor, inherited from the parent
};

__global__ void k_child_table(int32_t S, int32_t N, int32_t E, const int32_t *nbase,
                              const int32_t *hbase, const int32_t *k0, const int32_t *k1,
                              const int32_t *lo, const uint64_t *F, const uint64_t *nscan,
                              const uint64_t *hscan0,
                              const uint64_t *hscan1, const uint64_t *ntot, const uint64_t *htot0,
                              const uint64_t *htot1, ChildTable ct, LevelInfo *info)
{
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    int32_t c = 0, nb = 0, hb = 0, pb = 0;
    auto at = [&](const uint64_t *scan, const uint64_t *tot, int32_t i, int32_t n) -> uint64_t {
        return i < n ? scan[i] : *tot;
    };
    for (int32_t s = 0; s < S; s++) {
        uint64_t na = at(nscan, ntot, nbase[s], N), nz = at(nscan, ntot, nbase[s + 1], N);
        for (int sd = 0; sd < 2; sd++) {
            int32_t kk = sd ? k1[s] : k0[s];
            if (kk < 2) {
                ct.idx[2 * s + sd] = -1;
                continue;
            }
            const uint64_t *hs = sd ? hscan1 : hscan0;
            const uint64_t *ht = sd ? htot1 : htot0;
            uint64_t ha = at(hs, ht, hbase[s], E), hz = at(hs, ht, hbase[s + 1], E);
            int32_t nn = sd ? (int32_t)((nz >> 32) - (na >> 32)) : (int32_t)((nz & 0xffffffffu) - (na & 0xffffffffu));
            int32_t ne = (int32_t)((hz >> 32) - (ha >> 32));
            int32_t np = (int32_t)((hz & 0xffffffffu) - (ha & 0xffffffffu));
            ct.idx[2 * s + sd] = c;
            ct.nbase[c] = nb;
            ct.hbase[c] = hb;
            ct.pbase[c] = pb;
            ct.k[c] = kk;
            ct.lo[c] = lo[s] + (sd ? k0[s] : 0);
            ct.F[c] = F[s];
            nb += nn;
            hb += ne;
            pb += np;
            c++;
        }
    }
    ct.nbase[c] = nb;
    ct.hbase[c] = hb;
    ct.pbase[c] = pb;
    info->N = nb;
    info->E = hb;
    info->P = pb;
    info->active = c;
}

// nodes: renumber into their child, or write the final part id
__global__ __launch_bounds__(kBlock) void k_extract_nodes(
    int32_t N, const int32_t *nseg, const int32_t *nbase, const uint8_t *side,
    const uint64_t *nscan, const int32_t *orig, const int32_t *nw, const int32_t *k0,
    const int32_t *lo, ChildTable ct, int32_t *map, int32_t *c_orig, int32_t *c_nw,
    int32_t *c_nseg, int32_t *part)
{
    int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (v >= N) return;
    int32_t s = nseg[v], sd = side[v];
    int32_t ci = ct.idx[2 * s + sd];
    if (ci < 0) {
        part[orig[v]] = lo[s] + (sd ? k0[s] : 0);
        map[v] = -1;
        return;
    }
    uint64_t a = nscan[v], z = nscan[nbase[s]];
    int32_t rank = sd ? (int32_t)((a >> 32) - (z >> 32)) : (int32_t)((a & 0xffffffffu) - (z & 0xffffffffu));
    int32_t id = ct.nbase[ci] + rank;
    map[v] = id;
    c_orig[id] = orig[v];
    c_nw[id] = nw[v];
    c_nseg[id] = ci;
}

// hyperedges: emit each side's part when it keeps >= 2 pins
template <int S>
__global__ __launch_bounds__(kBlock) void k_extract_hedges(
    int32_t count, const int32_t *list, const int32_t *off, const int32_t *pins,
    const int32_t *hw, const int32_t *hseg, const int32_t *hbase, const uint8_t *side,
    const int32_t *n1, const uint64_t *hscan0, const uint64_t *hscan1, const int32_t *map,
    ChildTable ct, int32_t *c_off, int32_t *c_pins, int32_t *c_hw, int32_t *c_hseg)
{
    __shared__ int32_t lds[16];
    __shared__ int32_t carry;
    int lane, stride;
    int32_t e = sched_hedge<S>(count, list, lane, stride);
    if (e < 0) return;
    int32_t b = off[e], d = off[e + 1] - b;
    if (!thread_split<S>(d)) return;
    int32_t s = hseg[e];
    int32_t cnt1 = n1[e];
    for (int sd = 0; sd < 2; sd++) {
        int32_t ci = ct.idx[2 * s + sd];
        int32_t ns = sd ? cnt1 : d - cnt1;
        if (ci < 0 || ns < 2) continue;  // uniform over the group
        const uint64_t *hs = sd ? hscan1 : hscan0;
        uint64_t a = hs[e], z = hs[hbase[s]];
        int32_t id = ct.hbase[ci] + (int32_t)((a >> 32) - (z >> 32));
        int32_t po = ct.pbase[ci] + (int32_t)((a & 0xffffffffu) - (z & 0xffffffffu));
        if (lane == 0) {
            c_off[id] = po;
            c_hw[id] = hw[e];
            c_hseg[id] = ci;
        }
        if (S == SMALL) {
            int32_t k = 0;
            for (int i = 0; i < d; i++) {
                int32_t v = pins[b + i];
                if (side[v] == sd) c_pins[po + k++] = map[v];
            }
        } else if (S == WAVE) {
            int32_t base = 0;
            for (int i0 = 0; i0 < d; i0 += 64) {
                int i = i0 + lane;
                int32_t v = i < d ? pins[b + i] : 0;
                bool in = i < d && side[v] == sd;
                unsigned long long m = __ballot(in);
                if (in) c_pins[po + base + __popcll(m & ((1ull << lane) - 1))] = map[v];
                base += __popcll(m);
            }
        } else {
            if (threadIdx.x == 0) carry = 0;
            __syncthreads();
            for (int i0 = 0; i0 < d; i0 += blockDim.x) {
                int i = i0 + threadIdx.x;
                int32_t v = i < d ? pins[b + i] : 0;
                int32_t in = (i < d && side[v] == sd) ? 1 : 0;
                int32_t tot;
                int32_t ex = block_excl_scan(in, lds, &tot);
                if (in) c_pins[po + carry + ex] = map[v];
                __syncthreads();
                if (threadIdx.x == 0) carry += tot;
                __syncthreads();
            }
        }
    }
}

// ---- connectivity-1 cut of the final partition ----------------------------------

// Connectivity (number of distinct parts) of hyperedge e, computed by its
// schedule group: a part bitmask when every part id is below 64, else a
// count of parts not seen at an earlier pin (O(d^2), rare large hyperedges).
template <int S>
__device__ __forceinline__ int32_t hedge_lambda(int32_t e, int lane, int stride, const int32_t *off,
                                                const int32_t *pins, const int32_t *part, bool mask64,
                                                unsigned long long *orl, int32_t *lds)
{
    int32_t b = off[e], d = off[e + 1] - b;
    if (mask64) {
        unsigned long long m = 0;
        for (int i = lane; i < d; i += stride) m |= 1ull << (part[pins[b + i]] & 63);
        if (S != SMALL) {
#pragma unroll
            for (int o = 32; o > 0; o >>= 1) m |= __shfl_xor(m, o, 64);
        }
        if (S == BLOCK) {
            if ((threadIdx.x & 63) == 0) orl[threadIdx.x >> 6] = m;
            __syncthreads();
            m = 0;
            for (int i = 0; i < (int)(blockDim.x >> 6); i++) m |= orl[i];
            __syncthreads();
        }
        return __popcll(m);
    }
    int32_t lam = 0;
    for (int i = lane; i < d; i += stride) {
        int32_t p = part[pins[b + i]];
        bool first = true;
        for (int j = 0; j < i && first; j++) first = part[pins[b + j]] != p;
        lam += first ? 1 : 0;
    }
    return group_sum<S>(lam, lds);
}

// Connectivity-1 cut, summed over the hyperedges of one schedule (SMALL: all
// hyperedges of degree <= 8, one per thread; WAVE / BLOCK: the listed ones).
// Each workgroup writes its sum to partial[blockIdx.x] (no same-address
// atomics); k_sum_u64 adds the partial sums up.  SMALL: contiguous chunks of
// about two hyperedges a thread (at most kCutBlocks workgroups); WAVE / BLOCK: the listed
// hyperedges, as many workgroups as keep every wavefront on about one
// hyperedge (at most kCutBlocks).
constexpr int64_t kCutBlocks = 16384;

template <int S> inline int64_t cut_grid(int64_t count)
{
    if (S == SMALL) {  // two hyperedges a thread: enough loads in flight to cover the gathers
        int64_t g = ceil_div(count, (int64_t)2 * kBlock);
        return g < kCutBlocks ? g : kCutBlocks;
    }
    int64_t g = S == WAVE ? sched_grid<WAVE>(count) : count;
    return g < kCutBlocks ? g : kCutBlocks;
}

template <int S>
__global__ __launch_bounds__(kBlock) void k_cut(int32_t count, const int32_t *list, const int32_t *off,
                                                const int32_t *pins, const int32_t *hw, const int32_t *part,
                                                int mask64, unsigned long long *partial)
{
    __shared__ unsigned long long orl[16];
    __shared__ int32_t lds[16];
    __shared__ int64_t lds64[16];
    int64_t contrib = 0;
    if (S == SMALL) {
        for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < count;
             e += (int64_t)gridDim.x * blockDim.x) {
            if (!thread_split<SMALL>(off[e + 1] - off[e])) continue;
            int32_t lam = hedge_lambda<SMALL>((int32_t)e, 0, 1, off, pins, part, mask64, orl, lds);
            if (lam > 1) contrib += (int64_t)(hw ? hw[e] : 1) * (lam - 1);
        }
    } else if (S == WAVE) {
        int64_t wpb = blockDim.x >> 6;
        for (int64_t i = (int64_t)blockIdx.x * wpb + (threadIdx.x >> 6); i < count; i += (int64_t)gridDim.x * wpb) {
            int32_t e = list[i];
            if (!thread_split<WAVE>(off[e + 1] - off[e])) continue;
            int32_t lam = hedge_lambda<WAVE>(e, threadIdx.x & 63, 64, off, pins, part, mask64, orl, lds);
            if ((threadIdx.x & 63) == 0 && lam > 1) contrib += (int64_t)(hw ? hw[e] : 1) * (lam - 1);
        }
    } else {
        for (int64_t i = blockIdx.x; i < count; i += gridDim.x) {
            int32_t e = list[i];
            int32_t lam = hedge_lambda<BLOCK>(e, threadIdx.x, blockDim.x, off, pins, part, mask64, orl, lds);
            if (threadIdx.x == 0 && lam > 1) contrib += (int64_t)(hw ? hw[e] : 1) * (lam - 1);
        }
    }
    contrib = block_sum(contrib, lds64);
    if (threadIdx.x == 0) partial[blockIdx.x] = (unsigned long long)contrib;
}

// out[0] = the sum of a[0, n): one workgroup.
__global__ void k_sum_u64(int32_t n, const unsigned long long *a, unsigned long long *out)
{
    __shared__ unsigned long long lds[16];
    unsigned long long t = 0;
    for (int i = threadIdx.x; i < n; i += blockDim.x) t += a[i];
    t = wave_sum(t);
    if ((threadIdx.x & 63) == 0) lds[threadIdx.x >> 6] = t;
    __syncthreads();
    if (threadIdx.x == 0) {
        unsigned long long r = 0;
        for (int i = 0; i < (int)(blockDim.x >> 6); i++) r += lds[i];
        *out = r;
    }
}

// Part weights: registers for k <= 8, an LDS histogram for k <= 4096, else
// global atomics; one global atomic per part per workgroup otherwise.
__global__ __launch_bounds__(kBlock) void k_part_weights(int32_t N, int32_t k, const int32_t *part,
                                                         const int32_t *nw,
                                                         unsigned long long *pw)
{
    __shared__ unsigned long long acc[4096];
    __shared__ int64_t lds[16];
    int64_t stride = (int64_t)gridDim.x * blockDim.x;
    if (k <= 8) {
        int64_t r[8] = {0, 0, 0, 0, 0, 0, 0, 0};
        for (int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; v < N; v += stride) {
            int32_t p = part[v];
            int64_t w = nw ? nw[v] : 1;
#pragma unroll
            for (int j = 0; j < 8; j++) r[j] += p == j ? w : 0;
        }
#pragma unroll
        for (int j = 0; j < 8; j++) {
            int64_t t = block_sum(r[j], lds);
            if (threadIdx.x == 0 && j < k && t) atomicAdd(&pw[j], (unsigned long long)t);
        }
        return;
    }
    bool in_lds = k <= 4096;
    if (in_lds) {
        for (int i = threadIdx.x; i < k; i += blockDim.x) acc[i] = 0;
        __syncthreads();
    }
    for (int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; v < N; v += stride) {
        int32_t p = part[v];
        if (p < 0 || p >= k) continue;  // range is the caller's contract; never write outside
        unsigned long long w = (unsigned long long)(nw ? nw[v] : 1);
        if (in_lds) atomicAdd(&acc[p], w);
        else atomicAdd(&pw[p], w);
    }
    if (in_lds) {
        __syncthreads();
        for (int i = threadIdx.x; i < k; i += blockDim.x)
            if (acc[i]) atomicAdd(&pw[i], acc[i]);
    }
}

__global__ void k_max_u64(int32_t n, const unsigned long long *a, unsigned long long *out)
{
    __shared__ unsigned long long lds[16];
    unsigned long long m = 0;
    for (int i = threadIdx.x; i < n; i += blockDim.x) m = a[i] > m ? a[i] : m;
    m = wave_max(m);
    if ((threadIdx.x & 63) == 0) lds[threadIdx.x >> 6] = m;
    __syncthreads();
    if (threadIdx.x == 0) {
        unsigned long long r = 0;
        for (int i = 0; i < (int)(blockDim.x >> 6); i++) r = lds[i] > r ? lds[i] : r;
        *out = r;
    }
}

}  // namespace bp
