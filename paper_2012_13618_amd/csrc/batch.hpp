// Many independent hypergraphs as the segments of one level-0 CSR.
//
// The nested k-way scheme of Algorithm 6 already runs every bisection of a
// tree level as one segment of a shared CSR, with local ids, so a batch of
// input graphs is simply a wider first tree level: graph g becomes segment g
// with its own k, its own per-bisection factor and its own node and hyperedge
// ranges.  Results per graph are the ones the graph gets alone.
#pragma once
#include "kway.hpp"

namespace bp {

// One input graph, device-readable.
struct GraphDesc {
    const int32_t *off, *pins, *nw, *hw;  // caller's device CSR (nw/hw may be null)
    int32_t N, E;
    int64_t nbase, ebase, pbase;          // position in the concatenation
};

struct GraphCheck {
    int32_t bad_offsets, bad_pins, bad_weights, pad;
    unsigned long long sum_nw, sum_hw;
    int64_t P;
};

// Pin counts (offsets[E]) and the offsets[0] check, one thread per graph.
__global__ void k_batch_sizes(int32_t n, const GraphDesc *d, GraphCheck *chk)
{
    int32_t g = blockIdx.x * blockDim.x + threadIdx.x;
    if (g >= n) return;
    GraphDesc x = d[g];
    int32_t p = x.off[x.E];
    chk[g].P = p;
    chk[g].bad_offsets = (x.off[0] != 0 || p < 0) ? 1 : 0;
    chk[g].bad_pins = 0;
    chk[g].bad_weights = 0;
    chk[g].sum_nw = 0;
    chk[g].sum_hw = 0;
}

// Concatenation: blockIdx.y is the graph, blockIdx.x strides over its
// hyperedges, pins and nodes.  Node ids in pins become global (node base
// added); segment ids are written per node and per input hyperedge.  Every
// graph is checked the way a single input is.
__global__ __launch_bounds__(kBlock) void k_batch_gather(const GraphDesc *d, GraphCheck *chk,
                                                         int32_t *off, int32_t *pins, int32_t *nw,
                                                         int32_t *hw, int32_t *nseg, int32_t *eseg)
{
    __shared__ int64_t lds[16];
    int32_t g = blockIdx.y;
    GraphDesc x = d[g];
    int64_t P = chk[g].P;
    int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x, stride = (int64_t)gridDim.x * blockDim.x;
    int bo = 0, bpn = 0, bw = 0;
    int64_t snw = 0, shw = 0;
    for (int64_t e = t; e < x.E; e += stride) {
        int32_t a = x.off[e], b = x.off[e + 1];
        if (b < a) bo = 1;
        off[x.ebase + e] = (int32_t)(x.pbase + a);
        int32_t w = x.hw ? x.hw[e] : 1;
        if (w < 0) bw = 1;
        shw += w;
        hw[x.ebase + e] = w;
        eseg[x.ebase + e] = g;
    }
    if (!chk[g].bad_offsets)
        for (int64_t i = t; i < P; i += stride) {
            int32_t v = x.pins[i];
            if (v < 0 || v >= x.N) bpn = 1;
            pins[x.pbase + i] = (int32_t)(x.nbase + v);
        }
    for (int64_t v = t; v < x.N; v += stride) {
        int32_t w = x.nw ? x.nw[v] : 1;
        if (w < 0) bw = 1;
        snw += w;
        nw[x.nbase + v] = w;
        nseg[x.nbase + v] = g;
    }
    snw = block_sum(snw, lds);
    shw = block_sum(shw, lds);
    if (bo) atomicOr(&chk[g].bad_offsets, 1);
    if (bpn) atomicOr(&chk[g].bad_pins, 1);
    if (bw) atomicOr(&chk[g].bad_weights, 1);
    if (threadIdx.x == 0) {
        if (snw) atomicAdd(&chk[g].sum_nw, (unsigned long long)snw);
        if (shw) atomicAdd(&chk[g].sum_hw, (unsigned long long)shw);
    }
}

// Hyperedge and pin bases of every segment after normalisation: kept[e] is
// (kept hyperedges before input hyperedge e) << 32 | (their pins).
__global__ void k_batch_hbase(int32_t S, const int64_t *ebase_in, int64_t E_in, const uint64_t *kept,
                              const uint64_t *tot, int32_t *hbase, int32_t *pbase)
{
    int32_t s = blockIdx.x * blockDim.x + threadIdx.x;
    if (s > S) return;
    int64_t e = ebase_in[s];
    uint64_t k = e < E_in ? kept[e] : *tot;
    hbase[s] = (int32_t)(k >> 32);
    pbase[s] = (int32_t)(k & 0xffffffffu);
}

// Part ids of the concatenation back into every graph's own output buffer.
__global__ __launch_bounds__(kBlock) void k_batch_scatter(const GraphDesc *d, int32_t *const *out,
                                                          const int32_t *part)
{
    int32_t g = blockIdx.y;
    GraphDesc x = d[g];
    int32_t *o = out[g];
    for (int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; v < x.N;
         v += (int64_t)gridDim.x * blockDim.x)
        o[v] = part[x.nbase + v];
}

// ---- per-graph cut and part weights ------------------------------------------------

// Per-graph connectivity-1 cut.  Every schedule takes contiguous chunks (of
// hyperedges for SMALL, of the degree lists for WAVE / BLOCK, whose entries
// ascend roughly with the hyperedge id and so with the graph) and sums per
// graph in LDS, one global atomic per graph and chunk; a graph more than
// kAggLists past the chunk's first one adds globally.
template <int S>
__global__ __launch_bounds__(kBlock) void k_cut_seg(int32_t count, const int32_t *list,
                                                    const int32_t *off, const int32_t *pins,
                                                    const int32_t *hw, const int32_t *hseg,
                                                    const int32_t *part, int32_t kmax,
                                                    unsigned long long *cut)
{
    __shared__ unsigned long long orl[16];
    __shared__ int32_t lds[16];
    __shared__ unsigned long long acc[kAggLists];
    bool mask64 = kmax <= 64;
    int64_t lo, hi;
    if (S == SMALL) {
        reduce_chunk(count, gridDim.x, blockIdx.x, lo, hi);
    } else {  // list chunks as even as the grid allows (a wavefront or workgroup per entry)
        int64_t per = ceil_div((int64_t)count, (int64_t)gridDim.x);
        lo = min((int64_t)blockIdx.x * per, (int64_t)count);
        hi = min(lo + per, (int64_t)count);
    }
    if (lo >= hi) return;
    int32_t s0 = hseg[S == SMALL ? (int32_t)lo : list[lo]];
    for (int i = threadIdx.x; i < kAggLists; i += blockDim.x) acc[i] = 0;
    __syncthreads();
    auto add = [&](int32_t e, int32_t lam) {
        unsigned long long c = (unsigned long long)hw[e] * (lam - 1);
        int32_t q = hseg[e] - s0;
        if (q >= 0 && q < kAggLists) atomicAdd(&acc[q], c);
        else atomicAdd(&cut[hseg[e]], c);
    };
    if (S == SMALL) {
        // a wavefront's hyperedges nearly always belong to one graph: the lanes
        // of each graph present add up their cuts first, so that one lane adds
        // for all of them (per-lane LDS atomics on one address serialize)
        const int lane = threadIdx.x & 63;
        for (int64_t base = lo; base < hi; base += blockDim.x) {
            int64_t e = base + threadIdx.x;
            unsigned long long c = 0;
            int32_t g = -1;
            if (e < hi && thread_split<SMALL>(off[e + 1] - off[e])) {
                int32_t lam = hedge_lambda<SMALL>((int32_t)e, 0, 1, off, pins, part, mask64, orl, lds);
                if (lam > 1) {
                    c = (unsigned long long)hw[e] * (lam - 1);
                    g = hseg[e];
                }
            }
            unsigned long long left = __ballot(c != 0);
            while (left) {
                int32_t gl = __shfl(g, __ffsll((long long)left) - 1, 64);
                bool mine = c != 0 && g == gl;
                unsigned long long sum = wave_sum(mine ? c : 0ull);
                if (lane == __ffsll((long long)left) - 1) {
                    int32_t q = gl - s0;
                    if (q >= 0 && q < kAggLists) atomicAdd(&acc[q], sum);
                    else atomicAdd(&cut[gl], sum);
                }
                left &= ~__ballot(mine);
            }
        }
    } else if (S == WAVE) {
        for (int64_t i = lo + (threadIdx.x >> 6); i < hi; i += blockDim.x >> 6) {
            int32_t e = list[i];
            if (!thread_split<WAVE>(off[e + 1] - off[e])) continue;
            int32_t lam = hedge_lambda<WAVE>(e, threadIdx.x & 63, 64, off, pins, part, mask64, orl, lds);
            if ((threadIdx.x & 63) == 0 && lam > 1) add(e, lam);
        }
    } else {
        for (int64_t i = lo; i < hi; i++) {
            int32_t e = list[i];
            int32_t lam = hedge_lambda<BLOCK>(e, threadIdx.x, blockDim.x, off, pins, part, mask64, orl, lds);
            if (threadIdx.x == 0 && lam > 1) add(e, lam);
        }
    }
    __syncthreads();
    for (int i = threadIdx.x; i < kAggLists; i += blockDim.x)
        if (acc[i]) atomicAdd(&cut[s0 + i], acc[i]);
}

// part weights of every graph: pw[kbase[g] + part] (LDS histogram when a
// workgroup's nodes all belong to one graph with at most 1024 parts)
__global__ __launch_bounds__(kBlock) void k_part_weights_seg(int32_t N, const int32_t *nseg,
                                                             const int32_t *kbase, const int32_t *part,
                                                             const int32_t *nw, unsigned long long *pw)
{
    __shared__ unsigned long long acc[1024];
    int64_t vf = (int64_t)blockIdx.x * blockDim.x;
    int64_t v = vf + threadIdx.x;
    int64_t vl = vf + blockDim.x - 1 < N ? vf + blockDim.x - 1 : N - 1;
    int32_t g0 = nseg[vf];
    int32_t kg = kbase[g0 + 1] - kbase[g0];
    bool one = nseg[vl] == g0 && kg <= 1024;
    if (one) {
        for (int i = threadIdx.x; i < kg; i += blockDim.x) acc[i] = 0;
        __syncthreads();
    }
    if (v < N) {
        int32_t g = nseg[v], p = part[v];
        int32_t k = kbase[g + 1] - kbase[g];
        if (p >= 0 && p < k) {
            unsigned long long w = (unsigned long long)nw[v];
            if (one) atomicAdd(&acc[p], w);
            else atomicAdd(&pw[kbase[g] + p], w);
        }
    }
    if (one) {
        __syncthreads();
        for (int i = threadIdx.x; i < kg; i += blockDim.x)
            if (acc[i]) atomicAdd(&pw[kbase[g0] + i], acc[i]);
    }
}

__global__ void k_seg_max(int32_t n, const int32_t *kbase, const unsigned long long *pw,
                          unsigned long long *out)
{
    int32_t g = blockIdx.x * blockDim.x + threadIdx.x;
    if (g >= n) return;
    unsigned long long m = 0;
    for (int32_t i = kbase[g]; i < kbase[g + 1]; i++) m = pw[i] > m ? pw[i] : m;
    out[g] = m;
}

}  // namespace bp
