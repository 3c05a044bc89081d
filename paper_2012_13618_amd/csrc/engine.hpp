// Host driver of the device-resident multilevel bisection engine.
#pragma once
#include "batch.hpp"
#include "coarsen.hpp"
#include "kway.hpp"
#include "refine.hpp"
#include "uncoarsen.hpp"
#include "balance.hpp"
#include "transpose.hpp"

namespace bp {

struct Input {
    int32_t N = 0, E = 0;
    const int32_t *off = nullptr, *pins = nullptr, *nw = nullptr, *hw = nullptr;  // device
};

// Launch schedule (results never depend on it): see bp_schedule.
struct Schedule {
    int32_t incremental_min_pins = 1 << 16;
    int32_t seg_select_max_nodes = 1 << 14;
    int32_t round_chunk_max = 32;
    int32_t fused_pick_lists = 8;
    int32_t fuse_max_pins = 1 << 17;
    int32_t chunk_select_max_nodes = 1 << 18;
    int32_t graph_rounds = 0;
};

constexpr int kCaptureDevices = 64;

Schedule current_schedule();  // the process-wide schedule (a copy, taken under a lock)

struct Ctx {
    LaunchCtx lc;
    Schedule sched = current_schedule();
    Arena *ar = nullptr;
    LevelInfo *info_h = nullptr;  // pinned host
    LevelInfo *info_d = nullptr;  // device
    bp_params prm{};
    int64_t pins_coarsened = 0, pins_refined = 0;
    int32_t first_levels = -1;
    int32_t bisections = 0;
    bool no_graphs = false;  // the call may not capture (the allocation-free entry point)
    int32_t graph_replays = 0;
    std::vector<int32_t> tree_depth;  // most coarsening steps of a bisection, per tree level

    LevelInfo &readback()
    {
        BP_HIP(hipMemcpyAsync(info_h, info_d, sizeof(LevelInfo), hipMemcpyDeviceToHost, lc.stream));
        lc.sync();
        return *info_h;
    }
    void clear_info() { fill(lc, (int32_t *)info_d, (int64_t)(sizeof(LevelInfo) / 4), 0); }
};

// ---- small kernels used only by the driver -------------------------------------

__global__ void k_set_segs_root(int32_t N, int32_t E, int32_t *nbase, int32_t *hbase)
{
    nbase[0] = 0;
    nbase[1] = N;
    hbase[0] = 0;
    hbase[1] = E;
}

__global__ void k_set_i32(int32_t *p, int32_t v) { *p = v; }

__global__ void k_empty(int32_t) {}

// Segment weights W[s] (chunked; per-segment sums in LDS).
__global__ __launch_bounds__(kBlock) void k_seg_total(int32_t N, const int32_t *nseg,
                                                      const int32_t *nw, unsigned long long *W)
{
    __shared__ unsigned long long acc[kAggLists];
    int64_t lo, hi;
    reduce_chunk(N, gridDim.x, blockIdx.x, lo, hi);
    if (lo >= hi) return;
    int32_t s0 = nseg[lo], ns = nseg[hi - 1] + 1 - s0;
    bool local = ns <= kAggLists;
    for (int i = threadIdx.x; i < kAggLists; i += blockDim.x) acc[i] = 0;
    __syncthreads();
    for (int64_t v = lo + threadIdx.x; v < hi; v += blockDim.x) {
        unsigned long long w = (unsigned long long)nw[v];
        if (!w) continue;
        if (local) atomicAdd(&acc[nseg[v] - s0], w);
        else atomicAdd(&W[nseg[v]], w);
    }
    __syncthreads();
    if (local)
        for (int i = threadIdx.x; i < ns; i += blockDim.x)
            if (acc[i]) atomicAdd(&W[s0 + i], acc[i]);
}

// Bisection split, side bounds and coarsening start state of every segment.
// bound_s = max(ceil(W k_s / k_sub), floor(W k_s F / (k_sub 2^32))), with F the
// per-bisection fixed-point factor of the graph the segment descends from.
__global__ void k_seg_setup(int32_t S, const int32_t *ksub, const int32_t *k0_fixed,
                            const int64_t *W, const uint64_t *Fs,
                            const int32_t *nbase, const int32_t *hbase, const int32_t *off, int32_t max_levels,
                            int32_t min_nodes, int32_t *k0, int32_t *k1, int64_t *max0,
                            int64_t *max1, uint8_t *active, int32_t *coarsest, int32_t *stuck,
                            LevelInfo *info)
{
    int32_t s = blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= S) return;
    int32_t ks = ksub[s];
    int32_t a = k0_fixed ? k0_fixed[s] : (ks + 1) / 2, b = ks - a;
    k0[s] = a;
    k1[s] = b;
    uint64_t w = (uint64_t)W[s], F = Fs[s];
    for (int sd = 0; sd < 2; sd++) {
        uint64_t kk = sd ? b : a;
        uint64_t prod = w * kk;  // < 2^62
        uint64_t lo = prod * F, hi = __umul64hi(prod, F);
        uint64_t shifted = (hi << 32) | (lo >> 32);  // floor(prod * F / 2^32)
        uint64_t fl = shifted / (uint64_t)ks;
        uint64_t ce = (prod + (uint64_t)ks - 1) / (uint64_t)ks;
        int64_t mx = (int64_t)(fl > ce ? fl : ce);
        if (sd) max1[s] = mx;
        else max0[s] = mx;
    }
    int32_t ns = nbase[s + 1] - nbase[s], es = hbase[s + 1] - hbase[s];
    bool go = max_levels > 0 && es > 0 && ns > min_nodes;
    active[s] = go;
    coarsest[s] = 0;
    stuck[s] = 0;
    if (go) atomicAdd(&info->active, 1);
    atomicMax(&info->maxseg_nodes, ns);
    atomicMax(&info->maxseg_pins, off[hbase[s + 1]] - off[hbase[s]]);
    atomicMax(&info->maxseg_hedges, es);
}

// ---- level construction ----------------------------------------------------------

inline void alloc_lists(Arena &ar, Level &L, int64_t bound)
{
    L.lmid = ar.get<int32_t>(bound);
    L.lbig = ar.get<int32_t>(bound);
    L.lhuge = ar.get<int32_t>(bound);
}

// Classify a level's hyperedges into schedule lists (counts land in info).
inline void classify(Ctx &cx, Level &L, int32_t *counters)
{
    alloc_lists(*cx.ar, L, L.E);
    launch(cx.lc, "classify", 4.0 * L.E, k_classify, ceil_div(L.E, kClsItems), kBlock, 0, L.E,
           (const int32_t *)L.off, (const uint64_t *)nullptr, L.lmid, L.lbig, L.lhuge, counters);
}

// Level 0 of the root problem: the input without hyperedges of < 2 pins.
inline Level normalize(Ctx &cx, const Input &in)
{
    Arena &ar = *cx.ar;
    Level L;
    L.S = 1;
    L.N = in.N;
    const int32_t *off = in.off, *hw = in.hw;
    int32_t *dst = ar.get<int32_t>(in.E);
    L.off = ar.get<int32_t>((int64_t)in.E + 1);
    L.hw = ar.get<int32_t>(in.E);
    uint64_t *tot = ar.get<uint64_t>(1);
    int32_t *loff = L.off, *lhw = L.hw;
    scan<uint64_t>(
        cx.lc, ar, "normalize_scan", in.E,
        [=] __device__(int64_t e) -> uint64_t {
            int32_t d = off[e + 1] - off[e];
            return d >= 2 ? ((1ull << 32) | (uint32_t)d) : 0ull;
        },
        [=] __device__(int64_t e, uint64_t ex, uint64_t val) {
            if (!val) return;
            int32_t id = (int32_t)(ex >> 32);
            loff[id] = (int32_t)ex;
            lhw[id] = hw ? hw[e] : 1;
            dst[e] = (int32_t)ex;
        },
        tot);
    BP_HIP(hipMemcpyAsync(cx.info_h, tot, sizeof(uint64_t), hipMemcpyDeviceToHost, cx.lc.stream));
    cx.lc.sync();
    uint64_t t = *(uint64_t *)cx.info_h;
    L.E = (int32_t)(t >> 32);
    L.P = (int32_t)(t & 0xffffffffu);
    L.pins = ar.get<int32_t>(L.P);
    launch(cx.lc, "normalize_copy", 8.0 * L.P, k_norm_copy, ceil_div(in.E, kBlock), kBlock, 0, in.E,
           in.off, in.pins, (const int32_t *)dst, L.pins);
    launch(cx.lc, "normalize", 4.0, k_set_i32, 1, 1, 0, L.off + L.E, L.P);
    L.nw = ar.get<int32_t>(L.N);
    launch(cx.lc, "normalize", 8.0 * L.N, k_copy_weights, ceil_div(L.N, kBlock) < 4096 ? ceil_div(L.N, kBlock) : 4096,
           kBlock, 0, (int64_t)L.N, in.nw, L.nw);
    L.nseg = ar.get<int32_t>(L.N);
    L.hseg = ar.get<int32_t>(L.E);
    fill(cx.lc, L.nseg, L.N, 0);
    fill(cx.lc, L.hseg, L.E, 0);
    L.nbase = ar.get<int32_t>(2);
    L.hbase = ar.get<int32_t>(2);
    launch(cx.lc, "normalize", 16.0, k_set_segs_root, 1, 1, 0, L.N, L.E, L.nbase, L.hbase);
    return L;
}

// A level viewing a caller's CSR as one segment (single-step entry points).
inline Level view_level(Ctx &cx, const Input &in)
{
    Arena &ar = *cx.ar;
    Level L;
    L.S = 1;
    L.N = in.N;
    L.E = in.E;
    L.off = const_cast<int32_t *>(in.off);
    L.pins = const_cast<int32_t *>(in.pins);
    int32_t p = 0;
    BP_HIP(hipMemcpyAsync(cx.info_h, in.off + in.E, sizeof(int32_t), hipMemcpyDeviceToHost, cx.lc.stream));
    cx.lc.sync();
    p = *(int32_t *)cx.info_h;
    L.P = p;
    L.nw = ar.get<int32_t>(L.N);
    L.hw = ar.get<int32_t>(L.E);
    int64_t g = 4096;
    launch(cx.lc, "view", 8.0 * L.N, k_copy_weights, g, kBlock, 0, (int64_t)L.N, in.nw, L.nw);
    launch(cx.lc, "view", 8.0 * L.E, k_copy_weights, g, kBlock, 0, (int64_t)L.E, in.hw, L.hw);
    L.nseg = ar.get<int32_t>(L.N);
    L.hseg = ar.get<int32_t>(L.E);
    fill(cx.lc, L.nseg, L.N, 0);
    fill(cx.lc, L.hseg, L.E, 0);
    L.nbase = ar.get<int32_t>(2);
    L.hbase = ar.get<int32_t>(2);
    launch(cx.lc, "view", 16.0, k_set_segs_root, 1, 1, 0, L.N, L.E, L.nbase, L.hbase);
    return L;
}

inline Segs alloc_segs(Arena &ar, int32_t S)
{
    Segs g;
    g.S = S;
    g.k0 = ar.get<int32_t>(S);
    g.k1 = ar.get<int32_t>(S);
    g.lo = ar.get<int32_t>(S);
    g.W = ar.get<int64_t>(S);
    g.max0 = ar.get<int64_t>(S);
    g.max1 = ar.get<int64_t>(S);
    g.active = ar.get<uint8_t>(S);
    g.coarsest = ar.get<int32_t>(S);
    g.w = ar.get<int64_t>(2 * S);
    g.cnt1 = ar.get<int32_t>(S);
    g.mode = ar.get<uint8_t>(S);
    g.gmask = ar.get<uint8_t>(S);
    g.m = ar.get<int32_t>(S);
    g.need = ar.get<int64_t>(S);
    g.room = ar.get<int64_t>(S);
    g.bal_moved = ar.get<int64_t>(2 * S);
    g.done = ar.get<uint8_t>(S);
    g.stuck = ar.get<int32_t>(S);
    g.root_levels = ar.get<int32_t>(1);
    SelState &st = g.st;
    st.hist = ar.get<uint32_t>((int64_t)2 * S * kBins);
    st.tot = ar.get<int32_t>(2 * S);
    st.gmax = ar.get<int32_t>(2 * S);
    st.gmin = ar.get<int32_t>(2 * S);
    st.rsel = ar.get<int32_t>(2 * S);
    st.rem = ar.get<int32_t>(2 * S);
    st.kbits = ar.get<int32_t>(2 * S);
    st.kpre = ar.get<uint64_t>(2 * S);
    st.kthr = ar.get<uint64_t>(2 * S);
    st.done = ar.get<uint8_t>(2 * S);
    st.ctl = ar.get<int32_t>(4);
    st.tick = ar.get<int32_t>(S);
    g.go = ar.get<int32_t>(8);
    g.ccount = ar.get<int32_t>(S);
    return g;
}

// one graph of a batch (device arrays)
struct BatchItem {
    int32_t N = 0, E = 0;
    const int32_t *off = nullptr, *pins = nullptr, *nw = nullptr, *hw = nullptr;
    int32_t k = 1;
    double eps = 0.0;
};

struct BatchOut {
    int64_t cut = 0, maxw = 0, limit = 0, W = 0;
    int32_t balanced = 1, k = 1;
};

std::vector<BatchOut> partition_batch(Ctx &cx, const std::vector<BatchItem> &it,
                                      const std::vector<int32_t *> &d_out, int32_t *tree_levels);
int64_t part_limit(int64_t W, int32_t k, double eps);
uint64_t eps_factor(int32_t k, double eps);

void coarsen_level(Ctx &cx, Level &f, Segs &sg, uint8_t *&sact, uint8_t *&sact_next, int32_t l,
                   Level &c);
void build_incidence(Ctx &cx, Level &L);
// hkey: the level's hyperedge keys when already computed, else null
void run_match_keys(Ctx &cx, Level &L, const uint8_t *sact, uint64_t *key, const uint64_t *hkey = nullptr);
void bisect_all(Ctx &cx, Level &L0, Segs &sg, int32_t active0);
void run_gains(Ctx &cx, Level &L, Segs &sg, int32_t *gain, bool stats, const int32_t *go);
void run_select(Ctx &cx, Level &L, Segs &sg, const int32_t *gain, const int32_t *go, int32_t clip = 0);

}  // namespace bp
