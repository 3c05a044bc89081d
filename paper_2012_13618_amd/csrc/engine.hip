// Multilevel bisection engine and the C ABI (include/bipart.h).
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <string>
#include <vector>
#include <chrono>
#include <mutex>

#include "engine.hpp"

namespace bp {

// A sweep must never launch over a bucket whose list was not built.
static void check_lists(const Level &L)
{
    if ((L.nmid > 0 && !L.lmid) || (L.nbig > 0 && !L.lbig) || (L.nhuge > 0 && !L.lhuge))
        throw Error(BP_ERR_DEVICE, "internal: hyperedge schedule lists missing");
    if (L.noff && (!L.ncount || !L.chunk_node || !L.chunk_beg || !L.chunk_big || !L.big_chunks ||
                   !L.big_done))
        throw Error(BP_ERR_DEVICE, "internal: node schedule lists missing");
}

static std::mutex g_sched_mu;
static Schedule g_sched;

Schedule current_schedule()
{
    std::lock_guard<std::mutex> g(g_sched_mu);
    return g_sched;
}

static void set_schedule(const Schedule &s)
{
    std::lock_guard<std::mutex> g(g_sched_mu);
    g_sched = s;
}

// ---- one coarsening step ------------------------------------------------------

// The coarse level's hyperedge lists by degree (blocks [0, ncls)) and the copy
// of its pins (the other blocks, by degree bucket of the fine hyperedges), in
// one launch: their outputs are disjoint.
__global__ __launch_bounds__(kBlock) void k_classify_copy(int64_t ncls, int32_t E, const int32_t *coff,
                                                          const uint64_t *tot, int32_t *lmid, int32_t *lbig,
                                                          int32_t *lhuge, int32_t *counters, CopyPinsOp op,
                                                          int32_t nmid, const int32_t *flmid, int32_t nbig,
                                                          const int32_t *flbig)
{
    int64_t b = blockIdx.x;
    if (b < ncls) {
        classify_block(b, E, coff, tot, lmid, lbig, lhuge, counters);
        return;
    }
    b -= ncls;
    int64_t ns = ceil_div(E, kBlock), nw = ceil_div(nmid, kBlock / 64);
    if (b < ns) op.template run<SMALL>(b, E, nullptr);
    else if (b < ns + nw) op.template run<WAVE>(b - ns, nmid, flmid);
    else op.template run<BLOCK>(b - ns - nw, nbig, flbig);
}

void coarsen_level(Ctx &cx, Level &f, Segs &sg, uint8_t *&sact, uint8_t *&sact_next, int32_t l,
                   Level &c)
{
    Arena &ar = *cx.ar;
    LaunchCtx &lc = cx.lc;
    const int32_t N = f.N, E = f.E, P = f.P, S = f.S;
    check_lists(f);
    cx.pins_coarsened += P;
    CoarsenBufs b;
    b.key = ar.get<uint64_t>(N);
    b.match = ar.get<int32_t>(N);
    b.grp = ar.get<int32_t>(N);
    b.cid = ar.get<int32_t>(N);
    b.cg = ar.get<uint64_t>(E);
    b.lead = ar.get<int32_t>(E);
    b.qpins = ar.get<int32_t>(P);
    b.qlen = ar.get<int32_t>(E);
    b.fp = ar.get<uint64_t>(E);
    b.hslot = ar.get<int32_t>(E);
    b.rep = ar.get<int32_t>(E);
    b.wsum = ar.get<int32_t>(E);
    b.hdst = ar.get<int32_t>(E);
    b.hb_tmp = ar.get<int32_t>(S);
    int64_t T = 1024;
    while (T < 2 * (int64_t)E) T <<= 1;
    b.tmask = (int32_t)(T - 1);
    b.tkeys = ar.get<uint64_t>(T);
    b.tmin = ar.get<int32_t>(T);
    b.counters = ar.get<int32_t>(8);
    b.totN = ar.get<int32_t>(1);
    b.totEP = ar.get<uint64_t>(1);

    f.parent = ar.get<int32_t>(N);
    c.S = S;
    c.nw = ar.get<int32_t>(N);
    c.nseg = ar.get<int32_t>(N);
    c.off = ar.get<int32_t>((int64_t)E + 1);
    c.pins = ar.get<int32_t>(P);
    c.hw = ar.get<int32_t>(E);
    c.hseg = ar.get<int32_t>(E);
    c.nbase = ar.get<int32_t>(S + 1);
    c.hbase = ar.get<int32_t>(S + 1);
    alloc_lists(ar, c, E);

    int64_t initn = std::max<int64_t>(std::max<int64_t>(N, E), T);
    uint64_t *hkey = ar.get<uint64_t>(E);
    HedgeKeyArgs hk{(const int32_t *)f.off, (const int32_t *)f.hw, (const int32_t *)f.hseg,
                    (const int32_t *)f.hbase, sact, cx.prm.policy, hkey};
    launch(lc, "coarsen_init", 8.0 * N + 16.0 * E + 12.0 * T + 20.0 * E, k_coarsen_init,
           std::min<int64_t>(ceil_div(initn, kBlock), 8192), kBlock, 0, N, E, T, b.key, b.grp,
           c.nw, b.cg, b.lead, b.wsum, b.tkeys, b.tmin, b.counters, hk);

    // Algorithm 1: per-node minimum over its own hyperedges' keys
    run_match_keys(cx, f, sact, b.key, hkey);
    launch(lc, "decode", 16.0 * N, k_decode, ceil_div(N, kBlock), kBlock, 0, N,
           (const uint64_t *)b.key, (const int32_t *)f.nseg, (const int32_t *)f.hbase,
           (const uint8_t *)sact, (const int32_t *)f.nw, b.match, b.cg);

    // Algorithm 2, singletons
    AttachOp aop{(const int32_t *)f.off, (const int32_t *)f.pins, (const int32_t *)f.hseg, (const uint8_t *)sact,
                 (const int32_t *)b.match, (const uint64_t *)b.cg, b.grp};
    launch(lc, "attach", 4.0 * E, k_buckets<AttachOp>, buckets_grid(E, f.nmid, f.nbig), kBlock, 0, aop, E, f.nmid,
           (const int32_t *)f.lmid, f.nbig, (const int32_t *)f.lbig);
    launch(lc, "lead", 12.0 * N, k_lead, ceil_div(N, kBlock), kBlock, 0, N,
           (const int32_t *)f.nseg, (const uint8_t *)sact, (const int32_t *)b.match,
           (const uint64_t *)b.cg, b.grp, b.lead);

    // coarse node ids: exclusive scan of leader flags
    {
        const int32_t *nseg = f.nseg, *grp = b.grp, *lead = b.lead;
        const uint8_t *sa = sact;
        int32_t *cid = b.cid;
        scan<int32_t>(
            lc, ar, "node_ids", N,
            [=] __device__(int64_t v) -> int32_t {
                if (!sa[nseg[v]]) return 0;
                int32_t g = grp[v];
                return (g < 0 || lead[g] == v) ? 1 : 0;
            },
            [=] __device__(int64_t v, int32_t ex, int32_t) { cid[v] = ex; }, b.totN);
    }
    launch(lc, "parent", 20.0 * N, k_parent, ceil_div(N, kBlock), kBlock, 0, N,
           (const int32_t *)f.nseg, (const uint8_t *)sact, (const int32_t *)b.grp,
           (const int32_t *)b.lead, (const int32_t *)b.cid, (const int32_t *)f.nw, f.parent, c.nw,
           c.nseg);

    // Algorithm 2, coarse hyperedges
    launch(lc, "qbuild", 4.0 * E + 12.0 * P, k_qbuild_sw, ceil_div(E, kBlock) + ceil_div(f.nmid, kBlock / 64),
           kBlock, 0, E, f.nmid, (const int32_t *)f.lmid, (const int32_t *)f.off, (const int32_t *)f.pins,
           (const int32_t *)f.hseg, (const uint8_t *)sact, (const int32_t *)f.parent, b.qpins, b.qlen, b.fp);
    launch(lc, "qbuild_block", 0.0, k_qbuild_big_waves, ceil_div(f.nbig, kBlock / 64), kBlock, 0, f.nbig,
           (const int32_t *)f.lbig, (const int32_t *)f.off, (const int32_t *)f.pins, (const int32_t *)f.hseg,
           (const uint8_t *)sact, (const int32_t *)f.parent, b.qpins, b.qlen, b.fp);
    launch(lc, "qbuild_block", 0.0, k_qbuild_block, sched_grid<BLOCK>(f.nbig), kBlock,
           (size_t)kBigMax * sizeof(int32_t), f.nbig, (const int32_t *)f.lbig,
           (const int32_t *)f.off, (const int32_t *)f.pins, (const int32_t *)f.hseg,
           (const uint8_t *)sact, (const int32_t *)f.parent, b.qpins, b.qlen, b.fp);
    if (f.nhuge > 0) {
        b.huge_scratch = ar.get<int32_t>(next_pow2(P > 0 ? P : 1));
        for (int32_t i = 0; i < f.nhuge; i++)
            launch(lc, "qbuild_huge", 0.0, k_qbuild_huge, 1, 1024, 0, (const int32_t *)f.lhuge, i,
                   (const int32_t *)f.off, (const int32_t *)f.pins, (const int32_t *)f.hseg,
                   (const uint8_t *)sact, (const int32_t *)f.parent, b.huge_scratch, b.qpins,
                   b.qlen, b.fp);
    }

    // duplicate pin sets
    launch(lc, "dedup", 16.0 * E, k_dd_insert, ceil_div(E, kBlock), kBlock, 0, E,
           (const int32_t *)b.qlen, (const uint64_t *)b.fp, (const int32_t *)b.rep, 0,
           (unsigned long long *)b.tkeys, b.tmin, b.tmask, b.hslot);
    launch(lc, "dedup", 20.0 * E, k_dd_resolve, ceil_div(E, kBlock), kBlock, 0, E,
           (const int32_t *)f.off, (const int32_t *)b.qpins, (const int32_t *)b.qlen,
           (const int32_t *)f.hw, (const int32_t *)b.hslot, (const int32_t *)b.tmin, 0, b.rep,
           b.wsum, b.counters);

    auto compact = [&]() {
        const int32_t *rep = b.rep, *qlen = b.qlen, *hseg = f.hseg, *hbase = f.hbase,
                      *wsum = b.wsum;
        int32_t *coff = c.off, *chw = c.hw, *chseg = c.hseg, *hdst = b.hdst, *hbt = b.hb_tmp;
        scan<uint64_t>(
            lc, ar, "hedge_ids", E,
            [=] __device__(int64_t e) -> uint64_t {
                return rep[e] == e ? ((1ull << 32) | (uint32_t)qlen[e]) : 0ull;
            },
            [=] __device__(int64_t e, uint64_t ex, uint64_t val) {
                int32_t s = hseg[e];
                if (e == hbase[s]) hbt[s] = (int32_t)(ex >> 32);
                int32_t id = (int32_t)(ex >> 32);
                if (val) {
                    coff[id] = (int32_t)ex;
                    chw[id] = wsum[e];
                    chseg[id] = s;
                    hdst[e] = (int32_t)ex;
                }
            },
            b.totEP);
        CopyPinsOp cop{(const int32_t *)f.off, rep, qlen, (const int32_t *)b.qpins, (const int32_t *)b.hdst, c.pins};
        int64_t ncls = ceil_div(E, kClsItems);
        launch(lc, "copy_pins", 4.0 * E + 8.0 * P, k_classify_copy, ncls + buckets_grid(E, f.nmid, f.nbig), kBlock, 0,
               ncls, E, (const int32_t *)c.off, (const uint64_t *)b.totEP, c.lmid, c.lbig, c.lhuge, b.counters, cop,
               f.nmid, (const int32_t *)f.lmid, f.nbig, (const int32_t *)f.lbig);
        launch(lc, "level_fixup", 0.0, k_level_fixup, 1, kFixupThreads, 0, S, N, E, (const int32_t *)f.nbase,
               (const int32_t *)f.hbase, (const int32_t *)b.cid, (const int32_t *)b.hb_tmp,
               (const int32_t *)b.totN, (const uint64_t *)b.totEP, l + 1, cx.prm.max_levels,
               cx.prm.min_coarse_nodes, (const uint8_t *)sact, sact_next, sg.coarsest, c.nbase,
               c.hbase, c.off, (const int32_t *)b.counters, cx.info_d);
    };
    compact();
    LevelInfo inf = cx.readback();
    if (inf.unresolved > 0) {
        // a fingerprint shared by different pin sets: re-hash the open ones
        for (uint64_t salt = 1; inf.unresolved > 0; salt++) {
            if (salt > 64) throw Error(BP_ERR_DEVICE, "duplicate check did not converge");
            fill(lc, b.tkeys, T, kEmptySlot);
            fill(lc, b.tmin, T, INT32_MAX);
            fill(lc, b.counters, 8, 0);
            launch(lc, "dedup", 0.0, k_refingerprint, ceil_div(E, kBlock), kBlock, 0, E,
                   (const int32_t *)f.off, (const int32_t *)b.qpins, (const int32_t *)b.qlen,
                   (const int32_t *)b.rep, salt * 0x9E3779B97F4A7C15ull, b.fp);
            launch(lc, "dedup", 0.0, k_dd_insert, ceil_div(E, kBlock), kBlock, 0, E,
                   (const int32_t *)b.qlen, (const uint64_t *)b.fp, (const int32_t *)b.rep, 1,
                   (unsigned long long *)b.tkeys, b.tmin, b.tmask, b.hslot);
            launch(lc, "dedup", 0.0, k_dd_resolve, ceil_div(E, kBlock), kBlock, 0, E,
                   (const int32_t *)f.off, (const int32_t *)b.qpins, (const int32_t *)b.qlen,
                   (const int32_t *)f.hw, (const int32_t *)b.hslot, (const int32_t *)b.tmin, 1,
                   b.rep, b.wsum, b.counters);
            launch(lc, "dedup", 0.0, k_level_fixup, 1, kFixupThreads, 0, S, N, E, (const int32_t *)f.nbase,
                   (const int32_t *)f.hbase, (const int32_t *)b.cid, (const int32_t *)b.hb_tmp,
                   (const int32_t *)b.totN, (const uint64_t *)b.totEP, l + 1, cx.prm.max_levels,
                   cx.prm.min_coarse_nodes, (const uint8_t *)sact, sact_next, sg.coarsest,
                   c.nbase, c.hbase, c.off, (const int32_t *)b.counters, cx.info_d);
            inf = cx.readback();
        }
        fill(lc, b.counters, 8, 0);
        compact();
        inf = cx.readback();
    }
    c.N = inf.N;
    c.E = inf.E;
    c.P = inf.P;
    c.nmid = inf.nmid;
    c.nbig = inf.nbig;
    c.nhuge = inf.nhuge;
    c.maxseg_nodes = inf.maxseg_nodes;
    c.maxseg_pins = inf.maxseg_pins;
    c.maxseg_hedges = inf.maxseg_hedges;
    std::swap(sact, sact_next);
    build_incidence(cx, c);
}

// ---- node-major incidence ------------------------------------------------------------

void build_incidence(Ctx &cx, Level &L)
{
    Arena &ar = *cx.ar;
    LaunchCtx &lc = cx.lc;
    check_lists(L);
    const int32_t N = L.N, E = L.E, P = L.P;
    uint32_t *k0 = ar.get<uint32_t>(P), *k1 = ar.get<uint32_t>(P);
    int32_t *v0 = ar.get<int32_t>(P), *v1 = ar.get<int32_t>(P);
    ExpandPairsOp eop{(const int32_t *)L.off, v0};
    launch(lc, "incidence", 4.0 * P, k_buckets<ExpandPairsOp>, buckets_grid(E, L.nmid, L.nbig), kBlock, 0, eop, E,
           L.nmid, (const int32_t *)L.lmid, L.nbig, (const int32_t *)L.lbig);
    int bits = 0;
    while (bits < 31 && ((int64_t)1 << bits) < (int64_t)N) bits++;
    int64_t ntiles = ceil_div(P > 0 ? P : 1, kRsTile);
    uint32_t *counts = ar.get<uint32_t>(256 * ntiles), *offs = ar.get<uint32_t>(256 * ntiles);
    uint32_t *tot = ar.get<uint32_t>(1);
    // the first pass reads the keys (the pins) in place
    const uint32_t *kin = (const uint32_t *)L.pins;
    for (int shift = 0; shift < bits && P > 0; shift += 8) {
        launch(lc, "radix_hist", 4.0 * P, k_rs_hist, ntiles, kBlock, 0, kin, (int64_t)P, shift, counts, ntiles);
        const uint32_t *cnt = counts;
        uint32_t *of = offs;
        scan<uint32_t>(
            lc, ar, "radix_scan", 256 * ntiles, [=] __device__(int64_t i) -> uint32_t { return cnt[i]; },
            [=] __device__(int64_t i, uint32_t ex, uint32_t) { of[i] = ex; }, tot);
        launch(lc, "radix_scatter", 16.0 * P, k_rs_scatter, ntiles, kBlock, 0, kin, (const int32_t *)v0,
               (int64_t)P, shift, (const uint32_t *)offs, ntiles, k1, v1);
        kin = k1;
        std::swap(k0, k1);
        std::swap(v0, v1);
    }
    L.inc = v0;
    L.noff = ar.get<int32_t>((int64_t)N + 1);
    // (kin: the sorted keys, or the pins themselves when no pass ran)
    launch(lc, "incidence", 4.0 * N, k_node_offsets, ceil_div((int64_t)N + 1, kBlock), kBlock, 0, kin,
           (int64_t)P, N, L.noff);
    L.nmid_bound = std::min<int64_t>(N, P / (kNodeSmallMax + 1)) + 1;
    L.nbig_bound = std::min<int64_t>(N, P / (kNodeMidMax + 1)) + 1;
    L.lnmid = ar.get<int32_t>(L.nmid_bound);
    L.lnbig = ar.get<int32_t>(L.nbig_bound);
    L.ncount = ar.get<int32_t>(4);
    L.bigslot = ar.get<int32_t>(N);
    Fills().add(L.ncount, 4, 0).add(L.bigslot, (int64_t)N, -1).run(lc);
    launch(lc, "incidence", 8.0 * N, k_classify_nodes, ceil_div(N, kClsNodes), kBlock, 0, N,
           (const int32_t *)L.noff, L.lnmid, L.lnbig, L.ncount);
    L.nchunk_bound = (int64_t)P / kNodeChunk + L.nbig_bound + 1;
    L.chunk_node = ar.get<int32_t>(L.nchunk_bound);
    L.chunk_beg = ar.get<int32_t>(L.nchunk_bound);
    L.chunk_big = ar.get<int32_t>(L.nchunk_bound);
    L.big_chunks = ar.get<int32_t>(L.nbig_bound);
    L.big_done = ar.get<int32_t>(L.nbig_bound);
    launch(lc, "incidence", 0.0, k_big_chunks, 1, kBlock, 0, (const int32_t *)L.lnbig,
           (const int32_t *)L.noff, L.ncount, L.chunk_node, L.chunk_beg, L.chunk_big, L.big_chunks,
           L.bigslot);
    L.cc = ar.get<int2>(E);
}

void run_match_keys(Ctx &cx, Level &L, const uint8_t *sact, uint64_t *key, const uint64_t *hkey_ready)
{
    Arena &ar = *cx.ar;
    LaunchCtx &lc = cx.lc;
    const uint64_t *hkey = hkey_ready;
    if (!hkey) {
        uint64_t *h = ar.get<uint64_t>(L.E);
        launch(lc, "hedge_keys", 20.0 * L.E, k_hedge_keys, ceil_div(L.E, kBlock), kBlock, 0, L.E,
               (const int32_t *)L.off, (const int32_t *)L.hw, (const int32_t *)L.hseg,
               (const int32_t *)L.hbase, sact, cx.prm.policy, h);
        hkey = h;
    }
    double bytes = 8.0 * L.N + 4.0 * L.P + 8.0 * L.P + 8.0 * L.N;
    launch(lc, "match", bytes, k_match_sw, ceil_div(L.N, kBlock) + ceil_div(L.nmid_bound, kBlock / 64), kBlock, 0,
           L.N, (const int32_t *)L.ncount, (const int32_t *)L.lnmid, (const int32_t *)L.noff,
           (const int32_t *)L.inc, (const int32_t *)L.nseg, sact, (const uint64_t *)hkey, key);
    launch(lc, "match_chunks", 0.0, k_match_chunks, L.nchunk_bound, kBlock, 0, (const int32_t *)L.ncount,
           (const int32_t *)L.chunk_node, (const int32_t *)L.chunk_beg, (const int32_t *)L.noff,
           (const int32_t *)L.inc, (const int32_t *)L.nseg, sact, (const uint64_t *)hkey,
           (unsigned long long *)key);
}

// ---- gains and selection -----------------------------------------------------------

// Gains of the segments in sg.gmask: two launches.  With stats, the node pass
// also fills the per-list counts / gain extremes used by the selection.
void run_gains(Ctx &cx, Level &L, Segs &sg, int32_t *gain, bool stats, const int32_t *go)
{
    LaunchCtx &lc = cx.lc;
    check_lists(L);
    cx.pins_refined += L.P;
    int64_t hv = std::max<int64_t>(ceil_div(L.E, kBlock) + ceil_div(L.nmid, kBlock / 64) + L.nbig,
                                   ceil_div(L.nbig_bound, kBlock));
    double cb = L.cc_pk ? 4.0 : 8.0;  // bytes of one contribution pair
    double hb = 8.0 * L.E + 4.0 * L.E + 4.0 * L.P + 1.0 * L.P + cb * L.E;
    launch(lc, "gain_hedges", hb, k_gain_hedges, hv, kBlock, 0, L.E, (const int32_t *)L.lmid, L.nmid,
           (const int32_t *)L.lbig, L.nbig, (const int32_t *)L.off, (const int32_t *)L.pins,
           (const int32_t *)L.hw, (const int32_t *)L.hseg, (const uint8_t *)sg.gmask,
           (const uint8_t *)L.side, (void *)L.cc, L.cc_pk, go, (const int32_t *)L.lnbig, (const int32_t *)L.ncount, gain,
           L.big_done);
    int32_t nw = (int32_t)std::min<int64_t>(ceil_div(L.nmid_bound, kBlock / 64), kReduceBlocks);
    int64_t nv = reduce_grid(L.N) + nw + L.nchunk_bound;
    double nb = 8.0 * L.N + 4.0 * L.P + cb * L.P + 1.0 * L.N + 4.0 * L.N;
    launch(lc, "gain_nodes", nb, k_gain_nodes, nv, kBlock, 0, L.N, (const int32_t *)L.lnmid,
           (const int32_t *)L.lnbig, (const int32_t *)L.ncount, (const int32_t *)L.noff,
           (const int32_t *)L.inc, (const int32_t *)L.nseg, (const uint8_t *)sg.gmask,
           (const uint8_t *)L.side, (const void *)L.cc, L.cc_pk, gain, (const uint8_t *)sg.mode,
           stats ? sg.st.tot : nullptr, sg.st.gmax, sg.st.gmin, go, (const int32_t *)L.chunk_node,
           (const int32_t *)L.chunk_beg, (const int32_t *)L.chunk_big, (const int32_t *)L.big_chunks,
           L.big_done, L.S, nw);
}

static int id_bits(const Level &L)
{
    int bits = 0;
    while (bits < 31 && ((int64_t)1 << bits) < (int64_t)std::max(L.maxseg_nodes, 1)) bits++;
    return bits;
}

static SelView sel_view(Level &L, Segs &sg, const int32_t *gain)
{
    SelView sv;
    sv.gain = gain;
    sv.nseg = L.nseg;
    sv.nbase = L.nbase;
    sv.side = L.side;
    sv.mode = sg.mode;
    sv.m = sg.m;
    sv.idbits = id_bits(L);
    return sv;
}

// The first r nodes of every list in (gain desc, id asc) order: up to three
// digit passes over the gain span and then over the node id; passes that no
// list needs return at once.
// clip > 0: a balance round, whose finish orders the gathered nodes and
// keeps the first r, so a list may stop at a whole bin of at most clip keys
void run_select(Ctx &cx, Level &L, Segs &sg, const int32_t *gain, const int32_t *go, int32_t clip)
{
    LaunchCtx &lc = cx.lc;
    int idb = id_bits(L);
    // digits of the widest key: gain span (bounded per level) + node id
    int passes = std::max(1, (L.span_bits + idb + kDigit - 1) / kDigit);
    int32_t nl = 2 * L.S;
    // picks: by the last workgroup (few lists), by the last workgroup of each
    // segment (many lists), or by a launch of their own (no nodes at all)
    int fused = nl <= cx.sched.fused_pick_lists ? 1 : (L.N > 0 ? 2 : 0);
    SelView sv = sel_view(L, sg, gain);
    int64_t grid = std::max<int64_t>(1, ceil_div(L.N, kSelNodes));
    for (int p = 0; p < passes; p++) {
        launch(lc, "select", 10.0 * L.N, k_select_pass, grid, kBlock, 0, L.N, p, nl, idb, sv, sg.st,
               fused, go, clip);
        if (!fused)
            launch(lc, "select_pick", 0.0, k_select_pick, nl, kBlock, 0, nl, p, idb, sv, sg.st, go, clip);
    }
}

static void flip(Ctx &cx, Level &L, Segs &sg, const int32_t *gain, const int32_t *go);

// Whether a level's selections run in one workgroup per segment (kind 0:
// flips, kind 1: balance); that kernel computes its lists' sizes and gain
// extremes itself, so the gain passes need not.
static bool seg_path(const Ctx &cx, const Level &L, int kind)
{
    int32_t cap = kind == 0 ? seg_select_max<0, kSegThreads>() : seg_select_max<1, kSegThreads>();
    return L.maxseg_nodes <= std::min(cx.sched.seg_select_max_nodes, cap);
}

// Buffers of the chunked balance selection for levels of at most tab_n
// chunk table entries (none when tab_n is 0).
static void alloc_chunk_bufs(Arena &ar, Segs &sg, int64_t tab_n)
{
    sg.chunk_cand = nullptr;
    sg.chunk_tab_n = tab_n;
    if (tab_n == 0) return;
    sg.chunk_cand = ar.get<uint64_t>((int64_t)sg.S * kChunkMax * kChunkKeys);
    sg.chunk_ccnt = ar.get<int32_t>((int64_t)sg.S * kChunkMax);
    sg.chunk_tab = ar.get<int32_t>(2 * tab_n + 1);
}

// Whether a level's balance selections run in chunks (k_seg_select in chunk
// mode, then k_bal_merge): segments too large for one workgroup, but of at
// most kChunkMax chunks.
static bool chunk_path(const Ctx &cx, const Level &L)
{
    return !seg_path(cx, L, 1) && cx.sched.chunk_select_max_nodes > 0 &&
           L.maxseg_nodes <= std::min<int64_t>(cx.sched.chunk_select_max_nodes, (int64_t)kChunkMax * kChunkNodes);
}

// Selection and flip of the chosen nodes (Algorithm 3 rounds, Algorithm 5
// swaps): one workgroup per segment when every segment is small, else the
// multi-workgroup passes and a flip launch.
static void select_and_flip(Ctx &cx, Level &L, Segs &sg, const int32_t *gain, const int32_t *go)
{
    if (seg_path(cx, L, 0)) {
        BalFinish bf{};
        bf.side = L.side;
        if (L.maxseg_nodes <= seg_select_max<0, kSegThreadsSmall>())
            launch(cx.lc, "seg_select", 6.0 * L.N, k_seg_select<0, kSegThreadsSmall>, L.S, kSegThreadsSmall, 0,
                   L.S, sel_view(L, sg, gain), sg.st, id_bits(L), (const int32_t *)L.nw, (unsigned long long *)sg.w,
                   bf, go, ChunkArgs{});
        else
            launch(cx.lc, "seg_select", 6.0 * L.N, k_seg_select<0, kSegThreads>, L.S, kSegThreads, 0, L.S,
                   sel_view(L, sg, gain), sg.st, id_bits(L), (const int32_t *)L.nw, (unsigned long long *)sg.w,
                   bf, go, ChunkArgs{});
        return;
    }
    run_select(cx, L, sg, gain, go);
    flip(cx, L, sg, gain, go);
}

static void flip(Ctx &cx, Level &L, Segs &sg, const int32_t *gain, const int32_t *go)
{
    launch(cx.lc, "flip", 6.0 * L.N, k_flip, reduce_grid(L.N), kBlock, 0, L.N,
           sel_view(L, sg, gain), sg.st, L.side, (const int32_t *)L.nw, (unsigned long long *)sg.w, go);
}

// Rounds issued in chunks with one readback per chunk: the round kernels keep
// a device counter of segments still running and every later kernel of a
// finished round returns at once.
static bool trace_on()
{
    static int on = -1;
    if (on < 0) {
        const char *e = getenv("BP_TRACE");
        on = (e && *e && *e != '0') ? 1 : 0;
    }
    return on == 1;
}

// Graph replay of a level's rounds: every round after the first issues the
// same launches, which depend on the round index only through ri % 3 (its
// counter slot) and ri > 0, so three graphs, captured once from rounds
// 3, 4 and 5 on a private stream, replay every later round of the level on
// the call's stream.
struct RoundGraphs {
    hipGraph_t graph[3] = {nullptr, nullptr, nullptr};
    hipGraphExec_t exec[3] = {nullptr, nullptr, nullptr};
    int32_t launches[3] = {0, 0, 0};
    bool failed = false;
    ~RoundGraphs()
    {
        for (int k = 0; k < 3; k++) {
            if (exec[k]) (void)hipGraphExecDestroy(exec[k]);
            if (graph[k]) (void)hipGraphDestroy(graph[k]);
        }
    }
};

// A non-blocking stream of the current device for capturing (one per thread
// and device, kept for the process).
static hipStream_t capture_stream()
{
    thread_local hipStream_t st[kCaptureDevices] = {};
    int dev = 0;
    BP_HIP(hipGetDevice(&dev));
    if (dev < 0 || dev >= kCaptureDevices) return nullptr;
    if (!st[dev]) BP_HIP(hipStreamCreateWithFlags(&st[dev], hipStreamNonBlocking));
    return st[dev];
}

// Issues round ri through the level's graphs (capturing the slot's graph on
// first use); false when capture is not possible, the round then to be
// launched directly.
template <typename Round>
static bool replay_round(LaunchCtx &lc, Segs &sg, RoundGraphs &rg, int64_t ri, Round &round)
{
    int k = (int)(ri % 3);
    if (rg.failed) return false;
    if (!rg.exec[k]) {
        hipStream_t cs = capture_stream();
        if (!cs || hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal) != hipSuccess) {
            (void)hipGetLastError();
            rg.failed = true;
            return false;
        }
        hipStream_t own = lc.stream;
        int32_t before = lc.launches;
        lc.stream = cs;
        try {
            round((int32_t)(3 + k), sg.go + 4 + k);  // the same slot and ri > 0
        } catch (...) {
            lc.stream = own;
            hipGraph_t g = nullptr;
            (void)hipStreamEndCapture(cs, &g);
            if (g) (void)hipGraphDestroy(g);
            throw;
        }
        lc.stream = own;
        rg.launches[k] = lc.launches - before;
        lc.launches = before;
        BP_HIP(hipStreamEndCapture(cs, &rg.graph[k]));
        BP_HIP(hipGraphInstantiate(&rg.exec[k], rg.graph[k], nullptr, nullptr, 0));
    }
    BP_HIP(hipGraphLaunch(rg.exec[k], lc.stream));
    lc.launches += rg.launches[k];
    return true;
}

// With estimate (balance rounds), go[3] holds the rounds the segments still
// need as estimated by the last round: the next chunk is that long, and an
// estimate of zero ends the loop.  round(ri, gc) issues round ri; gc is its
// active-segment counter, which every kernel of the round checks.
template <typename Round>
static int64_t chunked_rounds(Ctx &cx, Segs &sg, int64_t limit, bool estimate, Round round)
{
    LaunchCtx &lc = cx.lc;
    int64_t issued = 0;
    int chunk = estimate ? 1 : 2;
    std::vector<int64_t> first;  // serial of each round's first launch (profiling)
    // graphs from round 6 on: a level that ends sooner never captures
    const bool graphs = cx.sched.graph_rounds && !lc.prof && !cx.no_graphs;
    RoundGraphs rg;
    lc.hold++;
    for (;;) {
        for (int i = 0; i < chunk; i++) {
            first.push_back(lc.serial);
            if (graphs && issued >= 6 && replay_round(lc, sg, rg, issued, round)) cx.graph_replays++;
            else round((int32_t)issued, sg.go + 4 + issued % 3);
            issued++;
        }
        BP_HIP(hipMemcpyAsync(cx.info_h, sg.go, 8 * sizeof(int32_t), hipMemcpyDeviceToHost, lc.stream));
        lc.sync(false);
        int32_t *g = (int32_t *)cx.info_h;
        int32_t last = g[4 + (issued - 1) % 3];
        int64_t ran = g[2] + (last > 0 ? 1 : 0);
        bool end = last == 0 || (estimate && g[3] == 0);
        if (lc.prof && ran < (int64_t)first.size()) lc.no_bytes(first[ran], lc.serial);
        if (end || issued > limit) {
            lc.hold--;
            if (lc.prof) lc.flush();
            if (!end) throw Error(BP_ERR_DEVICE, "round loop did not terminate");
            return ran;
        }
        // the estimate decides the next chunk, growing at most twofold
        int cap = cx.sched.round_chunk_max;
        chunk = estimate ? std::min({std::max(g[3], 1), 2 * chunk, cap}) : std::min(chunk * 2, cap);
    }
}

// Whether every segment of the level runs its rounds in one workgroup.
static bool fuse_all(const Ctx &cx, const Level &L)
{
    return cx.sched.fuse_max_pins > 0 && L.maxseg_nodes <= kFuseNodes && L.maxseg_pins <= cx.sched.fuse_max_pins &&
           L.maxseg_hedges <= kFuseHedges;
}

static int64_t fused_rounds_run(Ctx &cx, const int32_t *ctr)
{
    if (!trace_on()) return 0;
    int32_t r = 0;
    BP_HIP(hipMemcpyAsync(&r, ctr, sizeof(int32_t), hipMemcpyDeviceToHost, cx.lc.stream));
    cx.lc.sync();
    return r;
}

static int64_t initial_rounds(Ctx &cx, Level &L, Segs &sg, int32_t j, int32_t *gain)
{
    LaunchCtx &lc = cx.lc;
    int64_t gs = ceil_div(L.S, kBlock);
    fill(lc, sg.go, 8, 0);
    if (cx.sched.fuse_max_pins > 0) {
        // small segments: all rounds of Algorithm 3 in one workgroup each.  They
        // end with the loop test false, so the rounds below pass them by.
        FuseArgs fa{L.off, L.pins, L.hw, L.noff, L.inc, L.nw, L.nbase, L.hbase, L.side, sg.max0, sg.max1,
                    (unsigned long long *)sg.w, sg.done, sg.stuck, sg.go + 2, cx.sched.fuse_max_pins,
                    sg.coarsest, sg.k0, sg.k1, sg.W, j};
        launch(lc, "seg_initial", 8.0 * L.P, k_seg_fused<true>, L.S, kFuseThreads, 0, L.S, fa);
        if (fuse_all(cx, L)) return fused_rounds_run(cx, sg.go + 2);
        fill(lc, sg.go, 8, 0);
    }
    return chunked_rounds(cx, sg, (int64_t)L.N + 2, false, [&](int32_t ri, const int32_t *gc) {
        launch(lc, "round", 0.0, k_round_initial, gs, kBlock, 0, L.S, j, (const int32_t *)L.nbase,
               (const int32_t *)sg.coarsest, (const int32_t *)sg.k0, (const int32_t *)sg.k1,
               (const int64_t *)sg.W, (const unsigned long long *)sg.w, sg.cnt1, ri, sg.mode, sg.gmask, sg.m,
               sg.st, sg.go);
        run_gains(cx, L, sg, gain, !seg_path(cx, L, 0), gc);
        select_and_flip(cx, L, sg, gain, gc);
    });
}

static int64_t refine_level(Ctx &cx, Level &L, Segs &sg, int32_t j, int32_t *gain)
{
    LaunchCtx &lc = cx.lc;
    int64_t gs = ceil_div(L.S, kBlock);
    for (int it = 0; it < cx.prm.refine_iters; it++) {
        // a later iteration finds the modes and masks the first one set, unless
        // the multi-workgroup selection needs its lists reset
        if (it == 0 || !seg_path(cx, L, 0))
            launch(lc, "round", 0.0, k_round_refine, gs, kBlock, 0, L.S, j, (const int32_t *)sg.coarsest,
                   sg.mode, sg.gmask, sg.done, sg.st, sg.go);
        run_gains(cx, L, sg, gain, !seg_path(cx, L, 0), nullptr);
        select_and_flip(cx, L, sg, gain, nullptr);
    }
    if (cx.prm.refine_iters == 0)
        launch(lc, "round", 0.0, k_round_refine, gs, kBlock, 0, L.S, j, (const int32_t *)sg.coarsest,
               sg.mode, sg.gmask, sg.done, sg.st, sg.go);
    // balance step: the first round computes every gain; later rounds update
    // the gains from the hyperedges of the nodes the previous round moved
    // incremental gains pay off once a full recomputation is long against
    // the three short launches they take
    bool incr = (int64_t)L.P + L.N >= cx.sched.incremental_min_pins && !fuse_all(cx, L);
    Arena &ar = *cx.ar;
    MoveLog ml{L.noff, nullptr, nullptr, nullptr};
    uint32_t *bits = nullptr;
    int64_t nbits = ceil_div(L.E, 32);
    Fills zf;
    zf.add(sg.go, 8, 0).add(sg.bal_moved, (int64_t)2 * L.S, (int64_t)0);
    if (incr) {
        int64_t chunks = (int64_t)L.P / kLogChunk + L.N + 1;
        ml.cnode = ar.get<int32_t>(chunks);
        ml.cbeg = ar.get<int32_t>(chunks);
        ml.count = ar.get<int32_t>(4);
        bits = ar.get<uint32_t>(nbits);
        zf.add(bits, nbits, 0u).add(ml.count, 4, 0);
    }
    zf.run(lc);
    // small segments: the whole balance step in one workgroup each; when every
    // segment is small that is all, else the rounds below run the others
    if (cx.sched.fuse_max_pins > 0) {
        FuseArgs fa{L.off, L.pins, L.hw, L.noff, L.inc, L.nw, L.nbase, L.hbase, L.side, sg.max0, sg.max1,
                    (unsigned long long *)sg.w, sg.done, sg.stuck, sg.go + 2, cx.sched.fuse_max_pins,
                    nullptr, nullptr, nullptr, nullptr, 0};
        launch(lc, "seg_balance", 8.0 * L.P, k_seg_fused<false>, L.S, kFuseThreads, 0, L.S, fa);
        if (fuse_all(cx, L)) return fused_rounds_run(cx, sg.go + 2);
    }
    // LDS keys of the balance finish (32 KiB at most): room for a sorted
    // copy behind the candidates when the lists are short
    int32_t cap = sg.cand_stride <= 2048 ? 2 * sg.cand_stride : (sg.cand_stride <= 4096 ? sg.cand_stride : 0);
    BalFinish bf{sg.mode, L.nw, sg.need, sg.room, L.side, (unsigned long long *)sg.w, sg.done, sg.stuck, ml,
                 sg.go, sg.bal_moved, sg.st.rsel};
    // chunked selections: the level's chunk table (buffers of the whole
    // bisection, sized for its largest level)
    bool chunk = chunk_path(cx, L);
    ChunkArgs ca{};
    int64_t nct = 0;
    if (chunk) {
        nct = ceil_div(L.N, kChunkNodes) + L.S;
        if (!sg.chunk_cand || nct > sg.chunk_tab_n)
            throw Error(BP_ERR_DEVICE, "chunked selection buffers missing");
        int32_t *tseg = sg.chunk_tab, *tbeg = sg.chunk_tab + sg.chunk_tab_n, *tcnt = sg.chunk_tab + 2 * sg.chunk_tab_n;
        ca = ChunkArgs{tseg, tbeg, tcnt, L.N, sg.chunk_cand, sg.chunk_ccnt};
        launch(lc, "balance", 0.0, k_chunk_table, 1, 1024, 0, L.S, (const int32_t *)L.nbase, tseg, tbeg, tcnt);
    }
    int64_t lg = std::max<int64_t>(1, std::min<int64_t>(ceil_div((int64_t)L.P / kLogChunk + L.N, kBlock / 64), 1024));
    int64_t ugrid = std::max<int64_t>(1, std::min<int64_t>(ceil_div(nbits, kUpdWords), 2048));
    // profiling: the gain update counts its data-dependent bytes on the device
    unsigned long long *ubytes = nullptr;
    if (incr && lc.prof) {
        ubytes = ar.get<unsigned long long>(1);
        fill(lc, ubytes, 1, 0ull);
    }
    RoundBal rb{L.S, (const int32_t *)L.nbase, (const unsigned long long *)sg.w, (const int64_t *)sg.max0,
                (const int64_t *)sg.max1, sg.done, sg.mode, sg.gmask, sg.m, sg.need, sg.room, sg.ccount};
    int64_t rounds = chunked_rounds(cx, sg, (int64_t)L.N + L.S + 2, true, [&](int32_t ri, const int32_t *gc) {
        bool seg = seg_path(cx, L, 1);
        if (ri == 0 || !incr) {
            launch(lc, "round", 0.0, k_round_balance, gs, kBlock, 0, rb, sg.st, sg.go, ri);
            run_gains(cx, L, sg, gain, !seg && !chunk, gc);
        } else {
            // the round's test and the marking of the last round's moves: one launch
            launch(lc, "round", 0.0, k_round_balance_log, gs + lg, kBlock, 0, gs, rb, sg.st, sg.go, ri,
                   (const int32_t *)ml.count, (const int32_t *)ml.cnode, (const int32_t *)ml.cbeg,
                   (const int32_t *)L.noff, (const int32_t *)L.inc, bits, (const void *)L.cc, L.cc_pk,
                   (const uint8_t *)L.side, gain);
            launch(lc, "gain_update", 0.0, k_gain_update, ugrid, kBlock, 0, nbits, bits,
                   (const int32_t *)L.off, (const int32_t *)L.pins, (const int32_t *)L.hw,
                   (const uint8_t *)L.side, (void *)L.cc, L.cc_pk, gain, (const int32_t *)L.bigslot,
                   (const int32_t *)L.lnbig, (const int32_t *)L.ncount, gc, ml.count, ubytes);
            if (!seg && !chunk)
                launch(lc, "gain_stats", 10.0 * L.N, k_gain_stats, reduce_grid(L.N), kBlock, 0, L.N,
                   (const int32_t *)L.nseg, (const uint8_t *)sg.gmask, (const uint8_t *)L.side,
                   (const int32_t *)gain, (const uint8_t *)sg.mode, sg.st.tot, sg.st.gmax, sg.st.gmin,
                   ml.count, gc);
        }
        if (seg) {
            if (L.maxseg_nodes <= seg_select_max<1, kSegThreadsSmall>())
                launch(lc, "seg_select", 6.0 * L.N, k_seg_select<1, kSegThreadsSmall>, L.S, kSegThreadsSmall, 0,
                       L.S, sel_view(L, sg, gain), sg.st, id_bits(L), (const int32_t *)L.nw,
                       (unsigned long long *)sg.w, bf, gc, ChunkArgs{});
            else if (L.maxseg_nodes <= seg_select_max<1, kSegThreadsBal>())
                launch(lc, "seg_select", 6.0 * L.N, k_seg_select<1, kSegThreadsBal>, L.S, kSegThreadsBal, 0, L.S,
                       sel_view(L, sg, gain), sg.st, id_bits(L), (const int32_t *)L.nw,
                       (unsigned long long *)sg.w, bf, gc, ChunkArgs{});
            else
                launch(lc, "seg_select", 6.0 * L.N, k_seg_select<1, kSegThreads>, L.S, kSegThreads, 0, L.S,
                       sel_view(L, sg, gain), sg.st, id_bits(L), (const int32_t *)L.nw,
                       (unsigned long long *)sg.w, bf, gc, ChunkArgs{});
            return;
        }
        if (chunk) {
            launch(lc, "seg_select", 6.0 * L.N, k_seg_select<1, kChunkThreads, true>, nct, kChunkThreads, 0, L.S,
                   sel_view(L, sg, gain), sg.st, id_bits(L), (const int32_t *)L.nw, (unsigned long long *)sg.w, bf,
                   gc, ca);
            return;
        }
        run_select(cx, L, sg, gain, gc, sg.cand_stride);
        launch(lc, "balance", 10.0 * L.N, k_gather, ceil_div(L.N, kBlock), kBlock, 0, L.N,
               sel_view(L, sg, gain), sg.st, sg.ccount, sg.cand, sg.cand_stride, gc);
        launch(lc, "balance", 0.0, k_bal_finish, L.S, 1024, (size_t)cap * 8, L.S, (const int32_t *)sg.ccount,
               sg.cand, sg.cand_stride, cap, bf);
    });
    if (ubytes) {
        unsigned long long v = 0;
        BP_HIP(hipMemcpyAsync(&v, ubytes, sizeof(v), hipMemcpyDeviceToHost, lc.stream));
        lc.sync(false);
        Profiler::get().add_bytes("gain_update", (double)v);
    }
    return rounds;
}


// ---- the multilevel bisection of every segment of a level-0 CSR ---------------------

void bisect_all(Ctx &cx, Level &L0, Segs &sg, int32_t active0)
{
    Arena &ar = *cx.ar;
    LaunchCtx &lc = cx.lc;
    if (!L0.noff) build_incidence(cx, L0);
    std::vector<Level> lv;
    lv.push_back(L0);
    std::vector<int32_t> stops;  // segments whose coarsest level is l
    stops.push_back(L0.S - active0);
    uint8_t *sact = sg.active;
    uint8_t *sact_next = ar.get<uint8_t>(L0.S);
    int32_t active = active0;
    int32_t l = 0;
    auto trace_ms = [&]() -> double {
        // tracing only: wall time with the stream drained
        BP_HIP(hipStreamSynchronize(lc.stream));
        return std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now().time_since_epoch())
            .count();
    };
    while (active > 0) {
        Level c;
        double t0 = trace_on() ? trace_ms() : 0.0;
        coarsen_level(cx, lv[l], sg, sact, sact_next, l, c);
        if (trace_on())
            fprintf(stderr, "[bp] coarsen %d -> %d: N=%d P=%d  %.3f ms\n", l, l + 1, lv[l].N, lv[l].P,
                    trace_ms() - t0);
        lv.push_back(c);
        int32_t now = cx.info_h->active;
        stops.push_back(active - now);
        active = now;
        l++;
    }
    if (cx.first_levels < 0) cx.first_levels = l;
    cx.tree_depth.push_back(l);
    int32_t Lmax = l;

    // per level: a bound on the gain span, for the number of selection passes
    {
        unsigned long long *bd = ar.get<unsigned long long>(2 * (Lmax + 1));
        fill(lc, bd, 2 * (int64_t)(Lmax + 1), 0ull);
        for (int32_t j0 = 0; j0 <= Lmax; j0 += kBoundLevels) {
            LevelBoundArgs la{};
            int32_t nl = std::min<int32_t>(kBoundLevels, Lmax + 1 - j0);
            int64_t g = 1;
            double bytes = 0.0;
            for (int32_t q = 0; q < nl; q++) {
                const Level &x = lv[j0 + q];
                la.noff[q] = x.noff;
                la.hw[q] = x.hw;
                la.N[q] = x.N;
                la.E[q] = x.E;
                g = std::max<int64_t>(g, std::min<int64_t>(reduce_grid(std::max(x.N, x.E)), 128));
                bytes += 4.0 * (x.N + x.E);
            }
            launch3(lc, "level_bound", bytes, k_level_bound, dim3((unsigned)g, (unsigned)nl, 1), kBlock, 0, la,
                    bd + 2 * j0);
        }
        std::vector<unsigned long long> hb(2 * (Lmax + 1));
        BP_HIP(hipMemcpyAsync(hb.data(), bd, sizeof(unsigned long long) * hb.size(), hipMemcpyDeviceToHost,
                              lc.stream));
        lc.sync();
        for (int32_t j = 0; j <= Lmax; j++) {
            unsigned __int128 span = (unsigned __int128)2 * hb[2 * j] * hb[2 * j + 1];
            int bits = 0;
            while (bits < 32 && ((unsigned __int128)1 << bits) <= span) bits++;
            lv[j].span_bits = bits;
            lv[j].cc_pk = hb[2 * j + 1] < 32768;
        }
    }

    // balance candidate buffers sized for the largest segment
    int32_t maxn = 1;
    for (auto &x : lv) maxn = std::max(maxn, x.maxseg_nodes);
    int32_t mmax = (int32_t)ceil_sqrt_i64(maxn);
    sg.cand_stride = next_pow2(std::max(mmax, kBalGather));
    sg.cand = ar.get<uint64_t>((int64_t)sg.S * sg.cand_stride);
    // chunked balance selections, when some level takes them
    int64_t tab_n = 0;
    for (auto &x : lv)
        if (chunk_path(cx, x)) tab_n = std::max<int64_t>(tab_n, ceil_div(x.N, kChunkNodes) + x.S);
    alloc_chunk_bufs(ar, sg, tab_n);
    int32_t *gain = ar.get<int32_t>(lv[0].N);
    Fills()
        .add(sg.st.hist, (int64_t)2 * sg.S * kBins, 0u)
        .add(sg.st.ctl, 4, 0)
        .add(sg.st.tick, (int64_t)sg.S, 0)
        .add(sg.st.rsel, (int64_t)2 * sg.S, 0)
        .run(lc);

    for (int32_t j = Lmax; j >= 0; j--) {
        Level &L = lv[j];
        L.side = ar.get<uint8_t>(L.N);
        // (and the segments' side weights zeroed)
        launch(lc, "project", 6.0 * L.N, k_project, std::max<int64_t>(1, ceil_div(L.N, kBlock)), kBlock, 0, L.N, j,
               (const int32_t *)L.nseg, (const int32_t *)sg.coarsest,
               (const int32_t *)(j < Lmax ? L.parent : nullptr),
               (const uint8_t *)(j < Lmax ? lv[j + 1].side : nullptr), L.side, (unsigned long long *)sg.w,
               2 * sg.S);
        launch(lc, "side_weights", 5.0 * L.N, k_side_weights, reduce_grid(L.N), kBlock, 0, L.N,
               (const int32_t *)L.nseg, (const uint8_t *)L.side, (const int32_t *)L.nw,
               (unsigned long long *)sg.w);
        double t0 = trace_on() ? trace_ms() : 0.0;
        int64_t ir = stops[j] > 0 ? initial_rounds(cx, L, sg, j, gain) : 0;
        int64_t br = refine_level(cx, L, sg, j, gain);
        if (trace_on())
            fprintf(stderr, "[bp] level %d: S=%d N=%d E=%d P=%d initial_rounds=%lld balance_rounds=%lld  %.3f ms\n",
                    j, L.S, L.N, L.E, L.P, (long long)ir, (long long)br, trace_ms() - t0);
    }
    L0.side = lv[0].side;
}

// ---- nested k-way --------------------------------------------------------------------

struct TreeLevel {
    Level L;
    Segs sg;
    int32_t *ksub;  // [S]
    uint64_t *F;    // [S] per-bisection factor
    int32_t *orig;  // [N] input node id
    int32_t active0;
};

static void seg_setup(Ctx &cx, TreeLevel &t, const int32_t *k0_fixed = nullptr)
{
    LaunchCtx &lc = cx.lc;
    Level &L = t.L;
    fill(lc, t.sg.W, (int64_t)L.S, (int64_t)0);
    launch(lc, "seg_setup", 8.0 * L.N, k_seg_total, reduce_grid(L.N), kBlock, 0, L.N,
           (const int32_t *)L.nseg, (const int32_t *)L.nw, (unsigned long long *)t.sg.W);
    launch(lc, "seg_setup", 0.0, k_seg_setup, ceil_div(L.S, kBlock), kBlock, 0, L.S,
           (const int32_t *)t.ksub, k0_fixed, (const int64_t *)t.sg.W, (const uint64_t *)t.F,
           (const int32_t *)L.nbase,
           (const int32_t *)L.hbase, (const int32_t *)L.off, cx.prm.max_levels, cx.prm.min_coarse_nodes,
           t.sg.k0, t.sg.k1,
           t.sg.max0, t.sg.max1, t.sg.active, t.sg.coarsest, t.sg.stuck, cx.info_d);
}

// Children of every bisection of tree level t (cut-net splitting); final
// children write their part id.  Returns false when no child continues.
static bool extract(Ctx &cx, TreeLevel &t, int32_t *d_part, TreeLevel &nx)
{
    Arena &ar = *cx.ar;
    LaunchCtx &lc = cx.lc;
    Level &L = t.L;
    const int32_t N = L.N, E = L.E, S = L.S;
    check_lists(L);
    int32_t *n1 = ar.get<int32_t>(E);
    launch(lc, "extract_small", 4.0 * E + 5.0 * L.P, k_count_side1<SMALL>, sched_grid<SMALL>(E), kBlock, 0,
           E, (const int32_t *)nullptr, (const int32_t *)L.off, (const int32_t *)L.pins,
           (const uint8_t *)L.side, n1);
    launch(lc, "extract_wave", 0.0, k_count_side1<WAVE>, sched_grid<WAVE>(L.nmid), kBlock, 0, L.nmid,
           (const int32_t *)L.lmid, (const int32_t *)L.off, (const int32_t *)L.pins,
           (const uint8_t *)L.side, n1);
    launch(lc, "extract_block", 0.0, k_count_side1<BLOCK>, sched_grid<BLOCK>(L.nbig), kBlock, 0, L.nbig,
           (const int32_t *)L.lbig, (const int32_t *)L.off, (const int32_t *)L.pins,
           (const uint8_t *)L.side, n1);
    uint64_t *nscan = ar.get<uint64_t>(N), *hs0 = ar.get<uint64_t>(E), *hs1 = ar.get<uint64_t>(E);
    uint64_t *tots = ar.get<uint64_t>(3);
    {
        const uint8_t *side = L.side;
        scan<uint64_t>(
            lc, ar, "extract_scan", N,
            [=] __device__(int64_t v) -> uint64_t { return side[v] ? (1ull << 32) : 1ull; },
            [=] __device__(int64_t v, uint64_t ex, uint64_t) { nscan[v] = ex; }, tots);
        const int32_t *off = L.off, *hseg = L.hseg, *k0 = t.sg.k0, *k1 = t.sg.k1, *cn1 = n1;
        for (int sd = 0; sd < 2; sd++) {
            uint64_t *hs = sd ? hs1 : hs0;
            scan<uint64_t>(
                lc, ar, "extract_scan", E,
                [=] __device__(int64_t e) -> uint64_t {
                    int32_t s = hseg[e];
                    int32_t kk = sd ? k1[s] : k0[s];
                    int32_t d = off[e + 1] - off[e];
                    int32_t ns = sd ? cn1[e] : d - cn1[e];
                    return (kk >= 2 && ns >= 2) ? ((1ull << 32) | (uint32_t)ns) : 0ull;
                },
                [=] __device__(int64_t e, uint64_t ex, uint64_t) { hs[e] = ex; }, tots + 1 + sd);
        }
    }
    ChildTable ct;
    ct.idx = ar.get<int32_t>(2 * S);
    ct.nbase = ar.get<int32_t>(2 * S + 1);
    ct.hbase = ar.get<int32_t>(2 * S + 1);
    ct.pbase = ar.get<int32_t>(2 * S + 1);
    ct.k = ar.get<int32_t>(2 * S);
    ct.lo = ar.get<int32_t>(2 * S);
    ct.F = ar.get<uint64_t>(2 * S);
    cx.clear_info();
    launch(lc, "extract", 0.0, k_child_table, 1, 1, 0, S, N, E, (const int32_t *)L.nbase,
           (const int32_t *)L.hbase, (const int32_t *)t.sg.k0, (const int32_t *)t.sg.k1,
           (const int32_t *)t.sg.lo, (const uint64_t *)t.F, (const uint64_t *)nscan, (const uint64_t *)hs0,
           (const uint64_t *)hs1, (const uint64_t *)tots, (const uint64_t *)(tots + 1),
           (const uint64_t *)(tots + 2), ct, cx.info_d);
    LevelInfo inf = cx.readback();
    int32_t C = inf.active;
    Level &c = nx.L;
    c.S = C;
    c.N = inf.N;
    c.E = inf.E;
    c.P = inf.P;
    int32_t *map = ar.get<int32_t>(N);
    nx.orig = ar.get<int32_t>(c.N);
    c.nw = ar.get<int32_t>(c.N);
    c.nseg = ar.get<int32_t>(c.N);
    launch(lc, "extract", 24.0 * N, k_extract_nodes, ceil_div(N, kBlock), kBlock, 0, N,
           (const int32_t *)L.nseg, (const int32_t *)L.nbase, (const uint8_t *)L.side,
           (const uint64_t *)nscan, (const int32_t *)t.orig, (const int32_t *)L.nw,
           (const int32_t *)t.sg.k0, (const int32_t *)t.sg.lo, ct, map, nx.orig, c.nw, c.nseg,
           d_part);
    if (C == 0) return false;
    c.off = ar.get<int32_t>((int64_t)c.E + 1);
    c.pins = ar.get<int32_t>(c.P);
    c.hw = ar.get<int32_t>(c.E);
    c.hseg = ar.get<int32_t>(c.E);
    launch(lc, "extract_small", 12.0 * E + 9.0 * L.P, k_extract_hedges<SMALL>, sched_grid<SMALL>(E), kBlock, 0,
           E, (const int32_t *)nullptr, (const int32_t *)L.off, (const int32_t *)L.pins,
           (const int32_t *)L.hw, (const int32_t *)L.hseg, (const int32_t *)L.hbase,
           (const uint8_t *)L.side, (const int32_t *)n1, (const uint64_t *)hs0,
           (const uint64_t *)hs1, (const int32_t *)map, ct, c.off, c.pins, c.hw, c.hseg);
    launch(lc, "extract_wave", 0.0, k_extract_hedges<WAVE>, sched_grid<WAVE>(L.nmid), kBlock, 0, L.nmid,
           (const int32_t *)L.lmid, (const int32_t *)L.off, (const int32_t *)L.pins,
           (const int32_t *)L.hw, (const int32_t *)L.hseg, (const int32_t *)L.hbase,
           (const uint8_t *)L.side, (const int32_t *)n1, (const uint64_t *)hs0,
           (const uint64_t *)hs1, (const int32_t *)map, ct, c.off, c.pins, c.hw, c.hseg);
    launch(lc, "extract_block", 0.0, k_extract_hedges<BLOCK>, sched_grid<BLOCK>(L.nbig), kBlock, 0, L.nbig,
           (const int32_t *)L.lbig, (const int32_t *)L.off, (const int32_t *)L.pins,
           (const int32_t *)L.hw, (const int32_t *)L.hseg, (const int32_t *)L.hbase,
           (const uint8_t *)L.side, (const int32_t *)n1, (const uint64_t *)hs0,
           (const uint64_t *)hs1, (const int32_t *)map, ct, c.off, c.pins, c.hw, c.hseg);
    launch(lc, "extract", 4.0, k_set_i32, 1, 1, 0, c.off + c.E, c.P);
    c.nbase = ct.nbase;
    c.hbase = ct.hbase;
    nx.ksub = ct.k;
    nx.F = ct.F;
    nx.sg = alloc_segs(ar, C);
    BP_HIP(hipMemcpyAsync(nx.sg.lo, ct.lo, sizeof(int32_t) * C, hipMemcpyDeviceToDevice, lc.stream));
    return true;
}

static void prepare_tree_level(Ctx &cx, TreeLevel &t)
{
    int32_t *ctr = cx.ar->get<int32_t>(8);
    fill(cx.lc, ctr, 8, 0);
    classify(cx, t.L, ctr);
    cx.clear_info();
    seg_setup(cx, t);
    // fold the schedule counts into the same readback
    BP_HIP(hipMemcpyAsync(&cx.info_d->nmid, ctr + 1, 3 * sizeof(int32_t), hipMemcpyDeviceToDevice,
                          cx.lc.stream));
    LevelInfo inf = cx.readback();
    t.L.nmid = inf.nmid;
    t.L.nbig = inf.nbig;
    t.L.nhuge = inf.nhuge;
    t.L.maxseg_nodes = inf.maxseg_nodes;
    t.L.maxseg_pins = inf.maxseg_pins;
    t.L.maxseg_hedges = inf.maxseg_hedges;
    t.active0 = inf.active;
}

uint64_t eps_factor(int32_t k, double eps)
{
    int32_t levels = 0;
    while (((int64_t)1 << levels) < (int64_t)k) levels++;
    if (levels < 1) levels = 1;
    double f = std::pow(1.0 + eps, 1.0 / (double)levels);
    // A factor of 2^30 or more lets either side of any split hold all of the
    // weight (sums stay below 2^31 and a side's share is at least a third), so
    // every such factor gives the same bounds: cap it where the conversion and
    // the bound products stay in range.
    if (!(f < 1073741824.0)) return uint64_t(1) << 62;
    return (uint64_t)std::floor(std::ldexp(f, 32));
}

struct CutResult {
    int64_t cut = 0, maxw = 0, total_w = 0;
};

static CutResult compute_cut(Ctx &cx, Level &L, int32_t N_nodes, const int32_t *nw_in, int32_t k,
                             const int32_t *d_part)
{
    Arena &ar = *cx.ar;
    LaunchCtx &lc = cx.lc;
    check_lists(L);
    unsigned long long *acc = ar.get<unsigned long long>(4);
    int mask64 = k <= 64 ? 1 : 0;
    const int64_t gs = cut_grid<SMALL>(L.E), gw = cut_grid<WAVE>(L.nmid), gb = cut_grid<BLOCK>(L.nbig);
    unsigned long long *partial = ar.get<unsigned long long>(gs + gw + gb);
    launch(lc, "cut_small", 8.0 * L.E + 8.0 * L.P, k_cut<SMALL>, gs, kBlock, 0, L.E,
           (const int32_t *)nullptr, (const int32_t *)L.off, (const int32_t *)L.pins, (const int32_t *)L.hw,
           d_part, mask64, partial);
    launch(lc, "cut_wave", 0.0, k_cut<WAVE>, gw, kBlock, 0, L.nmid, (const int32_t *)L.lmid,
           (const int32_t *)L.off, (const int32_t *)L.pins, (const int32_t *)L.hw, d_part, mask64, partial + gs);
    launch(lc, "cut_block", 0.0, k_cut<BLOCK>, gb, kBlock, 0, L.nbig, (const int32_t *)L.lbig,
           (const int32_t *)L.off, (const int32_t *)L.pins, (const int32_t *)L.hw, d_part, mask64,
           partial + gs + gw);
    launch(lc, "cut", 0.0, k_sum_u64, 1, 1024, 0, (int32_t)(gs + gw + gb), (const unsigned long long *)partial,
           acc);
    unsigned long long *pw = ar.get<unsigned long long>(k);
    fill(lc, pw, k, 0ull);
    launch(lc, "part_weights", 8.0 * N_nodes, k_part_weights,
           std::max<int64_t>(1, reduce_grid(N_nodes)), kBlock, 0, N_nodes, k,
           d_part, nw_in, pw);
    launch(lc, "cut", 0.0, k_max_u64, 1, 1024, 0, k, (const unsigned long long *)pw, acc + 1);
    BP_HIP(hipMemcpyAsync(cx.info_h, acc, 2 * sizeof(uint64_t), hipMemcpyDeviceToHost, lc.stream));
    cx.lc.sync();
    CutResult r;
    r.cut = (int64_t)((uint64_t *)cx.info_h)[0];
    r.maxw = (int64_t)((uint64_t *)cx.info_h)[1];
    return r;
}

// Checks the CSR and weight sums on the device; returns the node weight total.
static int64_t validate_device(Ctx &cx, const Input &in)
{
    ValidateOut *vo = cx.ar->get<ValidateOut>(1);
    fill(cx.lc, (int32_t *)vo, (int64_t)(sizeof(ValidateOut) / 4), 0);
    int64_t work = std::max<int64_t>(std::max<int64_t>(in.N, in.E), 1);
    launch(cx.lc, "validate", 0.0, k_validate, std::min<int64_t>(ceil_div(work, kBlock), 2048), kBlock, 0,
           in.N, in.E, in.off, in.pins, in.nw, in.hw, vo);
    BP_HIP(hipMemcpyAsync(cx.info_h, vo, sizeof(ValidateOut), hipMemcpyDeviceToHost, cx.lc.stream));
    cx.lc.sync();
    ValidateOut v = *(ValidateOut *)cx.info_h;
    if (v.bad_offsets || v.bad_pins) throw Error(BP_ERR_INVALID_CSR, "invalid CSR (offsets or pin range)");
    if (v.bad_weights) throw Error(BP_ERR_WEIGHT_OVERFLOW, "negative weight");
    int64_t sn = in.nw ? (int64_t)v.sum_nw : in.N, sh = in.hw ? (int64_t)v.sum_hw : in.E;
    if (sn >= (int64_t(1) << 31) || sh >= (int64_t(1) << 31))
        throw Error(BP_ERR_WEIGHT_OVERFLOW, "weight sum >= 2^31");
    return sn;
}

// The balance limit of the problem statement, max(ceil(W/k), floor((1+eps) W / k)),
// with (1+eps) in 32.32 fixed point.
int64_t part_limit(int64_t W, int32_t k, double eps)
{
    // 1 + eps at or above 2^31 exceeds every k, so the limit is at least W either way.
    double f = 1.0 + eps;
    uint64_t F0 = f < 2147483648.0 ? (uint64_t)std::floor(std::ldexp(f, 32)) : uint64_t(1) << 63;
    unsigned __int128 a = (unsigned __int128)(uint64_t)W * F0;
    int64_t lim_f = (int64_t)(a / ((unsigned __int128)(uint64_t)k << 32));
    int64_t lim_c = (W + k - 1) / k;
    return std::max(lim_f, lim_c);
}

// Report fields shared by every form: coarsening depth per tree level,
// imbalance, graph replays.
static void report_extras(const Ctx &cx, int64_t maxw, int64_t W, int32_t k, bp_report &r)
{
    for (int t = 0; t < 64; t++) r.levels[t] = t < (int)cx.tree_depth.size() ? cx.tree_depth[t] : 0;
    r.imbalance = W > 0 ? (double)maxw * k / (double)W - 1.0 : 0.0;
    r.graph_replays = cx.graph_replays;
    r.reserved = 0;
}

bp_status partition_device(Ctx &cx, const Input &in, int32_t k, double eps, int32_t *d_part,
                           int64_t *cut_out, bp_report *rep)
{
    LaunchCtx &lc = cx.lc;
    int64_t W = validate_device(cx, in);
    Level root = normalize(cx, in);
    CutResult cr;
    int32_t tree_levels = 0;
    if (k == 1 || in.N == 0) {
        fill(lc, d_part, in.N, 0);
    } else {
        uint64_t F = eps_factor(k, eps);
        TreeLevel t;
        t.L = root;
        t.sg = alloc_segs(*cx.ar, 1);
        t.ksub = cx.ar->get<int32_t>(1);
        launch(lc, "seg_setup", 4.0, k_set_i32, 1, 1, 0, t.ksub, k);
        t.F = cx.ar->get<uint64_t>(1);
        fill(lc, t.F, 1, F);
        fill(lc, t.sg.lo, 1, 0);
        t.orig = cx.ar->get<int32_t>(in.N);
        launch(lc, "seg_setup", 4.0 * in.N, k_iota, std::min<int64_t>(ceil_div(in.N, kBlock), 4096), kBlock,
               0, (int64_t)in.N, t.orig);
        prepare_tree_level(cx, t);
        root = t.L;  // keep the schedule lists for the final cut
        for (;;) {
            tree_levels++;
            cx.bisections += t.L.S;
            bisect_all(cx, t.L, t.sg, t.active0);
            TreeLevel nx;
            if (!extract(cx, t, d_part, nx)) break;
            prepare_tree_level(cx, nx);
            t = nx;
        }
    }
    if (k > 1 && in.N > 0) cr = compute_cut(cx, root, in.N, in.nw, k, d_part);
    else {
        cr.cut = 0;
        cr.maxw = W;
    }
    if (cut_out) *cut_out = cr.cut;
    int64_t limit = part_limit(W, k, eps);
    bool balanced = cr.maxw <= limit;
    if (rep) {
        rep->cut = cr.cut;
        rep->max_part_weight = cr.maxw;
        rep->part_weight_limit = limit;
        rep->balanced = balanced ? 1 : 0;
        rep->tree_levels = tree_levels;
        rep->bisections = cx.bisections;
        rep->coarsen_levels = cx.first_levels < 0 ? 0 : cx.first_levels;
        rep->pins_coarsened = cx.pins_coarsened;
        rep->pins_refined = cx.pins_refined;
        rep->host_syncs = lc.syncs;
        rep->kernel_launches = lc.launches;
        rep->device_bytes = (int64_t)cx.ar->used();
        report_extras(cx, cr.maxw, W, k, *rep);
    }
    return balanced ? BP_OK : BP_WARN_IMBALANCED;
}

// ---- batches of independent graphs ----------------------------------------------------
//
// Graph g of the batch is segment g of the first tree level (graphs that need
// no bisection - k = 1 or no node - are placed after the others and only
// copied).  Every later step is the segmented k-way loop above, so each graph
// gets the partition it gets alone.

template <typename T> static T *upload_vec(Ctx &cx, const std::vector<T> &v)
{
    T *p = cx.ar->get<T>((int64_t)std::max<size_t>(v.size(), 1));
    if (!v.empty())
        BP_HIP(hipMemcpyAsync(p, v.data(), sizeof(T) * v.size(), hipMemcpyHostToDevice, cx.lc.stream));
    return p;
}

std::vector<BatchOut> partition_batch(Ctx &cx, const std::vector<BatchItem> &it,
                                      const std::vector<int32_t *> &d_out, int32_t *tree_levels)
{
    Arena &ar = *cx.ar;
    LaunchCtx &lc = cx.lc;
    const int32_t n = (int32_t)it.size();
    std::vector<BatchOut> res(n);
    if (tree_levels) *tree_levels = 0;
    if (n == 0) return res;
    if (n > 65535) throw Error(BP_ERR_INVALID_ARG, "batch of more than 65535 graphs");
    std::vector<int32_t> order;
    for (int32_t g = 0; g < n; g++)
        if (it[g].k >= 2 && it[g].N > 0) order.push_back(g);
    const int32_t S = (int32_t)order.size();
    for (int32_t g = 0; g < n; g++)
        if (!(it[g].k >= 2 && it[g].N > 0)) order.push_back(g);

    // sizes, then the concatenation (with the same checks as a single input)
    std::vector<GraphDesc> d(n);
    for (int32_t i = 0; i < n; i++) {
        const BatchItem &x = it[order[i]];
        d[i] = GraphDesc{x.off, x.pins, x.nw, x.hw, x.N, x.E, 0, 0, 0};
    }
    GraphDesc *dd = upload_vec(cx, d);
    GraphCheck *chk = ar.get<GraphCheck>(n);
    launch(lc, "batch", 0.0, k_batch_sizes, ceil_div(n, kBlock), kBlock, 0, n, (const GraphDesc *)dd, chk);
    std::vector<GraphCheck> ch(n);
    BP_HIP(hipMemcpyAsync(ch.data(), chk, sizeof(GraphCheck) * n, hipMemcpyDeviceToHost, lc.stream));
    lc.sync();
    int64_t nb = 0, eb = 0, pb = 0, work = 1;
    for (int32_t i = 0; i < n; i++) {
        if (ch[i].bad_offsets)
            throw Error(BP_ERR_INVALID_CSR, "graph " + std::to_string(order[i]) + ": invalid CSR offsets");
        d[i].nbase = nb;
        d[i].ebase = eb;
        d[i].pbase = pb;
        nb += d[i].N;
        eb += d[i].E;
        pb += ch[i].P;
        work = std::max({work, (int64_t)d[i].N, (int64_t)d[i].E, ch[i].P});
    }
    if (nb >= INT32_MAX || eb >= INT32_MAX || pb >= INT32_MAX)
        throw Error(BP_ERR_INVALID_ARG, "batch too large: nodes, hyperedges and pins must each total < 2^31");
    BP_HIP(hipMemcpyAsync(dd, d.data(), sizeof(GraphDesc) * n, hipMemcpyHostToDevice, lc.stream));
    int32_t *off = ar.get<int32_t>(eb + 1), *pins = ar.get<int32_t>(std::max<int64_t>(pb, 1));
    int32_t *nw = ar.get<int32_t>(std::max<int64_t>(nb, 1)), *hw = ar.get<int32_t>(std::max<int64_t>(eb, 1));
    int32_t *nseg = ar.get<int32_t>(std::max<int64_t>(nb, 1)), *eseg = ar.get<int32_t>(std::max<int64_t>(eb, 1));
    unsigned gx = (unsigned)std::min<int64_t>(ceil_div(work, kBlock), 64);
    launch3(lc, "batch", 4.0 * (2 * pb + 4 * eb + 3 * nb), k_batch_gather, dim3(gx, (unsigned)n), kBlock, 0,
            (const GraphDesc *)dd, chk, off, pins, nw, hw, nseg, eseg);
    launch(lc, "batch", 4.0, k_set_i32, 1, 1, 0, off + eb, (int32_t)pb);
    BP_HIP(hipMemcpyAsync(ch.data(), chk, sizeof(GraphCheck) * n, hipMemcpyDeviceToHost, lc.stream));
    lc.sync();
    std::vector<int64_t> W(n);
    for (int32_t i = 0; i < n; i++) {
        std::string gname = "graph " + std::to_string(order[i]) + ": ";
        if (ch[i].bad_offsets) throw Error(BP_ERR_INVALID_CSR, gname + "hedge offsets not monotone");
        if (ch[i].bad_pins) throw Error(BP_ERR_INVALID_CSR, gname + "pin out of range");
        if (ch[i].bad_weights) throw Error(BP_ERR_WEIGHT_OVERFLOW, gname + "negative weight");
        if (ch[i].sum_nw >= (1ull << 31) || ch[i].sum_hw >= (1ull << 31))
            throw Error(BP_ERR_WEIGHT_OVERFLOW, gname + "weight sum >= 2^31");
        W[i] = (int64_t)ch[i].sum_nw;
    }
    const int64_t Neng = S < n ? d[S].nbase : nb, Eeng = S < n ? d[S].ebase : eb;
    int32_t *part = ar.get<int32_t>(std::max<int64_t>(nb, 1));
    if (nb > Neng) fill(lc, part + Neng, nb - Neng, 0);
    for (int32_t i = S; i < n; i++) {
        const BatchItem &x = it[order[i]];
        BatchOut &r = res[order[i]];
        r.cut = 0;
        r.maxw = W[i];
        r.limit = part_limit(W[i], x.k, x.eps);
        r.W = W[i];
        r.k = x.k;
        r.balanced = r.maxw <= r.limit;
    }

    if (S > 0) {
        // level 0: hyperedges of >= 2 pins, per segment, in input order
        Level L;
        L.S = S;
        L.N = (int32_t)Neng;
        uint64_t *kept = ar.get<uint64_t>(std::max<int64_t>(Eeng, 1));
        int32_t *dst = ar.get<int32_t>(std::max<int64_t>(Eeng, 1));
        L.off = ar.get<int32_t>(Eeng + 1);
        L.hw = ar.get<int32_t>(std::max<int64_t>(Eeng, 1));
        L.hseg = ar.get<int32_t>(std::max<int64_t>(Eeng, 1));
        uint64_t *tot = ar.get<uint64_t>(1);
        {
            int32_t *loff = L.off, *lhw = L.hw, *lhseg = L.hseg;
            const int32_t *coff = off, *chw = hw, *ceseg = eseg;
            scan<uint64_t>(
                lc, ar, "normalize_scan", Eeng,
                [=] __device__(int64_t e) -> uint64_t {
                    int32_t dg = coff[e + 1] - coff[e];
                    return dg >= 2 ? ((1ull << 32) | (uint32_t)dg) : 0ull;
                },
                [=] __device__(int64_t e, uint64_t ex, uint64_t val) {
                    kept[e] = ex;
                    if (!val) return;
                    int32_t id = (int32_t)(ex >> 32);
                    loff[id] = (int32_t)ex;
                    lhw[id] = chw[e];
                    lhseg[id] = ceseg[e];
                    dst[e] = (int32_t)ex;
                },
                tot);
        }
        BP_HIP(hipMemcpyAsync(cx.info_h, tot, sizeof(uint64_t), hipMemcpyDeviceToHost, lc.stream));
        lc.sync();
        uint64_t tv = *(uint64_t *)cx.info_h;
        L.E = (int32_t)(tv >> 32);
        L.P = (int32_t)(tv & 0xffffffffu);
        L.pins = ar.get<int32_t>(std::max<int32_t>(L.P, 1));
        launch(lc, "normalize_copy", 8.0 * L.P, k_norm_copy, ceil_div(Eeng, kBlock), kBlock, 0, (int32_t)Eeng,
               (const int32_t *)off, (const int32_t *)pins, (const int32_t *)dst, L.pins);
        launch(lc, "normalize", 4.0, k_set_i32, 1, 1, 0, L.off + L.E, L.P);
        L.nw = nw;
        L.nseg = nseg;
        std::vector<int32_t> nbh(S + 1);
        std::vector<int64_t> ebh(S + 1);
        for (int32_t i = 0; i <= S; i++) {
            nbh[i] = (int32_t)(i < n ? d[i].nbase : nb);
            ebh[i] = i < n ? d[i].ebase : eb;
        }
        L.nbase = upload_vec(cx, nbh);
        int64_t *ebd = upload_vec(cx, ebh);
        L.hbase = ar.get<int32_t>(S + 1);
        int32_t *pbk = ar.get<int32_t>(S + 1);
        launch(lc, "normalize", 0.0, k_batch_hbase, ceil_div(S + 1, kBlock), kBlock, 0, S,
               (const int64_t *)ebd, Eeng, (const uint64_t *)kept, (const uint64_t *)tot, L.hbase, pbk);

        // first tree level: one segment per graph, its own k and factor
        std::vector<int32_t> kh(S), kb(S + 1, 0);
        std::vector<uint64_t> fh(S);
        int32_t kmax = 1;
        for (int32_t i = 0; i < S; i++) {
            const BatchItem &x = it[order[i]];
            kh[i] = x.k;
            fh[i] = eps_factor(x.k, x.eps);
            kb[i + 1] = kb[i] + x.k;
            kmax = std::max(kmax, x.k);
        }
        TreeLevel t;
        t.L = L;
        t.sg = alloc_segs(ar, S);
        t.ksub = upload_vec(cx, kh);
        t.F = upload_vec(cx, fh);
        fill(lc, t.sg.lo, S, 0);
        t.orig = ar.get<int32_t>(Neng);
        launch(lc, "seg_setup", 4.0 * Neng, k_iota, std::min<int64_t>(ceil_div(Neng, kBlock), 4096), kBlock, 0,
               Neng, t.orig);
        prepare_tree_level(cx, t);
        Level root = t.L;
        int32_t tl = 0;
        for (;;) {
            tl++;
            cx.bisections += t.L.S;
            bisect_all(cx, t.L, t.sg, t.active0);
            TreeLevel nx;
            if (!extract(cx, t, part, nx)) break;
            prepare_tree_level(cx, nx);
            t = nx;
        }
        if (tree_levels) *tree_levels = tl;

        // per-graph cut (connectivity - 1) and heaviest part
        int32_t *kbd = upload_vec(cx, kb);
        unsigned long long *acc = ar.get<unsigned long long>(2 * S);
        unsigned long long *pw = ar.get<unsigned long long>(kb[S]);
        fill(lc, acc, 2 * S, 0ull);
        fill(lc, pw, kb[S], 0ull);
        check_lists(root);
        launch(lc, "cut_small", 8.0 * root.E + 8.0 * root.P, k_cut_seg<SMALL>, cut_grid<SMALL>(root.E), kBlock,
               0, root.E, (const int32_t *)nullptr, (const int32_t *)root.off, (const int32_t *)root.pins,
               (const int32_t *)root.hw, (const int32_t *)root.hseg, (const int32_t *)part, kmax, acc);
        launch(lc, "cut_wave", 0.0, k_cut_seg<WAVE>, cut_grid<WAVE>(root.nmid), kBlock, 0, root.nmid,
               (const int32_t *)root.lmid, (const int32_t *)root.off, (const int32_t *)root.pins,
               (const int32_t *)root.hw, (const int32_t *)root.hseg, (const int32_t *)part, kmax, acc);
        launch(lc, "cut_block", 0.0, k_cut_seg<BLOCK>, std::min<int64_t>(root.nbig, kCutBlocks), kBlock, 0,
               root.nbig,
               (const int32_t *)root.lbig, (const int32_t *)root.off, (const int32_t *)root.pins,
               (const int32_t *)root.hw, (const int32_t *)root.hseg, (const int32_t *)part, kmax, acc);
        launch(lc, "part_weights", 8.0 * Neng, k_part_weights_seg, ceil_div(Neng, kBlock), kBlock, 0,
               (int32_t)Neng, (const int32_t *)nseg, (const int32_t *)kbd, (const int32_t *)part,
               (const int32_t *)nw, pw);
        launch(lc, "cut", 0.0, k_seg_max, ceil_div(S, kBlock), kBlock, 0, S, (const int32_t *)kbd,
               (const unsigned long long *)pw, acc + S);
        std::vector<unsigned long long> accv(2 * S);
        BP_HIP(hipMemcpyAsync(accv.data(), acc, sizeof(unsigned long long) * 2 * S, hipMemcpyDeviceToHost,
                              lc.stream));
        lc.sync();
        for (int32_t i = 0; i < S; i++) {
            const BatchItem &x = it[order[i]];
            BatchOut &r = res[order[i]];
            r.cut = (int64_t)accv[i];
            r.maxw = (int64_t)accv[S + i];
            r.limit = part_limit(W[i], x.k, x.eps);
            r.W = W[i];
            r.k = x.k;
            r.balanced = r.maxw <= r.limit;
        }
    }

    // part ids into every graph's own buffer
    std::vector<int32_t *> outs(n);
    int64_t maxn = 1;
    for (int32_t i = 0; i < n; i++) {
        outs[i] = d_out[order[i]];
        maxn = std::max<int64_t>(maxn, d[i].N);
    }
    int32_t **outd = upload_vec(cx, outs);
    launch3(lc, "batch", 8.0 * nb, k_batch_scatter, dim3((unsigned)std::min<int64_t>(ceil_div(maxn, kBlock), 64), (unsigned)n),
            kBlock, 0, (const GraphDesc *)dd, (int32_t *const *)outd, (const int32_t *)part);
    return res;
}

// ---- context pool -------------------------------------------------------------------
// Arenas of finished calls are kept per device for the next call, so steady
// calls allocate nothing.  A call that used much less than its arena holds
// trims it (a large input followed by small ones does not pin gigabytes), and
// bp_release_memory frees every idle arena of the current device.

constexpr int kMaxDevices = 64;
constexpr size_t kTrimFloor = size_t(1) << 30;

struct Pool {
    std::mutex mu;
    std::vector<Arena *> arenas[kMaxDevices];
    std::vector<void *> pinned;
    static Pool &get()
    {
        static Pool p;
        return p;
    }
};

static int current_device()
{
    int dev = 0;
    BP_HIP(hipGetDevice(&dev));
    if (dev < 0 || dev >= kMaxDevices) throw Error(BP_ERR_DEVICE, "device id beyond the supported range");
    return dev;
}

struct CtxGuard {
    Ctx cx;
    int dev = 0;
    bool pooled = true;
    CtxGuard(hipStream_t stream, const bp_params *p)
    {
        dev = current_device();
        Pool &pl = Pool::get();
        {
            std::lock_guard<std::mutex> g(pl.mu);
            if (!pl.arenas[dev].empty()) {
                cx.ar = pl.arenas[dev].back();
                pl.arenas[dev].pop_back();
            }
            if (!pl.pinned.empty()) {
                cx.info_h = (LevelInfo *)pl.pinned.back();
                pl.pinned.pop_back();
            }
        }
        if (!cx.ar) cx.ar = new Arena();
        if (!cx.info_h) BP_HIP(hipHostMalloc((void **)&cx.info_h, 4096, hipHostMallocDefault));
        init(stream, p, Profiler::get().on);
    }
    // A context over a caller-owned arena and host readback buffer, outside
    // the pool (no allocation at all, no profiling events).
    CtxGuard(hipStream_t stream, const bp_params *p, Arena *fixed, LevelInfo *info) : pooled(false)
    {
        cx.ar = fixed;
        cx.info_h = info;
        init(stream, p, false);
    }
    void init(hipStream_t stream, const bp_params *p, bool prof)
    {
        cx.lc.stream = stream;
        cx.lc.prof = prof;
        cx.info_d = cx.ar->get<LevelInfo>(1);
        bp_default_params(&cx.prm);
        if (p) cx.prm = *p;
    }
    ~CtxGuard()
    {
        try {
            cx.lc.flush();
        } catch (...) {
        }
        // everything queued must finish before the arena is reused
        (void)hipStreamSynchronize(cx.lc.stream);
        size_t used = cx.ar->used();
        cx.ar->reset();
        if (!pooled) return;
        if (cx.ar->reserved() > std::max(4 * used, kTrimFloor)) cx.ar->trim(std::max(2 * used, kTrimFloor));
        Pool &pl = Pool::get();
        std::lock_guard<std::mutex> g(pl.mu);
        pl.arenas[dev].push_back(cx.ar);
        pl.pinned.push_back(cx.info_h);
    }
};

// Frees the device memory of every idle arena of the current device.
static void release_idle_arenas()
{
    int dev = current_device();
    Pool &pl = Pool::get();
    std::vector<Arena *> idle;
    {
        std::lock_guard<std::mutex> g(pl.mu);
        idle.swap(pl.arenas[dev]);
    }
    for (Arena *a : idle) delete a;
}

}  // namespace bp

// ==== C ABI ==============================================================================

using namespace bp;

static thread_local std::string g_last_error;

static bp_status fail(bp_status s, const std::string &msg)
{
    g_last_error = msg;
    return s;
}

#define BP_GUARD_BEGIN try {
#define BP_GUARD_END                                                   \
    }                                                                  \
    catch (const bp::Error &e) { return fail(e.status, e.what()); }     \
    catch (const std::exception &e) { return fail(BP_ERR_DEVICE, e.what()); }

static bp_status check_params(const bp_params *p)
{
    if (!p) return BP_OK;
    if (p->policy < BP_LDH || p->policy > BP_RAND || p->max_levels < 0 || p->max_levels > 1000 ||
        p->refine_iters < 0 || p->min_coarse_nodes < 0)
        return fail(BP_ERR_INVALID_ARG, "invalid bp_params");
    return BP_OK;
}

// Host-side validation of a host CSR (including repeated pins).
static bp_status validate_host(const bp_hypergraph *hg)
{
    if (!hg) return fail(BP_ERR_INVALID_ARG, "hypergraph is NULL");
    int32_t N = hg->num_nodes, E = hg->num_hedges;
    if (N < 0 || E < 0) return fail(BP_ERR_INVALID_ARG, "negative size");
    if (!hg->hedge_offsets) return fail(BP_ERR_INVALID_ARG, "hedge_offsets is NULL");
    const int32_t *off = hg->hedge_offsets;
    if (off[0] != 0) return fail(BP_ERR_INVALID_CSR, "hedge_offsets[0] != 0");
    for (int32_t e = 0; e < E; e++)
        if (off[e + 1] < off[e]) return fail(BP_ERR_INVALID_CSR, "hedge_offsets not monotone");
    int64_t P = off[E];
    if (P > 0 && !hg->pins) return fail(BP_ERR_INVALID_ARG, "pins is NULL");
    std::vector<int32_t> stamp(N > 0 ? N : 1, -1);
    for (int32_t e = 0; e < E; e++)
        for (int32_t i = off[e]; i < off[e + 1]; i++) {
            int32_t v = hg->pins[i];
            if (v < 0 || v >= N) return fail(BP_ERR_INVALID_CSR, "pin out of range");
            if (stamp[v] == e) return fail(BP_ERR_INVALID_CSR, "node repeated in a hyperedge");
            stamp[v] = e;
        }
    int64_t s = 0;
    if (hg->node_weights)
        for (int32_t v = 0; v < N; v++) {
            if (hg->node_weights[v] < 0) return fail(BP_ERR_WEIGHT_OVERFLOW, "negative node weight");
            s += hg->node_weights[v];
        }
    else
        s = N;
    if (s >= (int64_t(1) << 31)) return fail(BP_ERR_WEIGHT_OVERFLOW, "node weight sum >= 2^31");
    s = 0;
    if (hg->hedge_weights)
        for (int32_t e = 0; e < E; e++) {
            if (hg->hedge_weights[e] < 0) return fail(BP_ERR_WEIGHT_OVERFLOW, "negative hedge weight");
            s += hg->hedge_weights[e];
        }
    else
        s = E;
    if (s >= (int64_t(1) << 31)) return fail(BP_ERR_WEIGHT_OVERFLOW, "hedge weight sum >= 2^31");
    return BP_OK;
}

// Copies a host CSR into arena memory; returns the device view.
static Input upload(Ctx &cx, const bp_hypergraph *hg)
{
    Input in;
    in.N = hg->num_nodes;
    in.E = hg->num_hedges;
    int64_t P = hg->hedge_offsets[in.E];
    int32_t *off = cx.ar->get<int32_t>((int64_t)in.E + 1);
    int32_t *pins = cx.ar->get<int32_t>(P);
    BP_HIP(hipMemcpyAsync(off, hg->hedge_offsets, sizeof(int32_t) * ((size_t)in.E + 1),
                          hipMemcpyHostToDevice, cx.lc.stream));
    if (P > 0)
        BP_HIP(hipMemcpyAsync(pins, hg->pins, sizeof(int32_t) * (size_t)P, hipMemcpyHostToDevice,
                              cx.lc.stream));
    in.off = off;
    in.pins = pins;
    if (hg->node_weights) {
        int32_t *nw = cx.ar->get<int32_t>(in.N);
        BP_HIP(hipMemcpyAsync(nw, hg->node_weights, sizeof(int32_t) * (size_t)in.N,
                              hipMemcpyHostToDevice, cx.lc.stream));
        in.nw = nw;
    }
    if (hg->hedge_weights) {
        int32_t *hw = cx.ar->get<int32_t>(in.E);
        BP_HIP(hipMemcpyAsync(hw, hg->hedge_weights, sizeof(int32_t) * (size_t)in.E,
                              hipMemcpyHostToDevice, cx.lc.stream));
        in.hw = hw;
    }
    return in;
}

static Input device_input(const bp_hypergraph *hg)
{
    Input in;
    in.N = hg->num_nodes;
    in.E = hg->num_hedges;
    in.off = hg->hedge_offsets;
    in.pins = hg->pins;
    in.nw = hg->node_weights;
    in.hw = hg->hedge_weights;
    return in;
}

static bp_status check_device_hg(const bp_hypergraph *hg)
{
    if (!hg) return fail(BP_ERR_INVALID_ARG, "hypergraph is NULL");
    if (hg->num_nodes < 0 || hg->num_hedges < 0) return fail(BP_ERR_INVALID_ARG, "negative size");
    if (!hg->hedge_offsets) return fail(BP_ERR_INVALID_ARG, "hedge_offsets is NULL");
    if (!hg->pins && hg->num_hedges > 0) return fail(BP_ERR_INVALID_ARG, "pins is NULL");
    return BP_OK;
}

#include "server.hpp"

extern "C" {

void bp_default_params(bp_params *p)
{
    if (!p) return;
    p->policy = BP_LDH;
    p->max_levels = 25;
    p->refine_iters = 2;
    p->min_coarse_nodes = 100;
}

const char *bp_status_string(bp_status s)
{
    switch (s) {
    case BP_OK: return "BP_OK";
    case BP_WARN_IMBALANCED: return "BP_WARN_IMBALANCED";
    case BP_ERR_INVALID_ARG: return "BP_ERR_INVALID_ARG";
    case BP_ERR_INVALID_CSR: return "BP_ERR_INVALID_CSR";
    case BP_ERR_WEIGHT_OVERFLOW: return "BP_ERR_WEIGHT_OVERFLOW";
    case BP_ERR_OUT_OF_MEMORY: return "BP_ERR_OUT_OF_MEMORY";
    case BP_ERR_DEVICE: return "BP_ERR_DEVICE";
    case BP_ERR_REJECTED: return "BP_ERR_REJECTED";
    case BP_ERR_SHUTDOWN: return "BP_ERR_SHUTDOWN";
    case BP_ERR_NOT_FOUND: return "BP_ERR_NOT_FOUND";
    default: return "BP_UNKNOWN_STATUS";
    }
}

const char *bp_last_error(void) { return g_last_error.c_str(); }

bp_status bp_partition(const bp_hypergraph *hg, int32_t k, double eps, const bp_params *params,
                       int32_t *part_out, int64_t *cut_out, bp_report *report)
{
    bp_status st = validate_host(hg);
    if (st != BP_OK) return st;
    if ((st = check_params(params)) != BP_OK) return st;
    if (k < 1 || !(eps >= 0.0) || std::isinf(eps)) return fail(BP_ERR_INVALID_ARG, "k < 1 or bad eps");
    if (!part_out && hg->num_nodes > 0) return fail(BP_ERR_INVALID_ARG, "part_out is NULL");
    BP_GUARD_BEGIN
    CtxGuard g(nullptr, params);
    Input in = upload(g.cx, hg);
    int32_t *d_part = g.cx.ar->get<int32_t>(hg->num_nodes);
    bp_status r = partition_device(g.cx, in, k, eps, d_part, cut_out, report);
    if (hg->num_nodes > 0)
        BP_HIP(hipMemcpyAsync(part_out, d_part, sizeof(int32_t) * (size_t)hg->num_nodes,
                              hipMemcpyDeviceToHost, g.cx.lc.stream));
    BP_HIP(hipStreamSynchronize(g.cx.lc.stream));
    return r;
    BP_GUARD_END
}

bp_status bp_partition_device(const bp_hypergraph *hg, int32_t k, double eps,
                              const bp_params *params, int32_t *d_part_out, int64_t *cut_out,
                              bp_report *report, void *stream)
{
    bp_status st = check_device_hg(hg);
    if (st != BP_OK) return st;
    if ((st = check_params(params)) != BP_OK) return st;
    if (k < 1 || !(eps >= 0.0) || std::isinf(eps)) return fail(BP_ERR_INVALID_ARG, "k < 1 or bad eps");
    if (!d_part_out && hg->num_nodes > 0) return fail(BP_ERR_INVALID_ARG, "d_part_out is NULL");
    BP_GUARD_BEGIN
    CtxGuard g((hipStream_t)stream, params);
    return partition_device(g.cx, device_input(hg), k, eps, d_part_out, cut_out, report);
    BP_GUARD_END
}

// The fixed device workspace of bp_partition_device_noalloc: a static device
// array, one copy per GPU the library runs on, held until the process ends.
// Host code reaches a device's copy only through the address that
// hipGetSymbolAddress returns for it (kept per device below).
constexpr size_t kScratchBytes = size_t(256) << 20;
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

struct ScratchDev {
    std::mutex mu;  // calls on one device share its workspace, so they run one at a time
    bool ready = false;
    void *ptr = nullptr;  // device address of this device's copy of `scratch`
    Arena ar;             // bump allocation inside that copy
    alignas(64) unsigned char info[4096];  // host readback buffer
};
static ScratchDev g_scratch[kMaxDevices];

// Upper bound of the workspace a partition takes: the bump allocations of one
// call, by the largest terms measured per pin, node and hyperedge and tree
// level, plus the fixed tables.
static int64_t workspace_bound(int64_t N, int64_t E, int64_t P, int32_t k)
{
    return footprint_bytes(N, E, P, k);
}

bp_status bp_partition_device_noalloc(const bp_hypergraph *hg, int32_t k, double eps,
                                      const bp_params *params, int32_t *d_part_out, int64_t *cut_out,
                                      bp_report *report, void *stream)
{
    bp_status st = check_device_hg(hg);
    if (st != BP_OK) return st;
    if ((st = check_params(params)) != BP_OK) return st;
    if (k < 1 || !(eps >= 0.0) || std::isinf(eps)) return fail(BP_ERR_INVALID_ARG, "k < 1 or bad eps");
    if (!d_part_out && hg->num_nodes > 0) return fail(BP_ERR_INVALID_ARG, "d_part_out is NULL");
    BP_GUARD_BEGIN
    int dev = current_device();
    ScratchDev &sd = g_scratch[dev];
    std::lock_guard<std::mutex> lock(sd.mu);
    if (!sd.ready) {
        void *ptr = nullptr;
        hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !ptr) {
            (void)hipGetLastError();
            return fail(BP_ERR_DEVICE, std::string("hipGetSymbolAddress of the workspace: ") + hipGetErrorString(e));
        }
        sd.ptr = ptr;
        sd.ar.adopt(ptr, kScratchBytes);
        sd.ready = true;
    }
    int64_t P = 0;
    if (hg->num_hedges > 0) {
        int32_t p32 = 0;
        BP_HIP(hipMemcpyAsync(&p32, hg->hedge_offsets + hg->num_hedges, sizeof(int32_t), hipMemcpyDeviceToHost,
                              (hipStream_t)stream));
        BP_HIP(hipStreamSynchronize((hipStream_t)stream));
        P = p32;
    }
    int64_t need = workspace_bound(hg->num_nodes, hg->num_hedges, P, k);
    if (need > (int64_t)kScratchBytes)
        return fail(BP_ERR_OUT_OF_MEMORY, "input needs up to " + std::to_string(need) +
                                              " bytes of workspace; the fixed workspace holds " +
                                              std::to_string(kScratchBytes));
    CtxGuard g((hipStream_t)stream, params, &sd.ar, (LevelInfo *)sd.info);
    g.cx.no_graphs = true;  // instantiating a graph allocates
    return partition_device(g.cx, device_input(hg), k, eps, d_part_out, cut_out, report);
    BP_GUARD_END
}

bp_status bp_set_memory_limit(int64_t bytes)
{
    if (bytes < 0) return fail(BP_ERR_INVALID_ARG, "negative memory limit");
    g_arena_limit.store(bytes);
    return BP_OK;
}

bp_status bp_release_memory(void)
{
    BP_GUARD_BEGIN
    release_idle_arenas();
    return BP_OK;
    BP_GUARD_END
}

static void fill_batch_reports(const Ctx &cx, const std::vector<BatchOut> &res, int32_t tree_levels,
                               int64_t *cut_out, bp_report *reports)
{
    for (size_t g = 0; g < res.size(); g++) {
        if (cut_out) cut_out[g] = res[g].cut;
        if (!reports) continue;
        bp_report &r = reports[g];
        r.cut = res[g].cut;
        r.max_part_weight = res[g].maxw;
        r.part_weight_limit = res[g].limit;
        r.balanced = res[g].balanced;
        r.tree_levels = tree_levels;
        r.bisections = cx.bisections;
        r.coarsen_levels = cx.first_levels < 0 ? 0 : cx.first_levels;
        r.pins_coarsened = cx.pins_coarsened;
        r.pins_refined = cx.pins_refined;
        r.host_syncs = cx.lc.syncs;
        r.kernel_launches = cx.lc.launches;
        r.device_bytes = (int64_t)cx.ar->used();
        report_extras(cx, res[g].maxw, res[g].W, res[g].k, r);
    }
}

static bp_status batch_status(const std::vector<BatchOut> &res)
{
    for (auto &r : res)
        if (!r.balanced) return BP_WARN_IMBALANCED;
    return BP_OK;
}

static bp_status check_batch_args(int32_t n, const bp_hypergraph *graphs, const int32_t *k, const double *eps,
                                  const void *outs, const bp_params *params)
{
    if (n < 0) return fail(BP_ERR_INVALID_ARG, "n < 0");
    if (n > 0 && (!graphs || !k || !eps || !outs)) return fail(BP_ERR_INVALID_ARG, "NULL batch array");
    bp_status st = check_params(params);
    if (st != BP_OK) return st;
    for (int32_t g = 0; g < n; g++)
        if (k[g] < 1 || !(eps[g] >= 0.0) || std::isinf(eps[g]))
            return fail(BP_ERR_INVALID_ARG, "graph " + std::to_string(g) + ": k < 1 or bad eps");
    return BP_OK;
}

bp_status bp_partition_batch(int32_t n, const bp_hypergraph *graphs, const int32_t *k, const double *eps,
                             const bp_params *params, int32_t *const *part_out, int64_t *cut_out,
                             bp_report *reports)
{
    bp_status st = check_batch_args(n, graphs, k, eps, part_out, params);
    if (st != BP_OK) return st;
    for (int32_t g = 0; g < n; g++) {
        if ((st = validate_host(&graphs[g])) != BP_OK)
            return fail(st, "graph " + std::to_string(g) + ": " + g_last_error);
        if (!part_out[g] && graphs[g].num_nodes > 0)
            return fail(BP_ERR_INVALID_ARG, "graph " + std::to_string(g) + ": part_out is NULL");
    }
    if (n == 0) return BP_OK;
    BP_GUARD_BEGIN
    CtxGuard gd(nullptr, params);
    Ctx &cx = gd.cx;
    std::vector<BatchItem> items(n);
    std::vector<int32_t *> outs(n);
    std::vector<int64_t> obase(n + 1, 0);
    for (int32_t g = 0; g < n; g++) obase[g + 1] = obase[g] + graphs[g].num_nodes;
    int32_t *dpart = cx.ar->get<int32_t>(std::max<int64_t>(obase[n], 1));
    for (int32_t g = 0; g < n; g++) {
        Input in = upload(cx, &graphs[g]);
        items[g] = BatchItem{in.N, in.E, in.off, in.pins, in.nw, in.hw, k[g], eps[g]};
        outs[g] = dpart + obase[g];
    }
    int32_t tl = 0;
    std::vector<BatchOut> res = partition_batch(cx, items, outs, &tl);
    std::vector<int32_t> host((size_t)obase[n]);
    if (obase[n] > 0)
        BP_HIP(hipMemcpyAsync(host.data(), dpart, sizeof(int32_t) * (size_t)obase[n], hipMemcpyDeviceToHost,
                              cx.lc.stream));
    BP_HIP(hipStreamSynchronize(cx.lc.stream));
    for (int32_t g = 0; g < n; g++)
        if (graphs[g].num_nodes > 0)
            std::memcpy(part_out[g], host.data() + obase[g], sizeof(int32_t) * (size_t)graphs[g].num_nodes);
    fill_batch_reports(cx, res, tl, cut_out, reports);
    return batch_status(res);
    BP_GUARD_END
}

bp_status bp_partition_batch_device(int32_t n, const bp_hypergraph *graphs, const int32_t *k,
                                    const double *eps, const bp_params *params,
                                    int32_t *const *d_part_out, int64_t *cut_out, bp_report *reports,
                                    void *stream)
{
    bp_status st = check_batch_args(n, graphs, k, eps, d_part_out, params);
    if (st != BP_OK) return st;
    for (int32_t g = 0; g < n; g++) {
        if ((st = check_device_hg(&graphs[g])) != BP_OK)
            return fail(st, "graph " + std::to_string(g) + ": " + g_last_error);
        if (!d_part_out[g] && graphs[g].num_nodes > 0)
            return fail(BP_ERR_INVALID_ARG, "graph " + std::to_string(g) + ": d_part_out is NULL");
    }
    if (n == 0) return BP_OK;
    BP_GUARD_BEGIN
    CtxGuard gd((hipStream_t)stream, params);
    Ctx &cx = gd.cx;
    std::vector<BatchItem> items(n);
    std::vector<int32_t *> outs(n);
    for (int32_t g = 0; g < n; g++) {
        Input in = device_input(&graphs[g]);
        items[g] = BatchItem{in.N, in.E, in.off, in.pins, in.nw, in.hw, k[g], eps[g]};
        outs[g] = d_part_out[g];
    }
    int32_t tl = 0;
    std::vector<BatchOut> res = partition_batch(cx, items, outs, &tl);
    BP_HIP(hipStreamSynchronize(cx.lc.stream));
    fill_batch_reports(cx, res, tl, cut_out, reports);
    return batch_status(res);
    BP_GUARD_END
}

static Schedule to_schedule(const bp_schedule *s)
{
    Schedule r;
    r.incremental_min_pins = s->incremental_min_pins;
    r.seg_select_max_nodes = s->seg_select_max_nodes;
    r.round_chunk_max = s->round_chunk_max;
    r.fused_pick_lists = s->fused_pick_lists;
    r.fuse_max_pins = s->fuse_max_pins;
    r.chunk_select_max_nodes = s->chunk_select_max_nodes;
    r.graph_rounds = s->graph_rounds;
    return r;
}

static void from_schedule(const Schedule &r, bp_schedule *s)
{
    s->incremental_min_pins = r.incremental_min_pins;
    s->seg_select_max_nodes = r.seg_select_max_nodes;
    s->round_chunk_max = r.round_chunk_max;
    s->fused_pick_lists = r.fused_pick_lists;
    s->fuse_max_pins = r.fuse_max_pins;
    s->chunk_select_max_nodes = r.chunk_select_max_nodes;
    s->graph_rounds = r.graph_rounds;
}

static bool schedule_ok(const bp_schedule *s)
{
    return s && s->incremental_min_pins >= 0 && s->seg_select_max_nodes >= 0 && s->round_chunk_max >= 1 &&
           s->round_chunk_max <= 64 && s->fused_pick_lists >= 0 && s->fused_pick_lists <= 4096 &&
           s->fuse_max_pins >= 0 && s->chunk_select_max_nodes >= 0 && (s->graph_rounds == 0 || s->graph_rounds == 1);
}

void bp_schedule_default(bp_schedule *s)
{
    if (s) from_schedule(Schedule{}, s);
}

bp_status bp_schedule_set(const bp_schedule *s)
{
    if (!schedule_ok(s)) return fail(BP_ERR_INVALID_ARG, "schedule out of range");
    set_schedule(to_schedule(s));
    return BP_OK;
}

bp_status bp_schedule_get(bp_schedule *s)
{
    if (!s) return fail(BP_ERR_INVALID_ARG, "NULL schedule");
    from_schedule(current_schedule(), s);
    return BP_OK;
}

bp_status bp_autotune_batch_device(int32_t n, const bp_hypergraph *graphs, const int32_t *k, const double *eps,
                                   const bp_params *params, int32_t *const *d_scratch_parts, int32_t trials,
                                   bp_schedule *best, double *best_ms, void *stream)
{
    bp_status st = check_batch_args(n, graphs, k, eps, d_scratch_parts, params);
    if (st != BP_OK) return st;
    if (trials < 1 || !best) return fail(BP_ERR_INVALID_ARG, "trials < 1 or NULL best");
    for (int32_t g = 0; g < n; g++)
        if ((st = check_device_hg(&graphs[g])) != BP_OK)
            return fail(st, "graph " + std::to_string(g) + ": " + g_last_error);
    BP_GUARD_BEGIN
    std::vector<BatchItem> items(n);
    std::vector<int32_t *> outs(n);
    int64_t total_nodes = 0;
    for (int32_t g = 0; g < n; g++) {
        Input in = device_input(&graphs[g]);
        items[g] = BatchItem{in.N, in.E, in.off, in.pins, in.nw, in.hw, k[g], eps[g]};
        outs[g] = d_scratch_parts[g];
        total_nodes += in.N;
    }
    // one run under a schedule: time and the results (cuts and all part ids)
    auto run = [&](const Schedule &sc, std::vector<int64_t> &cuts, std::vector<int32_t> &parts) -> double {
        CtxGuard gd((hipStream_t)stream, params);
        Ctx &cx = gd.cx;
        cx.sched = sc;
        BP_HIP(hipStreamSynchronize(cx.lc.stream));
        auto t0 = std::chrono::steady_clock::now();
        int32_t tl = 0;
        std::vector<BatchOut> res = partition_batch(cx, items, outs, &tl);
        BP_HIP(hipStreamSynchronize(cx.lc.stream));
        double ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
        cuts.resize(n);
        for (int32_t g = 0; g < n; g++) cuts[g] = res[g].cut;
        parts.resize((size_t)total_nodes);
        int64_t o = 0;
        for (int32_t g = 0; g < n; g++) {
            if (items[g].N > 0)
                BP_HIP(hipMemcpy(parts.data() + o, outs[g], sizeof(int32_t) * (size_t)items[g].N,
                                 hipMemcpyDeviceToHost));
            o += items[g].N;
        }
        return ms;
    };
    Schedule base = current_schedule();
    std::vector<int64_t> ref_cuts, cuts;
    std::vector<int32_t> ref_parts, parts;
    run(base, ref_cuts, ref_parts);  // also warms the device memory pool
    std::vector<Schedule> cand;
    for (int32_t inc : {1 << 16, 1 << 18, 1 << 20, INT32_MAX})
        for (int32_t seg : {0, 4096, 16384, 32768})
            for (int32_t chunk : {16, 32})
                cand.push_back(
                    Schedule{inc, seg, chunk, base.fused_pick_lists, base.fuse_max_pins, base.chunk_select_max_nodes,
                             base.graph_rounds});
    double best_t = 1e300;
    Schedule best_s = base;
    for (const Schedule &sc : cand) {
        double t = 1e300;
        for (int32_t r = 0; r < trials; r++) {
            t = std::min(t, run(sc, cuts, parts));
            if (cuts != ref_cuts || parts != ref_parts)
                throw Error(BP_ERR_DEVICE, "a launch schedule changed the results");
        }
        if (t < best_t) {
            best_t = t;
            best_s = sc;
        }
    }
    from_schedule(best_s, best);
    if (best_ms) *best_ms = best_t;
    return BP_OK;
    BP_GUARD_END
}

bp_status bp_compute_cut_device(const bp_hypergraph *hg, int32_t k, const int32_t *d_part,
                                int64_t *cut, int64_t *max_part_weight, void *stream)
{
    bp_status st = check_device_hg(hg);
    if (st != BP_OK) return st;
    if (k < 1 || (!d_part && hg->num_nodes > 0)) return fail(BP_ERR_INVALID_ARG, "bad k or part");
    BP_GUARD_BEGIN
    CtxGuard g((hipStream_t)stream, nullptr);
    Input in = device_input(hg);
    validate_device(g.cx, in);
    Level L = view_level(g.cx, in);
    int32_t *ctr = g.cx.ar->get<int32_t>(8);
    fill(g.cx.lc, ctr, 8, 0);
    classify(g.cx, L, ctr);
    BP_HIP(hipMemcpyAsync(g.cx.info_h, ctr, 8 * sizeof(int32_t), hipMemcpyDeviceToHost, g.cx.lc.stream));
    g.cx.lc.sync();
    L.nmid = ((int32_t *)g.cx.info_h)[1];
    L.nbig = ((int32_t *)g.cx.info_h)[2];
    CutResult r = compute_cut(g.cx, L, in.N, in.nw, k, d_part);
    if (cut) *cut = r.cut;
    if (max_part_weight) *max_part_weight = r.maxw;
    return BP_OK;
    BP_GUARD_END
}

bp_status bp_compute_cut(const bp_hypergraph *hg, int32_t k, const int32_t *part, int64_t *cut,
                         int64_t *max_part_weight)
{
    bp_status st = validate_host(hg);
    if (st != BP_OK) return st;
    if (k < 1 || (!part && hg->num_nodes > 0)) return fail(BP_ERR_INVALID_ARG, "bad k or part");
    for (int32_t v = 0; v < hg->num_nodes; v++)
        if (part[v] < 0 || part[v] >= k) return fail(BP_ERR_INVALID_ARG, "part id out of range");
    BP_GUARD_BEGIN
    CtxGuard g(nullptr, nullptr);
    Input in = upload(g.cx, hg);
    int32_t *d_part = g.cx.ar->get<int32_t>(hg->num_nodes);
    if (hg->num_nodes > 0)
        BP_HIP(hipMemcpyAsync(d_part, part, sizeof(int32_t) * (size_t)hg->num_nodes,
                              hipMemcpyHostToDevice, g.cx.lc.stream));
    Level L = view_level(g.cx, in);
    int32_t *ctr = g.cx.ar->get<int32_t>(8);
    fill(g.cx.lc, ctr, 8, 0);
    classify(g.cx, L, ctr);
    BP_HIP(hipMemcpyAsync(g.cx.info_h, ctr, 8 * sizeof(int32_t), hipMemcpyDeviceToHost, g.cx.lc.stream));
    g.cx.lc.sync();
    L.nmid = ((int32_t *)g.cx.info_h)[1];
    L.nbig = ((int32_t *)g.cx.info_h)[2];
    CutResult r = compute_cut(g.cx, L, in.N, in.nw, k, d_part);
    if (cut) *cut = r.cut;
    if (max_part_weight) *max_part_weight = r.maxw;
    return BP_OK;
    BP_GUARD_END
}

// ---- single steps ----------------------------------------------------------------------

// Prepares a one-segment level over the caller's device CSR with its schedule.
static Level step_level(Ctx &cx, const bp_hypergraph *hg)
{
    Input in = device_input(hg);
    Level L = view_level(cx, in);
    int32_t *ctr = cx.ar->get<int32_t>(8);
    fill(cx.lc, ctr, 8, 0);
    classify(cx, L, ctr);
    BP_HIP(hipMemcpyAsync(cx.info_h, ctr, 8 * sizeof(int32_t), hipMemcpyDeviceToHost, cx.lc.stream));
    cx.lc.sync();
    L.nmid = ((int32_t *)cx.info_h)[1];
    L.nbig = ((int32_t *)cx.info_h)[2];
    L.nhuge = ((int32_t *)cx.info_h)[3];
    L.maxseg_nodes = L.N;
    L.maxseg_pins = L.P;
    L.maxseg_hedges = L.E;
    build_incidence(cx, L);
    return L;
}

bp_status bp_step_match(const bp_hypergraph *hg, int32_t policy, int32_t *d_match, void *stream)
{
    bp_status st = check_device_hg(hg);
    if (st != BP_OK) return st;
    if (policy < BP_LDH || policy > BP_RAND) return fail(BP_ERR_INVALID_ARG, "bad policy");
    BP_GUARD_BEGIN
    CtxGuard g((hipStream_t)stream, nullptr);
    Ctx &cx = g.cx;
    cx.prm.policy = policy;
    Level L = step_level(cx, hg);
    uint8_t *sact = cx.ar->get<uint8_t>(1);
    fill(cx.lc, sact, 1, (uint8_t)1);
    uint64_t *key = cx.ar->get<uint64_t>(L.N);
    uint64_t *cg = cx.ar->get<uint64_t>(L.E);
    run_match_keys(cx, L, sact, key);
    fill(cx.lc, cg, L.E, (uint64_t)0);
    launch(cx.lc, "decode", 0.0, k_decode, ceil_div(L.N, kBlock), kBlock, 0, L.N,
           (const uint64_t *)key, (const int32_t *)L.nseg, (const int32_t *)L.hbase,
           (const uint8_t *)sact, (const int32_t *)L.nw, d_match, cg);
    return BP_OK;
    BP_GUARD_END
}

bp_status bp_step_coarsen(const bp_hypergraph *hg, int32_t policy, int32_t *d_parent,
                          int32_t *d_coarse_offsets, int32_t *d_coarse_pins,
                          int32_t *d_coarse_node_w, int32_t *d_coarse_hedge_w,
                          int32_t *coarse_nodes, int32_t *coarse_hedges, void *stream)
{
    bp_status st = check_device_hg(hg);
    if (st != BP_OK) return st;
    if (policy < BP_LDH || policy > BP_RAND) return fail(BP_ERR_INVALID_ARG, "bad policy");
    BP_GUARD_BEGIN
    CtxGuard g((hipStream_t)stream, nullptr);
    Ctx &cx = g.cx;
    cx.prm.policy = policy;
    cx.prm.max_levels = 1000;
    cx.prm.min_coarse_nodes = 0;
    Level L = step_level(cx, hg);
    Segs sg = alloc_segs(*cx.ar, 1);
    uint8_t *sact = sg.active, *sact_next = cx.ar->get<uint8_t>(1);
    fill(cx.lc, sact, 1, (uint8_t)1);
    Level c;
    coarsen_level(cx, L, sg, sact, sact_next, 0, c);
    hipStream_t s = cx.lc.stream;
    if (L.N > 0) {
        BP_HIP(hipMemcpyAsync(d_parent, L.parent, sizeof(int32_t) * L.N, hipMemcpyDeviceToDevice, s));
        if (c.N > 0)
            BP_HIP(hipMemcpyAsync(d_coarse_node_w, c.nw, sizeof(int32_t) * c.N, hipMemcpyDeviceToDevice, s));
    }
    BP_HIP(hipMemcpyAsync(d_coarse_offsets, c.off, sizeof(int32_t) * ((size_t)c.E + 1), hipMemcpyDeviceToDevice, s));
    if (c.P > 0)
        BP_HIP(hipMemcpyAsync(d_coarse_pins, c.pins, sizeof(int32_t) * c.P, hipMemcpyDeviceToDevice, s));
    if (c.E > 0)
        BP_HIP(hipMemcpyAsync(d_coarse_hedge_w, c.hw, sizeof(int32_t) * c.E, hipMemcpyDeviceToDevice, s));
    if (coarse_nodes) *coarse_nodes = c.N;
    if (coarse_hedges) *coarse_hedges = c.E;
    return BP_OK;
    BP_GUARD_END
}

bp_status bp_step_gains(const bp_hypergraph *hg, const uint8_t *d_side, int32_t *d_gain, void *stream)
{
    bp_status st = check_device_hg(hg);
    if (st != BP_OK) return st;
    BP_GUARD_BEGIN
    CtxGuard g((hipStream_t)stream, nullptr);
    Ctx &cx = g.cx;
    Level L = step_level(cx, hg);
    Segs sg = alloc_segs(*cx.ar, 1);
    fill(cx.lc, sg.gmask, 1, (uint8_t)1);
    L.side = const_cast<uint8_t *>(d_side);
    run_gains(cx, L, sg, d_gain, false, nullptr);
    return BP_OK;
    BP_GUARD_END
}

// one segment of k0 : k1 with explicit bounds, for the initial/refine steps
static Segs step_segs(Ctx &cx, Level &L, int32_t k0, int32_t k1, int64_t max0, int64_t max1)
{
    Segs sg = alloc_segs(*cx.ar, 1);
    fill(cx.lc, sg.k0, 1, k0);
    fill(cx.lc, sg.k1, 1, k1);
    fill(cx.lc, sg.coarsest, 1, 0);
    fill(cx.lc, sg.stuck, 1, 0);
    fill(cx.lc, sg.max0, 1, max0);
    fill(cx.lc, sg.max1, 1, max1);
    fill(cx.lc, sg.st.hist, 2 * kBins, 0u);
    fill(cx.lc, sg.st.ctl, 4, 0);
    fill(cx.lc, sg.st.tick, 1, 0);
    fill(cx.lc, sg.st.rsel, 2, 0);
    fill(cx.lc, sg.W, 1, (int64_t)0);
    launch(cx.lc, "seg_setup", 0.0, k_seg_total, reduce_grid(L.N), kBlock, 0, L.N,
           (const int32_t *)L.nseg, (const int32_t *)L.nw, (unsigned long long *)sg.W);
    int32_t mm = (int32_t)ceil_sqrt_i64(L.N);
    sg.cand_stride = next_pow2(std::max(mm, kBalGather));
    sg.cand = cx.ar->get<uint64_t>(sg.cand_stride);
    alloc_chunk_bufs(*cx.ar, sg, chunk_path(cx, L) ? ceil_div(L.N, kChunkNodes) + L.S : 0);
    return sg;
}

bp_status bp_step_initial(const bp_hypergraph *hg, int32_t k0, int32_t k1, uint8_t *d_side, void *stream)
{
    bp_status st = check_device_hg(hg);
    if (st != BP_OK) return st;
    if (k0 < 1 || k1 < 1) return fail(BP_ERR_INVALID_ARG, "k0, k1 must be >= 1");
    BP_GUARD_BEGIN
    CtxGuard g((hipStream_t)stream, nullptr);
    Ctx &cx = g.cx;
    Level L = step_level(cx, hg);
    Segs sg = step_segs(cx, L, k0, k1, INT64_MAX, INT64_MAX);
    L.side = d_side;
    int32_t *gain = cx.ar->get<int32_t>(L.N);
    launch(cx.lc, "project", 0.0, k_project, ceil_div(L.N, kBlock), kBlock, 0, L.N, 0,
           (const int32_t *)L.nseg, (const int32_t *)sg.coarsest, (const int32_t *)nullptr,
           (const uint8_t *)nullptr, L.side, (unsigned long long *)nullptr, 0);
    fill(cx.lc, sg.w, 2, (int64_t)0);
    launch(cx.lc, "side_weights", 0.0, k_side_weights, reduce_grid(L.N), kBlock, 0, L.N,
           (const int32_t *)L.nseg, (const uint8_t *)L.side, (const int32_t *)L.nw,
           (unsigned long long *)sg.w);
    initial_rounds(cx, L, sg, 0, gain);
    return BP_OK;
    BP_GUARD_END
}

bp_status bp_step_refine(const bp_hypergraph *hg, int32_t iters, int64_t max0, int64_t max1,
                         uint8_t *d_side, int32_t *stuck, void *stream)
{
    bp_status st = check_device_hg(hg);
    if (st != BP_OK) return st;
    if (iters < 0) return fail(BP_ERR_INVALID_ARG, "iters < 0");
    BP_GUARD_BEGIN
    CtxGuard g((hipStream_t)stream, nullptr);
    Ctx &cx = g.cx;
    cx.prm.refine_iters = iters;
    Level L = step_level(cx, hg);
    Segs sg = step_segs(cx, L, 1, 1, max0, max1);
    L.side = d_side;
    int32_t *gain = cx.ar->get<int32_t>(L.N);
    fill(cx.lc, sg.w, 2, (int64_t)0);
    launch(cx.lc, "side_weights", 0.0, k_side_weights, reduce_grid(L.N), kBlock, 0, L.N,
           (const int32_t *)L.nseg, (const uint8_t *)L.side, (const int32_t *)L.nw,
           (unsigned long long *)sg.w);
    refine_level(cx, L, sg, 0, gain);
    BP_HIP(hipMemcpyAsync(cx.info_h, sg.stuck, sizeof(int32_t), hipMemcpyDeviceToHost, cx.lc.stream));
    cx.lc.sync();
    if (stuck) *stuck = *(int32_t *)cx.info_h;
    return BP_OK;
    BP_GUARD_END
}

bp_status bp_step_bisect(const bp_hypergraph *hg, int32_t k0, int32_t k1, uint64_t F,
                         const bp_params *params, uint8_t *d_side, int32_t *levels, void *stream)
{
    bp_status st = check_device_hg(hg);
    if (st != BP_OK) return st;
    if ((st = check_params(params)) != BP_OK) return st;
    if (k0 < 1 || k1 < 1) return fail(BP_ERR_INVALID_ARG, "k0, k1 must be >= 1");
    BP_GUARD_BEGIN
    CtxGuard g((hipStream_t)stream, params);
    Ctx &cx = g.cx;
    Level L = step_level(cx, hg);
    TreeLevel t;
    t.L = L;
    t.sg = alloc_segs(*cx.ar, 1);
    t.ksub = cx.ar->get<int32_t>(1);
    fill(cx.lc, t.ksub, 1, k0 + k1);
    int32_t *k0_fixed = cx.ar->get<int32_t>(1);
    fill(cx.lc, k0_fixed, 1, k0);
    t.F = cx.ar->get<uint64_t>(1);
    fill(cx.lc, t.F, 1, F);
    cx.clear_info();
    seg_setup(cx, t, k0_fixed);
    LevelInfo inf = cx.readback();
    t.active0 = inf.active;
    bisect_all(cx, t.L, t.sg, t.active0);
    if (L.N > 0)
        BP_HIP(hipMemcpyAsync(d_side, t.L.side, L.N, hipMemcpyDeviceToDevice, cx.lc.stream));
    if (levels) *levels = cx.first_levels < 0 ? 0 : cx.first_levels;
    return BP_OK;
    BP_GUARD_END
}

// ---- profiling -----------------------------------------------------------------------

void bp_profile_enable(int32_t on) { Profiler::get().on = on != 0; }

bp_status bp_profile_floor(int32_t n, void *stream)
{
    if (n < 0) return fail(BP_ERR_INVALID_ARG, "n < 0");
    BP_GUARD_BEGIN
    CtxGuard g((hipStream_t)stream, nullptr);
    for (int32_t i = 0; i < n; i++) launch(g.cx.lc, "event_floor", 0.0, k_empty, 1, 64, 0, 0);
    return BP_OK;
    BP_GUARD_END
}

void bp_profile_reset(void)
{
    Profiler &p = Profiler::get();
    std::lock_guard<std::mutex> g(p.mu);
    p.acc.clear();
}

int32_t bp_profile_read(bp_kernel_stat *out, int32_t cap)
{
    Profiler &p = Profiler::get();
    std::lock_guard<std::mutex> g(p.mu);
    int32_t n = (int32_t)p.acc.size();
    for (int32_t i = 0; i < n && i < cap && out; i++) {
        memset(&out[i], 0, sizeof(bp_kernel_stat));
        strncpy(out[i].name, p.acc[i].name.c_str(), sizeof(out[i].name) - 1);
        out[i].launches = p.acc[i].launches;
        out[i].total_ms = p.acc[i].ms;
        out[i].bytes = p.acc[i].bytes;
    }
    return n;
}

}  // extern "C"
