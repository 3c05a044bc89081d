// Balance step of Algorithm 5 (and the rounds of Algorithm 3) for small
// segments, every round in one launch.
//
// One workgroup per segment keeps the segment's gains and sides in LDS and
// runs the rounds itself: the over-weight side, the ceil(sqrt n) best nodes
// of that side in (gain desc, id asc) order, the shortest prefix covering the
// excess cut back to what the other side can take, the moves, and the gain
// changes they cause, until the segment is balanced or no node can move.
// The gains start from a full computation (Algorithm 4) and follow the moves
// exactly: after a round, every hyperedge with a moved pin is recounted and
// each of its pins' gains changes by the difference of its contributions
// (integer sums, so equal to a recomputation).  Segments are independent, so
// each runs only the rounds it needs; no launch and no host check per round.
//
// Selection inside a round, with each thread's gains in registers: radix
// passes over u = gmax - gain (8-bit digits from the top) narrow the r-th
// node down to a bin; a bin of at most kFuseCand nodes is ranked directly by
// (u, id), a larger one whose nodes share one u by id with one scan.  The
// chosen set is the one the multi-launch path chooses.
#pragma once
#include "uncoarsen.hpp"

namespace bp {

constexpr int kFuseThreads = 1024;
constexpr int32_t kFuseNodes = 8192;                 // nodes of a segment (LDS gains, sides, weights)
constexpr int kFuseItems = kFuseNodes / kFuseThreads;  // per thread, strided
constexpr int32_t kFuseWords = kBins;                // hyperedge bitmap words (shares the histogram)
constexpr int32_t kFuseHedges = kFuseWords * 32;     // hyperedges of a segment
constexpr int kFuseKeys = 128;                       // >= ceil(sqrt(kFuseNodes))
constexpr int kFuseDigit = 8;                        // radix digit of the selection
constexpr int kFuseBins = 1 << kFuseDigit;
constexpr int kFuseSmallDeg = 16;                    // larger hyperedges: one wavefront each
constexpr int kFuseQueue = 1024;
constexpr int kFuseCand = 256;                       // bins this small are ranked directly

// Level arrays the rounds read, and the per-segment state they change.
struct FuseArgs {
    const int32_t *off, *pins, *hw, *noff, *inc, *nw, *nbase, *hbase;
    uint8_t *side;
    const int64_t *max0, *max1;
    unsigned long long *segw;
    uint8_t *done;
    int32_t *stuck;
    int32_t *rounds;    // atomicMax of the rounds any segment ran (may be null)
    int32_t max_pins;   // segments with more pins are left to the multi-launch rounds
    // initial bisection only: segments whose coarsest level is `level`, their
    // part counts and total weight
    const int32_t *coarsest, *k0, *k1;
    const int64_t *W;
    int32_t level;
};

// LDS the selection of a list's best nodes works in.
struct PickLds {
    uint32_t *hist;         // kFuseBins
    uint64_t *cand;         // kFuseCand
    int32_t *tcnt;          // ITEMS * TH / 64
    uint64_t *keys;         // KCAP (a power of two): the chosen nodes' order keys
    int32_t *ncand, *nkeys; // zero on entry
    int32_t *sbin;          // [3]
};

// Appends to pl.keys the order keys (gain desc, id asc) of the r nodes of
// smallest (u, id) among a list's c nodes, u = gmax - gain.  uat(j, u) tells
// whether item j of this thread (node id j * TH + threadIdx.x) is in the list
// and sets its u; T is the bit length of the largest u.  Every thread calls;
// the keys are complete after the caller's next barrier.
//
// Nodes with u < ulo are chosen, and the rem smallest of "the bin", u in
// [ulo, ulo + 2^lo): by rank when the bin is small (bmode 1), by id when its
// u are all equal (bmode 2).  Radix passes over u (8-bit digits from the top)
// narrow the bin down.
template <int TH, int ITEMS, int KCAP, typename UAt>
__device__ __forceinline__ void pick_best(UAt uat, int32_t gmax, int32_t a0, int32_t r, int32_t c, int T,
                                          const PickLds &pl)
{
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    uint64_t ulo = r == c ? ~0ull : 0ull;
    int lo = 0, bmode = 0;
    int32_t rem = 0;
    if (r > 0 && r < c) {
        uint32_t pre = 0;
        rem = r;
        for (int p = 0;; p++) {
            int hi = T - kFuseDigit * p;
            lo = hi - kFuseDigit > 0 ? hi - kFuseDigit : 0;
            if (tid < kFuseBins) pl.hist[tid] = 0;
            __syncthreads();
#pragma unroll
            for (int j = 0; j < ITEMS; j++) {
                uint32_t u = 0;
                bool in = uat(j, u);  // hi <= 24 when p > 0
                bool act = in && (p == 0 || ((u ^ pre) >> hi) == 0);
                lds_hist_add(act, (u >> lo) & ((1u << (hi - lo)) - 1u), pl.hist);
            }
            __syncthreads();
            if (wv == 0) {  // the bin holding the rem-th key: one wavefront
                constexpr int per = kFuseBins / 64;
                int32_t x[per], loc = 0;
#pragma unroll
                for (int j = 0; j < per; j++) {
                    x[j] = (int32_t)pl.hist[lane * per + j];
                    loc += x[j];
                }
                int32_t ex = wave_incl_scan(loc) - loc;
                if (ex < rem && rem <= ex + loc) {
                    int32_t acc = ex;
#pragma unroll
                    for (int j = 0; j < per; j++) {
                        if (acc < rem && rem <= acc + x[j]) {
                            pl.sbin[0] = lane * per + j;
                            pl.sbin[1] = acc;
                            pl.sbin[2] = x[j];
                        }
                        acc += x[j];
                    }
                }
            }
            __syncthreads();
            int32_t bin = pl.sbin[0], left = rem - pl.sbin[1], inb = pl.sbin[2];
            pre |= (uint32_t)bin << lo;
            rem = left;
            ulo = pre;
            if (left == inb) {  // the whole bin
                ulo = (uint64_t)pre + (1ull << lo);
                break;
            }
            if (inb <= kFuseCand) {
                bmode = 1;
                break;
            }
            if (lo == 0) {
                bmode = 2;
                break;
            }
        }
    }

    if (bmode == 1) {
        // the bin's nodes as (u, id) keys; each chosen iff fewer than rem of
        // them are smaller (TH / kFuseCand threads per key)
#pragma unroll
        for (int j = 0; j < ITEMS; j++) {
            uint32_t u = 0;
            bool in = uat(j, u);
            int32_t k = lds_wave_slot(in && (u >> lo) == (uint32_t)(ulo >> lo), pl.ncand);
            if (k >= 0) pl.cand[k] = ((uint64_t)u << 32) | (uint32_t)(j * TH + tid);
        }
        __syncthreads();
        constexpr int tpc = TH / kFuseCand;
        int32_t nc = *pl.ncand, ci = tid / tpc, part = tid % tpc;
        uint64_t x = ci < nc ? pl.cand[ci] : 0ull;
        int32_t rk = 0;
        if (ci < nc) {
#pragma unroll 8
            for (int32_t q = part; q < nc; q += tpc) rk += pl.cand[q] < x;
        }
#pragma unroll
        for (int o = 1; o < tpc; o <<= 1) rk += __shfl_xor(rk, o, 64);
        int32_t k = lds_wave_slot(ci < nc && part == 0 && rk < rem, pl.nkeys);
        if (k >= 0)
            pl.keys[k & (KCAP - 1)] = gain_order_key((int32_t)((int64_t)gmax - (uint32_t)(x >> 32)),
                                                     (uint32_t)(a0 + (int32_t)(x & 0xffffffffu)));
    } else if (bmode == 2) {
        // the bin's nodes all have u == ulo: the first rem by id (ids ascend
        // with (item j, wavefront, lane))
#pragma unroll
        for (int j = 0; j < ITEMS; j++) {
            uint32_t u = 0;
            bool t = uat(j, u) && u == (uint32_t)ulo;
            unsigned long long b = __ballot(t);
            if (lane == 0) pl.tcnt[j * (TH / 64) + wv] = __popcll(b);
        }
        __syncthreads();
        if (wv == 0) {
            constexpr int nc = ITEMS * (TH / 64), per = nc / 64;
            int32_t v[per], sum = 0;
#pragma unroll
            for (int q = 0; q < per; q++) {
                v[q] = pl.tcnt[lane * per + q];
                sum += v[q];
            }
            int32_t base = wave_incl_scan(sum) - sum;
#pragma unroll
            for (int q = 0; q < per; q++) {
                pl.tcnt[lane * per + q] = base;
                base += v[q];
            }
        }
        __syncthreads();
#pragma unroll
        for (int j = 0; j < ITEMS; j++) {
            uint32_t u = 0;
            bool t = uat(j, u) && u == (uint32_t)ulo;
            unsigned long long b = __ballot(t);
            int32_t k = lds_wave_slot(
                t && pl.tcnt[j * (TH / 64) + wv] + __popcll(b & ((1ull << lane) - 1ull)) < rem, pl.nkeys);
            if (k >= 0)
                pl.keys[k & (KCAP - 1)] = gain_order_key((int32_t)((int64_t)gmax - u), (uint32_t)(a0 + j * TH + tid));
        }
    }
    // and the nodes below the bin
    if (r > 0) {
#pragma unroll
        for (int j = 0; j < ITEMS; j++) {
            uint32_t u = 0;
            bool in = uat(j, u);
            int32_t k = lds_wave_slot(in && (uint64_t)u < ulo, pl.nkeys);
            if (k >= 0)
                pl.keys[k & (KCAP - 1)] = gain_order_key((int32_t)((int64_t)gmax - u), (uint32_t)(a0 + j * TH + tid));
        }
    }
}

// Whether segment s is balanced here (nodes, hyperedges and pins in range).
__device__ __forceinline__ bool fuse_fits(const FuseArgs &fa, int32_t s)
{
    int32_t n = fa.nbase[s + 1] - fa.nbase[s];
    int32_t e0 = fa.hbase[s], ne = fa.hbase[s + 1] - e0;
    int32_t np = fa.off[e0 + ne] - fa.off[e0];
    return n <= kFuseNodes && ne <= kFuseHedges && np <= fa.max_pins;
}

// Gain contributions of hyperedge e to its pins.  full: add the hyperedge's
// contribution (gains start at 0).  Otherwise the pins flagged in mv moved
// from side h to 1 - h in the last round: add new minus old contribution.
// Lanes lane, lane + stride, ... of the hyperedge's pins (stride 1: a thread
// alone, 64: a wavefront).
// The same for d <= R * stride: the pins are loaded once, all in flight
// together, and kept in registers for both the count and the deltas.
template <int R>
__device__ __forceinline__ void fuse_hedge_regs(int32_t e, int32_t b, int32_t d, bool full, int h, int lane,
                                                int stride, int32_t a0, const FuseArgs &fa, const uint8_t *sd,
                                                const uint32_t *mv, int32_t *g)
{
    int32_t u[R];
#pragma unroll
    for (int k = 0; k < R; k++) u[k] = fa.pins[b + min(lane + k * stride, d - 1)] - a0;
    int32_t n1 = 0, km = 0;
#pragma unroll
    for (int k = 0; k < R; k++)
        if (lane + k * stride < d) {
            n1 += sd[u[k]];
            if (!full) km += (mv[u[k] >> 5] >> (u[k] & 31)) & 1;
        }
    if (stride > 1) {
        n1 = wave_sum(n1);
        km = wave_sum(km);
    }
    int32_t w = fa.hw[e];
    int2 cn = hedge_contrib_value(w, d, n1);
    int2 co = make_int2(0, 0);
    if (!full) {
        if (km == 0) return;
        co = hedge_contrib_value(w, d, h ? n1 + km : n1 - km);
    }
#pragma unroll
    for (int k = 0; k < R; k++) {
        if (lane + k * stride >= d) continue;
        int sn = sd[u[k]];
        int so = full ? sn : (sn ^ (int)((mv[u[k] >> 5] >> (u[k] & 31)) & 1));
        int32_t delta = (sn ? cn.y : cn.x) - (full ? 0 : (so ? co.y : co.x));
        if (delta) atomicAdd(&g[u[k]], delta);
    }
}

__device__ __forceinline__ void fuse_hedge(int32_t e, bool full, int h, int lane, int stride, int32_t a0,
                                           const FuseArgs &fa, const uint8_t *sd, const uint32_t *mv,
                                           int32_t *g)
{
    int32_t b = fa.off[e], d = fa.off[e + 1] - b;
    // pins in registers when few (a thread: up to 4, or up to kFuseSmallDeg;
    // a wavefront: up to 512)
    if (stride == 1 && d <= kFuseSmallDeg) {
        if (__ballot(d > 4) == 0) fuse_hedge_regs<4>(e, b, d, full, h, lane, 1, a0, fa, sd, mv, g);
        else fuse_hedge_regs<kFuseSmallDeg>(e, b, d, full, h, lane, 1, a0, fa, sd, mv, g);
        return;
    }
    if (stride == 64 && d <= 512) {
        fuse_hedge_regs<8>(e, b, d, full, h, lane, 64, a0, fa, sd, mv, g);
        return;
    }
    int32_t n1 = 0, km = 0;
#pragma unroll 4
    for (int32_t i = lane; i < d; i += stride) {
        int32_t u = fa.pins[b + i] - a0;
        n1 += sd[u];
        if (!full) km += (mv[u >> 5] >> (u & 31)) & 1;
    }
    if (stride > 1) {
        n1 = wave_sum(n1);
        km = wave_sum(km);
    }
    int32_t w = fa.hw[e];
    int2 cn = hedge_contrib_value(w, d, n1);
    int2 co = make_int2(0, 0);
    if (!full) {
        if (km == 0) return;
        co = hedge_contrib_value(w, d, h ? n1 + km : n1 - km);
    }
#pragma unroll 4
    for (int32_t i = lane; i < d; i += stride) {
        int32_t u = fa.pins[b + i] - a0;
        int sn = sd[u];
        int so = full ? sn : (sn ^ (int)((mv[u >> 5] >> (u & 31)) & 1));
        int32_t delta = (sn ? cn.y : cn.x) - (full ? 0 : (so ? co.y : co.x));
        if (delta) atomicAdd(&g[u], delta);
    }
}

// INIT: the rounds of Algorithm 3 instead (segments at their coarsest
// level, all nodes starting on side 1): while side 0 is below its share
// W k0 / (k0 + k1) and side 1 has nodes, move the ceil(sqrt n) best nodes of
// side 1 to side 0 (all of them, no prefix).  The gains follow the moves in
// the same way.
template <bool INIT>
__global__ __launch_bounds__(kFuseThreads) void k_seg_fused(int32_t S, FuseArgs fa)
{
    __shared__ int32_t g[kFuseNodes], nwl[kFuseNodes], noffl[kFuseNodes + 1];
    __shared__ uint8_t sd[kFuseNodes];
    __shared__ uint32_t mv[kFuseNodes / 32];
    __shared__ uint32_t work[kFuseWords];  // radix histogram, then the hyperedge bitmap
    __shared__ uint64_t keys[kFuseKeys], sorted[kFuseKeys];
    __shared__ int32_t dpre[kFuseKeys + 1];
    __shared__ int32_t queue[kFuseQueue];
    __shared__ int32_t tcnt[kFuseItems * (kFuseThreads / 64)];
    __shared__ int32_t red[kFuseThreads / 64][3];
    __shared__ int64_t w01[2];
    __shared__ uint64_t cand[kFuseCand];
    __shared__ int32_t qn, nkeys, ncand, sbin[3], np_s;

    int32_t s = blockIdx.x;
    if (s >= S || (INIT ? fa.coarsest[s] != fa.level : fa.done[s] != 0) || !fuse_fits(fa, s)) return;
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    const int32_t a0 = fa.nbase[s], n = fa.nbase[s + 1] - a0;
    const int32_t e0 = fa.hbase[s], ne = fa.hbase[s + 1] - e0;
    const int32_t m = (int32_t)ceil_sqrt_i64(n);
    const int64_t mx0 = INIT ? 0 : fa.max0[s], mx1 = INIT ? 0 : fa.max1[s];
    const int64_t ks = INIT ? (int64_t)fa.k0[s] + fa.k1[s] : 0, Wk0 = INIT ? fa.W[s] * (int64_t)fa.k0[s] : 0;

    for (int32_t i = tid; i < n; i += kFuseThreads) {
        g[i] = 0;
        sd[i] = fa.side[a0 + i];
        nwl[i] = fa.nw[a0 + i];
        noffl[i] = fa.noff[a0 + i];
    }
    if (tid == 0) noffl[n] = fa.noff[a0 + n];
    for (int32_t i = tid; i < kFuseNodes / 32; i += kFuseThreads) mv[i] = 0;
    if (tid == 0) {
        qn = 0;
        w01[0] = (int64_t)fa.segw[2 * s];
        w01[1] = (int64_t)fa.segw[2 * s + 1];
    }
    __syncthreads();

    // every gain, hyperedge by hyperedge (large ones one wavefront each)
    for (int32_t i = tid; i < ne; i += kFuseThreads) {
        int32_t e = e0 + i;
        if (fa.off[e + 1] - fa.off[e] > kFuseSmallDeg) {
            int32_t q = atomicAdd(&qn, 1);
            if (q < kFuseQueue) {
                queue[q] = e;
                continue;
            }
        }
        fuse_hedge(e, true, 0, 0, 1, a0, fa, sd, mv, g);
    }
    __syncthreads();
    for (int32_t q = wv; q < min(qn, kFuseQueue); q += kFuseThreads / 64)
        fuse_hedge(queue[q], true, 0, lane, 64, a0, fa, sd, mv, g);
    __syncthreads();

    int32_t rounds = 0;
    for (;;) {
        // the side over its bound, the excess and the room
        int64_t w0 = w01[0], w1 = w01[1];
        int h = INIT ? 1 : (w0 > mx0 ? 0 : (w1 > mx1 ? 1 : -1));
        if (h < 0) break;
        if (rounds > n) {  // never: each round moves a node for good, so <= n rounds
            if (tid == 0 && !INIT) fa.stuck[s] = 1;
            break;
        }

        // this thread's nodes (ids j * kFuseThreads + tid): gains in registers,
        // bit j of `on` = node on side h
        int32_t gi[kFuseItems];
        uint32_t on = 0;
#pragma unroll
        for (int j = 0; j < kFuseItems; j++) {
            int32_t i = j * kFuseThreads + tid;
            gi[j] = 0;
            if (i < n) {
                gi[j] = g[i];
                if (sd[i] == h) on |= 1u << j;
            }
        }
        // list h: size and gain extremes
        int32_t c = __popc(on), gmax = INT32_MIN, gmin = INT32_MAX;
#pragma unroll
        for (int j = 0; j < kFuseItems; j++)
            if ((on >> j) & 1) {
                gmax = max(gmax, gi[j]);
                gmin = min(gmin, gi[j]);
            }
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) {
            c += __shfl_xor(c, o, 64);
            gmax = max(gmax, __shfl_xor(gmax, o, 64));
            gmin = min(gmin, __shfl_xor(gmin, o, 64));
        }
        if (lane == 0) {
            red[wv][0] = c;
            red[wv][1] = gmax;
            red[wv][2] = gmin;
        }
        if (tid == 0) {
            qn = 0;
            nkeys = 0;
            ncand = 0;
        }
        __syncthreads();
        c = 0;
        gmax = INT32_MIN;
        gmin = INT32_MAX;
#pragma unroll
        for (int w = 0; w < kFuseThreads / 64; w++) {
            c += red[w][0];
            gmax = max(gmax, red[w][1]);
            gmin = min(gmin, red[w][2]);
        }
        if (INIT && !(w0 * ks < Wk0 && c > 0)) break;  // Algorithm 3's loop test
        rounds++;
        int32_t r = c < m ? c : m;
        // from here on the registers hold u = gmax - gain
#pragma unroll
        for (int j = 0; j < kFuseItems; j++) gi[j] = (int32_t)(uint32_t)((int64_t)gmax - gi[j]);

        PickLds pl{work, cand, tcnt, keys, &ncand, &nkeys, sbin};
        pick_best<kFuseThreads, kFuseItems, kFuseKeys>(
            [=](int j, uint32_t &u) -> bool {
                u = (uint32_t)gi[j];
                return (on >> j) & 1;
            },
            gmax, a0, r, c, bitlen_u32((uint32_t)((int64_t)gmax - gmin)), pl);
        __syncthreads();
        int32_t cnt = min(nkeys, kFuseKeys);  // r of them
        // the moving nodes: all chosen ones (INIT), else a prefix in order
        const uint64_t *mlist = INIT ? keys : sorted;
        if (!INIT) block_rank_sort(keys, sorted, cnt);

        // prefix, moves and side weights (one wavefront)
        if (wv == 0) {
            int64_t need = h ? w1 - mx1 : w0 - mx0, room = h ? mx0 - w0 : mx1 - w1;
            int32_t p1 = cnt, fit = INIT ? cnt : 0;
            int64_t carry = 0;
            for (int32_t base = 0; !INIT && base < cnt; base += 64) {
                int32_t i = base + lane;
                int64_t w = i < cnt ? (int64_t)nwl[(uint32_t)(sorted[i] & 0xffffffffu) - a0] : 0;
                int64_t incl = wave_incl_scan(w) + carry;
                unsigned long long hit = __ballot(i < cnt && incl >= need);
                fit += __popcll(__ballot(i < cnt && incl <= room));
                if (hit) {
                    p1 = base + __ffsll((long long)hit);
                    break;
                }
                carry = __shfl(incl, 63, 64);
            }
            int32_t p = fit < p1 ? fit : p1;
            int64_t moved = 0;
            int32_t dcarry = 0;
            for (int32_t base = 0; base < p; base += 64) {
                int32_t i = base + lane;
                int32_t deg = 0;
                if (i < p) {
                    int32_t v = (int32_t)(uint32_t)(mlist[i] & 0xffffffffu), u = v - a0;
                    sd[u] = (uint8_t)(1 - h);
                    fa.side[v] = (uint8_t)(1 - h);
                    atomicOr(&mv[u >> 5], 1u << (u & 31));
                    moved += nwl[u];
                    deg = noffl[u + 1] - noffl[u];
                }
                int32_t incl = wave_incl_scan(deg) + dcarry;
                if (i < p) dpre[i + 1] = incl;
                dcarry = __shfl(incl, 63, 64);
            }
            moved = wave_sum(moved);
            if (lane == 0) {
                dpre[0] = 0;
                np_s = p;
                if (p > 0) {
                    w01[h] -= moved;
                    w01[1 - h] += moved;
                }
            }
        }
        __syncthreads();
        int32_t p = np_s;
        if (p == 0) {
            if (tid == 0 && !INIT) fa.stuck[s] = 1;
            break;
        }

        // mark the moved nodes' hyperedges, then update their pins' gains
        int32_t nwords = (ne + 31) >> 5;
        for (int32_t i = tid; i < nwords; i += kFuseThreads) work[i] = 0;
        __syncthreads();
        // one thread per incidence of a moved node; the thread that marks a
        // hyperedge first updates it (the moves are all made, so its counts
        // are final), large ones queued for a wavefront
        int32_t D = dpre[p];
        for (int32_t t = tid; t < D; t += kFuseThreads) {
            int32_t lo = 0, hi = p;  // dpre[lo] <= t < dpre[hi]
            while (hi - lo > 1) {
                int32_t mid = (lo + hi) >> 1;
                if (dpre[mid] <= t) lo = mid;
                else hi = mid;
            }
            int32_t u = (int32_t)(uint32_t)(mlist[lo] & 0xffffffffu) - a0;
            int32_t x = fa.inc[noffl[u] + (t - dpre[lo])] - e0;
            uint32_t bit = 1u << (x & 31);
            if (atomicOr(&work[x >> 5], bit) & bit) continue;
            int32_t e = e0 + x;
            if (fa.off[e + 1] - fa.off[e] > kFuseSmallDeg) {
                int32_t q = atomicAdd(&qn, 1);
                if (q < kFuseQueue) {
                    queue[q] = e;
                    continue;
                }
            }
            fuse_hedge(e, false, h, 0, 1, a0, fa, sd, mv, g);
        }
        __syncthreads();
        for (int32_t q = wv; q < min(qn, kFuseQueue); q += kFuseThreads / 64)
            fuse_hedge(queue[q], false, h, lane, 64, a0, fa, sd, mv, g);
        __syncthreads();
        // the move marks are spent
        for (int32_t i = tid; i < p; i += kFuseThreads) {
            int32_t u = (int32_t)(uint32_t)(mlist[i] & 0xffffffffu) - a0;
            atomicAnd(&mv[u >> 5], ~(1u << (u & 31)));
        }
        __syncthreads();
    }
    if (tid == 0) {
        fa.segw[2 * s] = (unsigned long long)w01[0];
        fa.segw[2 * s + 1] = (unsigned long long)w01[1];
        if (!INIT) fa.done[s] = 1;
        if (fa.rounds) atomicMax(fa.rounds, rounds);
    }
}

}  // namespace bp
