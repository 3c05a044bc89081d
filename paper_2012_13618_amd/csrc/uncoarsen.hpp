// Uncoarsening kernels with few launches per round (Algorithms 3-5).
//
// Gains (Algorithm 4) take two launches: a hyperedge pass computing what a pin
// on each side gains from its hyperedge (+w when alone on its side, -w when
// the hyperedge is uncut), and a node pass summing that over the node's
// hyperedges.  Each launch covers all degree buckets: virtual blocks
// [0, ns) take degree <= 8 (hyperedges) / <= 32 (nodes) one per thread, the
// next ones one listed item per wavefront, the last ones one per workgroup.
// The node pass also records, per list (one side of one segment), how many
// nodes are eligible and their largest and smallest gain.
//
// Selection of the first r nodes in (gain desc, id asc) order per list is an
// exact radix select over the pair (u, lid), u = max gain - gain (so ascending
// u = descending gain) and lid = node id within its segment: 12-bit digits,
// first over the significant bits of u (1 digit when the list's gains span
// < 4096 values), then over the bits of lid - each list follows its own digit
// schedule and stops as soon as the remaining count equals a bin's count.
// In balance rounds a list also stops at the bin holding its r-th key when
// the keys through that bin fit the candidate buffer: the balance finish
// orders what it gathers and keeps the first r.
// Each pass is one launch: blocks build their histograms and the workgroup
// that finishes last (atomic ticket) picks the digit of every list.
#pragma once
#include "level.hpp"
#include "refine.hpp"
#include "transpose.hpp"

namespace bp {

constexpr int kDigit = 12;
constexpr int kBins = 1 << kDigit;        // 4096
constexpr int kSelNodes = 1024;           // nodes per workgroup in histogram passes

__device__ __forceinline__ int bitlen_u32(uint32_t x) { return x ? 32 - __clz((int)x) : 0; }

// Per-hyperedge gain contributions (what a pin on side 0 / side 1 gains from
// the hyperedge: +w, -w or 0).  When every hyperedge weight of the level is
// below 2^15 (pk) the pair is stored as two 16-bit halves of one word, which
// halves the bytes of the node pass's random gathers; else as an int2.
__device__ __forceinline__ int2 cc_get(const void *cc, int pk, int32_t e)
{
    if (pk) {
        uint32_t v = ((const uint32_t *)cc)[e];
        return make_int2((int32_t)(int16_t)(v & 0xffffu), (int32_t)(int16_t)(v >> 16));
    }
    return ((const int2 *)cc)[e];
}
__device__ __forceinline__ void cc_put(void *cc, int pk, int32_t e, int2 c)
{
    if (pk) ((uint32_t *)cc)[e] = (uint32_t)(uint16_t)(int16_t)c.x | ((uint32_t)(uint16_t)(int16_t)c.y << 16);
    else ((int2 *)cc)[e] = c;
}

// ---- gains -------------------------------------------------------------------------

template <int S>
__device__ __forceinline__ void hedge_contrib_one(int32_t e, int lane, int stride, const int32_t *off,
                                                  const int32_t *pins, const int32_t *hw,
                                                  const int32_t *hseg, const uint8_t *gmask,
                                                  const uint8_t *side, void *cc, int pk, int32_t *lds)
{
    int32_t b = off[e], d = off[e + 1] - b;
    if (!thread_split<S>(d)) return;  // (eight pins' loads in flight at a time below)
    if (!gmask[hseg[e]]) return;
    int32_t n1 = 0;
    if (S == SMALL) {
        // eight pins at a time, straight-line loads (past the degree: the
        // last pin again) in flight together
        for (int32_t i0 = 0; i0 < d; i0 += 8) {
            int32_t u[8];
#pragma unroll
            for (int i = 0; i < 8; i++) u[i] = pins[b + min(i0 + i, d - 1)];
#pragma unroll
            for (int i = 0; i < 8; i++) {
                int32_t x = side[u[i]];
                if (i0 + i < d) n1 += x;
            }
        }
    } else {
#pragma unroll 4
        for (int i = lane; i < d; i += stride) n1 += side[pins[b + i]];
        n1 = group_sum<S>(n1, lds);
    }
    if (lane == 0) {
        int32_t w = hw[e], n0 = d - n1;
        int2 c;
        c.x = n0 == 1 ? w : (n0 == d ? -w : 0);
        c.y = n1 == 1 ? w : (n1 == d ? -w : 0);
        cc_put(cc, pk, e, c);
    }
}

__global__ __launch_bounds__(kBlock) void k_gain_hedges(int32_t E, const int32_t *lmid, int32_t nmid,
                                                        const int32_t *lbig, int32_t nbig,
                                                        const int32_t *off, const int32_t *pins,
                                                        const int32_t *hw, const int32_t *hseg,
                                                        const uint8_t *gmask, const uint8_t *side,
                                                        void *cc, int pk, const int32_t *go,
                                                        const int32_t *lnbig, const int32_t *ncount,
                                                        int32_t *gain, int32_t *big_done)
{
    __shared__ int32_t lds[16];
    if (go && *go == 0) return;
    // big nodes are summed chunk by chunk in the node pass: start them at 0
    int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t < ncount[1]) {
        gain[lnbig[t]] = 0;
        big_done[t] = 0;
    }
    int64_t ns = ceil_div(E, kBlock), nw = ceil_div(nmid, kBlock / 64);
    int64_t vb = blockIdx.x;
    if (vb < ns) {
        int64_t e = xcd_block(vb, ns) * kBlock + threadIdx.x;
        if (e < E) hedge_contrib_one<SMALL>((int32_t)e, 0, 1, off, pins, hw, hseg, gmask, side, cc, pk, lds);
    } else if (vb < ns + nw) {
        int64_t i = (vb - ns) * (kBlock / 64) + (threadIdx.x >> 6);
        if (i < nmid)
            hedge_contrib_one<WAVE>(lmid[i], threadIdx.x & 63, 64, off, pins, hw, hseg, gmask, side, cc, pk, lds);
    } else if (vb - ns - nw < nbig) {
        hedge_contrib_one<BLOCK>(lbig[vb - ns - nw], threadIdx.x, blockDim.x, off, pins, hw, hseg, gmask,
                                 side, cc, pk, lds);
    }
}

// ---- gains after a balance round: updated from what it moved -------------------------

// One wavefront per logged chunk of a moved node's incidences: marks each
// hyperedge in the bitmap.  The chunk's hyperedges ascend, so lanes sharing a
// bitmap word are adjacent and the first lane of each run sets the run's bits
// with one atomic (none when they are all set already).  Here: blocks b of nb
// (kBlock threads each) of the marking of the n logged chunks.
//
// It also settles the moved node's side change in its gain.  The gain update
// that follows treats every pin as unmoved (new contribution minus old, both
// for the pin's side now); a node that moved from side o to side s had gained
// the old contribution for o, so it is owed old[s] - old[o] per hyperedge,
// added here while the contributions are still the old ones.  That way the
// update reads one side byte per pin and no move flags.
__device__ __forceinline__ void log_hedges_blocks(int64_t b, int64_t nb, int32_t n, const int32_t *cnode,
                                                  const int32_t *cbeg, const int32_t *noff, const int32_t *inc,
                                                  uint32_t *bits, const void *cc, int pk, const uint8_t *side,
                                                  int32_t *gain)
{
    int lane = threadIdx.x & 63;
    const int64_t wpb = kBlock / 64;
    for (int64_t i = b * wpb + (threadIdx.x >> 6); i < n; i += nb * wpb) {
        int32_t v = cnode[i];
        int32_t j = cbeg[i] + lane, end = noff[v + 1];
        bool valid = j < end;
        int32_t e = valid ? inc[j] : 0;
        int sv = side[v];
        int32_t corr = 0;
        if (valid) {
            int2 oc = cc_get(cc, pk, e);
            corr = sv ? oc.y - oc.x : oc.x - oc.y;
        }
        corr = wave_sum(corr);
        if (lane == 0 && corr) atomicAdd(&gain[v], corr);
        int32_t w = valid ? (e >> 5) : -1;
        uint32_t bit = valid ? 1u << (e & 31) : 0u;
        int32_t pw = __shfl_up(w, 1, 64);
        bool head = valid && (lane == 0 || pw != w);
        unsigned long long heads = __ballot(head);
        int lead = 63 - __clzll((long long)(heads & ((2ull << lane) - 1ull)));
        uint32_t run = bit;
#pragma unroll
        for (int o = 1; o < 64; o <<= 1) {
            uint32_t t = __shfl_down(run, o, 64);
            int tl = __shfl_down(lead, o, 64);
            if (lane + o < 64 && tl == lead) run |= t;
        }
        if (head) {
            uint32_t old = __hip_atomic_load(&bits[w], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            if ((old & run) != run) atomicOr(&bits[w], run);
        }
    }
}

__device__ __forceinline__ int2 hedge_contrib_value(int32_t w, int32_t d, int32_t n1)
{
    int32_t n0 = d - n1;
    int2 c;
    c.x = n0 == 1 ? w : (n0 == d ? -w : 0);
    c.y = n1 == 1 ? w : (n1 == d ? -w : 0);
    return c;
}

constexpr int kUpdSlots = 1024;  // big nodes whose gain changes gather in LDS first

// adds delta to gain[u]: in the workgroup's LDS slot when u is one of the
// first kUpdSlots big nodes (many hyperedges, so many updates), else globally
__device__ __forceinline__ void add_gain(int32_t u, int32_t delta, const int32_t *bigslot, int32_t *slot,
                                        int32_t *gain)
{
    int32_t k = bigslot[u];
    if (k >= 0 && k < kUpdSlots) atomicAdd(&slot[k], delta);
    else atomicAdd(&gain[u], delta);
}

constexpr int kUpdWords = 64;                // bitmap words a workgroup sweeps per step
constexpr int kUpdChunk = 8;                 // ... as 8 chunks of this many words
constexpr int kUpdQueue = kUpdWords * 32;  // hyperedges those words can hold
constexpr int kUpdWaveMax = 512;           // larger marked hyperedges: the whole workgroup
constexpr int kUpdHugeRegs = 8;            // ... whose pins fit kUpdHugeRegs a thread in registers

// recount of hyperedge e (pins b .. b + d, d <= kSmallMax) after a round:
// its new contribution, with each pin's gain change added
__device__ __forceinline__ int2 recount_small(int32_t e, int32_t b, int32_t d, const int32_t *pins,
                                              const int32_t *hw, const uint8_t *side, int2 oc,
                                              const int32_t *bigslot, int32_t *slot, int32_t *gain)
{
    // straight-line loads (past the degree: pin 0 again), so that they fly together
    int32_t u[kSmallMax];
    uint32_t sn[kSmallMax];
    int32_t n1 = 0;
#pragma unroll
    for (int j = 0; j < kSmallMax; j++) u[j] = pins[b + (j < d ? j : 0)];
#pragma unroll
    for (int j = 0; j < kSmallMax; j++) sn[j] = side[u[j]];
#pragma unroll
    for (int j = 0; j < kSmallMax; j++)
        if (j < d) n1 += sn[j];
    int2 nc = hedge_contrib_value(hw[e], d, n1);
#pragma unroll
    for (int j = 0; j < kSmallMax; j++)
        if (j < d) {
            int32_t delta = sn[j] ? nc.y - oc.y : nc.x - oc.x;
            if (delta) add_gain(u[j], delta, bigslot, slot, gain);
        }
    return nc;
}

// The same for 9..kHedgeThreadMax pins by one thread, eight pins' loads in
// flight at a time; the pins are read again (from cache) for the deltas, unless
// the contribution did not change, when no pin's gain does.
__device__ __forceinline__ int2 recount_thread(int32_t e, int32_t b, int32_t d, const int32_t *pins,
                                               const int32_t *hw, const uint8_t *side, int2 oc,
                                               const int32_t *bigslot, int32_t *slot, int32_t *gain)
{
    int32_t n1 = 0;
    for (int32_t i0 = 0; i0 < d; i0 += 8) {
        int32_t u[8];
#pragma unroll
        for (int j = 0; j < 8; j++) u[j] = pins[b + min(i0 + j, d - 1)];
#pragma unroll
        for (int j = 0; j < 8; j++) {
            int32_t x = side[u[j]];
            if (i0 + j < d) n1 += x;
        }
    }
    int2 nc = hedge_contrib_value(hw[e], d, n1);
    if (nc.x == oc.x && nc.y == oc.y) return nc;
    for (int32_t i0 = 0; i0 < d; i0 += 8) {
        int32_t u[8];
        uint32_t sn[8];
#pragma unroll
        for (int j = 0; j < 8; j++) u[j] = pins[b + min(i0 + j, d - 1)];
#pragma unroll
        for (int j = 0; j < 8; j++) sn[j] = side[u[j]];
#pragma unroll
        for (int j = 0; j < 8; j++)
            if (i0 + j < d) {
                int32_t delta = sn[j] ? nc.y - oc.y : nc.x - oc.x;
                if (delta) add_gain(u[j], delta, bigslot, slot, gain);
            }
    }
    return nc;
}

// Marked hyperedges, found by sweeping the bitmap: recount the sides, replace
// the contribution, and add the change to every pin's gain, as if no pin had
// moved (the marking launch has already settled what the moved nodes are
// owed for changing sides).  Integer sums, so the result equals a
// recomputation.  The sweep clears the bitmap.
//
// The bitmap is dealt out in chunks of 8 words (256 hyperedges, in id order),
// chunk c to workgroup c mod G: a moved node's hyperedges crowd into a few
// chunks (ids follow locality), and consecutive chunks go to different
// workgroups.  Each step a workgroup takes 8 of its chunks; one wavefront
// lists their marked hyperedges in LDS (popcount scan), then degree <= 32 go
// one per thread, up to 512 one per wavefront, larger ones to the whole
// workgroup.  When abytes is set (profiling), adds the algorithmic bytes it
// moved: 4 per bitmap word, per hyperedge 12 (offsets, weight) plus the
// contribution in and out, 9 per pin (id, side, gain).
__global__ __launch_bounds__(kBlock) void k_gain_update(int64_t nwords, uint32_t *bits, const int32_t *off,
                                                        const int32_t *pins, const int32_t *hw,
                                                        const uint8_t *side, void *cc, int pk,
                                                        int32_t *gain, const int32_t *bigslot,
                                                        const int32_t *lnbig, const int32_t *ncount,
                                                        const int32_t *go, int32_t *logcount,
                                                        unsigned long long *abytes)
{
    __shared__ int32_t slot[kUpdSlots];
    __shared__ int32_t queue[kUpdQueue], bigq[kUpdQueue];  // bigq: wavefront ones from the front, workgroup ones from the back
    __shared__ int32_t nq, nbq, nhq, npins;
    __shared__ int32_t lds[16];
    const int32_t gv = go ? *go : 1, nbig = ncount[1];  // loaded together
    if (gv == 0) return;
    // the move log was read by the previous launch: empty it for this round's moves
    if (logcount && blockIdx.x == 0 && threadIdx.x == 0) *logcount = 0;
    int32_t nb = min(nbig, kUpdSlots);
    for (int i = threadIdx.x; i < nb; i += blockDim.x) slot[i] = 0;
    int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int64_t G = gridDim.x;
    int64_t words_done = 0, hedges_done = 0, pins_done = 0;  // thread 0's tally (profiling)
    for (int64_t step = 0; step * 8 * G * kUpdChunk < nwords; step++) {
        if (wv == 0) {
            int64_t chunk = step * 8 * G + (lane / kUpdChunk) * G + blockIdx.x;
            int64_t wi = chunk * kUpdChunk + (lane % kUpdChunk);
            uint32_t word = wi < nwords ? bits[wi] : 0u;
            if (word) bits[wi] = 0;
            int32_t c = __popc(word);
            int32_t at = wave_incl_scan(c) - c;
            while (word) {
                int k = __ffs((int)word) - 1;
                word &= word - 1;
                queue[at++] = (int32_t)(wi * 32 + k);
            }
            if (lane == 63) nq = at;
            if (lane == 0) {
                nbq = 0;
                nhq = 0;
                npins = 0;
            }
        }
        __syncthreads();
        int32_t n = nq;
        for (int32_t q = threadIdx.x; q < n; q += blockDim.x) {
            int32_t e = queue[q];
            int32_t b = off[e], d = off[e + 1] - b;
            if (abytes) atomicAdd(&npins, d);
            if (d <= kSmallMax)
                cc_put(cc, pk, e, recount_small(e, b, d, pins, hw, side, cc_get(cc, pk, e), bigslot, slot, gain));
            else if (d <= kHedgeThreadMax)
                cc_put(cc, pk, e, recount_thread(e, b, d, pins, hw, side, cc_get(cc, pk, e), bigslot, slot, gain));
            else if (d <= kUpdWaveMax) bigq[atomicAdd(&nbq, 1)] = e;
            else bigq[kUpdQueue - 1 - atomicAdd(&nhq, 1)] = e;  // front and back never meet
        }
        __syncthreads();
        int32_t nbig = nbq, nhuge = nhq;
        for (int32_t q = wv; q < nbig; q += blockDim.x >> 6) {
            int32_t e = bigq[q];
            int32_t b = off[e], d = off[e + 1] - b;
            int32_t w = hw[e];
            int2 oc = cc_get(cc, pk, e);
            // up to kUpdWaveMax / 64 pins a lane, held in registers: their ids,
            // then their sides, each group of loads in flight together, and
            // used by both the count and the deltas
            constexpr int kR = kUpdWaveMax / 64;
            int32_t u[kR];
            uint32_t sn[kR];
#pragma unroll
            for (int k = 0; k < kR; k++) u[k] = pins[b + min(lane + 64 * k, d - 1)];
#pragma unroll
            for (int k = 0; k < kR; k++) sn[k] = side[u[k]];
            int32_t n1 = 0;
#pragma unroll
            for (int k = 0; k < kR; k++)
                if (lane + 64 * k < d) n1 += sn[k];
            n1 = wave_sum(n1);
            int2 nc = hedge_contrib_value(w, d, n1);
#pragma unroll
            for (int k = 0; k < kR; k++) {
                if (lane + 64 * k >= d) continue;
                int32_t delta = sn[k] ? nc.y - oc.y : nc.x - oc.x;
                if (delta) add_gain(u[k], delta, bigslot, slot, gain);
            }
            if (lane == 0) cc_put(cc, pk, e, nc);
        }
        // the largest ones by the whole workgroup, one after another
        for (int32_t q = 0; q < nhuge; q++) {
            int32_t e = bigq[kUpdQueue - 1 - q];
            int32_t b = off[e], d = off[e + 1] - b;
            int2 oc = cc_get(cc, pk, e);
            int32_t w = hw[e];
            if (d <= kUpdHugeRegs * kBlock) {
                // up to kUpdHugeRegs pins a thread in registers (loaded once, in
                // flight together) for both the count and the deltas
                int32_t u[kUpdHugeRegs];
                uint32_t sn[kUpdHugeRegs];
#pragma unroll
                for (int k = 0; k < kUpdHugeRegs; k++) u[k] = pins[b + min((int32_t)threadIdx.x + kBlock * k, d - 1)];
#pragma unroll
                for (int k = 0; k < kUpdHugeRegs; k++) sn[k] = side[u[k]];
                int32_t n1 = 0;
#pragma unroll
                for (int k = 0; k < kUpdHugeRegs; k++)
                    if ((int32_t)threadIdx.x + kBlock * k < d) n1 += sn[k];
                n1 = block_sum(n1, lds);
                int2 nc = hedge_contrib_value(w, d, n1);
#pragma unroll
                for (int k = 0; k < kUpdHugeRegs; k++) {
                    if ((int32_t)threadIdx.x + kBlock * k >= d) continue;
                    int32_t delta = sn[k] ? nc.y - oc.y : nc.x - oc.x;
                    if (delta) add_gain(u[k], delta, bigslot, slot, gain);
                }
                __syncthreads();  // every thread has read the old contribution
                if (threadIdx.x == 0) cc_put(cc, pk, e, nc);
                continue;
            }
            int32_t n1 = 0;
#pragma unroll 4
            for (int j = threadIdx.x; j < d; j += blockDim.x) n1 += side[pins[b + j]];
            n1 = block_sum(n1, lds);
            int2 nc = hedge_contrib_value(w, d, n1);
#pragma unroll 4
            for (int j = threadIdx.x; j < d; j += blockDim.x) {
                int32_t u = pins[b + j];
                int sn = side[u];
                int32_t delta = sn ? nc.y - oc.y : nc.x - oc.x;
                if (delta) add_gain(u, delta, bigslot, slot, gain);
            }
            __syncthreads();  // every thread has read the old contribution
            if (threadIdx.x == 0) cc_put(cc, pk, e, nc);
        }
        __syncthreads();
        if (threadIdx.x == 0) {
            words_done += 64;
            hedges_done += n;
            pins_done += npins;
        }
    }
    __syncthreads();
    for (int i = threadIdx.x; i < nb; i += blockDim.x)
        if (slot[i]) atomicAdd(&gain[lnbig[i]], slot[i]);
    if (abytes && threadIdx.x == 0 && words_done)
        atomicAdd(abytes, (unsigned long long)(4 * words_done + (pk ? 20 : 28) * hedges_done + 9 * pins_done));
}

// eligibility of a node for its list under the segment's selection mode
__device__ __forceinline__ bool sel_list(int32_t s, int sd, int32_t g, const uint8_t *mode)
{
    uint8_t md = mode[s];
    if (!((md >> sd) & 1)) return false;
    return !((md & kGainNonNeg) && g < 0);
}

template <int S>
__device__ __forceinline__ void node_gain_one(int32_t v, int lane, int stride, const int32_t *noff,
                                              const int32_t *inc, const int32_t *nseg,
                                              const uint8_t *gmask, const uint8_t *side,
                                              const void *cc, int pk, int32_t *gain, int32_t *lds,
                                              const uint8_t *mode, int32_t *tot, int32_t *gmax,
                                              int32_t *gmin, bool stats)
{
    int32_t b = noff[v], d = noff[v + 1] - b;
    if (S == SMALL && d > kNodeSmallMax) return;
    int32_t s = nseg[v];
    if (!gmask[s]) return;
    int sd = side[v];
    int32_t g = 0;
    if (S == SMALL) {
        // eight incidences at a time, straight-line loads (past the degree: the
        // last incidence again), in flight together
        for (int i0 = 0; i0 < d; i0 += 8) {
            int32_t e8[8];
#pragma unroll
            for (int k = 0; k < 8; k++) e8[k] = inc[b + min(i0 + k, d - 1)];
#pragma unroll
            for (int k = 0; k < 8; k++) {
                int2 c = cc_get(cc, pk, e8[k]);
                if (i0 + k < d) g += sd ? c.y : c.x;
            }
        }
    } else {
#pragma unroll 4
        for (int i = lane; i < d; i += stride) {
            int2 c = cc_get(cc, pk, inc[b + i]);
            g += sd ? c.y : c.x;
        }
    }
    g = group_sum<S>(g, lds);
    if (lane == 0) {
        gain[v] = g;
        if (stats && sel_list(s, sd, g, mode)) {
            int32_t c = 2 * s + sd;
            atomicAdd(&tot[c], 1);
            atomicMax(&gmax[c], g);
            atomicMin(&gmin[c], g);
        }
    }
}

// Node pass.  Besides gain[v], per-list counts and gain extremes for the
// selection that follows (block-aggregated when a block is in one segment).
__global__ __launch_bounds__(kBlock) void k_gain_nodes(int32_t N, const int32_t *lnmid,
                                                       const int32_t *lnbig, const int32_t *ncount,
                                                       const int32_t *noff, const int32_t *inc,
                                                       const int32_t *nseg, const uint8_t *gmask,
                                                       const uint8_t *side, const void *cc, int pk,
                                                       int32_t *gain, const uint8_t *mode,
                                                       int32_t *tot, int32_t *gmax, int32_t *gmin,
                                                       const int32_t *go, const int32_t *chunk_node,
                                                       const int32_t *chunk_beg,
                                                       const int32_t *chunk_big,
                                                       const int32_t *big_chunks, int32_t *big_done,
                                                       int32_t S, int32_t nw)
{
    __shared__ int32_t lds[16];
    __shared__ int32_t at[kAggLists], amax[kAggLists], amin[kAggLists];
    if (go && *go == 0) return;
    bool stats = tot != nullptr;
    int32_t cm = ncount[0], ck = ncount[2];
    int64_t ns = reduce_grid(N);
    int64_t vb = blockIdx.x;
    if (vb < ns) {
        // nodes of degree <= 32, one per thread, over a contiguous chunk
        int64_t lo, hi;
        reduce_chunk(N, ns, xcd_block(vb, ns), lo, hi);
        if (lo >= hi) return;
        int32_t c0 = 2 * nseg[lo], nl = 2 * nseg[hi - 1] + 2 - c0;
        bool local = nl <= kAggLists;
        for (int i = threadIdx.x; i < kAggLists; i += blockDim.x) {
            at[i] = 0;
            amax[i] = INT32_MIN;
            amin[i] = INT32_MAX;
        }
        __syncthreads();
        for (int64_t v = lo + threadIdx.x; v < hi; v += blockDim.x) {
            int32_t b = noff[v], d = noff[v + 1] - b;
            int32_t s = nseg[v];
            if (d > kNodeSmallMax || !gmask[s]) continue;
            int sd = side[v];
            int32_t g = 0;
            // eight incidences at a time, straight-line loads in flight together
            for (int i0 = 0; i0 < d; i0 += 8) {
                int32_t e8[8];
#pragma unroll
                for (int k = 0; k < 8; k++) e8[k] = inc[b + min(i0 + k, d - 1)];
#pragma unroll
                for (int k = 0; k < 8; k++) {
                    int2 c = cc_get(cc, pk, e8[k]);
                    if (i0 + k < d) g += sd ? c.y : c.x;
                }
            }
            gain[v] = g;
            if (!stats || !sel_list(s, sd, g, mode)) continue;
            int32_t c = 2 * s + sd;
            if (local) {
                atomicAdd(&at[c - c0], 1);
                atomicMax(&amax[c - c0], g);
                atomicMin(&amin[c - c0], g);
            } else {
                atomicAdd(&tot[c], 1);
                atomicMax(&gmax[c], g);
                atomicMin(&gmin[c], g);
            }
        }
        __syncthreads();
        if (stats && local)
            for (int i = threadIdx.x; i < nl; i += blockDim.x)
                if (at[i]) {
                    atomicAdd(&tot[c0 + i], at[i]);
                    atomicMax(&gmax[c0 + i], amax[i]);
                    atomicMin(&gmin[c0 + i], amin[i]);
                }
    } else if (vb < ns + nw) {
        // nodes of degree 33..2048, one per wavefront, nw workgroups striding
        // over the list; with few segments the lists aggregate in LDS
        bool local = 2 * S <= kAggLists;
        for (int i = threadIdx.x; i < kAggLists; i += blockDim.x) {
            at[i] = 0;
            amax[i] = INT32_MIN;
            amin[i] = INT32_MAX;
        }
        __syncthreads();
        int lane = threadIdx.x & 63;
        for (int64_t i = (vb - ns) * (kBlock / 64) + (threadIdx.x >> 6); i < cm; i += (int64_t)nw * (kBlock / 64)) {
            int32_t v = lnmid[i];
            int32_t s = nseg[v];
            if (!gmask[s]) continue;
            int32_t b = noff[v], d = noff[v + 1] - b;
            int sd = side[v];
            int32_t g = 0;
#pragma unroll 4
            for (int j = lane; j < d; j += 64) {
                int2 c = cc_get(cc, pk, inc[b + j]);
                g += sd ? c.y : c.x;
            }
            g = wave_sum(g);
            if (lane != 0) continue;
            gain[v] = g;
            if (!stats || !sel_list(s, sd, g, mode)) continue;
            int32_t c = 2 * s + sd;
            if (local) {
                atomicAdd(&at[c], 1);
                atomicMax(&amax[c], g);
                atomicMin(&amin[c], g);
            } else {
                atomicAdd(&tot[c], 1);
                atomicMax(&gmax[c], g);
                atomicMin(&gmin[c], g);
            }
        }
        __syncthreads();
        if (stats && local)
            for (int i = threadIdx.x; i < 2 * S; i += blockDim.x)
                if (at[i]) {
                    atomicAdd(&tot[i], at[i]);
                    atomicMax(&gmax[i], amax[i]);
                    atomicMin(&gmin[i], amin[i]);
                }
    } else if (vb - ns - nw < ck) {
        // one chunk of a big node: partial sum, then the last chunk of the
        // node records its statistics
        int32_t q = (int32_t)(vb - ns - nw);
        int32_t v = chunk_node[q];
        int32_t s = nseg[v];
        if (!gmask[s]) return;
        int sd = side[v];
        int32_t b = chunk_beg[q], e = min(b + kNodeChunk, noff[v + 1]);
        int32_t g = 0;
        for (int32_t i = b + threadIdx.x; i < e; i += blockDim.x) {
            int2 c = cc_get(cc, pk, inc[i]);
            g += sd ? c.y : c.x;
        }
        g = block_sum(g, lds);
        if (threadIdx.x == 0) {
            atomicAdd(&gain[v], g);
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
            int32_t bi = chunk_big[q];
            if (atomicAdd(&big_done[bi], 1) == big_chunks[bi] - 1) {
                __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
                int32_t gv = __hip_atomic_load(&gain[v], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                if (stats && sel_list(s, sd, gv, mode)) {
                    int32_t c = 2 * s + sd;
                    atomicAdd(&tot[c], 1);
                    atomicMax(&gmax[c], gv);
                    atomicMin(&gmin[c], gv);
                }
            }
        }
    }
}

// Per-list counts and gain extremes after a gain update (what the node pass
// records otherwise); clears the move marks and the hyperedge list.  Chunked:
// the lists of a chunk aggregate in LDS and end in one atomic each.
__global__ __launch_bounds__(kBlock) void k_gain_stats(int32_t N, const int32_t *nseg, const uint8_t *gmask,
                                                       const uint8_t *side, const int32_t *gain,
                                                       const uint8_t *mode, int32_t *tot, int32_t *gmax,
                                                       int32_t *gmin, int32_t *counts,
                                                       const int32_t *go)
{
    __shared__ int32_t at[kAggLists], amax[kAggLists], amin[kAggLists];
    if (go && *go == 0) return;
    if (blockIdx.x == 0 && threadIdx.x == 0) counts[0] = 0;
    int64_t lo, hi;
    reduce_chunk(N, gridDim.x, blockIdx.x, lo, hi);
    if (lo >= hi) return;
    int32_t c0 = 2 * nseg[lo], nl = 2 * nseg[hi - 1] + 2 - c0;
    bool local = nl <= kAggLists;
    for (int i = threadIdx.x; i < kAggLists; i += blockDim.x) {
        at[i] = 0;
        amax[i] = INT32_MIN;
        amin[i] = INT32_MAX;
    }
    __syncthreads();
    for (int64_t v = lo + threadIdx.x; v < hi; v += blockDim.x) {
        int32_t s = nseg[v];
        if (!gmask[s]) continue;
        int sd = side[v];
        int32_t g = gain[v];
        if (!sel_list(s, sd, g, mode)) continue;
        int32_t c = 2 * s + sd;
        if (local) {
            atomicAdd(&at[c - c0], 1);
            atomicMax(&amax[c - c0], g);
            atomicMin(&amin[c - c0], g);
        } else {
            atomicAdd(&tot[c], 1);
            atomicMax(&gmax[c], g);
            atomicMin(&gmin[c], g);
        }
    }
    __syncthreads();
    if (local)
        for (int i = threadIdx.x; i < nl; i += blockDim.x)
            if (at[i]) {
                atomicAdd(&tot[c0 + i], at[i]);
                atomicMax(&gmax[c0 + i], amax[i]);
                atomicMin(&gmin[c0 + i], amin[i]);
            }
}

// ---- radix select ----------------------------------------------------------------------

struct SelView {
    const int32_t *gain, *nseg, *nbase;
    const uint8_t *side, *mode;
    const int32_t *m;
    int idbits;  // bits of the largest local node id of the level
};

// Selection key of a node in its list: u = gmax - gain (ascending u is
// descending gain) above the node's local id, so ascending keys are the
// (gain desc, id asc) order and every key of a list is distinct.
__device__ __forceinline__ uint64_t sel_key(int32_t gmax, int32_t g, uint32_t lid, int idbits)
{
    return ((uint64_t)(uint32_t)((int64_t)gmax - g) << idbits) | lid;
}

// Width in bits of a list's keys, from its gain extremes.
__device__ __forceinline__ int sel_kbits(int32_t gmax, int32_t gmin, int idbits)
{
    return bitlen_u32((uint32_t)((int64_t)gmax - gmin)) + idbits;
}

// Digit (12 bits, from the top of the T-bit key) of key k at pass p, or -1
// when k does not carry the prefix fixed by the earlier passes.
__device__ __forceinline__ int sel_digit_k(uint64_t k, int T, int p, uint64_t pre)
{
    int hi = T - kDigit * p;
    if (hi <= 0) return (p == 0 && T == 0) ? 0 : -1;  // a 0-bit key: one bin
    int lo = hi - kDigit > 0 ? hi - kDigit : 0;
    if (p > 0 && hi < 64 && ((k ^ pre) >> hi) != 0) return -1;
    return (int)((k >> lo) & ((1ull << (hi - lo)) - 1ull));
}

// Pick of list c after pass p: the digit holding the rem-th key.  One
// workgroup.  Clears the bins it read.  clip > 0 (balance rounds): the list
// may also stop at a whole bin once the keys up to its end are at most clip;
// the balance finish then orders them and keeps the first rsel.
__device__ void sel_pick_list(const SelState &st, int32_t c, int p, int idbits, const uint8_t *mode,
                              const int32_t *m, int64_t *lds, int32_t clip)
{
    __shared__ int sbin;
    __shared__ int32_t sbefore, sin_;
    uint32_t *hc = st.hist + (int64_t)c * kBins;
    if (p == 0) {
        // the number to choose: Algorithm 5 takes min(|L0|, |L1|) from both
        // lists, Algorithm 3 and the balance step at most ceil(sqrt n)
        if (threadIdx.x == 0) {
            int32_t s = c >> 1, sd = c & 1;
            uint8_t md = mode[s];
            int64_t r = 0;
            if ((md >> sd) & 1) {
                int64_t t = st.tot[c];
                if (md & kMinPair) {
                    int64_t o = st.tot[c ^ 1];
                    r = t < o ? t : o;
                } else {
                    r = t < (int64_t)m[s] ? t : (int64_t)m[s];
                }
            }
            st.rsel[c] = (int32_t)r;
            st.rem[c] = (int32_t)r;
            st.kpre[c] = 0;
            bool whole = r > 0 && r == st.tot[c];  // the whole list: no digit needed
            st.kthr[c] = whole ? ~0ull : 0ull;
            st.kbits[c] = r > 0 ? sel_kbits(st.gmax[c], st.gmin[c], idbits) : 0;
            st.done[c] = r == 0 || whole;
            if (r == 0 || whole) atomicSub(&st.ctl[0], 1);
        }
        __syncthreads();
    }
    int per = kBins / kBlock;
    if (st.done[c]) {
        // nothing to choose: still clear what pass 0 counted for this list
        if (p == 0)
            for (int j = 0; j < per; j++) hc[threadIdx.x * per + j] = 0;
        __syncthreads();
        return;
    }
    int32_t r = st.rem[c];
    int64_t loc = 0;
    for (int j = 0; j < per; j++) loc += hc[threadIdx.x * per + j];
    int64_t tot;
    int64_t ex = block_excl_scan(loc, lds, &tot);
    if (threadIdx.x == 0) sbin = -1;
    __syncthreads();
    if (ex < r && r <= ex + loc) {
        int64_t acc = ex;
        for (int j = 0; j < per; j++) {
            int64_t x = hc[threadIdx.x * per + j];
            if (acc + x >= r) {
                sbin = threadIdx.x * per + j;
                sbefore = (int32_t)acc;
                sin_ = (int32_t)x;
                break;
            }
            acc += x;
        }
    }
    __syncthreads();
    for (int j = 0; j < per; j++) hc[threadIdx.x * per + j] = 0;
    if (threadIdx.x == 0 && sbin >= 0) {
        int T = st.kbits[c];
        int hi = T - kDigit * p, lo = hi - kDigit > 0 ? hi - kDigit : 0;
        int32_t left = r - sbefore;
        uint64_t pre = st.kpre[c] | ((uint64_t)sbin << lo);
        st.kpre[c] = pre;
        st.rem[c] = left;
        // done when the whole bin is taken or the bin is a single key, or
        // (clip) when the keys through the end of the bin fit the finish
        if (left == sin_ || lo == 0 || (clip > 0 && (int64_t)st.rsel[c] - left + sin_ <= clip)) {
            st.kthr[c] = pre | (lo ? ((1ull << lo) - 1ull) : 0ull);
            st.done[c] = 1;
            atomicSub(&st.ctl[0], 1);
        }
    }
    __syncthreads();
}

// A list of a segment without nodes chooses nothing.
__device__ __forceinline__ void empty_segment_done(const SelState &st, int32_t s)
{
    for (int sd = 0; sd < 2; sd++) {
        int32_t c = 2 * s + sd;
        st.rsel[c] = 0;
        st.rem[c] = 0;
        st.done[c] = 1;
        atomicSub(&st.ctl[0], 1);
    }
}

// Per-segment tickets: every workgroup whose node range meets segment s
// counts itself in tick[s] after its histogram is flushed; the last one does
// the picks of the segment's two lists.  Segments without nodes are settled
// in pass 0 by the workgroup holding their position.
__device__ void seg_tickets_pick(int32_t N, int p, int32_t nlists, int idbits, const SelView &sv,
                                 const SelState &st, int64_t v0, int64_t *lds, int32_t clip)
{
    __shared__ int32_t picks[kBlock];
    __shared__ int npick;
    int64_t v1 = v0 + kSelNodes < N ? v0 + kSelNodes : N;
    int32_t S = nlists / 2;
    if (p == 0) {
        for (int64_t v = v0 + threadIdx.x; v < v1; v += blockDim.x) {
            int32_t lo = v == 0 ? -1 : sv.nseg[v - 1], hi = sv.nseg[v];
            for (int32_t s = lo + 1; s < hi; s++) empty_segment_done(st, s);
        }
        if (v1 == N)
            for (int32_t s = sv.nseg[N - 1] + 1 + (int32_t)threadIdx.x; s < S; s += blockDim.x)
                empty_segment_done(st, s);
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
        npick = 0;
    }
    __syncthreads();
    int32_t sf = sv.nseg[v0], sl = sv.nseg[v1 - 1];
    for (int32_t base = sf; base <= sl; base += blockDim.x) {
        int32_t s = base + (int32_t)threadIdx.x;
        if (s <= sl) {
            int32_t a = sv.nbase[s], b = sv.nbase[s + 1];
            if (b > a) {
                int32_t nb = (b - 1) / kSelNodes - a / kSelNodes + 1;
                if (atomicAdd(&st.tick[s], 1) == nb - 1) {
                    st.tick[s] = 0;
                    picks[atomicAdd(&npick, 1)] = s;
                }
            }
        }
        __syncthreads();
        int np = npick;
        if (np > 0) {
            if (threadIdx.x == 0) __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
            __syncthreads();
            for (int i = 0; i < np; i++) {
                sel_pick_list(st, 2 * picks[i], p, idbits, sv.mode, sv.m, lds, clip);
                sel_pick_list(st, 2 * picks[i] + 1, p, idbits, sv.mode, sv.m, lds, clip);
            }
        }
        __syncthreads();
        if (threadIdx.x == 0) npick = 0;
        __syncthreads();
    }
}

// Histogram of global pass p; the last workgroup to finish does the picks
// when there are few lists, the last one of each segment when there are many.
__global__ __launch_bounds__(kBlock) void k_select_pass(int32_t N, int p, int32_t nlists, int idbits,
                                                        SelView sv, SelState st, int fused,
                                                        const int32_t *go, int32_t clip)
{
    __shared__ uint32_t h[2 * kBins];
    __shared__ int64_t lds[16];
    __shared__ int last;
    const int32_t gv = go ? *go : 1, ctl = st.ctl[0];  // loaded together
    if (gv == 0) return;
    if (p > 0 && ctl <= 0) return;
    int64_t v0 = (int64_t)blockIdx.x * kSelNodes;
    if (v0 < N) {
        int64_t v1 = v0 + kSelNodes < N ? v0 + kSelNodes : N;
        int32_t cbase = 2 * sv.nseg[v0];
        bool use_lds = 2 * sv.nseg[v1 - 1] + 1 - cbase < 2;
        if (use_lds) {
            for (int i = threadIdx.x; i < 2 * kBins; i += blockDim.x) h[i] = 0;
            __syncthreads();
            // one segment: its two lists' state once per workgroup, then only
            // each node's side and gain
            int32_t s = cbase / 2, nb0 = sv.nbase[s];
            uint8_t md = sv.mode[s];
            bool on0 = md & 1, on1 = (md >> 1) & 1;
            if (p > 0) {
                on0 = on0 && !st.done[cbase];
                on1 = on1 && !st.done[cbase + 1];
            } else {  // a list taken whole needs no histogram
                int64_t t0 = st.tot[cbase], t1 = st.tot[cbase + 1], ms = sv.m[s];
                bool pair = md & kMinPair;
                on0 = on0 && (pair ? min(t0, t1) : min(t0, ms)) != t0;
                on1 = on1 && (pair ? min(t1, t0) : min(t1, ms)) != t1;
            }
            int32_t gx0 = st.gmax[cbase], gx1 = st.gmax[cbase + 1];
            int T0 = p == 0 ? sel_kbits(gx0, st.gmin[cbase], idbits) : st.kbits[cbase];
            int T1 = p == 0 ? sel_kbits(gx1, st.gmin[cbase + 1], idbits) : st.kbits[cbase + 1];
            uint64_t pr0 = p == 0 ? 0ull : st.kpre[cbase], pr1 = p == 0 ? 0ull : st.kpre[cbase + 1];
            bool nonneg = md & kGainNonNeg;
            if (on0 || on1) {
#pragma unroll 4
                for (int64_t v = v0 + threadIdx.x; v < v1; v += blockDim.x) {
                    int sd = sv.side[v];
                    int32_t g = sv.gain[v];
                    if (!(sd ? on1 : on0) || (nonneg && g < 0)) continue;
                    uint64_t k = sel_key(sd ? gx1 : gx0, g, (uint32_t)(v - nb0), idbits);
                    int dig = sel_digit_k(k, sd ? T1 : T0, p, sd ? pr1 : pr0);
                    if (dig >= 0) atomicAdd(&h[sd * kBins + dig], 1u);
                }
            }
        }
        for (int64_t v = v0 + threadIdx.x; !use_lds && v < v1; v += blockDim.x) {
            int32_t s = sv.nseg[v];
            int sd = sv.side[v];
            int32_t g = sv.gain[v];
            if (!sel_list(s, sd, g, sv.mode)) continue;
            int32_t c = 2 * s + sd;
            if (p > 0 && st.done[c]) continue;
            if (p == 0) {  // a list taken whole needs no histogram
                int64_t t = st.tot[c];
                int64_t r = (sv.mode[s] & kMinPair) ? min(t, (int64_t)st.tot[c ^ 1]) : min(t, (int64_t)sv.m[s]);
                if (r == t) continue;
            }
            uint64_t k = sel_key(st.gmax[c], g, (uint32_t)(v - sv.nbase[s]), idbits);
            // pass 0 runs before the pick has fixed the key width: from the
            // extremes the node pass recorded
            int T = p == 0 ? sel_kbits(st.gmax[c], st.gmin[c], idbits) : st.kbits[c];
            int dig = sel_digit_k(k, T, p, p == 0 ? 0ull : st.kpre[c]);
            if (dig < 0) continue;
            atomicAdd(&st.hist[(int64_t)c * kBins + dig], 1u);
        }
        if (use_lds) {
            __syncthreads();
            for (int i = threadIdx.x; i < 2 * kBins; i += blockDim.x) {
                uint32_t x = h[i];
                if (x) atomicAdd(&st.hist[(int64_t)(cbase + i / kBins) * kBins + (i % kBins)], x);
            }
        }
    }
    if (!fused) return;
    if (fused == 2) {
        seg_tickets_pick(N, p, nlists, idbits, sv, st, v0, lds, clip);
        return;
    }
    // ticket: the last workgroup sees every histogram
    __syncthreads();
    if (threadIdx.x == 0) {
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
        int t = atomicAdd(&st.ctl[1], 1);
        last = t == (int)gridDim.x - 1;
        if (last) __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
    }
    __syncthreads();
    if (!last) return;
    for (int32_t c = 0; c < nlists; c++) sel_pick_list(st, c, p, idbits, sv.mode, sv.m, lds, clip);
    if (threadIdx.x == 0) st.ctl[1] = 0;
}

__global__ __launch_bounds__(kBlock) void k_select_pick(int32_t nlists, int p, int idbits, SelView sv,
                                                        SelState st, const int32_t *go, int32_t clip)
{
    __shared__ int64_t lds[16];
    const int32_t gv = go ? *go : 1, ctl = st.ctl[0];  // loaded together
    if (gv == 0) return;
    if (p > 0 && ctl <= 0) return;
    int32_t c = blockIdx.x;
    if (c >= nlists) return;
    sel_pick_list(st, c, p, idbits, sv.mode, sv.m, lds, clip);
}

__device__ __forceinline__ bool sel_chosen(int64_t v, const SelView &sv, const SelState &st)
{
    int32_t s = sv.nseg[v];
    int sd = sv.side[v];
    int32_t g = sv.gain[v];
    if (!sel_list(s, sd, g, sv.mode)) return false;
    int32_t c = 2 * s + sd;
    if (st.rsel[c] <= 0) return false;
    return sel_key(st.gmax[c], g, (uint32_t)(v - sv.nbase[s]), sv.idbits) <= st.kthr[c];
}

// ---- small segments: the whole selection and the moves in one workgroup --------------------

constexpr int kSegThreads = 1024;     // flips above 4 K nodes
constexpr int kSegThreadsBal = 768;   // balance from 8 K to 24 K nodes
constexpr int kSegThreadsSmall = 256; // flips up to 4 K nodes, balance up to 8 K
// nodes per thread, kept in registers: the flipping kind holds both lists'
// thresholds as well.  1024 threads leave 128 registers per thread, 768
// threads 170: 32 balance nodes each without spilling
template <int KIND, int TH> constexpr int seg_items() { return KIND == 0 ? 16 : 32; }
template <int KIND, int TH> constexpr int32_t seg_select_max() { return TH * seg_items<KIND, TH>(); }
constexpr int kSegKeys = 256;                           // balance candidates: ceil(sqrt n) <= 182

// Balance selection of mid-size segments in chunks: each chunk of up to
// kChunkNodes nodes of a segment (1024 threads, 16 nodes each) orders its
// best ceil(sqrt n) nodes, then one workgroup per segment merges the chunks'
// lists.  The union holds the segment's best ceil(sqrt n), so the merge's
// first ones are those of the whole segment.
constexpr int kChunkThreads = 1024;
constexpr int32_t kChunkNodes = 16384;
constexpr int kChunkMax = 16;      // chunks per segment: segments up to 262144 nodes
constexpr int kChunkKeys = 512;    // per chunk: ceil(sqrt 262144) = 512 at most
struct ChunkArgs {
    const int32_t *seg, *beg, *count;  // chunk table: segment, first node; count[0] chunks
    int32_t N;                         // the level's nodes (bounds the chunk's loads)
    uint64_t *cand;                    // [S][kChunkMax][kChunkKeys]: each chunk's best, ascending
    int32_t *ccnt;                     // [S][kChunkMax]: how many
};

// The merge of a balancing segment's chunk lists (1024 threads of one
// workgroup, the last of the segment's chunks): each node of the chunks'
// ascending lists is ranked among all of them (its index in its
// own list plus, by binary search, the smaller keys of every other list); the
// first min(total, m) in order are the segment's chosen nodes.  Then the
// balance prefix over them (bal_finish_block: one chosen node a thread, as
// they fit the workgroup).
__device__ __forceinline__ void bal_merge_seg(int32_t s, const int32_t *nbase, const int32_t *m, ChunkArgs ca,
                                              BalFinish bf)
{
    static_assert(kChunkKeys <= 1024, "the chosen nodes fit the workgroup");
    __shared__ uint64_t a[kChunkMax * kChunkKeys];
    __shared__ uint64_t out[kChunkKeys];
    __shared__ int32_t cnt[kChunkMax];
    int32_t n = nbase[s + 1] - nbase[s];
    int ng = (int)((n + kChunkNodes - 1) / kChunkNodes);  // <= kChunkMax, checked by the caller
    const int32_t tid = threadIdx.x, nslot = ng * kChunkKeys;
    // every slot of the segment's lists (past a list's count: unused), with the
    // counts; the segment's balance state is loaded with them
    const uint64_t *src = ca.cand + (int64_t)s * kChunkMax * kChunkKeys;
    for (int32_t f = tid; f < nslot; f += 1024) a[f] = src[f];
    if (tid < kChunkMax) cnt[tid] = tid < ng ? ca.ccnt[s * kChunkMax + tid] : 0;
    const int h = (bf.mode[s] & kList1) ? 1 : 0;
    const int64_t nd = bf.need[s], rm = bf.room[s];
    int64_t bm0 = 0, bm1 = 0;
    if (tid == 0) {
        bm0 = bf.bal_moved[2 * s];
        bm1 = bf.bal_moved[2 * s + 1];
    }
    __syncthreads();
    int32_t tot = 0;
    for (int q = 0; q < ng; q++) tot += cnt[q];
    int32_t take = min(tot, m[s]);
    // list-major slots (a wavefront's keys are neighbours in one list, so
    // their searches read the same LDS words), the index range rotated by a
    // wavefront per pass so that no thread ranks the heads of several lists,
    // the keys with the most lists to search
    for (int32_t f = tid; f < nslot; f += 1024) {
        int q = f / kChunkKeys;
        int32_t i = ((f % kChunkKeys) + 64 * (f / 1024)) % kChunkKeys;
        if (i >= cnt[q] || i >= take) continue;
        uint64_t x = a[q * kChunkKeys + i];
        int32_t rank = i;
        for (int o = 0; o < ng && rank < take; o++) {
            if (o == q) continue;
            const uint64_t *b = a + o * kChunkKeys;
            int32_t lo = 0, hi = cnt[o];
            while (lo < hi) {
                int32_t mid = (lo + hi) >> 1;
                if (b[mid] < x) lo = mid + 1;
                else hi = mid;
            }
            rank += lo;
        }
        if (rank < take) out[rank] = x;
    }
    __syncthreads();
    bal_finish_block(s, out, take, bf, h, nd, rm, bm0, bm1);
}

// One workgroup per segment of at most seg_select_max<KIND, TH>() nodes: each list's
// r-th key by the same 12-bit radix select as the multi-workgroup passes,
// with the segment's gains in registers and the histogram in LDS, then the
// moves (bf.side is written): kind 0 flips the chosen nodes of both lists
// (Algorithm 3 and the swap of Algorithm 5); kind 1 orders the chosen nodes
// of the over-weight side (by counting, their weights and incidence ranges
// gathered meanwhile) and the workgroup takes the balance prefix (Algorithm
// 5).  The chosen set is the one the multi-workgroup path chooses: the same
// keys, the same r.
//
// CH (kind 1 only): one workgroup per chunk of the chunk table instead, whose
// ordered best nodes go to ca for the merge by the segment's last chunk; node
// ids in the selection keys are then local to the chunk, which keeps them
// short.
template <int KIND, int TH, bool CH = false>
__global__ __launch_bounds__(TH) void k_seg_select(int32_t S, SelView sv, SelState st, int idbits_lv,
                                                           const int32_t *nw,
                                                           unsigned long long *segw, BalFinish bf,
                                                           const int32_t *go, ChunkArgs ca)
{
    static_assert(!CH || (KIND == 1 && TH * 16 == kChunkNodes), "chunks: balance, 16 nodes a thread");
    constexpr int kSegItems = CH ? 16 : seg_items<KIND, TH>();
    constexpr int32_t kCap = TH * kSegItems;
    constexpr int kKeys = CH ? kChunkKeys : kSegKeys;
    __shared__ uint32_t hist[kBins];
    __shared__ int64_t lds64[16];
    __shared__ int32_t sbin, sbefore, sin_;
    __shared__ uint64_t keys[kKeys], sorted[KIND == 1 ? kKeys : 1];
    __shared__ uint8_t sdl[kCap];  // the segment's sides
    __shared__ int32_t nkeys;
    // the round's flag is loaded together with what the block reads next (all
    // in bounds: the grid never exceeds the segments or the chunk table, and a
    // chunk entry past the count is not used)
    const int32_t gv = go ? *go : 1;
    int32_t s, a0, n;
    uint8_t md;
    int64_t bnd = 0, brm = 0, bm0 = 0, bm1 = 0;  // balance (one workgroup): the segment's state, loaded early
    int32_t nld;  // nodes whose gains and sides are loaded (CH: from the level's end, not the segment's)
    if (CH) {
        int32_t ci = blockIdx.x;
        int32_t cc = ca.count[0];
        s = ca.seg[ci];
        a0 = ca.beg[ci];
        if (gv == 0 || ci >= cc) return;
        nld = min(ca.N - a0, kChunkNodes);
        n = min(sv.nbase[s + 1] - a0, kChunkNodes);
        md = sv.mode[s];
    } else {
        s = blockIdx.x;
        a0 = sv.nbase[s];
        int32_t a1 = sv.nbase[s + 1];
        md = sv.mode[s];
        if (KIND == 1) {
            bnd = bf.need[s];
            brm = bf.room[s];
            bm0 = bf.bal_moved[2 * s];
            bm1 = bf.bal_moved[2 * s + 1];
        }
        if (gv == 0) return;
        n = a1 - a0;
        nld = n;
    }
    const int idbits = CH ? bitlen_u32((uint32_t)max(n - 1, 0)) : idbits_lv;
    int32_t g[kSegItems];
    uint64_t sbits = 0, ebits = 0;  // bit j: item j's side, item j eligible for its side's list
    // per list: size and gain extremes, from the gains just loaded
    int32_t lc[2] = {0, 0}, lmax[2] = {INT32_MIN, INT32_MIN}, lmin[2] = {INT32_MAX, INT32_MAX};
    // the segment's sides by aligned 4-byte words (a word never leaves the
    // memory page of the bytes it covers) and its gains (indices past the
    // segment read its node 0): loads in flight together
    const uint8_t *sp = sv.side + a0;
    int32_t off0 = (int32_t)((uintptr_t)sp & 3), nwd = (off0 + n + 3) >> 2, nwl = (off0 + nld + 3) >> 2;
    const uint32_t *wp = (const uint32_t *)(sp - off0);
    constexpr int kW = kCap / 4 / TH + 1;
    uint32_t xw[kW];
    // (CH: issued before the segment's bounds arrive; nodes past the segment
    // are loaded but never used)
    if ((CH || md) && nld > 0) {
#pragma unroll
        for (int q = 0; q < kW; q++) xw[q] = wp[min(q * TH + (int32_t)threadIdx.x, nwl - 1)];
#pragma unroll
        for (int j = 0; j < kSegItems; j++) {
            int32_t i = j * TH + (int32_t)threadIdx.x;
            g[j] = sv.gain[a0 + (i < nld ? i : 0)];
        }
    }
    if (!md) return;
    // the histogram starts cleared (each radix pass clears the bins it read),
    // the balance key list empty
    for (int i = threadIdx.x; i < kBins; i += TH) hist[i] = 0;
    if (threadIdx.x == 0) nkeys = 0;
    if (n > 0) {
        // the sides staged in LDS
#pragma unroll
        for (int q = 0; q < kW; q++) {
            int32_t w = q * TH + (int32_t)threadIdx.x;
#pragma unroll
            for (int b = 0; b < 4; b++) {
                int32_t i = 4 * w + b - off0;
                if (w < nwd && i >= 0 && i < n) sdl[i] = (uint8_t)(xw[q] >> (8 * b));
            }
        }
    }
    __syncthreads();
#pragma unroll
    for (int j = 0; j < kSegItems; j++) {
        int32_t i = j * TH + (int32_t)threadIdx.x;
        int sd = i < n ? sdl[i] : 0;
        sbits |= (uint64_t)sd << j;
        if (i < n && ((md >> sd) & 1) && !((md & kGainNonNeg) && g[j] < 0)) {  // sel_list
            ebits |= 1ull << j;
            lc[sd]++;
            lmax[sd] = max(lmax[sd], g[j]);
            lmin[sd] = min(lmin[sd], g[j]);
        }
    }
    {
        __shared__ int32_t red[TH / 64][6];
        int32_t x[6] = {lc[0], lc[1], lmax[0], lmax[1], lmin[0], lmin[1]};
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) {
            x[0] += __shfl_xor(x[0], o, 64);
            x[1] += __shfl_xor(x[1], o, 64);
            x[2] = max(x[2], __shfl_xor(x[2], o, 64));
            x[3] = max(x[3], __shfl_xor(x[3], o, 64));
            x[4] = min(x[4], __shfl_xor(x[4], o, 64));
            x[5] = min(x[5], __shfl_xor(x[5], o, 64));
        }
        if ((threadIdx.x & 63) == 0)
            for (int q = 0; q < 6; q++) red[threadIdx.x >> 6][q] = x[q];
        __syncthreads();
        lc[0] = red[0][0];
        lc[1] = red[0][1];
        lmax[0] = red[0][2];
        lmax[1] = red[0][3];
        lmin[0] = red[0][4];
        lmin[1] = red[0][5];
#pragma unroll 1
        for (int w = 1; w < TH / 64; w++) {
            lc[0] += red[w][0];
            lc[1] += red[w][1];
            lmax[0] = max(lmax[0], red[w][2]);
            lmax[1] = max(lmax[1], red[w][3]);
            lmin[0] = min(lmin[0], red[w][4]);
            lmin[1] = min(lmin[1], red[w][5]);
        }
        // (red is not written again: no barrier before what follows)
    }
    uint64_t thr[2] = {0, 0};
    int32_t rr[2] = {0, 0};
    constexpr int per = (kBins + TH - 1) / TH;  // bins per thread (the last ones may run past kBins)
    for (int sd = 0; sd < 2; sd++) {
        int32_t c = 2 * s + sd;
        int64_t r = 0;
        if ((md >> sd) & 1) {
            int64_t t = lc[sd];
            if (md & kMinPair) {
                int64_t o = lc[sd ^ 1];
                r = t < o ? t : o;
            } else {
                r = t < (int64_t)sv.m[s] ? t : (int64_t)sv.m[s];
            }
        }
        rr[sd] = (int32_t)r;
        if (r == 0) continue;
        if (r == lc[sd]) {  // the whole list: no pass needed
            thr[sd] = ~0ull;
            continue;
        }
        int32_t gmax = lmax[sd];
        int T = bitlen_u32((uint32_t)((int64_t)gmax - lmin[sd])) + idbits;
        uint64_t pre = 0;
        int32_t rem = (int32_t)r;
        for (int p = 0;; p++) {
            int hi = T - kDigit * p, lo = hi - kDigit > 0 ? hi - kDigit : 0;
            uint64_t mine = ebits & (sd ? sbits : ~sbits);
#pragma unroll
            for (int j = 0; j < kSegItems; j++) {
                if (!((mine >> j) & 1)) continue;
                uint64_t k = sel_key(gmax, g[j], (uint32_t)(j * TH + threadIdx.x), idbits);
                if (p > 0 && ((k ^ pre) >> hi) != 0) continue;
                int dig = hi > 0 ? (int)((k >> lo) & ((1ull << (hi - lo)) - 1ull)) : 0;
                atomicAdd(&hist[dig], 1u);
            }
            __syncthreads();
            int64_t loc = 0;
            for (int j = 0; j < per; j++)
                if (threadIdx.x * per + j < kBins) loc += hist[threadIdx.x * per + j];
            // exclusive scan of the bin sums over the workgroup: the barrier
            // above already separates these LDS writes from the last pass's
            // reads, and the one below the bin pick from the next pass's writes
            int64_t ex = wave_incl_scan(loc);
            if ((threadIdx.x & 63) == 63) lds64[threadIdx.x >> 6] = ex;
            __syncthreads();
            for (int w = 0; w < (int)(threadIdx.x >> 6); w++) ex += lds64[w];
            ex -= loc;
            if (ex < rem && rem <= ex + loc) {
                int64_t acc = ex;
                for (int j = 0; j < per; j++) {
                    int64_t x = threadIdx.x * per + j < kBins ? hist[threadIdx.x * per + j] : 0;
                    if (acc + x >= rem) {
                        sbin = threadIdx.x * per + j;
                        sbefore = (int32_t)acc;
                        sin_ = (int32_t)x;
                        break;
                    }
                    acc += x;
                }
            }
            // only this thread reads its bins: clear them for the next pass
            for (int j = 0; j < per; j++)
                if (threadIdx.x * per + j < kBins) hist[threadIdx.x * per + j] = 0;
            __syncthreads();
            // (the next pass writes the pick only after two more barriers)
            int32_t bin = sbin, left = rem - sbefore, inb = sin_;
            pre |= (uint64_t)bin << lo;
            rem = left;
            if (left == inb || lo == 0) {
                thr[sd] = pre | (lo ? ((1ull << lo) - 1ull) : 0ull);
                break;
            }
        }
    }
    if (!CH && threadIdx.x == 0) {
        st.rsel[2 * s] = rr[0];
        st.rsel[2 * s + 1] = rr[1];
    }
    if (KIND == 0) {
        // flip the chosen nodes of both lists
        int64_t d01 = 0;  // weight moving from side 0 to side 1
#pragma unroll
        for (int j = 0; j < kSegItems; j++) {
            if (!((ebits >> j) & 1)) continue;
            int sd = (sbits >> j) & 1;
            if (rr[sd] == 0) continue;
            uint32_t lid = (uint32_t)(j * TH + threadIdx.x);
            if (sel_key(lmax[sd], g[j], lid, idbits) > thr[sd]) continue;
            int32_t v = a0 + (int32_t)lid;
            int64_t w = nw[v];
            bf.side[v] = (uint8_t)(1 - sd);
            d01 += sd ? -w : w;
        }
        d01 = block_sum(d01, lds64);
        if (threadIdx.x == 0 && d01 != 0) {
            atomicAdd(&segw[2 * s], (unsigned long long)(-d01));
            atomicAdd(&segw[2 * s + 1], (unsigned long long)d01);
        }
        return;
    }
    // balance: the chosen nodes of the over-weight side, sorted, then the prefix
    int h = (md & kList1) ? 1 : 0;
    if (rr[h] > 0) {
        uint64_t mine = ebits & (h ? sbits : ~sbits);
#pragma unroll
        for (int j = 0; j < kSegItems; j++) {
            if (!((mine >> j) & 1)) continue;
            uint32_t lid = (uint32_t)(j * TH + threadIdx.x);
            if (sel_key(lmax[h], g[j], lid, idbits) > thr[h]) continue;
            keys[atomicAdd(&nkeys, 1)] = gain_order_key(g[j], (uint32_t)(a0 + (int32_t)lid));
        }
    }
    __syncthreads();
    int32_t cnt = nkeys;
    if (!CH) {
        // counting order (as block_rank_sort), each chosen node's weight and
        // incidence range loaded while its rank is counted (for the finish)
        __shared__ int32_t pw[CH ? 1 : kKeys], pnb[CH ? 1 : kKeys], pne[CH ? 1 : kKeys];
        const bool logm = bf.ml.cnode != nullptr;
        int tpc = 1;
        while (tpc < 16 && cnt * 2 * tpc <= TH) tpc <<= 1;
        for (int base = 0; base < cnt * tpc; base += TH) {
            int t = base + (int)threadIdx.x, i = t / tpc, part = t & (tpc - 1);
            uint64_t x = keys[i < cnt ? i : 0];
            int32_t v = (int32_t)(uint32_t)(x & 0xffffffffu), xw = 0, xb = 0, xe = 0;
            if (i < cnt && part == 0) {
                xw = nw[v];
                if (logm) {
                    xb = bf.ml.noff[v];
                    xe = bf.ml.noff[v + 1];
                }
            }
            int r = 0;
            if (i < cnt) {
#pragma unroll 8
                for (int j = part; j < cnt; j += tpc) r += keys[j] < x;
            }
            for (int o = 1; o < tpc; o <<= 1) r += __shfl_xor(r, o, 64);
            if (i < cnt && part == 0) {
                sorted[r] = x;
                pw[r] = xw;
                pnb[r] = xb;
                pne[r] = xe;
            }
        }
        __syncthreads();
        bal_finish_block(s, sorted, cnt, bf, h, bnd, brm, bm0, bm1, BalPre{pw, pnb, pne});
        return;
    }
    block_rank_sort(keys, sorted, cnt);
    int32_t gi = (a0 - sv.nbase[s]) / kChunkNodes;
    uint64_t *dst = ca.cand + ((int64_t)s * kChunkMax + gi) * kChunkKeys;
    for (int32_t i = threadIdx.x; i < cnt; i += TH) dst[i] = sorted[i];
    if (threadIdx.x == 0) ca.ccnt[s * kChunkMax + gi] = cnt;
    // the segment's last chunk to finish (ticket) merges the lists
    __shared__ int32_t last;
    __syncthreads();
    if (threadIdx.x == 0) {
        int32_t nch = (sv.nbase[s + 1] - sv.nbase[s] + kChunkNodes - 1) / kChunkNodes;
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
        last = atomicAdd(&st.tick[s], 1) == nch - 1;
        if (last) {
            st.tick[s] = 0;
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
        }
    }
    __syncthreads();
    if (last) bal_merge_seg(s, sv.nbase, sv.m, ca, bf);
}

// The chunk table of a level: segment s gets ceil(n_s / kChunkNodes)
// consecutive entries (its segment and first node).  One workgroup.
__global__ __launch_bounds__(1024) void k_chunk_table(int32_t S, const int32_t *nbase, int32_t *seg,
                                                      int32_t *beg, int32_t *count)
{
    __shared__ int32_t lds[16];
    __shared__ int32_t carry;
    if (threadIdx.x == 0) carry = 0;
    __syncthreads();
    for (int32_t base = 0; base < S; base += blockDim.x) {
        int32_t s = base + (int32_t)threadIdx.x;
        int32_t a = s < S ? nbase[s] : 0, n = s < S ? nbase[s + 1] - a : 0;
        int32_t c = (n + kChunkNodes - 1) / kChunkNodes, tot;
        int32_t at = block_excl_scan(c, lds, &tot) + carry;
        for (int32_t i = 0; i < c; i++) {
            seg[at + i] = s;
            beg[at + i] = a + i * kChunkNodes;
        }
        __syncthreads();
        if (threadIdx.x == 0) carry += tot;
        __syncthreads();
    }
    if (threadIdx.x == 0) count[0] = carry;
}

// ---- moves ---------------------------------------------------------------------------------

__global__ __launch_bounds__(kBlock) void k_flip(int32_t N, SelView sv, SelState st, uint8_t *side,
                                                 const int32_t *nw, unsigned long long *segw,
                                                 const int32_t *go)
{
    __shared__ unsigned long long dw[kAggLists / 2];  // two's complement sums
    if (go && *go == 0) return;
    int64_t lo, hi;
    reduce_chunk(N, gridDim.x, blockIdx.x, lo, hi);
    if (lo >= hi) return;
    int32_t s0 = sv.nseg[lo], ns = sv.nseg[hi - 1] + 1 - s0;
    bool local = 2 * ns <= kAggLists;
    for (int i = threadIdx.x; i < kAggLists / 2; i += blockDim.x) dw[i] = 0;
    __syncthreads();
    for (int64_t v = lo + threadIdx.x; v < hi; v += blockDim.x) {
        if (!sel_chosen(v, sv, st)) continue;
        int32_t sd = side[v];
        int64_t w = nw[v];
        side[v] = (uint8_t)(1 - sd);
        int32_t s = sv.nseg[v];
        // weight moving from side 0 to side 1 (negative: the other way)
        if (local) {
            atomicAdd(&dw[s - s0], (unsigned long long)(sd ? -w : w));
        } else {
            atomicAdd(&segw[2 * s + sd], (unsigned long long)(-w));
            atomicAdd(&segw[2 * s + 1 - sd], (unsigned long long)w);
        }
    }
    __syncthreads();
    if (local)
        for (int i = threadIdx.x; i < ns; i += blockDim.x)
            if (dw[i]) {
                atomicAdd(&segw[2 * (s0 + i)], 0ull - dw[i]);
                atomicAdd(&segw[2 * (s0 + i) + 1], dw[i]);
            }
}

__global__ __launch_bounds__(kBlock) void k_gather(int32_t N, SelView sv, SelState st, int32_t *ccount,
                                                   uint64_t *cand, int32_t stride, const int32_t *go)
{
    if (go && *go == 0) return;
    int64_t v0 = (int64_t)blockIdx.x * blockDim.x, v = v0 + threadIdx.x;
    int64_t vl = min(v0 + (int64_t)blockDim.x, (int64_t)N) - 1;
    int32_t s0 = sv.nseg[v0];
    if (s0 != sv.nseg[vl]) {  // workgroup over several segments: node by node
        if (v >= N || !sel_chosen(v, sv, st)) return;
        int32_t s = sv.nseg[v];
        int32_t at = atomicAdd(&ccount[s], 1);
        if (at < stride) cand[(int64_t)s * stride + at] = gain_order_key(sv.gain[v], (uint32_t)v);
        return;
    }
    // one segment: its lists' state once, one append atomic per wavefront
    uint8_t md = sv.mode[s0];
    int32_t nb0 = sv.nbase[s0];
    bool chosen = false;
    int32_t g = 0;
    if (v < N) {
        int sd = sv.side[v];
        g = sv.gain[v];
        int32_t c = 2 * s0 + sd;
        chosen = ((md >> sd) & 1) && !((md & kGainNonNeg) && g < 0) && st.rsel[c] > 0 &&
                 sel_key(st.gmax[c], g, (uint32_t)(v - nb0), sv.idbits) <= st.kthr[c];
    }
    int32_t at = lds_wave_slot(chosen, &ccount[s0]);
    if (at >= 0 && at < stride) cand[(int64_t)s0 * stride + at] = gain_order_key(g, (uint32_t)v);
}

// ---- per-round modes: also reset the selection state of the lists --------------------------

__device__ __forceinline__ void reset_lists(SelState st, int32_t s)
{
    for (int sd = 0; sd < 2; sd++) {
        int32_t c = 2 * s + sd;
        st.tot[c] = 0;
        st.gmax[c] = INT32_MIN;
        st.gmin[c] = INT32_MAX;
        st.done[c] = 0;
    }
    st.tick[s] = 0;
}

// Algorithm 3 loop test per segment: P0 below its share and P1 non-empty.
// Round counters without a launch of their own: round ri counts its active
// segments in slot ri % 3, reads the previous round's count from slot
// (ri - 1) % 3 (complete) and clears slot (ri + 1) % 3 for the next round.
__device__ __forceinline__ int32_t round_counters(int32_t *go, int32_t ri, int32_t s)
{
    int32_t prev = ri > 0 ? go[4 + (ri + 2) % 3] : 0;
    if (s == 0) {
        go[4 + (ri + 1) % 3] = 0;
        go[1] = prev;
        if (prev) go[2] += 1;
        go[3] = 0;
    }
    return prev;
}

__global__ void k_round_initial(int32_t S, int32_t j, const int32_t *nbase, const int32_t *coarsest,
                                const int32_t *k0, const int32_t *k1, const int64_t *W,
                                const unsigned long long *segw, int32_t *cnt1, int32_t ri,
                                uint8_t *mode, uint8_t *gmask, int32_t *m, SelState st, int32_t *go)
{
    int32_t s = blockIdx.x * blockDim.x + threadIdx.x;
    bool first = ri == 0;
    if (s == 0) st.ctl[0] = 2 * S;
    int32_t prev = round_counters(go, ri, s);
    int32_t *cur = go + 4 + ri % 3;
    if (s >= S) return;
    if (prev == 0 && !first) {  // the previous round found nothing to do
        mode[s] = 0;
        gmask[s] = 0;
        return;
    }
    uint8_t md = 0;
    if (coarsest[s] == j) {
        int32_t n = nbase[s + 1] - nbase[s];
        if (first) cnt1[s] = n;
        else cnt1[s] -= st.rsel[2 * s + 1];
        int64_t ks = (int64_t)k0[s] + k1[s];
        bool run = (int64_t)segw[2 * s] * ks < W[s] * (int64_t)k0[s] && cnt1[s] > 0;
        if (run) {
            md = kList1;
            m[s] = (int32_t)ceil_sqrt_i64(n);
            atomicAdd(cur, 1);
        }
    }
    mode[s] = md;
    gmask[s] = md ? 1 : 0;
    reset_lists(st, s);
    st.rsel[2 * s] = 0;
    st.rsel[2 * s + 1] = 0;
}

__global__ void k_round_refine(int32_t S, int32_t j, const int32_t *coarsest, uint8_t *mode,
                               uint8_t *gmask, uint8_t *done, SelState st, int32_t *go)
{
    int32_t s = blockIdx.x * blockDim.x + threadIdx.x;
    if (s == 0) st.ctl[0] = 2 * S;
    if (s >= S) return;
    bool present = coarsest[s] >= j;
    mode[s] = present ? (kList0 | kList1 | kGainNonNeg | kMinPair) : 0;
    gmask[s] = present ? 1 : 0;
    done[s] = present ? 0 : 1;
    reset_lists(st, s);
}

// Balance test per segment: the side over its bound, the excess, the room.
struct RoundBal {
    int32_t S;
    const int32_t *nbase;
    const unsigned long long *segw;
    const int64_t *max0, *max1;
    uint8_t *done, *mode, *gmask;
    int32_t *m;
    int64_t *need, *room;
    int32_t *ccount;
};

__device__ __forceinline__ void round_balance_seg(int32_t s, const RoundBal &rb, SelState st, int32_t *go,
                                                  int32_t ri)
{
    int32_t S = rb.S;
    const int32_t *nbase = rb.nbase;
    const unsigned long long *segw = rb.segw;
    const int64_t *max0 = rb.max0, *max1 = rb.max1;
    uint8_t *done = rb.done, *mode = rb.mode, *gmask = rb.gmask;
    int32_t *m = rb.m, *ccount = rb.ccount;
    int64_t *need = rb.need, *room = rb.room;
    if (s == 0) st.ctl[0] = 2 * S;
    round_counters(go, ri, s);
    int32_t *cur = go + 4 + ri % 3;
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
            atomicAdd(cur, 1);
        }
    }
    mode[s] = md;
    gmask[s] = md ? 1 : 0;
    reset_lists(st, s);
}

__global__ void k_round_balance(RoundBal rb, SelState st, int32_t *go, int32_t ri)
{
    round_balance_seg(blockIdx.x * blockDim.x + threadIdx.x, rb, st, go, ri);
}

// A later balance round's test and the marking of the hyperedges of the nodes
// the previous round moved, in one launch: they are independent (the test
// reads the side weights, the marking the move log, both left by the previous
// round).  Blocks [0, gs) test, the others mark, when the previous round had
// anything to do.
__global__ __launch_bounds__(kBlock) void k_round_balance_log(int64_t gs, RoundBal rb, SelState st, int32_t *go,
                                                              int32_t ri, const int32_t *count,
                                                              const int32_t *cnode, const int32_t *cbeg,
                                                              const int32_t *noff, const int32_t *inc,
                                                              uint32_t *bits, const void *cc, int pk,
                                                              const uint8_t *side, int32_t *gain)
{
    if ((int64_t)blockIdx.x < gs) {
        round_balance_seg(blockIdx.x * blockDim.x + threadIdx.x, rb, st, go, ri);
        return;
    }
    // the previous round's counter and its log size, loaded together
    const int32_t prev = go[4 + (ri + 2) % 3], n = count[0];
    if (prev == 0) return;  // the previous round moved nothing
    log_hedges_blocks((int64_t)blockIdx.x - gs, (int64_t)gridDim.x - gs, n, cnode, cbeg, noff, inc, bits, cc, pk,
                      side, gain);
}


}  // namespace bp
