// Device-resident hypergraph levels and per-segment state.
//
// A Level holds the disjoint union of S independent (sub)hypergraphs
// ("segments") in one CSR: segment s owns nodes [nbase[s], nbase[s+1]) and
// hyperedges [hbase[s], hbase[s+1]).  Node and hyperedge ids inside a segment
// are ordered as in the segment's own numbering, so every comparison by id
// and every hash of a local id gives the same result as if the segment were
// partitioned alone (the nested k-way scheme of Algorithm 6).
#pragma once
#include "sched.hpp"

namespace bp {

struct Level {
    int32_t N = 0, E = 0, P = 0, S = 0;
    int32_t *off = nullptr;   // [E+1]
    int32_t *pins = nullptr;  // [P]
    int32_t *nw = nullptr;    // [N] node weights
    int32_t *hw = nullptr;    // [E] hyperedge weights
    int32_t *nseg = nullptr;  // [N] segment of each node
    int32_t *hseg = nullptr;  // [E] segment of each hyperedge
    int32_t *nbase = nullptr; // [S+1]
    int32_t *hbase = nullptr; // [S+1]
    // schedule lists (hyperedge ids) of the WAVE and BLOCK buckets; lhuge is
    // the subset of lbig above the LDS sort capacity
    int32_t *lmid = nullptr, *lbig = nullptr, *lhuge = nullptr;
    int32_t nmid = 0, nbig = 0, nhuge = 0;
    int32_t maxseg_nodes = 0;   // largest segment node count
    int32_t maxseg_pins = 0;    // largest segment pin count
    int32_t maxseg_hedges = 0;  // largest segment hyperedge count
    int32_t *parent = nullptr;  // [N] -> ids of the next level, once coarsened
    uint8_t *side = nullptr;    // [N] bisection side
    // node-major incidence: hyperedges of node v are inc[noff[v] .. noff[v+1])
    int32_t *noff = nullptr;    // [N+1]
    int32_t *inc = nullptr;     // [P]
    int32_t *lnmid = nullptr, *lnbig = nullptr;  // node buckets (degree > 32, > 2048)
    int32_t *ncount = nullptr;  // device: [0] = |lnmid|, [1] = |lnbig|, [2] = chunks of big nodes
    int64_t nmid_bound = 0, nbig_bound = 0;      // grid bounds for the node buckets
    // big nodes (degree > 2048) are reduced in chunks of 4096 incidences
    int32_t *chunk_node = nullptr, *chunk_beg = nullptr, *chunk_big = nullptr;
    int32_t *big_chunks = nullptr, *big_done = nullptr;  // per big node
    int64_t nchunk_bound = 0;
    int32_t *bigslot = nullptr;  // [N] index of a big node in lnbig, else -1
    // bits of a bound on any list's gain span (max - min gain): 2 max_v sum of
    // w(e) over v's hyperedges <= 2 (max degree)(max hyperedge weight)
    int32_t span_bits = 32;
    int2 *cc = nullptr;         // [E] per-hyperedge gain contributions (scratch)
    int32_t cc_pk = 0;          // contributions packed as two int16 (every w(e) < 2^15)
};

// Sizes and counters read back once per level.
struct LevelInfo {
    int32_t N, E, P;
    int32_t nmid, nbig, nhuge;
    int32_t unresolved;     // duplicate-check collisions still open
    int32_t active;         // segments that keep coarsening
    int32_t maxseg_nodes;   // largest segment
    int32_t flag;           // general-purpose count (rounds still running)
    int32_t maxseg_pins, maxseg_hedges;
    int32_t pad[4];
};

// Per-list selection state (device arrays of 2S unless noted).
struct SelState {
    uint32_t *hist;   // [2S * 4096], zero between passes
    int32_t *tot;     // eligible nodes
    int32_t *gmax, *gmin;
    int32_t *rsel;    // r, the number to choose (0 = none)
    int32_t *rem;     // remaining inside the current prefix
    int32_t *kbits;   // width of the list's key (u << idbits | lid)
    uint64_t *kpre;   // key bits fixed by the passes so far
    uint64_t *kthr;   // the r-th smallest key once found
    uint8_t *done;
    int32_t *ctl;     // [4]: [0] lists still open, [1] ticket
    int32_t *tick;    // [S] per-segment tickets of the fused picks
};

// Per-segment bisection state (device arrays; 2S entries where per side).
struct Segs {
    int32_t S = 0;
    int32_t *k0, *k1;         // parts on each side of this bisection
    int32_t *lo;              // first part id of the segment
    int64_t *W;               // total node weight
    int64_t *max0, *max1;     // side weight bounds
    uint8_t *active;          // still coarsening
    int32_t *coarsest;        // index of the coarsest level
    int64_t *w;               // [2S] side weights at the current level
    int32_t *cnt1;            // nodes on side 1 (initial bisection)
    uint8_t *mode;            // selection mode (see refine.hpp)
    uint8_t *gmask;           // segments whose gains are needed
    int32_t *m;               // ceil(sqrt(nodes)) at the current level
    int64_t *need, *room;     // balance step
    int64_t *bal_moved;       // [2S]: weight moved and rounds run by the level's balance step
    uint8_t *done;
    int32_t *stuck;           // balance stopped over the bound (any level)
    int32_t *root_levels;     // coarsening steps
    int32_t *ccount;          // balance candidates per segment
    uint64_t *cand;           // [S * cand_stride]
    int32_t cand_stride = 0;
    uint64_t *chunk_cand = nullptr;  // chunked balance selection: [S][kChunkMax][kChunkKeys], or null
    int32_t *chunk_ccnt = nullptr;   // [S][kChunkMax]
    int32_t *chunk_tab = nullptr;    // chunk table: segment, first node ([2][chunk_tab_n]), count
    int64_t chunk_tab_n = 0;
    int32_t *go;              // [8] round counters: [1] last count, [2] rounds run, [3] estimate,
                              // [4..6] per-round active counts (round i uses slot 4 + i % 3)
    SelState st;              // selection state of the 2S lists
};

}  // namespace bp
