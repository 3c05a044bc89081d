/*
 * Sequential oracle of BiPart's deterministic multilevel partitioner.
 *
 * TEST INFRASTRUCTURE ONLY.  This is a plain, slow, single-threaded C
 * rendering of the paper's method (problem statement of Section 1.1,
 * Algorithms 1-6 of Section 3) used to check the HIP library.  Only the test
 * suite, the smoke check and the benchmark's CPU-baseline leg may load it; the
 * product path never calls into it and shares no code with it.
 *
 * Hypergraphs are CSR over hyperedges: off[e+1], pins[off[e]..off[e+1]) are
 * the node ids of hyperedge e.  nw (node weights) and hw (hyperedge weights)
 * may be NULL, meaning all ones.  All arithmetic is integer except the one
 * conversion of the imbalance eps into a 32.32 fixed-point factor.
 */
#ifndef BIPART_ORACLE_H
#define BIPART_ORACLE_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* matching policies of Table 1 */
enum { OR_LDH = 0, OR_HDH = 1, OR_LWD = 2, OR_HWD = 3, OR_RAND = 4 };

typedef struct {
    int32_t policy;           /* Table 1 policy, default LDH */
    int32_t max_levels;       /* coarsening depth cap (Section 3.4), default 25 */
    int32_t refine_iters;     /* Algorithm 5 "iter", default 2 */
    int32_t min_coarse_nodes; /* stop coarsening at or below this many nodes, default 100 */
} oracle_params;

/* MurmurHash3 32-bit finalizer, the deterministic hash of hyperedge ids. */
uint32_t oracle_hash32(uint32_t x);

/* Problem statement: sum over hyperedges of w(e) * (lambda_e - 1); *maxw gets
 * the heaviest part.  Returns the cut. */
int64_t oracle_cut(int32_t n, int32_t e, const int32_t *off, const int32_t *pins,
                   const int32_t *nw, const int32_t *hw, int32_t k, const int32_t *part,
                   int64_t *maxw);

/* Algorithm 1: match[v] = incident hyperedge of highest priority, -1 if none. */
void oracle_match(int32_t n, int32_t e, const int32_t *off, const int32_t *pins,
                  const int32_t *hw, int32_t policy, int32_t *match);

/* Algorithm 2 (one coarsening step).  Caller provides parent[n], and coarse
 * buffers of the fine sizes: c_off[e+1], c_pins[P], c_nw[n], c_hw[e].  The
 * coarse sizes are returned in *cn, *ce. */
void oracle_coarsen(int32_t n, int32_t e, const int32_t *off, const int32_t *pins,
                    const int32_t *nw, const int32_t *hw, int32_t policy,
                    int32_t *parent, int32_t *cn, int32_t *ce, int32_t *c_off,
                    int32_t *c_pins, int32_t *c_nw, int32_t *c_hw);

/* Algorithm 4: move gains for the bisection side[] (0/1). */
void oracle_gains(int32_t n, int32_t e, const int32_t *off, const int32_t *pins,
                  const int32_t *hw, const uint8_t *side, int32_t *gain);

/* Per-side weight bounds of one bisection into k0 : k1 parts with the
 * 32.32 fixed-point factor F = floor((1+eps')*2^32). */
void oracle_bounds(int64_t total_w, int32_t k0, int32_t k1, uint64_t F, int64_t *max0,
                   int64_t *max1);

/* Algorithm 3: initial bisection of the coarsest graph (side[] out). */
void oracle_initial(int32_t n, int32_t e, const int32_t *off, const int32_t *pins,
                    const int32_t *nw, const int32_t *hw, int32_t k0, int32_t k1,
                    uint8_t *side);

/* Algorithm 5 (iters swap rounds, then the balance step); returns 1 when the
 * balance step had to stop with a side still over its bound, else 0. */
int32_t oracle_refine(int32_t n, int32_t e, const int32_t *off, const int32_t *pins,
                      const int32_t *nw, const int32_t *hw, int32_t iters, int64_t max0,
                      int64_t max1, uint8_t *side);

/* Multilevel bisection (Section 2.3 scheme with Algorithms 1-5).  levels_out
 * (nullable) receives the number of coarsening steps taken. */
void oracle_bisect(int32_t n, int32_t e, const int32_t *off, const int32_t *pins,
                   const int32_t *nw, const int32_t *hw, int32_t k0, int32_t k1, uint64_t F,
                   const oracle_params *prm, uint8_t *side, int32_t *levels_out);

/* Fixed-point factor of one bisection for a k-way run with imbalance eps. */
uint64_t oracle_eps_factor(int32_t k, double eps);

/* Full k-way partition (Algorithm 6).  Returns 0 on success, -1 on bad
 * arguments.  part_out[n], cut_out may be NULL. */
int32_t oracle_partition(int32_t n, int32_t e, const int32_t *off, const int32_t *pins,
                         const int32_t *nw, const int32_t *hw, int32_t k, double eps,
                         const oracle_params *prm, int32_t *part_out, int64_t *cut_out);

#ifdef __cplusplus
}
#endif
#endif
