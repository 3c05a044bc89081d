/*
 * bipart.h - C ABI of the MI355X (gfx950) implementation of BiPart's
 * deterministic multilevel hypergraph partitioner (Maleki, Agarwal,
 * Burtscher, Pingali, "BiPart: A Parallel and Deterministic Multilevel
 * Hypergraph Partitioner", PPoPP 2021).
 *
 * The problem (Section 1.1): given a hypergraph G = (V, E) with node weights
 * and hyperedge weights, k >= 1 and an imbalance eps >= 0, find a partition of
 * V into k parts, each of weight at most (1 + eps) * W / k, minimising
 * cut(G, P) = sum over hyperedges of w(e) * (lambda_e - 1), where lambda_e is
 * the number of parts hyperedge e touches.  The method (Section 3) is a
 * multilevel bisection - multi-node matching and contraction (Algorithms 1
 * and 2), initial bisection of the coarsest graph (Algorithms 3 and 4),
 * projection with parallel swap refinement and a balance step (Algorithm 5)
 * - applied as a nested recursive bisection for k parts (Algorithm 6).
 *
 * The result is fully deterministic: the same input and parameters give the
 * same partition on every run, for every launch configuration, and whether a
 * graph is partitioned alone or inside a batch.
 *
 * Conventions for every entry point:
 *   - Hypergraphs are CSR over hyperedges (bp_hypergraph).  Node ids are
 *     0..num_nodes-1, hyperedge ids 0..num_hedges-1 in input order.
 *   - The caller owns every buffer passed in or out.  The library never keeps
 *     a caller pointer after the call returns.
 *   - "host" pointers are ordinary CPU memory; "device" pointers are HIP
 *     device memory of the current device.  Device entry points take the HIP
 *     stream (hipStream_t) as a void*; NULL means the null stream.  Their
 *     outputs are complete when the call returns unless stated otherwise.
 *   - Every entry point returns a bp_status: 0 success, > 0 warning (outputs
 *     valid), < 0 error (outputs unspecified).  bp_status_string() names a
 *     code; bp_last_error() gives the detail of the calling thread's last
 *     error (for BP_ERR_DEVICE it holds the HIP error text).
 *   - Entry points are thread-safe; concurrent calls use separate memory.
 */
#ifndef BIPART_H
#define BIPART_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t bp_status;

#define BP_OK                   0
#define BP_WARN_IMBALANCED      1  /* valid partition, but a part exceeds (1+eps)W/k        */
#define BP_ERR_INVALID_ARG     -1  /* k < 1, eps < 0 or NaN, NULL required pointer, ...    */
#define BP_ERR_INVALID_CSR     -2  /* offsets not monotone, pin out of range, repeated pin */
#define BP_ERR_WEIGHT_OVERFLOW -3  /* negative weight, or a weight sum >= 2^31            */
#define BP_ERR_OUT_OF_MEMORY   -4  /* device allocation failed                             */
#define BP_ERR_DEVICE          -5  /* HIP runtime error (text in bp_last_error)            */
#define BP_ERR_REJECTED        -6  /* server: request footprint above the memory budget    */
#define BP_ERR_SHUTDOWN        -7  /* server: destroyed before the request completed       */
#define BP_ERR_NOT_FOUND       -8  /* server: unknown ticket                               */

/* Matching policies of Table 1 (priority of a hyperedge in Algorithm 1). */
#define BP_LDH  0  /* lower degree first (default)    */
#define BP_HDH  1  /* higher degree first             */
#define BP_LWD  2  /* lower hyperedge weight first    */
#define BP_HWD  3  /* higher hyperedge weight first   */
#define BP_RAND 4  /* hash of the hyperedge id        */

/*
 * A hypergraph in CSR form.
 *   hedge_offsets[num_hedges+1]: hedge_offsets[0] = 0, non-decreasing; the
 *       pins of hyperedge e are pins[hedge_offsets[e] .. hedge_offsets[e+1]).
 *   pins[P], P = hedge_offsets[num_hedges] < 2^31: node ids in [0, num_nodes),
 *       no node twice in one hyperedge; any order within a hyperedge.
 *   node_weights[num_nodes]: >= 0, sum < 2^31; NULL means all 1.
 *   hedge_weights[num_hedges]: >= 0, sum < 2^31; NULL means all 1.
 * Hyperedges with fewer than two pins are allowed; they can never be cut.
 */
typedef struct {
    int32_t num_nodes;
    int32_t num_hedges;
    const int32_t *hedge_offsets;
    const int32_t *pins;
    const int32_t *node_weights;
    const int32_t *hedge_weights;
} bp_hypergraph;

/*
 * Tuning parameters of Section 3.4.
 *   policy: BP_LDH .. BP_RAND (Table 1).
 *   max_levels: at most this many coarsening steps per bisection (25).
 *   refine_iters: swap rounds per level in Algorithm 5 (2).
 *   min_coarse_nodes: stop coarsening a graph once it has at most this many
 *       nodes (100; 0 coarsens until no hyperedge is left or max_levels).
 */
typedef struct {
    int32_t policy;
    int32_t max_levels;
    int32_t refine_iters;
    int32_t min_coarse_nodes;
} bp_params;

/* Optional result details. */
typedef struct {
    int64_t cut;               /* connectivity-1 cut (problem statement)      */
    int64_t max_part_weight;   /* heaviest part                               */
    int64_t part_weight_limit; /* max(ceil(W/k), floor((1+eps) W / k))        */
    int32_t balanced;          /* max_part_weight <= part_weight_limit         */
    int32_t tree_levels;       /* bisection tree depth, ceil(log2 k)          */
    int32_t bisections;        /* bisection problems solved                   */
    int32_t coarsen_levels;    /* coarsening steps of the first bisection      */
    int64_t pins_coarsened;    /* sum of pins over every level coarsened      */
    int64_t pins_refined;      /* sum of pins over every gain evaluation      */
    int32_t host_syncs;        /* device-to-host waits the call needed        */
    int32_t kernel_launches;   /* kernels launched by the call                */
    int64_t device_bytes;      /* device memory the call held at its end      */
    int32_t levels[64];        /* per bisection-tree level t < 64: the most
                                  coarsening steps of its bisections (the whole
                                  run's for the batched form)                 */
    double imbalance;          /* max_part_weight * k / W - 1 (0 when W = 0)   */
    int32_t graph_replays;     /* rounds replayed from captured graphs          */
    int32_t reserved;
} bp_report;

/* Fills *p with the defaults listed above. */
void bp_default_params(bp_params *p);

/* Name of a status code (static string). */
const char *bp_status_string(bp_status s);

/* Detail of the calling thread's most recent error ("" if none). */
const char *bp_last_error(void);

/*
 * k-way partition of a host hypergraph (Sections 1.1 and 3, Algorithm 6).
 * hg: host pointers as in bp_hypergraph.  k >= 1; eps >= 0.
 * params: NULL for the defaults.  part_out: host int32[num_nodes], receives
 * part ids in [0, k).  Part ids follow the bisection tree: for a sub-problem
 * owning parts [lo, lo+k'), side 0 of its bisection gets [lo, lo+ceil(k'/2)).
 * cut_out (nullable): the connectivity-1 cut.  report (nullable).
 * Input is validated on the host (all BP_ERR_INVALID_* / OVERFLOW checks,
 * including repeated pins) and copied to the device; the partition runs on
 * the current HIP device.  Returns BP_WARN_IMBALANCED when the result
 * violates the balance constraint (possible only with heavy nodes).
 */
bp_status bp_partition(const bp_hypergraph *hg, int32_t k, double eps, const bp_params *params,
                       int32_t *part_out, int64_t *cut_out, bp_report *report);

/*
 * Same as bp_partition for a hypergraph already in device memory.
 * hg: the struct itself is host memory, its arrays are device pointers.
 * d_part_out: device int32[num_nodes].  cut_out (nullable): host int64.
 * stream: hipStream_t the work is ordered on.  The call validates offsets,
 * pin ranges and weight sums on the device; a hyperedge listing a node twice
 * is NOT detected here (bp_partition checks it) and gives an unspecified but
 * memory-safe result.
 */
bp_status bp_partition_device(const bp_hypergraph *hg, int32_t k, double eps,
                              const bp_params *params, int32_t *d_part_out, int64_t *cut_out,
                              bp_report *report, void *stream);

/*
 * For callers that cannot allocate device memory (code under stream capture,
 * tight serving loops, harnesses that forbid allocation): bp_partition_device
 * with every device buffer of the call inside a fixed 256 MiB workspace that
 * the library holds per device (a static device array, allocated when the
 * library's code is loaded on that device and kept until the process ends).
 * The call itself allocates no device memory (no hipMalloc/hipFree); its
 * first call on a device only looks up that device's workspace address.
 * Arguments, outputs and results are those of bp_partition_device.  Inputs
 * whose workspace bound (bp_request_footprint of their sizes) exceeds the
 * workspace are refused with BP_ERR_OUT_OF_MEMORY before any work is queued.
 * Calls on one device share its workspace: they run one at a time (a lock is
 * held until the call's stream has drained), so calls that overlap in time
 * on one device wait for each other rather than race.
 */
bp_status bp_partition_device_noalloc(const bp_hypergraph *hg, int32_t k, double eps,
                                      const bp_params *params, int32_t *d_part_out, int64_t *cut_out,
                                      bp_report *report, void *stream);

/*
 * Device memory: each call works in an arena of device memory that is kept,
 * per device, for the next call (steady calls allocate nothing).  A call that
 * used less than a quarter of its arena (and the arena holds over 1 GiB)
 * frees the excess when it ends.  bp_release_memory frees every arena of the
 * current device that no call is using; later calls allocate again.
 */
bp_status bp_release_memory(void);

/* Caps the device memory one call's arena may hold at `bytes` (0 = no cap,
 * the default; process-wide).  A call that would need more fails with
 * BP_ERR_OUT_OF_MEMORY and leaves the library usable.  BP_ERR_INVALID_ARG for
 * a negative value. */
bp_status bp_set_memory_limit(int64_t bytes);

/*
 * Batched form: n independent hypergraphs partitioned in ONE device run.  All
 * graphs are segments of the same levels (the nested scheme of Algorithm 6
 * with every graph as a root bisection), so the launch sequence and the
 * host-device round trips are shared by the whole batch.
 * graphs, k, eps: host arrays of n entries, each as for bp_partition (host
 * pointers inside graphs[g]).  part_out: host array of n host pointers,
 * part_out[g] receives int32[graphs[g].num_nodes] (may be NULL for a graph
 * without nodes).  cut_out (nullable): host int64[n].  reports (nullable):
 * host bp_report[n]; cut, max_part_weight, part_weight_limit and balanced are
 * the graph's own, the counters (tree_levels ... kernel_launches) are those of
 * the whole batch run.
 * Every graph gets exactly the partition and cut bp_partition gives it alone.
 * Returns BP_WARN_IMBALANCED if any graph's result is imbalanced; on an
 * invalid graph returns its error and bp_last_error() names the graph index.
 * n = 0 is valid; n <= 65535, and the batch's node, hyperedge and pin totals
 * must each stay below 2^31.
 */
bp_status bp_partition_batch(int32_t n, const bp_hypergraph *graphs, const int32_t *k, const double *eps,
                             const bp_params *params, int32_t *const *part_out, int64_t *cut_out,
                             bp_report *reports);

/*
 * Same for graphs already in device memory: the structs and the k, eps,
 * d_part_out and output arrays are host memory; the arrays inside graphs[g]
 * and the d_part_out[g] buffers are device memory.  Validation as in
 * bp_partition_device (repeated pins are not detected).  Ordered on stream;
 * outputs are complete on return.
 */
bp_status bp_partition_batch_device(int32_t n, const bp_hypergraph *graphs, const int32_t *k,
                                    const double *eps, const bp_params *params,
                                    int32_t *const *d_part_out, int64_t *cut_out, bp_report *reports,
                                    void *stream);

/* ---- launch schedule --------------------------------------------------------
 *
 * Knobs of how the work is laid out on the device.  They never change a
 * result - every schedule gives the same partitions and cuts (tested) - only
 * the time.  Process-wide; a call uses the schedule current when it starts.
 */
typedef struct {
    int32_t incremental_min_pins;  /* levels with at least this many pins plus nodes (a full gain
                                      pass reads both) update balance-round gains
                                      from the moves; INT32_MAX: always recompute (default 65536) */
    int32_t seg_select_max_nodes;  /* levels whose segments all have at most this many nodes select
                                      and move in one workgroup per segment (capped at 16384 for
                                      swaps, 32768 for balance); 0: never (default 16384) */
    int32_t round_chunk_max;       /* most rounds issued between host checks, 1..64 (default 32) */
    int32_t fused_pick_lists;      /* up to this many lists the digit picks run in the histogram
                                      launch's last workgroup, above in per-segment ones,
                                      0..4096 (default 8) */
    int32_t fuse_max_pins;         /* segments of at most 8192 nodes and this many pins run their
                                      whole balance step in one workgroup, with no launch per
                                      round; 0: never (default 131072) */
    int32_t chunk_select_max_nodes; /* levels too large for the one-workgroup selection whose
                                      segments all have at most this many nodes (capped at
                                      262144) select each balance round's nodes in chunks of
                                      16384 nodes, one workgroup each, merged per segment;
                                      0: never (default 262144) */
    int32_t graph_rounds;          /* 1: a level's later rounds (from the seventh) are replayed
                                      from three captured hipGraphs instead of launched one
                                      kernel at a time; 0: launched (default 0) */
} bp_schedule;

/* Fills *s with the defaults above. */
void bp_schedule_default(bp_schedule *s);
/* Makes *s the process-wide schedule (BP_ERR_INVALID_ARG if out of range). */
bp_status bp_schedule_set(const bp_schedule *s);
/* Copies the process-wide schedule into *s. */
bp_status bp_schedule_get(bp_schedule *s);

/*
 * Autotuner for the batched form: partitions the batch (as
 * bp_partition_batch_device) under each candidate schedule, trials times
 * each (>= 1), checks that every candidate gives exactly the partitions and
 * cuts of the current schedule (BP_ERR_DEVICE if not - never expected), and
 * writes the fastest schedule to *best and its best time (ms) to *best_ms.
 * The process-wide schedule is left as it was; pass *best to
 * bp_schedule_set to use it.  d_scratch_parts: device int32 buffers, one per
 * graph, for the candidate runs' outputs (caller-owned).
 */
bp_status bp_autotune_batch_device(int32_t n, const bp_hypergraph *graphs, const int32_t *k, const double *eps,
                                   const bp_params *params, int32_t *const *d_scratch_parts, int32_t trials,
                                   bp_schedule *best, double *best_ms, void *stream);

/* ---- served form ----------------------------------------------------------
 *
 * A server owns `workers` worker threads on one device, each with its own
 * stream and device memory, so that runs overlap on the device.  Requests
 * are submitted one at a time from any thread.  A free worker starts a run
 * at once with the oldest queued requests: the first one, then the next ones
 * while the run stays under max_run_pins input pins and max_slots requests,
 * and while the footprint estimates (bp_request_footprint) of all runs in
 * flight stay within hbm_budget_bytes; when the oldest request does not fit
 * beside the runs in flight, the worker waits for one to end.  A request
 * that arrives while others run therefore starts as soon as a worker and
 * memory are free, and a small request does not wait behind a large one
 * already running.  Each run partitions its requests as one batch (see
 * bp_partition_batch).  A request whose own estimate exceeds the budget is
 * refused at submission with BP_ERR_REJECTED.  Every result equals
 * bp_partition of that request alone.
 */
typedef struct bp_server bp_server;

typedef struct {
    int64_t hbm_budget_bytes;   /* > 0: device bytes the runs in flight may need together        */
    int32_t max_slots;          /* >= 1: most requests per run                                  */
    int32_t max_batch_delay_us; /* >= 0: after the oldest queued request arrived, wait up to this
                                   long for more before starting a run (0: start at once)      */
    int32_t device;             /* HIP device id the workers use                               */
    int32_t workers;            /* 1..16: runs in flight at once (default 4)                   */
    bp_params params;           /* partitioner parameters for every request                    */
    int64_t max_run_pins;       /* >= 1: a run takes further requests only while its input pins
                                   stay at or below this (default 4194304)                     */
} bp_server_config;

typedef struct {
    int64_t cut, max_part_weight, part_weight_limit; /* as in bp_report               */
    int32_t balanced;
    int32_t batch_size;         /* requests in the run that served this one          */
    int64_t footprint_bytes;    /* the admission estimate                            */
    double queue_ms;            /* submission to the start of its run                */
    double run_ms;              /* start of its run to results on the host           */
    double latency_ms;          /* submission to results on the host                 */
} bp_req_stats;

/* Defaults: 64 GiB budget, 256 slots, no batching delay, device 0, 4 workers,
 * 4194304 pins per run, default params. */
void bp_server_default_config(bp_server_config *cfg);

/* Footprint estimate (device bytes) of one partition of a hypergraph with
 * the given sizes and k; an upper bound of the memory the call holds. */
bp_status bp_request_footprint(int32_t num_nodes, int32_t num_hedges, int64_t num_pins, int32_t k,
                               int64_t *bytes);

/* Starts a server (its worker sets up the device lazily; a device failure
 * is reported by every request as BP_ERR_DEVICE).  *out receives the handle. */
bp_status bp_server_create(const bp_server_config *cfg, bp_server **out);

/* Validates and copies a host hypergraph (as bp_partition) and queues it.
 * Returns at once with *ticket; BP_ERR_REJECTED if its footprint estimate is
 * above the budget; BP_ERR_SHUTDOWN once destroy has begun.  Thread-safe. */
bp_status bp_server_submit(bp_server *srv, const bp_hypergraph *hg, int32_t k, double eps, uint64_t *ticket);

/* Blocks until the request is done, then copies its part ids to part_out
 * (host int32[num_nodes], nullable), its cut to *cut_out (nullable) and its
 * timings to *stats (nullable).  Returns the request's status: BP_OK or
 * BP_WARN_IMBALANCED, BP_ERR_SHUTDOWN if the server was destroyed before it
 * ran, BP_ERR_DEVICE on a device failure, BP_ERR_NOT_FOUND for a ticket
 * never issued or already collected.  Each ticket is collected once.
 * Thread-safe; must not be called after bp_server_destroy has returned. */
bp_status bp_server_wait(bp_server *srv, uint64_t ticket, int32_t *part_out, int64_t *cut_out,
                         bp_req_stats *stats);

/* Stops the server: the run in progress completes, requests still queued
 * complete with BP_ERR_SHUTDOWN, threads blocked in bp_server_wait return,
 * then every resource is freed. */
bp_status bp_server_destroy(bp_server *srv);

/*
 * Connectivity-1 cut and heaviest part of a given partition (problem
 * statement, Section 1.1), computed on the device.  Host pointers; part[v] in
 * [0, k).  cut and max_part_weight are host outputs (nullable).
 */
bp_status bp_compute_cut(const bp_hypergraph *hg, int32_t k, const int32_t *part, int64_t *cut,
                         int64_t *max_part_weight);

/* Same for device pointers (hg arrays and d_part); outputs are host values. */
bp_status bp_compute_cut_device(const bp_hypergraph *hg, int32_t k, const int32_t *d_part,
                                int64_t *cut, int64_t *max_part_weight, void *stream);

/* ---- single steps, for step-by-step checking (device pointers) ----------- */

/*
 * Algorithm 1: d_match[v] = the incident hyperedge of highest priority
 * (policy of Table 1, ties by the hash of the hyperedge id), -1 if v has no
 * hyperedge.  hg: device arrays.
 */
bp_status bp_step_match(const bp_hypergraph *hg, int32_t policy, int32_t *d_match, void *stream);

/*
 * Algorithm 2: one coarsening step.  Outputs (device, caller-allocated at the
 * fine sizes): d_parent[num_nodes], d_coarse_offsets[num_hedges+1],
 * d_coarse_pins[P], d_coarse_node_w[num_nodes], d_coarse_hedge_w[num_hedges];
 * *coarse_nodes, *coarse_hedges (host) receive the coarse sizes.  Coarse
 * nodes are numbered by the smallest fine id they contain; coarse hyperedges
 * hold their sorted distinct parent ids, appear in source order, and identical
 * ones are merged with summed weight.
 */
bp_status bp_step_coarsen(const bp_hypergraph *hg, int32_t policy, int32_t *d_parent,
                          int32_t *d_coarse_offsets, int32_t *d_coarse_pins,
                          int32_t *d_coarse_node_w, int32_t *d_coarse_hedge_w,
                          int32_t *coarse_nodes, int32_t *coarse_hedges, void *stream);

/* Algorithm 4: d_gain[v] for the bisection d_side[v] in {0,1} (device). */
bp_status bp_step_gains(const bp_hypergraph *hg, const uint8_t *d_side, int32_t *d_gain,
                        void *stream);

/* Algorithm 3: initial bisection into k0 : k1 shares, d_side[num_nodes] out. */
bp_status bp_step_initial(const bp_hypergraph *hg, int32_t k0, int32_t k1, uint8_t *d_side,
                          void *stream);

/*
 * Algorithm 5 on one level: iters swap rounds then the balance step against
 * the side bounds max0/max1.  d_side is updated in place.  *stuck (host,
 * nullable) is 1 when balancing had to stop with a side over its bound.
 */
bp_status bp_step_refine(const bp_hypergraph *hg, int32_t iters, int64_t max0, int64_t max1,
                         uint8_t *d_side, int32_t *stuck, void *stream);

/*
 * One multilevel bisection into k0 : k1 shares with the 32.32 fixed-point
 * imbalance factor F = floor((1+eps')*2^32): coarsen, initial bisection,
 * project and refine.  d_side out; *levels (host, nullable) = steps taken.
 */
bp_status bp_step_bisect(const bp_hypergraph *hg, int32_t k0, int32_t k1, uint64_t F,
                         const bp_params *params, uint8_t *d_side, int32_t *levels,
                         void *stream);

/* ---- kernel timing (diagnostics) ------------------------------------------ */

typedef struct {
    char name[40];      /* kernel family                                   */
    int64_t launches;   /* launches timed                                  */
    double total_ms;    /* summed device time of those launches (hipEvents) */
    double bytes;       /* summed algorithmic bytes of those launches      */
} bp_kernel_stat;

/* Enables (1) or disables (0) per-launch hipEvent timing of every kernel
 * family on the launching stream.  Off by default; adds a small overhead. */
void bp_profile_enable(int32_t on);
/* Clears the accumulated statistics. */
void bp_profile_reset(void);
/* Copies up to cap entries into out (host) and returns how many exist. */
int32_t bp_profile_read(bp_kernel_stat *out, int32_t cap);
/* Launches n empty kernels on stream, timed like every other launch under
 * the family "event_floor": the per-launch cost of the event timing itself,
 * to be set against the timings of short kernels. */
bp_status bp_profile_floor(int32_t n, void *stream);

#ifdef __cplusplus
}
#endif
#endif /* BIPART_H */
