/*
 * upr.h -- C ABI of the MI355X (gfx950) unconstrained partition refinement
 * library, libupr.so.
 *
 * One call of upr_refine_round performs one deterministic synchronous round of
 * penalised unconstrained refinement for balanced k-way graph partitioning
 * (arXiv 2308.15494): build the gain table, pick every node's best penalised
 * move, filter conflicting moves in a fixed (score, id) order, apply the
 * survivors, then rebalance overloaded blocks. Every step runs in HIP kernels
 * on the caller's stream; all arithmetic is integer, so results are exact and
 * independent of launch geometry.
 *
 * Problem statement (Section 2): an undirected graph G = (V, E, c, omega) with
 * node weights c(v) >= 1 and edge weights omega(e) >= 1, a number of blocks k
 * and an imbalance eps > 0. A partition is balanced iff every block weight
 * c(V_i) <= L_max = (1 + eps) * ceil(c(V) / k) (rounded down to an integer).
 * The objective is the edge cut, the total weight of edges between blocks.
 *
 * Conventions for every entry point:
 *  - Pointers marked "device" must be device memory of the context's device
 *    (e.g. torch ROCm tensors). The caller owns all arrays it passes; the
 *    library never frees them and keeps no pointer to them after the call
 *    returns, except that a plan keeps the graph arrays it was created from
 *    (they must outlive the plan and must not change).
 *  - Work is enqueued on `stream` (0 = the null stream). Device outputs are
 *    valid once the stream has been synchronised. Entry points that need a
 *    host decision (the rebalancing loop) synchronise `stream` themselves.
 *  - Return value: UPR_OK (0) or a negative UPR_E_* code; upr_last_error()
 *    then describes it. On an argument error nothing is written.
 *  - A context is not thread-safe: calls on one context must not overlap.
 */
#ifndef UPR_H
#define UPR_H

#include <stdint.h>
#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

#define UPR_OK            0
#define UPR_E_ARG        -1   /* null pointer, bad k / eps / t / tau / mode, size out of range */
#define UPR_E_GRAPH      -2   /* CSR violates the invariants (upr_validate_graph only) */
#define UPR_E_INFEASIBLE -3   /* some node weight exceeds L_max: no balanced partition exists */
#define UPR_E_NOMEM      -4   /* device workspace allocation failed */
#define UPR_E_HIP        -5   /* a HIP runtime call or kernel launch failed */

#define UPR_MAX_K 8192        /* largest supported number of blocks (a gain-table row fits LDS) */
#define UPR_MAX_BATCH_BLOCKS 65536  /* largest graphs-times-k of a batch (sort key width) */

typedef struct upr_ctx upr_ctx;
typedef struct upr_plan upr_plan;
typedef struct upr_batch upr_batch;

/* Graph in symmetric CSR form (Section 2: G = (V, E, c, omega)). */
typedef struct {
    int64_t n;               /* number of nodes, 0 <= n < 2^31 */
    const int64_t *xadj;     /* device [n+1]; xadj[0] = 0, nondecreasing; nnz = xadj[n] */
    const int32_t *adjncy;   /* device [nnz]; row v lists N(v); symmetric, no self-loops,
                                no duplicates; may be NULL when nnz = 0 */
    const int32_t *adjwgt;   /* device [nnz], omega of each directed entry, > 0 and symmetric;
                                NULL means every edge weight is 1 */
    const int32_t *vwgt;     /* device [n], c(v) > 0; NULL means every node weight is 1 */
} upr_graph;

/* Parameters of one round. */
typedef struct {
    int32_t k;                   /* number of blocks, 2 <= k <= UPR_MAX_K */
    int32_t eps_num, eps_den;    /* eps = eps_num / eps_den > 0 (Section 8.1 uses 3/100) */
    int32_t t_num, t_den;        /* availability threshold t in [0, 1] (Section 5.3, 0.7) */
    int32_t tau_num, tau_den;    /* penalty factor tau in [0, 1] of this round (Section 5.5) */
    int32_t mode;                /* 0 penalised unconstrained moves (Section 5.3),
                                    1 constrained (moves that would overload are skipped),
                                    2 penalty-free unconstrained (Section 8.2 variant),
                                    3 limited imbalance (Section 8.2 variant): no penalty,
                                      moves may fill a target up to floor(alpha * L_max) */
    int32_t rebuild_table;       /* 1: conn and block_w are recomputed from part first;
                                    0: conn and block_w are trusted resident state */
    int32_t max_rebalance_iters; /* 0: k+1 for unit node weights, 4k otherwise */
    int32_t seq_penalty;         /* 1: the conflict filter prices each move against its target's
                                    weight as changed by the eligible earlier candidates
                                    (Section 5.3); 0: against the round-start weight only */
    int32_t alpha_num, alpha_den; /* mode 3: alpha = alpha_num / alpha_den >= 1 (the paper
                                    shrinks it from 2 to 1.1 over the rounds); else ignored */
    int32_t variant;             /* bit flags, 0 for the main configuration:
                                    UPR_VAR_OPTIMISTIC: the conflict filter counts an earlier
                                      candidate neighbour in its target block (moved) instead
                                      of the worse of its two blocks;
                                    UPR_VAR_PLAIN_PRIORITY: rebalancing ranks nodes by the
                                      gain alone, without the node weight (Section 8.2);
                                    UPR_VAR_BEST_PREFIX: after the rebalancing, the filtered
                                      and the rebalancing moves form one interleaved sequence
                                      with exact gains, and the round keeps its best balanced
                                      prefix (Section 5.4; single-graph rounds only) */
} upr_params;

#define UPR_VAR_OPTIMISTIC 1
#define UPR_VAR_PLAIN_PRIORITY 2
/* The interleaved sequence (Section 5.4 and the end of Algorithm 1): a node
 * moved by the filter (a -> b) and by the rebalancer (b -> c) makes one move
 * a -> c (none if c = a), placed as its filtered move; the filtered moves in
 * the filter's order, each followed, when it leaves its target b
 * overloaded, by the fewest unused rebalancing moves out of b (in the order
 * they were made: sub-iteration, priority bucket, id) that bring b back to
 * L_max. Gains are recomputed exactly in sequence order; of the boundaries
 * after each filtered move (and its rebalancing moves) that leave every
 * block within L_max, the one with the highest cumulative gain is kept
 * (the earliest on ties) and every other move of the round is undone. With
 * no balanced boundary the round's result stands. */
#define UPR_VAR_BEST_PREFIX 4

/* Round statistics, written to a device int64 array of UPR_STATS_LEN slots. */
enum {
    UPR_ST_LMAX = 0,          /* L_max */
    UPR_ST_CUT_BEFORE,        /* cut of the input partition */
    UPR_ST_CUT_AFTER_MOVES,   /* cut after the filtered moves, before rebalancing */
    UPR_ST_CUT_AFTER,         /* cut of the output partition */
    UPR_ST_CANDIDATES,        /* nodes whose best penalised score was > 0 */
    UPR_ST_ACCEPTED,          /* moves that passed the conflict filter */
    UPR_ST_REBAL_MOVES,       /* moves made by rebalancing */
    UPR_ST_REBAL_ITERS,       /* rebalancing sub-iterations */
    UPR_ST_STATUS,            /* 0 balanced; 1 rebalancing stuck or out of iterations */
    UPR_ST_PREFIX_STEPS,      /* best-prefix rounds: filtered moves kept, -1 if no boundary
                                 was balanced (nothing undone); 0 otherwise */
    UPR_ST_REVERTED,          /* best-prefix rounds: nodes returned to their round-start block */
    UPR_STATS_LEN = 12
};

/* Context: owns the device workspace on one device. Returns UPR_OK or a code.
 * A context serves one call at a time (its workspace is shared by the calls);
 * use one context per host thread or stream for concurrent work. */
int upr_create(upr_ctx **out, int device);
void upr_destroy(upr_ctx *ctx);
/* Message for the last nonzero return on this context (never NULL). */
const char *upr_last_error(const upr_ctx *ctx);

/* Plan: the per-graph preparation of Section 2's input -- weighted degrees
 * omega(I(v)), total node weight c(V), and the hubs: nodes whose adjacency
 * is traversed by several workgroups instead of inside their node tile.
 * Created once per graph; enqueued on
 * `stream` and synchronised. The graph arrays must outlive the plan. */
int upr_plan_create(upr_ctx *ctx, const upr_graph *graph, upr_plan **out, hipStream_t stream);

/* Traversal thresholds of a plan (0 = default: the environment variables
 * UPR_HUB_THRESHOLD / UPR_DIRTY_DIV if set, else 4096 / 16). Nodes of degree
 * above hub_threshold are hubs (split into edge chunks of whole workgroups);
 * the apply rebuilds table tiles instead of atomic deltas once the moving
 * nodes' degrees sum above nnz / dirty_div (from twice that on, or above
 * nnz / UPR_REBUILD_ALL_DIV when set but never below the marking threshold, every tile
 * without marking any). low_threshold is ignored (the
 * apply no longer splits nodes by degree; the field keeps the layout). They
 * change only the speed, never a result; paper_2308_15494_amd/tune.py picks
 * them by timing trial rounds. */
typedef struct {
    int64_t hub_threshold;
    int64_t low_threshold;
    int64_t dirty_div;
} upr_plan_opts;
int upr_plan_create_opts(upr_ctx *ctx, const upr_graph *graph, const upr_plan_opts *opts,
                         upr_plan **out, hipStream_t stream);
/* Frees the plan's device memory. A plan may be destroyed after its context
 * (it is usable only while the context lives). */
void upr_plan_destroy(upr_plan *plan);
/* Host-side facts of a plan (any output pointer may be NULL). */
int upr_plan_info(const upr_plan *plan, int64_t *n, int64_t *nnz, int64_t *total_weight,
                  int64_t *max_degree, int64_t *num_hubs);

/* Check the CSR invariants on the device (xadj monotone, ids in range, no
 * self-loops, rows strictly increasing so no duplicates, symmetric structure
 * and weights, positive weights). Rows must be sorted for this check.
 * Returns UPR_OK or UPR_E_GRAPH with the first violation in upr_last_error.
 * Synchronises `stream`. */
int upr_validate_graph(upr_ctx *ctx, const upr_graph *graph, hipStream_t stream);

/* Gain table (Section 7.1, reused from the shared-memory FM):
 * conn[v * k + j] = omega(v, V_j) for every node v and block j.
 * part: device int32 [n], values in [0, k). conn: device int32 [n * k], out.
 * Checks part first (one stream synchronisation); values outside [0, k)
 * give UPR_E_ARG with nothing written. */
int upr_gain_table(upr_ctx *ctx, const upr_plan *plan, int32_t k, const int32_t *part,
                   int32_t *conn, hipStream_t stream);

/* Block weights c(V_j): block_w device int64 [k], out. Checks part like
 * upr_gain_table. */
int upr_block_weights(upr_ctx *ctx, const upr_plan *plan, int32_t k, const int32_t *part,
                      int64_t *block_w, hipStream_t stream);

/* Edge cut of Section 2, sum over i < j of omega(E_ij), straight from the
 * adjacency: cut device int64 [1], out. */
int upr_edge_cut(upr_ctx *ctx, const upr_plan *plan, const int32_t *part, int64_t *cut,
                 hipStream_t stream);

/* Edge cut without device allocation. For callers that cannot allocate
 * device memory: code under HIP graph capture, tight serving loops and
 * harnesses that forbid hipMalloc. Same result as upr_edge_cut (the
 * Section 2 objective), taken from the graph directly, so no plan is needed:
 * graph: device arrays as in upr_graph (vwgt is not read); part: device
 * int32 [n], any values (only equality is tested); cut: device int64 [1],
 * out. The context is used for its device and its error message only.
 * Scratch: a static device array of 2^18 partial sums per device (2 MiB),
 * one per tile of 1024 nodes, held until the process ends; hence
 * n <= UPR_NOALLOC_MAX_NODES, and a larger n gives UPR_E_ARG with nothing
 * enqueued. Calls no allocating routine; every call on a device shares that
 * device's array, so calls that overlap on one device (other streams or
 * threads) race and must be serialised by the caller. */
#define UPR_NOALLOC_MAX_NODES ((int64_t)1 << 28)
int upr_edge_cut_noalloc(upr_ctx *ctx, const upr_graph *graph, const int32_t *part, int64_t *cut,
                         hipStream_t stream);

/* One refinement round, in place on (part, conn, block_w):
 *   S1 gain table and block weights (if params->rebuild_table), cut;
 *   penalty buckets of the rebalance-available nodes (Section 5.3);
 *   S2 best move per node maximising gain * 2^16 - penalty (Q16 fixed point;
 *      penalty tau * (3/2)^l * c(v), l the least slot covering the target's
 *      excess; moves with no covering slot are forbidden); candidates have a
 *      positive best score;
 *   S3 conflict filter: in (score desc, id asc) order, a candidate survives iff
 *      its gain, recomputed assuming every earlier candidate neighbour ends in
 *      the worse of its two blocks, times 2^16 still exceeds its penalty
 *      (with seq_penalty, the penalty for the target's weight after the
 *      eligible earlier candidates' moves in and out);
 *   S4 apply survivors with delta updates of conn and block_w;
 *   S5 rebalance (Section 7.1) while a block exceeds L_max;
 *   S6 cut and statistics.
 * part: device int32 [n] in/out; conn: device int32 [n * k] in/out;
 * block_w: device int64 [k] in/out; stats: device int64 [UPR_STATS_LEN] out.
 * Synchronises `stream` once per rebalancing decision. A part value outside
 * [0, k) is detected on the device and reported as UPR_E_ARG at the first
 * synchronisation; part, conn and block_w are then unspecified. */
int upr_refine_round(upr_ctx *ctx, const upr_plan *plan, const upr_params *params, int32_t *part,
                     int32_t *conn, int64_t *block_w, int64_t *stats, hipStream_t stream);

/* A schedule of rounds (Section 5.5: one round after another, each with its
 * own penalty factor tau and form): round r = 0 .. rounds - 1 with
 * params[r] (host array), in place on (part, conn, block_w), exactly as
 * `rounds` calls of upr_refine_round but without returning to the caller
 * between them. stats: device int64 [rounds * UPR_STATS_LEN], round r's at
 * r * UPR_STATS_LEN. Stops at the first round that fails and returns its
 * error (the rounds before it stand, later entries of stats are not
 * written). rounds = 0 does nothing. */
int upr_refine_rounds(upr_ctx *ctx, const upr_plan *plan, const upr_params *params, int32_t rounds,
                      int32_t *part, int32_t *conn, int64_t *block_w, int64_t *stats,
                      hipStream_t stream);

/* Rebalancing alone (Section 7.1): S1 if params->rebuild_table, then S5 and
 * S6. Same arrays as upr_refine_round; mode and tau are ignored. */
int upr_rebalance(upr_ctx *ctx, const upr_plan *plan, const upr_params *params, int32_t *part,
                  int32_t *conn, int64_t *block_w, int64_t *stats, hipStream_t stream);

/* Per-node results of the last round's move phase on this context, copied to
 * device arrays of length n (any may be NULL): target block of each candidate
 * (-1 otherwise), its score, its penalty, and whether it passed the filter.
 * Valid until the next call on the context. For diagnosis. */
int upr_last_moves(upr_ctx *ctx, int64_t n, int32_t *target, int64_t *score, int64_t *pen,
                   uint8_t *accept, hipStream_t stream);

/* Batches: many independent graphs refined by the same kernel launches.
 *
 * The batch holds the disjoint union of ng graphs with a common k and eps:
 * node v of graph g is node off[g] + v of the union (off from
 * upr_batch_info), and the union is refined as one graph whose blocks are
 * numbered globally: block j of graph g is g * k + j. Each graph keeps its
 * own L_max (from its own total node weight), its own penalty factor tau and
 * its own statistics, and no kernel lets two graphs interact, so every
 * graph's results are exactly those of upr_refine_round on it alone.
 * upr_batch_create copies the graphs into the union (the inputs may be
 * freed afterwards) and plans it; it validates like upr_plan_create, plus
 * that every graph names only its own nodes (unless trusted, below).
 * Enqueued on `stream` and synchronised. ng * k <= UPR_MAX_BATCH_BLOCKS. */
int upr_batch_create(upr_ctx *ctx, const upr_graph *graphs, const int64_t *nnz, int32_t ng,
                     int32_t k, int32_t eps_num, int32_t eps_den, int32_t flags,
                     const upr_plan_opts *opts, upr_batch **out, hipStream_t stream);
/* upr_batch_create arguments: nnz, a host array [ng] of each graph's xadj[n]
 * (or NULL to read them from the device); flags: 0, or UPR_BATCH_TRUSTED when
 * every graph has passed upr_validate_graph or an earlier batch (a server
 * rebuilding batches of admitted graphs): the checks are skipped; opts: the
 * union's plan thresholds (may be NULL). */
#define UPR_BATCH_TRUSTED 1
/* Frees the batch; like a plan, it may be destroyed after its context. */
void upr_batch_destroy(upr_batch *batch);
/* Union size, node offsets off[ng + 1] and L_max[ng] (any pointer may be NULL). */
int upr_batch_info(const upr_batch *batch, int64_t *n_total, int64_t *nnz_total, int64_t *node_off,
                   int64_t *lmax);
/* One round of every graph of the batch (the steps of upr_refine_round).
 * params: k and eps must be the batch's; tau_num / tau_den: host arrays [ng]
 * with each graph's penalty factor, or both NULL for params->tau everywhere.
 * part: device int32 [n_total], global block ids (graph g's nodes hold values
 * in [g*k, g*k + k)); conn: device int32 [n_total * k], row v indexed by the
 * local block j; block_w: device int64 [ng * k], indexed by global block;
 * stats: device int64 [ng * UPR_STATS_LEN], graph g's statistics at
 * g * UPR_STATS_LEN. A part value outside its graph's range is reported as
 * UPR_E_ARG. Rebalancing stops per graph as in upr_refine_round; the call
 * synchronises once per sub-iteration of the slowest graph. */
int upr_batch_refine_round(upr_ctx *ctx, upr_batch *batch, const upr_params *params,
                           const int32_t *tau_num, const int32_t *tau_den, int32_t *part,
                           int32_t *conn, int64_t *block_w, int64_t *stats, hipStream_t stream);
/* Carry graphs' round state between batches on the device, for a server
 * that rebuilds its batch when membership changes: for every graph g of
 * dst with src_index[g] >= 0 (host int32 [dst's ng]), graph src_index[g] of
 * src -- the same graph, same node count and k -- has its partition copied
 * (block ids renumbered from its old to its new global range), its table
 * rows and its block weights. Graphs with src_index[g] < 0 are not touched.
 * src_part / src_conn / src_block_w and the dst arrays: the device state
 * arrays of the two batches, laid out as for upr_batch_refine_round.
 * Enqueued on `stream`; the arrays of src must stay valid until it has run. */
int upr_batch_carry(upr_ctx *ctx, const upr_batch *src, const int32_t *src_part,
                    const int32_t *src_conn, const int64_t *src_block_w, const upr_batch *dst,
                    const int32_t *src_index, int32_t *dst_part, int32_t *dst_conn,
                    int64_t *dst_block_w, hipStream_t stream);
/* Rebalancing alone of every graph of the batch (as upr_rebalance). */
int upr_batch_rebalance(upr_ctx *ctx, upr_batch *batch, const upr_params *params, int32_t *part,
                        int32_t *conn, int64_t *block_w, int64_t *stats, hipStream_t stream);

/* Refinement driver: the rounds around the round (Sections 5.5 and 6).
 *   Label propagation: penalty-free rounds (mode 2) on an active set, which
 *   starts as the boundary nodes (a neighbour in another block) and then holds
 *   every node that did not move and has a neighbour that moved; a round that
 *   does not lower the cut (rebalancing included) is rolled back and ends the
 *   phase, as do lp_rounds rounds, an empty active set, or an improvement
 *   below lp_min (a fraction of the cut before the round).
 *   FM: at most fm_rounds rounds; penalised (mode 0) while unconstrained, with
 *   tau rising linearly from tau_1 to 1 over fm_rounds - 1 rounds; a round that
 *   improves by less than fm_switch (a fraction of its starting cut) switches
 *   to constrained rounds (mode 1), which stop at the first one that improves
 *   by less than fm_switch; the last round of the budget is always
 *   constrained. Every round rebuilds the table. */
typedef struct {
    int32_t k, eps_num, eps_den, t_num, t_den;  /* as in upr_params */
    int32_t lp_rounds;                         /* paper: 5 */
    int32_t lp_min_num, lp_min_den;            /* paper: 1/1000 */
    int32_t fm_rounds;                         /* e.g. 10 */
    int32_t tau1_num, tau1_den;                /* tau_1, e.g. 1/2 */
    int32_t fm_switch_num, fm_switch_den;      /* paper: 2/1000 */
    int32_t seq_penalty;                       /* as in upr_params */
} upr_driver;

/* Kinds of the driver's log entries. */
enum { UPR_LOG_LP = 0, UPR_LOG_ROLLBACK = 1, UPR_LOG_UNCONSTRAINED = 2, UPR_LOG_CONSTRAINED = 3 };

/* Run the driver in place on (part, conn, block_w) of one graph. log_stats:
 * device int64 [(lp_rounds + 1 + fm_rounds) * UPR_STATS_LEN], one entry per
 * round (a rollback repeats the rolled-back round's entry); log_kind: host
 * int32 of the same count; *n_log: host, entries written. conn and block_w
 * end consistent with part. Synchronises `stream` after every round. */
int upr_refine(upr_ctx *ctx, const upr_plan *plan, const upr_driver *driver, int32_t *part,
               int32_t *conn, int64_t *block_w, int64_t *log_stats, int32_t *log_kind,
               int32_t *n_log, hipStream_t stream);

/* Host-side helpers (no device work). */
/* L_max = floor((1 + eps) * ceil(total / k)) with eps = eps_num / eps_den. */
int64_t upr_lmax(int64_t total, int32_t k, int32_t eps_num, int32_t eps_den);
/* Best move decides a node of degree <= this bound from its adjacency, every
 * other node from its table row (the same result either way), for a graph
 * with k blocks and the given largest degree; 0: every node from its row.
 * The environment variable UPR_ADJ_DEG overrides the bound (at most 16). */
int32_t upr_best_move_adjacency_degree(int32_t k, int64_t max_degree);
/* Q16 penalty factors floor(tau * (3/2)^l * 2^16), l = 0..53, into out[54]. */
int upr_penalty_table(int32_t tau_num, int32_t tau_den, int64_t *out);

/* Captured move phases, for callers that run many rounds of one
 * configuration: with enable != 0, a round's kernels from the partition
 * copies to the cut after the filtered moves (S1 to S4) are captured into a
 * HIP graph on the context's own stream the first time a configuration is
 * seen, and replayed from it afterwards; the round's first kernel (which
 * holds the round's penalty factors) and the rebalancing stay eager. A
 * configuration is the plan, k, eps, t, mode, rebuild_table, seq_penalty,
 * variant, alpha and the part / conn / block_w arrays (a graph replays the
 * kernel arguments it was captured with; a batch is keyed by its own plan,
 * its per-graph penalty factors stay eager). Used for single graphs and
 * batches, without the best prefix, without an activity mask (the driver's
 * label-propagation rounds), with the segment path of the sequence-aware
 * price and with phase timing off; every other round runs eagerly. Results are identical either
 * way. At most 16 graphs are kept per context; they are freed when the
 * workspace grows, when capture is disabled (which synchronises the device)
 * and by upr_destroy. */
int upr_capture_enable(upr_ctx *ctx, int enable);

/* Per-phase device time of the calls on this context, accumulated in
 * milliseconds by HIP events while timing is enabled (each timed phase
 * records two events on the call's stream). Phases: 0 gain table,
 * 1 penalty buckets, 2 best move, 3 filter, 4 apply, 5 rebalance, 6 cut,
 * 7 whole call, 8 the best-move kernel alone, 9 the filter's edge-tile
 * kernel alone. Phase 0 is the gain-table kernel (its tiles and the hubs'
 * edge chunks), 1 the node statistics and penalty buckets, 2 the bucket
 * prefix sums and the best-move kernel, 3 the whole conflict filter (edge
 * tiles, hub chunks, sequence-aware price), 4 the apply of the filtered
 * moves (table deltas or tile rebuilds included).
 * phase_mask: bit p times phase p (0 = off, UPR_TIMING_ALL = every phase).
 * ms and counts: arrays of UPR_NUM_PHASES; counts[p] = number of intervals
 * accumulated. */
#define UPR_NUM_PHASES 10
#define UPR_TIMING_ALL 0x3FF
int upr_timing_enable(upr_ctx *ctx, int phase_mask);
int upr_timing_read(upr_ctx *ctx, double *ms, int64_t *counts, int reset);

#ifdef __cplusplus
}
#endif

#endif /* UPR_H */
