/*
 * CPU ORACLE for one synchronous round of penalised unconstrained refinement
 * for balanced k-way graph partitioning (arXiv 2308.15494).
 *
 * TEST INFRASTRUCTURE ONLY. Nothing in the product path may call, link or
 * load this file: only the tests, the smoke check and the CPU-baseline leg of
 * the benchmark do. It is deliberately plain: one thread, straight loops,
 * qsort where an order is needed, exact integer arithmetic (unsigned __int128
 * where a product can exceed 64 bits), no blocking, fusion or reordering
 * beyond what the definitions state. It shares no code or header with the GPU
 * library.
 *
 * Notation follows Section 2 (Preliminaries): G = (V, E, c, omega), k blocks,
 * Pi(v) the block of v, omega(v, V_j) the edge weight from v into block j
 * ("conn[v][j]", the gain table), omega(I(v)) the weighted degree ("wdeg"),
 * c(V_j) the block weight ("W[j]"), L_max = (1+eps) * ceil(c(V)/k).
 *
 * The paper's refinement (localized parallel FM with multi-queue rebalancing,
 * Sections 5 and 7) is nondeterministic. The round computed here is the
 * deterministic synchronous form of it, with every open choice fixed:
 *
 *   S0  L_max, penalty table PENQ[l] = floor(tau * (3/2)^l * 2^16)
 *   S1  gain table and block weights from the partition; cut_before
 *   S1b rebalance-available set V_r (t = t_num/t_den), slots, bucket
 *       weights c(B_{l,j}) and their prefix sums (Section 5.3)
 *   S2  per node, the target block maximising
 *          s(v,j) = (omega(v,V_j) - omega(v,V_a)) * 2^16 - P(v,j)
 *       where P is the Section 5.3 penalty in Q16 fixed point; a node is a
 *       candidate iff the best s is > 0 (label-propagation style positive
 *       moves, Section 6)
 *   S3  conflict filter: order candidates by (s desc, id asc); for each
 *       candidate recompute a pessimistic gain assuming every earlier
 *       candidate neighbour ends in whichever of its two blocks is worse for
 *       this move (the candidate is eligible if that gain is > 0); with the
 *       sequence-aware penalty, price the move against its target's weight
 *       as changed by the eligible earlier candidates: plus those moving in,
 *       minus those moving out unless they are available for rebalancing
 *       (Section 5.3 prices a move by c(V_j + u) + c~_j when it is made, and
 *       c~_j keeps the weight of available nodes that left; Lemma 1 sums
 *       pen(u_i, V_1 + U^{i-1})); accept iff gain * 2^16 - P > 0.
 *       Applying the accepted moves one by one in that order lowers the
 *       cut at every step.
 *   S4  apply accepted moves; delta-update the gain table and block weights
 *   S5  rebalance (Section 7.1) in synchronous sub-iterations
 *   S6  final cut and statistics
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define ORC_SLOTS 54               /* slots 0..53; 1.5^53 > 2^31 covers any int32 ratio */
#define ORC_RB_BUCKETS (2 * ORC_SLOTS + 1)
#define ORC_PEN_CAP ((int64_t)1 << 62)

typedef unsigned __int128 u128;

typedef struct {
    int64_t n;
    const int64_t *xadj;
    const int32_t *adjncy;
    const int32_t *adjwgt; /* NULL: every edge weight is 1 */
    const int32_t *vwgt;   /* NULL: every node weight is 1 */
} orc_graph;

typedef struct {
    int32_t k;
    int32_t eps_num, eps_den;
    int32_t t_num, t_den;
    int32_t tau_num, tau_den;
    int32_t mode;            /* 0 penalised, 1 constrained, 2 penalty-free,
                                3 limited imbalance: no penalty, targets capped at
                                floor(alpha * L_max) (Section 8.2) */
    int32_t rebuild_table;   /* 1: conn and W are recomputed from part */
    int32_t max_rebalance_iters; /* 0: default */
    int32_t seq_penalty;     /* 1: S3 re-prices moves with earlier candidates' inflow */
    int32_t alpha_num, alpha_den; /* mode 3: alpha = alpha_num / alpha_den >= 1 */
    int32_t variant;         /* bit 0: optimistic filter (an earlier candidate neighbour
                                counts in its target block); bit 1: rebalancing priority
                                by the plain gain, without the node weight (Section 8.2) */
} orc_params;

#define ORC_VAR_OPTIMISTIC 1
#define ORC_VAR_PLAIN_PRIORITY 2
#define ORC_VAR_BEST_PREFIX 4     /* interleaved move sequence and best prefix (Section 5.4) */

/* Statistics, same order as the int64 slots the tests read. */
enum {
    ST_LMAX = 0, ST_CUT_BEFORE, ST_CUT_AFTER_MOVES, ST_CUT_AFTER, ST_CANDIDATES,
    ST_ACCEPTED, ST_REBAL_MOVES, ST_REBAL_ITERS, ST_STATUS,
    ST_PREFIX_STEPS,  /* best-prefix rounds: moves of the filtered sequence kept (-1: no
                         balanced boundary, nothing reverted) */
    ST_REVERTED,      /* best-prefix rounds: nodes returned to their round-start block */
    ST_COUNT = 12
};

/* Optional per-node outputs of the move phase (any pointer may be NULL). */
typedef struct {
    int32_t *target;  /* best target if candidate, else -1 */
    int64_t *score;   /* s(v, target) if candidate, else 0 */
    int64_t *pen;     /* P(v, target) if candidate, else 0 */
    uint8_t *accept;  /* 1 if the move survived the conflict filter */
    int64_t *pen_seq; /* S3 penalty of a candidate (-1: forbidden), else 0 */
    int64_t *gp;      /* S3 pessimistic gain of a candidate, else 0 */
    /* best-prefix rounds (any may be NULL): */
    int64_t *seq;     /* [4 n] the interleaved sequence: (node, from, to, step) per move */
    int64_t *bgain;   /* [n + 1] exact cumulative gain at each step boundary */
    uint8_t *bbal;    /* [n + 1] 1 iff the partition at that boundary is balanced */
    int64_t *pref;    /* [4] moves in the sequence, steps, best boundary, moves kept */
    int64_t *rrec;    /* [n] rebalancing moves: sub-iteration << 8 | bucket, else 0 */
} orc_debug;

static int64_t edge_w(const orc_graph *g, int64_t e) { return g->adjwgt ? g->adjwgt[e] : 1; }
static int64_t node_c(const orc_graph *g, int64_t v) { return g->vwgt ? g->vwgt[v] : 1; }

/* ---------------------------------------------------------------- S0 -- */

/* Balance constraint of Section 2: L_max = (1 + eps) * ceil(c(V) / k), with
 * eps = eps_num / eps_den rational and the product rounded down, since block
 * weights are integers and c(V_i) <= L_max is the constraint. */
int64_t orc_lmax(int64_t total, int32_t k, int32_t eps_num, int32_t eps_den)
{
    int64_t per = (total + k - 1) / k;                       /* ceil(c(V)/k) */
    u128 num = (u128)per * (u128)((int64_t)eps_den + eps_num);
    return (int64_t)(num / (u128)eps_den);
}

/* Slot of Section 5.3: slot = ceil(log_{3/2}(w / c)), i.e. the smallest l
 * with (3/2)^l >= w/c, i.e. w * 2^l <= c * 3^l. Clamped to [0, 53]: ratios
 * below 1 (and w = 0) land in slot 0, the sums of Section 5.3 start there. */
int32_t orc_slot(int64_t w, int64_t c)
{
    u128 p3 = 1;
    for (int l = 0; l < ORC_SLOTS; ++l) {
        if (((u128)w << l) <= (u128)c * p3) return l;
        p3 *= 3;
    }
    return ORC_SLOTS - 1;
}

/* Penalty factor of slot l (Section 5.3 penalty (3/2)^l * c(u), scaled by the
 * round's tau from Section 5.5), in Q16 fixed point, rounded down:
 * PENQ[l] = floor(tau_num * 3^l * 2^16 / (tau_den * 2^l)). */
void orc_penq(int32_t tau_num, int32_t tau_den, int64_t *out)
{
    u128 p3 = 1;
    for (int l = 0; l < ORC_SLOTS; ++l) {
        u128 num = (u128)(uint64_t)tau_num * p3;
        u128 den = (u128)(uint64_t)tau_den << l;
        u128 q = num / den, r = num % den;
        out[l] = (int64_t)(q * 65536 + (r * 65536) / den);
        p3 *= 3;
    }
}

int64_t orc_total_weight(const orc_graph *g)
{
    int64_t s = 0;
    for (int64_t v = 0; v < g->n; ++v) s += node_c(g, v);
    return s;
}

/* ---------------------------------------------------------------- S1 -- */

/* Gain table of the shared-memory FM (Section 7.1): conn[v][j] = omega(v, V_j). */
void orc_gain_table(const orc_graph *g, int32_t k, const int32_t *part, int32_t *conn)
{
    for (int64_t v = 0; v < g->n; ++v) {
        int32_t *row = conn + v * (int64_t)k;
        for (int32_t j = 0; j < k; ++j) row[j] = 0;
        for (int64_t e = g->xadj[v]; e < g->xadj[v + 1]; ++e)
            row[part[g->adjncy[e]]] += (int32_t)edge_w(g, e);
    }
}

/* c(V_j) for every block. */
void orc_block_weights(const orc_graph *g, int32_t k, const int32_t *part, int64_t *W)
{
    for (int32_t j = 0; j < k; ++j) W[j] = 0;
    for (int64_t v = 0; v < g->n; ++v) W[part[v]] += node_c(g, v);
}

/* Edge cut straight from the definition of Section 2: total weight of edges
 * whose endpoints lie in different blocks, each undirected edge once. */
int64_t orc_cut_edges(const orc_graph *g, const int32_t *part)
{
    int64_t cut = 0;
    for (int64_t v = 0; v < g->n; ++v)
        for (int64_t e = g->xadj[v]; e < g->xadj[v + 1]; ++e) {
            int64_t u = g->adjncy[e];
            if (v < u && part[v] != part[u]) cut += edge_w(g, e);
        }
    return cut;
}

static int64_t wdeg(const orc_graph *g, int64_t v)
{
    int64_t s = 0;
    for (int64_t e = g->xadj[v]; e < g->xadj[v + 1]; ++e) s += edge_w(g, e);
    return s;
}

/* Cut from the gain table: every cut edge leaves its two endpoints' own
 * blocks, so 2 * cut = sum_v (omega(I(v)) - omega(v, Pi(v))). */
int64_t orc_cut_table(const orc_graph *g, int32_t k, const int32_t *part, const int32_t *conn)
{
    int64_t twice = 0;
    for (int64_t v = 0; v < g->n; ++v) twice += wdeg(g, v) - conn[v * (int64_t)k + part[v]];
    return twice / 2;
}

/* ---------------------------------------------------------------- S4 -- */

/* Move v from its block to b, keeping conn and W consistent (Section 7.1:
 * block weights and the gain table are updated as nodes move). */
static void apply_move(const orc_graph *g, int32_t k, int32_t *part, int32_t *conn, int64_t *W,
                       int64_t v, int32_t b)
{
    int32_t a = part[v];
    if (a == b) return;
    W[a] -= node_c(g, v);
    W[b] += node_c(g, v);
    for (int64_t e = g->xadj[v]; e < g->xadj[v + 1]; ++e) {
        int64_t u = g->adjncy[e];
        conn[u * (int64_t)k + a] -= (int32_t)edge_w(g, e);
        conn[u * (int64_t)k + b] += (int32_t)edge_w(g, e);
    }
    part[v] = b;
}

/* ---------------------------------------------------------------- S5 -- */

/* One node in a selection list: grouped by blk, then ordered by (beta, id). */
typedef struct { int32_t blk; int32_t beta; int64_t id; int64_t c; } rb_item;

static int rb_cmp(const void *x, const void *y)
{
    const rb_item *a = (const rb_item *)x, *b = (const rb_item *)y;
    if (a->blk != b->blk) return a->blk < b->blk ? -1 : 1;
    if (a->beta != b->beta) return a->beta < b->beta ? -1 : 1;
    return a->id < b->id ? -1 : (a->id > b->id);
}

/* Rebalancing of Section 7.1, made synchronous.
 *
 * While some block is overloaded (W[j] > L_max), one sub-iteration:
 *  1. Every node v of an overloaded block a (just-moved nodes included)
 *     picks its move with the best gain among targets that stay balanced
 *     (W[j] + c(v) <= L_max, j != a); if it is connected to none of them it
 *     picks the lightest block (ties to the smaller id). No valid target:
 *     v cannot move. Gain g = omega(v, target) - omega(v, a).
 *     Priority (higher first): g * c(v) if g >= 0, g / c(v) if g < 0. It is
 *     bucketed monotonically into beta (lower first):
 *        g >  0: beta = S - 1 - slot(g * c(v), 1)
 *        g == 0: beta = S
 *        g <  0: beta = S + 1 + slot(-g, c(v))
 *  2. Every movable node of an overloaded block is offered to its target.
 *  3. Each target j accepts the maximal prefix, in (beta, id) order, of the
 *     offers aimed at it whose weight fits L_max - W[j] (a target is never
 *     overloaded, like the atomic weight check of Section 7.1).
 *  4. Each source a keeps the minimal prefix, in (beta, id) order, of its
 *     accepted nodes whose weight covers W[a] - L_max (all of them if they do
 *     not suffice): like the priority queue, the cheapest nodes go first and
 *     nodes of a block that is balanced again stay.
 *  5. The kept nodes move (as in S4). If nothing moved, stop stuck.
 * All of 1-4 read the sub-iteration's starting W and conn.
 */
static int rebalance_iterate(const orc_graph *g, const orc_params *p, int64_t lmax, int32_t *part,
                             int32_t *conn, int64_t *W, int64_t *moves_out, int64_t *iters_out,
                             int64_t *rec_iter, int32_t *rec_beta)
{
    const int32_t k = p->k;
    const int64_t n = g->n;
    int64_t it_max = p->max_rebalance_iters > 0 ? p->max_rebalance_iters
                     : (g->vwgt ? 4 * (int64_t)k : (int64_t)k + 1);
    int32_t *tgt = (int32_t *)malloc(sizeof(int32_t) * (size_t)(n > 0 ? n : 1));
    int32_t *beta = (int32_t *)malloc(sizeof(int32_t) * (size_t)(n > 0 ? n : 1));
    uint8_t *sel = (uint8_t *)malloc((size_t)(n > 0 ? n : 1));
    rb_item *items = (rb_item *)malloc(sizeof(rb_item) * (size_t)(n > 0 ? n : 1));
    int64_t *W0 = (int64_t *)malloc(sizeof(int64_t) * (size_t)k);
    int64_t moves = 0, iters = 0;
    int status = 0;

    for (;;) {
        int any_over = 0;
        for (int32_t j = 0; j < k; ++j) any_over |= (W[j] > lmax);
        if (!any_over) break;
        if (iters >= it_max) { status = 1; break; }
        ++iters;
        memcpy(W0, W, sizeof(int64_t) * (size_t)k);

        /* step 1 */
        for (int64_t v = 0; v < n; ++v) {
            tgt[v] = -1;
            sel[v] = 0;
            int32_t a = part[v];
            if (W0[a] <= lmax) continue;
            int64_t cv = node_c(g, v);
            const int32_t *row = conn + v * (int64_t)k;
            int32_t best = -1;
            for (int32_t j = 0; j < k; ++j) {
                if (j == a || W0[j] + cv > lmax || row[j] <= 0) continue;
                if (best < 0 || row[j] > row[best]) best = j;
            }
            if (best < 0) {
                for (int32_t j = 0; j < k; ++j) {
                    if (j == a || W0[j] + cv > lmax) continue;
                    if (best < 0 || W0[j] < W0[best]) best = j;
                }
            }
            if (best < 0) continue;
            tgt[v] = best;
            int64_t gain = (int64_t)row[best] - row[a];
            /* the plain-gain variant ranks by the gain alone: as if c(v) = 1 */
            const int64_t cp = (p->variant & ORC_VAR_PLAIN_PRIORITY) ? 1 : cv;
            if (gain > 0)
                beta[v] = ORC_SLOTS - 1 - orc_slot(gain * cp, 1);
            else if (gain == 0)
                beta[v] = ORC_SLOTS;
            else
                beta[v] = ORC_SLOTS + 1 + orc_slot(-gain, cp);
        }

        /* steps 2-3: every movable node is offered; per target, the maximal
         * prefix within capacity is accepted */
        int64_t moved_now = 0;
        int64_t cnt = 0;
        for (int64_t v = 0; v < n; ++v)
            if (tgt[v] >= 0) {
                items[cnt].blk = tgt[v]; items[cnt].beta = beta[v];
                items[cnt].id = v; items[cnt].c = node_c(g, v); ++cnt;
            }
        qsort(items, (size_t)cnt, sizeof(rb_item), rb_cmp);
        for (int64_t i = 0; i < cnt;) {
            int32_t j = items[i].blk;
            int64_t cap = lmax - W0[j], used = 0;
            int full = 0;
            for (; i < cnt && items[i].blk == j; ++i) {
                if (full || used + items[i].c > cap) { full = 1; continue; }
                used += items[i].c;
                sel[items[i].id] = 1; /* accepted by its target */
            }
        }

        /* step 4: per source, the minimal covering prefix of its accepted nodes */
        cnt = 0;
        for (int64_t v = 0; v < n; ++v)
            if (sel[v]) {
                items[cnt].blk = part[v]; items[cnt].beta = beta[v];
                items[cnt].id = v; items[cnt].c = node_c(g, v); ++cnt;
            }
        qsort(items, (size_t)cnt, sizeof(rb_item), rb_cmp);
        for (int64_t i = 0; i < cnt;) {
            int32_t a = items[i].blk;
            int64_t need = W0[a] - lmax, got = 0;
            for (; i < cnt && items[i].blk == a; ++i)
                if (got < need) { sel[items[i].id] = 2; got += items[i].c; }
        }

        /* step 5 (rec_iter / rec_beta, if given: the sub-iteration and the
         * priority bucket of each move, the order in which it was made) */
        for (int64_t v = 0; v < n; ++v)
            if (sel[v] == 2) {
                if (rec_iter) { rec_iter[v] = iters; rec_beta[v] = beta[v]; }
                apply_move(g, k, part, conn, W, v, tgt[v]);
                ++moved_now;
            }
        moves += moved_now;
        if (moved_now == 0) { status = 1; break; }
    }
    free(tgt); free(beta); free(sel); free(items); free(W0);
    *moves_out = moves;
    *iters_out = iters;
    return status;
}

/* --------------------------------------------------------------- S1b -- */

/* Rebalance-available set and penalty buckets of Section 5.3: v is available
 * iff omega(v, Pi(v)) >= t * omega(I(v)) (exact: t_den * inner >= t_num * wdeg);
 * an available node goes to bucket (Pi(v), slot(omega(v, Pi(v)), c(v))), and
 * bucket[j * 54 + l] = c(B_{l,j}) is the node weight collected there.
 * avail[v] (optional) receives 1 + slot for available nodes, 0 otherwise. */
void orc_penalty_buckets(const orc_graph *g, int32_t k, const int32_t *part, const int32_t *conn,
                         int32_t t_num, int32_t t_den, int64_t *bucket, int32_t *avail)
{
    for (int64_t i = 0; i < (int64_t)k * ORC_SLOTS; ++i) bucket[i] = 0;
    for (int64_t v = 0; v < g->n; ++v) {
        int32_t a = part[v];
        int64_t inner = conn[v * (int64_t)k + a];
        int32_t s = -1;
        if ((int64_t)t_den * inner >= (int64_t)t_num * wdeg(g, v)) {
            s = orc_slot(inner, node_c(g, v));
            bucket[(int64_t)a * ORC_SLOTS + s] += node_c(g, v);
        }
        if (avail) avail[v] = s + 1;
    }
}

/* Penalty of Section 5.3 for a node of weight cv whose move leaves its target
 * with excess X = c(V_j + v) - bound (bound = L_max, or the cap of mode 3),
 * given the target's bucket weights: 0 if X <= 0; otherwise constrained
 * (mode 1) and limited imbalance (mode 3): forbidden; penalty-free (mode 2):
 * 0; penalised (mode 0): tau * (3/2)^l * c(v) in Q16 (saturated at 2^62) for
 * the least slot l whose cumulative bucket weight covers X, forbidden if none.
 * Returns 0 when the move is forbidden. */
static int move_penalty(const int64_t *bucket_row, const int64_t *penq, int mode, int64_t X,
                        int64_t cv, int64_t *P)
{
    *P = 0;
    if (X <= 0 || mode == 2) return 1;
    if (mode == 1 || mode == 3) return 0;
    int64_t acc = 0;
    for (int i = 0; i < ORC_SLOTS; ++i) {
        acc += bucket_row[i];
        if (acc >= X) {
            if (penq[i] != 0 && cv > ORC_PEN_CAP / penq[i]) *P = ORC_PEN_CAP;
            else *P = penq[i] * cv;
            if (*P > ORC_PEN_CAP) *P = ORC_PEN_CAP;
            return 1;
        }
    }
    return 0;
}

/* The weight a move may bring its target to before it is penalised or
 * forbidden: L_max, or in the limited-imbalance variant of Section 8.2 the
 * round's cap floor(alpha * L_max). */
static int64_t move_bound(const orc_params *p, int64_t lmax)
{
    if (p->mode != 3) return lmax;
    return (int64_t)(((unsigned __int128)(uint64_t)lmax * (uint32_t)p->alpha_num) /
                     (uint32_t)p->alpha_den);
}

/* Candidate order of S3: score descending, then id ascending. */
static const int64_t *cmp_score;
static int cand_cmp(const void *x, const void *y)
{
    const int64_t u = *(const int64_t *)x, v = *(const int64_t *)y;
    if (cmp_score[u] != cmp_score[v]) return cmp_score[u] > cmp_score[v] ? -1 : 1;
    return u < v ? -1 : (u > v);
}

/* ------------------------------------------------------------ prefix -- */

/* A rebalancing move in its list R_i: grouped by the block it left, in the
 * order the rebalancer made it (sub-iteration, then priority bucket, then
 * id: the order in which a source keeps its nodes). */
typedef struct { int32_t from; int64_t iter; int32_t beta; int64_t id; } rmove;

static int rmove_cmp(const void *x, const void *y)
{
    const rmove *a = (const rmove *)x, *b = (const rmove *)y;
    if (a->from != b->from) return a->from < b->from ? -1 : 1;
    if (a->iter != b->iter) return a->iter < b->iter ? -1 : 1;
    if (a->beta != b->beta) return a->beta < b->beta ? -1 : 1;
    return a->id < b->id ? -1 : (a->id > b->id);
}

static int all_balanced(const int64_t *W, int32_t k, int64_t lmax)
{
    for (int32_t j = 0; j < k; ++j)
        if (W[j] > lmax) return 0;
    return 1;
}

/* Interleaved move sequence and best prefix (Section 5.4, the last two steps
 * of Algorithm 1), after S4 and S5 have run.
 *
 * part0 / W0: the round-start partition and block weights; part: after S5.
 * order[0..nc): the candidates in the filter's order; accept: its decisions.
 * rec_iter / rec_beta: sub-iteration (0: none) and bucket of S5's moves.
 *
 *  1. A node moved by both the filtered moves (a -> b) and the rebalancer
 *     (b -> c) is combined into one move a -> c in the place of the first
 *     (the footnote of Section 5.4); if c = a it is dropped. M is the
 *     filtered moves in the filter's order, so combined; R_i the other
 *     rebalancing moves out of block i, in the order they were made.
 *  2. Interleave: starting from W0, append the moves of M one by one; when a
 *     move m into block b leaves b overloaded, append the minimal prefix of
 *     the unused moves of R_b that brings b back to L_max (all of them if
 *     they do not suffice). A step is m with the moves it pulled in; the
 *     boundaries after each step are the candidate prefixes.
 *  3. Recompute each move's gain exactly at its position: a neighbour sits
 *     in its new block if its move comes earlier in the sequence, else in
 *     its round-start block.
 *  4. Keep the prefix ending at the balanced boundary with the highest
 *     cumulative gain (the earliest on ties); every other move of the round
 *     is undone. With no balanced boundary nothing is undone.
 * Returns the boundary kept (-1: none) and fills stats and dbg. */
static int64_t best_prefix(const orc_graph *g, int32_t k, int64_t lmax, const int32_t *part0,
                           const int64_t *W0, int32_t *part, int32_t *conn, int64_t *W,
                           const int64_t *order, int64_t nc, const uint8_t *accept,
                           const int64_t *rec_iter, const int32_t *rec_beta, int64_t *stats,
                           const orc_debug *dbg)
{
    const int64_t n = g->n;
    const size_t N = (size_t)(n > 0 ? n : 1);
    /* 1. M (filter order, combined moves) and the lists R_i */
    int64_t *mlist = (int64_t *)malloc(sizeof(int64_t) * N);
    int64_t nm = 0;
    for (int64_t i = 0; i < nc; ++i) {
        const int64_t v = order[i];
        if (accept[v] && part[v] != part0[v]) mlist[nm++] = v;
    }
    rmove *rl = (rmove *)malloc(sizeof(rmove) * N);
    int64_t nr = 0;
    for (int64_t v = 0; v < n; ++v)
        if (rec_iter[v] > 0 && !accept[v]) {
            rl[nr].from = part0[v]; rl[nr].iter = rec_iter[v];
            rl[nr].beta = rec_beta[v]; rl[nr].id = v; ++nr;
        }
    qsort(rl, (size_t)nr, sizeof(rmove), rmove_cmp);
    int64_t *rstart = (int64_t *)calloc((size_t)k + 1, sizeof(int64_t));
    for (int64_t i = 0; i < nr; ++i) rstart[rl[i].from + 1]++;
    for (int32_t j = 0; j < k; ++j) rstart[j + 1] += rstart[j];
    int64_t *used = (int64_t *)calloc((size_t)k, sizeof(int64_t));

    /* 2. interleave */
    int64_t *Wc = (int64_t *)malloc(sizeof(int64_t) * (size_t)k);
    memcpy(Wc, W0, sizeof(int64_t) * (size_t)k);
    int64_t *seq_node = (int64_t *)malloc(sizeof(int64_t) * N);
    int64_t *seq_step = (int64_t *)malloc(sizeof(int64_t) * N);
    int32_t *seq_to = (int32_t *)malloc(sizeof(int32_t) * N);
    uint8_t *bal = (uint8_t *)malloc((size_t)nm + 1);
    int64_t len = 0;
    bal[0] = (uint8_t)all_balanced(Wc, k, lmax);
    for (int64_t j = 0; j < nm; ++j) {
        const int64_t v = mlist[j];
        const int32_t b = part[v];
        Wc[part0[v]] -= node_c(g, v);
        Wc[b] += node_c(g, v);
        seq_node[len] = v; seq_step[len] = j; seq_to[len] = b; ++len;
        while (Wc[b] > lmax && rstart[b] + used[b] < rstart[b + 1]) {
            const int64_t r = rl[rstart[b] + used[b]].id;
            ++used[b];
            Wc[b] -= node_c(g, r);
            Wc[part[r]] += node_c(g, r);
            seq_node[len] = r; seq_step[len] = j; seq_to[len] = part[r]; ++len;
        }
        bal[j + 1] = (uint8_t)all_balanced(Wc, k, lmax);
    }

    /* 3. exact gains in sequence order */
    int64_t *pos = (int64_t *)malloc(sizeof(int64_t) * N);
    for (int64_t v = 0; v < n; ++v) pos[v] = -1;
    for (int64_t i = 0; i < len; ++i) pos[seq_node[i]] = i;
    int64_t *bgain = (int64_t *)calloc((size_t)nm + 1, sizeof(int64_t));
    for (int64_t i = 0; i < len; ++i) {
        const int64_t u = seq_node[i];
        const int32_t a = part0[u], b = part[u];
        int64_t gain = 0;
        for (int64_t e = g->xadj[u]; e < g->xadj[u + 1]; ++e) {
            const int64_t x = g->adjncy[e];
            const int32_t bx = (pos[x] >= 0 && pos[x] < i) ? part[x] : part0[x];
            gain += edge_w(g, e) * ((bx == b) - (bx == a));
        }
        bgain[seq_step[i] + 1] += gain;
    }
    for (int64_t j = 0; j < nm; ++j) bgain[j + 1] += bgain[j];

    /* 4. best balanced boundary, earliest on ties */
    int64_t best = -1;
    for (int64_t j = 0; j <= nm; ++j)
        if (bal[j] && (best < 0 || bgain[j] > bgain[best])) best = j;
    int64_t kept = 0, reverted = 0;
    if (best >= 0) {
        for (int64_t v = 0; v < n; ++v) {
            if (part[v] == part0[v]) continue;
            if (pos[v] >= 0 && seq_step[pos[v]] < best) { ++kept; continue; }
            apply_move(g, k, part, conn, W, v, part0[v]);
            ++reverted;
        }
    }
    stats[ST_PREFIX_STEPS] = best;
    stats[ST_REVERTED] = reverted;
    if (dbg) {
        if (dbg->seq)
            for (int64_t i = 0; i < len; ++i) {
                const int64_t u = seq_node[i];
                dbg->seq[4 * i] = u;
                dbg->seq[4 * i + 1] = part0[u];
                dbg->seq[4 * i + 2] = seq_to[i];
                dbg->seq[4 * i + 3] = seq_step[i];
            }
        if (dbg->bgain) memcpy(dbg->bgain, bgain, sizeof(int64_t) * ((size_t)nm + 1));
        if (dbg->bbal) memcpy(dbg->bbal, bal, (size_t)nm + 1);
        if (dbg->pref) {
            dbg->pref[0] = len; dbg->pref[1] = nm; dbg->pref[2] = best; dbg->pref[3] = kept;
        }
        if (dbg->rrec)
            for (int64_t v = 0; v < n; ++v)
                dbg->rrec[v] = rec_iter[v] > 0 ? (rec_iter[v] << 8) | rec_beta[v] : 0;
    }
    free(mlist); free(rl); free(rstart); free(used); free(Wc); free(seq_node); free(seq_step);
    free(seq_to); free(bal); free(pos); free(bgain);
    return best;
}

/* ------------------------------------------------------------- rounds -- */

static int check_params(const orc_graph *g, const orc_params *p, const int32_t *part)
{
    if (p->k < 2 || p->eps_num <= 0 || p->eps_den <= 0) return -1;
    if (p->t_num < 0 || p->t_den <= 0 || p->t_num > p->t_den) return -1;
    if (p->tau_num < 0 || p->tau_den <= 0 || p->tau_num > p->tau_den) return -1;
    if (p->mode < 0 || p->mode > 3) return -1;
    if (p->mode == 3 && (p->alpha_den <= 0 || p->alpha_num < p->alpha_den)) return -1;
    if (p->variant & ~(ORC_VAR_OPTIMISTIC | ORC_VAR_PLAIN_PRIORITY | ORC_VAR_BEST_PREFIX)) return -1;
    for (int64_t v = 0; v < g->n; ++v)
        if (part[v] < 0 || part[v] >= p->k) return -1;
    return 0;
}

/* S0 + S1 shared by both entry points. */
static void prepare(const orc_graph *g, const orc_params *p, const int32_t *part, int32_t *conn,
                    int64_t *W, int64_t *stats, int64_t *lmax)
{
    for (int i = 0; i < ST_COUNT; ++i) stats[i] = 0;
    *lmax = orc_lmax(orc_total_weight(g), p->k, p->eps_num, p->eps_den);
    stats[ST_LMAX] = *lmax;
    if (p->rebuild_table) {
        orc_gain_table(g, p->k, part, conn);
        orc_block_weights(g, p->k, part, W);
    }
    stats[ST_CUT_BEFORE] = orc_cut_table(g, p->k, part, conn);
}

/* One round. active (may be NULL: every node): only nodes with active[v] != 0
 * look for a move in S2 (the active set of Section 6's label propagation). */
int orc_refine_round_active(const orc_graph *g, const orc_params *p, int32_t *part,
                            int32_t *conn, int64_t *W, int64_t *stats, const orc_debug *dbg,
                            const uint8_t *active)
{
    if (check_params(g, p, part)) return -1;
    const int32_t k = p->k;
    const int64_t n = g->n;
    int64_t lmax;
    prepare(g, p, part, conn, W, stats, &lmax);

    /* S0 penalty table for this round's tau */
    int64_t penq[ORC_SLOTS];
    orc_penq(p->tau_num, p->tau_den, penq);

    /* S1b */
    int64_t *bucket = (int64_t *)calloc((size_t)k * ORC_SLOTS, sizeof(int64_t));
    int32_t *avail = (int32_t *)malloc(sizeof(int32_t) * (size_t)(n > 0 ? n : 1));
    orc_penalty_buckets(g, k, part, conn, p->t_num, p->t_den, bucket, avail);

    /* S2: best penalised move per node, against the round-start W. */
    const int64_t bound = move_bound(p, lmax);
    int32_t *target = (int32_t *)malloc(sizeof(int32_t) * (size_t)(n > 0 ? n : 1));
    int64_t *score = (int64_t *)malloc(sizeof(int64_t) * (size_t)(n > 0 ? n : 1));
    int64_t *pen = (int64_t *)malloc(sizeof(int64_t) * (size_t)(n > 0 ? n : 1));
    int64_t candidates = 0;
    for (int64_t v = 0; v < n; ++v) {
        int32_t a = part[v];
        int64_t cv = node_c(g, v);
        const int32_t *row = conn + v * (int64_t)k;
        int32_t best = -1;
        int64_t best_s = 0, best_p = 0;
        for (int32_t j = 0; j < k && (!active || active[v]); ++j) {
            if (j == a || row[j] <= 0) continue;      /* adjacent blocks only */
            int64_t delta = (int64_t)row[j] - row[a];  /* gain of the move v -> j */
            int64_t excess = W[j] + cv - bound;        /* c(V_j + v) - L_max (or the cap) */
            int64_t P;
            if (!move_penalty(bucket + (int64_t)j * ORC_SLOTS, penq, p->mode, excess, cv, &P))
                continue;                              /* forbidden */
            int64_t s = delta * 65536 - P;
            if (best < 0 || s > best_s) { best = j; best_s = s; best_p = P; }
        }
        if (best >= 0 && best_s > 0) {
            target[v] = best; score[v] = best_s; pen[v] = best_p; ++candidates;
        } else {
            target[v] = -1; score[v] = 0; pen[v] = 0;
        }
    }
    stats[ST_CANDIDATES] = candidates;

    /* S3: conflict filter in (score desc, id asc) order. For candidate v
     * moving a -> b, f(x) = +1 if x == b, -1 if x == a, else 0 is the change
     * in v's internal edge weight contributed by a neighbour sitting in x.
     * An earlier candidate neighbour u (before v in the order) may or may
     * not move; take the worse of its two positions. With the
     * sequence-aware penalty, each block's weight is tracked along the
     * order: an eligible candidate (pessimistic gain > 0) adds its weight to
     * its target and, unless it is available for rebalancing, removes it
     * from its own block; every move is priced against the weight reached
     * before it. */
    uint8_t *accept = (uint8_t *)calloc((size_t)(n > 0 ? n : 1), 1);
    int64_t *pen_seq = (int64_t *)calloc((size_t)(n > 0 ? n : 1), sizeof(int64_t));
    int64_t *gps = (int64_t *)calloc((size_t)(n > 0 ? n : 1), sizeof(int64_t));
    int64_t *order = (int64_t *)malloc(sizeof(int64_t) * (size_t)(candidates > 0 ? candidates : 1));
    int64_t *net = (int64_t *)calloc((size_t)k, sizeof(int64_t));
    int64_t nc = 0;
    for (int64_t v = 0; v < n; ++v)
        if (target[v] >= 0) order[nc++] = v;
    cmp_score = score;
    qsort(order, (size_t)nc, sizeof(int64_t), cand_cmp);
    int64_t accepted = 0;
    for (int64_t i = 0; i < nc; ++i) {
        const int64_t v = order[i];
        int32_t a = part[v], b = target[v];
        int64_t gp = 0;
        for (int64_t e = g->xadj[v]; e < g->xadj[v + 1]; ++e) {
            int64_t u = g->adjncy[e];
            int32_t pu = part[u];
            int fu = pu == b ? 1 : (pu == a ? -1 : 0);
            int earlier = target[u] >= 0 &&
                          (score[u] > score[v] || (score[u] == score[v] && u < v));
            if (earlier) {
                int32_t tu = target[u];
                int ft = tu == b ? 1 : (tu == a ? -1 : 0);
                /* pessimistic: the worse of its two blocks; optimistic
                 * variant: the neighbour is assumed to have moved */
                if ((p->variant & ORC_VAR_OPTIMISTIC) || ft < fu) fu = ft;
            }
            gp += edge_w(g, e) * fu;
        }
        gps[v] = gp;
        int64_t P = pen[v];
        int allowed = 1;
        const int eligible = gp > 0;
        if (p->seq_penalty) {
            const int64_t cv = node_c(g, v);
            allowed = move_penalty(bucket + (int64_t)b * ORC_SLOTS, penq, p->mode,
                                   W[b] + net[b] + cv - bound, cv, &P);
            pen_seq[v] = allowed ? P : -1;
            if (eligible) {
                net[b] += cv;
                if (!avail[v]) net[a] -= cv;
            }
        } else {
            pen_seq[v] = P;
        }
        if (eligible && allowed && gp * 65536 - P > 0) { accept[v] = 1; ++accepted; }
    }
    free(net);
    free(avail);
    stats[ST_ACCEPTED] = accepted;

    /* the round-start state, for the best prefix */
    const int prefix = (p->variant & ORC_VAR_BEST_PREFIX) != 0;
    int32_t *part0 = NULL;
    int64_t *W0 = NULL, *rec_iter = NULL;
    int32_t *rec_beta = NULL;
    if (prefix) {
        part0 = (int32_t *)malloc(sizeof(int32_t) * (size_t)(n > 0 ? n : 1));
        W0 = (int64_t *)malloc(sizeof(int64_t) * (size_t)k);
        rec_iter = (int64_t *)calloc((size_t)(n > 0 ? n : 1), sizeof(int64_t));
        rec_beta = (int32_t *)calloc((size_t)(n > 0 ? n : 1), sizeof(int32_t));
        memcpy(part0, part, sizeof(int32_t) * (size_t)n);
        memcpy(W0, W, sizeof(int64_t) * (size_t)k);
    }

    /* S4: apply (commutative updates; the order does not matter). */
    for (int64_t v = 0; v < n; ++v)
        if (accept[v]) apply_move(g, k, part, conn, W, v, target[v]);
    stats[ST_CUT_AFTER_MOVES] = orc_cut_table(g, k, part, conn);

    /* S5 */
    int64_t moves = 0, iters = 0;
    stats[ST_STATUS] = rebalance_iterate(g, p, lmax, part, conn, W, &moves, &iters, rec_iter,
                                         rec_beta);
    stats[ST_REBAL_MOVES] = moves;
    stats[ST_REBAL_ITERS] = iters;

    /* interleaved move sequence and best prefix */
    if (prefix) {
        if (best_prefix(g, k, lmax, part0, W0, part, conn, W, order, nc, accept, rec_iter,
                        rec_beta, stats, dbg) >= 0)
            stats[ST_STATUS] = 0;
        free(part0); free(W0); free(rec_iter); free(rec_beta);
    }

    /* S6 */
    stats[ST_CUT_AFTER] = orc_cut_table(g, k, part, conn);

    if (dbg) {
        for (int64_t v = 0; v < n; ++v) {
            if (dbg->target) dbg->target[v] = target[v];
            if (dbg->score) dbg->score[v] = score[v];
            if (dbg->pen) dbg->pen[v] = pen[v];
            if (dbg->accept) dbg->accept[v] = accept[v];
            if (dbg->pen_seq) dbg->pen_seq[v] = pen_seq[v];
            if (dbg->gp) dbg->gp[v] = gps[v];
        }
    }
    free(bucket); free(target); free(score); free(pen); free(accept); free(pen_seq); free(gps);
    free(order);
    return 0;
}

/* A standalone rebalancing call: S0, S1 (if rebuilding), S5, S6. */
int orc_refine_round(const orc_graph *g, const orc_params *p, int32_t *part, int32_t *conn,
                     int64_t *W, int64_t *stats, const orc_debug *dbg)
{
    return orc_refine_round_active(g, p, part, conn, W, stats, dbg, NULL);
}

int orc_rebalance(const orc_graph *g, const orc_params *p, int32_t *part, int32_t *conn,
                  int64_t *W, int64_t *stats)
{
    if (check_params(g, p, part)) return -1;
    int64_t lmax;
    prepare(g, p, part, conn, W, stats, &lmax);
    stats[ST_CUT_AFTER_MOVES] = stats[ST_CUT_BEFORE];
    int64_t moves = 0, iters = 0;
    stats[ST_STATUS] = rebalance_iterate(g, p, lmax, part, conn, W, &moves, &iters, NULL, NULL);
    stats[ST_REBAL_MOVES] = moves;
    stats[ST_REBAL_ITERS] = iters;
    stats[ST_CUT_AFTER] = orc_cut_table(g, p->k, part, conn);
    return 0;
}
