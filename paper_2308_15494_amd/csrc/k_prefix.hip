// Interleaved move sequence and best prefix (Section 5.4, the last two steps
// of Algorithm 1), run after a round's rebalancing.
//
// The sequence is defined one move at a time: the filtered moves M in the
// filter's order (a node moved by both M and the rebalancer is one move from
// its round-start block to its final block, dropped if those are equal),
// and after each move m into block b that leaves b overloaded, the fewest
// unused rebalancing moves out of b (R_b, in the order the rebalancer made
// them: sub-iteration, bucket, id) that bring b back to L_max. Walking it
// move by move would be a single thread over up to millions of moves, so
// the walk is solved in parallel instead:
//
//  * b's weight right after step j (before its own rebalancing moves of that
//    step) is W0[b] + (filtered moves in and out of b up to j) + (rebalancing
//    moves into b taken at steps before j), and the number of R_b's moves
//    taken by step j is the running maximum, over b's steps up to j, of the
//    fewest moves whose weight covers that excess. With the rebalancing
//    moves into each block known, every block's schedule is a segmented
//    scan over its own events.
//  * Those moves into b come from the other blocks' schedules. Starting
//    from "none taken" and recomputing all schedules from the previous
//    round's take-times only makes blocks heavier, so the take-times only
//    move earlier; the unique fixed point (by induction over the steps) is
//    the sequential walk. A few iterations suffice; each costs a host read
//    of one flag.
//
// Then each move's exact gain at its position (a neighbour sits in its new
// block iff its own move comes earlier), the cumulative gain and the number
// of overloaded blocks at every step boundary, and the balanced boundary
// with the highest gain (earliest on ties). Every move of the round past it
// is undone through the ordinary apply (table deltas or tile rebuilds).
#include "upr_common.h"

#include <algorithm>
#include <cstring>

#include <rocprim/rocprim.hpp>

namespace upr {

namespace {

constexpr int32_t kInf = 0x7FFFFFFF;  // "never taken"
constexpr int kBestGroups = 1024;     // workgroups of the boundary argmax

__host__ __device__ __forceinline__ uint32_t ev_block(uint64_t k) { return (uint32_t)(k >> 32); }
__host__ __device__ __forceinline__ int32_t ev_step(uint64_t k) { return (int32_t)((k >> 1) & 0x7FFFFFFFu); }

struct KeyBlock {
    __host__ __device__ uint32_t operator()(uint64_t k) const { return ev_block(k); }
};

struct MaxI32 {
    __host__ __device__ int32_t operator()(int32_t a, int32_t b) const { return a > b ? a : b; }
};

struct FlagSet {
    const uint8_t *f;
    __host__ __device__ bool operator()(int32_t v) const { return f[v] != 0; }
};

__device__ __forceinline__ int64_t cw(const int32_t *vwgt, int64_t v) { return vwgt ? (int64_t)vwgt[v] : 1; }

// Weight of the first t moves of a block's list (rwi: inclusive prefix
// weights of the sorted list, the block's entries from `start`).
__device__ __forceinline__ int64_t rw_sum(const int64_t *rwi, int32_t start, int32_t t)
{
    return t > 0 ? rwi[start + t - 1] : 0;
}

// Fewest moves of the list [start, start + len) whose weight covers x.
__device__ __forceinline__ int32_t fewest_covering(const int64_t *rwi, int32_t start, int32_t len, int64_t x)
{
    if (x <= 0) return 0;
    int32_t lo = 1, hi = len;  // rw_sum(t) >= x for t = hi if at all
    if (len == 0 || rw_sum(rwi, start, len) < x) return len;
    while (lo < hi) {
        const int32_t mid = (lo + hi) >> 1;
        if (rw_sum(rwi, start, mid) >= x) hi = mid;
        else lo = mid + 1;
    }
    return lo;
}

// ---------------------------------------------------------------- kernels --

// Which nodes carry a move of the sequence: a filtered move that did not
// end where it started (fm), or a rebalancing move of a node the filter did
// not move (fr). Also resets the per-node position and step. The filter's
// flag is meaningful for this round's candidates only (key >= 0).
__global__ void k_bp_classify(int64_t n, const int32_t *part0, const int32_t *part,
                              const uint8_t *accflag, const int64_t *key, const int32_t *rbrec,
                              uint8_t *fm, uint8_t *fr, int64_t *pos, int32_t *stepof)
{
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; v < n; v += stride) {
        const bool moved = part[v] != part0[v];
        const bool acc = key[v] >= 0 && accflag[v] != 0;
        fm[v] = (acc && moved) ? 1 : 0;
        fr[v] = (!acc && rbrec[v] != 0) ? 1 : 0;
        pos[v] = -1;
        stepof[v] = -1;
    }
}

// Sort keys: the filtered moves by score descending ((2^48 - 1) - score;
// ties keep the id order of the selection), the rebalancing moves by
// (block left, sub-iteration, bucket).
__global__ void k_bp_keys(int32_t nm, const int32_t *mids, const int64_t *key, int32_t nr,
                          const int32_t *rids, const int32_t *part0, const int32_t *rbrec,
                          uint64_t *mkey, uint64_t *rkey)
{
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < (int64_t)nm + nr; i += stride) {
        if (i < nm) {
            const int64_t score = key[mids[i]] >> 16;
            mkey[i] = (((uint64_t)1 << 48) - 1) - (uint64_t)score;
        } else {
            const int64_t v = rids[i - nm];
            const uint32_t rec = (uint32_t)rbrec[v];
            rkey[i - nm] = ((uint64_t)(uint32_t)part0[v] << 40) | ((uint64_t)(rec >> 8) << 8) | (rec & 0xFFu);
        }
    }
}

// Per step j: the filtered move's two events (leaving its block, entering
// its target), keyed (block, step, in?); per rebalancing move: its blocks
// and weight; per-block counts of both lists.
__global__ void k_bp_lists(int32_t nm, const int32_t *mlist, int32_t nr, const int32_t *rlist,
                           const int32_t *part0, const int32_t *part, const int32_t *vwgt,
                           uint64_t *evkey, int32_t *rfrom, int32_t *rto, int64_t *rc,
                           int32_t *ecnt, int32_t *rcnt, int32_t *tau, int32_t *stepof)
{
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < (int64_t)nm + nr; i += stride) {
        if (i < nm) {
            const int64_t u = mlist[i];
            const uint32_t a = (uint32_t)part0[u], b = (uint32_t)part[u];
            evkey[2 * i] = ((uint64_t)a << 32) | ((uint64_t)i << 1);
            evkey[2 * i + 1] = ((uint64_t)b << 32) | ((uint64_t)i << 1) | 1u;
            atomicAdd(&ecnt[a], 1);
            atomicAdd(&ecnt[b], 1);
            stepof[u] = (int32_t)i;
        } else {
            const int64_t r = i - nm;
            const int64_t v = rlist[r];
            rfrom[r] = part0[v];
            rto[r] = part[v];
            rc[r] = cw(vwgt, v);
            tau[r] = kInf;
            atomicAdd(&rcnt[part0[v]], 1);
        }
    }
}

// Exclusive scans of up to three per-block count arrays of K entries, one
// workgroup of 1024 threads (out[K] = total).
__global__ __launch_bounds__(1024) void k_bp_offsets(int32_t K, const int32_t *c0, int32_t *o0,
                                                     const int32_t *c1, int32_t *o1)
{
    __shared__ int32_t carry[2];
    __shared__ int32_t wsum[2][16];
    if (threadIdx.x < 2) carry[threadIdx.x] = 0;
    __syncthreads();
    for (int32_t base = 0; base < K; base += 1024) {
        const int32_t j = base + threadIdx.x;
        int32_t x[2] = {j < K && c0 ? c0[j] : 0, j < K && c1 ? c1[j] : 0};
        int32_t inc[2];
        for (int s = 0; s < 2; ++s) {
            inc[s] = wave_incl_scan(x[s]);
            if (lane_id() == 63) wsum[s][threadIdx.x >> 6] = inc[s];
        }
        __syncthreads();
        for (int s = 0; s < 2; ++s) {
            int32_t pre = carry[s];
            for (int w = 0; w < (int)(threadIdx.x >> 6); ++w) pre += wsum[s][w];
            int32_t *o = s == 0 ? o0 : o1;
            if (o && j < K) o[j] = pre + inc[s] - x[s];
        }
        __syncthreads();
        if (threadIdx.x == 0)
            for (int s = 0; s < 2; ++s) {
                int32_t t = 0;
                for (int w = 0; w < 16; ++w) t += wsum[s][w];
                carry[s] += t;
            }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        if (o0) o0[K] = carry[0];
        if (o1) o1[K] = carry[1];
    }
}

// Event deltas for the segmented scan: -c leaving, +c entering.
__global__ void k_bp_ev_delta(int64_t ne, const uint64_t *evs, const int32_t *mlist,
                              const int32_t *vwgt, int64_t *delta)
{
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < ne; e += stride) {
        const uint64_t k = evs[e];
        const int64_t c = cw(vwgt, mlist[ev_step(k)]);
        delta[e] = (k & 1u) ? c : -c;
    }
}

// Rebalancing moves already taken, keyed (target block, take-step) for the
// lookup of the weight each block receives before a step; never-taken ones
// sort past every block.
__global__ void k_bp_rin_keys(int32_t nr, int32_t K, const int32_t *rto, const int32_t *tau,
                              uint64_t *key)
{
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < nr; i += stride)
        key[i] = tau[i] < kInf ? (((uint64_t)(uint32_t)rto[i] << 32) | (uint32_t)tau[i])
                               : ((uint64_t)(uint32_t)K << 32);
}

// First index of each block's entries in a list sorted by (block << 32 | x):
// off[b] = lower bound of b << 32 (b = 0..K).
__global__ void k_bp_bounds(int64_t cnt, const uint64_t *sorted, int32_t K, int32_t *off)
{
    const int32_t b = blockIdx.x * blockDim.x + threadIdx.x;
    if (b > K) return;
    const uint64_t x = (uint64_t)(uint32_t)b << 32;
    int64_t lo = 0, hi = cnt;
    while (lo < hi) {
        const int64_t mid = (lo + hi) >> 1;
        if (sorted[mid] < x) lo = mid + 1;
        else hi = mid;
    }
    off[b] = (int32_t)lo;
}

// Fewest moves of the block's list needed after each entering event: the
// block's weight with every filtered move up to the step and every
// rebalancing move taken into it before the step, over L_max.
__global__ void k_bp_need(int64_t ne, const uint64_t *evs, const int64_t *acc, const int64_t *W0,
                          int64_t lmax, const int32_t *roff, const int64_t *rwi,
                          const uint64_t *rin_key, const int64_t *rin_inc, const int32_t *rinoff,
                          int32_t *need)
{
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < ne; e += stride) {
        const uint64_t k = evs[e];
        if (!(k & 1u)) {
            need[e] = 0;
            continue;
        }
        const uint32_t b = ev_block(k);
        const int32_t j = ev_step(k);
        // weight received from rebalancing moves taken before step j
        const int32_t s0 = rinoff[b], s1 = rinoff[b + 1];
        const uint64_t lim = ((uint64_t)b << 32) | (uint32_t)j;
        int32_t lo = s0, hi = s1;
        while (lo < hi) {
            const int32_t mid = (lo + hi) >> 1;
            if (rin_key[mid] < lim) lo = mid + 1;
            else hi = mid;
        }
        const int64_t rin = lo > s0 ? rin_inc[lo - 1] : 0;
        const int64_t x = W0[b] + acc[e] + rin - lmax;
        need[e] = fewest_covering(rwi, roff[b], roff[b + 1] - roff[b], x);
    }
}

// Take-step of each rebalancing move: the first step of its block whose
// running count of needed moves passes the move's index in the list (the
// counts are nondecreasing along the block's events). Counts changes.
__global__ void k_bp_take(int32_t nr, const int32_t *rfrom, const int32_t *roff, const int32_t *eoff,
                          const uint64_t *evs, const int32_t *tcum, int32_t *tau,
                          unsigned long long *changed)
{
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    unsigned long long ch = 0;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < nr; i += stride) {
        const int32_t x = rfrom[i];
        const int32_t ii = (int32_t)i - roff[x];
        int32_t lo = eoff[x], hi = eoff[x + 1];
        while (lo < hi) {
            const int32_t mid = (lo + hi) >> 1;
            if (tcum[mid] > ii) hi = mid;
            else lo = mid + 1;
        }
        const int32_t t = lo < eoff[x + 1] ? ev_step(evs[lo]) : kInf;
        if (t != tau[i]) {
            tau[i] = t;
            ++ch;
        }
    }
    ch = wave_sum(ch);
    if (lane_id() == 0 && ch) atomicAdd(changed, ch);
}

// Rebalancing moves taken per step (for the positions).
__global__ void k_bp_count_steps(int32_t nr, const int32_t *tau, int32_t *cstep)
{
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < nr; i += stride)
        if (tau[i] < kInf) atomicAdd(&cstep[tau[i]], 1);
}

// Positions in the sequence: step j's filtered move at j plus the
// rebalancing moves of earlier steps, its rebalancing moves right after it
// in list order.
__global__ void k_bp_positions(int32_t nm, const int32_t *mlist, int32_t nr, const int32_t *rlist,
                               const int32_t *rfrom, const int32_t *roff, const int32_t *tau,
                               const int32_t *rbefore, int64_t *pos, int32_t *stepof)
{
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < (int64_t)nm + nr; i += stride) {
        if (i < nm) {
            pos[mlist[i]] = i + rbefore[i];
            continue;
        }
        const int32_t r = (int32_t)(i - nm);
        const int32_t t = tau[r];
        if (t >= kInf) continue;
        const int32_t x = rfrom[r];
        // first move of the block taken at the same step
        int32_t lo = roff[x], hi = r;
        while (lo < hi) {
            const int32_t mid = (lo + hi) >> 1;
            if (tau[mid] < t) lo = mid + 1;
            else hi = mid;
        }
        const int64_t v = rlist[r];
        pos[v] = (int64_t)t + rbefore[t] + 1 + (r - lo);
        stepof[v] = t;
    }
}

// Exact gain of every move of the sequence at its position, one wave per
// moving node over its row, summed per step.
__global__ __launch_bounds__(kBlock) void k_bp_gains(GraphView g, int32_t nm, const int32_t *mlist,
                                                      int32_t nr, const int32_t *rlist,
                                                      const int32_t *tau, const int32_t *part0,
                                                      const int32_t *part, const int64_t *pos,
                                                      const int32_t *stepof, int64_t *stepgain)
{
    const int lane = lane_id();
    const int64_t waves = (int64_t)gridDim.x * (kBlock / 64);
    for (int64_t i = (int64_t)blockIdx.x * (kBlock / 64) + (threadIdx.x >> 6); i < (int64_t)nm + nr;
         i += waves) {
        int64_t u;
        if (i < nm) {
            u = mlist[i];
        } else {
            if (tau[i - nm] >= kInf) continue;  // wave-uniform
            u = rlist[i - nm];
        }
        const int32_t a = part0[u], b = part[u];
        const int64_t pu = pos[u];
        int64_t s = 0;
        for (int64_t e = g.xadj[u] + lane; e < g.xadj[u + 1]; e += 64) {
            const int64_t x = g.adjncy[e];
            const int64_t px = pos[x];
            const int32_t bx = (px >= 0 && px < pu) ? part[x] : part0[x];
            s += (int64_t)edge_weight(g, e) * ((bx == b) - (bx == a));
        }
        s = wave_sum(s);
        if (lane == 0 && s) atomic_add_i64(&stepgain[stepof[u]], s);
    }
}

// Balance events: every filtered event (an entering one also loses the
// block's rebalancing moves of its step) and every taken rebalancing move's
// arrival. Keys as the filtered events.
__global__ void k_bp_bal_events(int64_t ne, const uint64_t *evs, const int64_t *delta,
                                const int32_t *tcum, const int32_t *roff, const int64_t *rwi,
                                int32_t nr, const int32_t *rto, const int32_t *tau,
                                const int64_t *rc, uint64_t *bkey, int64_t *bdelta)
{
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < ne + nr; e += stride) {
        if (e < ne) {
            const uint64_t k = evs[e];
            int64_t d = delta[e];
            if (k & 1u) {
                const uint32_t b = ev_block(k);
                const bool first = e == 0 || ev_block(evs[e - 1]) != b;
                const int32_t tp = first ? 0 : tcum[e - 1];
                d -= rw_sum(rwi, roff[b], tcum[e]) - rw_sum(rwi, roff[b], tp);
            }
            bkey[e] = k;
            bdelta[e] = d;
        } else {
            const int64_t r = e - ne;
            const int32_t t = tau[r];
            // an arrival sorts with the filtered events of its block at that
            // step; untaken moves go past every block
            bkey[e] = t < kInf ? (((uint64_t)(uint32_t)rto[r] << 32) | ((uint64_t)t << 1) | 1u)
                               : ~0ull;
            bdelta[e] = t < kInf ? rc[r] : 0;
        }
    }
}

// Changes of the number of overloaded blocks per step: each event compares
// its block's weight after it with the weight before it.
__global__ void k_bp_bal_diff(int64_t ne, const uint64_t *bkey, const int64_t *bacc,
                              const int64_t *W0, int64_t lmax, int32_t *diff)
{
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < ne; e += stride) {
        const uint64_t k = bkey[e];
        if (k == ~0ull) continue;
        const uint32_t b = ev_block(k);
        const bool first = e == 0 || ev_block(bkey[e - 1]) != b;
        const int64_t after = W0[b] + bacc[e];
        const int64_t before = first ? W0[b] : W0[b] + bacc[e - 1];
        const int d = (after > lmax ? 1 : 0) - (before > lmax ? 1 : 0);
        if (d) atomicAdd(&diff[ev_step(k)], d);
    }
}

// Best balanced boundary: boundary j (0..nm) is balanced iff no block is
// overloaded after steps 0..j-1; its gain is the sum of those steps' gains.
// Pass 1: per workgroup the best (gain, earliest j); pass 2 reduces.
__global__ __launch_bounds__(kBlock) void k_bp_best(int32_t nm, const int64_t *W0, int32_t K,
                                                     int64_t lmax, const int32_t *over_incl,
                                                     const int64_t *gain_incl, int64_t *part_g,
                                                     int32_t *part_j)
{
    __shared__ int32_t over0_lds;
    __shared__ int64_t bg[kBlock];
    __shared__ int32_t bj[kBlock];
    if (threadIdx.x == 0) over0_lds = 0;
    __syncthreads();
    int32_t o = 0;
    for (int32_t b = threadIdx.x; b < K; b += kBlock) o += W0[b] > lmax ? 1 : 0;
    if (o) atomicAdd(&over0_lds, o);
    __syncthreads();
    const int32_t over0 = over0_lds;
    int64_t best_g = 0;
    int32_t best_j = -1;
    const int64_t stride = (int64_t)gridDim.x * kBlock;
    for (int64_t j = (int64_t)blockIdx.x * kBlock + threadIdx.x; j <= nm; j += stride) {
        const int32_t over = over0 + (j > 0 ? over_incl[j - 1] : 0);
        if (over != 0) continue;
        const int64_t gsum = j > 0 ? gain_incl[j - 1] : 0;
        if (best_j < 0 || gsum > best_g) {  // j ascends per thread: keeps the earliest
            best_g = gsum;
            best_j = (int32_t)j;
        }
    }
    bg[threadIdx.x] = best_g;
    bj[threadIdx.x] = best_j;
    __syncthreads();
    for (int w = kBlock / 2; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) {
            const int64_t g2 = bg[threadIdx.x + w];
            const int32_t j2 = bj[threadIdx.x + w];
            const int32_t j1 = bj[threadIdx.x];
            if (j2 >= 0 && (j1 < 0 || g2 > bg[threadIdx.x] || (g2 == bg[threadIdx.x] && j2 < j1))) {
                bg[threadIdx.x] = g2;
                bj[threadIdx.x] = j2;
            }
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        part_g[blockIdx.x] = bg[0];
        part_j[blockIdx.x] = bj[0];
    }
}

__global__ __launch_bounds__(kBlock) void k_bp_best_final(int32_t groups, const int64_t *part_g,
                                                           const int32_t *part_j, int64_t *scal,
                                                           unsigned long long *counters)
{
    if (threadIdx.x != 0) return;
    int64_t g = 0;
    int32_t j = -1;
    for (int32_t i = 0; i < groups; ++i) {
        const int32_t ji = part_j[i];
        if (ji >= 0 && (j < 0 || part_g[i] > g || (part_g[i] == g && ji < j))) {
            g = part_g[i];
            j = ji;
        }
    }
    scal[0] = j;
    scal[1] = 0;  // reverted nodes, counted by the revert pass
    // the undo moves' degrees decide the apply's table update
    cnt_set(counters, CNT_MOVED_DEG, 0);
}

// Undo every move of the round past the kept boundary: the node returns to
// its round-start block through the apply (mvto).
__global__ void k_bp_revert(GraphView g, const int32_t *part0, const int32_t *part,
                            const int64_t *pos, const int32_t *stepof, int64_t *scal, int32_t *mvto,
                            unsigned long long *counters)
{
    __shared__ unsigned long long deg, cnt;
    if (threadIdx.x == 0) {
        deg = 0;
        cnt = 0;
    }
    __syncthreads();
    const int64_t best = scal[0];
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; v < g.n && best >= 0; v += stride) {
        if (part[v] == part0[v]) continue;
        if (pos[v] >= 0 && stepof[v] < best) continue;
        mvto[v] = part0[v];
        atomicAdd(&deg, (unsigned long long)(g.xadj[v + 1] - g.xadj[v]));
        atomicAdd(&cnt, 1ull);
    }
    __syncthreads();
    if (threadIdx.x == 0 && cnt) {
        cnt_add(counters, CNT_MOVED_DEG, deg);
        atomic_add_i64(&scal[1], (int64_t)cnt);
    }
}

__global__ void k_bp_stats(const int64_t *scal, int64_t *stats)
{
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    stats[9] = scal[0];
    stats[10] = scal[1];
    if (scal[0] >= 0) stats[8] = 0;
}

int grid_of(int64_t items, int per = kBlock, int cap = 4096)
{
    int64_t g = (items + per - 1) / per;
    if (g < 1) g = 1;
    if (g > cap) g = cap;
    return (int)g;
}

}  // namespace

size_t bp_temp_bytes(int64_t n)
{
    const size_t N = (size_t)(n > 0 ? n : 1);
    size_t mx = 16, b = 0;
    FlagSet fs{nullptr};
    int32_t *i32 = nullptr;
    int64_t *i64 = nullptr;
    uint64_t *u64 = nullptr;
    int32_t *cnt = nullptr;
    (void)rocprim::select(nullptr, b, rocprim::counting_iterator<int32_t>(0), i32, cnt, N, fs, (hipStream_t)0);
    mx = std::max(mx, b);
    (void)rocprim::radix_sort_pairs(nullptr, b, u64, u64, i32, i32, N, 0, 64, (hipStream_t)0);
    mx = std::max(mx, b);
    (void)rocprim::radix_sort_pairs(nullptr, b, u64, u64, i64, i64, 3 * N, 0, 64, (hipStream_t)0);
    mx = std::max(mx, b);
    (void)rocprim::radix_sort_keys(nullptr, b, u64, u64, 2 * N, 0, 64, (hipStream_t)0);
    mx = std::max(mx, b);
    auto kb = rocprim::make_transform_iterator(u64, KeyBlock{});
    (void)rocprim::inclusive_scan_by_key(nullptr, b, kb, i64, i64, 3 * N, rocprim::plus<int64_t>(),
                                   rocprim::equal_to<uint32_t>(), (hipStream_t)0);
    mx = std::max(mx, b);
    (void)rocprim::inclusive_scan_by_key(nullptr, b, kb, i32, i32, 2 * N, MaxI32{},
                                   rocprim::equal_to<uint32_t>(), (hipStream_t)0);
    mx = std::max(mx, b);
    (void)rocprim::inclusive_scan_by_key(nullptr, b, i32, i64, i64, N, rocprim::plus<int64_t>(),
                                   rocprim::equal_to<int32_t>(), (hipStream_t)0);
    mx = std::max(mx, b);
    (void)rocprim::inclusive_scan(nullptr, b, i32, i32, N + 1, rocprim::plus<int32_t>(), (hipStream_t)0);
    mx = std::max(mx, b);
    (void)rocprim::inclusive_scan(nullptr, b, i64, i64, N + 1, rocprim::plus<int64_t>(), (hipStream_t)0);
    mx = std::max(mx, b);
    (void)rocprim::exclusive_scan(nullptr, b, i32, i32, 0, N + 1, rocprim::plus<int32_t>(), (hipStream_t)0);
    mx = std::max(mx, b);
    return mx;
}

hipError_t launch_bp_record_start(int64_t n, int32_t K, const int32_t *part, const int64_t *W,
                                  const BpWs &ws, hipStream_t s)
{
    hipError_t e;
    if (n > 0 && (e = hipMemcpyAsync(ws.part0, part, sizeof(int32_t) * n, hipMemcpyDeviceToDevice, s)) != hipSuccess)
        return e;
    if ((e = hipMemcpyAsync(ws.W0, W, sizeof(int64_t) * K, hipMemcpyDeviceToDevice, s)) != hipSuccess) return e;
    return launch_fill_i32(ws.rbrec, n, 0, s);
}

hipError_t run_best_prefix(const GraphView &g, int32_t K, int64_t lmax, int32_t *part,
                           const PartView &pv, int32_t *conn, int64_t *W, const uint8_t *accflag,
                           const int64_t *key, int32_t *mvto, unsigned long long *counters,
                           const BpWs &ws, const BpApply &apply, int64_t *stats, int *iterations,
                           hipStream_t s)
{
    const int64_t n = g.n;
    hipError_t e;
#define BP_TRY(x)                                 \
    do {                                          \
        if ((e = (x)) != hipSuccess) return e;   \
    } while (0)
#define BP_LAUNCH(...)                            \
    do {                                          \
        hipLaunchKernelGGL(__VA_ARGS__);          \
        BP_TRY(hipGetLastError());                \
    } while (0)
    size_t tb = ws.temp_bytes;
    *iterations = 0;
    // 1. the sequence's nodes, in id order
    BP_LAUNCH(k_bp_classify, dim3(grid_of(n)), dim3(kBlock), 0, s, n, ws.part0, part, accflag, key,
              ws.rbrec, ws.fm, ws.fr, ws.pos, ws.stepof);
    BP_TRY(rocprim::select(ws.temp, tb, rocprim::counting_iterator<int32_t>(0), ws.ids, ws.cnt,
                           (size_t)n, FlagSet{ws.fm}, s));
    BP_TRY(rocprim::select(ws.temp, tb, rocprim::counting_iterator<int32_t>(0), ws.ids2, ws.cnt + 1,
                           (size_t)n, FlagSet{ws.fr}, s));
    int32_t cnt[2] = {0, 0};
    BP_TRY(hipMemcpyAsync(cnt, ws.cnt, sizeof cnt, hipMemcpyDeviceToHost, s));
    BP_TRY(hipStreamSynchronize(s));
    const int32_t nm = cnt[0], nr = cnt[1];
    // 2. filtered moves in the filter's order, rebalancing moves in list order
    BP_LAUNCH(k_bp_keys, dim3(grid_of((int64_t)nm + nr)), dim3(kBlock), 0, s, nm, ws.ids, key, nr,
              ws.ids2, ws.part0, ws.rbrec, ws.k0, ws.k0 + nm);
    if (nm > 0) BP_TRY(rocprim::radix_sort_pairs(ws.temp, tb, ws.k0, ws.k1, ws.ids, ws.mlist, (size_t)nm, 0, 48, s));
    if (nr > 0)
        BP_TRY(rocprim::radix_sort_pairs(ws.temp, tb, ws.k0 + nm, ws.k1 + nm, ws.ids2, ws.rlist, (size_t)nr, 0, 56, s));
    BP_TRY(launch_fill_i32(ws.ecnt, (int64_t)K + 1, 0, s));
    BP_TRY(launch_fill_i32(ws.rcnt, (int64_t)K + 1, 0, s));
    BP_LAUNCH(k_bp_lists, dim3(grid_of((int64_t)nm + nr)), dim3(kBlock), 0, s, nm, ws.mlist, nr, ws.rlist,
              ws.part0, part, g.vwgt, ws.k0, ws.rfrom, ws.rto, ws.rc, ws.ecnt, ws.rcnt, ws.tau,
              ws.stepof);
    BP_LAUNCH(k_bp_offsets, dim3(1), dim3(1024), 0, s, K, ws.ecnt, ws.eoff, ws.rcnt, ws.roff);
    // inclusive weights of each block's rebalancing list
    if (nr > 0)
        BP_TRY(rocprim::inclusive_scan_by_key(ws.temp, tb, ws.rfrom, ws.rc, ws.rwi, (size_t)nr,
                                              rocprim::plus<int64_t>(), rocprim::equal_to<int32_t>(), s));
    // 3. the filtered events by (block, step) and each block's weight after
    // each of them (filtered moves only)
    const int64_t ne = 2 * (int64_t)nm;
    if (ne > 0) {
        BP_TRY(rocprim::radix_sort_keys(ws.temp, tb, ws.k0, ws.evs, (size_t)ne, 0, 48, s));
        BP_LAUNCH(k_bp_ev_delta, dim3(grid_of(ne)), dim3(kBlock), 0, s, ne, ws.evs, ws.mlist, g.vwgt,
                  ws.d0);
        BP_TRY(rocprim::inclusive_scan_by_key(ws.temp, tb, rocprim::make_transform_iterator(ws.evs, KeyBlock{}),
                                              ws.d0, ws.acc, (size_t)ne, rocprim::plus<int64_t>(),
                                              rocprim::equal_to<uint32_t>(), s));
    }
    // 4. take-steps of the rebalancing moves: the fixed point from "none taken"
    if (ne > 0 && nr > 0) {
        for (;;) {
            ++*iterations;
            if (*iterations > 4096) return hipErrorUnknown;  // cannot happen: the steps only decrease
            BP_LAUNCH(k_bp_rin_keys, dim3(grid_of(nr)), dim3(kBlock), 0, s, nr, K, ws.rto, ws.tau, ws.k1);
            BP_TRY(rocprim::radix_sort_pairs(ws.temp, tb, ws.k1, ws.rin_key, ws.rc, ws.d1, (size_t)nr, 0, 48, s));
            BP_LAUNCH(k_bp_bounds, dim3((K + 1 + kBlock - 1) / kBlock), dim3(kBlock), 0, s, (int64_t)nr,
                      ws.rin_key, K, ws.rinoff);
            BP_TRY(rocprim::inclusive_scan_by_key(ws.temp, tb, rocprim::make_transform_iterator(ws.rin_key, KeyBlock{}),
                                                  ws.d1, ws.rin_inc, (size_t)nr, rocprim::plus<int64_t>(),
                                                  rocprim::equal_to<uint32_t>(), s));
            BP_LAUNCH(k_bp_need, dim3(grid_of(ne)), dim3(kBlock), 0, s, ne, ws.evs, ws.acc, ws.W0, lmax,
                      ws.roff, ws.rwi, ws.rin_key, ws.rin_inc, ws.rinoff, ws.need);
            BP_TRY(rocprim::inclusive_scan_by_key(ws.temp, tb, rocprim::make_transform_iterator(ws.evs, KeyBlock{}),
                                                  ws.need, ws.tcum, (size_t)ne, MaxI32{},
                                                  rocprim::equal_to<uint32_t>(), s));
            BP_TRY(hipMemsetAsync(ws.changed, 0, sizeof(unsigned long long), s));
            BP_LAUNCH(k_bp_take, dim3(grid_of(nr)), dim3(kBlock), 0, s, nr, ws.rfrom, ws.roff, ws.eoff,
                      ws.evs, ws.tcum, ws.tau, ws.changed);
            unsigned long long ch = 0;
            BP_TRY(hipMemcpyAsync(&ch, ws.changed, sizeof ch, hipMemcpyDeviceToHost, s));
            BP_TRY(hipStreamSynchronize(s));
            if (ch == 0) break;
        }
    } else if (ne > 0) {
        BP_TRY(launch_fill_i32(ws.tcum, ne, 0, s));
    }
    // 5. positions and exact gains
    BP_TRY(launch_fill_i32(ws.cstep, (int64_t)nm + 1, 0, s));
    BP_LAUNCH(k_bp_count_steps, dim3(grid_of(nr)), dim3(kBlock), 0, s, nr, ws.tau, ws.cstep);
    BP_TRY(rocprim::exclusive_scan(ws.temp, tb, ws.cstep, ws.rbefore, 0, (size_t)nm + 1,
                                   rocprim::plus<int32_t>(), s));
    BP_LAUNCH(k_bp_positions, dim3(grid_of((int64_t)nm + nr)), dim3(kBlock), 0, s, nm, ws.mlist, nr, ws.rlist,
              ws.rfrom, ws.roff, ws.tau, ws.rbefore, ws.pos, ws.stepof);
    BP_TRY(launch_fill_i64(ws.stepgain, (int64_t)nm + 1, 0, s));
    BP_LAUNCH(k_bp_gains, dim3(grid_of((int64_t)nm + nr, kBlock / 64, 8192)), dim3(kBlock), 0, s, g, nm,
              ws.mlist, nr, ws.rlist, ws.tau, ws.part0, part, ws.pos, ws.stepof, ws.stepgain);
    if (nm > 0)
        BP_TRY(rocprim::inclusive_scan(ws.temp, tb, ws.stepgain, ws.gain_incl, (size_t)nm,
                                       rocprim::plus<int64_t>(), s));
    // 6. overloaded blocks at every boundary
    BP_TRY(launch_fill_i32(ws.cstep, (int64_t)nm + 1, 0, s));  // now the per-step changes
    const int64_t nb = ne + nr;
    if (nb > 0) {
        BP_LAUNCH(k_bp_bal_events, dim3(grid_of(nb)), dim3(kBlock), 0, s, ne, ws.evs, ws.d0, ws.tcum,
                  ws.roff, ws.rwi, nr, ws.rto, ws.tau, ws.rc, ws.k1, ws.d1);
        BP_TRY(rocprim::radix_sort_pairs(ws.temp, tb, ws.k1, ws.k0, ws.d1, ws.d0, (size_t)nb, 0, 64, s));
        BP_TRY(rocprim::inclusive_scan_by_key(ws.temp, tb, rocprim::make_transform_iterator(ws.k0, KeyBlock{}),
                                              ws.d0, ws.acc, (size_t)nb, rocprim::plus<int64_t>(),
                                              rocprim::equal_to<uint32_t>(), s));
        BP_LAUNCH(k_bp_bal_diff, dim3(grid_of(nb)), dim3(kBlock), 0, s, nb, ws.k0, ws.acc, ws.W0, lmax,
                  ws.cstep);
    }
    if (nm > 0)
        BP_TRY(rocprim::inclusive_scan(ws.temp, tb, ws.cstep, ws.over_incl, (size_t)nm,
                                       rocprim::plus<int32_t>(), s));
    // 7. best balanced boundary; undo the rest
    const int groups = grid_of((int64_t)nm + 1, kBlock, kBestGroups);
    BP_LAUNCH(k_bp_best, dim3(groups), dim3(kBlock), 0, s, nm, ws.W0, K, lmax, ws.over_incl, ws.gain_incl,
              ws.best_g, ws.best_j);
    BP_LAUNCH(k_bp_best_final, dim3(1), dim3(64), 0, s, groups, ws.best_g, ws.best_j, ws.scal, counters);
    BP_LAUNCH(k_bp_revert, dim3(grid_of(n)), dim3(kBlock), 0, s, g, ws.part0, part, ws.pos, ws.stepof,
              ws.scal, mvto, counters);
    BP_TRY(launch_apply(g, apply.bk, part, pv, conn, W, mvto, apply.hub_t, apply.h, counters,
                        apply.dirty_threshold, apply.dirty, apply.tg, apply.tpv, apply.pc2, apply.perm,
                        apply.all_threshold, s));
    (void)stats;
#undef BP_LAUNCH
#undef BP_TRY
    return hipSuccess;
}

hipError_t launch_bp_stats(const BpWs &ws, int64_t *stats, hipStream_t s)
{
    hipLaunchKernelGGL(k_bp_stats, dim3(1), dim3(64), 0, s, ws.scal, stats);
    return hipGetLastError();
}

}  // namespace upr
