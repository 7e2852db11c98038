// Move phase of one round: penalty buckets to prefix sums, penalised best
// move, conflict filter and scatter-apply.
//
// Degree classes: low-degree nodes are handled by groups of 8 lanes,
// mid-degree nodes by a whole wave64, hubs by several workgroups over chunks
// of their edges (the chunk list is built once per graph).
#include "upr_common.h"

namespace upr {

constexpr int kLowLanes = 8;
constexpr int kMidLanes = 64;

static int grid_cap(int64_t items, int per_block, int cap)
{
    int64_t g = (items + per_block - 1) / per_block;
    if (g < 1) g = 1;
    if (g > cap) g = cap;
    return (int)g;
}

// ----------------------------------------------------------- round init --

// Zero the counters, the penalty buckets and (rebuild form) the block
// weights; publish the round's Q16 penalty table.
__global__ void k_round_init(int32_t k, int64_t *bucket, int64_t *W, PenTable pq, int64_t *penq,
                             unsigned long long *counters, int zero_w)
{
    const int64_t tid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = tid; i < (int64_t)k * kSlots; i += stride) bucket[i] = 0;
    if (zero_w)
        for (int64_t i = tid; i < k; i += stride) W[i] = 0;
    if (tid < kSlots) penq[tid] = pq.q[tid];
    if (tid < CNT_COUNT) counters[tid] = 0;
}

hipError_t launch_round_init(int32_t k, int64_t *bucket, int64_t *W, const PenTable &pq,
                             int64_t *penq, unsigned long long *counters, int zero_w, hipStream_t s)
{
    hipLaunchKernelGGL(k_round_init, dim3(grid_cap((int64_t)k * kSlots, kBlock * 4, 1024)),
                       dim3(kBlock), 0, s, k, bucket, W, pq, penq, counters, zero_w);
    return hipGetLastError();
}

// Prefix sums over slots: cb[j][l] = sum_{i <= l} c(B_{i,j}).
__global__ void k_cb_prefix(int32_t k, int64_t *bucket)
{
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= k) return;
    int64_t *b = bucket + (int64_t)j * kSlots;
    int64_t run = 0;
    for (int l = 0; l < kSlots; ++l) {
        run += b[l];
        b[l] = run;
    }
}

hipError_t launch_cb_prefix(int32_t k, int64_t *bucket, hipStream_t s)
{
    hipLaunchKernelGGL(k_cb_prefix, dim3((k + kBlock - 1) / kBlock), dim3(kBlock), 0, s, k, bucket);
    return hipGetLastError();
}

// ------------------------------------------------------------- best move --

// Least l with cb[l] >= x (cb nondecreasing), kSlots if none.
__device__ __forceinline__ int covering_slot(const int64_t *cb, int64_t x)
{
    if (cb[kSlots - 1] < x) return kSlots;
    int lo = 0, hi = kSlots - 1;
    while (lo < hi) {
        int mid = (lo + hi) >> 1;
        if (cb[mid] >= x) hi = mid;
        else lo = mid + 1;
    }
    return lo;
}

// S2: per node v in block a, over blocks j != a with omega(v, V_j) >
// omega(v, V_a) (only those can give a positive score):
//   X = W[j] + c(v) - L_max; P = 0 if X <= 0; constrained: skip if X > 0;
//   penalised: l = least slot with cb[j][l] >= X (skip if none),
//   P = min(penq[l] * c(v), 2^62); score = delta * 2^16 - P.
// The best score (ties to the smaller j) is reduced over a group of G lanes
// as the packed value (score << 16 | (0xFFFF - j)). key[v] = score << 16 | j
// for candidates (score > 0), -1 otherwise.
template <int G>
__global__ __launch_bounds__(kBlock) void k_best_move(
    GraphView g, int32_t k, const int32_t *__restrict__ part, const int32_t *__restrict__ conn,
    const int64_t *__restrict__ W, const int64_t *__restrict__ cb, const int64_t *__restrict__ penq,
    int64_t lmax, int mode, int64_t low_t, int64_t hub_t, int64_t *__restrict__ key,
    int64_t *__restrict__ pen, int32_t *cl_low, int32_t *cl_mid, unsigned long long *counters)
{
    constexpr int GPB = kBlock / G;
    const int gl = threadIdx.x & (G - 1);
    const int64_t stride = (int64_t)gridDim.x * GPB;
    const int64_t first = (int64_t)blockIdx.x * GPB + threadIdx.x / G;
    // all groups of a wave iterate the same number of times (wave-uniform
    // bound), so the wave-level append below sees every lane
    const int64_t wave_first = (int64_t)blockIdx.x * GPB + (threadIdx.x & ~63) / G;
    for (int64_t vb = wave_first; vb < g.n; vb += stride) {
        const int64_t v = vb + (first - wave_first);
        const bool valid = v < g.n;
        int64_t best = 0, bestP = 0;
        int32_t a = 0;
        int64_t cv = 1;
        if (valid) {
            a = part[v];
            cv = node_weight(g, v);
            if ((unsigned)a < (unsigned)k) {
                const int32_t *row = conn + v * (int64_t)k;
                const int32_t ca = row[a];
                for (int j = gl; j < k; j += G) {
                    const int32_t cj = row[j];
                    if (cj <= ca || j == a) continue;
                    const int64_t delta = (int64_t)cj - ca;
                    const int64_t x = W[j] + cv - lmax;
                    int64_t P = 0;
                    if (x > 0) {
                        if (mode == 1) continue;
                        if (mode == 0) {
                            const int l = covering_slot(cb + (int64_t)j * kSlots, x);
                            if (l >= kSlots) continue;
                            P = sat_mul_pen(penq[l], cv);
                        }
                    }
                    const int64_t sc = delta * 65536 - P;
                    if (sc <= 0) continue;
                    const int64_t packed = (sc << 16) | (int64_t)(0xFFFF - j);
                    if (packed > best) {
                        best = packed;
                        bestP = P;
                    }
                }
            }
        }
#pragma unroll
        for (int off = G / 2; off > 0; off >>= 1) {
            const int64_t ob = __shfl_xor(best, off);
            const int64_t op = __shfl_xor(bestP, off);
            if (ob > best) {
                best = ob;
                bestP = op;
            }
        }
        const bool leader = valid && gl == 0;
        const bool cand = leader && best > 0;
        int64_t deg = 0;
        if (leader) {
            if (cand) {
                const int64_t sc = best >> 16;
                const int32_t j = 0xFFFF - (int32_t)(best & 0xFFFF);
                key[v] = (sc << 16) | j;
                pen[v] = bestP;
                deg = g.xadj[v + 1] - g.xadj[v];
            } else {
                key[v] = -1;
            }
        }
        const bool is_low = cand && deg <= low_t;
        const bool is_mid = cand && deg > low_t && deg <= hub_t;
        const int64_t sl = wave_append(is_low, &counters[CNT_CL_LOW]);
        if (is_low) cl_low[sl] = (int32_t)v;
        const int64_t sm = wave_append(is_mid, &counters[CNT_CL_MID]);
        if (is_mid) cl_mid[sm] = (int32_t)v;
        const uint64_t cm = __ballot(cand);
        if (lane_id() == 0 && cm) atomicAdd(&counters[CNT_CAND], (unsigned long long)__popcll(cm));
    }
}

hipError_t launch_best_move(const GraphView &g, int32_t k, const int32_t *part, const int32_t *conn,
                            const int64_t *W, const int64_t *cb, const int64_t *penq, int64_t lmax,
                            int mode, int64_t low_t, int64_t hub_t, int64_t *key, int64_t *pen,
                            int32_t *cl_low, int32_t *cl_mid, unsigned long long *counters,
                            hipStream_t s)
{
    if (g.n <= 0) return hipSuccess;
#define UPR_BM(GG)                                                                                \
    hipLaunchKernelGGL(k_best_move<GG>, dim3(grid_cap(g.n, kBlock / GG, 16384)), dim3(kBlock), 0, \
                       s, g, k, part, conn, W, cb, penq, lmax, mode, low_t, hub_t, key, pen,      \
                       cl_low, cl_mid, counters)
    if (k <= 4) UPR_BM(4);
    else if (k <= 8) UPR_BM(8);
    else if (k <= 16) UPR_BM(16);
    else if (k <= 32) UPR_BM(32);
    else UPR_BM(64);
#undef UPR_BM
    return hipGetLastError();
}

// ---------------------------------------------------------------- filter --

// Contribution f(x) of a neighbour in block x to the move a -> b.
__device__ __forceinline__ int move_sign(int32_t x, int32_t a, int32_t b)
{
    return (x == b) - (x == a);
}

// S3 for candidate v (a -> b, score sv): pessimistic gain over its row
// [e0, e1) strided by `step` starting at e0 + off.
__device__ __forceinline__ int64_t pessimistic_part(const GraphView &g, const int32_t *part,
                                                    const int64_t *key, int64_t v, int32_t a,
                                                    int32_t b, int64_t sv, int64_t e0, int64_t e1,
                                                    int off, int step)
{
    int64_t acc = 0;
    for (int64_t e = e0 + off; e < e1; e += step) {
        const int32_t u = g.adjncy[e];
        int f = move_sign(part[u], a, b);
        const int64_t ku = key[u];
        if (ku >= 0) {
            const int64_t su = ku >> 16;
            if (su > sv || (su == sv && (int64_t)u < v)) {
                const int ft = move_sign((int32_t)(ku & 0xFFFF), a, b);
                f = ft < f ? ft : f;
            }
        }
        acc += (int64_t)edge_weight(g, e) * f;
    }
    return acc;
}

template <int G>
__global__ __launch_bounds__(kBlock) void k_filter(GraphView g, const int32_t *__restrict__ part,
                                                    const int64_t *__restrict__ key,
                                                    const int64_t *__restrict__ pen,
                                                    const int32_t *__restrict__ list, int cnt_slot,
                                                    Move *out, int out_slot, uint8_t *accflag,
                                                    unsigned long long *counters)
{
    constexpr int GPB = kBlock / G;
    const int gl = threadIdx.x & (G - 1);
    const int64_t cnt = (int64_t)counters[cnt_slot];
    const int64_t stride = (int64_t)gridDim.x * GPB;
    const int64_t first = (int64_t)blockIdx.x * GPB + threadIdx.x / G;
    const int64_t wave_first = (int64_t)blockIdx.x * GPB + (threadIdx.x & ~63) / G;
    for (int64_t ib = wave_first; ib < cnt; ib += stride) {
        const int64_t i = ib + (first - wave_first);
        const bool valid = i < cnt;
        int64_t acc = 0, v = 0, kv = 0;
        int32_t a = 0, b = 0;
        if (valid) {
            v = list[i];
            kv = key[v];
            a = part[v];
            b = (int32_t)(kv & 0xFFFF);
            acc = pessimistic_part(g, part, key, v, a, b, kv >> 16, g.xadj[v], g.xadj[v + 1], gl, G);
        }
        acc = group_sum<G>(acc);
        bool ok = false;
        if (valid && gl == 0) {
            ok = acc * 65536 - pen[v] > 0;
            accflag[v] = ok ? 1 : 0;
        }
        const int64_t slot = wave_append(ok, &counters[out_slot]);
        if (ok) out[slot] = Move{(int32_t)v, b};
        const uint64_t am = __ballot(ok);
        if (lane_id() == 0 && am) atomicAdd(&counters[CNT_ACC], (unsigned long long)__popcll(am));
    }
}

hipError_t launch_filter(const GraphView &g, const int32_t *part, const int64_t *key,
                         const int64_t *pen, const int32_t *cl_low, const int32_t *cl_mid,
                         Move *mv_low, Move *mv_mid, uint8_t *accflag,
                         unsigned long long *counters, hipStream_t s)
{
    if (g.n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_filter<kLowLanes>, dim3(grid_cap(g.n, kBlock / kLowLanes, 4096)),
                       dim3(kBlock), 0, s, g, part, key, pen, cl_low, (int)CNT_CL_LOW, mv_low,
                       (int)CNT_MV_LOW, accflag, counters);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_filter<kMidLanes>, dim3(grid_cap(g.n, kBlock / kMidLanes, 4096)),
                       dim3(kBlock), 0, s, g, part, key, pen, cl_mid, (int)CNT_CL_MID, mv_mid,
                       (int)CNT_MV_MID, accflag, counters);
    return hipGetLastError();
}

// Hub candidates: each chunk adds its part of the pessimistic gain.
__global__ __launch_bounds__(kBlock) void k_filter_hub(GraphView g, const int32_t *part,
                                                        const int64_t *key, HubView h)
{
    __shared__ int64_t red[4];
    const HubChunk c = h.chunks[blockIdx.x];
    const int64_t v = h.ids[c.hub];
    const int64_t kv = key[v];
    if (kv < 0) return;  // uniform over the workgroup
    const int32_t a = part[v], b = (int32_t)(kv & 0xFFFF);
    int64_t acc = pessimistic_part(g, part, key, v, a, b, kv >> 16, c.e0, c.e1, threadIdx.x, kBlock);
    acc = block_sum(acc, red);
    if (threadIdx.x == 0 && acc) atomic_add_i64(&h.gacc[c.hub], acc);
}

// Hub candidates: decide, record the move for the apply step, reset gacc.
__global__ void k_filter_hub_final(const int32_t *part, const int64_t *key, const int64_t *pen,
                                   HubView h, uint8_t *accflag, unsigned long long *counters)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= h.nh) return;
    const int64_t v = h.ids[i];
    const int64_t kv = key[v];
    const int64_t acc = h.gacc[i];
    h.gacc[i] = 0;
    if (kv < 0) return;
    const bool ok = acc * 65536 - pen[v] > 0;
    accflag[v] = ok ? 1 : 0;
    if (ok) {
        h.from[i] = part[v];
        h.to[i] = (int32_t)(kv & 0xFFFF);
        atomicAdd(&counters[CNT_ACC], 1ull);
    }
}

hipError_t launch_filter_hub(const GraphView &g, const int32_t *part, const int64_t *key,
                             const int64_t *pen, const HubView &h, uint8_t *accflag,
                             unsigned long long *counters, hipStream_t s)
{
    if (h.nh <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_filter_hub, dim3((unsigned)h.nchunks), dim3(kBlock), 0, s, g, part, key,
                       h);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_filter_hub_final, dim3((h.nh + kBlock - 1) / kBlock), dim3(kBlock), 0, s,
                       part, key, pen, h, accflag, counters);
    return hipGetLastError();
}

// ----------------------------------------------------------------- apply --

// S4 (and the rebalancing moves): for a move v: a -> b, part[v] = b,
// W[a] -= c(v), W[b] += c(v), and for every neighbour u
// conn[u][a] -= omega(v, u), conn[u][b] += omega(v, u). Integer atomics
// commute, so the result does not depend on the order of the moves.
template <int G>
__global__ __launch_bounds__(kBlock) void k_apply(GraphView g, int32_t k, int32_t *part,
                                                   int32_t *conn, int64_t *W,
                                                   const Move *__restrict__ list, int cnt_slot,
                                                   unsigned long long *counters)
{
    extern __shared__ __align__(16) unsigned char lds_raw[];
    int64_t *wloc = (int64_t *)lds_raw;
    const bool use_lds = k <= 2048;
    const int64_t cnt = (int64_t)counters[cnt_slot];
    if (cnt == 0) return;  // uniform
    if (use_lds) {
        for (int j = threadIdx.x; j < k; j += kBlock) wloc[j] = 0;
        __syncthreads();
    }
    constexpr int GPB = kBlock / G;
    const int gl = threadIdx.x & (G - 1);
    const int64_t stride = (int64_t)gridDim.x * GPB;
    for (int64_t i = (int64_t)blockIdx.x * GPB + threadIdx.x / G; i < cnt; i += stride) {
        const Move m = list[i];
        const int64_t v = m.v;
        const int32_t b = m.to;
        int32_t a = 0;
        if (gl == 0) a = part[v];
        a = __shfl(a, (int)(threadIdx.x & 63) & ~(G - 1));
        const int64_t e0 = g.xadj[v], e1 = g.xadj[v + 1];
        for (int64_t e = e0 + gl; e < e1; e += G) {
            const int64_t u = g.adjncy[e];
            const int32_t w = edge_weight(g, e);
            atomicAdd(&conn[u * k + a], -w);
            atomicAdd(&conn[u * k + b], w);
        }
        if (gl == 0) {
            const int64_t cv = node_weight(g, v);
            part[v] = b;
            if (use_lds) {
                atomicAdd((unsigned long long *)&wloc[a], (unsigned long long)(-cv));
                atomicAdd((unsigned long long *)&wloc[b], (unsigned long long)cv);
            } else {
                atomic_add_i64(&W[a], -cv);
                atomic_add_i64(&W[b], cv);
            }
        }
    }
    if (use_lds) {
        __syncthreads();
        for (int j = threadIdx.x; j < k; j += kBlock)
            if (wloc[j]) atomic_add_i64(&W[j], wloc[j]);
    }
}

// Hub moves: each chunk updates the rows of its neighbours.
__global__ __launch_bounds__(kBlock) void k_apply_hub(GraphView g, int32_t k, int32_t *conn,
                                                       HubView h)
{
    const HubChunk c = h.chunks[blockIdx.x];
    const int32_t b = h.to[c.hub];
    if (b < 0) return;
    const int32_t a = h.from[c.hub];
    for (int64_t e = c.e0 + threadIdx.x; e < c.e1; e += kBlock) {
        const int64_t u = g.adjncy[e];
        const int32_t w = edge_weight(g, e);
        atomicAdd(&conn[u * k + a], -w);
        atomicAdd(&conn[u * k + b], w);
    }
}

// Hub moves: part and block weights, then clear the move record.
__global__ void k_apply_hub_final(GraphView g, int32_t *part, int64_t *W, HubView h)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= h.nh) return;
    const int32_t b = h.to[i];
    if (b < 0) return;
    const int64_t v = h.ids[i];
    const int32_t a = h.from[i];
    const int64_t cv = node_weight(g, v);
    part[v] = b;
    atomic_add_i64(&W[a], -cv);
    atomic_add_i64(&W[b], cv);
    h.to[i] = -1;
}

hipError_t launch_apply(const GraphView &g, int32_t k, int32_t *part, int32_t *conn, int64_t *W,
                        const Move *mv_low, const Move *mv_mid, const HubView &h,
                        unsigned long long *counters, hipStream_t s)
{
    if (g.n <= 0) return hipSuccess;
    const size_t lds = k <= 2048 ? (size_t)k * 8 : 0;
    hipLaunchKernelGGL(k_apply<kLowLanes>, dim3(grid_cap(g.n, kBlock / kLowLanes, 2048)),
                       dim3(kBlock), lds, s, g, k, part, conn, W, mv_low, (int)CNT_MV_LOW, counters);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_apply<kMidLanes>, dim3(grid_cap(g.n, kBlock / kMidLanes, 2048)),
                       dim3(kBlock), lds, s, g, k, part, conn, W, mv_mid, (int)CNT_MV_MID, counters);
    e = hipGetLastError();
    if (e != hipSuccess || h.nh <= 0) return e;
    hipLaunchKernelGGL(k_apply_hub, dim3((unsigned)h.nchunks), dim3(kBlock), 0, s, g, k, conn, h);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_apply_hub_final, dim3((h.nh + kBlock - 1) / kBlock), dim3(kBlock), 0, s, g,
                       part, W, h);
    return hipGetLastError();
}

// ----------------------------------------------------------------- stats --

__global__ void k_stats_final(int64_t *stats, const unsigned long long *c, int64_t lmax,
                              int64_t iters, int64_t status)
{
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    stats[0] = lmax;
    stats[1] = (int64_t)c[CNT_CUT2_BEFORE] / 2;
    stats[2] = (int64_t)c[CNT_CUT2_MOVES] / 2;
    stats[3] = (int64_t)c[CNT_CUT2_AFTER] / 2;
    stats[4] = (int64_t)c[CNT_CAND];
    stats[5] = (int64_t)c[CNT_ACC];
    stats[6] = (int64_t)c[CNT_REBAL_MOVES];
    stats[7] = iters;
    stats[8] = status;
    for (int i = 9; i < 12; ++i) stats[i] = 0;
}

hipError_t launch_stats_final(int64_t *stats, const unsigned long long *counters, int64_t lmax,
                              int64_t iters, int64_t status, hipStream_t s)
{
    hipLaunchKernelGGL(k_stats_final, dim3(1), dim3(64), 0, s, stats, counters, lmax, iters, status);
    return hipGetLastError();
}

__global__ void k_export_moves(int64_t n, const int64_t *key, const int64_t *pen,
                               const uint8_t *accflag, int32_t *target, int64_t *score,
                               int64_t *pen_out, uint8_t *accept)
{
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; v < n; v += stride) {
        const int64_t kv = key[v];
        const bool c = kv >= 0;
        if (target) target[v] = c ? (int32_t)(kv & 0xFFFF) : -1;
        if (score) score[v] = c ? (kv >> 16) : 0;
        if (pen_out) pen_out[v] = c ? pen[v] : 0;
        if (accept) accept[v] = c ? accflag[v] : 0;
    }
}

hipError_t launch_export_moves(int64_t n, const int64_t *key, const int64_t *pen,
                               const uint8_t *accflag, int32_t *target, int64_t *score,
                               int64_t *pen_out, uint8_t *accept, hipStream_t s)
{
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_export_moves, dim3(grid_cap(n, kBlock * 4, 4096)), dim3(kBlock), 0, s, n,
                       key, pen, accflag, target, score, pen_out, accept);
    return hipGetLastError();
}

}  // namespace upr
