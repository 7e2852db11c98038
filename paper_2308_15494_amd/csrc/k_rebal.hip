// Rebalancing (Section 7.1), one synchronous sub-iteration per call of
// launch_rb_iteration.
//
// The paper's rebalancer pops nodes of overloaded blocks from a relaxed
// concurrent priority queue. Here the same priorities are bucketed and the
// order "bucket, then node id" is realised without sorting:
//   prepare   every node of an overloaded block picks its best-gain target
//             among blocks that stay balanced (or the lightest such block if
//             it is connected to none) and its priority bucket; per source
//             block a histogram of node weight over buckets
//   source    the cutoff bucket is the first whose cumulative weight covers
//             the excess; inside it, chunk sums over id ranges and a scan of
//             one chunk give the id bound of the minimal covering prefix
//   target    the same over the selected nodes aimed at each target: the
//             maximal prefix that fits the target's remaining capacity
//   moves     accepted nodes become moves, applied by the apply kernels
// Histogram rows and chunk rows are cleared by the kernel that reads them,
// so they are zero again at the start of the next sub-iteration.
#include "upr_common.h"

namespace upr {

static int grid_cap(int64_t items, int per_block, int cap)
{
    int64_t g = (items + per_block - 1) / per_block;
    if (g < 1) g = 1;
    if (g > cap) g = cap;
    return (int)g;
}

struct RbView {
    const int32_t *rtgt;
    const uint8_t *rbeta;
    const int64_t *W0;
    const int32_t *cbeta_src;
    const int32_t *theta_src;
    const int32_t *cbeta_tgt;
    const int32_t *theta_tgt;
};

__device__ __forceinline__ bool rb_selected(const RbView &r, int64_t v, int32_t a)
{
    const int cb = r.cbeta_src[a];
    const int be = r.rbeta[v];
    return be < cb || (be == cb && v < (int64_t)r.theta_src[a]);
}

__device__ __forceinline__ bool rb_accepted(const RbView &r, int64_t v, int32_t a, int32_t j)
{
    if (!rb_selected(r, v, a)) return false;
    const int cb = r.cbeta_tgt[j];
    const int be = r.rbeta[v];
    return be < cb || (be == cb && v < (int64_t)r.theta_tgt[j]);
}

// ------------------------------------------------------------------ begin --

// Count overloaded blocks, snapshot W, reset the overloaded-node list.
__global__ void k_rb_begin(int32_t k, const int64_t *W, int64_t lmax, int64_t *W0,
                           unsigned long long *counters)
{
    __shared__ unsigned long long red[4];
    unsigned long long over = 0;
    for (int j = threadIdx.x; j < k; j += kBlock) {
        const int64_t w = W[j];
        W0[j] = w;
        over += w > lmax;
    }
    over = block_sum(over, red);
    if (threadIdx.x == 0) {
        counters[CNT_OVER] = over;
        counters[CNT_OLIST] = 0;
    }
}

hipError_t launch_rb_begin(int32_t k, const int64_t *W, int64_t lmax, const RebalWs &r,
                           unsigned long long *counters, hipStream_t s)
{
    hipLaunchKernelGGL(k_rb_begin, dim3(1), dim3(kBlock), 0, s, k, W, lmax, r.W0, counters);
    return hipGetLastError();
}

// ---------------------------------------------------------------- prepare --

template <int G>
__global__ __launch_bounds__(kBlock) void k_rb_prepare(GraphView g, int32_t k,
                                                        const int32_t *__restrict__ part,
                                                        const int32_t *__restrict__ conn,
                                                        int64_t lmax, RebalWs r,
                                                        unsigned long long *counters)
{
    constexpr int GPB = kBlock / G;
    const int gl = threadIdx.x & (G - 1);
    const int64_t stride = (int64_t)gridDim.x * GPB;
    const int64_t first = (int64_t)blockIdx.x * GPB + threadIdx.x / G;
    const int64_t wave_first = (int64_t)blockIdx.x * GPB + (threadIdx.x & ~63) / G;
    for (int64_t vb = wave_first; vb < g.n; vb += stride) {
        const int64_t v = vb + (first - wave_first);
        bool active = false;
        int32_t a = 0;
        int64_t cv = 1;
        if (v < g.n) {
            a = part[v];
            if ((unsigned)a < (unsigned)k && r.W0[a] > lmax) {
                active = true;
                cv = node_weight(g, v);
            }
        }
        // best connected valid target: max (conn, -j); lightest valid: min (W, j)
        int64_t best = -1, lw = INT64_MAX;
        int32_t lj = 0x7fffffff;
        if (active) {
            const int32_t *row = conn + v * (int64_t)k;
            for (int j = gl; j < k; j += G) {
                if (j == a) continue;
                const int64_t wj = r.W0[j];
                if (wj + cv > lmax) continue;
                const int32_t cj = row[j];
                if (cj > 0) {
                    const int64_t p = ((int64_t)cj << 16) | (int64_t)(0xFFFF - j);
                    if (p > best) best = p;
                }
                if (wj < lw || (wj == lw && j < lj)) {
                    lw = wj;
                    lj = j;
                }
            }
        }
#pragma unroll
        for (int off = G / 2; off > 0; off >>= 1) {
            const int64_t ob = __shfl_xor(best, off);
            const int64_t ow = __shfl_xor(lw, off);
            const int32_t oj = __shfl_xor(lj, off);
            if (ob > best) best = ob;
            if (ow < lw || (ow == lw && oj < lj)) {
                lw = ow;
                lj = oj;
            }
        }
        bool push = false;
        if (active && gl == 0) {
            int32_t tgt = -1;
            int64_t ct = 0;
            if (best >= 0) {
                tgt = 0xFFFF - (int32_t)(best & 0xFFFF);
                ct = best >> 16;
            } else if (lj != 0x7fffffff) {
                tgt = lj;
                ct = 0;
            }
            r.rtgt[v] = tgt;
            if (tgt >= 0) {
                const int64_t ca = conn[v * (int64_t)k + a];
                const int be = rebalance_bucket(ct - ca, cv);
                r.rbeta[v] = (uint8_t)be;
                atomic_add_i64(&r.hist_src[(int64_t)a * kRbBuckets + be], cv);
                push = true;
            }
        }
        const int64_t slot = wave_append(push, &counters[CNT_OLIST]);
        if (push) r.olist[slot] = (int32_t)v;
    }
}

// ------------------------------------------------------------- cutoffs --

// Source: first bucket whose cumulative weight covers the excess.
// Target: first bucket whose cumulative weight exceeds the capacity.
// Rows are cleared after reading. Also resets the per-sub-iteration move
// counters (their previous users have finished).
__global__ void k_rb_cutoffs(int32_t k, int64_t lmax, RebalWs r, int target_side,
                             unsigned long long *counters)
{
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    if (!target_side && j == 0) {
        counters[CNT_MV_LOW] = 0;
        counters[CNT_MV_MID] = 0;
        counters[CNT_MOVED_NOW] = 0;
    }
    if (j >= k) return;
    int64_t *h = (target_side ? r.hist_tgt : r.hist_src) + (int64_t)j * kRbBuckets;
    const int64_t w0 = r.W0[j];
    int cut = kRbBuckets;
    int64_t rest = 0;
    if (!target_side) {
        if (w0 <= lmax) {
            r.cbeta_src[j] = kRbBuckets;
            return;
        }
        const int64_t excess = w0 - lmax;
        int64_t cum = 0;
        for (int b = 0; b < kRbBuckets; ++b) {
            const int64_t x = h[b];
            if (x) h[b] = 0;
            if (cut == kRbBuckets && cum + x >= excess) {
                cut = b;
                rest = excess - cum;
            }
            cum += x;
        }
        r.cbeta_src[j] = cut;
        r.need_src[j] = rest;
    } else {
        if (w0 > lmax) {  // an overloaded block is never a target
            r.cbeta_tgt[j] = kRbBuckets;
            return;
        }
        const int64_t cap = lmax - w0;
        int64_t cum = 0;
        for (int b = 0; b < kRbBuckets; ++b) {
            const int64_t x = h[b];
            if (x) h[b] = 0;
            if (cut == kRbBuckets && cum + x > cap) {
                cut = b;
                rest = cap - cum;
            }
            cum += x;
        }
        r.cbeta_tgt[j] = cut;
        r.room_tgt[j] = rest;
    }
}

// ------------------------------------------------------ chunk histograms --

// Nodes in the cutoff bucket add their weight to the chunk of their id.
__global__ __launch_bounds__(kBlock) void k_rb_chunks(GraphView g, const int32_t *part,
                                                       RebalWs r, RbView rv, int target_side,
                                                       const unsigned long long *counters)
{
    const int64_t cnt = (int64_t)counters[CNT_OLIST];
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < cnt; i += stride) {
        const int64_t v = r.olist[i];
        const int32_t a = part[v];
        const int be = r.rbeta[v];
        if (!target_side) {
            if (be == r.cbeta_src[a])
                atomic_add_i64(&r.chunk_src[(int64_t)a * r.nchunks + (v >> r.chunk_shift)],
                               node_weight(g, v));
        } else {
            const int32_t j = r.rtgt[v];
            if (be == r.cbeta_tgt[j] && rb_selected(rv, v, a))
                atomic_add_i64(&r.chunk_tgt[(int64_t)j * r.nchunks + (v >> r.chunk_shift)],
                               node_weight(g, v));
        }
    }
}

// Selected nodes add their weight to their target's bucket histogram.
__global__ __launch_bounds__(kBlock) void k_rb_tgt_hist(GraphView g, const int32_t *part,
                                                         RebalWs r, RbView rv,
                                                         const unsigned long long *counters)
{
    const int64_t cnt = (int64_t)counters[CNT_OLIST];
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < cnt; i += stride) {
        const int64_t v = r.olist[i];
        const int32_t a = part[v];
        if (rb_selected(rv, v, a))
            atomic_add_i64(&r.hist_tgt[(int64_t)r.rtgt[v] * kRbBuckets + r.rbeta[v]],
                           node_weight(g, v));
    }
}

// ------------------------------------------------------------- id bounds --

// One workgroup per block. Within the cutoff bucket, find the id bound:
//   source: theta = (first id at which the cumulative weight reaches need) + 1
//   target: theta = first id at which the cumulative weight exceeds room
// First over chunk sums (clearing the row), then over the ids of one chunk.
__global__ __launch_bounds__(kBlock) void k_rb_theta(GraphView g, int32_t k, const int32_t *part,
                                                      int64_t lmax, RebalWs r, RbView rv,
                                                      int target_side)
{
    __shared__ int64_t scan_lds[4];
    __shared__ int64_t found_lds[2];
    const int32_t j = blockIdx.x;
    int cb;
    int64_t limit;
    if (!target_side) {
        if (r.W0[j] <= lmax) return;
        cb = r.cbeta_src[j];
        limit = r.need_src[j];
    } else {
        cb = r.cbeta_tgt[j];
        limit = r.room_tgt[j];
    }
    if (cb >= kRbBuckets) return;
    int64_t *row = (target_side ? r.chunk_tgt : r.chunk_src) + (int64_t)j * r.nchunks;
    // reached(x): source x >= need, target x > room
    if (threadIdx.x == 0) {
        found_lds[0] = -1;
        found_lds[1] = 0;
    }
    __syncthreads();
    int64_t base = 0;
    for (int64_t c0 = 0; c0 < r.nchunks; c0 += kBlock) {
        const int64_t c = c0 + threadIdx.x;
        int64_t x = 0;
        if (c < r.nchunks) {
            x = row[c];
            if (x) row[c] = 0;
        }
        int64_t total;
        const int64_t inc = block_incl_scan(x, scan_lds, &total);
        const int64_t cum = base + inc;
        const bool hit = c < r.nchunks && x > 0 &&
                         (target_side ? (cum > limit) : (cum >= limit)) &&
                         !(target_side ? (cum - x > limit) : (cum - x >= limit));
        if (hit) {
            found_lds[0] = c;       // unique: the first chunk where the bound is reached
            found_lds[1] = cum - x; // weight before this chunk
        }
        base += total;
    }
    __syncthreads();
    const int64_t chunk = found_lds[0];
    int64_t before = found_lds[1];
    __syncthreads();
    if (chunk < 0) return;  // cannot happen when cb < kRbBuckets
    const int64_t id0 = chunk << r.chunk_shift;
    int64_t id1 = (chunk + 1) << r.chunk_shift;
    if (id1 > g.n) id1 = g.n;
    if (threadIdx.x == 0) found_lds[0] = -1;
    __syncthreads();
    for (int64_t b0 = id0; b0 < id1; b0 += kBlock) {
        const int64_t v = b0 + threadIdx.x;
        int64_t x = 0;
        if (v < id1) {
            const int32_t a = part[v];
            if ((unsigned)a < (unsigned)k && r.W0[a] > lmax && r.rtgt[v] >= 0 &&
                (int)r.rbeta[v] == cb) {
                if (!target_side) {
                    if (a == j) x = node_weight(g, v);
                } else {
                    if (r.rtgt[v] == j && rb_selected(rv, v, a)) x = node_weight(g, v);
                }
            }
        }
        int64_t total;
        const int64_t inc = block_incl_scan(x, scan_lds, &total);
        const int64_t cum = before + inc;
        const bool hit = x > 0 && (target_side ? (cum > limit) : (cum >= limit)) &&
                         !(target_side ? (cum - x > limit) : (cum - x >= limit));
        if (hit) found_lds[0] = v;
        __syncthreads();
        const int64_t fv = found_lds[0];
        __syncthreads();
        if (fv >= 0) {
            if (threadIdx.x == 0) {
                if (!target_side) r.theta_src[j] = (int32_t)(fv + 1);
                else r.theta_tgt[j] = (int32_t)fv;
            }
            return;
        }
        before += total;
    }
}

// ------------------------------------------------------------------ moves --

__device__ __forceinline__ int hub_index(const HubView &h, int64_t v)
{
    int lo = 0, hi = h.nh - 1;
    while (lo < hi) {
        int mid = (lo + hi) >> 1;
        if ((int64_t)h.ids[mid] < v) lo = mid + 1;
        else hi = mid;
    }
    return lo;
}

__global__ __launch_bounds__(kBlock) void k_rb_moves(GraphView g, const int32_t *part, RebalWs r,
                                                      RbView rv, HubView h, int64_t hub_t,
                                                      int64_t low_t, Move *mv_low, Move *mv_mid,
                                                      unsigned long long *counters)
{
    const int64_t cnt = (int64_t)counters[CNT_OLIST];
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    const int64_t wave_base = (int64_t)blockIdx.x * blockDim.x + (threadIdx.x & ~63);
    for (int64_t ib = wave_base; ib < cnt; ib += stride) {
        const int64_t i = ib + (threadIdx.x & 63);
        bool acc = false, lo = false, mid = false;
        int64_t v = 0;
        int32_t j = 0;
        if (i < cnt) {
            v = r.olist[i];
            const int32_t a = part[v];
            j = r.rtgt[v];
            acc = rb_accepted(rv, v, a, j);
            if (acc) {
                const int64_t deg = g.xadj[v + 1] - g.xadj[v];
                if (deg > hub_t) {
                    const int hi = hub_index(h, v);
                    h.from[hi] = a;
                    h.to[hi] = j;
                } else if (deg > low_t) {
                    mid = true;
                } else {
                    lo = true;
                }
            }
        }
        const int64_t sl = wave_append(lo, &counters[CNT_MV_LOW]);
        if (lo) mv_low[sl] = Move{(int32_t)v, j};
        const int64_t sm = wave_append(mid, &counters[CNT_MV_MID]);
        if (mid) mv_mid[sm] = Move{(int32_t)v, j};
        const uint64_t am = __ballot(acc);
        if (lane_id() == 0 && am) {
            atomicAdd(&counters[CNT_MOVED_NOW], (unsigned long long)__popcll(am));
            atomicAdd(&counters[CNT_REBAL_MOVES], (unsigned long long)__popcll(am));
        }
    }
}

// --------------------------------------------------------------- sequence --

hipError_t launch_rb_iteration(const GraphView &g, int32_t k, const int32_t *part,
                               const int32_t *conn, int64_t lmax, int64_t hub_t, int64_t low_t,
                               const RebalWs &r, const HubView &h, Move *mv_low, Move *mv_mid,
                               unsigned long long *counters, hipStream_t s)
{
    hipError_t e;
    const RbView rv{r.rtgt, r.rbeta, r.W0, r.cbeta_src, r.theta_src, r.cbeta_tgt, r.theta_tgt};
#define UPR_RP(GG)                                                                                 \
    hipLaunchKernelGGL(k_rb_prepare<GG>, dim3(grid_cap(g.n, kBlock / GG, 16384)), dim3(kBlock), 0, \
                       s, g, k, part, conn, lmax, r, counters)
    if (k <= 4) UPR_RP(4);
    else if (k <= 8) UPR_RP(8);
    else if (k <= 16) UPR_RP(16);
    else if (k <= 32) UPR_RP(32);
    else UPR_RP(64);
#undef UPR_RP
    if ((e = hipGetLastError()) != hipSuccess) return e;
    const dim3 kg((k + kBlock - 1) / kBlock);
    const int lg = grid_cap(g.n, kBlock, 2048);
    hipLaunchKernelGGL(k_rb_cutoffs, kg, dim3(kBlock), 0, s, k, lmax, r, 0, counters);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    hipLaunchKernelGGL(k_rb_chunks, dim3(lg), dim3(kBlock), 0, s, g, part, r, rv, 0, counters);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    hipLaunchKernelGGL(k_rb_theta, dim3(k), dim3(kBlock), 0, s, g, k, part, lmax, r, rv, 0);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    hipLaunchKernelGGL(k_rb_tgt_hist, dim3(lg), dim3(kBlock), 0, s, g, part, r, rv, counters);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    hipLaunchKernelGGL(k_rb_cutoffs, kg, dim3(kBlock), 0, s, k, lmax, r, 1, counters);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    hipLaunchKernelGGL(k_rb_chunks, dim3(lg), dim3(kBlock), 0, s, g, part, r, rv, 1, counters);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    hipLaunchKernelGGL(k_rb_theta, dim3(k), dim3(kBlock), 0, s, g, k, part, lmax, r, rv, 1);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    hipLaunchKernelGGL(k_rb_moves, dim3(lg), dim3(kBlock), 0, s, g, part, r, rv, h, hub_t, low_t,
                       mv_low, mv_mid, counters);
    return hipGetLastError();
}

}  // namespace upr
