// Graph preparation, block weights, cut and per-node statistics kernels:
// fills, the plan's degree scan and input validation, block weights, the
// statistics pass (cut, block weights, penalty buckets and availability),
// cut edges, and the compact partition copy.
#include "upr_common.h"

#include <cstring>

#include <rocprim/rocprim.hpp>

namespace upr {

// ------------------------------------------------------------------ fill --

template <typename T>
__global__ void k_fill(T *p, int64_t count, T value)
{
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < count;
         i += (int64_t)gridDim.x * blockDim.x)
        p[i] = value;
}

static int grid_for(int64_t items, int per_block, int cap = 8192)
{
    int64_t g = (items + per_block - 1) / per_block;
    if (g < 1) g = 1;
    if (g > cap) g = cap;
    return (int)g;
}

hipError_t launch_fill_i64(int64_t *p, int64_t count, int64_t value, hipStream_t s)
{
    if (count <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_fill<int64_t>, dim3(grid_for(count, kBlock * 4)), dim3(kBlock), 0, s, p,
                       count, value);
    return hipGetLastError();
}

hipError_t launch_fill_i32(int32_t *p, int64_t count, int32_t value, hipStream_t s)
{
    if (count <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_fill<int32_t>, dim3(grid_for(count, kBlock * 4)), dim3(kBlock), 0, s, p,
                       count, value);
    return hipGetLastError();
}

// ------------------------------------------------------------------ plan --

// Per node: weighted degree (lane group of 64 for weighted rows), maximum
// degree, hub list (unordered; the host sorts it).
// counters[0] = number of hubs, [1] = max degree, [2] = max weighted degree,
// [3] = total node weight, [4] = max node weight.
__global__ __launch_bounds__(kBlock) void k_plan_scan(GraphView g, int32_t *wdeg, int64_t hub_t,
                                                       int32_t *hub_list,
                                                       unsigned long long *counters)
{
    const int lane = lane_id();
    const int64_t waves = (int64_t)gridDim.x * (kBlock / 64);
    unsigned long long maxdeg = 0, maxw = 0, totw = 0, maxvw = 0;
    for (int64_t v = (int64_t)blockIdx.x * (kBlock / 64) + (threadIdx.x >> 6); v < g.n; v += waves) {
        const int64_t e0 = g.xadj[v], e1 = g.xadj[v + 1];
        const int64_t deg = e1 - e0;
        int64_t w = deg;
        if (g.adjwgt) {
            int64_t s = 0;
            for (int64_t e = e0 + lane; e < e1; e += 64) s += g.adjwgt[e];
            w = wave_sum(s);
        }
        if (lane == 0) {
            wdeg[v] = (int32_t)(w < 0x7fffffff ? w : 0x7fffffff);
            if ((unsigned long long)deg > maxdeg) maxdeg = deg;
            if ((unsigned long long)w > maxw) maxw = w;
            const unsigned long long cv = g.vwgt ? (unsigned long long)g.vwgt[v] : 1ull;
            totw += cv;
            if (cv > maxvw) maxvw = cv;
            if (deg > hub_t) {
                unsigned long long slot = atomicAdd(&counters[0], 1ull);
                hub_list[slot] = (int32_t)v;
            }
        }
    }
    // reduce (lane 0 of each wave holds values)
    unsigned long long m1 = maxdeg, m2 = maxw, m3 = maxvw;
    if (lane != 0) { m1 = 0; m2 = 0; m3 = 0; totw = 0; }
    for (int off = 32; off > 0; off >>= 1) {
        unsigned long long o1 = __shfl_xor(m1, off), o2 = __shfl_xor(m2, off);
        unsigned long long o3 = __shfl_xor(m3, off);
        m1 = o1 > m1 ? o1 : m1;
        m2 = o2 > m2 ? o2 : m2;
        m3 = o3 > m3 ? o3 : m3;
    }
    totw = wave_sum(totw);
    if (lane == 0) {
        atomicMax(&counters[1], m1);
        atomicMax(&counters[2], m2);
        atomicAdd(&counters[3], totw);
        atomicMax(&counters[4], m3);
    }
}

hipError_t launch_plan_scan(const GraphView &g, int32_t *wdeg, int64_t hub_t, int32_t *hub_list,
                            unsigned long long *counters, hipStream_t s)
{
    if (g.n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_plan_scan, dim3(grid_for(g.n, kBlock / 64, 2048)), dim3(kBlock), 0, s, g,
                       wdeg, hub_t, hub_list, counters);
    return hipGetLastError();
}

// CSR invariants. flags[0]: first bad xadj index + 1; flags[1]: bad entry
// (out of range / self-loop / unsorted or duplicate) + 1; flags[2]:
// asymmetric entry + 1; flags[3]: bad weight + 1. Each holds the minimum
// offending index (atomicMin over index + 1, 0 = none is encoded as ~0).
__device__ __forceinline__ bool has_entry(const GraphView &g, int64_t u, int64_t v, int32_t w,
                                          bool *wmatch)
{
    int64_t lo = g.xadj[u], hi = g.xadj[u + 1];
    while (lo < hi) {
        int64_t mid = (lo + hi) >> 1;
        if (g.adjncy[mid] < v) lo = mid + 1;
        else hi = mid;
    }
    if (lo < g.xadj[u + 1] && g.adjncy[lo] == v) {
        *wmatch = !g.adjwgt || g.adjwgt[lo] == w;
        return true;
    }
    return false;
}

__global__ __launch_bounds__(kBlock) void k_validate(GraphView g, unsigned long long *flags)
{
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; v < g.n; v += stride) {
        if (g.xadj[v + 1] < g.xadj[v]) atomicMin(&flags[0], (unsigned long long)v);
        if (g.vwgt && g.vwgt[v] <= 0) atomicMin(&flags[3], (unsigned long long)v);
    }
    if (blockIdx.x == 0 && threadIdx.x == 0 && g.xadj[0] != 0) atomicMin(&flags[0], 0ull);
}

__global__ __launch_bounds__(kBlock) void k_validate_edges(GraphView g, unsigned long long *flags,
                                                            int full)
{
    // one wave per node, lanes over the row
    const int lane = lane_id();
    const int64_t waves = (int64_t)gridDim.x * (kBlock / 64);
    for (int64_t v = (int64_t)blockIdx.x * (kBlock / 64) + (threadIdx.x >> 6); v < g.n; v += waves) {
        const int64_t e0 = g.xadj[v], e1 = g.xadj[v + 1];
        for (int64_t e = e0 + lane; e < e1; e += 64) {
            const int64_t u = g.adjncy[e];
            if (u < 0 || u >= g.n) {
                atomicMin(&flags[1], (unsigned long long)e);
                continue;
            }
            const int32_t w = g.adjwgt ? g.adjwgt[e] : 1;
            if (w <= 0) atomicMin(&flags[3], (unsigned long long)(g.n + e));
            if (!full) continue;
            if (u == v || (e > e0 && g.adjncy[e - 1] >= u)) {
                atomicMin(&flags[1], (unsigned long long)e);
                continue;
            }
            bool wm = true;
            if (!has_entry(g, u, v, w, &wm) || !wm) atomicMin(&flags[2], (unsigned long long)e);
        }
    }
}

hipError_t launch_validate(const GraphView &g, unsigned long long *flags, int stage,
                           hipStream_t s)
{
    if (g.n <= 0) return hipSuccess;
    if (stage == 0)
        hipLaunchKernelGGL(k_validate, dim3(grid_for(g.n, kBlock)), dim3(kBlock), 0, s, g, flags);
    else
        hipLaunchKernelGGL(k_validate_edges, dim3(grid_for(g.n, kBlock / 64, 16384)), dim3(kBlock),
                           0, s, g, flags, stage == 2 ? 1 : 0);
    return hipGetLastError();
}

// ---------------------------------------------------------- block weights --

__global__ __launch_bounds__(kBlock) void k_block_weights(GraphView g, int32_t k,
                                                           const int32_t *part, int64_t *W,
                                                           unsigned long long *counters)
{
    extern __shared__ __align__(16) unsigned char lds_raw[];
    int64_t *loc = (int64_t *)lds_raw;
    const bool use_lds = k <= 2048;
    if (use_lds) {
        for (int j = threadIdx.x; j < k; j += kBlock) loc[j] = 0;
        __syncthreads();
    }
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; v < g.n; v += stride) {
        const int32_t a = part[v];
        if ((unsigned)a >= (unsigned)k) {
            cnt_add(counters, CNT_BAD_INPUT, 1ull);
            continue;
        }
        const int64_t c = node_weight(g, v);
        if (use_lds) atomicAdd((unsigned long long *)&loc[a], (unsigned long long)c);
        else atomic_add_i64(&W[a], c);
    }
    if (use_lds) {
        __syncthreads();
        for (int j = threadIdx.x; j < k; j += kBlock)
            if (loc[j]) atomic_add_i64(&W[j], loc[j]);
    }
}

hipError_t launch_block_weights(const GraphView &g, int32_t k, const int32_t *part, int64_t *W,
                                unsigned long long *counters, hipStream_t s)
{
    if (g.n <= 0) return hipSuccess;
    const size_t lds = k <= 2048 ? (size_t)k * 8 : 0;
    hipLaunchKernelGGL(k_block_weights, dim3(grid_for(g.n, kBlock * 8, 2048)), dim3(kBlock), lds, s,
                       g, k, part, W, counters);
    return hipGetLastError();
}

// ------------------------------------------------------------------- cut --

// Per node, from a finished table: 2 * cut contribution
// omega(I(v)) - omega(v, Pi(v)), block weight (if W), and the penalty bucket
// of rebalance-available nodes (Section 5.3: t_den * omega(v, Pi(v)) >=
// t_num * omega(I(v)); slot(omega(v, Pi(v)), c(v))). One pass, each
// workgroup over a contiguous node range: 2 * cut into counters[cut_slot]
// and, for a batch, per graph into gstat[g][gs_slot]; out-of-range part
// values count in counters[CNT_BAD_INPUT]. Sums over the blocks of the
// graphs that own the range (the window) are kept in LDS when the window
// has at most cap_w (W) / cap_b (bucket) blocks, otherwise they go to
// global memory aggregated per wave.
constexpr int kStatsGraphs = 64;   // graphs of a window summed in LDS
__global__ __launch_bounds__(kBlock) void k_node_stats(GraphView g, Blocks bk,
                                                        const int64_t *__restrict__ goff,
                                                        int64_t span, int cap_w, int cap_b,
                                                        const int32_t *__restrict__ part,
                                                        const int32_t *__restrict__ conn,
                                                        const int32_t *__restrict__ wdeg,
                                                        int64_t *W, int64_t *bucket,
                                                        int32_t t_num, int32_t t_den,
                                                        unsigned long long *counters, int cut_slot,
                                                        uint8_t *avail_out, int64_t *gstat,
                                                        int gs_slot,
                                                        const int32_t *__restrict__ inner,
                                                        const uint32_t *__restrict__ hub_bits,
                                                        int cut_cond, int64_t *wsp, int64_t *bsp,
                                                        int ncopies)
{
    if (cut_cond && wave_cnt_get(counters, CNT_CUT_STALE) == 0) {
        // every apply since the first pass summed its change of the cut
        if (blockIdx.x == 0 && threadIdx.x < 64)
            wave_cnt_set(counters, cut_slot,
                         wave_cnt_get(counters, CNT_CUT2_BEFORE) +
                             wave_cnt_get(counters, CNT_CUT2_DELTA));
        return;
    }
    extern __shared__ __align__(16) unsigned char lds_raw[];
    __shared__ unsigned long long red[4];
    __shared__ unsigned long long bad;
    __shared__ int32_t win[2];
    __shared__ int64_t gsl[kStatsGraphs];
    const int32_t K = bk.total();
    const int32_t k = bk.k;
    const int64_t lo = (int64_t)blockIdx.x * span;
    const int64_t hi = lo + span < g.n ? lo + span : g.n;
    if (threadIdx.x == 0) {
        bad = 0;
        node_block_window(bk, goff, lo, hi, &win[0], &win[1]);
    }
    __syncthreads();
    const int32_t B0 = win[0], nb = win[1];
    const int32_t g0 = bk.graph(B0);
    // with copies (wsp / bsp) the sums go to this workgroup's copy, which the
    // bucket prefix pass adds into W and the histogram
    const unsigned cp = ncopies > 1 ? blockIdx.x % (unsigned)ncopies : 0u;
    int64_t *Wd = (W && wsp) ? wsp + (int64_t)cp * K : W;
    int64_t *Bd = (bucket && bsp) ? bsp + (int64_t)cp * K * kSlots : bucket;
    const bool w_lds = W && nb <= cap_w;
    const bool b_lds = bucket && nb <= cap_b;
    const bool s_lds = gstat && (nb + k - 1) / k <= kStatsGraphs;
    int64_t *lw = (int64_t *)lds_raw;
    int64_t *lb = (int64_t *)(lds_raw + (size_t)cap_w * 8);
    if (w_lds)
        for (int j = threadIdx.x; j < nb; j += kBlock) lw[j] = 0;
    if (b_lds)
        for (int j = threadIdx.x; j < nb * kSlots; j += kBlock) lb[j] = 0;
    if (s_lds)
        for (int j = threadIdx.x; j < kStatsGraphs; j += kBlock) gsl[j] = 0;
    __syncthreads();

    unsigned long long s = 0;
    // kStatsUnroll nodes per thread and step: their part entries, then their
    // table entries and degrees are loaded together (from clamped indices,
    // without a branch). Loop bound uniform per wave (wave_hist_add needs
    // whole waves).
    constexpr int kStatsUnroll = 8;
    for (int64_t vb = lo + (threadIdx.x & ~63); vb < hi; vb += (int64_t)kBlock * kStatsUnroll) {
        int32_t au[kStatsUnroll];
        int32_t inu[kStatsUnroll], wdu[kStatsUnroll];
#pragma unroll
        for (int i = 0; i < kStatsUnroll; ++i) {
            const int64_t v = vb + (int64_t)i * kBlock + lane_id();
            au[i] = part[v < hi ? v : hi - 1];
        }
#pragma unroll
        for (int i = 0; i < kStatsUnroll; ++i) {
            const int64_t v = vb + (int64_t)i * kBlock + lane_id();
            const int64_t vc = v < hi ? v : hi - 1;
            const int32_t a = (unsigned)au[i] < (unsigned)K ? au[i] : 0;
            inu[i] = inner ? inner[vc] : conn[vc * (int64_t)k + bk.local(a)];
            wdu[i] = wdeg[vc];
            if (inner && hub_bits && ((hub_bits[vc >> 5] >> (vc & 31)) & 1u))
                inu[i] = conn[vc * (int64_t)k + bk.local(a)];  // a hub (rare)
        }
#pragma unroll
        for (int i = 0; i < kStatsUnroll; ++i) {
            const int64_t v = vb + (int64_t)i * kBlock + lane_id();
            bool ok = v < hi;
            int32_t a = 0;
            int64_t cv = 1, inner = 0, wd = 0;
            if (ok) {
                a = au[i];
                if ((unsigned)a >= (unsigned)K) {
                    atomicAdd(&bad, 1ull);
                    ok = false;
                } else {
                    inner = inu[i];
                    wd = wdu[i];
                    cv = node_weight(g, v);
                    s += (unsigned long long)(wd - inner);
                }
            }
            const uint32_t x = (uint32_t)(a - B0);
            const bool inw = ok && x < (uint32_t)nb;
            if (gstat) {
                if (s_lds && inw) atomicAdd((unsigned long long *)&gsl[bk.graph(a) - g0],
                                            (unsigned long long)(wd - inner));
                wave_hist_add(gstat, (int64_t)bk.graph(a) * GS_COUNT + gs_slot, wd - inner,
                              ok && !(s_lds && inw));
            }
            if (W) {
                if (w_lds && inw) atomicAdd((unsigned long long *)&lw[x], (unsigned long long)cv);
                if (!w_lds) wave_hist_add(Wd, a, cv, ok);
                else wave_hist_add(Wd, a, cv, ok && !inw);
            }
            if (bucket) {
                const bool avail = ok && (int64_t)t_den * inner >= (int64_t)t_num * wd;
                if (avail_out && v < hi) avail_out[v] = avail ? 1 : 0;
                const int l = avail ? slot_of(inner, cv) : 0;
                if (b_lds && avail && inw)
                    atomicAdd((unsigned long long *)&lb[(int64_t)x * kSlots + l],
                              (unsigned long long)cv);
                wave_hist_add(Bd, (int64_t)a * kSlots + l, cv, avail && !(b_lds && inw));
            }
        }
    }
    s = block_sum(s, red);
    if (threadIdx.x == 0) {
        if (s) cnt_add(counters, cut_slot, s);
        if (bad) cnt_add(counters, CNT_BAD_INPUT, bad);
    }
    __syncthreads();
    if (w_lds)
        for (int j = threadIdx.x; j < nb; j += kBlock)
            if (lw[j]) atomic_add_i64(&Wd[B0 + j], lw[j]);
    if (b_lds)
        for (int j = threadIdx.x; j < nb * kSlots; j += kBlock)
            if (lb[j]) atomic_add_i64(&Bd[(int64_t)B0 * kSlots + j], lb[j]);
    if (s_lds)
        for (int j = threadIdx.x; j < kStatsGraphs; j += kBlock)
            if (gsl[j]) atomic_add_i64(&gstat[(int64_t)(g0 + j) * GS_COUNT + gs_slot], gsl[j]);
}

constexpr int kStatsRows = 512;                // workgroups of the statistics pass (one graph)
constexpr size_t kStatsWBytes = 8192;           // LDS block weights of a window
constexpr size_t kStatsBucketBytes = 57344;     // LDS slot histogram of a window

int64_t stats_span(int64_t n, int64_t max_span)
{
    int64_t G = (n + kBlock - 1) / kBlock;
    if (G > kStatsRows) G = kStatsRows;
    if (G < 1) G = 1;
    int64_t span = (n + G - 1) / G;
    if (max_span > 0 && span > max_span) span = max_span;
    return span < 1 ? 1 : span;
}

hipError_t launch_node_stats(const GraphView &g, const Blocks &bk, const StatsGeom &sg,
                             const int32_t *part, const int32_t *conn, const int32_t *wdeg,
                             int64_t *W, int64_t *bucket, int32_t t_num, int32_t t_den,
                             unsigned long long *counters, int cut_slot, uint8_t *avail,
                             int64_t *gstat, int gs_slot, hipStream_t s, const int32_t *inner,
                             const uint32_t *hub_bits, bool cut_cond, int64_t *wsp, int64_t *bsp,
                             int ncopies)
{
    if (g.n <= 0) return hipSuccess;
    const int64_t span = sg.span > 0 ? sg.span : stats_span(g.n, 0);
    const int32_t win = sg.window > 0 ? sg.window : bk.total();
    const int cap_w = (size_t)win * 8 <= kStatsWBytes ? win : 0;
    const int cap_b = (size_t)win * kSlots * 8 <= kStatsBucketBytes ? win : 0;
    const size_t lds = (W ? (size_t)cap_w * 8 : 0) + (bucket ? (size_t)cap_b * kSlots * 8 : 0);
    const int64_t rows = (g.n + span - 1) / span;
    hipLaunchKernelGGL(k_node_stats, dim3((unsigned)rows), dim3(kBlock), lds, s, g, bk, sg.goff,
                       span, W ? cap_w : 0, bucket ? cap_b : 0, part, conn, wdeg, W, bucket, t_num,
                       t_den, counters, cut_slot, avail, gstat, gs_slot, inner, hub_bits,
                       cut_cond && !W && !bucket && !gstat ? 1 : 0, wsp, bsp, ncopies);
    return hipGetLastError();
}

__global__ void k_store_half(const unsigned long long *counters, int slot, int64_t *out)
{
    const unsigned long long v = wave_cnt_get(counters, slot);
    if (threadIdx.x == 0 && blockIdx.x == 0) out[0] = (int64_t)(v / 2);
}

hipError_t launch_store_half(const unsigned long long *counters, int slot, int64_t *out,
                             hipStream_t s)
{
    hipLaunchKernelGGL(k_store_half, dim3(1), dim3(64), 0, s, counters, slot, out);
    return hipGetLastError();
}

// Hub row ranges: e0[i] = xadj[ids[i]], e1[i] = xadj[ids[i] + 1].
__global__ void k_hub_ranges(const int64_t *xadj, const int32_t *ids, int32_t nh, int64_t *e01)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= nh) return;
    e01[2 * i] = xadj[ids[i]];
    e01[2 * i + 1] = xadj[ids[i] + 1];
}

hipError_t launch_hub_ranges(const int64_t *xadj, const int32_t *ids, int32_t nh, int64_t *e01,
                             hipStream_t s)
{
    if (nh <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_hub_ranges, dim3((nh + kBlock - 1) / kBlock), dim3(kBlock), 0, s, xadj,
                       ids, nh, e01);
    return hipGetLastError();
}

// 2 * cut straight from the adjacency (Section 2 definition): one wave per
// node, lanes over the row.
__global__ __launch_bounds__(kBlock) void k_cut_edges(GraphView g,
                                                       const int32_t *__restrict__ part,
                                                       unsigned long long *counters, int slot)
{
    __shared__ unsigned long long red[4];
    const int lane = lane_id();
    const int64_t waves = (int64_t)gridDim.x * (kBlock / 64);
    unsigned long long s = 0;
    for (int64_t v = (int64_t)blockIdx.x * (kBlock / 64) + (threadIdx.x >> 6); v < g.n; v += waves) {
        const int32_t a = part[v];
        for (int64_t e = g.xadj[v] + lane; e < g.xadj[v + 1]; e += 64)
            if (part[g.adjncy[e]] != a) s += (unsigned long long)edge_weight(g, e);
    }
    s = block_sum(s, red);
    if (threadIdx.x == 0 && s) cnt_add(counters, slot, s);
}

hipError_t launch_cut_edges(const GraphView &g, const int32_t *part, unsigned long long *counters,
                            int slot, hipStream_t s)
{
    if (g.n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_cut_edges, dim3(grid_for(g.n, kBlock / 64, 16384)), dim3(kBlock), 0, s, g,
                       part, counters, slot);
    return hipGetLastError();
}

// pc2 (may be null): the same values in label order, pc2[i] = local block of
// order[i] (a gather of part; a bad value there is counted through its own
// node v).
__global__ void k_pack_part(int64_t n, Blocks bk, const int64_t *goff, const int32_t *part,
                            void *pc, int bytes, unsigned long long *counters,
                            const int32_t *order, void *pc2)
{
    const int32_t K = bk.total();
    bool bad = false;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; v < n; v += stride) {
        const int32_t B = part[v];
        if (pc2) {
            const int32_t B2 = part[order[v]];
            pset(pc2, bytes, v, (unsigned)B2 < (unsigned)K ? bk.local(B2) : 0);
        }
        if ((unsigned)B >= (unsigned)K) {
            bad = true;
            continue;
        }
        if (goff && bk.graph(B) != graph_of_node(goff, bk.ng, v)) bad = true;
        pset(pc, bytes, v, bk.local(B));
    }
    if (__ballot(bad) && lane_id() == 0) cnt_add(counters, CNT_BAD_INPUT, 1ull);
}

hipError_t launch_pack_part(int64_t n, const Blocks &bk, const int64_t *goff, const int32_t *part,
                            void *pc, int bytes, unsigned long long *counters, hipStream_t s,
                            const int32_t *order, void *pc2)
{
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_pack_part, dim3(grid_for(n, kBlock * 4, 4096)), dim3(kBlock), 0, s, n, bk,
                       goff, part, pc, bytes, counters, order, pc2);
    return hipGetLastError();
}

__global__ void k_check_part(int64_t n, int32_t k, const int32_t *part, unsigned long long *counters)
{
    bool bad = false;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; v < n; v += stride)
        bad |= (unsigned)part[v] >= (unsigned)k;
    if (__ballot(bad) && lane_id() == 0) cnt_add(counters, CNT_BAD_INPUT, 1ull);
}

hipError_t launch_check_part(int64_t n, int32_t k, const int32_t *part,
                             unsigned long long *counters, hipStream_t s)
{
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_check_part, dim3(grid_for(n, kBlock * 8, 2048)), dim3(kBlock), 0, s, n, k,
                       part, counters);
    return hipGetLastError();
}

// ------------------------------------------------------------- relabelling --

// The table build gathers the block of every neighbour; R-MAT-like graphs
// send most edges to few high-degree nodes. With neighbour ids renumbered by
// descending degree (ties by id), those nodes' entries of the compact
// partition copy share a few cache lines that stay in L1. Rows stay in place:
// only the neighbour ids in the table build's copy of the adjacency change.
__global__ void k_degree_keys(GraphView g, uint32_t *keys, int32_t *ids)
{
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; v < g.n; v += stride) {
        const int64_t d = g.xadj[v + 1] - g.xadj[v];
        keys[v] = 0xFFFFFFFFu - (uint32_t)(d < 0xFFFFFFFFll ? d : 0xFFFFFFFFll);
        ids[v] = (int32_t)v;
    }
}
__global__ void k_inverse(int64_t n, const int32_t *order, int32_t *perm)
{
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride)
        perm[order[i]] = (int32_t)i;
}
__global__ void k_relabel_adj(int64_t nnz, const int32_t *adjncy, const int32_t *perm, int32_t *adj_r)
{
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < nnz; e += stride)
        adj_r[e] = perm[adjncy[e]];
}

hipError_t launch_degree_relabel(const GraphView &g, int64_t nnz, int32_t *order, int32_t *perm,
                                 int32_t *adj_r, hipStream_t s)
{
    if (g.n <= 0) return hipSuccess;
    uint32_t *keys = nullptr, *keys2 = nullptr;
    int32_t *ids = nullptr;
    void *temp = nullptr;
    size_t bytes = 0;
    hipError_t e = hipMalloc((void **)&keys, sizeof(uint32_t) * g.n);
    if (e == hipSuccess) e = hipMalloc((void **)&keys2, sizeof(uint32_t) * g.n);
    if (e == hipSuccess) e = hipMalloc((void **)&ids, sizeof(int32_t) * g.n);
    if (e == hipSuccess)
        e = rocprim::radix_sort_pairs(nullptr, bytes, keys, keys2, ids, order, (size_t)g.n, 0, 32, s);
    if (e == hipSuccess) e = hipMalloc(&temp, bytes > 0 ? bytes : 1);
    if (e == hipSuccess) {
        hipLaunchKernelGGL(k_degree_keys, dim3(grid_for(g.n, kBlock * 4)), dim3(kBlock), 0, s, g, keys,
                           ids);
        e = hipGetLastError();
    }
    // a stable sort: equal degrees keep ascending ids
    if (e == hipSuccess)
        e = rocprim::radix_sort_pairs(temp, bytes, keys, keys2, ids, order, (size_t)g.n, 0, 32, s);
    if (e == hipSuccess) {
        hipLaunchKernelGGL(k_inverse, dim3(grid_for(g.n, kBlock * 4)), dim3(kBlock), 0, s, g.n, order,
                           perm);
        e = hipGetLastError();
    }
    if (e == hipSuccess && nnz > 0) {
        hipLaunchKernelGGL(k_relabel_adj, dim3(grid_for(nnz, kBlock * 4)), dim3(kBlock), 0, s, nnz,
                           g.adjncy, perm, adj_r);
        e = hipGetLastError();
    }
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    (void)hipFree(keys);
    (void)hipFree(keys2);
    (void)hipFree(ids);
    (void)hipFree(temp);
    return e;
}

}  // namespace upr
