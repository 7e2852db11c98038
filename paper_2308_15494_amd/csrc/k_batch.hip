// Batches: many independent graphs refined by the same launches.
//
// A batch is the disjoint union of its graphs, built once: node ids of graph
// g are shifted by its node offset, so the union is an ordinary CSR graph and
// every kernel of the round runs over it unchanged except for the block ids
// (global id g*k + j, see Blocks). This file holds the union construction and
// the per-graph statistics.
#include "upr_common.h"

#include <algorithm>

namespace upr {

namespace {

int grid_for(int64_t items, int per_block, int cap)
{
    int64_t g = (items + per_block - 1) / per_block;
    if (g < 1) g = 1;
    if (g > cap) g = cap;
    return (int)g;
}

}  // namespace

// Copy graph g into the union: rows shifted by the edge offset, neighbour
// ids by the node offset; missing weights become 1.
__global__ void k_batch_copy(GraphView src, int64_t node_off, int64_t edge_off, int64_t *xadj,
                             int32_t *adjncy, int32_t *adjwgt, int32_t *vwgt, int last)
{
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    for (int64_t v = t; v < src.n; v += stride) {
        xadj[node_off + v] = edge_off + src.xadj[v];
        if (vwgt) vwgt[node_off + v] = src.vwgt ? src.vwgt[v] : 1;
    }
    if (last && t == 0 && src.n > 0) xadj[node_off + src.n] = edge_off + src.xadj[src.n];
    const int64_t nnz = src.n > 0 ? src.xadj[src.n] : 0;
    for (int64_t e = t; e < nnz; e += stride) {
        adjncy[edge_off + e] = (int32_t)(node_off + src.adjncy[e]);
        if (adjwgt) adjwgt[edge_off + e] = src.adjwgt ? src.adjwgt[e] : 1;
    }
}

hipError_t launch_batch_copy(const GraphView &src, int64_t node_off, int64_t edge_off,
                             int64_t nnz, int64_t *xadj, int32_t *adjncy, int32_t *adjwgt,
                             int32_t *vwgt, int last, hipStream_t s)
{
    const int64_t items = std::max<int64_t>(src.n, nnz);
    hipLaunchKernelGGL(k_batch_copy, dim3(grid_for(items, kBlock, 4096)), dim3(kBlock), 0, s, src,
                       node_off, edge_off, xadj, adjncy, adjwgt, vwgt, last);
    return hipGetLastError();
}

// Carry graphs' round state from one batch into another: record r =
// (source node offset, destination node offset, nodes, source graph,
// destination graph); workgroups (x, r) copy strided parts of graph r's
// partition (block ids moved from the source graph's range to the
// destination's), its table rows and its block weights.
__global__ void k_batch_carry(const int64_t *rec, int32_t k, const int32_t *src_part,
                              const int32_t *src_conn, const int64_t *src_W, int32_t *dst_part,
                              int32_t *dst_conn, int64_t *dst_W)
{
    const int64_t *r = rec + 5 * (int64_t)blockIdx.y;
    const int64_t so = r[0], d0 = r[1], n = r[2];
    const int32_t shift = (int32_t)((r[4] - r[3]) * k);
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    for (int64_t v = t; v < n; v += stride) dst_part[d0 + v] = src_part[so + v] + shift;
    const int64_t cells = n * k;
    const int32_t *sc = src_conn + so * k;
    int32_t *dc = dst_conn + d0 * k;
    for (int64_t i = t; i < cells; i += stride) dc[i] = sc[i];
    for (int64_t j = t; j < k; j += stride) dst_W[r[4] * k + j] = src_W[r[3] * k + j];
}

hipError_t launch_batch_carry(const int64_t *rec, int32_t nrec, int64_t max_cells, int32_t k,
                              const int32_t *src_part, const int32_t *src_conn,
                              const int64_t *src_W, int32_t *dst_part, int32_t *dst_conn,
                              int64_t *dst_W, hipStream_t s)
{
    const int gx = grid_for(max_cells, kBlock * 4, 256);
    for (int32_t r0 = 0; r0 < nrec; r0 += 65535) {  // grid y is at most 65535
        const int32_t nr = nrec - r0 < 65535 ? nrec - r0 : 65535;
        hipLaunchKernelGGL(k_batch_carry, dim3(gx, nr), dim3(kBlock), 0, s, rec + 5 * (int64_t)r0, k,
                           src_part, src_conn, src_W, dst_part, dst_conn, dst_W);
        const hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

// Per graph (one workgroup each): total node weight and the largest one.
__global__ void k_batch_totals(const int64_t *goff, const int32_t *vwgt, int64_t *out)
{
    __shared__ int64_t red[4];
    const int g = blockIdx.x;
    const int64_t v0 = goff[g], v1 = goff[g + 1];
    int64_t sum = 0, mx = 0;
    for (int64_t v = v0 + threadIdx.x; v < v1; v += kBlock) {
        const int64_t c = vwgt ? vwgt[v] : 1;
        sum += c;
        mx = c > mx ? c : mx;
    }
    sum = block_sum(sum, red);
    for (int off = 32; off > 0; off >>= 1) {
        const int64_t o = __shfl_xor(mx, off);
        mx = o > mx ? o : mx;
    }
    __shared__ int64_t mred[4];
    if (lane_id() == 0) mred[threadIdx.x >> 6] = mx;
    __syncthreads();
    if (threadIdx.x == 0) {
        int64_t m = mred[0];
        for (int i = 1; i < kBlock / 64; ++i) m = mred[i] > m ? mred[i] : m;
        out[2 * g] = sum;
        out[2 * g + 1] = m;
    }
}

hipError_t launch_batch_totals(const int64_t *goff, int32_t ng, const int32_t *vwgt, int64_t *out,
                               hipStream_t s)
{
    if (ng <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_batch_totals, dim3(ng), dim3(kBlock), 0, s, goff, vwgt, out);
    return hipGetLastError();
}

// Per-graph candidate and accepted counts after the filter. Each workgroup
// takes a contiguous node range and sums per graph in LDS over the graphs
// that own it (a range meets few graphs), then adds one value per graph.
constexpr int kMoveStatsGraphs = 64;
__global__ __launch_bounds__(kBlock) void k_batch_move_stats(int64_t n, int64_t span, Blocks bk,
                                                              const int64_t *goff,
                                                              const int32_t *part,
                                                              const int64_t *key,
                                                              const uint8_t *accflag,
                                                              int64_t *gstat)
{
    __shared__ unsigned long long lc[kMoveStatsGraphs], la[kMoveStatsGraphs];
    __shared__ int32_t g0s;
    const int64_t lo = (int64_t)blockIdx.x * span;
    const int64_t hi = lo + span < n ? lo + span : n;
    if (threadIdx.x == 0) g0s = graph_of_node(goff, bk.ng, lo);
    for (int j = threadIdx.x; j < kMoveStatsGraphs; j += kBlock) {
        lc[j] = 0;
        la[j] = 0;
    }
    __syncthreads();
    const int32_t g0 = g0s;
    for (int64_t v = lo + threadIdx.x; v < hi; v += kBlock) {
        if (key[v] < 0) continue;
        const bool acc = accflag[v] != 0;
        const int32_t gi = bk.graph(part[v]);
        const uint32_t x = (uint32_t)(gi - g0);
        if (x < (uint32_t)kMoveStatsGraphs) {
            atomicAdd(&lc[x], 1ull);
            if (acc) atomicAdd(&la[x], 1ull);
        } else {
            atomic_add_i64(&gstat[(int64_t)gi * GS_COUNT + GS_CAND], 1);
            if (acc) atomic_add_i64(&gstat[(int64_t)gi * GS_COUNT + GS_ACC], 1);
        }
    }
    __syncthreads();
    for (int j = threadIdx.x; j < kMoveStatsGraphs; j += kBlock) {
        if (lc[j]) atomic_add_i64(&gstat[(int64_t)(g0 + j) * GS_COUNT + GS_CAND], (int64_t)lc[j]);
        if (la[j]) atomic_add_i64(&gstat[(int64_t)(g0 + j) * GS_COUNT + GS_ACC], (int64_t)la[j]);
    }
}

hipError_t launch_batch_move_stats(int64_t n, int64_t span, const Blocks &bk, const int64_t *goff,
                                   const int32_t *part, const int64_t *key,
                                   const uint8_t *accflag, int64_t *gstat, hipStream_t s)
{
    if (n <= 0) return hipSuccess;
    if (span < 1) span = stats_span(n, 0);
    hipLaunchKernelGGL(k_batch_move_stats, dim3((unsigned)((n + span - 1) / span)), dim3(kBlock),
                       0, s, n, span, bk, goff, part, key, accflag, gstat);
    return hipGetLastError();
}

// Per-graph round statistics (UPR_STATS_LEN = 12 per graph, same slots as a
// single graph's). host3[g] = {rebalancing sub-iterations, status, moves}.
__global__ void k_batch_stats_final(int32_t ng, const int64_t *gstat, const int64_t *lmax,
                                    const int64_t *host3, int moved, int64_t *stats)
{
    const int g = blockIdx.x * blockDim.x + threadIdx.x;
    if (g >= ng) return;
    const int64_t *gs = gstat + (int64_t)g * GS_COUNT;
    int64_t *st = stats + (int64_t)g * 12;
    st[0] = lmax[g];
    st[1] = gs[GS_CUT2_BEFORE] / 2;
    st[2] = (moved ? gs[GS_CUT2_MOVES] : gs[GS_CUT2_BEFORE]) / 2;
    st[3] = gs[GS_CUT2_AFTER] / 2;
    st[4] = gs[GS_CAND];
    st[5] = gs[GS_ACC];
    st[6] = host3[3 * g + 2];
    st[7] = host3[3 * g];
    st[8] = host3[3 * g + 1];
    for (int i = 9; i < 12; ++i) st[i] = 0;
}

hipError_t launch_batch_stats_final(int32_t ng, const int64_t *gstat, const int64_t *lmax,
                                    const int64_t *host3, int moved, int64_t *stats, hipStream_t s)
{
    if (ng <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_batch_stats_final, dim3((ng + kBlock - 1) / kBlock), dim3(kBlock), 0, s,
                       ng, gstat, lmax, host3, moved, stats);
    return hipGetLastError();
}

// ------------------------------------------------------------ driver --

// Active set of the label-propagation rounds (Section 6): the boundary nodes
// (a neighbour in another block), one wave per node over its row.
__global__ __launch_bounds__(kBlock) void k_boundary(GraphView g, const int32_t *part,
                                                      uint8_t *active)
{
    const int lane = lane_id();
    const int64_t waves = (int64_t)gridDim.x * (kBlock / 64);
    for (int64_t v = (int64_t)blockIdx.x * (kBlock / 64) + (threadIdx.x >> 6); v < g.n; v += waves) {
        const int32_t a = part[v];
        bool diff = false;
        for (int64_t e = g.xadj[v] + lane; e < g.xadj[v + 1] && !diff; e += 64)
            diff = part[g.adjncy[e]] != a;
        const bool any = __ballot(diff) != 0;
        if (lane == 0) active[v] = any ? 1 : 0;
    }
}

// Next active set: nodes that did not move and have a neighbour that moved
// (before / after: the partition at the start and at the end of the round).
__global__ __launch_bounds__(kBlock) void k_next_active(GraphView g, const int32_t *before,
                                                         const int32_t *after, uint8_t *active)
{
    const int lane = lane_id();
    const int64_t waves = (int64_t)gridDim.x * (kBlock / 64);
    for (int64_t v = (int64_t)blockIdx.x * (kBlock / 64) + (threadIdx.x >> 6); v < g.n; v += waves) {
        const bool moved = before[v] != after[v];
        bool nb = false;
        if (!moved)
            for (int64_t e = g.xadj[v] + lane; e < g.xadj[v + 1] && !nb; e += 64) {
                const int64_t u = g.adjncy[e];
                nb = before[u] != after[u];
            }
        const bool any = __ballot(nb) != 0;
        if (lane == 0) active[v] = any ? 1 : 0;
    }
}

// out[0] = number of nonzero bytes of a[0, n) (one workgroup).
__global__ void k_count_u8(const uint8_t *a, int64_t n, int64_t *out)
{
    __shared__ int64_t red[4];
    int64_t c = 0;
    for (int64_t i = threadIdx.x; i < n; i += kBlock) c += a[i] != 0;
    c = block_sum(c, red);
    if (threadIdx.x == 0) out[0] = c;
}

hipError_t launch_count_u8(const uint8_t *a, int64_t n, int64_t *out, hipStream_t s)
{
    hipLaunchKernelGGL(k_count_u8, dim3(1), dim3(kBlock), 0, s, a, n, out);
    return hipGetLastError();
}

hipError_t launch_boundary(const GraphView &g, const int32_t *part, uint8_t *active, hipStream_t s)
{
    if (g.n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_boundary, dim3(grid_for(g.n, kBlock / 64, 16384)), dim3(kBlock), 0, s, g,
                       part, active);
    return hipGetLastError();
}

hipError_t launch_next_active(const GraphView &g, const int32_t *before, const int32_t *after,
                              uint8_t *active, hipStream_t s)
{
    if (g.n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_next_active, dim3(grid_for(g.n, kBlock / 64, 16384)), dim3(kBlock), 0, s,
                       g, before, after, active);
    return hipGetLastError();
}

}  // namespace upr
