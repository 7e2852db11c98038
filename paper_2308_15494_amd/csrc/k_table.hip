// Gain table, block weights, cut and per-graph preparation kernels.
//
// Gain table (Section 7.1, the shared-memory FM's table): conn[v][j] is the
// edge weight from v into block j. It is built tile by tile: a workgroup owns
// T consecutive nodes, zeroes their T x k rows in LDS, walks the tile's
// adjacency edge-parallel (coalesced adjncy/adjwgt reads, one gather of
// part[u] per edge, an LDS atomic per edge) and writes the rows back as one
// contiguous, coalesced span of conn. Hubs (degree above the plan's hub
// threshold) are left out of the tiles and accumulated by several
// workgroups, each over a chunk of the hub's edges, into the row in global
// memory.
#include "upr_common.h"

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

// ------------------------------------------------------------- gain tile --

constexpr int kTileInts = 8192;  // LDS ints of one tile's rows (32 KiB)
constexpr int kTileMaxNodes = 1024;

int gain_tile_nodes(int32_t k)
{
    int t = kTileInts / k;
    if (t > kTileMaxNodes) t = kTileMaxNodes;
    if (t < 1) t = 1;
    return t;
}

static size_t gain_tile_lds(int32_t k, int T, bool p16)
{
    size_t rows = (size_t)T * k * (p16 ? 2 : 4);
    if (rows < 4) rows = 4;
    return rows + (size_t)(T + 1) * 4 + (size_t)T * 8 + 64;
}

// One workgroup per tile of T consecutive nodes: zero the T x k rows in
// LDS, accumulate every non-hub edge of the tile (edge-parallel; the edge ->
// node map is a binary search over the tile's degree prefix), write the rows
// back as one contiguous span. Hub rows are written as zeros here and filled
// by k_gain_hub.
//
// P16: when every tiled row sum fits 16 bits (non-hub weighted degrees below
// 2^16), two counters share an LDS word (entry i in the low half of word
// i / 2 if i is even, the high half otherwise). A sum never carries into the
// neighbouring half, the tile takes half the LDS and twice as many
// workgroups stay resident per CU to hide the gathers' latency.
template <bool WEIGHTED, bool P16>
__device__ __forceinline__ void gain_tile_body(const GraphView &g, int32_t k, int T,
                                               const PartView &part,
                                               int32_t *__restrict__ conn, int64_t hub_t)
{
    extern __shared__ __align__(16) unsigned char lds_raw[];
    int32_t *tile = (int32_t *)lds_raw;
    const size_t rows_bytes = ((size_t)T * k * (P16 ? 2 : 4) + 15) & ~(size_t)15;
    int32_t *vstart = (int32_t *)(lds_raw + rows_bytes);
    int64_t *gstart = (int64_t *)(lds_raw + rows_bytes + (((size_t)(T + 1) * 4 + 15) & ~(size_t)15));
    __shared__ int32_t scan_lds[4];

    const int64_t v0 = (int64_t)blockIdx.x * T;
    const int nt = (int)((g.n - v0) < T ? (g.n - v0) : T);
    const int tid = threadIdx.x;
    const int64_t kk = k;
    const int entries = nt * k;

    {
        int4 *t4 = (int4 *)tile;
        const int words = P16 ? (entries + 1) >> 1 : entries;
        const int n4 = words >> 2;
        for (int i = tid; i < n4; i += kBlock) t4[i] = make_int4(0, 0, 0, 0);
        for (int i = (n4 << 2) + tid; i < words; i += kBlock) tile[i] = 0;
    }

    // virtual degrees (hubs contribute none) and their exclusive prefix,
    // in chunks of kBlock nodes
    int32_t run = 0;
    for (int base = 0; base < nt; base += kBlock) {
        const int i = base + tid;
        int32_t vd = 0;
        if (i < nt) {
            const int64_t a = g.xadj[v0 + i], b = g.xadj[v0 + i + 1];
            gstart[i] = a;
            vd = (b - a) > hub_t ? 0 : (int32_t)(b - a);
        }
        int32_t total;
        const int32_t inc = block_incl_scan(vd, scan_lds, &total);
        if (i < nt) vstart[i] = run + inc - vd;
        run += total;
    }
    if (tid == 0) vstart[nt] = run;
    __syncthreads();

    // kUnroll independent edges per thread and step, so that their loads
    // (adjncy, then the part gathers) are in flight together
    constexpr int kUnroll = 4;
    const int32_t E = run;
    for (int32_t p0 = tid; p0 < E; p0 += kBlock * kUnroll) {
        int node[kUnroll];
        int64_t e[kUnroll];
        int32_t u[kUnroll], w[kUnroll], pu[kUnroll];
#pragma unroll
        for (int i = 0; i < kUnroll; ++i) {
            const int32_t p = p0 + i * kBlock;
            node[i] = p < E ? upper_index(vstart, nt, p) : -1;
            e[i] = node[i] >= 0 ? gstart[node[i]] + (p - vstart[node[i]]) : 0;
        }
#pragma unroll
        for (int i = 0; i < kUnroll; ++i) {
            u[i] = node[i] >= 0 ? g.adjncy[e[i]] : 0;
            w[i] = (WEIGHTED && node[i] >= 0) ? g.adjwgt[e[i]] : 1;
        }
#pragma unroll
        for (int i = 0; i < kUnroll; ++i) pu[i] = node[i] >= 0 ? pget(part, u[i]) : -1;
#pragma unroll
        for (int i = 0; i < kUnroll; ++i)
            if ((unsigned)pu[i] < (unsigned)k) {
                const int idx = node[i] * k + pu[i];
                if (P16) atomicAdd(&tile[idx >> 1], w[i] << ((idx & 1) << 4));
                else atomicAdd(&tile[idx], w[i]);
            }
    }
    __syncthreads();

    // coalesced write-back of the contiguous rows [v0, v0 + nt)
    int32_t *dst = conn + v0 * kk;
    const int64_t total_ints = entries;
    int64_t done = 0;
    if (((uintptr_t)dst & 15) == 0) {
        const int64_t n4 = total_ints >> 2;
        int4 *d4 = (int4 *)dst;
        if (P16) {
            const uint2 *s2 = (const uint2 *)tile;
            for (int64_t i = tid; i < n4; i += kBlock) {
                const uint2 x = s2[i];
                d4[i] = make_int4((int)(x.x & 0xFFFF), (int)(x.x >> 16), (int)(x.y & 0xFFFF),
                                  (int)(x.y >> 16));
            }
        } else {
            const int4 *s4 = (const int4 *)tile;
            for (int64_t i = tid; i < n4; i += kBlock) d4[i] = s4[i];
        }
        done = n4 << 2;
    }
    if (P16) {
        const uint16_t *t16 = (const uint16_t *)tile;
        for (int64_t i = done + tid; i < total_ints; i += kBlock) dst[i] = t16[i];
    } else {
        for (int64_t i = done + tid; i < total_ints; i += kBlock) dst[i] = tile[i];
    }
}
template <bool WEIGHTED, bool P16>
__global__ __launch_bounds__(kBlock) void k_gain_tile(GraphView g, int32_t k, int T, PartView part,
                                                       int32_t *__restrict__ conn, int64_t hub_t)
{
    gain_tile_body<WEIGHTED, P16>(g, k, T, part, conn, hub_t);
}
template <bool WEIGHTED, bool P16>
__global__ __launch_bounds__(kBlock) void k_gain_refresh(GraphView g, int32_t k, int T,
                                                          PartView part,
                                                          int32_t *__restrict__ conn,
                                                          int64_t hub_t, uint8_t *dirty)
{
    if (!dirty[blockIdx.x]) return;
    __syncthreads();
    if (threadIdx.x == 0) dirty[blockIdx.x] = 0;
    gain_tile_body<WEIGHTED, P16>(g, k, T, part, conn, hub_t);
}

hipError_t launch_gain_tile(const GraphView &g, int32_t k, const PartView &part, int32_t *conn,
                            int64_t hub_t, uint8_t *dirty, hipStream_t s)
{
    if (g.n <= 0) return hipSuccess;
    const int T = gain_tile_nodes(k);
    const int64_t tiles = (g.n + T - 1) / T;
    const size_t lds = gain_tile_lds(k, T, g.tile16 != 0);
#define UPR_TILE(KERN, WW, PP, ...)                                                                 \
    hipLaunchKernelGGL((KERN<WW, PP>), dim3((unsigned)tiles), dim3(kBlock), lds, s, g, k, T, part, \
                       conn, hub_t __VA_ARGS__)
#define UPR_TILE_ALL(KERN, ...)                                                                     \
    do {                                                                                            \
        if (g.adjwgt) {                                                                             \
            if (g.tile16) UPR_TILE(KERN, true, true, __VA_ARGS__);                                  \
            else UPR_TILE(KERN, true, false, __VA_ARGS__);                                          \
        } else {                                                                                    \
            if (g.tile16) UPR_TILE(KERN, false, true, __VA_ARGS__);                                 \
            else UPR_TILE(KERN, false, false, __VA_ARGS__);                                         \
        }                                                                                           \
    } while (0)
    if (dirty) UPR_TILE_ALL(k_gain_refresh, , dirty);
    else UPR_TILE_ALL(k_gain_tile, );
#undef UPR_TILE_ALL
#undef UPR_TILE
    return hipGetLastError();
}

// --------------------------------------------------------------- hub rows --

// One workgroup per chunk of a hub's edges: accumulate into an LDS row, then
// add the non-zero entries into the hub's row of conn (zeroed by the tile).
__global__ __launch_bounds__(kBlock) void k_gain_hub(GraphView g, int32_t k, PartView part,
                                                      int32_t *conn, HubView h)
{
    extern __shared__ __align__(16) unsigned char lds_raw[];
    int32_t *row = (int32_t *)lds_raw;
    const HubChunk c = h.chunks[blockIdx.x];
    const int64_t v = h.ids[c.hub];
    for (int j = threadIdx.x; j < k; j += kBlock) row[j] = 0;
    __syncthreads();
    for (int64_t e = c.e0 + threadIdx.x; e < c.e1; e += kBlock) {
        const int32_t pu = pget(part, g.adjncy[e]);
        if ((unsigned)pu < (unsigned)k) atomicAdd(&row[pu], edge_weight(g, e));
    }
    __syncthreads();
    int32_t *dst = conn + v * (int64_t)k;
    for (int j = threadIdx.x; j < k; j += kBlock)
        if (row[j]) atomicAdd(&dst[j], row[j]);
}

__global__ void k_zero_hub_rows(int32_t k, int32_t *conn, HubView h)
{
    int32_t *row = conn + (int64_t)h.ids[blockIdx.x] * k;
    for (int j = threadIdx.x; j < k; j += kBlock) row[j] = 0;
}

__global__ void k_hub_bits(HubView h, uint32_t *bits)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= h.nh) return;
    const int32_t v = h.ids[i];
    atomicOr(&bits[v >> 5], 1u << (v & 31));
}

hipError_t launch_hub_bits(const HubView &h, uint32_t *bits, hipStream_t s)
{
    if (h.nh <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_hub_bits, dim3((h.nh + kBlock - 1) / kBlock), dim3(kBlock), 0, s, h, bits);
    return hipGetLastError();
}

hipError_t launch_rebuild_hub_rows(const GraphView &g, int32_t k, const PartView &part,
                                   int32_t *conn, const HubView &h, hipStream_t s)
{
    if (h.nh <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_zero_hub_rows, dim3(h.nh), dim3(kBlock), 0, s, k, conn, h);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    return launch_gain_hub(g, k, part, conn, h, s);
}

hipError_t launch_gain_hub(const GraphView &g, int32_t k, const PartView &part, int32_t *conn,
                           const HubView &h, hipStream_t s)
{
    if (h.nchunks <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_gain_hub, dim3((unsigned)h.nchunks), dim3(kBlock), (size_t)k * 4, s, g, k,
                       part, conn, h);
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
// t_num * omega(I(v)); slot(omega(v, Pi(v)), c(v))). Block weights and
// buckets are accumulated in LDS when they fit, else by wave-aggregated
// global atomics.
constexpr int kStatsLdsBytes = 32768;

__global__ __launch_bounds__(kBlock) void k_node_stats(GraphView g, Blocks bk,
                                                        const int32_t *__restrict__ part,
                                                        const int32_t *__restrict__ conn,
                                                        const int32_t *__restrict__ wdeg,
                                                        int64_t *W, int64_t *bucket,
                                                        int32_t t_num, int32_t t_den,
                                                        unsigned long long *counters, int cut_slot,
                                                        uint8_t *avail_out, int64_t *gstat,
                                                        int gs_slot)
{
    extern __shared__ __align__(16) unsigned char lds_raw[];
    __shared__ unsigned long long red[4];
    __shared__ unsigned long long bad;
    const int32_t K = bk.total();
    const int32_t k = bk.k;
    const bool w_lds = W && (size_t)K * 8 <= 16384;
    const bool b_lds = bucket && (size_t)K * kSlots * 8 <= kStatsLdsBytes;
    int64_t *lw = (int64_t *)lds_raw;
    int64_t *lb = (int64_t *)(lds_raw + (w_lds ? (size_t)K * 8 : 0));
    if (threadIdx.x == 0) bad = 0;
    if (w_lds)
        for (int j = threadIdx.x; j < K; j += kBlock) lw[j] = 0;
    if (b_lds)
        for (int j = threadIdx.x; j < K * kSlots; j += kBlock) lb[j] = 0;
    __syncthreads();

    unsigned long long s = 0;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    const int64_t nn = g.n;
    // loop bound uniform per wave (wave_hist_add needs whole waves)
    for (int64_t vb = (int64_t)blockIdx.x * blockDim.x + (threadIdx.x & ~63); vb < nn; vb += stride) {
        const int64_t v = vb + lane_id();
        bool ok = v < nn;
        int32_t a = 0;
        int64_t cv = 1, inner = 0, wd = 0;
        if (ok) {
            a = part[v];
            if ((unsigned)a >= (unsigned)K) {
                atomicAdd(&bad, 1ull);
                ok = false;
            } else {
                inner = conn[v * (int64_t)k + bk.local(a)];
                wd = wdeg[v];
                cv = node_weight(g, v);
                s += (unsigned long long)(wd - inner);
            }
        }
        if (gstat) wave_hist_add(gstat, (int64_t)bk.graph(a) * GS_COUNT + gs_slot, wd - inner, ok);
        if (W) {
            if (w_lds) {
                if (ok) atomicAdd((unsigned long long *)&lw[a], (unsigned long long)cv);
            } else {
                wave_hist_add(W, a, cv, ok);
            }
        }
        if (bucket) {
            const bool avail = ok && (int64_t)t_den * inner >= (int64_t)t_num * wd;
            if (avail_out && v < nn) avail_out[v] = avail ? 1 : 0;
            const int64_t key = (int64_t)a * kSlots + (avail ? slot_of(inner, cv) : 0);
            if (b_lds) {
                if (avail) atomicAdd((unsigned long long *)&lb[key], (unsigned long long)cv);
            } else {
                wave_hist_add(bucket, key, cv, avail);
            }
        }
    }
    s = block_sum(s, red);
    if (threadIdx.x == 0) {
        if (s) cnt_add(counters, cut_slot, s);
        if (bad) cnt_add(counters, CNT_BAD_INPUT, bad);
    }
    if (w_lds)
        for (int j = threadIdx.x; j < K; j += kBlock)
            if (lw[j]) atomic_add_i64(&W[j], lw[j]);
    if (b_lds)
        for (int j = threadIdx.x; j < K * kSlots; j += kBlock)
            if (lb[j]) atomic_add_i64(&bucket[j], lb[j]);
}

hipError_t launch_node_stats(const GraphView &g, const Blocks &bk, const int32_t *part,
                             const int32_t *conn, const int32_t *wdeg, int64_t *W,
                             int64_t *bucket, int32_t t_num, int32_t t_den,
                             unsigned long long *counters, int cut_slot, uint8_t *avail,
                             int64_t *gstat, int gs_slot, hipStream_t s)
{
    if (g.n <= 0) return hipSuccess;
    const int32_t K = bk.total();
    size_t lds = 0;
    if (W && (size_t)K * 8 <= 16384) lds += (size_t)K * 8;
    if (bucket && (size_t)K * kSlots * 8 <= kStatsLdsBytes) lds += (size_t)K * kSlots * 8;
    hipLaunchKernelGGL(k_node_stats, dim3(grid_for(g.n, kBlock * 8, 2048)), dim3(kBlock), lds, s,
                       g, bk, part, conn, wdeg, W, bucket, t_num, t_den, counters, cut_slot, avail,
                       gstat, gs_slot);
    return hipGetLastError();
}

__global__ void k_store_half(const unsigned long long *counters, int slot, int64_t *out)
{
    if (threadIdx.x == 0 && blockIdx.x == 0) out[0] = (int64_t)(cnt_get(counters, slot) / 2);
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

// Graph of node v in a batch: the g with goff[g] <= v < goff[g + 1].
__device__ __forceinline__ int32_t graph_of_node(const int64_t *goff, int32_t ng, int64_t v)
{
    int lo = 0, hi = ng - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (goff[mid] <= v) lo = mid;
        else hi = mid - 1;
    }
    return lo;
}

__global__ void k_pack_part(int64_t n, Blocks bk, const int64_t *goff, const int32_t *part,
                            void *pc, int bytes, unsigned long long *counters)
{
    const int32_t K = bk.total();
    bool bad = false;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; v < n; v += stride) {
        const int32_t B = part[v];
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
                            void *pc, int bytes, unsigned long long *counters, hipStream_t s)
{
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_pack_part, dim3(grid_for(n, kBlock * 4, 4096)), dim3(kBlock), 0, s, n, bk,
                       goff, part, pc, bytes, counters);
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

}  // namespace upr
