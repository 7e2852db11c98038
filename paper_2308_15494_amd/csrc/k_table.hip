// Gain table kernels.
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

// ------------------------------------------------------------- gain tile --

constexpr int kTileInts = 8192;  // LDS ints of one tile's rows (32 KiB)
constexpr int kTileMaxNodes = 1024;

// Nodes per tile: as many rows as kTileInts LDS ints hold (at most
// kTileMaxNodes), halved (down to kTileMinNodes) while the graph would get
// fewer than kTileMinTiles tiles, so that a small graph still spreads over
// the CUs.
constexpr int kTileMinNodes = 16;
constexpr int64_t kTileMinTiles = 2048;

int gain_tile_nodes(int32_t k, int64_t n)
{
    int t = kTileInts / k;
    if (t > kTileMaxNodes) t = kTileMaxNodes;
    if (t < 1) t = 1;
    while (t > kTileMinNodes && (n + t - 1) / t < kTileMinTiles) t /= 2;
    return t;
}

static size_t gain_tile_lds(int32_t k, int T, bool p16)
{
    size_t rows = (size_t)T * k * (p16 ? 2 : 4);
    if (rows < 4) rows = 4;
    return rows + (size_t)(T + 1) * 4 + (size_t)T * 8 + (size_t)T * 2 + 64;
}

// One workgroup per tile of T consecutive nodes: zero the T x k rows in
// LDS, accumulate every non-hub edge of the tile (edge-parallel; the edge ->
// node map is a binary search over the tile's degree prefix), write the rows
// back as one contiguous span. Hub rows are left alone: their chunks, in the
// same launch, write them.
//
// P16: when every tiled row sum fits 16 bits (non-hub weighted degrees below
// 2^16), two counters share an LDS word (entry i in the low half of word
// i / 2 if i is even, the high half otherwise). A sum never carries into the
// neighbouring half, the tile takes half the LDS and twice as many
// workgroups stay resident per CU to hide the gathers' latency.
// PB: bytes per entry of the partition view (1, 2 or 4).
// inner (may be null): each non-hub node's own entry conn[v][own block] is
// also written to inner[v] (own: the partition in node order), so that the
// statistics pass need not gather it from the row.
template <bool WEIGHTED, bool P16, int PB>
__device__ __forceinline__ void gain_tile_body(const GraphView &g, int32_t k, int T,
                                               const PartView &part,
                                               int32_t *__restrict__ conn, int64_t hub_t,
                                               int32_t *__restrict__ inner, const PartView &own,
                                               int64_t tile_id)
{
    extern __shared__ __align__(16) unsigned char lds_raw[];
    int32_t *tile = (int32_t *)lds_raw;
    const size_t rows_bytes = ((size_t)T * k * (P16 ? 2 : 4) + 15) & ~(size_t)15;
    int32_t *vstart = (int32_t *)(lds_raw + rows_bytes);
    int64_t *gstart = (int64_t *)(lds_raw + rows_bytes + (((size_t)(T + 1) * 4 + 15) & ~(size_t)15));
    int16_t *sown = (int16_t *)(gstart + T);  // own block of each node (with inner)
    __shared__ int32_t scan_lds[4];
    __shared__ int32_t any_hub;

    const int64_t v0 = tile_id * T;
    const int nt = (int)((g.n - v0) < T ? (g.n - v0) : T);
    const int tid = threadIdx.x;
    const int64_t kk = k;
    const int entries = nt * k;
    const int32_t pmask = part_mask(part);

    {
        int4 *t4 = (int4 *)tile;
        const int words = P16 ? (entries + 1) >> 1 : entries;
        const int n4 = words >> 2;
        for (int i = tid; i < n4; i += kBlock) t4[i] = make_int4(0, 0, 0, 0);
        for (int i = (n4 << 2) + tid; i < words; i += kBlock) tile[i] = 0;
    }

    // virtual degrees (hubs contribute none) and their exclusive prefix,
    // in chunks of kBlock nodes; a hub is marked by gstart = -1 (its edges
    // are never visited) and with inner, each node's own block goes to LDS
    if (tid == 0) any_hub = 0;  // ordered before the flag writes by the scan's barriers
    int32_t run = 0;
    for (int base = 0; base < nt; base += kBlock) {
        const int i = base + tid;
        int32_t vd = 0;
        if (i < nt) {
            const int64_t a = g.xadj[v0 + i], b = g.xadj[v0 + i + 1];
            const bool hub = (b - a) > hub_t;
            gstart[i] = hub ? -1 : a;
            vd = hub ? 0 : (int32_t)(b - a);
            if (inner) sown[i] = (int16_t)(pget(own, v0 + i) & part_mask(own));
        }
        int32_t total;
        const int32_t inc = block_incl_scan(vd, scan_lds, &total);
        if (i < nt) {
            vstart[i] = run + inc - vd;
            if (gstart[i] < 0) any_hub = 1;
        }
        run += total;
    }
    if (tid == 0) vstart[nt] = run;
    __syncthreads();

    // kUnroll independent edges per thread and step. Every load is issued
    // unconditionally (a slot past the tile's last edge reads that last edge
    // again and adds nothing), so the adjacency loads and then the part
    // gathers of all slots are in flight together.
    constexpr int kUnroll = 8;
    const int32_t E = run;
    for (int32_t p0 = tid; p0 < E; p0 += kBlock * kUnroll) {
        bool ok[kUnroll];
        int node[kUnroll];
        int64_t e[kUnroll];
        int32_t u[kUnroll], w[kUnroll], pu[kUnroll];
#pragma unroll
        for (int i = 0; i < kUnroll; ++i) {
            const int32_t p = p0 + i * kBlock;
            ok[i] = p < E;
            const int32_t pc = ok[i] ? p : E - 1;
            node[i] = upper_index(vstart, nt, pc);
            e[i] = gstart[node[i]] + (pc - vstart[node[i]]);
        }
#pragma unroll
        for (int i = 0; i < kUnroll; ++i) {
            u[i] = g.adjncy[e[i]];
            w[i] = WEIGHTED ? g.adjwgt[e[i]] : 1;
        }
#pragma unroll
        for (int i = 0; i < kUnroll; ++i) pu[i] = pget_w<PB>(part.p, u[i], pmask);
#pragma unroll
        for (int i = 0; i < kUnroll; ++i)
            if (ok[i] && (unsigned)pu[i] < (unsigned)k) {
                const int idx = node[i] * k + pu[i];
                if (P16) atomicAdd(&tile[idx >> 1], w[i] << ((idx & 1) << 4));
                else atomicAdd(&tile[idx], w[i]);
            }
    }
    __syncthreads();

    // coalesced write-back of the contiguous rows [v0, v0 + nt); a tile
    // that holds a hub skips the hub's row. The stores are non-temporal: the
    // table streams through the L2 without evicting the partition copy that
    // the other tiles gather from.
    int32_t *dst = conn + v0 * kk;
    const int64_t total_ints = entries;
    int64_t done = 0;
    if (any_hub) {
        for (int i = tid; i < entries; i += kBlock)
            if (gstart[i / k] >= 0) dst[i] = P16 ? (int32_t)((const uint16_t *)tile)[i] : tile[i];
        done = total_ints;
    } else if (((uintptr_t)dst & 15) == 0) {
        const int64_t n4 = total_ints >> 2;
        int4 *d4 = (int4 *)dst;
        if (P16) {
            const uint2 *s2 = (const uint2 *)tile;
            for (int64_t i = tid; i < n4; i += kBlock) {
                const uint2 x = s2[i];
                v4i32 y;
                y.x = (int)(x.x & 0xFFFF);
                y.y = (int)(x.x >> 16);
                y.z = (int)(x.y & 0xFFFF);
                y.w = (int)(x.y >> 16);
                __builtin_nontemporal_store(y, (v4i32 *)d4 + i);
            }
        } else {
            const v4i32 *s4 = (const v4i32 *)tile;
            for (int64_t i = tid; i < n4; i += kBlock) __builtin_nontemporal_store(s4[i], (v4i32 *)d4 + i);
        }
        done = n4 << 2;
    }
    if (P16) {
        const uint16_t *t16 = (const uint16_t *)tile;
        for (int64_t i = done + tid; i < total_ints; i += kBlock) dst[i] = t16[i];
    } else {
        for (int64_t i = done + tid; i < total_ints; i += kBlock) dst[i] = tile[i];
    }
    if (inner) {
        for (int i = tid; i < nt; i += kBlock) {
            const int32_t j = sown[i];
            if (gstart[i] < 0 || (unsigned)j >= (unsigned)k) continue;  // a hub: its row comes later
            const int idx = i * k + j;
            inner[v0 + i] = P16 ? (int32_t)((const uint16_t *)tile)[idx] : tile[idx];
        }
    }
}
// A chunk of a hub's edges: accumulate the chunk's counts in an LDS row,
// then add its non-zero entries into the hub's row of conn (which is zero
// before the first chunk adds: no chunk waits for another).
template <bool WEIGHTED, int PB>
__device__ __forceinline__ void gain_hub_chunk(const GraphView &g, int32_t k, const PartView &part,
                                               int32_t *__restrict__ conn, const HubView &h,
                                               int64_t ci)
{
    extern __shared__ __align__(16) unsigned char lds_raw[];
    int32_t *row = (int32_t *)lds_raw;
    const int tid = threadIdx.x;
    const HubChunk c = h.chunks[ci];
    const int64_t v = h.ids[c.hub];
    const int32_t pmask = part_mask(part);
    for (int j = tid; j < k; j += kBlock) row[j] = 0;
    __syncthreads();
    // as in the tile: every load issued unconditionally (a slot past the
    // chunk's end reads its last edge again and adds nothing)
    constexpr int kUnroll = 8;
    for (int64_t p0 = c.e0 + tid; p0 < c.e1; p0 += (int64_t)kBlock * kUnroll) {
        bool ok[kUnroll];
        int64_t e[kUnroll];
        int32_t u[kUnroll], w[kUnroll], pu[kUnroll];
#pragma unroll
        for (int i = 0; i < kUnroll; ++i) {
            const int64_t q = p0 + i * kBlock;
            ok[i] = q < c.e1;
            e[i] = ok[i] ? q : c.e1 - 1;
        }
#pragma unroll
        for (int i = 0; i < kUnroll; ++i) {
            u[i] = g.adjncy[e[i]];
            w[i] = WEIGHTED ? g.adjwgt[e[i]] : 1;
        }
#pragma unroll
        for (int i = 0; i < kUnroll; ++i) pu[i] = pget_w<PB>(part.p, u[i], pmask);
#pragma unroll
        for (int i = 0; i < kUnroll; ++i)
            if (ok[i] && (unsigned)pu[i] < (unsigned)k) atomicAdd(&row[pu[i]], w[i]);
    }
    __syncthreads();
    int32_t *dst = conn + v * (int64_t)k;
    for (int j = tid; j < k; j += kBlock)
        if (row[j]) atomicAdd(&dst[j], row[j]);
}

// The hubs' chunks take the first h.nchunks workgroups (they start first:
// a chunk's edges are many more than a tile's), the tiles the rest.
template <bool WEIGHTED, bool P16, int PB>
__global__ __launch_bounds__(kBlock) void k_gain_tile(GraphView g, int32_t k, int T, PartView part,
                                                       int32_t *__restrict__ conn, int64_t hub_t,
                                                       HubView h, int32_t *__restrict__ inner,
                                                       PartView own)
{
    if ((int64_t)blockIdx.x < h.nchunks) {
        gain_hub_chunk<WEIGHTED, PB>(g, k, part, conn, h, blockIdx.x);
        return;
    }
    gain_tile_body<WEIGHTED, P16, PB>(g, k, T, part, conn, hub_t, inner, own,
                                      (int64_t)blockIdx.x - h.nchunks);
}
// Rebuilds the marked tiles, or every tile when the moving nodes' degrees
// (counters[CNT_MOVED_DEG]) sum above all_threshold (the apply then marks
// nothing: nearly every tile would be marked), and the hub rows when they
// sum above dirty_threshold.
template <bool WEIGHTED, bool P16, int PB>
__global__ __launch_bounds__(kBlock) void k_gain_refresh(GraphView g, int32_t k, int T,
                                                          PartView part,
                                                          int32_t *__restrict__ conn,
                                                          int64_t hub_t, HubView h, uint8_t *dirty,
                                                          const unsigned long long *counters,
                                                          int64_t dirty_threshold,
                                                          int64_t all_threshold)
{
    const int64_t moved_deg = (int64_t)wave_cnt_get(counters, CNT_MOVED_DEG);
    if ((int64_t)blockIdx.x < h.nchunks) {
        if (moved_deg > dirty_threshold) gain_hub_chunk<WEIGHTED, PB>(g, k, part, conn, h, blockIdx.x);
        return;
    }
    const int64_t t = (int64_t)blockIdx.x - h.nchunks;
    if (moved_deg <= all_threshold && !dirty[t]) return;  // uniform over the workgroup
    __syncthreads();
    if (threadIdx.x == 0) dirty[t] = 0;
    gain_tile_body<WEIGHTED, P16, PB>(g, k, T, part, conn, hub_t, nullptr, part, t);
}

namespace {
size_t table_lds(int32_t k, int T, bool p16)
{
    return std::max(gain_tile_lds(k, T, p16), (size_t)k * 4);
}
bool hubs_ready(const HubView &h)
{
    return h.nchunks <= 0 || (h.chunks && h.ids);
}
}  // namespace

#define UPR_TILE_B(KERN, WW, PP, ...)                                                               \
    do {                                                                                            \
        if (part.bytes == 1) hipLaunchKernelGGL((KERN<WW, PP, 1>), __VA_ARGS__);                    \
        else if (part.bytes == 2) hipLaunchKernelGGL((KERN<WW, PP, 2>), __VA_ARGS__);               \
        else hipLaunchKernelGGL((KERN<WW, PP, 4>), __VA_ARGS__);                                    \
    } while (0)
#define UPR_TILE_ALL(KERN, ...)                                                                     \
    do {                                                                                            \
        if (g.adjwgt) {                                                                             \
            if (g.tile16) UPR_TILE_B(KERN, true, true, __VA_ARGS__);                                \
            else UPR_TILE_B(KERN, true, false, __VA_ARGS__);                                        \
        } else {                                                                                    \
            if (g.tile16) UPR_TILE_B(KERN, false, true, __VA_ARGS__);                               \
            else UPR_TILE_B(KERN, false, false, __VA_ARGS__);                                       \
        }                                                                                           \
    } while (0)

hipError_t launch_gain_table(const GraphView &g, int32_t k, const PartView &part, int32_t *conn,
                             int64_t hub_t, const HubView &h, hipStream_t s, int32_t *inner,
                             const PartView &own)
{
    if (g.n <= 0) return hipSuccess;
    if (!hubs_ready(h)) return hipErrorInvalidValue;
    const int T = gain_tile_nodes(k, g.n);
    const int64_t grid = (g.n + T - 1) / T + std::max<int64_t>(h.nchunks, 0);
    const size_t lds = table_lds(k, T, g.tile16 != 0);
    UPR_TILE_ALL(k_gain_tile, dim3((unsigned)grid), dim3(kBlock), lds, s, g, k, T, part, conn,
                 hub_t, h, inner, own);
    return hipGetLastError();
}

hipError_t launch_gain_refresh(const GraphView &g, int32_t k, const PartView &part, int32_t *conn,
                               int64_t hub_t, const HubView &h, uint8_t *dirty,
                               const unsigned long long *counters, int64_t dirty_threshold,
                               int64_t all_threshold, hipStream_t s)
{
    if (g.n <= 0) return hipSuccess;
    if (!hubs_ready(h) || !dirty || !counters) return hipErrorInvalidValue;
    const int T = gain_tile_nodes(k, g.n);
    const int64_t grid = (g.n + T - 1) / T + std::max<int64_t>(h.nchunks, 0);
    const size_t lds = table_lds(k, T, g.tile16 != 0);
    UPR_TILE_ALL(k_gain_refresh, dim3((unsigned)grid), dim3(kBlock), lds, s, g, k, T, part, conn,
                 hub_t, h, dirty, counters, dirty_threshold, all_threshold);
    return hipGetLastError();
}
#undef UPR_TILE_ALL
#undef UPR_TILE_B

// --------------------------------------------------------------- hub rows --

__global__ void k_zero_hub_rows(HubView h, int32_t *conn, int32_t k)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= (int64_t)h.nh * k) return;
    conn[(int64_t)h.ids[i / k] * k + i % k] = 0;
}

hipError_t launch_zero_hub_rows(const HubView &h, int32_t *conn, int32_t k, hipStream_t s)
{
    const int64_t total = (int64_t)h.nh * k;
    if (total <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_zero_hub_rows, dim3((unsigned)((total + kBlock - 1) / kBlock)), dim3(kBlock),
                       0, s, h, conn, k);
    return hipGetLastError();
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


}  // namespace upr
