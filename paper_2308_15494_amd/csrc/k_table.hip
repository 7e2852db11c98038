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
    return rows + (size_t)(T + 1) * 4 + (size_t)T * 8 + (size_t)T * 2 + 64;
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
// PB: bytes per entry of the partition view (1, 2 or 4).
// inner (may be null): each non-hub node's own entry conn[v][own block] is
// also written to inner[v] (own: the partition in node order), so that the
// statistics pass need not gather it from the row.
template <bool WEIGHTED, bool P16, int PB>
__device__ __forceinline__ void gain_tile_body(const GraphView &g, int32_t k, int T,
                                               const PartView &part,
                                               int32_t *__restrict__ conn, int64_t hub_t,
                                               int32_t *__restrict__ inner, const PartView &own)
{
    extern __shared__ __align__(16) unsigned char lds_raw[];
    int32_t *tile = (int32_t *)lds_raw;
    const size_t rows_bytes = ((size_t)T * k * (P16 ? 2 : 4) + 15) & ~(size_t)15;
    int32_t *vstart = (int32_t *)(lds_raw + rows_bytes);
    int64_t *gstart = (int64_t *)(lds_raw + rows_bytes + (((size_t)(T + 1) * 4 + 15) & ~(size_t)15));
    int16_t *sown = (int16_t *)(gstart + T);  // own block of each node (with inner)
    __shared__ int32_t scan_lds[4];

    const int64_t v0 = (int64_t)blockIdx.x * T;
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
    // in chunks of kBlock nodes; with inner, each node's own block goes to
    // LDS and a hub is marked by gstart = -1 (its edges are never visited)
    int32_t run = 0;
    for (int base = 0; base < nt; base += kBlock) {
        const int i = base + tid;
        int32_t vd = 0;
        if (i < nt) {
            const int64_t a = g.xadj[v0 + i], b = g.xadj[v0 + i + 1];
            const bool hub = (b - a) > hub_t;
            gstart[i] = hub && inner ? -1 : a;
            vd = hub ? 0 : (int32_t)(b - a);
            if (inner) sown[i] = (int16_t)(pget(own, v0 + i) & part_mask(own));
        }
        int32_t total;
        const int32_t inc = block_incl_scan(vd, scan_lds, &total);
        if (i < nt) vstart[i] = run + inc - vd;
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
    if (inner) {
        for (int i = tid; i < nt; i += kBlock) {
            const int32_t j = sown[i];
            if (gstart[i] < 0 || (unsigned)j >= (unsigned)k) continue;  // a hub: its row comes later
            const int idx = i * k + j;
            inner[v0 + i] = P16 ? (int32_t)((const uint16_t *)tile)[idx] : tile[idx];
        }
    }
}
template <bool WEIGHTED, bool P16, int PB>
__global__ __launch_bounds__(kBlock) void k_gain_tile(GraphView g, int32_t k, int T, PartView part,
                                                       int32_t *__restrict__ conn, int64_t hub_t,
                                                       int32_t *__restrict__ inner, PartView own)
{
    gain_tile_body<WEIGHTED, P16, PB>(g, k, T, part, conn, hub_t, inner, own);
}
template <bool WEIGHTED, bool P16, int PB>
// Rebuilds the marked tiles, or every tile when the moving nodes' degrees
// (counters[CNT_MOVED_DEG]) sum above all_threshold (the apply then marks
// nothing: nearly every tile would be marked).
__global__ __launch_bounds__(kBlock) void k_gain_refresh(GraphView g, int32_t k, int T,
                                                          PartView part,
                                                          int32_t *__restrict__ conn,
                                                          int64_t hub_t, uint8_t *dirty,
                                                          const unsigned long long *counters,
                                                          int64_t all_threshold)
{
    const bool all = counters && (int64_t)wave_cnt_get(counters, CNT_MOVED_DEG) > all_threshold;
    if (!all && !dirty[blockIdx.x]) return;  // uniform over the workgroup
    __syncthreads();
    if (threadIdx.x == 0) dirty[blockIdx.x] = 0;
    gain_tile_body<WEIGHTED, P16, PB>(g, k, T, part, conn, hub_t, nullptr, part);
}

hipError_t launch_gain_tile(const GraphView &g, int32_t k, const PartView &part, int32_t *conn,
                            int64_t hub_t, uint8_t *dirty, hipStream_t s, int32_t *inner,
                            const PartView &own, const unsigned long long *counters,
                            int64_t all_threshold)
{
    if (g.n <= 0) return hipSuccess;
    const int T = gain_tile_nodes(k);
    const int64_t tiles = (g.n + T - 1) / T;
    const size_t lds = gain_tile_lds(k, T, g.tile16 != 0);
#define UPR_TILE(KERN, WW, PP, BB, ...)                                                             \
    hipLaunchKernelGGL((KERN<WW, PP, BB>), dim3((unsigned)tiles), dim3(kBlock), lds, s, g, k, T,    \
                       part, conn, hub_t __VA_ARGS__)
#define UPR_TILE_B(KERN, WW, PP, ...)                                                               \
    do {                                                                                            \
        if (part.bytes == 1) UPR_TILE(KERN, WW, PP, 1, __VA_ARGS__);                                \
        else if (part.bytes == 2) UPR_TILE(KERN, WW, PP, 2, __VA_ARGS__);                           \
        else UPR_TILE(KERN, WW, PP, 4, __VA_ARGS__);                                                \
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
    if (dirty) UPR_TILE_ALL(k_gain_refresh, , dirty, counters, all_threshold);
    else UPR_TILE_ALL(k_gain_tile, , inner, own);
#undef UPR_TILE_ALL
#undef UPR_TILE_B
#undef UPR_TILE
    return hipGetLastError();
}

// --------------------------------------------------------------- hub rows --

// One workgroup per chunk of a hub's edges: accumulate into an LDS row, then
// add the non-zero entries into the hub's row of conn (zeroed by the tile,
// or by the hub apply). counters != null: only if the apply before rebuilt
// the table.
__global__ __launch_bounds__(kBlock) void k_gain_hub(GraphView g, int32_t k, PartView part,
                                                      int32_t *conn, HubView h,
                                                      const unsigned long long *counters,
                                                      int64_t dirty_threshold)
{
    extern __shared__ __align__(16) unsigned char lds_raw[];
    int32_t *row = (int32_t *)lds_raw;
    if (counters && (int64_t)wave_cnt_get(counters, CNT_MOVED_DEG) <= dirty_threshold) return;
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

hipError_t launch_gain_hub(const GraphView &g, int32_t k, const PartView &part, int32_t *conn,
                           const HubView &h, hipStream_t s, const unsigned long long *counters,
                           int64_t dirty_threshold)
{
    if (h.nchunks <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_gain_hub, dim3((unsigned)h.nchunks), dim3(kBlock), (size_t)k * 4, s, g, k,
                       part, conn, h, counters, dirty_threshold);
    return hipGetLastError();
}

}  // namespace upr
