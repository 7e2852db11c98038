// Internal declarations of libupr: constants, device helpers and kernel
// launchers shared by the HIP sources. Not part of the public ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace upr {

constexpr int kSlots = 54;                  // penalty slots 0..53 (1.5^53 > 2^31)
constexpr int kRbBuckets = 2 * kSlots + 1;  // rebalancing priority buckets
constexpr int kBlock = 256;                 // threads per workgroup (4 wave64)
constexpr int64_t kPenCap = int64_t(1) << 62;

// Device counters (unsigned long long slots of ws.counters).
enum Counter {
    CNT_CAND = 0,      // candidates
    CNT_ACC,           // accepted moves
    CNT_CUT2_BEFORE,   // 2 * cut before
    CNT_CUT2_MOVES,    // 2 * cut after the filtered moves
    CNT_CUT2_AFTER,    // 2 * cut after rebalancing
    CNT_REBAL_MOVES,   // moves made by rebalancing
    CNT_MOVED_NOW,     // moves of the current rebalancing sub-iteration
    CNT_OVER,          // number of overloaded blocks
    CNT_BAD_INPUT,     // nonzero: a part value was out of range
    CNT_TMP,           // scratch accumulator for standalone calls
    CNT_MOVED_DEG,     // sum of the degrees of the nodes marked to move
    CNT_ELIG,          // eligible candidates (pessimistic gain > 0), sequence-aware filter
    CNT_OVER0,         // overloaded blocks when rebalancing starts
    CNT_CUT2_DELTA,    // change of 2 * cut by the round's applies so far (two's complement)
    CNT_CUT_STALE,     // nonzero: an apply rebuilt tiles, so CNT_CUT2_DELTA is incomplete
    CNT_COUNT = 32
};

// The counters are kept in kCntCopies copies (CNT_COUNT slots each, 256 bytes
// apart): a workgroup adds to the copy of its blockIdx.x modulo kCntCopies.
// Atomics on one address serialise in the L2 at about 12 ns each, so a
// single copy costs about 100 us for 8192 workgroups; spread over 64 copies
// it costs nothing measurable. Readers sum the copies.
constexpr int kCntCopies = 64;
constexpr int kCntWords = kCntCopies * CNT_COUNT;

struct PenTable {
    int64_t q[kSlots];
};

// The blocks a round works on. One graph: k blocks, block id B = j. A batch:
// the disjoint union of ng graphs with k blocks each, refined together. Node
// v of graph g lies in the global block B = g*k + j, and its gain-table row
// (k wide) is indexed by the local block j. Block weights, penalty buckets
// and rebalancing state are indexed by B. Every graph has its own L_max and
// penalty table; the rounds of different graphs never interact.
struct Blocks {
    int32_t k = 0;
    int32_t ng = 1;
    const int64_t *lmax = nullptr;      // [ng] L_max of each graph
    const int64_t *src_lmax = nullptr;  // [ng] rebalancing: a block is a source iff heavier
    const int64_t *penq = nullptr;      // [ng * kSlots] Q16 penalty table of each graph
    // moves may fill a target up to floor(alpha * L_max) before they are
    // penalised or forbidden (alpha = 1 except in the limited-imbalance mode)
    int32_t alpha_num = 1, alpha_den = 1;
    __host__ __device__ int32_t total() const { return k * ng; }
    __device__ int32_t graph(int32_t B) const { return ng == 1 ? 0 : B / k; }
    __device__ int32_t base(int32_t B) const { return ng == 1 ? 0 : (B / k) * k; }
    __device__ int32_t local(int32_t B) const { return ng == 1 ? B : B % k; }
    __device__ int64_t lmax_of(int32_t B) const { return lmax[graph(B)]; }
    __device__ int64_t src_lmax_of(int32_t B) const { return src_lmax[graph(B)]; }
    __device__ const int64_t *penq_of(int32_t B) const { return penq + (int64_t)graph(B) * kSlots; }
    __device__ int64_t move_lmax_of(int32_t B) const
    {
        const int64_t L = lmax_of(B);
        if (alpha_num == alpha_den) return L;
        return (int64_t)(((unsigned __int128)(uint64_t)L * (uint32_t)alpha_num) / (uint32_t)alpha_den);
    }
};

// Bit flags of upr_params.variant.
constexpr int kVarOptimistic = 1;
constexpr int kVarPlainPriority = 2;

// Per-graph statistics of a batch (int64 [ng][GS_COUNT]).
enum GraphStat {
    GS_CUT2_BEFORE = 0,
    GS_CUT2_MOVES,
    GS_CUT2_AFTER,
    GS_CAND,
    GS_ACC,
    GS_REBAL_MOVES,
    GS_MOVED_NOW,  // moves of the current rebalancing sub-iteration
    GS_OVER,       // overloaded blocks at the start of a sub-iteration
    GS_COUNT
};

struct GraphView {
    int64_t n;
    const int64_t *xadj;
    const int32_t *adjncy;
    const int32_t *adjwgt;  // may be null: unit edge weights
    const int32_t *vwgt;    // may be null: unit node weights
    int32_t tile16 = 0;     // every non-hub weighted degree is below 2^16
};

// Read-only view of the partition for neighbour gathers: the caller's int32
// array, or a compact copy with 1 (k <= 256) or 2 bytes per node that stays
// resident in L2. flagged (1 byte, k <= 128): bit 7 marks the move
// candidates of the round (set by the best-move pass, cleared when the copy
// is rebuilt), so the conflict filter reads a neighbour's key only when it is
// a candidate.
struct PartView {
    const void *p;
    int bytes;
    int flagged = 0;
};
constexpr uint8_t kCandFlag = 0x80;

__device__ __forceinline__ int32_t pget(const PartView &pv, int64_t u)
{
    if (pv.bytes == 1) {
        const int32_t x = ((const uint8_t *)pv.p)[u];
        return pv.flagged ? (x & (kCandFlag - 1)) : x;
    }
    if (pv.bytes == 2) return ((const uint16_t *)pv.p)[u];
    return ((const int32_t *)pv.p)[u];
}

// The same with the width fixed at compile time: a plain load, no branch (a
// load inside a branch is waited for before the branch joins, which
// serialises loads that are meant to be in flight together). mask: 0x7F for
// a flagged copy, else all ones.
template <int PB>
__device__ __forceinline__ int32_t pget_w(const void *p, int64_t u, int32_t mask)
{
    if constexpr (PB == 1) return ((const uint8_t *)p)[u] & mask;
    else if constexpr (PB == 2) return ((const uint16_t *)p)[u];
    else return ((const int32_t *)p)[u];
}
__device__ __forceinline__ int32_t part_mask(const PartView &pv)
{
    return pv.flagged ? (int32_t)(kCandFlag - 1) : -1;
}

__device__ __forceinline__ void pset(void *pc, int bytes, int64_t v, int32_t b)
{
    if (bytes == 1) ((uint8_t *)pc)[v] = (uint8_t)b;
    else if (bytes == 2) ((uint16_t *)pc)[v] = (uint16_t)b;
}

struct HubChunk {
    int32_t hub;     // index into the sorted hub id list
    int32_t nchunk;  // chunks of this hub
    int64_t e0, e1;
};

// Hub description handed to kernels.
struct HubView {
    int32_t nh;
    const int32_t *ids;   // sorted node ids of hubs
    const HubChunk *chunks;
    int64_t nchunks;
    int64_t *gacc;        // [nh] filter gain accumulator
    const uint32_t *bits; // [ceil(n/32)] bit v set iff v is a hub
    unsigned int *ticket; // [nh] chunks of the filter done (the last one decides)
};

__device__ __forceinline__ bool is_hub(const HubView &h, int64_t u)
{
    return h.nh > 0 && ((h.bits[u >> 5] >> (u & 31)) & 1u);
}

// ---------------------------------------------------------------- device --
// Marks tile t of the gain table for a rebuild. The flag is read first and
// written only while it is clear: once a tile is marked, the moves of its
// other neighbours only read the cached byte instead of queueing stores on
// the few cache lines that hold every tile's flag.
__device__ __forceinline__ void mark_dirty(uint8_t *dirty, int64_t t)
{
    if (dirty[t] == 0) dirty[t] = 1;
}


__device__ __forceinline__ int64_t node_weight(const GraphView &g, int64_t v)
{
    return g.vwgt ? (int64_t)g.vwgt[v] : 1;
}

__device__ __forceinline__ int32_t edge_weight(const GraphView &g, int64_t e)
{
    return g.adjwgt ? g.adjwgt[e] : 1;
}

// Streaming reads: data read once per pass (adjacency, table rows) carry the
// non-temporal hint, so that the L2 favours the small arrays gathered at
// random (compact partition, keys).
typedef int32_t v4i32 __attribute__((ext_vector_type(4)));
__device__ __forceinline__ int32_t stream_load(const int32_t *p)
{
    return __builtin_nontemporal_load(p);
}
__device__ __forceinline__ v4i32 stream_load4(const int32_t *p16)
{
    return __builtin_nontemporal_load((const v4i32 *)p16);
}
__device__ __forceinline__ int32_t stream_edge_weight(const GraphView &g, int64_t e)
{
    return g.adjwgt ? stream_load(g.adjwgt + e) : 1;
}

// 3^l for l < kSlots as 128-bit values (low and high words), built at
// compile time.
struct Pow3Table {
    uint64_t lo[kSlots], hi[kSlots];
};
constexpr Pow3Table make_pow3_table()
{
    Pow3Table t{};
    unsigned __int128 r = 1;
    for (int l = 0; l < kSlots; ++l) {
        t.lo[l] = (uint64_t)r;
        t.hi[l] = (uint64_t)(r >> 64);
        r *= 3;
    }
    return t;
}
static __constant__ Pow3Table kPow3 = make_pow3_table();

// Least l in [0, kSlots) with w * 2^l <= c * 3^l (l = ceil(log_1.5(w / c))
// for w > c, 0 for w <= c), kSlots - 1 if none. Binary search: the predicate
// is monotone in l because 3^l / 2^l grows. w < 2^63 and c < 2^31, so both
// sides fit 128 bits (3^53 < 2^85).
__device__ __forceinline__ int slot_of(int64_t w, int64_t c)
{
    if (w <= c) return 0;
    const unsigned __int128 W = (uint64_t)w, C = (uint64_t)c;
    int lo = 1, hi = kSlots - 1;  // predicate false at 0, answer in [1, kSlots - 1]
    while (lo < hi) {
        const int mid = (lo + hi) >> 1;
        const unsigned __int128 p = ((unsigned __int128)kPow3.hi[mid] << 64) | kPow3.lo[mid];
        if ((W << mid) <= C * p) hi = mid;
        else lo = mid + 1;
    }
    return lo;
}

// Rebalancing priority bucket (lower first): gain*c for gain >= 0 and gain/c
// for gain < 0, higher priority first, bucketed by ceil(log_1.5).
__device__ __forceinline__ int rebalance_bucket(int64_t gain, int64_t c)
{
    if (gain > 0) return kSlots - 1 - slot_of(gain * c, 1);
    if (gain == 0) return kSlots;
    return kSlots + 1 + slot_of(-gain, c);
}

// min(q * c, kPenCap) for q, c >= 0 (a Q16 penalty factor and a node
// weight), from the exact 128-bit product: no 64-bit division.
__device__ __forceinline__ int64_t sat_mul_pen(int64_t q, int64_t c)
{
    const uint64_t lo = (uint64_t)q * (uint64_t)c;
    const uint64_t hi = __umul64hi((uint64_t)q, (uint64_t)c);
    return (hi != 0 || lo > (uint64_t)kPenCap) ? kPenCap : (int64_t)lo;
}

__device__ __forceinline__ int lane_id() { return (int)__lane_id(); }

// Sum over an aligned group of G lanes (G a power of two <= 64).
template <int G, typename T>
__device__ __forceinline__ T group_sum(T x)
{
#pragma unroll
    for (int off = G / 2; off > 0; off >>= 1) x += __shfl_xor(x, off);
    return x;
}

template <typename T>
__device__ __forceinline__ T wave_sum(T x)
{
    return group_sum<64, T>(x);
}

// Block-wide sum (blockDim.x == kBlock); result valid in every thread.
template <typename T>
__device__ __forceinline__ T block_sum(T x, T *lds /* >= 4 */)
{
    x = wave_sum(x);
    const int w = threadIdx.x >> 6;
    __syncthreads();
    if (lane_id() == 0) lds[w] = x;
    __syncthreads();
    T s = lds[0] + lds[1] + lds[2] + lds[3];
    __syncthreads();
    return s;
}

// Inclusive scan over the wave.
template <typename T>
__device__ __forceinline__ T wave_incl_scan(T x)
{
    const int lane = lane_id();
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
        T y = __shfl_up(x, off);
        if (lane >= off) x += y;
    }
    return x;
}

// Block-wide inclusive scan (blockDim.x == 64 * NW, kBlock by default);
// returns the inclusive prefix of the calling thread and the block total in
// *total.
template <typename T, int NW = kBlock / 64>
__device__ __forceinline__ T block_incl_scan(T x, T *lds /* >= NW */, T *total)
{
    T inc = wave_incl_scan(x);
    const int w = threadIdx.x >> 6;
    __syncthreads();
    if (lane_id() == 63) lds[w] = inc;
    __syncthreads();
    T base = 0, all = 0;
#pragma unroll
    for (int i = 0; i < NW; ++i) {
        if (i < w) base += lds[i];
        all += lds[i];
    }
    *total = all;
    __syncthreads();
    return base + inc;
}

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

// Blocks [B0, B0 + nb) of the graphs that own nodes [lo, hi) (a batch's
// graphs own consecutive node ranges and consecutive block ranges).
__device__ __forceinline__ void node_block_window(const Blocks &bk, const int64_t *goff,
                                                  int64_t lo, int64_t hi, int32_t *B0, int32_t *nb)
{
    if (!goff || bk.ng == 1) {
        *B0 = 0;
        *nb = bk.total();
        return;
    }
    const int32_t g0 = graph_of_node(goff, bk.ng, lo);
    const int32_t g1 = graph_of_node(goff, bk.ng, hi - 1);
    *B0 = g0 * bk.k;
    *nb = (g1 - g0 + 1) * bk.k;
}

// Largest i in [0, cnt) with a[i] <= p (a nondecreasing, a[0] <= p).
__device__ __forceinline__ int upper_index(const int32_t *a, int cnt, int32_t p)
{
    int lo = 0, hi = cnt - 1;
    while (lo < hi) {
        int mid = (lo + hi + 1) >> 1;
        if (a[mid] <= p) lo = mid;
        else hi = mid - 1;
    }
    return lo;
}

// Wave-aggregated append: lanes with pred reserve consecutive slots of a
// list whose length lives in *counter. Returns the slot (or -1).
__device__ __forceinline__ int64_t wave_append(bool pred, unsigned long long *counter)
{
    const uint64_t mask = __ballot(pred);
    if (mask == 0) return -1;
    const int lane = lane_id();
    const int leader = __ffsll((unsigned long long)mask) - 1;
    unsigned long long base = 0;
    if (lane == leader) base = atomicAdd(counter, (unsigned long long)__popcll(mask));
    base = __shfl(base, leader);
    if (!pred) return -1;
    const uint64_t below = lane == 0 ? 0 : (mask & ((~0ull) >> (64 - lane)));
    return (int64_t)(base + __popcll(below));
}

__device__ __forceinline__ void atomic_add_i64(int64_t *p, int64_t v)
{
    atomicAdd((unsigned long long *)p, (unsigned long long)v);
}

// Position of the n-th (0-based) set bit of mask (n < popcount(mask)).
__device__ __forceinline__ int nth_set_bit(uint64_t mask, int n)
{
    int pos = 0;
#pragma unroll
    for (int w = 32; w >= 1; w >>= 1) {
        const int c = __popcll((mask >> pos) & ((1ull << w) - 1));
        if (n >= c) {
            n -= c;
            pos += w;
        }
    }
    return pos;
}

// base[key] += val for every active lane, one global atomic per distinct key
// of the wave (lanes with equal keys are summed first).
__device__ __forceinline__ void wave_hist_add(int64_t *base, int64_t key, int64_t val, bool active)
{
    uint64_t pending = __ballot(active);
    const int lane = lane_id();
    while (pending) {
        const int leader = __ffsll((unsigned long long)pending) - 1;
        const int64_t lk = __shfl(key, leader);
        const bool same = active && key == lk;
        const uint64_t sm = __ballot(same);
        const int64_t sum = wave_sum(same ? val : (int64_t)0);
        if (lane == leader) atomic_add_i64(base + lk, sum);
        pending &= ~sm;
        active = active && !same;
    }
}

// Spread counters (see kCntCopies).
__device__ __forceinline__ void cnt_add(unsigned long long *c, int slot, unsigned long long v)
{
    atomicAdd(&c[(blockIdx.x & (kCntCopies - 1)) * CNT_COUNT + slot], v);
}
__device__ __forceinline__ unsigned long long cnt_get(const unsigned long long *c, int slot)
{
    unsigned long long s = 0;
#pragma unroll 16
    for (int i = 0; i < kCntCopies; ++i) s += c[i * CNT_COUNT + slot];
    return s;
}
// The same sum read by a whole wave (every lane active): lane i loads copy i,
// so the copies arrive in one round trip; every lane gets the sum.
__device__ __forceinline__ unsigned long long wave_cnt_get(const unsigned long long *c, int slot)
{
    static_assert(kCntCopies == 64, "one copy per lane");
    return wave_sum(c[lane_id() * CNT_COUNT + slot]);
}
// One thread sets a counter: copy 0 holds the value, the others 0.
__device__ __forceinline__ void cnt_set(unsigned long long *c, int slot, unsigned long long v)
{
    for (int i = 0; i < kCntCopies; ++i) c[i * CNT_COUNT + slot] = i == 0 ? v : 0ull;
}

// The same by a whole wave: lane i writes copy i.
__device__ __forceinline__ void wave_cnt_set(unsigned long long *c, int slot, unsigned long long v)
{
    const int i = lane_id();
    c[i * CNT_COUNT + slot] = i == 0 ? v : 0ull;
}

// Add the number of lanes with pred to an LDS counter (lane 0 of the wave).
__device__ __forceinline__ void wave_count(bool pred, unsigned long long *lds_counter)
{
    const uint64_t m = __ballot(pred);
    if (lane_id() == 0 && m) atomicAdd(lds_counter, (unsigned long long)__popcll(m));
}

// ------------------------------------------------------------ launchers --
// Each returns hipGetLastError() after enqueueing on `s`.

hipError_t launch_fill_i64(int64_t *p, int64_t count, int64_t value, hipStream_t s);
hipError_t launch_fill_i32(int32_t *p, int64_t count, int32_t value, hipStream_t s);

// plan
hipError_t launch_plan_scan(const GraphView &g, int32_t *wdeg, int64_t hub_t, int32_t *hub_list,
                            unsigned long long *counters, hipStream_t s);
// stage 0: xadj and node weights; 1: ids in range, edge weights; 2: also
// self-loops, sorted rows, symmetry.
hipError_t launch_validate(const GraphView &g, unsigned long long *flags, int stage,
                           hipStream_t s);
hipError_t launch_hub_ranges(const int64_t *xadj, const int32_t *ids, int32_t nh, int64_t *e01,
                             hipStream_t s);

// table (S1)
int gain_tile_nodes(int32_t k, int64_t n);
// The full table: one workgroup per tile of non-hub rows and, in the same
// launch, one per chunk of a hub's edges, which adds the chunk's counts into
// the hub's row: the hub rows must be zero (launch_zero_hub_rows).
// inner / own: each non-hub node's conn[v][own block] also goes to inner[v];
// own is the partition in node order.
hipError_t launch_gain_table(const GraphView &g, int32_t k, const PartView &part, int32_t *conn,
                             int64_t hub_t, const HubView &h, hipStream_t s,
                             int32_t *inner = nullptr, const PartView &own = PartView{});
// After an apply: the tiles whose dirty flag is set (flags are cleared), or
// every tile once the moving nodes' degrees (counters[CNT_MOVED_DEG]) sum
// above all_threshold, and the hub rows (cleared by the hub apply) once they
// sum above dirty_threshold. In the delta mode every workgroup returns at
// once.
hipError_t launch_gain_refresh(const GraphView &g, int32_t k, const PartView &part, int32_t *conn,
                               int64_t hub_t, const HubView &h, uint8_t *dirty,
                               const unsigned long long *counters, int64_t dirty_threshold,
                               int64_t all_threshold, hipStream_t s);
// Clears the hubs' rows of conn.
hipError_t launch_zero_hub_rows(const HubView &h, int32_t *conn, int32_t k, hipStream_t s);
// Compact copy of the local blocks (bytes = 1 or 2). Checks every value: a
// global block id below bk.total() and, for a batch (goff = node offsets of
// the graphs, ng + 1 entries), a block of the node's own graph; violations
// count in counters[CNT_BAD_INPUT]. With order / pc2: also the copy in the
// plan's label order, pc2[i] = local block of node order[i].
hipError_t launch_pack_part(int64_t n, const Blocks &bk, const int64_t *goff, const int32_t *part,
                            void *pc, int bytes, unsigned long long *counters, hipStream_t s,
                            const int32_t *order = nullptr, void *pc2 = nullptr);
hipError_t launch_hub_bits(const HubView &h, uint32_t *bits, hipStream_t s);
// Neighbour ids renumbered by descending degree (ties by id) for the table
// build: order[i] = node of label i, perm[v] = label of v, adj_r[e] =
// perm[adjncy[e]]. Allocates and frees its own sort space; synchronises s.
hipError_t launch_degree_relabel(const GraphView &g, int64_t nnz, int32_t *order, int32_t *perm,
                                 int32_t *adj_r, hipStream_t s);

// Per node: 2*cut into counters[cut_slot], penalty buckets of the available
// nodes (bucket may be null), block weights W[part] += c (W may be null),
// availability for rebalancing (avail may be null).
// gstat (batch): the cut also goes to gstat[graph][gs_slot].
// Geometry: each workgroup takes span consecutive nodes; window bounds the
// blocks of the graphs owning such a range (a batch's goff; zeros: one
// graph, default span).
struct StatsGeom {
    const int64_t *goff = nullptr;
    int64_t span = 0;
    int32_t window = 0;
};
// inner (may be null): conn[v][part[v]] of the non-hub nodes, written by the
// table build; hub_bits marks the hubs, whose entry is gathered from the row.
// cut_cond (one graph, cut statistics only): unless counters[CNT_CUT_STALE]
// is set, the pass stores CNT_CUT2_BEFORE + CNT_CUT2_DELTA into cut_slot
// and reads nothing else.
// Node range of the statistics pass for n nodes, at most max_span (> 0).
int64_t stats_span(int64_t n, int64_t max_span);
hipError_t launch_node_stats(const GraphView &g, const Blocks &bk, const StatsGeom &sg,
                             const int32_t *part, const int32_t *conn, const int32_t *wdeg,
                             int64_t *W, int64_t *bucket, int32_t t_num, int32_t t_den,
                             unsigned long long *counters, int cut_slot, uint8_t *avail,
                             int64_t *gstat, int gs_slot, hipStream_t s,
                             const int32_t *inner = nullptr, const uint32_t *hub_bits = nullptr,
                             bool cut_cond = false, int64_t *wsp = nullptr,
                             int64_t *bsp = nullptr, int ncopies = 1);
// Copies of the statistics pass's block weights and slot histogram for K
// blocks (wsp [ncopies * K], bsp [ncopies * K * kSlots]; a workgroup adds to
// copy blockIdx.x mod ncopies, so that the pass's workgroups do not all add
// to the same entries): launch_cb_prefix with the same copies adds their sums
// into W and the histogram and clears them. 1: no copies.
constexpr int kStatsCopiesMax = 8;
inline int stats_copies(int64_t K)
{
    return K * kSlots * kStatsCopiesMax <= ((int64_t)1 << 20) ? kStatsCopiesMax : 1;
}
hipError_t launch_block_weights(const GraphView &g, int32_t k, const int32_t *part, int64_t *W,
                                unsigned long long *counters, hipStream_t s);
// 2 * cut from the adjacency into the spread counter `slot`; out = that / 2.
hipError_t launch_cut_edges(const GraphView &g, const int32_t *part, unsigned long long *counters,
                            int slot, hipStream_t s);
hipError_t launch_store_half(const unsigned long long *counters, int slot, int64_t *out,
                             hipStream_t s);
// Spread counter dst = src.
hipError_t launch_cnt_copy(unsigned long long *counters, int dst, int src, hipStream_t s);
// Spread counter slot = v.
hipError_t launch_cnt_set(unsigned long long *counters, int slot, unsigned long long v,
                          hipStream_t s);
hipError_t launch_check_part(int64_t n, int32_t k, const int32_t *part,
                             unsigned long long *counters, hipStream_t s);

// moves (S0, S2-S4)
// Zero the counters, the buckets ([K][kSlots]), zero2 ([zero2_count]) and,
// if zero_w, W ([K]). With single (one graph) also publish its penalty table
// and L_max into bk.penq / bk.lmax / bk.src_lmax (writable workspace).
// With hub_conn: also clears the hubs' rows of the table (k entries each).
hipError_t launch_round_init(const Blocks &bk, int64_t *bucket, int64_t *W, const PenTable &pq,
                             int64_t lmax, int single, unsigned long long *counters, int zero_w,
                             unsigned long long *zero2, int64_t zero2_count, hipStream_t s,
                             const HubView &h = HubView{}, int32_t *hub_conn = nullptr,
                             int32_t k = 0);
// Prefix sums of the buckets; pen1[B] = penalty of a unit-weight node moving
// into B (0 if it fits, -1 if forbidden).
hipError_t launch_cb_prefix(const Blocks &bk, int64_t *bucket, int64_t *W, int mode,
                            int64_t *pen1, hipStream_t s, int64_t *wsp = nullptr,
                            int64_t *bsp = nullptr, int ncopies = 1);
// active (may be null: every node): only nodes with active[v] != 0 look for
// a move. cflag (may be null): the compact partition copy whose bit 7 marks
// the candidates; cflag2 / key2 / perm (may be null): the flagged copy and
// the candidates' keys in the plan's label order.
// pv / adj_deg: nodes of degree <= adj_deg (0: none) are decided from their
// adjacency with the neighbours' blocks from the compact copy pv (1 or 2
// bytes), the others from their table row; best_move_adj_deg(k, bytes,
// max_deg) is the default bound. max_deg: the graph's largest degree (with max_deg <=
// adj_deg the row kernel is not launched).
int32_t best_move_adj_deg(int32_t k, int pv_bytes, int64_t max_deg);
hipError_t launch_best_move(const GraphView &g, const Blocks &bk, const int32_t *part,
                            const int32_t *conn, const int64_t *W, const int64_t *cb,
                            const int64_t *pen1, int mode, const uint8_t *active, int64_t *key,
                            int64_t *pen, unsigned long long *counters, uint8_t *cflag,
                            hipStream_t s, uint8_t *cflag2 = nullptr, int64_t *key2 = nullptr,
                            const int32_t *perm = nullptr, const PartView &pv = PartView{},
                            int32_t adj_deg = 0, int64_t max_deg = 0);
// With gp_out the pessimistic gains are stored (decided by launch_filter_seq).
// adj_r / pv2 / key2 / order (may be null; one-byte flagged pv only):
// neighbours' blocks and keys read by label from the copies in the plan's
// degree order, and a neighbour's id (for a tie of scores) from order.
// optimistic: an earlier candidate neighbour counts in its target block.
hipError_t launch_filter(const GraphView &g, const Blocks &bk, int optimistic, const int32_t *part,
                         const PartView &pv,
                         const int64_t *key, const int64_t *pen, int64_t hub_t,
                         int32_t *mvto, uint8_t *accflag, unsigned long long *counters,
                         int64_t *gp_out, hipStream_t s, const int32_t *adj_r = nullptr,
                         const PartView &pv2 = PartView{}, const int64_t *key2 = nullptr,
                         const int32_t *order = nullptr);
hipError_t launch_filter_hub(const GraphView &g, const Blocks &bk, int optimistic,
                             const int32_t *part, const PartView &pv,
                             const int64_t *key, const int64_t *pen, const HubView &h,
                             int32_t *mvto, uint8_t *accflag, unsigned long long *counters,
                             int64_t *gp_out, hipStream_t s);
hipError_t launch_filter_seq(const GraphView &g, const Blocks &bk, const int32_t *part,
                             const int32_t *cand, int64_t ne, const int64_t *key,
                             const int64_t *gp, const int64_t *netpre, const int64_t *W,
                             const int64_t *cb, int mode, int64_t hub_t, int32_t *mvto,
                             uint8_t *accflag, unsigned long long *counters, hipStream_t s);

// Sequence-aware penalty (k_seq.hip): the eligible candidates (pessimistic
// gain > 0) in id order, then the weight change of each one's target
// accumulated before it. Score bits: scores are below 2^seq_score_bits.
int seq_score_bits(int64_t max_wdeg);
size_t seq_temp_bytes(int64_t n);
hipError_t launch_seq_select(int64_t n, const int64_t *key, const int64_t *gp, int32_t *cand,
                             unsigned long long *count, void *temp, size_t temp_bytes,
                             hipStream_t s);
hipError_t launch_seq_net(int64_t ne, const int32_t *cand, const int64_t *key, const int32_t *part,
                          const int32_t *vwgt, const uint8_t *avail, const Blocks &bk, int sb,
                          uint64_t *ev_key, uint64_t *ev_key2, uint32_t *ev_val,
                          uint32_t *ev_val2, int64_t *prefix, int64_t *netpre, void *temp,
                          size_t temp_bytes, hipStream_t s);
// Segment path: events grouped by block, each block's segment (split into
// buckets by sampled splitters when it is long) sorted, scanned and decided
// by one workgroup per bucket (accflag, mvto, CNT_ACC, CNT_MOVED_DEG as
// launch_filter_seq). Usable iff seq_segments_fit(sb, n): an event (order,
// node id, outflow flag) fits 64 bits. NB = seq_bucket_bound(n, K).
constexpr int kSegCopyEntries = 4096;  // counter copies of all blocks (when there are few)
constexpr int kSegCopyPad = 16;        // counters per cache line
struct SegWs {
    unsigned long long *cur;    // [max(K, kSegCopyEntries * kSegCopyPad)] counts, then cursors
    int64_t *seg_off;           // [K + 1] segment starts
    int32_t *boff, *cpre;       // [K + 1] first bucket / first bucketing chunk of each block
    int32_t *slist;             // [K] blocks whose segment is split
    int32_t *meta;              // [4] meta[0]: number of split blocks
    int32_t *bblk;              // [NB] block of each bucket
    int64_t *bpos, *bsize;      // [NB] bucket start and size
    int64_t *bdel;              // [NB] weight-change sums, then carries
    unsigned long long *bcnt;   // [NB] counts, then cursors
    int64_t *scan_c, *scan_d;   // [NB] scratch of the bucket offsets
    uint64_t *spl;              // [NB] splitters
    uint64_t *ev, *tmp;         // [2n] event keys, bucket / merge buffer
    int32_t bucket_avg;         // target bucket size of a split segment (>= seq_bucket_avg_min())
};
int seq_id_bits(int64_t n);
int64_t seq_bucket_bound(int64_t n, int K);
int seq_bucket_avg_min();
// Entries of ws.cur the segment path uses for K blocks; they must be zero
// when it starts (the round's init clears them).
int64_t seq_counter_words(int K);
bool seq_segments_fit(int sb, int64_t n);
// goff: a batch's node offsets (null for one graph).
hipError_t launch_seq_segments(const GraphView &g, const Blocks &bk, const int64_t *goff,
                               const int64_t *key, const int64_t *gp, const int32_t *part,
                               const uint8_t *avail, int sb, const SegWs &ws, const int64_t *W, const int64_t *cb,
                               int mode, int64_t hub_t, int32_t *mvto, uint8_t *accflag,
                               unsigned long long *counters, hipStream_t s);
// Apply every move recorded in mvto (target block, -1 = none) and clear it.
// If the moving nodes' degrees sum to at most dirty_threshold
// (counters[CNT_MOVED_DEG]) the neighbours' rows get integer-atomic deltas;
// otherwise their gain-table tiles are marked and rebuilt from the new
// partition, and the hub rows are rebuilt; above all_threshold no tile is
// marked and every tile is rebuilt.
// pv: the compact partition copy to keep in step (pv.p writable, or bytes 4).
// tg / tpv: the graph and partition views the table build reads (the
// relabelled ones when the plan has them); pc2 / perm (may be null): the
// compact copy in label order, kept in step with pv.
// cut_delta (one graph): before the apply changes anything, the change of
// 2 * cut the moves make is added to counters[CNT_CUT2_DELTA] in the delta
// mode; when tiles are rebuilt instead, counters[CNT_CUT_STALE] is raised.
hipError_t launch_apply(const GraphView &g, const Blocks &bk, int32_t *part, const PartView &pv,
                        int32_t *conn, int64_t *W, int32_t *mvto, int64_t hub_t,
                        const HubView &h, unsigned long long *counters,
                        int64_t dirty_threshold, uint8_t *dirty, const GraphView &tg,
                        const PartView &tpv, void *pc2, const int32_t *perm,
                        int64_t all_threshold, hipStream_t s, bool cut_delta = false,
                        int64_t *wcp = nullptr, int ncopies = 1);
// Copies of the apply's block-weight sums (wcp [ncopies * K]; a workgroup
// adds to copy blockIdx.x mod ncopies instead of all of them to W): the next
// launch_rb_begin with the same copies adds them into W and clears them.
constexpr int kApplyCopiesMax = 8;
// iters < 0: iters and status derived on the device for a rebalancing that
// ended after its speculative first sub-iteration.
hipError_t launch_stats_final(int64_t *stats, const unsigned long long *counters, int64_t lmax,
                              int64_t iters, int64_t status, hipStream_t s);
hipError_t launch_export_moves(int64_t n, const int64_t *key, const int64_t *pen,
                               const uint8_t *accflag, int32_t *target, int64_t *score,
                               int64_t *pen_out, uint8_t *accept, hipStream_t s);

// rebalance (S5)
// Rebalancing workspace; K = bk.total() blocks (global block ids).
struct RebalWs {
    int32_t *rtgt;       // [n] target block of a node of an overloaded block, -1 if none
    uint8_t *rbeta;      // [n] its priority bucket
    int64_t *W0;         // [K] block weights at sub-iteration start
    int64_t *hist_src;   // [hist_copies * K * kRbBuckets]: copy c from c * K * kRbBuckets on
    int64_t *hist_tgt;   // [hist_copies * K * kRbBuckets]
    int32_t *cbeta_src;  // [K] cutoff bucket per source block
    int32_t *cbeta_tgt;  // [K] cutoff bucket per target block
    int64_t *need_src;   // [K] weight still needed inside the cutoff bucket
    int64_t *room_tgt;   // [K] capacity left inside the cutoff bucket
    int32_t *theta_src;  // [K] id bound inside the cutoff bucket (exclusive)
    int32_t *theta_tgt;  // [K]
    int64_t *chunk_src;  // [K * nchunks]
    int64_t *chunk_tgt;  // [K * nchunks]
    int chunk_shift;     // a chunk holds 2^chunk_shift consecutive node ids of one graph
    int64_t nchunks;
    const int64_t *goff;  // batch: node offset of each graph (ng + 1 entries); null: one graph
    int hist_copies;      // copies of each histogram (a node scan's workgroup adds to one)
};

// Copies of the rebalancing histograms for up to K blocks (their sum is read).
constexpr int kRbHistCopiesMax = 8;
inline int rb_hist_copies(int64_t K)
{
    return K * kRbBuckets * kRbHistCopiesMax <= ((int64_t)1 << 20) ? kRbHistCopiesMax : 1;
}

// Snapshot W and count the source blocks (weight above src_lmax): in total
// (counters[CNT_OVER]) and, for a batch, per graph (gstat[g][GS_OVER]).
// pub (host-coherent memory, may be null): the sums of all CNT_COUNT counters
// go to pub[1 + slot], then pub[0] = seq with a system-scope release, so the
// host can read them without waiting for the stream.
hipError_t launch_rb_begin(const Blocks &bk, int64_t *W, const RebalWs &r,
                           unsigned long long *counters, int64_t *gstat, hipStream_t s,
                           int first = 0, unsigned long long *pub = nullptr,
                           unsigned long long seq = 0, int64_t *wcp = nullptr, int ncopies = 1);
// One sub-iteration up to the move marks: targets and buckets, source and
// target selection; accepted nodes get mvto[v] = target. hist32: the
// per-workgroup histograms may use 32-bit LDS counters (no overflow).
// gstat (batch): moves per graph in gstat[g][GS_MOVED_NOW] (reset first) and
// gstat[g][GS_REBAL_MOVES].
// plain: rebalancing priority by the gain alone (node weight left out).
// rbrec (may be null): moved nodes get (iter << 8) | priority bucket.
hipError_t launch_rb_iteration(const GraphView &g, const Blocks &bk, const int32_t *part,
                               const int32_t *conn, const RebalWs &r, int32_t *mvto, int hist32,
                               int plain, int64_t hub_t, unsigned long long *counters,
                               int64_t *gstat, hipStream_t s, int32_t *rbrec = nullptr,
                               int32_t iter = 0);
int rb_scan_grid(int64_t n);

// interleaved move sequence and best prefix (k_prefix.hip). Workspace for
// n nodes and K blocks (one graph).
struct BpWs {
    int32_t *part0, *rbrec;                      // [n] round-start partition; S5 move records
    int64_t *W0;                                 // [K] round-start block weights
    uint8_t *fm, *fr;                            // [n] in the filtered list / the rebalancing list
    int32_t *ids, *ids2, *mlist, *rlist;         // [n] selections and their sorted orders
    int32_t *rfrom, *rto, *tau, *stepof;         // [n]
    int64_t *rc, *rwi, *rin_inc;                 // [n]
    uint64_t *rin_key;                           // [n]
    uint64_t *k0, *k1, *evs;                     // [3n] sort keys, [2n] sorted events
    int64_t *d0, *d1, *acc;                      // [3n]
    int32_t *need, *tcum;                        // [2n]
    int64_t *pos;                                // [n]
    int32_t *ecnt, *rcnt, *eoff, *roff, *rinoff; // [K + 1] each (rcnt inside ecnt's allocation)
    int32_t *cstep, *rbefore, *over_incl;        // [n + 1]
    int64_t *stepgain, *gain_incl;               // [n + 1]
    int64_t *best_g;                             // [1024]
    int32_t *best_j;                             // [1024]
    int32_t *cnt;                                // [2]
    unsigned long long *changed;                 // [1]
    int64_t *scal;                               // [4]: best boundary, nodes undone
    void *temp;
    size_t temp_bytes;
};
// What the undo needs to call the apply.
struct BpApply {
    Blocks bk;
    int64_t hub_t;
    HubView h;
    int64_t dirty_threshold;
    uint8_t *dirty;
    GraphView tg;
    PartView tpv;
    void *pc2;
    const int32_t *perm;
    int64_t all_threshold;
};
size_t bp_temp_bytes(int64_t n);
// Before the moves: copies part and W, clears the rebalancing records.
hipError_t launch_bp_record_start(int64_t n, int32_t K, const int32_t *part, const int64_t *W,
                                  const BpWs &ws, hipStream_t s);
// After S5: builds the sequence, keeps the best balanced prefix and undoes
// the rest (synchronises s a few times). iterations: fixed-point rounds.
hipError_t run_best_prefix(const GraphView &g, int32_t K, int64_t lmax, int32_t *part,
                           const PartView &pv, int32_t *conn, int64_t *W, const uint8_t *accflag,
                           const int64_t *key, int32_t *mvto, unsigned long long *counters,
                           const BpWs &ws, const BpApply &apply, int64_t *stats, int *iterations,
                           hipStream_t s);
// Statistics slots 8 (status 0 when a balanced boundary was kept), 9 and 10.
hipError_t launch_bp_stats(const BpWs &ws, int64_t *stats, hipStream_t s);

// no-allocation edge cut (noalloc.hip): the device address of the scratch
// array on `device` (which the caller made current), taken once per device;
// then the two-pass cut with that address.
hipError_t noalloc_init(int device, void **ptr);
hipError_t launch_cut_noalloc(const GraphView &g, const int32_t *part, int64_t *cut,
                              void *scratch_ptr, hipStream_t s);

// batches (k_batch.hip)
hipError_t launch_batch_copy(const GraphView &src, int64_t node_off, int64_t edge_off,
                             int64_t nnz, int64_t *xadj, int32_t *adjncy, int32_t *adjwgt,
                             int32_t *vwgt, int last, hipStream_t s);
// rec: device int64 [nrec][5] = (source node offset, destination node
// offset, nodes, source graph, destination graph); max_cells: the largest
// nodes * k among them.
hipError_t launch_batch_carry(const int64_t *rec, int32_t nrec, int64_t max_cells, int32_t k,
                              const int32_t *src_part, const int32_t *src_conn,
                              const int64_t *src_W, int32_t *dst_part, int32_t *dst_conn,
                              int64_t *dst_W, hipStream_t s);
// out[2g] = total node weight of graph g, out[2g + 1] = its largest node weight.
hipError_t launch_batch_totals(const int64_t *goff, int32_t ng, const int32_t *vwgt, int64_t *out,
                               hipStream_t s);
hipError_t launch_batch_move_stats(int64_t n, int64_t span, const Blocks &bk, const int64_t *goff,
                                   const int32_t *part, const int64_t *key,
                                   const uint8_t *accflag, int64_t *gstat, hipStream_t s);
hipError_t launch_batch_stats_final(int32_t ng, const int64_t *gstat, const int64_t *lmax,
                                    const int64_t *host3, int moved, int64_t *stats, hipStream_t s);
// driver: count of nonzero bytes; boundary nodes; nodes that did not move
// with a neighbour that moved
hipError_t launch_count_u8(const uint8_t *a, int64_t n, int64_t *out, hipStream_t s);
hipError_t launch_boundary(const GraphView &g, const int32_t *part, uint8_t *active, hipStream_t s);
hipError_t launch_next_active(const GraphView &g, const int32_t *before, const int32_t *after,
                              uint8_t *active, hipStream_t s);

}  // namespace upr
