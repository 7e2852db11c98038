// Sequence-aware penalty of the conflict filter.
//
// Candidates are ordered by (score desc, id asc). Section 5.3 prices a move
// into V_j by the block's weight when the move is made, c(V_j + u) + c~_j,
// where c~_j keeps the weight of rebalance-available nodes that left. Along
// the order each eligible candidate (pessimistic gain > 0) therefore adds
// its weight to its target block and, unless it is available for
// rebalancing, removes it from its own block. For every candidate the filter
// needs the change of its target's weight accumulated before it.
//
// The eligible candidates are listed in id order; each emits two events:
// (target(v), +c(v)) and, if v is not available, (part(v), -c(v)); both
// carry v's order key. Events are sorted by (block, score desc) with a stable
// radix sort over the id-ordered input, so equal scores stay in id order; an
// exclusive scan by block gives, at v's inflow event, the weight change of
// v's target before v.
//
// Two implementations. The segment path (used whenever an event fits one
// 64-bit key: order, id and the outflow flag) groups the events by block
// with a counting sort and lets one workgroup per block sort its segment,
// scan it and decide its inflow events: a candidate's decision involves
// only its target block, so no list of eligible candidates, no host
// synchronisation and no separate decision pass are needed. The general
// path sorts (block, order) keys with a device-wide radix sort.
#include "upr_common.h"

#include <cstring>

#include <rocprim/rocprim.hpp>

namespace upr {

namespace {

// Events are sorted on (block << sb | order) with sb = score bits: a score
// is below (max weighted degree + 1) * 2^16, and order = 2^sb - 1 - score
// puts higher scores first. Blocks are global ids (a batch's graphs never
// share one). The block field also holds the sentinel K (number of blocks) for
// the outflow events of available candidates (they change no block).
// rocPRIM's merge-sort path costs about ten passes on mid-sized inputs; the
// onesweep radix path is used from the single-block size up.
using SortConfig = rocprim::radix_sort_config<rocprim::default_config, rocprim::default_config,
                                              rocprim::default_config, 0>;

struct IsEligible {
    const int64_t *key;
    const int64_t *gp;
    __host__ __device__ bool operator()(int32_t v) const { return key[v] >= 0 && gp[v] > 0; }
};

struct EventBlock {
    int sb;
    __host__ __device__ uint32_t operator()(uint64_t k) const { return (uint32_t)(k >> sb); }
};

struct EventDelta {
    const int32_t *vwgt;
    __host__ __device__ int64_t operator()(uint32_t ev) const
    {
        const int64_t v = ev >> 1;
        const int64_t c = vwgt ? (int64_t)vwgt[v] : 1;
        return (ev & 1u) ? -c : c;
    }
};

// Two events per eligible candidate: inflow at its target, outflow at its
// own block (the sentinel block if it is available for rebalancing).
__global__ void k_seq_events(int64_t ne, const int32_t *cand, const int64_t *key,
                             const int32_t *part, const uint8_t *avail, Blocks bk, int sb,
                             uint64_t sentinel, uint64_t *ev_key, uint32_t *ev_val)
{
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    const uint64_t top = ((uint64_t)1 << sb) - 1;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < ne; i += stride) {
        const int32_t v = cand[i];
        const int64_t kv = key[v];
        const uint64_t order = top - (uint64_t)(kv >> 16);  // score desc
        const int32_t A = part[v];
        const uint64_t b = (uint64_t)(bk.base(A) + (int32_t)(kv & 0xFFFF));
        const uint64_t a = (uint64_t)A;
        ev_key[2 * i] = (b << sb) | order;
        ev_val[2 * i] = ((uint32_t)v << 1);
        ev_key[2 * i + 1] = avail[v] ? sentinel : ((a << sb) | order);
        ev_val[2 * i + 1] = ((uint32_t)v << 1) | 1u;
    }
}

// The exclusive prefix at an inflow event is the weight change of the
// candidate's target before it.
__global__ void k_seq_scatter(int64_t nev, const uint32_t *ev_val, const int64_t *prefix,
                              int64_t *netpre)
{
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < nev; i += stride) {
        const uint32_t ev = ev_val[i];
        if ((ev & 1u) == 0) netpre[ev >> 1] = prefix[i];
    }
}

int grid_for(int64_t items)
{
    int64_t g = (items + kBlock - 1) / kBlock;
    if (g < 1) g = 1;
    if (g > 8192) g = 8192;
    return (int)g;
}

int bit_width(uint64_t x)
{
    int b = 0;
    while (x) {
        ++b;
        x >>= 1;
    }
    return b;
}

}  // namespace

int seq_score_bits(int64_t max_wdeg)
{
    return bit_width((uint64_t)(max_wdeg < 1 ? 1 : max_wdeg)) + 16;
}

size_t seq_temp_bytes(int64_t n)
{
    if (n <= 0) return 16;
    size_t a = 0, b = 0, c = 0;
    IsEligible pred{nullptr, nullptr};
    int32_t *out = nullptr;
    unsigned long long *cnt = nullptr;
    rocprim::select(nullptr, a, rocprim::counting_iterator<int32_t>(0), out, cnt, (size_t)n, pred,
                    (hipStream_t)0);
    uint64_t *k0 = nullptr, *k1 = nullptr;
    uint32_t *v0 = nullptr, *v1 = nullptr;
    rocprim::radix_sort_pairs<SortConfig>(nullptr, b, k0, k1, v0, v1, (size_t)(2 * n), 0, 64,
                                          (hipStream_t)0);
    int64_t *pre = nullptr;
    rocprim::exclusive_scan_by_key(
        nullptr, c, rocprim::make_transform_iterator(k1, EventBlock{0}),
        rocprim::make_transform_iterator(v1, EventDelta{nullptr}), pre, (int64_t)0,
        (size_t)(2 * n), rocprim::plus<int64_t>(), rocprim::equal_to<uint32_t>(), (hipStream_t)0);
    return std::max(a, std::max(b, c)) + 256;
}

hipError_t launch_seq_select(int64_t n, const int64_t *key, const int64_t *gp, int32_t *cand,
                             unsigned long long *count, void *temp, size_t temp_bytes,
                             hipStream_t s)
{
    size_t bytes = temp_bytes;
    return rocprim::select(temp, bytes, rocprim::counting_iterator<int32_t>(0), cand, count,
                           (size_t)n, IsEligible{key, gp}, s);
}

hipError_t launch_seq_net(int64_t ne, const int32_t *cand, const int64_t *key, const int32_t *part,
                          const int32_t *vwgt, const uint8_t *avail, const Blocks &bk, int sb,
                          uint64_t *ev_key, uint64_t *ev_key2, uint32_t *ev_val,
                          uint32_t *ev_val2, int64_t *prefix, int64_t *netpre, void *temp,
                          size_t temp_bytes, hipStream_t s)
{
    if (ne <= 0) return hipSuccess;
    const int64_t nev = 2 * ne;
    const uint64_t K = (uint64_t)bk.total();
    const uint64_t sentinel = K << sb;
    const int end_bit = sb + bit_width(K);
    hipLaunchKernelGGL(k_seq_events, dim3(grid_for(ne)), dim3(kBlock), 0, s, ne, cand, key, part,
                       avail, bk, sb, sentinel, ev_key, ev_val);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    size_t bytes = temp_bytes;
    e = rocprim::radix_sort_pairs<SortConfig>(temp, bytes, ev_key, ev_key2, ev_val, ev_val2,
                                              (size_t)nev, 0, end_bit, s);
    if (e != hipSuccess) return e;
    bytes = temp_bytes;
    e = rocprim::exclusive_scan_by_key(
        temp, bytes, rocprim::make_transform_iterator(ev_key2, EventBlock{sb}),
        rocprim::make_transform_iterator(ev_val2, EventDelta{vwgt}), prefix, (int64_t)0,
        (size_t)nev, rocprim::plus<int64_t>(), rocprim::equal_to<uint32_t>(), s);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_seq_scatter, dim3(grid_for(nev)), dim3(kBlock), 0, s, nev, ev_val2,
                       prefix, netpre);
    return hipGetLastError();
}

// ------------------------------------------------------- segment path --
//
// Events are grouped by block with a counting sort (per-block counts, their
// offsets, placement). Each workgroup of the counting passes takes a
// contiguous node range; in a batch its events fall into the blocks of the
// few graphs that own those nodes, so it counts them in LDS over that window
// of blocks and reserves its slots with one global atomic per block. A
// block's segment of at most kRun events is sorted in LDS by one workgroup.
// A longer segment is split into buckets of about SegWs::bucket_avg events
// (at least kBucketAvg) by splitters taken from a sorted sample of it
// (sample sort: the keys are distinct, so ties in the order cannot
// unbalance the buckets); its events are counted and scattered into the
// buckets by workgroups over chunks of kChunk events, and every bucket is
// sorted by its own workgroup. The scan of a bucket starts from the weight
// change of the buckets before it in its block, summed while counting. A
// bucket of up to 2 kRun events (a sampling outlier) is sorted in two
// halves merged in LDS; a larger one in runs merged pairwise through global
// memory (slow, but correct). Bucket boundaries depend on the placement
// order, the sorted order and the decisions do not.

namespace {

constexpr int kSegBins = 2048;          // block window up to which a workgroup aggregates in LDS
constexpr int kSegRows = 512;           // most workgroups of the counting and placement passes
constexpr int kSortItems = 4;           // keys per thread of the workgroup sorts
constexpr int kWaveKeys = 64 * kSortItems;
constexpr int kDecideThreads = 512;     // threads of the decide kernel (one bucket each)
constexpr int kRun = kDecideThreads * kSortItems;  // a segment or bucket sorted in LDS in one piece
constexpr int kSplitThreads = 1024;     // threads of the splitter kernel
constexpr int kSample = kSplitThreads * kSortItems;  // largest sample
constexpr int kBucketAvg = 768;         // average bucket of a split segment
constexpr int kMaxBuckets = 2048;       // buckets of one segment at most
constexpr int kOversample = 8;          // samples per bucket
constexpr int kChunk = 2048;            // events per workgroup while bucketing
constexpr int kSegMergeItems = 8;       // outputs per thread and step of a merge pass
constexpr int kOffThreads = 1024;       // threads of the offsets kernels

__host__ __device__ __forceinline__ int seg_buckets(int64_t m, int avg)
{
    if (m <= kRun) return 1;
    const int64_t p = (m + avg - 1) / avg;
    return p < kMaxBuckets ? (int)p : kMaxBuckets;
}

__host__ __device__ __forceinline__ int seg_chunks(int64_t m)
{
    return m <= kRun ? 0 : (int)((m + kChunk - 1) / kChunk);
}

// Grid bound of the bucketing passes: the sum over split blocks (fewer than
// 2n / kRun of them) of m / kChunk + 1.
int64_t seg_chunk_bound(int64_t n) { return 2 * n / kChunk + 2 * n / kRun + 2; }

// ----------------------------------------------------- workgroup sort --
//
// Ascending sort of kSortItems keys per thread, blocked (thread t holds
// positions t * kSortItems .. + kSortItems - 1). Each wave sorts its
// kWaveKeys keys with a bitonic network (partners less than kSortItems
// apart are in the same thread's registers, farther ones in the lane
// stride / kSortItems away, reached by a shuffle), then the waves' sorted
// runs are merged pairwise through LDS: each thread finds where its
// kSortItems outputs start by a binary search over the diagonal (merge
// path) and merges them sequentially.

__device__ __forceinline__ void wave_bitonic(uint64_t (&k)[kSortItems])
{
    const int lane = lane_id();
#pragma unroll
    for (int size = 2; size <= kWaveKeys; size <<= 1) {
#pragma unroll
        for (int stride = size >> 1; stride > 0; stride >>= 1) {
            if (stride >= kSortItems) {
                // all partners first (independent shuffles in flight together)
                const int lx = stride / kSortItems;
                uint64_t o[kSortItems];
#pragma unroll
                for (int j = 0; j < kSortItems; ++j) o[j] = __shfl_xor(k[j], lx);
                // stride and size are multiples of kSortItems here: the pair's
                // position bits come from the lane alone
                const int e = lane * kSortItems;
                const bool keep_min = ((e & stride) == 0) == ((e & size) == 0);
#pragma unroll
                for (int j = 0; j < kSortItems; ++j)
                    k[j] = ((k[j] < o[j]) == keep_min) ? k[j] : o[j];
            } else {
#pragma unroll
                for (int j = 0; j < kSortItems; ++j) {
                    if (j & stride) continue;
                    const int j2 = j | stride;
                    const bool asc = ((lane * kSortItems + j) & size) == 0;
                    const uint64_t a = k[j], b = k[j2];
                    const bool sw = (a > b) == asc;
                    k[j] = sw ? b : a;
                    k[j2] = sw ? a : b;
                }
            }
        }
    }
}

// live (uniform over the workgroup): only the first live positions hold
// keys that matter, the rest hold ~0; merging stops once one sorted run
// covers them.
template <int BLOCK>
__device__ __forceinline__ void block_sort_keys(uint64_t (&k)[kSortItems], uint64_t *lds,
                                                int64_t live = (int64_t)BLOCK * kSortItems)
{
    wave_bitonic(k);
    constexpr int N = BLOCK * kSortItems;
    const int d0 = (int)threadIdx.x * kSortItems;
#pragma unroll 1
    for (int r = kWaveKeys; r < N && r < live; r <<= 1) {
#pragma unroll
        for (int j = 0; j < kSortItems; ++j) lds[d0 + j] = k[j];
        __syncthreads();
        const int a0 = (d0 / (2 * r)) * (2 * r);
        const uint64_t *A = lds + a0;
        const uint64_t *Bv = lds + a0 + r;
        const int diag = d0 - a0;
        int lo = diag > r ? diag - r : 0;
        int hi = diag < r ? diag : r;
        while (lo < hi) {
            const int mid = (lo + hi) >> 1;
            if (A[mid] <= Bv[diag - 1 - mid]) lo = mid + 1;
            else hi = mid;
        }
        int ia = lo, ib = diag - lo;
        uint64_t va = ia < r ? A[ia] : ~0ull;
        uint64_t vb = ib < r ? Bv[ib] : ~0ull;
#pragma unroll
        for (int q = 0; q < kSortItems; ++q) {
            if (va <= vb) {
                k[q] = va;
                ++ia;
                va = ia < r ? A[ia] : ~0ull;
            } else {
                k[q] = vb;
                ++ib;
                vb = ib < r ? Bv[ib] : ~0ull;
            }
        }
        __syncthreads();
    }
}

// ------------------------------------------------------ counting sort --

struct SegGeom {
    int64_t span;  // nodes per workgroup (contiguous)
    int rows;      // workgroups
};

SegGeom seg_geom(int64_t n)
{
    SegGeom g;
    int64_t G = std::min<int64_t>(kSegRows, (n + kBlock - 1) / kBlock);
    if (G < 1) G = 1;
    g.span = (n + G - 1) / G;
    g.rows = (int)((n + g.span - 1) / g.span);
    return g;
}

constexpr int kNodeUnroll = 4;  // nodes per thread and step of the node passes

// Counter copies per block for the counting sort: with few blocks every
// workgroup would add to the same few addresses, so block B's count and
// cursor are split over C copies (workgroup w uses copy w mod C), laid out
// as the sub-ranges B * C + c of B's segment.
__host__ __device__ __forceinline__ int seg_copies(int K)
{
    int c = 1;
    while (c < 8 && (int64_t)K * c * 2 <= kSegCopyEntries) c <<= 1;
    return c;
}

// Counter of copy c of block B; with copies, each counter has a cache line
// of its own (atomics on one line are serialised).
__host__ __device__ __forceinline__ int64_t seg_slot(int B, int c, int C)
{
    return ((int64_t)B * C + c) * (C > 1 ? kSegCopyPad : 1);
}

// The eligible candidates among kNodeUnroll nodes v0 + u * kBlock (u <
// kNodeUnroll, below hi): inflow block T and own block A (global ids), or
// T = -1. The loads of the nodes are issued together.
__device__ __forceinline__ void seg_event_blocks(const int64_t *key, const int64_t *gp,
                                                 const int32_t *part, const uint8_t *avail,
                                                 const Blocks &bk, int K, int64_t v0, int64_t hi,
                                                 int64_t (&kv)[kNodeUnroll],
                                                 int32_t (&A)[kNodeUnroll],
                                                 int32_t (&T)[kNodeUnroll],
                                                 bool (&out)[kNodeUnroll])
{
    // every load from a clamped index and without a branch (gp and part of a
    // node that is no candidate are read and unused), so that all are in
    // flight together
    int64_t g4[kNodeUnroll];
    int32_t a4[kNodeUnroll];
#pragma unroll
    for (int u = 0; u < kNodeUnroll; ++u) {
        const int64_t v = v0 + (int64_t)u * kBlock;
        const int64_t vc = v < hi ? v : hi - 1;
        kv[u] = key[vc];
        g4[u] = gp[vc];
        a4[u] = part[vc];
        out[u] = avail[vc] == 0;  // an outflow event too (source not in V_r)
        if (v >= hi) kv[u] = -1;
    }
#pragma unroll
    for (int u = 0; u < kNodeUnroll; ++u) {
        T[u] = -1;
        A[u] = -1;
        if (kv[u] >= 0 && g4[u] > 0) {
            const int32_t a = a4[u];
            if ((unsigned)a < (unsigned)K) {
                const int32_t t = bk.base(a) + (int32_t)(kv[u] & 0xFFFF);
                if ((unsigned)t < (unsigned)K) {
                    A[u] = a;
                    T[u] = t;
                }
            }
        }
    }
}

// Node range and block window of this workgroup; zeroes the LDS counts if
// the window fits. Returns whether it does.
__device__ __forceinline__ bool seg_window(int64_t n, int64_t span, const Blocks &bk,
                                           const int64_t *goff, uint32_t *h, int32_t *win,
                                           int64_t *lo, int64_t *hi, int32_t *B0, int32_t *nb)
{
    *lo = (int64_t)blockIdx.x * span;
    *hi = *lo + span < n ? *lo + span : n;
    if (threadIdx.x == 0) node_block_window(bk, goff, *lo, *hi, &win[0], &win[1]);
    __syncthreads();
    *B0 = win[0];
    *nb = win[1];
    const bool lds = *nb <= kSegBins;
    if (lds)
        for (int j = threadIdx.x; j < *nb; j += kBlock) h[j] = 0;
    __syncthreads();
    return lds;
}

// Events per block into cnt (zeroed before).
__global__ __launch_bounds__(kBlock) void k_seg_count(int64_t n, int64_t span,
                                                      const int64_t *__restrict__ key,
                                                      const int64_t *__restrict__ gp,
                                                      const int32_t *__restrict__ part,
                                                      const uint8_t *__restrict__ avail, Blocks bk,
                                                      const int64_t *__restrict__ goff,
                                                      unsigned long long *cnt)
{
    __shared__ uint32_t h[kSegBins];
    __shared__ int32_t win[2];
    const int K = bk.total();
    const int C = seg_copies(K);
    const int copy = (int)blockIdx.x & (C - 1);
    int64_t lo, hi;
    int32_t B0, nb;
    const bool lds = seg_window(n, span, bk, goff, h, win, &lo, &hi, &B0, &nb);
    for (int64_t v0 = lo + threadIdx.x; v0 < hi; v0 += (int64_t)kNodeUnroll * kBlock) {
        int64_t kv[kNodeUnroll];
        int32_t A[kNodeUnroll], T[kNodeUnroll];
        bool out[kNodeUnroll];
        seg_event_blocks(key, gp, part, avail, bk, K, v0, hi, kv, A, T, out);
#pragma unroll
        for (int u = 0; u < kNodeUnroll; ++u) {
            if (T[u] < 0) continue;
            const uint32_t xt = (uint32_t)(T[u] - B0), xa = (uint32_t)(A[u] - B0);
            if (lds && xt < (uint32_t)nb) atomicAdd(&h[xt], 1u);
            else atomicAdd(&cnt[seg_slot(T[u], copy, C)], 1ull);
            if (out[u]) {
                if (lds && xa < (uint32_t)nb) atomicAdd(&h[xa], 1u);
                else atomicAdd(&cnt[seg_slot(A[u], copy, C)], 1ull);
            }
        }
    }
    __syncthreads();
    if (lds)
        for (int j = threadIdx.x; j < nb; j += kBlock)
            if (h[j]) atomicAdd(&cnt[seg_slot(B0 + j, copy, C)], (unsigned long long)h[j]);
}

// Exclusive scans over the 1024 threads: each wave scans its values, wave 0
// scans the 16 wave totals and publishes every wave's base and the total
// (kScanSlots entries of lds per scan), so that a thread holds one base
// rather than all 16 totals (with 1024 threads a thread has at most 128
// registers).
constexpr int kScanSlots = kOffThreads / 64 + 1;

__device__ __forceinline__ void scan_wave_totals(int64_t *lds)
{
    if ((threadIdx.x >> 6) == 0) {
        const int l = lane_id();
        const int64_t t = l < kScanSlots - 1 ? lds[l] : 0;
        const int64_t it = wave_incl_scan(t);
        if (l < kScanSlots - 1) lds[l] = it - t;
        if (l == kScanSlots - 2) lds[kScanSlots - 1] = it;
    }
}

__device__ __forceinline__ int64_t excl_scan_1024(int64_t x, int64_t *lds /* >= kScanSlots */,
                                                  int64_t *total)
{
    const int64_t inc = wave_incl_scan(x);
    const int w = threadIdx.x >> 6;
    __syncthreads();
    if (lane_id() == 63) lds[w] = inc;
    __syncthreads();
    scan_wave_totals(lds);
    __syncthreads();
    const int64_t base = lds[w];
    *total = lds[kScanSlots - 1];
    __syncthreads();
    return base + inc - x;
}

// Three exclusive scans at once (one set of barriers).
__device__ __forceinline__ void excl_scan3_1024(const int64_t (&x)[3], int64_t (&ex)[3],
                                                int64_t (&total)[3],
                                                int64_t *lds /* >= 3 * kScanSlots */)
{
    int64_t inc[3];
#pragma unroll
    for (int q = 0; q < 3; ++q) inc[q] = wave_incl_scan(x[q]);
    const int w = threadIdx.x >> 6;
    __syncthreads();
    if (lane_id() == 63)
#pragma unroll
        for (int q = 0; q < 3; ++q) lds[q * kScanSlots + w] = inc[q];
    __syncthreads();
#pragma unroll
    for (int q = 0; q < 3; ++q) scan_wave_totals(lds + q * kScanSlots);
    __syncthreads();
#pragma unroll
    for (int q = 0; q < 3; ++q) {
        ex[q] = lds[q * kScanSlots + w] + inc[q] - x[q];
        total[q] = lds[q * kScanSlots + kScanSlots - 1];
    }
    __syncthreads();
}

// Segment starts seg_off[0..K] (cur[B] becomes B's placement cursor). Then
// the buckets: boff[B] is B's first bucket (boff[K] buckets in all), cpre[B]
// the first bucketing chunk of a split block, slist the split blocks
// (meta[0] of them); a block that is not split is one bucket at its
// segment, a split block's buckets get zeroed accumulators. Up to kOffLds
// blocks, the offsets are also kept in LDS for the second pass.
constexpr int kOffLds = 2048;
__global__ __launch_bounds__(kOffThreads) void k_seg_offsets(int K, SegWs ws)
{
    __shared__ int64_t wtot[3 * kScanSlots];
    __shared__ int64_t s_off[kOffLds + 1];
    __shared__ int32_t s_boff[kOffLds + 1];
    const int t = threadIdx.x;
    const int C = seg_copies(K);
    const int KC = K * C;
    const bool lds = K <= kOffLds;
    int64_t carry = 0;
    for (int b0 = 0; b0 < KC; b0 += kOffThreads) {
        const int i = b0 + t;
        const int64_t slot = seg_slot(i / C, i & (C - 1), C);
        const int64_t x = i < KC ? (int64_t)ws.cur[slot] : 0;
        int64_t total;
        const int64_t ex = excl_scan_1024(x, wtot, &total);
        if (i < KC) {
            if ((i & (C - 1)) == 0) {
                ws.seg_off[i / C] = carry + ex;
                if (lds) s_off[i / C] = carry + ex;
            }
            ws.cur[slot] = (unsigned long long)(carry + ex);
        }
        carry += total;
    }
    if (t == 0) {
        ws.seg_off[K] = carry;
        if (lds) s_off[K] = carry;
    }
    __syncthreads();
    const int64_t *off = lds ? s_off : ws.seg_off;
    int64_t carry_p = 0, carry_q = 0, carry_s = 0;
    for (int b0 = 0; b0 < K; b0 += kOffThreads) {
        const int B = b0 + t;
        const int64_t m = B < K ? off[B + 1] - off[B] : 0;
        const int P = B < K ? seg_buckets(m, ws.bucket_avg) : 0;
        const int64_t x[3] = {P, B < K ? seg_chunks(m) : 0, P > 1 ? 1 : 0};
        int64_t ex[3], tot[3];
        excl_scan3_1024(x, ex, tot, wtot);
        if (B < K) {
            const int32_t f = (int32_t)(carry_p + ex[0]);
            ws.boff[B] = f;
            if (lds) s_boff[B] = f;
            ws.cpre[B] = (int32_t)(carry_q + ex[1]);
            if (P == 1) {
                ws.bblk[f] = B;
                ws.bpos[f] = off[B];
                ws.bsize[f] = m;
                ws.bdel[f] = 0;
            } else {
                ws.slist[carry_s + ex[2]] = B;
            }
        }
        carry_p += tot[0];
        carry_q += tot[1];
        carry_s += tot[2];
    }
    if (t == 0) {
        ws.boff[K] = (int32_t)carry_p;
        if (lds) s_boff[K] = (int32_t)carry_p;
        ws.cpre[K] = (int32_t)carry_q;
        ws.meta[0] = (int32_t)carry_s;
    }
    __syncthreads();
    // the buckets of split blocks, by all threads
    if (lds) {
        // one bucket per thread and step: its block is the last B with
        // boff[B] <= f (every block has at least one bucket)
        const int nbk = s_boff[K];
        for (int f = t; f < nbk; f += kOffThreads) {
            int lo = 0, hi = K - 1;
            while (lo < hi) {
                const int mid = (lo + hi + 1) >> 1;
                if (s_boff[mid] <= f) lo = mid;
                else hi = mid - 1;
            }
            if (s_boff[lo + 1] - s_boff[lo] > 1) {
                ws.bblk[f] = lo;
                ws.bcnt[f] = 0;
                ws.bdel[f] = 0;
            }
        }
        return;
    }
    for (int j = 0; j < (int)carry_s; ++j) {
        const int B = ws.slist[j];
        const int f = ws.boff[B], P = ws.boff[B + 1] - f;
        for (int i = t; i < P; i += kOffThreads) {
            ws.bblk[f + i] = B;
            ws.bcnt[f + i] = 0;
            ws.bdel[f + i] = 0;
        }
    }
}

// Each event's key, (order << (idb + 1)) | (v << 1) | outflow, at a free
// position of its block's segment (the order within a segment is
// irrelevant: the keys are distinct and are sorted next). The workgroup
// counts its events per block of its window, reserves each block's slots
// with one atomic, then hands them out in LDS.
__global__ __launch_bounds__(kBlock) void k_seg_place(int64_t n, int64_t span,
                                                      const int64_t *__restrict__ key,
                                                      const int64_t *__restrict__ gp,
                                                      const int32_t *__restrict__ part,
                                                      const uint8_t *__restrict__ avail, Blocks bk,
                                                      const int64_t *__restrict__ goff, SegWs ws,
                                                      int sb, int idb)
{
    __shared__ uint32_t h[kSegBins];
    __shared__ int32_t win[2];
    const int K = bk.total();
    const int C = seg_copies(K);
    const int copy = (int)blockIdx.x & (C - 1);
    int64_t lo, hi;
    int32_t B0, nb;
    const bool lds = seg_window(n, span, bk, goff, h, win, &lo, &hi, &B0, &nb);
    if (lds) {
        for (int64_t v0 = lo + threadIdx.x; v0 < hi; v0 += (int64_t)kNodeUnroll * kBlock) {
            int64_t kv[kNodeUnroll];
            int32_t A[kNodeUnroll], T[kNodeUnroll];
            bool out[kNodeUnroll];
            seg_event_blocks(key, gp, part, avail, bk, K, v0, hi, kv, A, T, out);
#pragma unroll
            for (int u = 0; u < kNodeUnroll; ++u) {
                if (T[u] < 0) continue;
                const uint32_t xt = (uint32_t)(T[u] - B0), xa = (uint32_t)(A[u] - B0);
                if (xt < (uint32_t)nb) atomicAdd(&h[xt], 1u);
                if (out[u] && xa < (uint32_t)nb) atomicAdd(&h[xa], 1u);
            }
        }
        __syncthreads();
        for (int j = threadIdx.x; j < nb; j += kBlock)
            if (h[j])
                h[j] = (uint32_t)atomicAdd(&ws.cur[seg_slot(B0 + j, copy, C)],
                                           (unsigned long long)h[j]);
        __syncthreads();
    }
    const uint64_t top = ((uint64_t)1 << sb) - 1;
    for (int64_t v0 = lo + threadIdx.x; v0 < hi; v0 += (int64_t)kNodeUnroll * kBlock) {
        int64_t kv[kNodeUnroll];
        int32_t A[kNodeUnroll], T[kNodeUnroll];
        bool out[kNodeUnroll];
        seg_event_blocks(key, gp, part, avail, bk, K, v0, hi, kv, A, T, out);
#pragma unroll
        for (int u = 0; u < kNodeUnroll; ++u) {
            if (T[u] < 0) continue;
            const int64_t v = v0 + (int64_t)u * kBlock;
            const uint64_t order = top - (uint64_t)(kv[u] >> 16);  // score desc
            const uint64_t kin = (order << (idb + 1)) | ((uint64_t)v << 1);
            const uint32_t xt = (uint32_t)(T[u] - B0), xa = (uint32_t)(A[u] - B0);
            const uint64_t pt = (lds && xt < (uint32_t)nb)
                                    ? (uint64_t)atomicAdd(&h[xt], 1u)
                                    : atomicAdd(&ws.cur[seg_slot(T[u], copy, C)], 1ull);
            ws.ev[pt] = kin;
            if (out[u]) {
                const uint64_t pa = (lds && xa < (uint32_t)nb)
                                        ? (uint64_t)atomicAdd(&h[xa], 1u)
                                        : atomicAdd(&ws.cur[seg_slot(A[u], copy, C)], 1ull);
                ws.ev[pa] = kin | 1ull;
            }
        }
    }
}

// ---------------------------------------------------------- buckets --

// Splitters of a split block: S keys sampled at evenly spaced positions of
// its segment (kOversample per bucket, at most kSample), sorted; splitter i
// (1 <= i < P) is sample i * S / P.
__global__ __launch_bounds__(kSplitThreads) void k_seg_split(SegWs ws)
{
    __shared__ uint64_t lds[kSample];
    if ((int)blockIdx.x >= ws.meta[0]) return;  // uniform over the workgroup
    const int B = ws.slist[blockIdx.x];
    const int f = ws.boff[B], P = ws.boff[B + 1] - f;
    const int64_t s0 = ws.seg_off[B], m = ws.seg_off[B + 1] - s0;
    int64_t S = (int64_t)P * kOversample;
    if (S > kSample) S = kSample;
    if (S > m) S = m;
    uint64_t k[kSortItems];
#pragma unroll
    for (int j = 0; j < kSortItems; ++j) {
        const int64_t idx = (int64_t)threadIdx.x * kSortItems + j;
        const uint64_t x = ws.ev[s0 + ((idx < S ? idx : S - 1) * m) / S];  // clamped: no load in a branch
        k[j] = idx < S ? x : ~0ull;
    }
    // the S samples fill the first positions: the runs past them stay ~0
    block_sort_keys<kSplitThreads>(k, lds, S);
#pragma unroll
    for (int j = 0; j < kSortItems; ++j) lds[threadIdx.x * kSortItems + j] = k[j];
    __syncthreads();
    for (int i = 1 + threadIdx.x; i < P; i += kSplitThreads)
        ws.spl[f + i - 1] = lds[((int64_t)i * S) / P];
}

// Bucket of a key: the number of splitters not above it.
__device__ __forceinline__ int bucket_of(const uint64_t *sp, int ns, uint64_t key)
{
    int lo = 0, hi = ns;
    while (lo < hi) {
        const int mid = (lo + hi) >> 1;
        if (sp[mid] <= key) lo = mid + 1;
        else hi = mid;
    }
    return lo;
}

// One chunk of a split block's segment per workgroup: count its events per
// bucket and sum their weight changes (PLACE false), or scatter them into
// the buckets at the cursors (PLACE true).
template <bool PLACE>
__global__ __launch_bounds__(kBlock) void k_seg_bucket(GraphView g, int K, SegWs ws, int idb)
{
    constexpr int kPer = kChunk / kBlock;
    __shared__ uint64_t ssp[kMaxBuckets];
    __shared__ uint32_t hcnt[kMaxBuckets];
    __shared__ int64_t hdel[PLACE ? 1 : kMaxBuckets];
    const int j = blockIdx.x;
    if (j >= ws.cpre[K]) return;  // uniform over the workgroup
    const int B = upper_index(ws.cpre, K, j);
    const int c = j - ws.cpre[B];
    const int64_t s0 = ws.seg_off[B], m = ws.seg_off[B + 1] - s0;
    const int f = ws.boff[B], P = ws.boff[B + 1] - f;
    const int64_t lo = (int64_t)c * kChunk;
    for (int i = threadIdx.x; i < P - 1; i += kBlock) ssp[i] = ws.spl[f + i];
    for (int i = threadIdx.x; i < P; i += kBlock) {
        hcnt[i] = 0;
        if (!PLACE) hdel[i] = 0;
    }
    uint64_t key[kPer];
#pragma unroll
    for (int u = 0; u < kPer; ++u) {
        const int64_t p = lo + threadIdx.x + (int64_t)u * kBlock;
        const uint64_t x = ws.ev[s0 + (p < m ? p : m - 1)];  // clamped: no load in a branch
        key[u] = p < m ? x : ~0ull;
    }
    __syncthreads();
    const uint64_t idmask = ((uint64_t)1 << idb) - 1;
    int bk[kPer];
#pragma unroll
    for (int u = 0; u < kPer; ++u) {
        bk[u] = -1;
        if (lo + threadIdx.x + (int64_t)u * kBlock < m) {
            bk[u] = bucket_of(ssp, P - 1, key[u]);
            if (!PLACE) {
                atomicAdd(&hcnt[bk[u]], 1u);
                const int64_t cv = node_weight(g, (int64_t)((key[u] >> 1) & idmask));
                atomicAdd((unsigned long long *)&hdel[bk[u]],
                          (unsigned long long)((key[u] & 1ull) ? -cv : cv));
            } else {
                atomicAdd(&hcnt[bk[u]], 1u);
            }
        }
    }
    __syncthreads();
    if (!PLACE) {
        for (int i = threadIdx.x; i < P; i += kBlock)
            if (hcnt[i]) {
                atomicAdd(&ws.bcnt[f + i], (unsigned long long)hcnt[i]);
                atomic_add_i64(&ws.bdel[f + i], hdel[i]);
            }
        return;
    }
    for (int i = threadIdx.x; i < P; i += kBlock)
        if (hcnt[i]) hcnt[i] = (uint32_t)atomicAdd(&ws.bcnt[f + i], (unsigned long long)hcnt[i]);
    __syncthreads();
#pragma unroll
    for (int u = 0; u < kPer; ++u)
        if (bk[u] >= 0) ws.tmp[atomicAdd(&hcnt[bk[u]], 1u)] = key[u];
}

// Buckets of split blocks: start (segment start plus the sizes of the
// block's earlier buckets), size, carry (the weight change of the block's
// earlier buckets), and the placement cursor.
__global__ __launch_bounds__(kOffThreads) void k_seg_boffsets(int K, SegWs ws)
{
    __shared__ int64_t wtot[kScanSlots];
    const int NB = ws.boff[K];
    const int t = threadIdx.x;
    int64_t cc = 0, cd = 0;
    for (int i0 = 0; i0 < NB; i0 += kOffThreads) {
        const int i = i0 + t;
        bool split = false;
        if (i < NB) {
            const int B = ws.bblk[i];
            split = ws.boff[B + 1] - ws.boff[B] > 1;
        }
        const int64_t x = split ? (int64_t)ws.bcnt[i] : 0;
        const int64_t y = split ? ws.bdel[i] : 0;
        int64_t tx, ty;
        const int64_t ex = excl_scan_1024(x, wtot, &tx);
        const int64_t ey = excl_scan_1024(y, wtot, &ty);
        if (i < NB) {
            ws.scan_c[i] = cc + ex;
            ws.scan_d[i] = cd + ey;
        }
        cc += tx;
        cd += ty;
    }
    __syncthreads();
    for (int i = t; i < NB; i += kOffThreads) {
        const int B = ws.bblk[i];
        const int f = ws.boff[B];
        if (ws.boff[B + 1] - f <= 1) continue;
        const int64_t pos = ws.seg_off[B] + ws.scan_c[i] - ws.scan_c[f];
        ws.bsize[i] = (int64_t)ws.bcnt[i];
        ws.bpos[i] = pos;
        ws.bdel[i] = ws.scan_d[i] - ws.scan_d[f];
        ws.bcnt[i] = (unsigned long long)pos;
    }
}

// ----------------------------------------------------------- decide --

// What the decision of an inflow event into block B needs.
struct SegDecide {
    GraphView g;
    int32_t B;
    int mode;
    int64_t WB;           // W[B]
    int64_t move_lmax;    // the fill limit of B's graph
    const int64_t *cbB;   // B's slot prefix sums
    const int64_t *penB;  // the penalty table of B's graph
    uint64_t idmask;
    const int64_t *gp;
    int64_t hub_t;
    int32_t *mvto;
    uint8_t *accflag;
};

// The move of v into B, priced against W[B] plus the weight change of the
// events before it (netpre); returns whether it is taken.
__device__ __forceinline__ bool seg_decide_one(const SegDecide &d, int64_t v, int64_t cv,
                                               int64_t gv, int64_t netpre)
{
    bool allowed = gv > 0;
    int64_t P = 0;
    const int64_t x = d.WB + netpre + cv - d.move_lmax;
    if (allowed && x > 0) {
        if (d.mode == 1 || d.mode == 3) allowed = false;
        else if (d.mode == 0) {
            const int l = covering_slot(d.cbB, x);
            if (l >= kSlots) allowed = false;
            else P = sat_mul_pen(d.penB[l], cv);
        }
    }
    const bool take = allowed && gv * 65536 - P > 0;
    d.accflag[v] = take ? 1 : 0;
    if (take) d.mvto[v] = d.B;
    return take;
}

// Scan and decide the IPT sorted keys of each thread (blocked: the
// thread's first key is at position pos0 of the bucket); carry is the
// weight change of the positions before this piece.
template <int IPT>
__device__ __forceinline__ void seg_scan_decide(const uint64_t (&k)[IPT], int64_t pos0,
                                                int64_t m, int64_t &carry, const SegDecide &d,
                                                int64_t *scan_lds, unsigned long long *acc_lds,
                                                unsigned long long *deg_lds)
{
    // the events' node weights, the inflow events' pessimistic gains and
    // degrees (for the moved-degree count), loaded together (node 0 stands in
    // for the slots past the bucket's end, whose keys hold no node id), so
    // that the decisions below wait on no load
    int64_t w[IPT], gv[IPT], cw[IPT], dg[IPT];
    int64_t vs[IPT];
#pragma unroll
    for (int j = 0; j < IPT; ++j) vs[j] = pos0 + j < m ? (int64_t)((k[j] >> 1) & d.idmask) : 0;
    if (d.g.vwgt) {  // uniform: the two forms keep their loads together
#pragma unroll
        for (int j = 0; j < IPT; ++j) {
            gv[j] = d.gp[vs[j]];
            cw[j] = d.g.vwgt[vs[j]];
            dg[j] = d.g.xadj[vs[j] + 1] - d.g.xadj[vs[j]];
        }
    } else {
#pragma unroll
        for (int j = 0; j < IPT; ++j) {
            gv[j] = d.gp[vs[j]];
            cw[j] = 1;
            dg[j] = d.g.xadj[vs[j] + 1] - d.g.xadj[vs[j]];
        }
    }
    int64_t ts = 0;
#pragma unroll
    for (int j = 0; j < IPT; ++j) {
        const bool ok = pos0 + j < m;
        w[j] = ok ? ((k[j] & 1ull) ? -cw[j] : cw[j]) : 0;
        gv[j] = (ok && !(k[j] & 1ull)) ? gv[j] : 0;
        ts += w[j];
    }
    int64_t total;
    const int64_t inc = block_incl_scan<int64_t, kDecideThreads / 64>(ts, scan_lds, &total);
    int64_t run = carry + inc - ts;
    unsigned long long nacc = 0, ndeg = 0;
#pragma unroll
    for (int j = 0; j < IPT; ++j) {
        if (pos0 + j < m && !(k[j] & 1ull) &&
            seg_decide_one(d, (int64_t)((k[j] >> 1) & d.idmask), w[j], gv[j], run)) {
            ++nacc;
            ndeg += (unsigned long long)dg[j];
        }
        run += w[j];
    }
    // one LDS atomic per wave for each count
    nacc = wave_sum(nacc);
    ndeg = wave_sum(ndeg);
    if (lane_id() == 0 && nacc) {
        atomicAdd(acc_lds, nacc);
        atomicAdd(deg_lds, ndeg);
    }
    carry += total;
}

// One workgroup per bucket: sort it, scan the weight changes from the
// bucket's carry, decide the inflow events. Up to 2 kRun keys the two
// halves are sorted in turn into LDS and merged there (merge path, the
// merged order in two pieces of kSortItems outputs per thread); a larger
// bucket is sorted in runs of kRun and merged pairwise through the other
// buffer (merge path over global memory, kSegMergeItems outputs per thread
// and step).
// k[j] = src[pos0 + j] below m, else the largest key (m >= 1): loads from
// clamped indices without a branch, so that all are in flight together.
__device__ __forceinline__ void seg_load_keys(uint64_t (&k)[kSortItems], const uint64_t *src,
                                              int64_t pos0, int64_t m)
{
#pragma unroll
    for (int j = 0; j < kSortItems; ++j) {
        const int64_t p = pos0 + j;
        const uint64_t x = src[p < m ? p : m - 1];
        k[j] = p < m ? x : ~0ull;
    }
}

__global__ __launch_bounds__(kDecideThreads) void k_seg_decide(GraphView g, Blocks bk, SegWs ws,
                                                               int idb,
                                                       const int64_t *__restrict__ gp,
                                                       const int64_t *__restrict__ W,
                                                       const int64_t *__restrict__ cb, int mode,
                                                       int64_t hub_t, int32_t *mvto,
                                                       uint8_t *accflag,
                                                       unsigned long long *counters)
{
    __shared__ uint64_t lds[2 * kRun];
    __shared__ int64_t scan_lds[kDecideThreads / 64];
    __shared__ int64_t s_cb[kSlots], s_pen[kSlots];
    __shared__ unsigned long long acc_lds, deg_lds;
    const int K = bk.total();
    const int i = blockIdx.x;
    if (i >= ws.boff[K]) return;  // uniform over the workgroup
    const int32_t B = ws.bblk[i];
    const bool split = ws.boff[B + 1] - ws.boff[B] > 1;
    const int64_t m = ws.bsize[i];
    if (m <= 0) return;
    const int64_t s0 = ws.bpos[i];
    int64_t carry = split ? ws.bdel[i] : 0;
    if (threadIdx.x == 0) {
        acc_lds = 0;
        deg_lds = 0;
    }
    // the block's slot prefix sums and penalty table (the price search reads them per event)
    if (threadIdx.x < kSlots) {
        s_cb[threadIdx.x] = cb[(int64_t)B * kSlots + threadIdx.x];
        s_pen[threadIdx.x] = bk.penq_of(B)[threadIdx.x];
    }
    __syncthreads();
    SegDecide d;
    d.g = g;
    d.B = B;
    d.mode = mode;
    d.WB = W[B];
    d.move_lmax = bk.move_lmax_of(B);
    d.cbB = s_cb;
    d.penB = s_pen;
    d.idmask = ((uint64_t)1 << idb) - 1;
    d.gp = gp;
    d.hub_t = hub_t;
    d.mvto = mvto;
    d.accflag = accflag;
    uint64_t *src = (split ? ws.tmp : ws.ev) + s0;
    uint64_t k[kSortItems];
    if (m <= kRun) {
        const int64_t pos0 = (int64_t)threadIdx.x * kSortItems;
        seg_load_keys(k, src, pos0, m);
        block_sort_keys<kDecideThreads>(k, lds, m);
        seg_scan_decide<kSortItems>(k, pos0, m, carry, d, scan_lds, &acc_lds, &deg_lds);
    } else if (m <= 2 * kRun) {
        // each half sorted with the upper half of the buffer as scratch, then
        // stored; the second half's sort leaves the first half untouched
        for (int hf = 0; hf < 2; ++hf) {
            const int64_t pos0 = (int64_t)hf * kRun + (int64_t)threadIdx.x * kSortItems;
            seg_load_keys(k, src, pos0, m);
            block_sort_keys<kDecideThreads>(k, lds + kRun, hf == 0 ? (int64_t)kRun : m - kRun);
#pragma unroll
            for (int j = 0; j < kSortItems; ++j) lds[pos0 + j] = k[j];
            __syncthreads();
        }
        // the merged order in two pieces: outputs [0, kRun), then [kRun, 2 kRun),
        // kSortItems consecutive ones per thread (blocked) in each
        const uint64_t *A = lds, *Bv = lds + kRun;
        for (int hf = 0; hf < 2; ++hf) {
            const int diag = hf * kRun + (int)threadIdx.x * kSortItems;
            int lo = diag > kRun ? diag - kRun : 0;
            int hi = diag < kRun ? diag : kRun;
            while (lo < hi) {
                const int mid = (lo + hi) >> 1;
                if (A[mid] <= Bv[diag - 1 - mid]) lo = mid + 1;
                else hi = mid;
            }
            int ia = lo, ib = diag - lo;
            uint64_t va = ia < kRun ? A[ia] : ~0ull;
            uint64_t vb = ib < kRun ? Bv[ib] : ~0ull;
#pragma unroll
            for (int q = 0; q < kSortItems; ++q) {
                if (va <= vb) {
                    k[q] = va;
                    ++ia;
                    va = ia < kRun ? A[ia] : ~0ull;
                } else {
                    k[q] = vb;
                    ++ib;
                    vb = ib < kRun ? Bv[ib] : ~0ull;
                }
            }
            seg_scan_decide<kSortItems>(k, diag, m, carry, d, scan_lds, &acc_lds, &deg_lds);
        }
    } else {
        uint64_t *dst = (split ? ws.ev : ws.tmp) + s0;
        // sorted runs
        for (int64_t r0 = 0; r0 < m; r0 += kRun) {
            const int64_t pos0 = r0 + (int64_t)threadIdx.x * kSortItems;
            seg_load_keys(k, src, pos0, m);
            block_sort_keys<kDecideThreads>(k, lds, m - r0 < kRun ? m - r0 : (int64_t)kRun);
#pragma unroll
            for (int j = 0; j < kSortItems; ++j)
                if (pos0 + j < m) src[pos0 + j] = k[j];
            __syncthreads();
        }
        // pairwise merges of runs of width w
        for (int64_t w = kRun; w < m; w <<= 1) {
            for (int64_t o0 = 0; o0 < m; o0 += (int64_t)kDecideThreads * kSegMergeItems) {
                const int64_t d0 = o0 + (int64_t)threadIdx.x * kSegMergeItems;
                if (d0 >= m) continue;
                const int64_t a0 = (d0 / (2 * w)) * (2 * w);
                const int64_t a1 = a0 + w < m ? a0 + w : m;
                const int64_t b1 = a1 + w < m ? a1 + w : m;
                const int64_t la = a1 - a0, lb = b1 - a1, diag = d0 - a0;
                int64_t lo = diag - lb > 0 ? diag - lb : 0;
                int64_t hi = diag < la ? diag : la;
                while (lo < hi) {
                    const int64_t mid = (lo + hi) >> 1;
                    if (src[a0 + mid] <= src[a1 + diag - 1 - mid]) lo = mid + 1;
                    else hi = mid;
                }
                int64_t ia = lo, ib = diag - lo;
                for (int q = 0; q < kSegMergeItems && d0 + q < b1; ++q) {
                    const bool ta = ia < la && (ib >= lb || src[a0 + ia] <= src[a1 + ib]);
                    dst[d0 + q] = ta ? src[a0 + ia++] : src[a1 + ib++];
                }
            }
            __syncthreads();
            uint64_t *t = src;
            src = dst;
            dst = t;
        }
        // scan and decide in pieces of kRun
        for (int64_t r0 = 0; r0 < m; r0 += kRun) {
            const int64_t pos0 = r0 + (int64_t)threadIdx.x * kSortItems;
            seg_load_keys(k, src, pos0, m);
            seg_scan_decide<kSortItems>(k, pos0, m, carry, d, scan_lds, &acc_lds, &deg_lds);
        }
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        if (acc_lds) cnt_add(counters, CNT_ACC, acc_lds);
        if (deg_lds) cnt_add(counters, CNT_MOVED_DEG, deg_lds);
    }
}

}  // namespace

int seq_id_bits(int64_t n)
{
    return bit_width((uint64_t)(n > 1 ? n - 1 : 1));
}

// Keys stay below 2^63, so the all-ones padding of the sorts sorts last.
bool seq_segments_fit(int sb, int64_t n)
{
    return sb + seq_id_bits(n) + 1 <= 63;
}

int64_t seq_counter_words(int K)
{
    return seg_slot(K, 0, seg_copies(K));
}

int seq_bucket_avg_min() { return kBucketAvg; }

int64_t seq_bucket_bound(int64_t n, int K)
{
    return (int64_t)K + 2 * n / kBucketAvg + 2 * n / kRun + 2;
}

hipError_t launch_seq_segments(const GraphView &g, const Blocks &bk, const int64_t *goff,
                               const int64_t *key, const int64_t *gp, const int32_t *part,
                               const uint8_t *avail, int sb, const SegWs &ws, const int64_t *W,
                               const int64_t *cb, int mode, int64_t hub_t, int32_t *mvto,
                               uint8_t *accflag, unsigned long long *counters, hipStream_t s)
{
    if (g.n <= 0) return hipSuccess;
    const int K = bk.total();
    const int idb = seq_id_bits(g.n);
    const SegGeom geo = seg_geom(g.n);
    hipError_t e;
    hipLaunchKernelGGL(k_seg_count, dim3(geo.rows), dim3(kBlock), 0, s, g.n, geo.span, key, gp,
                       part, avail, bk, goff, ws.cur);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    hipLaunchKernelGGL(k_seg_offsets, dim3(1), dim3(kOffThreads), 0, s, K, ws);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    hipLaunchKernelGGL(k_seg_place, dim3(geo.rows), dim3(kBlock), 0, s, g.n, geo.span, key, gp,
                       part, avail, bk, goff, ws, sb, idb);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    // split blocks hold more than kRun events each
    const int64_t splits = std::min<int64_t>(K, 2 * g.n / kRun + 1);
    hipLaunchKernelGGL(k_seg_split, dim3((unsigned)splits), dim3(kSplitThreads), 0, s, ws);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    const unsigned chunks = (unsigned)seg_chunk_bound(g.n);
    hipLaunchKernelGGL(k_seg_bucket<false>, dim3(chunks), dim3(kBlock), 0, s, g, K, ws, idb);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    hipLaunchKernelGGL(k_seg_boffsets, dim3(1), dim3(kOffThreads), 0, s, K, ws);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    hipLaunchKernelGGL(k_seg_bucket<true>, dim3(chunks), dim3(kBlock), 0, s, g, K, ws, idb);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    hipLaunchKernelGGL(k_seg_decide, dim3((unsigned)seq_bucket_bound(g.n, K)), dim3(kDecideThreads), 0, s,
                       g, bk, ws, idb, gp, W, cb, mode, hub_t, mvto, accflag, counters);
    return hipGetLastError();
}

}  // namespace upr
