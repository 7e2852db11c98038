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

}  // namespace upr
