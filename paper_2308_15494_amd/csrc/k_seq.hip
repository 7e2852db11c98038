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
// Each eligible candidate v emits two events: (target(v), +c(v)) and, if v
// is not available, (part(v), -c(v)); both carry v's order key. Events are
// sorted by (block, score desc) with a stable radix sort over an id-ordered
// input, so equal scores stay in id order; an exclusive scan by block gives,
// at v's inflow event, the weight change of v's target before v.
#include "upr_common.h"

#include <cstring>

#include <rocprim/rocprim.hpp>

namespace upr {

namespace {

constexpr int kBlockBits = 14;                        // block id or the sentinel 8192
constexpr uint64_t kSentinel = (uint64_t)8192 << 47;  // events of ineligible candidates

struct IsCandidate {
    const int64_t *key;
    __host__ __device__ bool operator()(int32_t v) const { return key[v] >= 0; }
};

struct EventBlock {
    __host__ __device__ uint32_t operator()(uint64_t k) const { return (uint32_t)(k >> 47); }
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

__global__ void k_seq_events(int64_t nc, const int32_t *cand, const int64_t *key,
                             const int32_t *part, const int64_t *gp, const uint8_t *avail,
                             uint64_t *ev_key, uint32_t *ev_val)
{
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < nc; i += stride) {
        const int32_t v = cand[i];
        const int64_t kv = key[v];
        const uint64_t order = ((uint64_t)1 << 47) - 1 - (uint64_t)(kv >> 16);  // score desc
        const bool eligible = gp[v] > 0;
        const uint64_t b = (uint64_t)(kv & 0xFFFF);
        const uint64_t a = (uint64_t)part[v];
        ev_key[2 * i] = eligible ? ((b << 47) | order) : kSentinel;
        ev_val[2 * i] = ((uint32_t)v << 1);
        ev_key[2 * i + 1] = (eligible && !avail[v]) ? ((a << 47) | order) : kSentinel;
        ev_val[2 * i + 1] = ((uint32_t)v << 1) | 1u;
    }
}

__global__ void k_seq_scatter(int64_t ne, const uint64_t *ev_key, const uint32_t *ev_val,
                              const int64_t *prefix, int64_t *netpre)
{
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < ne; i += stride) {
        const uint32_t ev = ev_val[i];
        if ((ev & 1u) == 0 && ev_key[i] != kSentinel) netpre[ev >> 1] = prefix[i];
    }
}

int grid_for(int64_t items)
{
    int64_t g = (items + kBlock - 1) / kBlock;
    if (g < 1) g = 1;
    if (g > 8192) g = 8192;
    return (int)g;
}

}  // namespace

size_t seq_temp_bytes(int64_t n)
{
    if (n <= 0) return 16;
    size_t a = 0, b = 0, c = 0;
    const int64_t *key = nullptr;
    int32_t *out = nullptr;
    int32_t *cnt = nullptr;
    rocprim::select(nullptr, a, rocprim::counting_iterator<int32_t>(0), out, cnt, (size_t)n,
                    IsCandidate{key}, (hipStream_t)0);
    uint64_t *k0 = nullptr, *k1 = nullptr;
    uint32_t *v0 = nullptr, *v1 = nullptr;
    rocprim::radix_sort_pairs(nullptr, b, k0, k1, v0, v1, (size_t)(2 * n), 0, 47 + kBlockBits,
                              (hipStream_t)0);
    int64_t *pre = nullptr;
    rocprim::exclusive_scan_by_key(
        nullptr, c, rocprim::make_transform_iterator(k1, EventBlock{}),
        rocprim::make_transform_iterator(v1, EventDelta{nullptr}), pre, (int64_t)0,
        (size_t)(2 * n), rocprim::plus<int64_t>(), rocprim::equal_to<uint32_t>(), (hipStream_t)0);
    return std::max(a, std::max(b, c)) + 256;
}

hipError_t launch_seq_select(int64_t n, const int64_t *key, int32_t *cand, int32_t *count,
                             void *temp, size_t temp_bytes, hipStream_t s)
{
    size_t bytes = temp_bytes;
    return rocprim::select(temp, bytes, rocprim::counting_iterator<int32_t>(0), cand, count,
                           (size_t)n, IsCandidate{key}, s);
}

hipError_t launch_seq_net(int64_t nc, const int32_t *cand, const int64_t *key, const int32_t *part,
                          const int32_t *vwgt, const int64_t *gp, const uint8_t *avail,
                          uint64_t *ev_key, uint64_t *ev_key2, uint32_t *ev_val,
                          uint32_t *ev_val2, int64_t *prefix, int64_t *netpre, void *temp,
                          size_t temp_bytes, hipStream_t s)
{
    if (nc <= 0) return hipSuccess;
    const int64_t ne = 2 * nc;
    hipLaunchKernelGGL(k_seq_events, dim3(grid_for(nc)), dim3(kBlock), 0, s, nc, cand, key, part, gp,
                       avail, ev_key, ev_val);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    size_t bytes = temp_bytes;
    e = rocprim::radix_sort_pairs(temp, bytes, ev_key, ev_key2, ev_val, ev_val2, (size_t)ne, 0,
                                  47 + kBlockBits, s);
    if (e != hipSuccess) return e;
    bytes = temp_bytes;
    e = rocprim::exclusive_scan_by_key(
        temp, bytes, rocprim::make_transform_iterator(ev_key2, EventBlock{}),
        rocprim::make_transform_iterator(ev_val2, EventDelta{vwgt}), prefix, (int64_t)0,
        (size_t)ne, rocprim::plus<int64_t>(), rocprim::equal_to<uint32_t>(), s);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_seq_scatter, dim3(grid_for(ne)), dim3(kBlock), 0, s, ne, ev_key2, ev_val2,
                       prefix, netpre);
    return hipGetLastError();
}

}  // namespace upr
