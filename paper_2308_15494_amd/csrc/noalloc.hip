// Edge cut without any device allocation, for callers that cannot allocate
// (work under HIP graph capture, tight serving loops, harnesses that forbid
// hipMalloc). The cut is the Section 2 objective, the total weight of the
// edges whose ends lie in different blocks, taken straight from the
// adjacency as upr_edge_cut does.
//
// Its scratch memory is a file-scope device array of kNoallocTiles partial
// sums, one per tile of kNoallocTileNodes consecutive nodes (2 MiB, so at
// most 2^28 nodes). Every device the library runs on holds its own copy
// until the process ends. Host code never names the array in a launch or a
// copy: the array's host-side symbol is only a stand-in, so its device
// address is taken once per device, with that device current, by
// hipGetSymbolAddress (noalloc_init, called by upr_create), and the kernels
// get that address as an argument.
//
// Two passes on the caller's stream: each tile's workgroup overwrites its
// own partial sum (no slot has to start at zero, and slots past the last
// tile are never read), then one workgroup sums the partials. Calls that
// overlap on one device share the array and race.
#include "upr.h"
#include "upr_common.h"

#include <mutex>

namespace upr {

namespace {

constexpr int kNoallocTileNodes = 1024;
constexpr int64_t kNoallocTiles = int64_t(1) << 18;
constexpr int kNoallocSumThreads = 1024;
constexpr int kMaxDevices = 64;
static_assert(kNoallocTiles * kNoallocTileNodes == UPR_NOALLOC_MAX_NODES,
              "the header's node limit is the scratch capacity");

static __device__ __align__(256) unsigned long long scratch[kNoallocTiles];

std::mutex g_mu;
void *g_ptr[kMaxDevices] = {};

// One workgroup per tile: the tile's node offsets and blocks go to LDS, its
// edges are spread over the threads (each finds its row by a binary search
// over the tile's offsets) and every edge into another block adds its
// weight. The sum (twice the tile's share of the cut) overwrites the tile's
// slot of the scratch array.
__global__ __launch_bounds__(kBlock) void k_cut_tiles(GraphView g, const int32_t *__restrict__ part,
                                                      unsigned long long *partial)
{
    __shared__ int64_t s_off[kNoallocTileNodes + 1];
    __shared__ int32_t s_part[kNoallocTileNodes];
    __shared__ unsigned long long red[4];
    const int64_t v0 = (int64_t)blockIdx.x * kNoallocTileNodes;
    const int nt = (int)min<int64_t>(kNoallocTileNodes, g.n - v0);
    for (int i = threadIdx.x; i <= nt; i += kBlock) s_off[i] = g.xadj[v0 + i];
    for (int i = threadIdx.x; i < nt; i += kBlock) s_part[i] = part[v0 + i];
    __syncthreads();
    const int64_t e0 = s_off[0], e1 = s_off[nt];
    unsigned long long sum = 0;
    for (int64_t e = e0 + threadIdx.x; e < e1; e += kBlock) {
        // row of edge e: the last i with s_off[i] <= e
        int lo = 0, hi = nt - 1;
        while (lo < hi) {
            const int mid = (lo + hi + 1) >> 1;
            if (s_off[mid] <= e) lo = mid;
            else hi = mid - 1;
        }
        if (part[g.adjncy[e]] != s_part[lo]) sum += (unsigned long long)edge_weight(g, e);
    }
    sum = block_sum(sum, red);
    if (threadIdx.x == 0) partial[blockIdx.x] = sum;
}

// One workgroup: cut = (sum of the tiles' partial sums) / 2.
__global__ __launch_bounds__(kNoallocSumThreads) void k_cut_total(const unsigned long long *partial,
                                                                  int64_t tiles, int64_t *cut)
{
    __shared__ unsigned long long red[kNoallocSumThreads / 64];
    unsigned long long s = 0;
    for (int64_t t = threadIdx.x; t < tiles; t += kNoallocSumThreads) s += partial[t];
    s = wave_sum(s);
    if (lane_id() == 0) red[threadIdx.x >> 6] = s;
    __syncthreads();
    if (threadIdx.x == 0) {
        unsigned long long tot = 0;
        for (int w = 0; w < kNoallocSumThreads / 64; ++w) tot += red[w];
        cut[0] = (int64_t)(tot / 2);
    }
}

}  // namespace

hipError_t noalloc_init(int device, void **ptr)
{
    if (device < 0 || device >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(g_mu);
    if (!g_ptr[device]) {
        // the caller made `device` current
        void *p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        g_ptr[device] = p;
    }
    *ptr = g_ptr[device];
    return hipSuccess;
}

hipError_t launch_cut_noalloc(const GraphView &g, const int32_t *part, int64_t *cut,
                              void *scratch_ptr, hipStream_t s)
{
    unsigned long long *partial = (unsigned long long *)scratch_ptr;
    const int64_t tiles = (g.n + kNoallocTileNodes - 1) / kNoallocTileNodes;
    if (tiles > 0)
        hipLaunchKernelGGL(k_cut_tiles, dim3((unsigned)tiles), dim3(kBlock), 0, s, g, part, partial);
    hipLaunchKernelGGL(k_cut_total, dim3(1), dim3(kNoallocSumThreads), 0, s, partial, tiles, cut);
    return hipGetLastError();
}

}  // namespace upr
