// Rebalancing (Section 7.1), one synchronous sub-iteration per call of
// launch_rb_iteration.
//
// The paper's rebalancer pops nodes of overloaded blocks from a relaxed
// concurrent priority queue. Here the same priorities are bucketed and the
// order "bucket, then node id" is realised without sorting:
//   prepare   every node of an overloaded block picks its best-gain target
//             among blocks that stay balanced (or the lightest such block if
//             it is connected to none) and its priority bucket, and offers
//             itself: per target a histogram of offered weight over buckets
//   target    the cutoff bucket is the first whose cumulative weight exceeds
//             the target's capacity; inside it, chunk sums over id ranges and
//             a scan of one chunk give the id bound of the maximal prefix
//             that fits
//   source    the same over each overloaded block's accepted nodes: the
//             minimal prefix that covers the block's excess is kept
//   moves     kept nodes are marked (mvto) for the apply kernels
// Blocks are global ids (a batch's graphs have disjoint blocks); a node's row
// is indexed by its local block. A block is a source iff its weight exceeds
// src_lmax of its graph (L_max, or "never" once that graph has stopped);
// targets must stay within L_max.
// Histogram rows and chunk rows are cleared by the kernel that reads them,
// so they are zero again at the start of the next sub-iteration. Node scans
// run over all ids in wave-sized runs; membership of a node in an overloaded
// block is re-derived from part and the sub-iteration's starting weights.
#include "upr_common.h"

namespace upr {

static int grid_cap(int64_t items, int per_block, int cap)
{
    int64_t g = (items + per_block - 1) / per_block;
    if (g < 1) g = 1;
    if (g > cap) g = cap;
    return (int)g;
}

struct RbView {
    const int32_t *rtgt;
    const uint8_t *rbeta;
    const int64_t *W0;
    const int32_t *cbeta_src;
    const int32_t *theta_src;
    const int32_t *cbeta_tgt;
    const int32_t *theta_tgt;
};

// Accepted by its target j (offers are ordered by (bucket, id)).
__device__ __forceinline__ bool rb_accepted(const RbView &r, int64_t v, int32_t j)
{
    const int cb = r.cbeta_tgt[j];
    const int be = r.rbeta[v];
    return be < cb || (be == cb && v < (int64_t)r.theta_tgt[j]);
}

// Accepted and kept by its source a.
__device__ __forceinline__ bool rb_kept(const RbView &r, int64_t v, int32_t a, int32_t j)
{
    if (!rb_accepted(r, v, j)) return false;
    const int cb = r.cbeta_src[a];
    const int be = r.rbeta[v];
    return be < cb || (be == cb && v < (int64_t)r.theta_src[a]);
}

// ------------------------------------------------------------------ begin --

// Count source blocks and snapshot W (one workgroup). For a batch, also per
// graph: gstat[g][GS_OVER]. first: the count also goes to CNT_OVER0. wcp
// (may be null): the apply's copies of its block-weight sums, added into W
// first and cleared.
__global__ __launch_bounds__(kBlock) void k_rb_begin(Blocks bk, int64_t *W, int64_t *W0,
                                                      unsigned long long *counters, int64_t *gstat,
                                                      int first, unsigned long long *pub,
                                                      unsigned long long seq, int64_t *wcp,
                                                      int ncopies)
{
    __shared__ unsigned long long red[4];
    const int32_t K = bk.total();
    if (gstat) {
        for (int gi = threadIdx.x; gi < bk.ng; gi += kBlock) gstat[(int64_t)gi * GS_COUNT + GS_OVER] = 0;
        __syncthreads();
    }
    unsigned long long over = 0;
    for (int j = threadIdx.x; j < K; j += kBlock) {
        int64_t w = W[j];
        if (wcp) {
            int64_t y[kApplyCopiesMax];
#pragma unroll
            for (int c = 0; c < kApplyCopiesMax; ++c)
                y[c] = c < ncopies ? wcp[(int64_t)c * K + j] : 0;
            int64_t d = 0;
#pragma unroll
            for (int c = 0; c < kApplyCopiesMax; ++c) {
                d += y[c];
                if (y[c]) wcp[(int64_t)c * K + j] = 0;
            }
            if (d) W[j] = w + d;
            w += d;
        }
        W0[j] = w;
        const bool o = w > bk.src_lmax_of(j);
        over += o;
        if (gstat && o) atomic_add_i64(&gstat[(int64_t)bk.graph(j) * GS_COUNT + GS_OVER], 1);
    }
    over = block_sum(over, red);
    if (threadIdx.x < 64) {
        wave_cnt_set(counters, CNT_OVER, over);
        if (first) wave_cnt_set(counters, CNT_OVER0, over);
    }
    if (!pub) return;
    // publish every counter's sum: wave w sums slots 8w .. 8w + 7 (the ones
    // set above take the value computed here)
    static_assert(CNT_COUNT == 32 && kBlock == 256, "four waves of eight slots");
    const int w = threadIdx.x >> 6;
    unsigned long long v[8];
#pragma unroll
    for (int i = 0; i < 8; ++i) v[i] = wave_cnt_get(counters, w * 8 + i);
    if (lane_id() < 8) {
        const int slot = w * 8 + lane_id();
        unsigned long long x = v[0];
#pragma unroll
        for (int i = 1; i < 8; ++i) x = lane_id() == i ? v[i] : x;
        if (slot == CNT_OVER || (first && slot == CNT_OVER0)) x = over;
        pub[1 + slot] = x;
    }
    __threadfence_system();
    __syncthreads();
    if (threadIdx.x == 0) __hip_atomic_store(&pub[0], seq, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_SYSTEM);
}

hipError_t launch_rb_begin(const Blocks &bk, int64_t *W, const RebalWs &r,
                           unsigned long long *counters, int64_t *gstat, hipStream_t s, int first,
                           unsigned long long *pub, unsigned long long seq, int64_t *wcp,
                           int ncopies)
{
    if (!wcp || ncopies < 2) wcp = nullptr;
    hipLaunchKernelGGL(k_rb_begin, dim3(1), dim3(kBlock), 0, s, bk, W, r.W0, counters, gstat,
                       first, pub, seq, wcp, ncopies);
    return hipGetLastError();
}

// This workgroup's copy of a rebalancing histogram (copy blockIdx.x mod
// hist_copies, each K * kRbBuckets entries): with few blocks the workgroups
// of a node scan add to the same few entries, and atomics on one address
// are serialised.
__device__ __forceinline__ int64_t *rb_hist_copy(int64_t *h, const RebalWs &r, int32_t K)
{
    const unsigned c = r.hist_copies > 0 ? (unsigned)r.hist_copies : 1u;
    return h + (int64_t)(blockIdx.x % c) * K * kRbBuckets;
}

// ---------------------------------------------------------------- prepare --

constexpr int kHistLdsBytes = 49152;
// 64-node runs per wave and step of the node scans (their loads in flight together)
constexpr int kRbRuns = 4;

// Nodes of overloaded blocks: target and priority bucket. G lanes per node
// scan its row (V ints per lane per vector): best connected target that
// stays balanced (max conn, ties to the smaller id) and the lightest such
// block (min W, ties to the smaller id) as fallback.

// One vector of V columns starting at column j0 of a source row.
template <int V>
__device__ __forceinline__ void rb_scan_cols(const int32_t (&c)[V], int j0, int32_t a,
                                             int32_t base, int64_t cv, int64_t lmax,
                                             const int64_t *W0, int64_t &best, int64_t &lw,
                                             int32_t &lj, int32_t &ca_mine)
{
#pragma unroll
    for (int t = 0; t < V; ++t) {
        const int j = j0 + t;
        if (j == a) {
            ca_mine = c[t];
            continue;
        }
        const int64_t wj = W0[base + j];
        if (wj + cv > lmax) continue;
        if (c[t] > 0) {
            const int64_t pk = ((int64_t)c[t] << 16) | (int64_t)(0xFFFF - j);
            if (pk > best) best = pk;
        }
        if (wj < lw || (wj == lw && j < lj)) {
            lw = wj;
            lj = j;
        }
    }
}

template <int V>
__device__ __forceinline__ void rb_load_vec(const int32_t *row, int q, int32_t (&c)[V])
{
    if constexpr (V == 4) {
        const v4i32 x = stream_load4(row + 4 * q);
        c[0] = x.x;
        c[1] = x.y;
        c[2] = x.z;
        c[3] = x.w;
    } else {
        c[0] = stream_load(row + q);
    }
}

// U source nodes per lane group at a time (their rows loaded together); with
// U > 1 or R > 1 a lane holds R vectors of the row, vector q = gl + r * G
// (k / V <= G * R). Fewer lanes per node mean fewer shuffle rounds per entry.
// A wave lists the sources among its kRbRuns runs of 64 nodes first and
// takes them GPW * U at a time, so that the rows of all its sources are
// loaded in as few round trips as possible (a source block holds a few
// percent of the nodes: run by run, each run cost a round trip of its own).
template <int G, int V, int U, int R>
__global__ __launch_bounds__(kBlock) void k_rb_prepare(GraphView g, Blocks bk,
                                                        const int32_t *__restrict__ part,
                                                        const int32_t *__restrict__ conn,
                                                        RebalWs r, int hist32, int plain)
{
    extern __shared__ __align__(16) unsigned char lds_raw[];
    const int32_t k = bk.k;
    const int32_t K = bk.total();
    int64_t *sW = (int64_t *)lds_raw;
    const bool w_lds = (size_t)K * 8 <= 16384;
    const bool h_lds = hist32 && (size_t)K * kRbBuckets * 4 <= kHistLdsBytes;
    uint32_t *sH = (uint32_t *)(sW + (w_lds ? K : 0));
    if (w_lds)
        for (int j = threadIdx.x; j < K; j += kBlock) sW[j] = r.W0[j];
    if (h_lds)
        for (int j = threadIdx.x; j < K * kRbBuckets; j += kBlock) sH[j] = 0;
    __syncthreads();
    // the node scan, instantiated once per source of the block weights (the
    // LDS copy or global memory), so that the weights are read with LDS
    // loads rather than generic ones
    auto scan_nodes = [&](const int64_t *W0) {
        constexpr int GPW = 64 / G;  // lane groups per wave
        const int lane = lane_id();
        const int grp = lane / G;
        const int gl = lane & (G - 1);
        const int nvec = k / V;
        // kRbRuns runs of 64 node ids per wave and step: their part entries and
        // block weights are loaded before any run is worked on
        const int64_t stride = (int64_t)gridDim.x * kBlock * kRbRuns;
        for (int64_t base0 = ((int64_t)blockIdx.x * kBlock + (threadIdx.x & ~63)) * kRbRuns; base0 < g.n;
             base0 += stride) {
            int32_t lar[kRbRuns];
            uint64_t maskr[kRbRuns];
    #pragma unroll
            for (int i = 0; i < kRbRuns; ++i) {
                const int64_t lv = base0 + 64 * i + lane;
                lar[i] = part[lv < g.n ? lv : g.n - 1];
            }
    #pragma unroll
            for (int i = 0; i < kRbRuns; ++i) {
                const int64_t lv = base0 + 64 * i + lane;
                const bool ok = lv < g.n && (unsigned)lar[i] < (unsigned)K;
                const int32_t a = ok ? lar[i] : 0;
                maskr[i] = __ballot(ok && W0[a] > bk.src_lmax_of(a));
            }
            int cntr[kRbRuns];
            int cnt = 0;
    #pragma unroll
            for (int i = 0; i < kRbRuns; ++i) {
                cntr[i] = __popcll(maskr[i]);
                cnt += cntr[i];
            }
            // source p of the wave's list: the q-th set bit of the run that holds it
            {
                for (int p0 = 0; p0 < cnt; p0 += GPW * U) {
                    int64_t vu[U];
                    int32_t Au[U];
                    bool oku[U];
                    int32_t cu[U][R][V];
    #pragma unroll
                    for (int u = 0; u < U; ++u) {
                        const int p = p0 + u * GPW + grp;
                        oku[u] = p < cnt;
                        int q = oku[u] ? p : 0, run = 0;
                        uint64_t mask = maskr[0];
    #pragma unroll
                        for (int i = 0; i + 1 < kRbRuns; ++i)
                            if (run == i && q >= cntr[i]) {
                                q -= cntr[i];
                                run = i + 1;
                                mask = maskr[i + 1];
                            }
                        // an unused slot takes the wave's first source (cnt > 0)
                        vu[u] = base0 + 64 * run + (oku[u] ? nth_set_bit(mask, q) : nth_set_bit(mask, 0));
                        Au[u] = part[vu[u]];
                    }
                    if constexpr (U > 1 || R > 1) {
                        // unconditional loads (an unused slot holds the wave's first
                        // source; q >= nvec rereads the last vector, unused), so
                        // that all rows are in flight together
    #pragma unroll
                        for (int u = 0; u < U; ++u) {
    #pragma unroll
                            for (int r = 0; r < R; ++r) {
                                const int q = gl + r * G;
                                rb_load_vec<V>(conn + vu[u] * (int64_t)k, q < nvec ? q : nvec - 1, cu[u][r]);
                            }
                        }
                    }
    #pragma unroll
                    for (int u = 0; u < U; ++u) {
                        const bool ok = oku[u];
                        const int64_t v = vu[u];
                        const int32_t A = Au[u];
                        const int32_t a = ok ? bk.local(A) : 0;     // row index of the source
                        const int32_t base = ok ? bk.base(A) : 0;  // global id of local block 0
                        const int64_t lmax = ok ? bk.lmax_of(A) : 0;
                        int64_t best = -1, lw = INT64_MAX, cv = 1;
                        int32_t lj = 0x7fffffff;
                        int32_t ca_mine = 0;  // omega(v, V_a), held by the lane that loads column a
                        if (ok) {
                            cv = node_weight(g, v);
                            if constexpr (U > 1 || R > 1) {
    #pragma unroll
                                for (int r = 0; r < R; ++r) {
                                    const int q = gl + r * G;
                                    if (q < nvec)
                                        rb_scan_cols<V>(cu[u][r], q * V, a, base, cv, lmax, W0, best, lw,
                                                        lj, ca_mine);
                                }
                            } else {
                                const int32_t *row = conn + v * (int64_t)k;
                                for (int q = gl; q < nvec; q += G) {
                                    int32_t c[V];
                                    rb_load_vec<V>(row, q, c);
                                    rb_scan_cols<V>(c, q * V, a, base, cv, lmax, W0, best, lw, lj,
                                                    ca_mine);
                                }
                            }
                        }
    #pragma unroll
                        for (int off = G / 2; off > 0; off >>= 1) {
                            const int64_t ob = __shfl_xor(best, off);
                            const int64_t ow = __shfl_xor(lw, off);
                            const int32_t oj = __shfl_xor(lj, off);
                            if (ob > best) best = ob;
                            if (ow < lw || (ow == lw && oj < lj)) {
                                lw = ow;
                                lj = oj;
                            }
                        }
                        // column a sits in vector a / V, loaded by lane (a / V) mod G of the group
                        const int32_t ca = __shfl(ca_mine, (lane & ~(G - 1)) + ((a / V) & (G - 1)));
                        bool push = false;
                        int64_t hkey = 0;
                        if (ok && gl == 0) {
                            int32_t tgt = -1;
                            int64_t ct = 0;
                            if (best >= 0) {
                                tgt = 0xFFFF - (int32_t)(best & 0xFFFF);
                                ct = best >> 16;
                            } else if (lj != 0x7fffffff) {
                                tgt = lj;
                            }
                            r.rtgt[v] = tgt >= 0 ? base + tgt : -1;
                            if (tgt >= 0) {
                                // the plain-gain variant ranks by the gain alone (c(v) = 1)
                                const int be = rebalance_bucket(ct - (int64_t)ca, plain ? 1 : cv);
                                r.rbeta[v] = (uint8_t)be;
                                hkey = (int64_t)(base + tgt) * kRbBuckets + be;
                                push = true;
                            }
                        }
                        if (h_lds) {
                            if (push) atomicAdd(&sH[hkey], (uint32_t)cv);
                        } else {
                            wave_hist_add(rb_hist_copy(r.hist_tgt, r, K), hkey, cv, push);
                        }
                    }
                }
            }
        }
    };
    if (w_lds) scan_nodes(sW);
    else scan_nodes(r.W0);
    if (h_lds) {
        __syncthreads();
        int64_t *hT = rb_hist_copy(r.hist_tgt, r, K);
        for (int j = threadIdx.x; j < K * kRbBuckets; j += kBlock)
            if (sH[j]) atomic_add_i64(&hT[j], (int64_t)sH[j]);
    }
}

// ------------------------------------------------------------- cutoffs --

// Source: first bucket whose cumulative weight covers the excess.
// Target: first bucket whose cumulative weight exceeds the capacity.
// One wave per block: each lane holds buckets lane and lane + 64, a wave scan
// gives the cumulative weights. Rows are cleared after reading. The target
// pass (the first) also resets the sub-iteration's move counters.
__global__ __launch_bounds__(kBlock) void k_rb_cutoffs(Blocks bk, RebalWs r, int target_side,
                                                        unsigned long long *counters,
                                                        int64_t *gstat)
{
    const int j = blockIdx.x * (kBlock / 64) + (threadIdx.x >> 6);
    const int lane = lane_id();
    if (target_side && j == 0 && lane == 0) {
        cnt_set(counters, CNT_MOVED_NOW, 0);
        cnt_set(counters, CNT_MOVED_DEG, 0);
    }
    if (j >= bk.total()) return;  // wave-uniform
    if (target_side && gstat && lane == 0 && bk.local(j) == 0)
        gstat[(int64_t)bk.graph(j) * GS_COUNT + GS_MOVED_NOW] = 0;
    const int64_t w0 = r.W0[j];
    const int64_t lmax = bk.lmax_of(j);
    if (!target_side ? (w0 <= bk.src_lmax_of(j)) : (w0 > lmax)) {
        // not a source / not a target: the row was never filled
        if (lane == 0) {
            if (!target_side) r.cbeta_src[j] = kRbBuckets;
            else r.cbeta_tgt[j] = kRbBuckets;
        }
        return;
    }
    int64_t *h = (target_side ? r.hist_tgt : r.hist_src) + (int64_t)j * kRbBuckets;
    const int64_t limit = !target_side ? w0 - lmax : lmax - w0;  // excess or capacity
    const int b1 = lane + 64;
    // the row summed over the histogram's copies (all loads issued first),
    // each copy cleared after reading
    const int64_t cstride = (int64_t)bk.total() * kRbBuckets;
    int64_t y0[kRbHistCopiesMax], y1[kRbHistCopiesMax];
#pragma unroll
    for (int c = 0; c < kRbHistCopiesMax; ++c) {
        const bool in = c < r.hist_copies;
        y0[c] = in ? h[c * cstride + lane] : 0;
        y1[c] = (in && b1 < kRbBuckets) ? h[c * cstride + b1] : 0;
    }
    int64_t x0 = 0, x1 = 0;
#pragma unroll
    for (int c = 0; c < kRbHistCopiesMax; ++c) {
        x0 += y0[c];
        x1 += y1[c];
        if (y0[c]) h[c * cstride + lane] = 0;
        if (y1[c]) h[c * cstride + b1] = 0;
    }
    const int64_t c0 = wave_incl_scan(x0);
    const int64_t t0 = __shfl(c0, 63);
    const int64_t c1 = t0 + wave_incl_scan(x1);
    const bool h0 = !target_side ? c0 >= limit : c0 > limit;
    const bool h1 = b1 < kRbBuckets && (!target_side ? c1 >= limit : c1 > limit);
    const uint64_t m0 = __ballot(h0), m1 = __ballot(h1);
    int cut = kRbBuckets;
    if (m0) cut = __ffsll((unsigned long long)m0) - 1;
    else if (m1) cut = 64 + __ffsll((unsigned long long)m1) - 1;
    if (cut < kRbBuckets) {
        const bool mine = (cut < 64) ? lane == cut : lane == cut - 64;
        if (mine) {
            const int64_t before = (cut < 64) ? c0 - x0 : c1 - x1;
            if (!target_side) {
                r.cbeta_src[j] = cut;
                r.need_src[j] = limit - before;
            } else {
                r.cbeta_tgt[j] = cut;
                r.room_tgt[j] = limit - before;
            }
        }
    } else if (lane == 0) {
        if (!target_side) r.cbeta_src[j] = kRbBuckets;
        else r.cbeta_tgt[j] = kRbBuckets;
    }
}

// ------------------------------------------------------ chunk histograms --

// Movable node of an overloaded block (its rtgt/rbeta are this
// sub-iteration's).
__device__ __forceinline__ bool rb_member(const RebalWs &r, const Blocks &bk, int64_t v, int32_t a)
{
    return (unsigned)a < (unsigned)bk.total() && r.W0[a] > bk.src_lmax_of(a) && r.rtgt[v] >= 0;
}

// One wave's kRbRuns runs of 64 node ids (run i: base + 64 i + lane) for the
// rebalancer's node scans. Every load of all runs is issued before any is
// used (from clamped indices, without a branch): a node's loads depend on
// each other (part, then its block's weights), and taken one node at a time
// they were a chain of round trips.
struct RbRuns {
    int64_t v[kRbRuns];
    int32_t a[kRbRuns], j[kRbRuns];
    int be[kRbRuns];
    bool mem[kRbRuns];  // movable node of an overloaded block (rb_member)
    int64_t cv[kRbRuns];
};
__device__ __forceinline__ void rb_load_runs(const GraphView &g, const Blocks &bk,
                                             const int32_t *part, const RebalWs &r, int64_t base,
                                             RbRuns &x)
{
    const int32_t K = bk.total();
    const int lane = lane_id();
    int64_t vc[kRbRuns];
#pragma unroll
    for (int i = 0; i < kRbRuns; ++i) {
        x.v[i] = base + 64 * i + lane;
        vc[i] = x.v[i] < g.n ? x.v[i] : g.n - 1;
        x.a[i] = part[vc[i]];
        x.j[i] = r.rtgt[vc[i]];
        x.be[i] = r.rbeta[vc[i]];
        x.cv[i] = node_weight(g, vc[i]);
    }
#pragma unroll
    for (int i = 0; i < kRbRuns; ++i) {
        const bool ok = x.v[i] < g.n && (unsigned)x.a[i] < (unsigned)K;
        const int32_t a = ok ? x.a[i] : 0;
        x.mem[i] = ok && r.W0[a] > bk.src_lmax_of(a) && x.j[i] >= 0;
    }
}

// Nodes in the cutoff bucket add their weight to the chunk of their id
// (target side: every offer; source side: accepted offers).
__global__ __launch_bounds__(kBlock) void k_rb_chunks(GraphView g, Blocks bk, const int32_t *part,
                                                       RebalWs r, RbView rv, int target_side)
{
    const int64_t stride = (int64_t)gridDim.x * kBlock * kRbRuns;
    for (int64_t base = ((int64_t)blockIdx.x * kBlock + (threadIdx.x & ~63)) * kRbRuns; base < g.n;
         base += stride) {
        RbRuns x;
        rb_load_runs(g, bk, part, r, base, x);
#pragma unroll
        for (int i = 0; i < kRbRuns; ++i) {
            if (!x.mem[i]) continue;
            const int32_t a = x.a[i], j = x.j[i];
            // chunks count node ids from the start of the node's graph
            const int64_t c = (x.v[i] - (r.goff ? r.goff[bk.graph(a)] : 0)) >> r.chunk_shift;
            if (target_side) {
                if (x.be[i] == r.cbeta_tgt[j])
                    atomic_add_i64(&r.chunk_tgt[(int64_t)j * r.nchunks + c], x.cv[i]);
            } else {
                if (x.be[i] == r.cbeta_src[a] && rb_accepted(rv, x.v[i], j))
                    atomic_add_i64(&r.chunk_src[(int64_t)a * r.nchunks + c], x.cv[i]);
            }
        }
    }
}

// Accepted nodes add their weight to their source's bucket histogram.
__global__ __launch_bounds__(kBlock) void k_rb_src_hist(GraphView g, Blocks bk, const int32_t *part,
                                                         RebalWs r, RbView rv, int hist32)
{
    extern __shared__ __align__(16) unsigned char lds_raw[];
    uint32_t *sH = (uint32_t *)lds_raw;
    const int32_t K = bk.total();
    const bool h_lds = hist32 && (size_t)K * kRbBuckets * 4 <= kHistLdsBytes;
    if (h_lds) {
        for (int j = threadIdx.x; j < K * kRbBuckets; j += kBlock) sH[j] = 0;
        __syncthreads();
    }
    const int64_t stride = (int64_t)gridDim.x * kBlock * kRbRuns;
    for (int64_t base = ((int64_t)blockIdx.x * kBlock + (threadIdx.x & ~63)) * kRbRuns; base < g.n;
         base += stride) {
        RbRuns x;
        rb_load_runs(g, bk, part, r, base, x);
#pragma unroll
        for (int i = 0; i < kRbRuns; ++i) {
            const bool sel = x.mem[i] && rb_accepted(rv, x.v[i], x.j[i]);
            const int64_t hkey = sel ? (int64_t)x.a[i] * kRbBuckets + x.be[i] : 0;
            if (h_lds) {
                if (sel) atomicAdd(&sH[hkey], (uint32_t)x.cv[i]);
            } else {
                wave_hist_add(rb_hist_copy(r.hist_src, r, K), hkey, sel ? x.cv[i] : 0, sel);
            }
        }
    }
    if (h_lds) {
        __syncthreads();
        int64_t *hS = rb_hist_copy(r.hist_src, r, K);
        for (int j = threadIdx.x; j < K * kRbBuckets; j += kBlock)
            if (sH[j]) atomic_add_i64(&hS[j], (int64_t)sH[j]);
    }
}

// ------------------------------------------------------------- id bounds --

constexpr int kThetaRun = 16;  // chunks per thread: nchunks <= 4096 = kThetaRun * kBlock

// One workgroup per block. Within the cutoff bucket, find the id bound:
//   source: theta = (first id at which the cumulative weight reaches need) + 1
//   target: theta = first id at which the cumulative weight exceeds room
// First over chunk sums (clearing the row), then over the ids of one chunk.
__global__ __launch_bounds__(kBlock) void k_rb_theta(GraphView g, Blocks bk, const int32_t *part,
                                                      RebalWs r, RbView rv, int target_side)
{
    __shared__ int64_t scan_lds[4];
    __shared__ int64_t found_lds[2];
    const int32_t j = blockIdx.x;
    int cb;
    int64_t limit;
    if (!target_side) {
        if (r.W0[j] <= bk.src_lmax_of(j)) return;
        cb = r.cbeta_src[j];
        limit = r.need_src[j];
    } else {
        cb = r.cbeta_tgt[j];
        limit = r.room_tgt[j];
    }
    if (cb >= kRbBuckets) return;
    int64_t *row = (target_side ? r.chunk_tgt : r.chunk_src) + (int64_t)j * r.nchunks;
    // reached(x): source x >= need, target x > room. Each thread owns a run
    // of consecutive chunks (reads and clears them); one block scan of the
    // run totals locates the chunk where the bound is first reached.
    if (threadIdx.x == 0) {
        found_lds[0] = -1;
        found_lds[1] = 0;
    }
    // a run of at most kThetaRun chunks per thread (nchunks <= 4096), held in
    // registers: all its loads are issued together
    const int64_t per = (r.nchunks + kBlock - 1) / kBlock;
    const int64_t c_lo = threadIdx.x * per;
    int64_t xs[kThetaRun];
    int64_t run_sum = 0;
#pragma unroll
    for (int i = 0; i < kThetaRun; ++i) {
        const int64_t c = c_lo + i;
        const bool in = i < per && c < r.nchunks;
        const int64_t x = row[in ? c : 0];
        xs[i] = in ? x : 0;
        run_sum += xs[i];
    }
    int64_t total;
    const int64_t incl = block_incl_scan(run_sum, scan_lds, &total);
    int64_t cum = incl - run_sum;
#pragma unroll
    for (int i = 0; i < kThetaRun; ++i) {
        const int64_t x = xs[i];
        if (x) {
            const int64_t c = c_lo + i;
            row[c] = 0;
            const int64_t nxt = cum + x;
            const bool reach = target_side ? (nxt > limit) : (nxt >= limit);
            const bool before = target_side ? (cum > limit) : (cum >= limit);
            if (reach && !before) {
                found_lds[0] = c;
                found_lds[1] = cum;
            }
            cum = nxt;
        }
    }
    __syncthreads();
    const int64_t chunk = found_lds[0];
    int64_t before = found_lds[1];
    __syncthreads();
    if (chunk < 0) return;  // cannot happen when cb < kRbBuckets
    const int64_t off = r.goff ? r.goff[bk.graph(j)] : 0;
    const int64_t end = r.goff ? r.goff[bk.graph(j) + 1] : g.n;
    const int64_t id0 = off + (chunk << r.chunk_shift);
    int64_t id1 = off + ((chunk + 1) << r.chunk_shift);
    if (id1 > end) id1 = end;
    if (threadIdx.x == 0) found_lds[0] = -1;
    __syncthreads();
    for (int64_t b0 = id0; b0 < id1; b0 += kBlock) {
        const int64_t v = b0 + threadIdx.x;
        int64_t x = 0;
        if (v < id1) {
            const int32_t a = part[v];
            if (rb_member(r, bk, v, a) && (int)r.rbeta[v] == cb) {
                if (target_side) {
                    if (r.rtgt[v] == j) x = node_weight(g, v);
                } else {
                    if (a == j && rb_accepted(rv, v, r.rtgt[v])) x = node_weight(g, v);
                }
            }
        }
        int64_t total;
        const int64_t inc = block_incl_scan(x, scan_lds, &total);
        const int64_t cum = before + inc;
        const bool hit = x > 0 && (target_side ? (cum > limit) : (cum >= limit)) &&
                         !(target_side ? (cum - x > limit) : (cum - x >= limit));
        if (hit) found_lds[0] = v;
        __syncthreads();
        const int64_t fv = found_lds[0];
        __syncthreads();
        if (fv >= 0) {
            if (threadIdx.x == 0) {
                if (!target_side) r.theta_src[j] = (int32_t)(fv + 1);
                else r.theta_tgt[j] = (int32_t)fv;
            }
            return;
        }
        before += total;
    }
}

// ------------------------------------------------------------------ moves --

// Accepted nodes get mvto[v] = target; counts per workgroup. rbrec (may be
// null): each moved node's sub-iteration and priority bucket, iter << 8 |
// bucket (the order in which the move was made).
__global__ __launch_bounds__(kBlock) void k_rb_moves(GraphView g, Blocks bk, const int32_t *part,
                                                      RebalWs r, RbView rv, int32_t *mvto,
                                                      int64_t hub_t, unsigned long long *counters,
                                                      int64_t *gstat, int32_t *rbrec, int32_t iter)
{
    __shared__ unsigned long long moved, mdeg;
    if (threadIdx.x == 0) {
        moved = 0;
        mdeg = 0;
    }
    __syncthreads();
    const int64_t stride = (int64_t)gridDim.x * kBlock * kRbRuns;
    for (int64_t base = ((int64_t)blockIdx.x * kBlock + (threadIdx.x & ~63)) * kRbRuns; base < g.n;
         base += stride) {
        RbRuns x;
        rb_load_runs(g, bk, part, r, base, x);
#pragma unroll
        for (int i = 0; i < kRbRuns; ++i) {
            const bool acc = x.mem[i] && rb_kept(rv, x.v[i], x.a[i], x.j[i]);
            if (acc) {
                const int64_t v = x.v[i];
                mvto[v] = x.j[i];
                if (rbrec) rbrec[v] = (iter << 8) | (int32_t)r.rbeta[v];
                atomicAdd(&mdeg, (unsigned long long)(g.xadj[v + 1] - g.xadj[v]));
            }
            wave_count(acc, &moved);
            if (gstat)
                wave_hist_add(gstat, (int64_t)bk.graph(acc ? x.a[i] : 0) * GS_COUNT + GS_MOVED_NOW, 1,
                              acc);
        }
    }
    __syncthreads();
    if (threadIdx.x == 0 && moved) {
        cnt_add(counters, CNT_MOVED_NOW, moved);
        cnt_add(counters, CNT_REBAL_MOVES, moved);
        cnt_add(counters, CNT_MOVED_DEG, mdeg);
    }
}

// --------------------------------------------------------------- sequence --

// Node scans of the rebalancer: few enough workgroups that the per-workgroup
// histogram flushes do not pile up on the same addresses.
int rb_scan_grid(int64_t n) { return grid_cap(n, kBlock, 1024); }

hipError_t launch_rb_iteration(const GraphView &g, const Blocks &bk, const int32_t *part,
                               const int32_t *conn, const RebalWs &r, int32_t *mvto, int hist32,
                               int plain, int64_t hub_t, unsigned long long *counters,
                               int64_t *gstat, hipStream_t s, int32_t *rbrec, int32_t iter)
{
    hipError_t e;
    const RbView rv{r.rtgt, r.rbeta, r.W0, r.cbeta_src, r.theta_src, r.cbeta_tgt, r.theta_tgt};
    const int32_t k = bk.k;
    const int32_t K = bk.total();
    const int lg = rb_scan_grid(g.n);
    const bool h_lds = hist32 && (size_t)K * kRbBuckets * 4 <= kHistLdsBytes;
    const size_t plds = ((size_t)K * 8 <= 16384 ? (size_t)K * 8 : 0) +
                        (h_lds ? (size_t)K * kRbBuckets * 4 : 0);
    const bool vec = (k % 4) == 0;
    const int nvec = vec ? k / 4 : k;
#define UPR_RP(GG, VV, UU, RR)                                                                  \
    hipLaunchKernelGGL((k_rb_prepare<GG, VV, UU, RR>), dim3(lg), dim3(kBlock), plds, s, g, bk,     \
                       part, conn, r, hist32, plain)
    if (vec) {
        // up to four int4 of the row per lane
        if (nvec <= 1) UPR_RP(1, 4, 4, 1);
        else if (nvec <= 2) UPR_RP(1, 4, 2, 2);
        else if (nvec <= 4) UPR_RP(1, 4, 1, 4);
        else if (nvec <= 8) UPR_RP(2, 4, 2, 4);
        else if (nvec <= 16) UPR_RP(4, 4, 2, 4);
        else if (nvec <= 32) UPR_RP(8, 4, 1, 4);
        else if (nvec <= 64) UPR_RP(16, 4, 1, 4);
        else UPR_RP(64, 4, 1, 1);
    } else {
        if (nvec <= 2) UPR_RP(2, 1, 4, 1);
        else if (nvec <= 4) UPR_RP(4, 1, 4, 1);
        else if (nvec <= 8) UPR_RP(8, 1, 4, 1);
        else if (nvec <= 16) UPR_RP(16, 1, 4, 1);
        else if (nvec <= 32) UPR_RP(32, 1, 4, 1);
        else if (nvec <= 64) UPR_RP(64, 1, 4, 1);
        else UPR_RP(64, 1, 1, 1);
    }
#undef UPR_RP
    if ((e = hipGetLastError()) != hipSuccess) return e;
    const dim3 kg((K + 3) / 4);  // one wave per block
    // target side over all offers
    hipLaunchKernelGGL(k_rb_cutoffs, kg, dim3(kBlock), 0, s, bk, r, 1, counters, gstat);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    hipLaunchKernelGGL(k_rb_chunks, dim3(lg), dim3(kBlock), 0, s, g, bk, part, r, rv, 1);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    hipLaunchKernelGGL(k_rb_theta, dim3(K), dim3(kBlock), 0, s, g, bk, part, r, rv, 1);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    // source side over the accepted offers
    hipLaunchKernelGGL(k_rb_src_hist, dim3(lg), dim3(kBlock), h_lds ? (size_t)K * kRbBuckets * 4 : 0,
                       s, g, bk, part, r, rv, hist32);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    hipLaunchKernelGGL(k_rb_cutoffs, kg, dim3(kBlock), 0, s, bk, r, 0, counters, gstat);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    hipLaunchKernelGGL(k_rb_chunks, dim3(lg), dim3(kBlock), 0, s, g, bk, part, r, rv, 0);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    hipLaunchKernelGGL(k_rb_theta, dim3(K), dim3(kBlock), 0, s, g, bk, part, r, rv, 0);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    hipLaunchKernelGGL(k_rb_moves, dim3(lg), dim3(kBlock), 0, s, g, bk, part, r, rv, mvto, hub_t,
                       counters, gstat, rbrec, iter);
    return hipGetLastError();
}

}  // namespace upr
