// Move phase of one round: penalty prefix sums, penalised best move,
// conflict filter and scatter-apply.
//
// Best move gives each node a lane group that holds its table row in
// registers. The filter and the apply take tiles of consecutive nodes and
// spread the tile's edges (of candidates, of movers) over all threads of the
// workgroup; hubs are split into edge chunks processed by whole workgroups.
// Loads meant to be in flight together are issued without branches.
// Counters are summed per workgroup in LDS and added to global memory once
// per workgroup.
#include "upr_common.h"

#include <cstdlib>

namespace upr {


static int grid_cap(int64_t items, int per_block, int cap)
{
    int64_t g = (items + per_block - 1) / per_block;
    if (g < 1) g = 1;
    if (g > cap) g = cap;
    return (int)g;
}

// ----------------------------------------------------------- round init --

// Zero the counters, the penalty buckets and (rebuild form) the block
// weights; for a single graph publish the round's Q16 penalty table and L_max.
__global__ void k_round_init(Blocks bk, int64_t *bucket, int64_t *W, PenTable pq, int64_t lmax,
                             int single, unsigned long long *counters, int zero_w,
                             unsigned long long *zero2, int64_t zero2_count, HubView h,
                             int32_t *hub_conn, int32_t k)
{
    const int64_t K = bk.total();
    const int64_t tid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = tid; i < K * kSlots; i += stride) bucket[i] = 0;
    if (zero_w)
        for (int64_t i = tid; i < K; i += stride) W[i] = 0;
    if (single) {
        if (tid < kSlots) ((int64_t *)bk.penq)[tid] = pq.q[tid];
        if (tid == 0) {
            ((int64_t *)bk.lmax)[0] = lmax;
            ((int64_t *)bk.src_lmax)[0] = lmax;
        }
    }
    for (int64_t i = tid; i < kCntWords; i += stride) counters[i] = 0;
    for (int64_t i = tid; i < zero2_count; i += stride) zero2[i] = 0;
    if (hub_conn)
        for (int64_t i = tid; i < (int64_t)h.nh * k; i += stride)
            hub_conn[(int64_t)h.ids[i / k] * k + i % k] = 0;
}

hipError_t launch_round_init(const Blocks &bk, int64_t *bucket, int64_t *W, const PenTable &pq,
                             int64_t lmax, int single, unsigned long long *counters, int zero_w,
                             unsigned long long *zero2, int64_t zero2_count, hipStream_t s,
                             const HubView &h, int32_t *hub_conn, int32_t k)
{
    if (hub_conn && (h.nh <= 0 || k <= 0)) hub_conn = nullptr;
    hipLaunchKernelGGL(k_round_init, dim3(grid_cap((int64_t)bk.total() * kSlots, kBlock * 4, 1024)),
                       dim3(kBlock), 0, s, bk, bucket, W, pq, lmax, single, counters, zero_w, zero2,
                       zero2_count, h, hub_conn, k);
    return hipGetLastError();
}

// Per block B: prefix sums over slots, cb[B][l] = sum_{i <= l} c(B_{i,B}), and
// the penalty a node of weight 1 pays to enter B: 0 if W[B] + 1 <= L_max
// (limited imbalance: the cap floor(alpha * L_max)); otherwise constrained and
// limited imbalance: -1 (forbidden); penalty-free: 0; penalised: penq[l] for
// the least covering slot l, -1 if none.
// One wave per block j: lane l holds slot l, a wave scan turns the slot
// weights into cumulative ones, and the least slot that covers the excess is
// the lowest lane of a ballot. With the statistics pass's copies (wsp, bsp),
// block j's entries of every copy are first added into W[j] and its slot
// weights, and cleared.
__global__ __launch_bounds__(kBlock) void k_cb_prefix(Blocks bk, int64_t *bucket, int64_t *W,
                                                       int mode, int64_t *pen1, int64_t *wsp,
                                                       int64_t *bsp, int ncopies)
{
    static_assert(kSlots <= 64, "one slot per lane");
    static_assert(kStatsCopiesMax <= 64, "one copy per lane");
    const int64_t j = ((int64_t)blockIdx.x * kBlock + threadIdx.x) >> 6;
    const int64_t K = bk.total();
    if (j >= K) return;  // whole waves
    const int l = lane_id();
    int64_t *b = bucket + j * kSlots;
    int64_t own = l < kSlots ? b[l] : (int64_t)0;
    int64_t wj = W[j];
    if (wsp) {
        // every copy's entries loaded first, then summed and cleared
        int64_t yb[kStatsCopiesMax];
#pragma unroll
        for (int c = 0; c < kStatsCopiesMax; ++c)
            yb[c] = (c < ncopies && l < kSlots) ? bsp[((int64_t)c * K + j) * kSlots + l] : 0;
        const int64_t yw = l < ncopies ? wsp[(int64_t)l * K + j] : 0;
#pragma unroll
        for (int c = 0; c < kStatsCopiesMax; ++c) {
            own += yb[c];
            if (yb[c]) bsp[((int64_t)c * K + j) * kSlots + l] = 0;
        }
        if (yw) wsp[(int64_t)l * K + j] = 0;
        const int64_t sw = wave_sum(yw);
        wj += sw;
        if (l == 0 && sw) W[j] = wj;
    }
    const int64_t run = wave_incl_scan(own);
    if (l < kSlots) b[l] = run;
    const int64_t x = wj + 1 - bk.move_lmax_of((int32_t)j);
    const uint64_t cov = __ballot(l < kSlots && run >= x);
    if (l != 0) return;
    int64_t p = 0;
    if (x > 0) {
        if (mode == 1 || mode == 3) p = -1;
        else if (mode == 0) {
            const int ls = cov ? __ffsll((unsigned long long)cov) - 1 : kSlots;
            p = ls >= kSlots ? -1 : bk.penq_of((int32_t)j)[ls];
        }
    }
    pen1[j] = p;
}

hipError_t launch_cb_prefix(const Blocks &bk, int64_t *bucket, int64_t *W, int mode,
                            int64_t *pen1, hipStream_t s, int64_t *wsp, int64_t *bsp, int ncopies)
{
    if (!wsp || !bsp || ncopies < 2) wsp = bsp = nullptr;
    hipLaunchKernelGGL(k_cb_prefix, dim3((unsigned)(((int64_t)bk.total() * 64 + kBlock - 1) / kBlock)),
                       dim3(kBlock), 0, s, bk, bucket, W, mode, pen1, wsp, bsp, ncopies);
    return hipGetLastError();
}

// ------------------------------------------------------------- best move --

// S2: per node v in block a, over blocks j != a with omega(v, V_j) >
// omega(v, V_a) (only those can score above 0):
//   X = W[j] + c(v) - L_max; P = 0 if X <= 0; constrained: skip if X > 0;
//   penalised: l = least slot with cb[j][l] >= X (skip if none),
//   P = min(penq[l] * c(v), 2^62); score = delta * 2^16 - P.
// G lanes per node, each reading V consecutive ints of the row per step. The
// best score (ties to the smaller j) is reduced as (score << 16 | 0xFFFF - j).
// key[v] = score << 16 | j for candidates (score > 0), -1 otherwise. j is the
// local block (row index); W, cb and pen1 are read at the global id base + j.
template <int G, int V, bool LW>
__global__ __launch_bounds__(kBlock) void k_best_move(
    GraphView g, Blocks bk, const int32_t *__restrict__ part, const int32_t *__restrict__ conn,
    const int64_t *__restrict__ W, const int64_t *__restrict__ cb,
    const int64_t *__restrict__ pen1, int mode, const uint8_t *__restrict__ active,
    int64_t *__restrict__ key, int64_t *__restrict__ pen, unsigned long long *counters,
    uint8_t *cflag, uint8_t *cflag2, int64_t *key2, const int32_t *perm, int32_t adj_deg)
{
    extern __shared__ __align__(16) unsigned char lds_raw[];
    const int32_t k = bk.k;
    const int32_t K = bk.total();
    int64_t *sW = (int64_t *)lds_raw;
    int64_t *sP = sW + K;
    __shared__ unsigned long long cand_lds;
    // LW (K <= 2048): block weights and penalties from their LDS copies; a
    // compile-time choice, so that no load goes through a generic pointer
    constexpr bool use_lds = LW;
    const bool unit = g.vwgt == nullptr;
    if (threadIdx.x == 0) cand_lds = 0;
    if (use_lds)
        for (int j = threadIdx.x; j < K; j += kBlock) {
            sW[j] = W[j];
            sP[j] = pen1[j];
        }
    __syncthreads();
    // values, not a pointer that may point to either: LDS or global loads, not generic ones
    auto Wr = [&](int64_t i) { return use_lds ? sW[i] : W[i]; };
    auto Pr = [&](int64_t i) { return use_lds ? sP[i] : pen1[i]; };

    constexpr int GPB = kBlock / G;
    const int gl = threadIdx.x & (G - 1);
    const int nvec = k / V;  // row length in vectors (V divides k)
    const int64_t stride = (int64_t)gridDim.x * GPB;
    const int64_t first = (int64_t)blockIdx.x * GPB + threadIdx.x / G;
    for (int64_t v = first; v < g.n; v += stride) {
        // nodes of degree <= adj_deg are decided by the adjacency form
        if (adj_deg > 0 && g.xadj[v + 1] - g.xadj[v] <= adj_deg) continue;  // group-uniform
        int64_t best = 0, bestP = 0;
        const int32_t A = part[v];
        const int64_t cv = node_weight(g, v);
        if ((unsigned)A < (unsigned)K && (!active || active[v])) {
            const int32_t a = bk.local(A);
            const int32_t base = bk.base(A);
            const int64_t lmax = bk.move_lmax_of(A);  // L_max, or the limited-imbalance cap
            const int64_t *penq = bk.penq_of(A);
            const int32_t *row = conn + v * (int64_t)k;
            const int32_t ca = row[a];
            for (int q = gl; q < nvec; q += G) {
                int32_t c4[V];
                if constexpr (V == 4) {
                    const v4i32 x = stream_load4(row + 4 * q);
                    c4[0] = x.x;
                    c4[1] = x.y;
                    c4[2] = x.z;
                    c4[3] = x.w;
                } else {
                    c4[0] = stream_load(row + q);
                }
#pragma unroll
                for (int t = 0; t < V; ++t) {
                    const int32_t cj = c4[t];
                    const int j = q * V + t;
                    if (cj <= ca || j == a) continue;
                    const int64_t delta = (int64_t)cj - ca;
                    int64_t P;
                    if (unit) {
                        P = Pr(base + j);
                        if (P < 0) continue;
                    } else {
                        P = 0;
                        const int64_t x = Wr(base + j) + cv - lmax;
                        if (x > 0) {
                            if (mode == 1 || mode == 3) continue;
                            if (mode == 0) {
                                const int l = covering_slot(cb + (int64_t)(base + j) * kSlots, x);
                                if (l >= kSlots) continue;
                                P = sat_mul_pen(penq[l], cv);
                            }
                        }
                    }
                    const int64_t sc = delta * 65536 - P;
                    if (sc <= 0) continue;
                    const int64_t packed = (sc << 16) | (int64_t)(0xFFFF - j);
                    if (packed > best) {
                        best = packed;
                        bestP = P;
                    }
                }
            }
        }
#pragma unroll
        for (int off = G / 2; off > 0; off >>= 1) {
            const int64_t ob = __shfl_xor(best, off);
            const int64_t op = __shfl_xor(bestP, off);
            if (ob > best) {
                best = ob;
                bestP = op;
            }
        }
        if (gl == 0) {
            if (best > 0) {
                const int64_t sc = best >> 16;
                const int32_t j = 0xFFFF - (int32_t)(best & 0xFFFF);
                key[v] = (sc << 16) | j;
                pen[v] = bestP;
                if (cflag) cflag[v] = (uint8_t)(bk.local(A) | kCandFlag);
                if (cflag2) {  // the same in the plan's label order
                    const int32_t lv = perm[v];
                    cflag2[lv] = (uint8_t)(bk.local(A) | kCandFlag);
                    key2[lv] = (sc << 16) | j;
                }
                atomicAdd(&cand_lds, 1ull);
            } else {
                key[v] = -1;
            }
        }
    }
    __syncthreads();
    if (threadIdx.x == 0 && cand_lds) cnt_add(counters, CNT_CAND, cand_lds);
}

// The same move choice with the row held in registers (k a multiple of 4, at
// most 1024): G lanes per node, R int4 per lane (q = r * G + lane), U nodes
// per lane group and step. The row loads, part[v] and the next node's loads
// are in flight together, and omega(v, V_a) comes from the loaded row by a
// shuffle instead of a dependent load.
template <int G, int R, int U, bool LW>
__global__ __launch_bounds__(kBlock) void k_best_move_reg(
    GraphView g, Blocks bk, const int32_t *__restrict__ part, const int32_t *__restrict__ conn,
    const int64_t *__restrict__ W, const int64_t *__restrict__ cb,
    const int64_t *__restrict__ pen1, int mode, const uint8_t *__restrict__ active,
    int64_t *__restrict__ key, int64_t *__restrict__ pen, unsigned long long *counters,
    uint8_t *cflag, uint8_t *cflag2, int64_t *key2, const int32_t *perm, int32_t adj_deg)
{
    extern __shared__ __align__(16) unsigned char lds_raw[];
    const int32_t k = bk.k;
    const int32_t K = bk.total();
    int64_t *sW = (int64_t *)lds_raw;
    int64_t *sP = sW + K;
    __shared__ unsigned long long cand_lds;
    // LW (K <= 2048): block weights and penalties from their LDS copies; a
    // compile-time choice, so that no load goes through a generic pointer
    constexpr bool use_lds = LW;
    const bool unit = g.vwgt == nullptr;
    // unit node weights with the table in LDS: a forbidden target (P < 0)
    // gets a penalty above any gain (a gain is below 2^31, its score below
    // 2^47), so that one signed comparison decides every entry
    const bool lean = unit && use_lds;
    if (threadIdx.x == 0) cand_lds = 0;
    if (use_lds)
        for (int j = threadIdx.x; j < K; j += kBlock) {
            sW[j] = W[j];
            const int64_t P = pen1[j];
            sP[j] = (lean && P < 0) ? kPenCap : P;
        }
    __syncthreads();
    // values, not a pointer that may point to either: LDS or global loads, not generic ones
    auto Wr = [&](int64_t i) { return use_lds ? sW[i] : W[i]; };
    auto Pr = [&](int64_t i) { return use_lds ? sP[i] : pen1[i]; };

    constexpr int GPB = kBlock / G;
    const int lane = lane_id();
    const int gl = lane & (G - 1);
    const int gbase = lane & ~(G - 1);
    const int nvec = k >> 2;
    const int64_t stride = (int64_t)gridDim.x * GPB * U;
    for (int64_t v0 = ((int64_t)blockIdx.x * GPB + threadIdx.x / G) * U; v0 < g.n; v0 += stride) {
        int32_t A[U];
        bool skip[U];
        v4i32 x[U][R];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int64_t v = v0 + u;
            // nodes of degree <= adj_deg are decided by the adjacency form
            skip[u] = v < g.n && adj_deg > 0 && g.xadj[v + 1] - g.xadj[v] <= adj_deg;
            const bool valid = v < g.n && !skip[u];
            A[u] = valid ? part[v] : -1;
            if (valid && active && !active[v]) A[u] = -1;
            const int32_t *row = conn + v * (int64_t)k;
#pragma unroll
            for (int r = 0; r < R; ++r) {
                const int q = r * G + gl;
                if (valid && q < nvec) {
                    x[u][r] = stream_load4(row + 4 * q);
                } else {
                    x[u][r].x = x[u][r].y = x[u][r].z = x[u][r].w = 0;
                }
            }
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int64_t v = v0 + u;
            const int32_t Au = A[u];
            const bool ok = (unsigned)Au < (unsigned)K;  // group-uniform
            const int32_t a = ok ? bk.local(Au) : 0;
            const int32_t base = ok ? bk.base(Au) : 0;
            // omega(v, V_a) from the lane and register that hold column a
            const int qa = a >> 2;
            const int ra = qa / G;
            v4i32 xr = x[u][0];
#pragma unroll
            for (int r = 1; r < R; ++r)
                if (ra == r) xr = x[u][r];
            const int comp = a & 3;
            const int32_t mine = comp == 0 ? xr.x : comp == 1 ? xr.y : comp == 2 ? xr.z : xr.w;
            const int32_t ca = __shfl(mine, gbase + (qa & (G - 1)));
            int64_t best = 0, bestP = 0;
            const int64_t cv = node_weight(g, ok ? v : 0);
            if (ok && lean) {
                // score (c_j - c_a) 2^16 - P_j for every column: the own
                // block (0 - P) and columns with c_j <= c_a never score above
                // zero, so no test of their own is needed; columns come in
                // increasing order, a strict comparison keeps the smallest j
                // of a tie
                int64_t bsc = 0;
                int32_t bj = 0;
#pragma unroll
                for (int r = 0; r < R; ++r) {
                    const int q = r * G + gl;
                    if (q >= nvec) continue;
                    const int32_t c4[4] = {x[u][r].x, x[u][r].y, x[u][r].z, x[u][r].w};
#pragma unroll
                    for (int t = 0; t < 4; ++t) {
                        const int j = q * 4 + t;
                        // (sP itself, not the generic Pr: LDS loads instead of flat ones)
                        const int64_t sc = ((int64_t)(c4[t] - ca) << 16) - sP[base + j];
                        if (sc > bsc) {
                            bsc = sc;
                            bj = j;
                        }
                    }
                }
                if (bsc > 0) {
                    best = (bsc << 16) | (int64_t)(0xFFFF - bj);
                    bestP = sP[base + bj];
                }
            } else if (ok) {
                const int64_t lmax = bk.move_lmax_of(Au);
                const int64_t *penq = bk.penq_of(Au);
#pragma unroll
                for (int r = 0; r < R; ++r) {
                    const int q = r * G + gl;
                    if (q >= nvec) continue;
                    const int32_t c4[4] = {x[u][r].x, x[u][r].y, x[u][r].z, x[u][r].w};
#pragma unroll
                    for (int t = 0; t < 4; ++t) {
                        const int32_t cj = c4[t];
                        const int j = q * 4 + t;
                        if (cj <= ca || j == a) continue;
                        const int64_t delta = (int64_t)cj - ca;
                        int64_t P;
                        if (unit) {
                            P = Pr(base + j);
                            if (P < 0) continue;
                        } else {
                            P = 0;
                            const int64_t xx = Wr(base + j) + cv - lmax;
                            if (xx > 0) {
                                if (mode == 1 || mode == 3) continue;
                                if (mode == 0) {
                                    const int l = covering_slot(cb + (int64_t)(base + j) * kSlots, xx);
                                    if (l >= kSlots) continue;
                                    P = sat_mul_pen(penq[l], cv);
                                }
                            }
                        }
                        const int64_t sc = delta * 65536 - P;
                        if (sc <= 0) continue;
                        const int64_t packed = (sc << 16) | (int64_t)(0xFFFF - j);
                        if (packed > best) {
                            best = packed;
                            bestP = P;
                        }
                    }
                }
            }
#pragma unroll
            for (int off = G / 2; off > 0; off >>= 1) {
                const int64_t ob = __shfl_xor(best, off);
                const int64_t op = __shfl_xor(bestP, off);
                if (ob > best) {
                    best = ob;
                    bestP = op;
                }
            }
            if (gl == 0 && v < g.n && !skip[u]) {
                if (best > 0) {
                    const int64_t sc = best >> 16;
                    const int32_t j = 0xFFFF - (int32_t)(best & 0xFFFF);
                    key[v] = (sc << 16) | j;
                    pen[v] = bestP;
                    if (cflag) cflag[v] = (uint8_t)(a | kCandFlag);
                    if (cflag2) {  // the same in the plan's label order
                        const int32_t lv = perm[v];
                        cflag2[lv] = (uint8_t)(a | kCandFlag);
                        key2[lv] = (sc << 16) | j;
                    }
                    atomicAdd(&cand_lds, 1ull);
                } else {
                    key[v] = -1;
                }
            }
        }
    }
    __syncthreads();
    if (threadIdx.x == 0 && cand_lds) cnt_add(counters, CNT_CAND, cand_lds);
}

// The same move choice from the adjacency instead of the table row (the
// row scan costs 4k bytes per node, this one xadj and about 5 bytes per
// edge): one thread per node of degree <= maxd (at most D), which sums its neighbours'
// edge weights per block in a register list (their blocks from the compact
// partition copy) and scores every listed block against the sum for its
// own block. Nodes of higher degree are left to the row kernel.
template <int D, int PB, bool LW>
__global__ __launch_bounds__(kBlock) void k_best_move_adj(
    GraphView g, Blocks bk, const int32_t *__restrict__ part, PartView pv,
    const int64_t *__restrict__ W, const int64_t *__restrict__ cb,
    const int64_t *__restrict__ pen1, int mode, const uint8_t *__restrict__ active,
    int64_t *__restrict__ key, int64_t *__restrict__ pen, unsigned long long *counters,
    uint8_t *cflag, uint8_t *cflag2, int64_t *key2, const int32_t *perm, int32_t maxd)
{
    extern __shared__ __align__(16) unsigned char lds_raw[];
    const int32_t K = bk.total();
    int64_t *sW = (int64_t *)lds_raw;
    int64_t *sP = sW + K;
    __shared__ unsigned long long cand_lds;
    // LW (K <= 2048): block weights and penalties from their LDS copies; a
    // compile-time choice, so that no load goes through a generic pointer
    constexpr bool use_lds = LW;
    const bool unit = g.vwgt == nullptr;
    if (threadIdx.x == 0) cand_lds = 0;
    if (use_lds)
        for (int j = threadIdx.x; j < K; j += kBlock) {
            sW[j] = W[j];
            sP[j] = pen1[j];
        }
    __syncthreads();
    // values, not a pointer that may point to either: LDS or global loads, not generic ones
    auto Wr = [&](int64_t i) { return use_lds ? sW[i] : W[i]; };
    auto Pr = [&](int64_t i) { return use_lds ? sP[i] : pen1[i]; };
    const int32_t pmask = part_mask(pv);
    unsigned long long cands = 0;
    const int64_t stride = (int64_t)gridDim.x * kBlock;
    for (int64_t v = (int64_t)blockIdx.x * kBlock + threadIdx.x; v < g.n; v += stride) {
        const int64_t e0 = g.xadj[v];
        const int32_t d = (int32_t)(g.xadj[v + 1] - e0);
        if (d > maxd) continue;  // maxd <= D; the row kernel takes the rest
        const int32_t A = part[v];
        bool ok = (unsigned)A < (unsigned)K && d > 0 && (!active || active[v]);
        const int32_t a = ok ? bk.local(A) : 0;
        // the neighbours' blocks and edge weights, loaded together (a slot
        // past the row rereads its last edge and is ignored)
        int32_t nb[D], nw[D];
#pragma unroll
        for (int i = 0; i < D; ++i) {
            const int64_t e = e0 + (i < d ? i : (d > 0 ? d - 1 : 0));
            const int32_t u = ok ? g.adjncy[e] : 0;
            nw[i] = ok ? edge_weight(g, e) : 0;
            nb[i] = u;
        }
#pragma unroll
        for (int i = 0; i < D; ++i) nb[i] = pget_w<PB>(pv.p, nb[i], pmask);
        // per-block sums: list of distinct blocks other than a
        int32_t lb[D], ls[D];
        int32_t cnt = 0, ca = 0;
#pragma unroll
        for (int i = 0; i < D; ++i) {
            lb[i] = -1;
            ls[i] = 0;
        }
#pragma unroll
        for (int i = 0; i < D; ++i) {
            if (i >= d) break;
            const int32_t j = nb[i];
            if (j == a) {
                ca += nw[i];
                continue;
            }
            bool found = false;
#pragma unroll
            for (int t = 0; t < D; ++t)
                if (lb[t] == j) {
                    ls[t] += nw[i];
                    found = true;
                }
#pragma unroll
            for (int t = 0; t < D; ++t)
                if (!found && t == cnt) {
                    lb[t] = j;
                    ls[t] = nw[i];
                }
            cnt += found ? 0 : 1;
        }
        int64_t best = 0, bestP = 0;
        if (ok) {
            const int32_t base = bk.base(A);
            const int64_t cv = node_weight(g, v);
            const int64_t lmax = bk.move_lmax_of(A);
            const int64_t *penq = bk.penq_of(A);
#pragma unroll
            for (int t = 0; t < D; ++t) {
                const int32_t cj = ls[t];
                const int32_t j = lb[t];
                if (j < 0 || j >= bk.k || cj <= ca) continue;
                const int64_t delta = (int64_t)cj - ca;
                int64_t P;
                if (unit) {
                    P = Pr(base + j);
                    if (P < 0) continue;
                } else {
                    P = 0;
                    const int64_t xx = Wr(base + j) + cv - lmax;
                    if (xx > 0) {
                        if (mode == 1 || mode == 3) continue;
                        if (mode == 0) {
                            const int l = covering_slot(cb + (int64_t)(base + j) * kSlots, xx);
                            if (l >= kSlots) continue;
                            P = sat_mul_pen(penq[l], cv);
                        }
                    }
                }
                const int64_t sc = delta * 65536 - P;
                if (sc <= 0) continue;
                const int64_t packed = (sc << 16) | (int64_t)(0xFFFF - j);
                if (packed > best) {
                    best = packed;
                    bestP = P;
                }
            }
        }
        if (best > 0) {
            const int64_t sc = best >> 16;
            const int32_t j = 0xFFFF - (int32_t)(best & 0xFFFF);
            key[v] = (sc << 16) | j;
            pen[v] = bestP;
            if (cflag) cflag[v] = (uint8_t)(a | kCandFlag);
            if (cflag2) {
                const int32_t lv = perm[v];
                cflag2[lv] = (uint8_t)(a | kCandFlag);
                key2[lv] = (sc << 16) | j;
            }
            ++cands;
        } else {
            key[v] = -1;
        }
    }
    cands = wave_sum(cands);
    if (lane_id() == 0 && cands) atomicAdd(&cand_lds, cands);
    __syncthreads();
    if (threadIdx.x == 0 && cand_lds) cnt_add(counters, CNT_CAND, cand_lds);
}

// Largest degree the adjacency form takes for k blocks. The row is 4k bytes
// streamed; the adjacency costs xadj, 4 bytes per edge streamed and one
// random gather per edge, which costs about as much as 32 streamed bytes
// (at k = 64 the adjacency form for nodes of degree up to 16 made R-MAT's
// best move twice as slow, the 4-neighbour grid's 30% faster). Its register
// list holds at most kAdjMaxDeg blocks. Splitting the nodes between the two
// forms costs a second pass over xadj and a launch, which pays only for long
// rows: the adjacency form is used when it takes every node (max_deg within
// the bound) or when rows are at least 1 KB (k >= 256; at k = 64 the split
// made R-MAT's best move 50% slower). 0: the row form for every node
// (UPR_ADJ_DEG overrides: 0 disables, else the bound, capped).
constexpr int kAdjMaxDeg = 16;
int32_t best_move_adj_deg(int32_t k, int pv_bytes, int64_t max_deg)
{
    if (pv_bytes > 2) return 0;
    const char *env = getenv("UPR_ADJ_DEG");
    if (env && *env) {
        const long x = strtol(env, nullptr, 10);
        return (int32_t)(x < 0 ? 0 : (x > kAdjMaxDeg ? kAdjMaxDeg : x));
    }
    int32_t d = (4 * k - 16) / 36;
    if (d > kAdjMaxDeg) d = kAdjMaxDeg;
    if (d < 4) return 0;
    return (max_deg <= d || k >= 256) ? d : 0;
}

hipError_t launch_best_move(const GraphView &g, const Blocks &bk, const int32_t *part,
                            const int32_t *conn, const int64_t *W, const int64_t *cb,
                            const int64_t *pen1, int mode, const uint8_t *active, int64_t *key,
                            int64_t *pen, unsigned long long *counters, uint8_t *cflag,
                            hipStream_t s, uint8_t *cflag2, int64_t *key2, const int32_t *perm,
                            const PartView &pv, int32_t adj_deg, int64_t max_deg)
{
    if (g.n <= 0) return hipSuccess;
    const int32_t k = bk.k;
    const bool lw = bk.total() <= 2048;
    const size_t lds = lw ? (size_t)bk.total() * 16 : 0;
    if (adj_deg > 0) {
        if (adj_deg > kAdjMaxDeg || pv.bytes > 2) return hipErrorInvalidValue;
        // the register list no longer than the graph's largest degree
        const int32_t dl = max_deg < adj_deg ? (int32_t)max_deg : adj_deg;
#define UPR_BA(DD, PP)                                                                             \
    do {                                                                                           \
        if (lw)                                                                                    \
            hipLaunchKernelGGL((k_best_move_adj<DD, PP, true>), dim3(grid_cap(g.n, kBlock, 8192)), \
                               dim3(kBlock), lds, s, g, bk, part, pv, W, cb, pen1, mode, active,   \
                               key, pen, counters, cflag, cflag2, key2, perm, adj_deg);            \
        else                                                                                       \
            hipLaunchKernelGGL((k_best_move_adj<DD, PP, false>), dim3(grid_cap(g.n, kBlock, 8192)),\
                               dim3(kBlock), lds, s, g, bk, part, pv, W, cb, pen1, mode, active,   \
                               key, pen, counters, cflag, cflag2, key2, perm, adj_deg);            \
    } while (0)
        if (dl <= 4) {
            if (pv.bytes == 1) UPR_BA(4, 1);
            else UPR_BA(4, 2);
        } else if (dl <= 8) {
            if (pv.bytes == 1) UPR_BA(8, 1);
            else UPR_BA(8, 2);
        } else {
            if (pv.bytes == 1) UPR_BA(16, 1);
            else UPR_BA(16, 2);
        }
#undef UPR_BA
        const hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
        if (max_deg <= adj_deg) return hipSuccess;  // no node is left for the row
    }
    const bool vec = (k % 4) == 0;
    const int nvec = vec ? k / 4 : k;
    if (vec && nvec <= 256) {
#define UPR_BR(GG, RR, UU)                                                                          \
    do {                                                                                            \
        if (lw)                                                                                     \
            hipLaunchKernelGGL((k_best_move_reg<GG, RR, UU, true>),                                 \
                               dim3(grid_cap((g.n + UU - 1) / UU, kBlock / GG, 8192)), dim3(kBlock), \
                               lds, s, g, bk, part, conn, W, cb, pen1, mode, active, key, pen,      \
                               counters, cflag, cflag2, key2, perm, adj_deg);                       \
        else                                                                                        \
            hipLaunchKernelGGL((k_best_move_reg<GG, RR, UU, false>),                                \
                               dim3(grid_cap((g.n + UU - 1) / UU, kBlock / GG, 8192)), dim3(kBlock), \
                               lds, s, g, bk, part, conn, W, cb, pen1, mode, active, key, pen,      \
                               counters, cflag, cflag2, key2, perm, adj_deg);                       \
    } while (0)
        // each lane holds up to four int4 of the row: fewer lanes per node
        // mean fewer shuffle rounds per scored entry (at k = 64, 4 lanes per
        // node took 80 us where 16 lanes took 102)
        if (nvec <= 1) UPR_BR(1, 1, 2);
        else if (nvec <= 2) UPR_BR(1, 2, 2);
        else if (nvec <= 4) UPR_BR(1, 4, 1);
        else if (nvec <= 8) UPR_BR(2, 4, 1);
        else if (nvec <= 16) UPR_BR(4, 4, 1);
        else if (nvec <= 32) UPR_BR(8, 4, 1);
        else if (nvec <= 64) UPR_BR(16, 4, 1);
        else if (nvec <= 128) UPR_BR(32, 4, 1);
        else UPR_BR(64, 4, 1);
#undef UPR_BR
        return hipGetLastError();
    }
#define UPR_BM(GG, VV)                                                                             \
    do {                                                                                           \
        if (lw)                                                                                    \
            hipLaunchKernelGGL((k_best_move<GG, VV, true>), dim3(grid_cap(g.n, kBlock / GG, 8192)),  \
                               dim3(kBlock), lds, s, g, bk, part, conn, W, cb, pen1, mode, active,  \
                               key, pen, counters, cflag, cflag2, key2, perm, adj_deg);             \
        else                                                                                       \
            hipLaunchKernelGGL((k_best_move<GG, VV, false>), dim3(grid_cap(g.n, kBlock / GG, 8192)), \
                               dim3(kBlock), lds, s, g, bk, part, conn, W, cb, pen1, mode, active,  \
                               key, pen, counters, cflag, cflag2, key2, perm, adj_deg);             \
    } while (0)
    if (vec) {
        if (nvec <= 1) UPR_BM(1, 4);
        else if (nvec <= 2) UPR_BM(2, 4);
        else if (nvec <= 4) UPR_BM(4, 4);
        else if (nvec <= 8) UPR_BM(8, 4);
        else if (nvec <= 16) UPR_BM(16, 4);
        else if (nvec <= 32) UPR_BM(32, 4);
        else UPR_BM(64, 4);
    } else {
        if (nvec <= 2) UPR_BM(2, 1);
        else if (nvec <= 4) UPR_BM(4, 1);
        else if (nvec <= 8) UPR_BM(8, 1);
        else if (nvec <= 16) UPR_BM(16, 1);
        else if (nvec <= 32) UPR_BM(32, 1);
        else UPR_BM(64, 1);
    }
#undef UPR_BM
    return hipGetLastError();
}

// ---------------------------------------------------------------- filter --

// Contribution f(x) of a neighbour in block x to the move a -> b.
__device__ __forceinline__ int move_sign(int32_t x, int32_t a, int32_t b)
{
    return (x == b) - (x == a);
}

// S3 for candidate v (a -> b, score sv): pessimistic gain over its row
// [e0, e1) strided by `step` starting at e0 + off. An earlier candidate
// neighbour u ((score, id) before v) contributes the worse of its current
// and its target block (optimistic variant: its target block). kEdgeUnroll
// edges per lane are loaded before their gathers, so their latencies overlap.
constexpr int kEdgeUnroll = 4;
__device__ __forceinline__ int64_t pessimistic_part(const GraphView &g, const PartView &part,
                                                    const int64_t *key, int64_t v, int32_t a,
                                                    int32_t b, int64_t sv, int64_t e0, int64_t e1,
                                                    int off, int step, int optimistic)
{
    int64_t acc = 0;
    for (int64_t e = e0 + off; e < e1; e += (int64_t)kEdgeUnroll * step) {
        int32_t u[kEdgeUnroll], w[kEdgeUnroll];
#pragma unroll
        for (int i = 0; i < kEdgeUnroll; ++i) {
            const int64_t ei = e + (int64_t)i * step;
            u[i] = ei < e1 ? stream_load(g.adjncy + ei) : -1;
            w[i] = ei < e1 ? stream_edge_weight(g, ei) : 0;
        }
        int32_t pu[kEdgeUnroll];
        int64_t ku[kEdgeUnroll];
#pragma unroll
        for (int i = 0; i < kEdgeUnroll; ++i) {
            pu[i] = u[i] >= 0 ? pget(part, u[i]) : -1;
            ku[i] = u[i] >= 0 ? key[u[i]] : -1;
        }
#pragma unroll
        for (int i = 0; i < kEdgeUnroll; ++i) {
            int f = move_sign(pu[i], a, b);
            if (ku[i] >= 0) {
                const int64_t su = ku[i] >> 16;
                if (su > sv || (su == sv && (int64_t)u[i] < v)) {
                    const int ft = move_sign((int32_t)(ku[i] & 0xFFFF), a, b);
                    f = (optimistic || ft < f) ? ft : f;
                }
            }
            acc += (int64_t)w[i] * f;
        }
    }
    return acc;
}

// Candidates of degree up to the hub threshold, one workgroup per tile of
// kFilterTile consecutive nodes. The tile's candidate edges are spread over
// all threads (edge -> node by a binary search over the tile's degree
// prefix), kFilterUnroll edges per thread and step so that their loads overlap;
// each edge adds its term w * f to the node's 32-bit LDS sum (a node's sum is
// bounded by its weighted degree, below 2^31). One LDS atomic per edge was
// faster than a segmented wave scan over the runs of equal nodes.
constexpr int kFilterTile = 256;
constexpr int kFilterUnroll = 8;  // edges per thread and step (8 measured best of 2, 4, 8)

// RL: a neighbour's block and key are read by its label (adj_r[e]) from the
// copies in the plan's degree order (pv2 with candidate flags, key2), where
// the high-degree nodes share cache lines; its id (ties) still from adjncy.
template <int PB, bool RL>
__global__ __launch_bounds__(kBlock) void k_filter(GraphView g, Blocks bk, int optimistic,
                                                    const int32_t *__restrict__ part,
                                                    PartView pv, const int64_t *__restrict__ key,
                                                    const int64_t *__restrict__ pen, int64_t hub_t,
                                                    int32_t *mvto, uint8_t *accflag,
                                                    unsigned long long *counters, int64_t *gp_out,
                                                    const int32_t *__restrict__ adj_r, PartView pv2,
                                                    const int64_t *__restrict__ key2,
                                                    const int32_t *__restrict__ order)
{
    __shared__ int32_t vstart[kFilterTile + 1];
    __shared__ int64_t estart[kFilterTile];
    __shared__ int64_t skey[kFilterTile];
    __shared__ int32_t sa[kFilterTile];  // local source block; -1: not decided here
    __shared__ int32_t sacc[kFilterTile];  // |sum| <= weighted degree < 2^31
    __shared__ int32_t scan_lds[4];
    __shared__ unsigned long long acc_lds, deg_lds;
    const int tid = threadIdx.x;
    if (tid == 0) {
        acc_lds = 0;
        deg_lds = 0;
    }
    const int64_t v0 = (int64_t)blockIdx.x * kFilterTile;
    const int nt = (int)((g.n - v0) < kFilterTile ? (g.n - v0) : kFilterTile);

    // candidates of the tile, their degrees and the degree prefix
    int32_t run = 0;
    for (int base = 0; base < nt; base += kBlock) {
        const int i = base + tid;
        int32_t vd = 0;
        if (i < nt) {
            const int64_t v = v0 + i;
            const int64_t kv = key[v];
            int32_t a = -1;
            if (kv >= 0) {
                const int64_t e0 = g.xadj[v], e1 = g.xadj[v + 1];
                if (e1 - e0 <= hub_t) {
                    a = bk.local(part[v]);
                    vd = (int32_t)(e1 - e0);
                    estart[i] = e0;
                }
            }
            skey[i] = kv;
            sa[i] = a;
            sacc[i] = 0;
        }
        int32_t total;
        const int32_t inc = block_incl_scan(vd, scan_lds, &total);
        if (i < nt) vstart[i] = run + inc - vd;
        run += total;
    }
    if (tid == 0) vstart[nt] = run;
    __syncthreads();

    // S3 terms over all candidate edges of the tile; an earlier candidate
    // neighbour u ((score, id) before v) counts in the worse of its current
    // and its target block (optimistic variant: its target block). Every
    // load is issued unconditionally (a slot past the last edge rereads that
    // edge and adds nothing), so the loads of all slots are in flight
    // together.
    const int32_t E = run;
    const int32_t pmask = part_mask(pv);
    for (int32_t q0 = tid; q0 < E; q0 += kBlock * kFilterUnroll) {
        bool ok[kFilterUnroll];
        int node[kFilterUnroll];
        int64_t e[kFilterUnroll];
#pragma unroll
        for (int i = 0; i < kFilterUnroll; ++i) {
            const int32_t p = q0 + i * kBlock;
            ok[i] = p < E;
            const int32_t pc = ok[i] ? p : E - 1;
            node[i] = upper_index(vstart, nt, pc);
            e[i] = estart[node[i]] + (pc - vstart[node[i]]);
        }
        // with the label copy the neighbour's id is needed only to break a
        // tie of scores; it is then taken from the label's node (order)
        int32_t u[kFilterUnroll], w[kFilterUnroll], ur[kFilterUnroll];
#pragma unroll
        for (int i = 0; i < kFilterUnroll; ++i) {
            if constexpr (RL) ur[i] = stream_load(adj_r + e[i]);
            else u[i] = stream_load(g.adjncy + e[i]);
            w[i] = stream_edge_weight(g, e[i]);
        }
        int32_t raw[kFilterUnroll];
#pragma unroll
        for (int i = 0; i < kFilterUnroll; ++i)
            raw[i] = RL ? pget_w<PB>(pv2.p, ur[i], -1) : pget_w<PB>(pv.p, u[i], -1);
        // a neighbour's key only if it is a candidate (flag bit of the
        // compact copy; without flags every neighbour's key)
        int64_t kraw[kFilterUnroll];
        bool cand[kFilterUnroll];
#pragma unroll
        for (int i = 0; i < kFilterUnroll; ++i) {
            cand[i] = !pv.flagged || (raw[i] & kCandFlag);
            // (a neighbour that is no candidate reads entry 0, one cached
            // line, unused: no load in a branch, and a global load rather than
            // a generic one that could also reach LDS)
            if constexpr (RL) kraw[i] = key2[cand[i] ? ur[i] : 0];
            else kraw[i] = key[cand[i] ? u[i] : 0];
        }
#pragma unroll
        for (int i = 0; i < kFilterUnroll; ++i) {
            if (!ok[i]) continue;
            const int nd = node[i];
            const int32_t pu = raw[i] & pmask;
            const int64_t ku = cand[i] ? kraw[i] : -1;
            const int64_t kv = skey[nd];
            const int32_t a = sa[nd], b = (int32_t)(kv & 0xFFFF);
            int f = move_sign(pu, a, b);
            if (ku >= 0) {
                const int64_t su = ku >> 16, sv = kv >> 16;
                bool earlier = su > sv;
                if (su == sv) {
                    const int64_t uid = RL ? (int64_t)order[ur[i]] : (int64_t)u[i];
                    earlier = uid < v0 + nd;
                }
                if (earlier) {
                    const int ft = move_sign((int32_t)(ku & 0xFFFF), a, b);
                    f = (optimistic || ft < f) ? ft : f;
                }
            }
            const int32_t t = w[i] * f;
            if (t != 0) atomicAdd(&sacc[nd], t);
        }
    }
    __syncthreads();

    // decisions
    for (int base = 0; base < nt; base += kBlock) {
        const int i = base + tid;
        bool take = false;
        if (i < nt && sa[i] >= 0) {
            const int64_t v = v0 + i;
            const int64_t acc = sacc[i];
            if (gp_out) {
                gp_out[v] = acc;  // eligible ones are decided against the sequence-aware price
                accflag[v] = 0;
            } else {
                take = acc * 65536 - pen[v] > 0;
                accflag[v] = take ? 1 : 0;
                if (take) {
                    const int32_t A = part[v];
                    mvto[v] = bk.base(A) + (int32_t)(skey[i] & 0xFFFF);
                    atomicAdd(&deg_lds, (unsigned long long)(vstart[i + 1] - vstart[i]));
                }
            }
        }
        wave_count(take, &acc_lds);
    }
    __syncthreads();
    if (tid == 0) {
        if (acc_lds) cnt_add(counters, CNT_ACC, acc_lds);
        if (deg_lds) cnt_add(counters, CNT_MOVED_DEG, deg_lds);
    }
}

hipError_t launch_filter(const GraphView &g, const Blocks &bk, int optimistic, const int32_t *part,
                         const PartView &pv, const int64_t *key, const int64_t *pen, int64_t hub_t,
                         int32_t *mvto, uint8_t *accflag, unsigned long long *counters,
                         int64_t *gp_out, hipStream_t s, const int32_t *adj_r, const PartView &pv2,
                         const int64_t *key2, const int32_t *order)
{
    if (g.n <= 0) return hipSuccess;
    const int64_t tiles = (g.n + kFilterTile - 1) / kFilterTile;
#define UPR_FI(BB, RR)                                                                             \
    hipLaunchKernelGGL((k_filter<BB, RR>), dim3((unsigned)tiles), dim3(kBlock), 0, s, g, bk,         \
                       optimistic, part, pv, key, pen, hub_t, mvto, accflag, counters, gp_out,     \
                       adj_r, pv2, key2, order)
    if (adj_r && pv2.p && key2 && order && pv.bytes == 1 && pv.flagged) UPR_FI(1, true);
    else if (pv.bytes == 1) UPR_FI(1, false);
    else if (pv.bytes == 2) UPR_FI(2, false);
    else UPR_FI(4, false);
#undef UPR_FI
    return hipGetLastError();
}

// Hub candidates: each chunk adds its part of the pessimistic gain; the
// chunk that finishes last (a per-hub ticket) decides the move (or, with
// the sequence-aware price, stores the pessimistic gain) and resets the
// accumulator and the ticket.
__global__ __launch_bounds__(kBlock) void k_filter_hub(GraphView g, Blocks bk, int optimistic,
                                                        const int32_t *part, PartView pv,
                                                        const int64_t *key, const int64_t *pen,
                                                        HubView h, int32_t *mvto,
                                                        uint8_t *accflag,
                                                        unsigned long long *counters,
                                                        int64_t *gp_out)
{
    __shared__ int64_t red[4];
    const HubChunk c = h.chunks[blockIdx.x];
    const int64_t v = h.ids[c.hub];
    const int64_t kv = key[v];
    if (kv < 0) return;  // uniform over the workgroup
    const int32_t a = bk.local(part[v]), b = (int32_t)(kv & 0xFFFF);
    int64_t acc = pessimistic_part(g, pv, key, v, a, b, kv >> 16, c.e0, c.e1, threadIdx.x, kBlock,
                                   optimistic);
    acc = block_sum(acc, red);
    if (threadIdx.x != 0) return;
    if (acc) atomic_add_i64(&h.gacc[c.hub], acc);
    __threadfence();
    if (atomicAdd(&h.ticket[c.hub], 1u) != (unsigned)(c.nchunk - 1)) return;
    __threadfence();
    const int64_t total = (int64_t)atomicExch((unsigned long long *)&h.gacc[c.hub], 0ull);
    h.ticket[c.hub] = 0;
    if (gp_out) {
        gp_out[v] = total;
        accflag[v] = 0;
        return;
    }
    const bool ok = total * 65536 - pen[v] > 0;
    accflag[v] = ok ? 1 : 0;
    if (ok) {
        mvto[v] = bk.base(part[v]) + b;
        cnt_add(counters, CNT_ACC, 1ull);
        cnt_add(counters, CNT_MOVED_DEG, (unsigned long long)(g.xadj[v + 1] - g.xadj[v]));
    }
}

hipError_t launch_filter_hub(const GraphView &g, const Blocks &bk, int optimistic,
                             const int32_t *part, const PartView &pv, const int64_t *key,
                             const int64_t *pen, const HubView &h, int32_t *mvto, uint8_t *accflag,
                             unsigned long long *counters, int64_t *gp_out, hipStream_t s)
{
    if (h.nh <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_filter_hub, dim3((unsigned)h.nchunks), dim3(kBlock), 0, s, g, bk,
                       optimistic, part, pv, key, pen, h, mvto, accflag, counters, gp_out);
    return hipGetLastError();
}

// Sequence-aware decision for each eligible candidate (id-ordered list; the
// filter pass already rejected the others): the
// move into b is priced against W[b] plus the weight change netpre[v]
// accumulated by the eligible candidates before v (Section 5.3: the penalty
// of a move depends on c(V_j + u) when it is made). Accept iff the
// pessimistic gain is positive, the move is not forbidden, and
// gain * 2^16 - P > 0.
__global__ __launch_bounds__(kBlock) void k_filter_seq(
    GraphView g, Blocks bk, const int32_t *__restrict__ part, const int32_t *__restrict__ cand,
    int64_t nc, const int64_t *__restrict__ key, const int64_t *__restrict__ gp,
    const int64_t *__restrict__ netpre, const int64_t *__restrict__ W,
    const int64_t *__restrict__ cb, int mode, int64_t hub_t, int32_t *mvto, uint8_t *accflag,
    unsigned long long *counters)
{
    __shared__ unsigned long long acc_lds, deg_lds;
    if (threadIdx.x == 0) {
        acc_lds = 0;
        deg_lds = 0;
    }
    __syncthreads();
    const int64_t stride = (int64_t)gridDim.x * kBlock;
    for (int64_t base = (int64_t)blockIdx.x * kBlock + (threadIdx.x & ~63); base < nc;
         base += stride) {
        const int64_t i = base + lane_id();
        bool take = false;
        if (i < nc) {
            const int64_t v = cand[i];
            const int64_t kv = key[v];
            const int32_t A = part[v];
            const int32_t b = bk.base(A) + (int32_t)(kv & 0xFFFF);  // global target
            const int64_t gv = gp[v];
            bool allowed = gv > 0;
            int64_t P = 0;
            if (allowed) {
                const int64_t cv = node_weight(g, v);
                const int64_t x = W[b] + netpre[v] + cv - bk.move_lmax_of(A);
                if (x > 0) {
                    if (mode == 1 || mode == 3) allowed = false;
                    else if (mode == 0) {
                        const int l = covering_slot(cb + (int64_t)b * kSlots, x);
                        if (l >= kSlots) allowed = false;
                        else P = sat_mul_pen(bk.penq_of(A)[l], cv);
                    }
                }
            }
            take = allowed && gv * 65536 - P > 0;
            accflag[v] = take ? 1 : 0;
            if (take) {
                mvto[v] = b;
                const int64_t deg = g.xadj[v + 1] - g.xadj[v];
                atomicAdd(&deg_lds, (unsigned long long)deg);
            }
        }
        wave_count(take, &acc_lds);
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        if (acc_lds) cnt_add(counters, CNT_ACC, acc_lds);
        if (deg_lds) cnt_add(counters, CNT_MOVED_DEG, deg_lds);
    }
}

hipError_t launch_filter_seq(const GraphView &g, const Blocks &bk, const int32_t *part,
                             const int32_t *cand, int64_t ne, const int64_t *key,
                             const int64_t *gp, const int64_t *netpre, const int64_t *W,
                             const int64_t *cb, int mode, int64_t hub_t, int32_t *mvto,
                             uint8_t *accflag, unsigned long long *counters, hipStream_t s)
{
    if (ne <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_filter_seq, dim3(grid_cap(ne, kBlock, 8192)), dim3(kBlock), 0, s, g, bk,
                       part, cand, ne, key, gp, netpre, W, cb, mode, hub_t, mvto, accflag,
                       counters);
    return hipGetLastError();
}

// ----------------------------------------------------------------- apply --

// S4 (and the rebalancing moves): for a move v: a -> b, part[v] = b,
// W[a] -= c(v), W[b] += c(v), and for every neighbour u
// conn[u][a] -= omega(v, u), conn[u][b] += omega(v, u). Integer atomics
// commute, so the result does not depend on the order of the moves. a and b
// are global block ids (W); the rows use their local ids.
//
// One workgroup per tile of kApplyTile consecutive nodes. Each mover of the
// tile is bookkept by its own thread (part, compact copy, mvto, block
// weights summed in LDS); then the movers' edges are spread over all threads
// of the workgroup (edge -> node by a binary search over the tile's degree
// prefix), so a mover of high degree is split over many lanes instead of
// holding up one wave. Delta mode: the two atomics per edge; rebuild mode
// (moving degrees above dirty_threshold): the neighbours' tiles are marked.
// Hubs: bookkeeping only, their edges were applied by k_apply_pre (which
// read the old part).
constexpr int kApplyTile = 1024;

template <bool LW>
__global__ __launch_bounds__(kBlock) void k_apply(GraphView g, Blocks bk, int32_t *part,
                                                   PartView pv, int32_t *conn, int64_t *W,
                                                   int32_t *mvto, int64_t hub_t,
                                                   const unsigned long long *counters,
                                                   int64_t dirty_threshold, uint8_t *dirty_flags,
                                                   int T, void *pc2, const int32_t *perm,
                                                   int64_t all_threshold, int64_t *wcp,
                                                   int ncopies)
{
    __shared__ int32_t vstart[kApplyTile + 1];
    __shared__ int64_t estart[kApplyTile];
    __shared__ uint32_t sab[kApplyTile];  // local source | local target << 16
    __shared__ int32_t scan_lds[4];
    extern __shared__ __align__(16) unsigned char lds_raw[];
    const int64_t moved_deg = (int64_t)wave_cnt_get(counters, CNT_MOVED_DEG);
    uint8_t *dirty = moved_deg > dirty_threshold ? dirty_flags : (uint8_t *)nullptr;
    // above all_threshold every tile is rebuilt: no edge walk at all
    const bool all = moved_deg > all_threshold;
    int64_t *wloc = (int64_t *)lds_raw;
    const int32_t K = bk.total();
    // LW (K <= 2048): block weights summed in LDS, a compile-time choice so
    // that the atomics are LDS ones rather than generic ones
    constexpr bool use_lds = LW;
    if (use_lds)
        for (int j = threadIdx.x; j < K; j += kBlock) wloc[j] = 0;
    __syncthreads();

    const int64_t v0 = (int64_t)blockIdx.x * kApplyTile;
    const int nt = (int)((g.n - v0) < kApplyTile ? (g.n - v0) : kApplyTile);

    // bookkeeping per mover, the movers' degrees (hubs: none) and their
    // prefix: thread t takes the tile's nodes 4t .. 4t + 3 (one 16-byte load
    // of mvto), one scan over the threads' sums
    static_assert(kApplyTile == 4 * kBlock, "four nodes per thread");
    const int i0 = 4 * threadIdx.x;
    int32_t to4[4] = {-1, -1, -1, -1};
    if (i0 + 3 < nt) {
        const int4 t4 = *(const int4 *)(mvto + v0 + i0);
        to4[0] = t4.x;
        to4[1] = t4.y;
        to4[2] = t4.z;
        to4[3] = t4.w;
    } else {
        for (int j = 0; j < 4; ++j)
            if (i0 + j < nt) to4[j] = mvto[v0 + i0 + j];
    }
    int32_t vd4[4] = {0, 0, 0, 0};
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        const int32_t to = to4[j];
        if (to < 0) continue;
        const int i = i0 + j;
        const int64_t v = v0 + i;
        const int64_t e0 = g.xadj[v], e1 = g.xadj[v + 1];
        const int32_t A = part[v];
        const uint32_t lb = (uint32_t)bk.local(to);
        if (e1 - e0 <= hub_t) {
            vd4[j] = (int32_t)(e1 - e0);
            estart[i] = e0;
            sab[i] = (uint32_t)bk.local(A) | (lb << 16);
        }
        const int64_t cv = node_weight(g, v);
        part[v] = to;
        pset((void *)pv.p, pv.bytes, v, (int32_t)lb);
        if (pc2) pset(pc2, pv.bytes, perm[v], (int32_t)lb);
        mvto[v] = -1;
        if (use_lds) {  // (LDS atomics, not generic ones)
            atomicAdd((unsigned long long *)&wloc[A], (unsigned long long)(-cv));
            atomicAdd((unsigned long long *)&wloc[to], (unsigned long long)cv);
        } else {
            atomicAdd((unsigned long long *)&W[A], (unsigned long long)(-cv));
            atomicAdd((unsigned long long *)&W[to], (unsigned long long)cv);
        }
    }
    int32_t run;
    {
        const int32_t sum = vd4[0] + vd4[1] + vd4[2] + vd4[3];
        const int32_t inc = block_incl_scan(sum, scan_lds, &run);
        int32_t x = inc - sum;
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            if (i0 + j < nt) vstart[i0 + j] = x;
            x += vd4[j];
        }
    }
    if (threadIdx.x == 0) vstart[nt] = run;
    __syncthreads();

    // the movers' edges, kEdgeUnroll per thread and step so that their loads overlap
    const int32_t E = all ? 0 : run;
    const int32_t k = bk.k;
    for (int32_t p0 = threadIdx.x; p0 < E; p0 += kBlock * kEdgeUnroll) {
        // loads from clamped indices without a branch, so that they are in
        // flight together (a slot past the last edge rereads it, unused)
        bool ok[kEdgeUnroll];
        int node[kEdgeUnroll];
        int64_t e[kEdgeUnroll];
        int32_t u[kEdgeUnroll];
#pragma unroll
        for (int i = 0; i < kEdgeUnroll; ++i) {
            const int32_t p = p0 + i * kBlock;
            ok[i] = p < E;
            const int32_t pc = ok[i] ? p : E - 1;
            node[i] = upper_index(vstart, nt, pc);
            e[i] = estart[node[i]] + (pc - vstart[node[i]]);
        }
#pragma unroll
        for (int i = 0; i < kEdgeUnroll; ++i) u[i] = g.adjncy[e[i]];
        if (dirty) {
#pragma unroll
            for (int i = 0; i < kEdgeUnroll; ++i)
                if (ok[i]) mark_dirty(dirty, u[i] / T);
        } else {
            int32_t w[kEdgeUnroll];
#pragma unroll
            for (int i = 0; i < kEdgeUnroll; ++i) w[i] = edge_weight(g, e[i]);
#pragma unroll
            for (int i = 0; i < kEdgeUnroll; ++i) {
                if (!ok[i]) continue;
                const uint32_t ab = sab[node[i]];
                int32_t *row = conn + (int64_t)u[i] * k;
                atomicAdd(&row[ab & 0xFFFF], -w[i]);
                atomicAdd(&row[ab >> 16], w[i]);
            }
        }
    }
    if (use_lds) {
        // with copies (wcp) into this workgroup's copy, which the next
        // rebalancing begin adds into W
        int64_t *Wd = wcp ? wcp + (int64_t)(blockIdx.x % (unsigned)ncopies) * K : W;
        __syncthreads();
        for (int j = threadIdx.x; j < K; j += kBlock)
            if (wloc[j]) atomic_add_i64(&Wd[j], wloc[j]);
    }
}

// The term of the directed entry (v, u) in the change of 2 * cut when v
// moves a -> b and u sits in pu with target tu (-1: u stays); see
// k_apply_pre.
__device__ __forceinline__ int64_t cut_term(int32_t a, int32_t b, int32_t pu, int32_t tu,
                                            int32_t w)
{
    const int32_t pn = tu >= 0 ? tu : pu;
    const int x = (b != pn ? 1 : 0) - (a != pu ? 1 : 0);
    return (int64_t)w * x * (tu >= 0 ? 1 : 2);
}

// Before k_apply, in one launch: the hub movers' edges, one workgroup per hub
// chunk (part of a hub is still its source block here), and with CUT the
// change of 2 * cut the moves make, summed into counters[CNT_CUT2_DELTA]
// (two's complement) by the hub chunks for the hub movers and by tiles of
// kApplyTile nodes (the workgroups after the chunks) for the others. Nothing
// here changes part or mvto, which k_apply updates afterwards.
//
// Hub rows: when the apply rebuilds the table, the first chunk of every hub
// clears the hub's own row, which the refresh after the apply rebuilds; in
// the delta mode hub rows get their deltas like every other row.
//
// The cut (Section 2) is a sum over the directed entries of the symmetric
// adjacency, each edge twice; an entry's term w [p(v) != p(u)] changes only
// if v or u moves. The entries out of a mover v are summed here; an entry
// into v from a neighbour u that stays has the same term as (v, u), so such
// an entry counts twice, and one between two movers is met from both ends.
// With the moving degrees above cut_max (the apply rebuilds tiles, or the
// walk would cost more than a recount) nothing is summed and
// counters[CNT_CUT_STALE] is raised, so that the cut is recounted.
template <bool CUT>
__global__ __launch_bounds__(kBlock) void k_apply_pre(GraphView g, Blocks bk,
                                                       const int32_t *__restrict__ part,
                                                       int32_t *conn,
                                                       const int32_t *__restrict__ mvto,
                                                       HubView h, unsigned long long *counters,
                                                       int64_t dirty_threshold, uint8_t *dirty,
                                                       int T, int64_t all_threshold, int64_t hub_t,
                                                       int64_t cut_max)
{
    __shared__ int32_t vstart[CUT ? kApplyTile + 1 : 1];
    __shared__ int64_t estart[CUT ? kApplyTile : 1];
    __shared__ int32_t sa[CUT ? kApplyTile : 1], sb[CUT ? kApplyTile : 1];
    __shared__ int32_t scan_lds[4];
    __shared__ int64_t red[4];
    const int32_t k = bk.k;
    const int64_t moved_deg = (int64_t)wave_cnt_get(counters, CNT_MOVED_DEG);
    const bool cut = CUT && moved_deg <= cut_max;
    if (CUT && !cut && blockIdx.x == 0 && threadIdx.x == 0) cnt_add(counters, CNT_CUT_STALE, 1ull);
    const int64_t nhc = h.nh > 0 ? h.nchunks : 0;
    int64_t acc = 0;
    if ((int64_t)blockIdx.x < nhc) {
        const HubChunk c = h.chunks[blockIdx.x];
        const int64_t v = h.ids[c.hub];
        const bool rebuild = moved_deg > dirty_threshold;
        if (rebuild && c.e0 == g.xadj[v])
            for (int j = threadIdx.x; j < k; j += kBlock) conn[v * (int64_t)k + j] = 0;
        const int32_t B = mvto[v];
        if (B < 0) return;  // uniform over the workgroup
        if (rebuild) {
            if (moved_deg <= all_threshold)  // else every tile is rebuilt
                for (int64_t e = c.e0 + threadIdx.x; e < c.e1; e += kBlock)
                    mark_dirty(dirty, g.adjncy[e] / T);
            return;
        }
        const int32_t A = part[v];
        const int32_t a = bk.local(A), b = bk.local(B);
        // kHubUnroll edges per thread and step, their loads in flight together
        // (a slot past the chunk rereads its last edge, unused)
        constexpr int kHubUnroll = 8;
        for (int64_t e0 = c.e0 + threadIdx.x; e0 < c.e1; e0 += (int64_t)kBlock * kHubUnroll) {
            bool ok[kHubUnroll];
            int32_t u[kHubUnroll], w[kHubUnroll], pu[kHubUnroll], tu[kHubUnroll];
#pragma unroll
            for (int i = 0; i < kHubUnroll; ++i) {
                const int64_t e = e0 + (int64_t)i * kBlock;
                ok[i] = e < c.e1;
                const int64_t ec = ok[i] ? e : c.e1 - 1;
                u[i] = g.adjncy[ec];
                w[i] = edge_weight(g, ec);
            }
            if (cut) {
#pragma unroll
                for (int i = 0; i < kHubUnroll; ++i) {
                    pu[i] = part[u[i]];
                    tu[i] = mvto[u[i]];
                }
            }
#pragma unroll
            for (int i = 0; i < kHubUnroll; ++i) {
                if (!ok[i]) continue;
                int32_t *row = conn + (int64_t)u[i] * k;
                atomicAdd(&row[a], -w[i]);
                atomicAdd(&row[b], w[i]);
                if (cut) acc += cut_term(A, B, pu[i], tu[i], w[i]);
            }
        }
    } else {
        if (!cut) return;  // uniform over the grid
        const int64_t v0 = ((int64_t)blockIdx.x - nhc) * kApplyTile;
        const int nt = (int)((g.n - v0) < kApplyTile ? (g.n - v0) : kApplyTile);
        const int i0 = 4 * threadIdx.x;
        int32_t vd4[4] = {0, 0, 0, 0};
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const int i = i0 + j;
            if (i >= nt) continue;
            const int64_t v = v0 + i;
            const int32_t to = mvto[v];
            if (to < 0) continue;
            const int64_t e0 = g.xadj[v], e1 = g.xadj[v + 1];
            if (e1 - e0 > hub_t) continue;  // a hub: its chunks
            vd4[j] = (int32_t)(e1 - e0);
            estart[i] = e0;
            sa[i] = part[v];
            sb[i] = to;
        }
        int32_t run;
        {
            const int32_t sum = vd4[0] + vd4[1] + vd4[2] + vd4[3];
            const int32_t inc = block_incl_scan(sum, scan_lds, &run);
            int32_t x = inc - sum;
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                if (i0 + j < nt) vstart[i0 + j] = x;
                x += vd4[j];
            }
        }
        if (threadIdx.x == 0) vstart[nt] = run;
        __syncthreads();
        const int32_t E = run;
        for (int32_t p0 = threadIdx.x; p0 < E; p0 += kBlock * kEdgeUnroll) {
            // loads from clamped indices without a branch, in flight together
            bool ok[kEdgeUnroll];
            int node[kEdgeUnroll];
            int32_t u[kEdgeUnroll], w[kEdgeUnroll], pu[kEdgeUnroll], tu[kEdgeUnroll];
#pragma unroll
            for (int i = 0; i < kEdgeUnroll; ++i) {
                const int32_t p = p0 + i * kBlock;
                ok[i] = p < E;
                const int32_t pc = ok[i] ? p : E - 1;
                node[i] = upper_index(vstart, nt, pc);
                const int64_t e = estart[node[i]] + (pc - vstart[node[i]]);
                u[i] = g.adjncy[e];
                w[i] = edge_weight(g, e);
            }
#pragma unroll
            for (int i = 0; i < kEdgeUnroll; ++i) {
                pu[i] = part[u[i]];
                tu[i] = mvto[u[i]];
            }
#pragma unroll
            for (int i = 0; i < kEdgeUnroll; ++i)
                if (ok[i]) acc += cut_term(sa[node[i]], sb[node[i]], pu[i], tu[i], w[i]);
        }
    }
    if (CUT) {
        acc = block_sum(acc, red);
        if (threadIdx.x == 0 && acc != 0) cnt_add(counters, CNT_CUT2_DELTA, (unsigned long long)acc);
    }
}

hipError_t launch_apply(const GraphView &g, const Blocks &bk, int32_t *part, const PartView &pv,
                        int32_t *conn, int64_t *W, int32_t *mvto, int64_t hub_t,
                        const HubView &h, unsigned long long *counters,
                        int64_t dirty_threshold, uint8_t *dirty, const GraphView &tg,
                        const PartView &tpv, void *pc2, const int32_t *perm,
                        int64_t all_threshold, hipStream_t s, bool cut_delta, int64_t *wcp,
                        int ncopies)
{
    if (g.n <= 0) return hipSuccess;
    if (!wcp || ncopies < 2) wcp = nullptr;
    const int32_t k = bk.k;
    const int T = gain_tile_nodes(k, g.n);
    const size_t lds = bk.total() <= 2048 ? (size_t)bk.total() * 8 : 0;
    const int64_t tiles = (g.n + kApplyTile - 1) / kApplyTile;
    hipError_t e;
    // the hub movers and, for one graph, the change of the cut (a walk over
    // more moving degrees than n / 8, three loads per edge and two of them
    // gathers, costs more than the recount's one table line per node)
    const int64_t nhc = h.nh > 0 ? h.nchunks : 0;
    const int64_t cut_max = std::min<int64_t>(dirty_threshold, g.n / 8);
    if (cut_delta)
        hipLaunchKernelGGL(k_apply_pre<true>, dim3((unsigned)(nhc + tiles)), dim3(kBlock), 0, s, g,
                           bk, part, conn, mvto, h, counters, dirty_threshold, dirty, T,
                           all_threshold, hub_t, cut_max);
    else if (nhc > 0)
        hipLaunchKernelGGL(k_apply_pre<false>, dim3((unsigned)nhc), dim3(kBlock), 0, s, g, bk, part,
                           conn, mvto, h, counters, dirty_threshold, dirty, T, all_threshold, hub_t,
                           cut_max);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    if (bk.total() <= 2048)
        hipLaunchKernelGGL(k_apply<true>, dim3((unsigned)tiles), dim3(kBlock), lds, s, g, bk, part,
                           pv, conn, W, mvto, hub_t, counters, dirty_threshold, dirty, T, pc2, perm,
                           all_threshold, wcp, ncopies);
    else
        hipLaunchKernelGGL(k_apply<false>, dim3((unsigned)tiles), dim3(kBlock), lds, s, g, bk, part,
                           pv, conn, W, mvto, hub_t, counters, dirty_threshold, dirty, T, pc2, perm,
                           all_threshold, nullptr, 1);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    // rebuild the marked tiles and the hub rows (nothing in the delta mode)
    return launch_gain_refresh(tg, k, tpv, conn, hub_t, h, dirty, counters, dirty_threshold,
                               all_threshold, s);
}

// ----------------------------------------------------------------- stats --

// iters < 0: the statistics follow one speculative rebalancing sub-iteration
// that no other followed: one sub-iteration counts if blocks were overloaded
// when rebalancing began, and the status is 1 iff some still are.
__global__ void k_stats_final(int64_t *stats, const unsigned long long *c, int64_t lmax,
                              int64_t iters, int64_t status)
{
    // one wave: every lane reads its copy of each counter
    const int64_t cb = (int64_t)wave_cnt_get(c, CNT_CUT2_BEFORE) / 2;
    const int64_t cm = (int64_t)wave_cnt_get(c, CNT_CUT2_MOVES) / 2;
    const int64_t ca = (int64_t)wave_cnt_get(c, CNT_CUT2_AFTER) / 2;
    const int64_t nc = (int64_t)wave_cnt_get(c, CNT_CAND);
    const int64_t na = (int64_t)wave_cnt_get(c, CNT_ACC);
    const int64_t nr = (int64_t)wave_cnt_get(c, CNT_REBAL_MOVES);
    const unsigned long long over0 = wave_cnt_get(c, CNT_OVER0);
    const unsigned long long over = wave_cnt_get(c, CNT_OVER);
    if (iters < 0) {
        iters = over0 != 0 ? 1 : 0;
        status = over != 0 ? 1 : 0;
    }
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    stats[0] = lmax;
    stats[1] = cb;
    stats[2] = cm;
    stats[3] = ca;
    stats[4] = nc;
    stats[5] = na;
    stats[6] = nr;
    stats[7] = iters;
    stats[8] = status;
    for (int i = 9; i < 12; ++i) stats[i] = 0;
}

// dst = src (summed over the copies) for a spread counter.
__global__ void k_cnt_copy(unsigned long long *c, int dst, int src)
{
    wave_cnt_set(c, dst, wave_cnt_get(c, src));
}

hipError_t launch_cnt_copy(unsigned long long *counters, int dst, int src, hipStream_t s)
{
    hipLaunchKernelGGL(k_cnt_copy, dim3(1), dim3(64), 0, s, counters, dst, src);
    return hipGetLastError();
}

__global__ void k_cnt_set(unsigned long long *c, int slot, unsigned long long v)
{
    wave_cnt_set(c, slot, v);
}

hipError_t launch_cnt_set(unsigned long long *counters, int slot, unsigned long long v,
                          hipStream_t s)
{
    hipLaunchKernelGGL(k_cnt_set, dim3(1), dim3(64), 0, s, counters, slot, v);
    return hipGetLastError();
}

hipError_t launch_stats_final(int64_t *stats, const unsigned long long *counters, int64_t lmax,
                              int64_t iters, int64_t status, hipStream_t s)
{
    hipLaunchKernelGGL(k_stats_final, dim3(1), dim3(64), 0, s, stats, counters, lmax, iters, status);
    return hipGetLastError();
}

__global__ void k_export_moves(int64_t n, const int64_t *key, const int64_t *pen,
                               const uint8_t *accflag, int32_t *target, int64_t *score,
                               int64_t *pen_out, uint8_t *accept)
{
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; v < n; v += stride) {
        const int64_t kv = key[v];
        const bool c = kv >= 0;
        if (target) target[v] = c ? (int32_t)(kv & 0xFFFF) : -1;
        if (score) score[v] = c ? (kv >> 16) : 0;
        if (pen_out) pen_out[v] = c ? pen[v] : 0;
        if (accept) accept[v] = c ? accflag[v] : 0;
    }
}

hipError_t launch_export_moves(int64_t n, const int64_t *key, const int64_t *pen,
                               const uint8_t *accflag, int32_t *target, int64_t *score,
                               int64_t *pen_out, uint8_t *accept, hipStream_t s)
{
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_export_moves, dim3(grid_cap(n, kBlock * 4, 4096)), dim3(kBlock), 0, s, n,
                       key, pen, accflag, target, score, pen_out, accept);
    return hipGetLastError();
}

}  // namespace upr
