// Host side of libupr: the C ABI declared in include/upr.h.
//
// A context owns the device workspace (grown on demand) and a small pinned
// buffer for the counters the rebalancing loop decides on. A plan holds a
// prepared graph: weighted degrees, total node weight and the hub list with
// its edge chunks. Every round is a fixed sequence of kernels on the caller's
// stream; the only host decisions are the rebalancing sub-iterations.
#include "upr.h"
#include "upr_common.h"

#include <algorithm>
#include <atomic>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <string>
#include <vector>

using namespace upr;

namespace {

constexpr int64_t kHubChunkEdges = 4096;
constexpr int64_t kDefaultHubThreshold = 4096;
constexpr int64_t kRelabelMinNodes = 65536;  // relabel the table build's adjacency from here on
constexpr int64_t kChunkEntries = int64_t(1) << 20;  // rebalancing id-chunk sums per side

constexpr int kCaptureKey = 16;       // words of a captured span's key
constexpr size_t kCaptureMax = 16;    // captured spans kept per context

struct Timing {
    uint32_t mask = 0;  // phases timed (bit p = phase p)
    std::vector<hipEvent_t> pool;
    struct Pending {
        int phase;
        hipEvent_t a, b;
    };
    std::vector<Pending> pending;
    double ms[UPR_NUM_PHASES] = {0};
    int64_t counts[UPR_NUM_PHASES] = {0};
};

int64_t env_int(const char *name, int64_t dflt)
{
    const char *s = getenv(name);
    if (!s || !*s) return dflt;
    return strtoll(s, nullptr, 10);
}

}  // namespace

struct upr_ctx {
    int device = 0;
    // device address of the no-allocation scratch array on this device (null:
    // not available, upr_edge_cut_noalloc then fails)
    void *noalloc = nullptr;
    // target bucket size of the sequence-aware price's split segments
    // (UPR_SEQ_BUCKET_AVG, read at creation; never below the default, which
    // sizes the bucket tables)
    int32_t seq_bucket_avg = 0;
    char err[512] = {0};  // last error (fixed storage: reporting an error allocates nothing)
    // workspace
    int64_t cap_n = 0, cap_k = 0;
    int64_t *key = nullptr, *pen = nullptr;
    int64_t *key2 = nullptr;  // [n] the candidates' keys in the plan's label order
    uint8_t *accflag = nullptr;
    int32_t *mvto = nullptr;     // [n] pending move target, -1 = none
    uint8_t *dirty = nullptr;    // [n] gain-table tiles to rebuild
    uint16_t *pc = nullptr;      // [n] compact copy of part for neighbour gathers
    uint16_t *pc2 = nullptr;     // [n] the same in the plan's label order (table build)
    int32_t *inner = nullptr;    // [n] conn[v][part[v]] of non-hub nodes, from the table build
    // sequence-aware penalty
    int64_t *gp = nullptr;       // [n] pessimistic gains of candidates
    uint8_t *avail = nullptr;    // [n] available for rebalancing
    int32_t *cand = nullptr;     // [n] eligible candidates in id order
    uint64_t *ev_key = nullptr, *ev_key2 = nullptr;  // [2n]
    uint32_t *ev_val = nullptr, *ev_val2 = nullptr;  // [2n]
    int64_t *ev_prefix = nullptr;                     // [2n]
    int64_t *netpre = nullptr;                        // [n]
    unsigned long long *seg_cur = nullptr;            // [K]
    int32_t *seg_slist = nullptr;                     // [K]
    int32_t *seg_meta = nullptr;                      // [4]
    int64_t *seg_off = nullptr;                       // [K + 1]
    int32_t *seg_boff = nullptr, *seg_cpre = nullptr; // [K + 1]
    int32_t *seg_bblk = nullptr;                      // [NB] (NB = seq_bucket_bound)
    int64_t *seg_bpos = nullptr, *seg_bsize = nullptr, *seg_bdel = nullptr;
    int64_t *seg_scan_c = nullptr, *seg_scan_d = nullptr;
    unsigned long long *seg_bcnt = nullptr;
    uint64_t *seg_spl = nullptr;
    void *seq_temp = nullptr;
    size_t seq_temp_size = 0;
    int64_t *bucket = nullptr, *penq = nullptr;
    int64_t *lmax1 = nullptr, *srcl1 = nullptr;  // one graph: its L_max (device, one entry each)
    int64_t *pen1 = nullptr;     // [K] unit-weight penalty per target block
    unsigned long long *counters = nullptr;
    unsigned long long *flags = nullptr;  // validation flags [4]
    RebalWs rb{};
    int64_t *stat_wsp = nullptr;  // [stat_copies * K] copies of the statistics pass's W sums
    int64_t *stat_bsp = nullptr;  // [stat_copies * K * kSlots] and of its slot histogram
    int stat_copies = 1;
    int64_t *apply_wcp = nullptr;  // [kApplyCopiesMax * K] copies of the applies' W sums
    unsigned long long *pinned = nullptr;  // host mirror of the counters' copies
    unsigned long long cnt[CNT_COUNT] = {0};  // their sums, after sync_counters
    // host-coherent [1 + CNT_COUNT]: a sequence number, then the counter sums
    // published by the rebalancer's begin kernel (null: not available)
    unsigned long long *pub = nullptr;
    unsigned long long *pub_d = nullptr;  // its device address
    unsigned long long pub_seq = 0;
    // pinned host area of the batches run on this context (grown on demand;
    // pinned allocations are slow, and batches are rebuilt often by a server)
    int64_t *bpinned = nullptr;
    int64_t bpinned_cap = 0;  // int64 entries
    bool rb_dirty = false;
    Timing timing;
    // captured move phases (upr_capture_enable): a non-blocking stream of the
    // context's own (default priority) to capture on, and the graphs by key
    bool capture = false;
    hipStream_t cap_stream = nullptr;
    struct Captured {
        uint64_t key[kCaptureKey];
        hipGraphExec_t exec;
    };
    std::vector<Captured> captured;
    uint64_t ws_gen = 0;  // bumped whenever the workspace is reallocated
    // carry records of upr_batch_carry (device, grown on demand)
    int64_t *carry = nullptr;
    int64_t carry_cap = 0;
    // interleaved best prefix (allocated on first use)
    BpWs bp{};
    int64_t bp_cap_n = 0;
    int32_t bp_cap_k = 0;
};

struct upr_plan {
    upr_ctx *ctx = nullptr;
    uint64_t serial = 0;  // unique per plan created in this process (keys of captured spans)
    int device = 0;  // the context's device (a plan may outlive its context)
    GraphView g{};
    int64_t nnz = 0, total = 0, maxdeg = 0, maxwdeg = 0, maxvw = 0;
    int32_t *wdeg = nullptr;
    int32_t nh = 0;
    int32_t *hub_ids = nullptr;
    HubChunk *chunks = nullptr;
    int64_t nchunks = 0;
    int64_t *gacc = nullptr;
    unsigned int *hub_ticket = nullptr;
    uint32_t *hub_bits = nullptr;  // [ceil(n/32)]
    int64_t hub_t = kDefaultHubThreshold;
    int64_t dirty_threshold = 0;  // moved-degree sum above which tiles are rebuilt
    int64_t all_threshold = 0;    // ... above which every tile is (nothing is marked)
    // neighbour ids renumbered by descending degree for the table build (null:
    // not built, the table build reads the graph as given)
    int32_t *adj_r = nullptr;  // [nnz] perm[adjncy[e]]
    int32_t *perm = nullptr;   // [n] label of node v
    int32_t *order = nullptr;  // [n] node of label i

    HubView hubs() const
    {
        return HubView{nh, hub_ids, chunks, nchunks, gacc, hub_bits, hub_ticket};
    }
    // the graph as the table build reads it
    GraphView table_graph() const
    {
        GraphView t = g;
        if (adj_r) t.adjncy = adj_r;
        return t;
    }
};

// A batch: the disjoint union of ng graphs with k blocks each (see Blocks),
// its plan, and the per-graph constants and statistics.
struct upr_batch {
    upr_ctx *ctx = nullptr;
    int device = 0;  // the context's device (a batch may outlive its context)
    upr_plan *plan = nullptr;  // plan of the union graph
    int32_t ng = 0, k = 0, eps_num = 0, eps_den = 0;
    int64_t n = 0, nnz = 0, max_n = 0;
    // the union CSR (owned)
    int64_t *xadj = nullptr;
    int32_t *adjncy = nullptr, *adjwgt = nullptr, *vwgt = nullptr;
    // host copies: node offsets [ng + 1], L_max, largest node weight, node-weighted flag
    std::vector<int64_t> off, lmax, maxvw;
    std::vector<uint8_t> weighted;
    // device: node offsets, L_max, rebalancing source bound, penalty tables,
    // statistics [ng][GS_COUNT], per-graph rebalancing results [ng][3]
    int64_t *goff_d = nullptr, *lmax_d = nullptr, *srcl_d = nullptr, *penq_d = nullptr;
    int64_t *gstat_d = nullptr, *host3_d = nullptr;
    // pinned mirrors (in the context's batch area, valid while the batch runs)
    int64_t *gstat_h = nullptr, *srcl_h = nullptr, *penq_h = nullptr, *host3_h = nullptr;
    // statistics pass: nodes per workgroup (at most the smallest graph) and
    // the most blocks the graphs of such a range own
    int64_t stats_span = 0;
    int32_t stats_window = 0;
};

namespace {

int fail(upr_ctx *c, int code, const char *fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    if (c) snprintf(c->err, sizeof c->err, "%s", buf);
    return code;
}

#define HIP_TRY(ctx, expr)                                                                  \
    do {                                                                                    \
        hipError_t e_ = (expr);                                                             \
        if (e_ != hipSuccess)                                                               \
            return fail((ctx), UPR_E_HIP, "%s failed: %s", #expr, hipGetErrorString(e_));  \
    } while (0)

template <typename T>
hipError_t dalloc(T **p, int64_t count)
{
    *p = nullptr;
    if (count <= 0) count = 1;
    return hipMalloc((void **)p, sizeof(T) * (size_t)count);
}

template <typename T>
void dfree(T *&p)
{
    if (p) (void)hipFree((void *)p);
    p = nullptr;
}

// The captured spans of a context (their kernels hold workspace addresses).
void drop_captured(upr_ctx *c)
{
    for (auto &g : c->captured) (void)hipGraphExecDestroy(g.exec);
    c->captured.clear();
}

void free_workspace(upr_ctx *c)
{
    dfree(c->key);
    dfree(c->key2);
    dfree(c->pen);
    dfree(c->accflag);
    dfree(c->mvto);
    dfree(c->dirty);
    dfree(c->pc);
    dfree(c->pc2);
    dfree(c->inner);
    dfree(c->gp);
    dfree(c->avail);
    dfree(c->cand);
    dfree(c->ev_key);
    dfree(c->ev_key2);
    dfree(c->ev_val);
    dfree(c->ev_val2);
    dfree(c->ev_prefix);
    dfree(c->netpre);
    dfree(c->seg_slist);
    dfree(c->seg_meta);
    dfree(c->seg_cur);
    dfree(c->seg_off);
    dfree(c->seg_boff);
    dfree(c->seg_cpre);
    dfree(c->seg_bblk);
    dfree(c->seg_bpos);
    dfree(c->seg_bsize);
    dfree(c->seg_bdel);
    dfree(c->seg_scan_c);
    dfree(c->seg_scan_d);
    dfree(c->seg_bcnt);
    dfree(c->seg_spl);
    if (c->seq_temp) (void)hipFree(c->seq_temp);
    c->seq_temp = nullptr;
    c->seq_temp_size = 0;
    dfree(c->bucket);
    dfree(c->pen1);
    dfree(c->rb.rtgt);
    dfree(c->rb.rbeta);
    dfree(c->rb.W0);
    dfree(c->rb.hist_src);
    dfree(c->stat_wsp);
    dfree(c->apply_wcp);
    dfree(c->stat_bsp);
    dfree(c->rb.hist_tgt);
    dfree(c->rb.cbeta_src);
    dfree(c->rb.cbeta_tgt);
    dfree(c->rb.need_src);
    dfree(c->rb.room_tgt);
    dfree(c->rb.theta_src);
    dfree(c->rb.theta_tgt);
    dfree(c->rb.chunk_src);
    dfree(c->rb.chunk_tgt);
    c->cap_n = c->cap_k = 0;
}

// Grow the workspace to hold n nodes and k blocks (all graphs' blocks for a
// batch).
int ensure_workspace(upr_ctx *c, int64_t n, int32_t k)
{
    if (n <= c->cap_n && k <= c->cap_k && !c->rb_dirty) return UPR_OK;
    const int64_t N = std::max<int64_t>(std::max(n, c->cap_n), 1);
    const int64_t K = std::max<int64_t>(std::max<int64_t>(k, c->cap_k), 2);
    HIP_TRY(c, hipDeviceSynchronize());
    free_workspace(c);
    drop_captured(c);  // their kernels hold the old workspace's addresses
    ++c->ws_gen;
    const int64_t NB = seq_bucket_bound(N, (int)K);
    bool ok = dalloc(&c->key, N) == hipSuccess && dalloc(&c->pen, N) == hipSuccess &&
              dalloc(&c->key2, N) == hipSuccess &&
              dalloc(&c->accflag, N) == hipSuccess && dalloc(&c->mvto, N) == hipSuccess &&
              dalloc(&c->dirty, N) == hipSuccess && dalloc(&c->gp, N) == hipSuccess &&
              dalloc(&c->pc, N) == hipSuccess && dalloc(&c->pc2, N) == hipSuccess &&
              dalloc(&c->inner, N) == hipSuccess &&
              dalloc(&c->avail, N) == hipSuccess && dalloc(&c->cand, N) == hipSuccess &&
              dalloc(&c->ev_key, 2 * N) == hipSuccess &&
              dalloc(&c->ev_key2, 2 * N) == hipSuccess && dalloc(&c->ev_val, 2 * N) == hipSuccess &&
              dalloc(&c->ev_val2, 2 * N) == hipSuccess && dalloc(&c->ev_prefix, 2 * N) == hipSuccess &&
              dalloc(&c->netpre, N) == hipSuccess &&
              dalloc(&c->seg_slist, K) == hipSuccess && dalloc(&c->seg_meta, 4) == hipSuccess &&
              dalloc(&c->seg_cur, std::max<int64_t>(K, (int64_t)kSegCopyEntries * kSegCopyPad)) == hipSuccess && dalloc(&c->seg_off, K + 1) == hipSuccess &&
              dalloc(&c->seg_boff, K + 1) == hipSuccess && dalloc(&c->seg_cpre, K + 1) == hipSuccess &&
              dalloc(&c->seg_bblk, NB) == hipSuccess && dalloc(&c->seg_bpos, NB) == hipSuccess &&
              dalloc(&c->seg_bsize, NB) == hipSuccess && dalloc(&c->seg_bdel, NB) == hipSuccess &&
              dalloc(&c->seg_scan_c, NB) == hipSuccess &&
              dalloc(&c->seg_scan_d, NB) == hipSuccess && dalloc(&c->seg_bcnt, NB) == hipSuccess &&
              dalloc(&c->seg_spl, NB) == hipSuccess &&
              dalloc(&c->bucket, K * kSlots) == hipSuccess && dalloc(&c->pen1, K) == hipSuccess &&
              dalloc(&c->rb.rtgt, N) == hipSuccess && dalloc(&c->rb.rbeta, N) == hipSuccess &&
              dalloc(&c->rb.W0, K) == hipSuccess &&
              dalloc(&c->rb.hist_src, rb_hist_copies(K) * K * kRbBuckets) == hipSuccess &&
              dalloc(&c->stat_wsp, stats_copies(K) * K) == hipSuccess &&
              dalloc(&c->apply_wcp, (int64_t)kApplyCopiesMax * K) == hipSuccess &&
              dalloc(&c->stat_bsp, stats_copies(K) * K * kSlots) == hipSuccess &&
              dalloc(&c->rb.hist_tgt, rb_hist_copies(K) * K * kRbBuckets) == hipSuccess &&
              dalloc(&c->rb.cbeta_src, K) == hipSuccess && dalloc(&c->rb.cbeta_tgt, K) == hipSuccess &&
              dalloc(&c->rb.need_src, K) == hipSuccess && dalloc(&c->rb.room_tgt, K) == hipSuccess &&
              dalloc(&c->rb.theta_src, K) == hipSuccess && dalloc(&c->rb.theta_tgt, K) == hipSuccess &&
              dalloc(&c->rb.chunk_src, kChunkEntries) == hipSuccess &&
              dalloc(&c->rb.chunk_tgt, kChunkEntries) == hipSuccess;
    if (!ok) {
        (void)hipGetLastError();
        free_workspace(c);
        return fail(c, UPR_E_NOMEM, "workspace allocation failed for n=%lld k=%lld", (long long)N,
                    (long long)K);
    }
    c->rb.hist_copies = rb_hist_copies(K);
    c->stat_copies = stats_copies(K);
    HIP_TRY(c, hipMemset(c->stat_wsp, 0, sizeof(int64_t) * c->stat_copies * K));
    HIP_TRY(c, hipMemset(c->apply_wcp, 0, sizeof(int64_t) * kApplyCopiesMax * K));
    HIP_TRY(c, hipMemset(c->stat_bsp, 0, sizeof(int64_t) * c->stat_copies * K * kSlots));
    HIP_TRY(c, hipMemset(c->rb.hist_src, 0, sizeof(int64_t) * c->rb.hist_copies * K * kRbBuckets));
    HIP_TRY(c, hipMemset(c->rb.hist_tgt, 0, sizeof(int64_t) * c->rb.hist_copies * K * kRbBuckets));
    HIP_TRY(c, hipMemset(c->rb.chunk_src, 0, sizeof(int64_t) * kChunkEntries));
    HIP_TRY(c, hipMemset(c->rb.chunk_tgt, 0, sizeof(int64_t) * kChunkEntries));
    HIP_TRY(c, hipMemset(c->key, 0xff, sizeof(int64_t) * N));
    HIP_TRY(c, hipMemset(c->mvto, 0xff, sizeof(int32_t) * N));
    HIP_TRY(c, hipMemset(c->dirty, 0, N));
    c->seq_temp_size = seq_temp_bytes(N);
    if (hipMalloc(&c->seq_temp, c->seq_temp_size) != hipSuccess) {
        (void)hipGetLastError();
        c->seq_temp = nullptr;
        free_workspace(c);
        return fail(c, UPR_E_NOMEM, "workspace allocation failed for n=%lld", (long long)N);
    }
    HIP_TRY(c, hipDeviceSynchronize());
    c->cap_n = N;
    c->cap_k = K;
    c->rb_dirty = false;
    return UPR_OK;
}

void free_bp(upr_ctx *c)
{
    BpWs &w = c->bp;
    for (void **p : {(void **)&w.part0, (void **)&w.rbrec, (void **)&w.W0, (void **)&w.fm,
                     (void **)&w.fr, (void **)&w.ids, (void **)&w.ids2, (void **)&w.mlist,
                     (void **)&w.rlist, (void **)&w.rfrom, (void **)&w.rto, (void **)&w.tau,
                     (void **)&w.stepof, (void **)&w.rc, (void **)&w.rwi, (void **)&w.rin_inc,
                     (void **)&w.rin_key, (void **)&w.k0, (void **)&w.k1, (void **)&w.evs,
                     (void **)&w.d0, (void **)&w.d1, (void **)&w.acc, (void **)&w.need,
                     (void **)&w.tcum, (void **)&w.pos, (void **)&w.ecnt, (void **)&w.eoff,
                     (void **)&w.roff, (void **)&w.rinoff, (void **)&w.cstep, (void **)&w.rbefore,
                     (void **)&w.over_incl, (void **)&w.stepgain, (void **)&w.gain_incl,
                     (void **)&w.best_g, (void **)&w.best_j, (void **)&w.cnt, (void **)&w.changed,
                     (void **)&w.scal, &w.temp}) {
        if (*p) (void)hipFree(*p);
        *p = nullptr;
    }
    w.rcnt = nullptr;
    w.temp_bytes = 0;
    c->bp_cap_n = 0;
    c->bp_cap_k = 0;
}

// The best-prefix workspace for n nodes and K blocks.
int ensure_bp(upr_ctx *c, int64_t n, int32_t K)
{
    if (n <= c->bp_cap_n && K <= c->bp_cap_k) return UPR_OK;
    const int64_t N = std::max<int64_t>(std::max(n, c->bp_cap_n), 1);
    const int32_t KK = std::max<int32_t>(std::max(K, c->bp_cap_k), 2);
    HIP_TRY(c, hipDeviceSynchronize());
    free_bp(c);
    BpWs &w = c->bp;
    bool ok = dalloc(&w.part0, N) == hipSuccess && dalloc(&w.rbrec, N) == hipSuccess &&
              dalloc(&w.W0, KK) == hipSuccess && dalloc(&w.fm, N) == hipSuccess &&
              dalloc(&w.fr, N) == hipSuccess && dalloc(&w.ids, N) == hipSuccess &&
              dalloc(&w.ids2, N) == hipSuccess && dalloc(&w.mlist, N) == hipSuccess &&
              dalloc(&w.rlist, N) == hipSuccess && dalloc(&w.rfrom, N) == hipSuccess &&
              dalloc(&w.rto, N) == hipSuccess && dalloc(&w.tau, N) == hipSuccess &&
              dalloc(&w.stepof, N) == hipSuccess && dalloc(&w.rc, N) == hipSuccess &&
              dalloc(&w.rwi, N) == hipSuccess && dalloc(&w.rin_inc, N) == hipSuccess &&
              dalloc(&w.rin_key, N) == hipSuccess && dalloc(&w.k0, 3 * N) == hipSuccess &&
              dalloc(&w.k1, 3 * N) == hipSuccess && dalloc(&w.evs, 2 * N) == hipSuccess &&
              dalloc(&w.d0, 3 * N) == hipSuccess && dalloc(&w.d1, 3 * N) == hipSuccess &&
              dalloc(&w.acc, 3 * N) == hipSuccess && dalloc(&w.need, 2 * N) == hipSuccess &&
              dalloc(&w.tcum, 2 * N) == hipSuccess && dalloc(&w.pos, N) == hipSuccess &&
              dalloc(&w.ecnt, 2 * ((int64_t)KK + 1)) == hipSuccess &&
              dalloc(&w.eoff, (int64_t)KK + 1) == hipSuccess &&
              dalloc(&w.roff, (int64_t)KK + 1) == hipSuccess &&
              dalloc(&w.rinoff, (int64_t)KK + 1) == hipSuccess &&
              dalloc(&w.cstep, N + 1) == hipSuccess && dalloc(&w.rbefore, N + 1) == hipSuccess &&
              dalloc(&w.over_incl, N + 1) == hipSuccess && dalloc(&w.stepgain, N + 1) == hipSuccess &&
              dalloc(&w.gain_incl, N + 1) == hipSuccess && dalloc(&w.best_g, 1024) == hipSuccess &&
              dalloc(&w.best_j, 1024) == hipSuccess && dalloc(&w.cnt, 2) == hipSuccess &&
              dalloc(&w.changed, 1) == hipSuccess && dalloc(&w.scal, 4) == hipSuccess;
    if (ok) {
        w.temp_bytes = bp_temp_bytes(N);
        ok = hipMalloc(&w.temp, w.temp_bytes) == hipSuccess;
    }
    if (!ok) {
        (void)hipGetLastError();
        free_bp(c);
        return fail(c, UPR_E_NOMEM, "best-prefix workspace allocation failed for n=%lld", (long long)N);
    }
    w.rcnt = w.ecnt + KK + 1;
    c->bp_cap_n = N;
    c->bp_cap_k = KK;
    return UPR_OK;
}

// Chunking of node ids for the rebalancer's in-bucket id bounds: n = the
// largest graph's node count, k = number of blocks.
void set_chunking(RebalWs &r, int64_t n, int32_t k)
{
    int64_t nch_max = kChunkEntries / std::max<int32_t>(k, 1);
    if (nch_max > 4096) nch_max = 4096;
    int shift = 0;
    while (((n + ((int64_t)1 << shift) - 1) >> shift) > nch_max) ++shift;
    r.chunk_shift = shift;
    r.nchunks = std::max<int64_t>((n + ((int64_t)1 << shift) - 1) >> shift, 1);
}

hipEvent_t take_event(upr_ctx *c)
{
    if (!c->timing.pool.empty()) {
        hipEvent_t e = c->timing.pool.back();
        c->timing.pool.pop_back();
        return e;
    }
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    return e;
}

struct PhaseTimer {
    upr_ctx *c;
    int phase;
    hipStream_t s;
    hipEvent_t a = nullptr;
    PhaseTimer(upr_ctx *c_, int p, hipStream_t s_) : c(c_), phase(p), s(s_)
    {
        if (((c->timing.mask >> phase) & 1u) && (a = take_event(c))) (void)hipEventRecord(a, s);
    }
    ~PhaseTimer()
    {
        if (!a) return;
        hipEvent_t b = take_event(c);
        if (!b) {
            c->timing.pool.push_back(a);
            return;
        }
        (void)hipEventRecord(b, s);
        c->timing.pending.push_back({phase, a, b});
    }
};

int check_params(upr_ctx *c, const upr_plan *p, const upr_params *q)
{
    if (!q) return fail(c, UPR_E_ARG, "params is NULL");
    if (q->k < 2 || q->k > UPR_MAX_K) return fail(c, UPR_E_ARG, "k=%d outside [2, %d]", q->k, UPR_MAX_K);
    if (q->eps_num <= 0 || q->eps_den <= 0) return fail(c, UPR_E_ARG, "eps must be > 0");
    if (q->t_den <= 0 || q->t_num < 0 || q->t_num > q->t_den) return fail(c, UPR_E_ARG, "t must be in [0, 1]");
    if (q->tau_den <= 0 || q->tau_num < 0 || q->tau_num > q->tau_den)
        return fail(c, UPR_E_ARG, "tau must be in [0, 1]");
    if (q->mode < 0 || q->mode > 3) return fail(c, UPR_E_ARG, "mode=%d not in {0,1,2,3}", q->mode);
    if (q->mode == 3 && (q->alpha_den <= 0 || q->alpha_num < q->alpha_den))
        return fail(c, UPR_E_ARG, "alpha must be a rational >= 1");
    if (q->variant & ~(UPR_VAR_OPTIMISTIC | UPR_VAR_PLAIN_PRIORITY | UPR_VAR_BEST_PREFIX))
        return fail(c, UPR_E_ARG, "unknown variant bits 0x%x", q->variant);
    if (q->max_rebalance_iters < 0) return fail(c, UPR_E_ARG, "max_rebalance_iters < 0");
    if (q->seq_penalty != 0 && q->seq_penalty != 1) return fail(c, UPR_E_ARG, "seq_penalty not 0/1");
    (void)p;
    return UPR_OK;
}

int check_plan(upr_ctx *c, const upr_plan *p)
{
    if (!c) return UPR_E_ARG;
    if (!p) return fail(c, UPR_E_ARG, "plan is NULL");
    if (p->ctx != c) return fail(c, UPR_E_ARG, "plan belongs to another context");
    return UPR_OK;
}

void sum_counters(upr_ctx *c)
{
    for (int j = 0; j < CNT_COUNT; ++j) {
        unsigned long long t = 0;
        for (int i = 0; i < kCntCopies; ++i) t += c->pinned[i * CNT_COUNT + j];
        c->cnt[j] = t;
    }
}

// Copy the counters to the pinned mirror, wait, and sum the copies.
int sync_counters(upr_ctx *c, hipStream_t s)
{
    HIP_TRY(c, hipMemcpyAsync(c->pinned, c->counters, sizeof(unsigned long long) * kCntWords,
                              hipMemcpyDeviceToHost, s));
    HIP_TRY(c, hipStreamSynchronize(s));
    sum_counters(c);
    return UPR_OK;
}

// Wait for the counter sums that the last k_rb_begin published with
// sequence number seq. The host spins on pub[0] (a sleeping stream wait
// wakes up tens of microseconds late); every 1024 polls it asks whether the
// stream has drained, which ends the wait with an error if the stream failed
// or finished without publishing.
static int wait_published(upr_ctx *c, hipStream_t s, unsigned long long seq)
{
    for (uint64_t i = 1;; ++i) {
        if (__atomic_load_n(&c->pub[0], __ATOMIC_ACQUIRE) == seq) break;
        if ((i & 1023) == 0) {
            const hipError_t q = hipStreamQuery(s);
            if (q == hipErrorNotReady) continue;
            if (q != hipSuccess) {
                (void)hipGetLastError();
                return fail(c, UPR_E_HIP, "HIP error %d (%s) while waiting for the counters", (int)q,
                            hipGetErrorString(q));
            }
            if (__atomic_load_n(&c->pub[0], __ATOMIC_ACQUIRE) == seq) break;
            return fail(c, UPR_E_HIP, "the stream finished without publishing the counters");
        }
        __builtin_ia32_pause();
    }
    for (int j = 0; j < CNT_COUNT; ++j) c->cnt[j] = __atomic_load_n(&c->pub[1 + j], __ATOMIC_RELAXED);
    return UPR_OK;
}

int64_t default_iters(const upr_plan *p, int32_t k)
{
    return p->g.vwgt ? 4 * (int64_t)k : (int64_t)k + 1;
}

// 32-bit per-workgroup histograms are exact when no workgroup can add up
// 2^32 of node weight: nodes scanned per workgroup times the largest c(v).
int hist32_ok(const upr_plan *p)
{
    const int64_t per_wg = ((p->g.n + (int64_t)rb_scan_grid(p->g.n) * kBlock - 1) /
                            ((int64_t)rb_scan_grid(p->g.n) * kBlock)) * kBlock;
    return (unsigned __int128)per_wg * (uint64_t)std::max<int64_t>(p->maxvw, 1) <
           ((unsigned __int128)1 << 32);
}

// The table build's view of the partition: the label-order copy when the
// plan has relabelled its adjacency, else pv itself.
static PartView table_part(const upr_ctx *c, const upr_plan *p, const PartView &pv)
{
    return p->order ? PartView{c->pc2, pv.bytes, pv.flagged} : pv;
}

// S4 for the moves marked in mvto; rebuilt tiles and hub rows are built from
// the table build's views. cut_delta (one graph without the best prefix): the
// apply also sums its change of the cut, which spares the statistics pass
// after it, and adds its block-weight sums into copies that the rebalancing
// begin after it (W's next reader) adds into W.
static hipError_t apply_moves(upr_ctx *c, const upr_plan *p, const Blocks &bk, int32_t *part,
                              const PartView &pv, int32_t *conn, int64_t *W, hipStream_t s,
                              bool cut_delta)
{
    return launch_apply(p->g, bk, part, pv, conn, W, c->mvto, p->hub_t, p->hubs(), c->counters,
                        p->dirty_threshold, c->dirty, p->table_graph(), table_part(c, p, pv),
                        p->order ? (void *)c->pc2 : nullptr, p->perm, p->all_threshold, s,
                        cut_delta, cut_delta ? c->apply_wcp : nullptr, kApplyCopiesMax);
}

// S5: the host loop over synchronous sub-iterations (one graph).
// early_tail (may be null): enqueued right after the speculative first
// sub-iteration, before the host waits for its counts; *tail_kept tells
// whether no sub-iteration followed it.
int rebalance_loop(upr_ctx *c, const upr_plan *p, const Blocks &bk, int plain, int32_t *part,
                   const PartView &pv, int32_t *conn, int64_t *W, int64_t it_max,
                   int64_t *iters_out, int64_t *status_out, hipStream_t s, bool speculate,
                   int32_t *rbrec, bool cut_delta, const std::function<int()> *early_tail,
                   bool *tail_kept)
{
    int32_t launched = 0;  // sub-iterations launched (numbers the records in rbrec)
    const HubView h = p->hubs();
    int64_t iters = 0, status = 0;
    const int hist32 = hist32_ok(p);
    c->rb_dirty = true;
    // every k_rb_begin publishes the counters (when the context can); the
    // host waits for the last one's
    auto begin = [&](int first) -> int {
        HIP_TRY(c, launch_rb_begin(bk, W, c->rb, c->counters, nullptr, s, first, c->pub_d,
                                   ++c->pub_seq, cut_delta ? c->apply_wcp : nullptr,
                                   kApplyCopiesMax));
        return UPR_OK;
    };
    auto sync = [&]() -> int {
        return c->pub ? wait_published(c, s, c->pub_seq) : sync_counters(c, s);
    };
    auto sub_iteration = [&]() -> int {
        HIP_TRY(c, launch_rb_iteration(p->g, bk, part, conn, c->rb, c->mvto, hist32, plain,
                                       p->hub_t, c->counters, nullptr, s, rbrec, ++launched));
        HIP_TRY(c, apply_moves(c, p, bk, part, pv, conn, W, s, cut_delta));
        return begin(0);
    };
    int rc;
    if ((rc = begin(1))) return rc;
    const bool early = speculate && early_tail;
    if (speculate) {
        // the first sub-iteration without waiting for the count of overloaded
        // blocks: with none it finds no movable node and changes nothing
        if ((rc = sub_iteration())) return rc;
        if (early && (rc = (*early_tail)())) return rc;
    }
    if (tail_kept) *tail_kept = early;
    rc = sync();
    if (rc) return rc;
    if (c->cnt[CNT_BAD_INPUT]) return fail(c, UPR_E_ARG, "part holds values outside [0, k)");
    if (speculate && c->cnt[CNT_OVER0] != 0) iters = 1;
    for (;;) {
        if (c->cnt[CNT_OVER] == 0) break;
        if (iters > 0 && c->cnt[CNT_MOVED_NOW] == 0) {
            status = 1;
            break;
        }
        if (iters >= it_max) {
            status = 1;
            break;
        }
        ++iters;
        if (tail_kept) *tail_kept = false;
        if ((rc = sub_iteration())) return rc;
        rc = sync();
        if (rc) return rc;
    }
    c->rb_dirty = false;
    *iters_out = iters;
    *status_out = status;
    return UPR_OK;
}

// Point a batch's host mirrors into the context's pinned area, growing it.
int bind_batch_pinned(upr_ctx *c, upr_batch *b)
{
    const int64_t need = (int64_t)b->ng * (GS_COUNT + 1 + kSlots + 3);
    if (need > c->bpinned_cap) {
        if (c->bpinned) {
            (void)hipDeviceSynchronize();
            (void)hipHostFree(c->bpinned);
        }
        c->bpinned = nullptr;
        c->bpinned_cap = 0;
        const int64_t cap = std::max<int64_t>(need, 4096);
        if (hipHostMalloc((void **)&c->bpinned, sizeof(int64_t) * cap) != hipSuccess) {
            (void)hipGetLastError();
            return UPR_E_NOMEM;
        }
        c->bpinned_cap = cap;
    }
    b->gstat_h = c->bpinned;
    b->srcl_h = b->gstat_h + (int64_t)b->ng * GS_COUNT;
    b->penq_h = b->srcl_h + b->ng;
    b->host3_h = b->penq_h + (int64_t)b->ng * kSlots;
    return UPR_OK;
}

// Counters and per-graph statistics to the pinned mirrors, then wait.
int sync_batch(upr_ctx *c, const upr_batch *b, hipStream_t s)
{
    HIP_TRY(c, hipMemcpyAsync(c->pinned, c->counters, sizeof(unsigned long long) * kCntWords,
                              hipMemcpyDeviceToHost, s));
    HIP_TRY(c, hipMemcpyAsync(b->gstat_h, b->gstat_d, sizeof(int64_t) * GS_COUNT * b->ng,
                              hipMemcpyDeviceToHost, s));
    HIP_TRY(c, hipStreamSynchronize(s));
    sum_counters(c);
    return UPR_OK;
}

// S5 for a batch: every graph follows the single-graph loop on its own (stop
// when balanced, when a sub-iteration moved nothing, or at its iteration
// cap); a graph that stopped is excluded from later sub-iterations by
// raising its source bound. Results per graph go to b->host3_h.
int rebalance_loop_batch(upr_ctx *c, const upr_plan *p, upr_batch *b, const Blocks &bk, int plain,
                         int32_t *part, const PartView &pv, int32_t *conn, int64_t *W,
                         int64_t it_user, hipStream_t s)
{
    const HubView h = p->hubs();
    const int32_t ng = b->ng, k = b->k;
    const int hist32 = hist32_ok(p);
    c->rb_dirty = true;
    HIP_TRY(c, hipMemcpyAsync(b->srcl_d, b->lmax_d, sizeof(int64_t) * ng, hipMemcpyDeviceToDevice, s));
    HIP_TRY(c, launch_rb_begin(bk, W, c->rb, c->counters, b->gstat_d, s));
    int rc = sync_batch(c, b, s);
    if (rc) return rc;
    if (c->cnt[CNT_BAD_INPUT]) return fail(c, UPR_E_ARG, "part holds a block outside its graph's range");
    std::vector<int64_t> iters(ng, 0), status(ng, 0), moves(ng, 0);
    std::vector<uint8_t> active(ng, 1);
    for (;;) {
        bool any = false;
        for (int32_t g = 0; g < ng; ++g) {
            if (!active[g]) continue;
            const int64_t *gs = b->gstat_h + (int64_t)g * GS_COUNT;
            if (iters[g] > 0) moves[g] += gs[GS_MOVED_NOW];
            const int64_t cap = it_user > 0 ? it_user : (b->weighted[g] ? 4 * (int64_t)k : (int64_t)k + 1);
            if (gs[GS_OVER] == 0) {
                active[g] = 0;
            } else if (iters[g] > 0 && gs[GS_MOVED_NOW] == 0) {
                status[g] = 1;
                active[g] = 0;
            } else if (iters[g] >= cap) {
                status[g] = 1;
                active[g] = 0;
            } else {
                ++iters[g];
                any = true;
            }
        }
        if (!any) break;
        for (int32_t g = 0; g < ng; ++g) b->srcl_h[g] = active[g] ? b->lmax[g] : INT64_MAX;
        HIP_TRY(c, hipMemcpyAsync(b->srcl_d, b->srcl_h, sizeof(int64_t) * ng, hipMemcpyHostToDevice, s));
        HIP_TRY(c, launch_rb_iteration(p->g, bk, part, conn, c->rb, c->mvto, hist32, plain,
                                       p->hub_t, c->counters, b->gstat_d, s));
        HIP_TRY(c, apply_moves(c, p, bk, part, pv, conn, W, s, false));
        HIP_TRY(c, launch_rb_begin(bk, W, c->rb, c->counters, b->gstat_d, s));
        rc = sync_batch(c, b, s);
        if (rc) return rc;
    }
    c->rb_dirty = false;
    for (int32_t g = 0; g < ng; ++g) {
        b->host3_h[3 * g] = iters[g];
        b->host3_h[3 * g + 1] = status[g];
        b->host3_h[3 * g + 2] = moves[g];
    }
    return UPR_OK;
}

void host_penq(int32_t tau_num, int32_t tau_den, int64_t *out)
{
    // floor(tau_num * 3^l * 2^16 / (tau_den * 2^l)) by exact long division:
    // numerator N = tau_num * 3^l (< 2^117), denominator D = tau_den * 2^l.
    for (int l = 0; l < kSlots; ++l) {
        unsigned __int128 N = (unsigned __int128)(uint32_t)tau_num;
        for (int i = 0; i < l; ++i) N *= 3;
        const unsigned __int128 D = (unsigned __int128)(uint32_t)tau_den << l;
        const unsigned __int128 q = N / D;
        const unsigned __int128 r = N - q * D;
        out[l] = (int64_t)((q << 16) + ((r << 16) / D));
    }
}

}  // namespace

// ==================================================================== ABI ==

extern "C" {

int64_t upr_lmax(int64_t total, int32_t k, int32_t eps_num, int32_t eps_den)
{
    if (k <= 0 || eps_den <= 0 || total < 0) return -1;
    const int64_t avg = total / k + (total % k != 0);
    const unsigned __int128 x = (unsigned __int128)(uint64_t)avg * (uint64_t)((int64_t)eps_den + eps_num);
    return (int64_t)(x / (uint64_t)eps_den);
}

int32_t upr_best_move_adjacency_degree(int32_t k, int64_t max_degree)
{
    if (k < 2 || k > UPR_MAX_K) return 0;
    return best_move_adj_deg(k, k <= 256 ? 1 : 2, max_degree);
}

int upr_penalty_table(int32_t tau_num, int32_t tau_den, int64_t *out)
{
    if (!out || tau_den <= 0 || tau_num < 0 || tau_num > tau_den) return UPR_E_ARG;
    host_penq(tau_num, tau_den, out);
    return UPR_OK;
}

int upr_create(upr_ctx **out, int device)
{
    if (!out) return UPR_E_ARG;
    *out = nullptr;
    int count = 0;
    if (hipGetDeviceCount(&count) != hipSuccess || device < 0 || device >= count) {
        (void)hipGetLastError();
        return UPR_E_HIP;
    }
    upr_ctx *c = new upr_ctx();
    c->device = device;
    c->seq_bucket_avg = (int32_t)std::min<int64_t>(
        std::max<int64_t>(env_int("UPR_SEQ_BUCKET_AVG", seq_bucket_avg_min()), seq_bucket_avg_min()),
        1 << 20);
    if (hipSetDevice(device) != hipSuccess ||
        hipMalloc((void **)&c->counters, sizeof(unsigned long long) * kCntWords) != hipSuccess ||
        hipMalloc((void **)&c->flags, sizeof(unsigned long long) * 8) != hipSuccess ||
        hipMalloc((void **)&c->penq, sizeof(int64_t) * kSlots) != hipSuccess ||
        hipMalloc((void **)&c->lmax1, sizeof(int64_t)) != hipSuccess ||
        hipMalloc((void **)&c->srcl1, sizeof(int64_t)) != hipSuccess ||
        hipHostMalloc((void **)&c->pinned, sizeof(unsigned long long) * kCntWords) != hipSuccess) {
        (void)hipGetLastError();
        upr_destroy(c);
        return UPR_E_NOMEM;
    }
    (void)hipMemset(c->counters, 0, sizeof(unsigned long long) * kCntWords);
    // the no-allocation scratch of this device (its address is taken once per
    // device; without it only upr_edge_cut_noalloc is unavailable)
    if (noalloc_init(device, &c->noalloc) != hipSuccess) {
        (void)hipGetLastError();
        c->noalloc = nullptr;
    }
    // the published counters: without host-coherent memory the rebalancing
    // loop copies the counters and waits for the stream instead
    if (hipHostMalloc((void **)&c->pub, sizeof(unsigned long long) * (1 + CNT_COUNT),
                      hipHostMallocMapped | hipHostMallocCoherent) != hipSuccess ||
        hipHostGetDevicePointer((void **)&c->pub_d, c->pub, 0) != hipSuccess) {
        (void)hipGetLastError();
        if (c->pub) (void)hipHostFree(c->pub);
        c->pub = c->pub_d = nullptr;
    } else {
        for (int i = 0; i <= CNT_COUNT; ++i) c->pub[i] = 0;
    }
    *out = c;
    return UPR_OK;
}

void upr_destroy(upr_ctx *c)
{
    if (!c) return;
    (void)hipSetDevice(c->device);
    (void)hipDeviceSynchronize();
    free_workspace(c);
    free_bp(c);
    dfree(c->carry);
    dfree(c->counters);
    dfree(c->flags);
    dfree(c->penq);
    dfree(c->lmax1);
    dfree(c->srcl1);
    if (c->pinned) (void)hipHostFree(c->pinned);
    if (c->pub) (void)hipHostFree(c->pub);
    if (c->bpinned) (void)hipHostFree(c->bpinned);
    for (auto &p : c->timing.pending) {
        (void)hipEventDestroy(p.a);
        (void)hipEventDestroy(p.b);
    }
    for (auto e : c->timing.pool) (void)hipEventDestroy(e);
    drop_captured(c);
    if (c->cap_stream) (void)hipStreamDestroy(c->cap_stream);
    delete c;
}

const char *upr_last_error(const upr_ctx *c)
{
    if (!c) return "null context";
    return c->err;
}

int upr_validate_graph(upr_ctx *c, const upr_graph *graph, hipStream_t s)
{
    if (!c) return UPR_E_ARG;
    if (!graph) return fail(c, UPR_E_ARG, "graph is NULL");
    if (graph->n < 0 || graph->n >= ((int64_t)1 << 31)) return fail(c, UPR_E_ARG, "n out of range");
    if (graph->n > 0 && !graph->xadj) return fail(c, UPR_E_ARG, "xadj NULL");
    HIP_TRY(c, hipSetDevice(c->device));
    const GraphView g{graph->n, graph->xadj, graph->adjncy, graph->adjwgt, graph->vwgt};
    if (g.n == 0) return UPR_OK;
    {
        int64_t nnz = 0;
        HIP_TRY(c, hipMemcpy(&nnz, g.xadj + g.n, sizeof nnz, hipMemcpyDeviceToHost));
        if (nnz > 0 && !g.adjncy) return fail(c, UPR_E_ARG, "adjncy NULL with %lld entries", (long long)nnz);
    }
    unsigned long long init[4] = {~0ull, ~0ull, ~0ull, ~0ull}, got[4];
    for (int stage = 0; stage < 3; ++stage) {
        HIP_TRY(c, hipMemcpyAsync(c->flags, init, sizeof init, hipMemcpyHostToDevice, s));
        HIP_TRY(c, launch_validate(g, c->flags, stage, s));
        HIP_TRY(c, hipMemcpyAsync(got, c->flags, sizeof got, hipMemcpyDeviceToHost, s));
        HIP_TRY(c, hipStreamSynchronize(s));
        if (stage == 0) {
            int64_t x0 = -1;
            HIP_TRY(c, hipMemcpy(&x0, g.xadj, sizeof x0, hipMemcpyDeviceToHost));
            if (x0 != 0) return fail(c, UPR_E_GRAPH, "xadj[0] = %lld, expected 0", (long long)x0);
            if (got[0] != ~0ull) return fail(c, UPR_E_GRAPH, "xadj decreases at %llu", got[0]);
            if (got[3] != ~0ull) return fail(c, UPR_E_GRAPH, "node weight <= 0 at node %llu", got[3]);
        } else {
            if (got[1] != ~0ull)
                return fail(c, UPR_E_GRAPH,
                            stage == 1 ? "neighbour id out of range at entry %llu"
                                       : "self-loop, unsorted row or duplicate at entry %llu",
                            got[1]);
            if (got[3] != ~0ull) return fail(c, UPR_E_GRAPH, "edge weight <= 0 at entry %llu", got[3] - g.n);
            if (stage == 2 && got[2] != ~0ull)
                return fail(c, UPR_E_GRAPH, "entry %llu has no symmetric counterpart (or its weight differs)",
                            got[2]);
        }
    }
    return UPR_OK;
}

static int plan_create(upr_ctx *c, const upr_graph *graph, upr_plan **out, hipStream_t s,
                       bool validate, int64_t known_nnz, const upr_plan_opts *opts,
                       bool batch = false);

int upr_plan_create(upr_ctx *c, const upr_graph *graph, upr_plan **out, hipStream_t s)
{
    return plan_create(c, graph, out, s, true, -1, nullptr);
}

int upr_plan_create_opts(upr_ctx *c, const upr_graph *graph, const upr_plan_opts *opts,
                         upr_plan **out, hipStream_t s)
{
    return plan_create(c, graph, out, s, true, -1, opts);
}

// validate = false: the caller has checked the graph already (a batch of
// graphs validated before); known_nnz >= 0: xadj[n], known on the host;
// batch: the union graph of a batch (not relabelled by default).
static int plan_create(upr_ctx *c, const upr_graph *graph, upr_plan **out, hipStream_t s,
                       bool validate, int64_t known_nnz, const upr_plan_opts *opts, bool batch)
{
    if (!c) return UPR_E_ARG;
    if (!out) return fail(c, UPR_E_ARG, "out is NULL");
    *out = nullptr;
    if (!graph) return fail(c, UPR_E_ARG, "graph is NULL");
    if (graph->n < 0 || graph->n >= ((int64_t)1 << 31)) return fail(c, UPR_E_ARG, "n out of range");
    if (graph->n > 0 && !graph->xadj) return fail(c, UPR_E_ARG, "xadj NULL");
    HIP_TRY(c, hipSetDevice(c->device));
    const GraphView g{graph->n, graph->xadj, graph->adjncy, graph->adjwgt, graph->vwgt};
    if (g.n > 0 && known_nnz < 0) {
        int64_t nnz = 0;
        HIP_TRY(c, hipMemcpy(&nnz, g.xadj + g.n, sizeof nnz, hipMemcpyDeviceToHost));
        if (nnz < 0) return fail(c, UPR_E_GRAPH, "xadj[n] < 0");
        if (nnz > 0 && !g.adjncy) return fail(c, UPR_E_ARG, "adjncy NULL with %lld entries", (long long)nnz);
    }

    // basic validation: xadj, ids in range, positive weights (kernels rely on it)
    if (g.n > 0 && validate) {
        unsigned long long init[4] = {~0ull, ~0ull, ~0ull, ~0ull}, got[4];
        for (int stage = 0; stage < 2; ++stage) {
            HIP_TRY(c, hipMemcpyAsync(c->flags, init, sizeof init, hipMemcpyHostToDevice, s));
            HIP_TRY(c, launch_validate(g, c->flags, stage, s));
            HIP_TRY(c, hipMemcpyAsync(got, c->flags, sizeof got, hipMemcpyDeviceToHost, s));
            HIP_TRY(c, hipStreamSynchronize(s));
            int64_t x0 = 0;
            if (stage == 0) HIP_TRY(c, hipMemcpy(&x0, g.xadj, sizeof x0, hipMemcpyDeviceToHost));
            if (x0 != 0 || got[0] != ~0ull) return fail(c, UPR_E_GRAPH, "xadj is not a valid offset array");
            if (got[1] != ~0ull) return fail(c, UPR_E_GRAPH, "neighbour id out of range at entry %llu", got[1]);
            if (got[3] != ~0ull) return fail(c, UPR_E_GRAPH, "non-positive node or edge weight");
        }
    }

    upr_plan *p = new upr_plan();
    static std::atomic<uint64_t> plan_serial{0};
    p->serial = ++plan_serial;
    p->ctx = c;
    p->device = c->device;
    p->g = g;
    // thresholds: the options, else the environment, else the defaults
    p->hub_t = opts && opts->hub_threshold > 0 ? opts->hub_threshold
                                               : env_int("UPR_HUB_THRESHOLD", kDefaultHubThreshold);
    const int64_t dirty_div = opts && opts->dirty_div > 0 ? opts->dirty_div : env_int("UPR_DIRTY_DIV", 16);
    // a tile's edge count (nodes per tile x hub threshold) must fit int32
    p->hub_t = std::min<int64_t>(std::max<int64_t>(p->hub_t, 1), (int64_t)1 << 20);
    int32_t *hub_list = nullptr;
    auto bail = [&](int code, const char *msg) {
        dfree(hub_list);
        upr_plan_destroy(p);
        return fail(c, code, "%s", msg);
    };
    if (g.n > 0) {
        if (known_nnz >= 0) p->nnz = known_nnz;
        else if (hipMemcpy(&p->nnz, g.xadj + g.n, sizeof(int64_t), hipMemcpyDeviceToHost) != hipSuccess)
            return bail(UPR_E_HIP, "reading xadj[n] failed");
        // integer-atomic deltas cost about as much per moved edge as a
        // rebuild costs per edge of the whole graph divided by this factor
        p->dirty_threshold = p->nnz / std::max<int64_t>(dirty_div, 1);
        // from twice that on, marking tiles is not worth its edge walk
        // (UPR_REBUILD_ALL_DIV: from nnz / div on)
        const int64_t all_div = env_int("UPR_REBUILD_ALL_DIV", 0);
        p->all_threshold = all_div > 0 ? p->nnz / all_div : 2 * p->dirty_threshold;
        // never below the marking threshold: between the two, the apply would
        // skip the movers' edge walk (every tile is rebuilt) while the hub
        // rows, rebuilt only above the marking threshold, still wait for deltas
        p->all_threshold = std::max(p->all_threshold, p->dirty_threshold);
        if (dalloc(&p->wdeg, g.n) != hipSuccess || dalloc(&hub_list, g.n) != hipSuccess)
            return bail(UPR_E_NOMEM, "plan allocation failed");
        unsigned long long zero[8] = {0}, res[8];
        if (hipMemcpyAsync(c->flags, zero, sizeof zero, hipMemcpyHostToDevice, s) != hipSuccess ||
            launch_plan_scan(g, p->wdeg, p->hub_t, hub_list, c->flags, s) != hipSuccess ||
            hipMemcpyAsync(res, c->flags, sizeof res, hipMemcpyDeviceToHost, s) != hipSuccess ||
            hipStreamSynchronize(s) != hipSuccess)
            return bail(UPR_E_HIP, "plan scan failed");
        p->nh = (int32_t)res[0];
        p->maxdeg = (int64_t)res[1];
        p->maxwdeg = (int64_t)res[2];
        p->total = (int64_t)res[3];
        p->maxvw = (int64_t)res[4];
        if (p->maxwdeg >= ((int64_t)1 << 31) - 1)
            return bail(UPR_E_GRAPH, "a weighted degree does not fit int32 (gain table entries are int32)");
        if (p->total >= ((int64_t)1 << 62)) return bail(UPR_E_GRAPH, "total node weight >= 2^62");
        // 16-bit gain-table counters in LDS: unit weights and a hub threshold
        // below 2^16 bound every tiled row sum, else the largest weighted degree
        p->g.tile16 = ((!g.adjwgt && p->hub_t < 65536) || p->maxwdeg < 65536) ? 1 : 0;
        if (p->nh > 0) {
            std::vector<int32_t> ids(p->nh);
            if (hipMemcpy(ids.data(), hub_list, sizeof(int32_t) * p->nh, hipMemcpyDeviceToHost) != hipSuccess)
                return bail(UPR_E_HIP, "reading the hub list failed");
            std::sort(ids.begin(), ids.end());
            if (dalloc(&p->hub_ids, p->nh) != hipSuccess || dalloc(&p->gacc, p->nh) != hipSuccess ||
                dalloc(&p->hub_ticket, p->nh) != hipSuccess)
                return bail(UPR_E_NOMEM, "plan allocation failed");
            std::vector<int64_t> e01(2 * (size_t)p->nh);
            int64_t *d_e01 = nullptr;
            if (dalloc(&d_e01, 2 * (int64_t)p->nh) != hipSuccess) return bail(UPR_E_NOMEM, "plan allocation failed");
            bool ok = hipMemcpy(p->hub_ids, ids.data(), sizeof(int32_t) * p->nh, hipMemcpyHostToDevice) == hipSuccess &&
                      launch_hub_ranges(g.xadj, p->hub_ids, p->nh, d_e01, s) == hipSuccess &&
                      hipStreamSynchronize(s) == hipSuccess &&
                      hipMemcpy(e01.data(), d_e01, sizeof(int64_t) * 2 * p->nh, hipMemcpyDeviceToHost) == hipSuccess;
            dfree(d_e01);
            if (!ok) return bail(UPR_E_HIP, "hub preparation failed");
            std::vector<HubChunk> chunks;
            for (int32_t i = 0; i < p->nh; ++i) {
                const int32_t nc =
                    (int32_t)((e01[2 * i + 1] - e01[2 * i] + kHubChunkEdges - 1) / kHubChunkEdges);
                for (int64_t e = e01[2 * i]; e < e01[2 * i + 1]; e += kHubChunkEdges)
                    chunks.push_back(HubChunk{i, nc, e, std::min(e + kHubChunkEdges, e01[2 * i + 1])});
            }
            p->nchunks = (int64_t)chunks.size();
            const int64_t words = (g.n + 31) / 32;
            if (dalloc(&p->chunks, p->nchunks) != hipSuccess || dalloc(&p->hub_bits, words) != hipSuccess)
                return bail(UPR_E_NOMEM, "plan allocation failed");
            if (hipMemset(p->hub_bits, 0, sizeof(uint32_t) * words) != hipSuccess)
                return bail(UPR_E_HIP, "hub bitmap clear failed");
            ok = hipMemcpy(p->chunks, chunks.data(), sizeof(HubChunk) * chunks.size(), hipMemcpyHostToDevice) == hipSuccess &&
                 launch_fill_i64(p->gacc, p->nh, 0, s) == hipSuccess &&
                 launch_fill_i32((int32_t *)p->hub_ticket, p->nh, 0, s) == hipSuccess &&
                 launch_hub_bits(p->hubs(), p->hub_bits, s) == hipSuccess &&
                 hipStreamSynchronize(s) == hipSuccess;
            if (!ok) return bail(UPR_E_HIP, "hub preparation failed");
        }
        dfree(hub_list);
        // relabelled adjacency for the table build: UPR_RELABEL=0 never, 2
        // always, else (default) for single graphs whose compact partition
        // copy outgrows an L1 (kRelabelMinNodes). Not for a batch by default:
        // a server rebuilds batches often and the sort costs more there than
        // it saves. Skipped, not an error, if its memory cannot be had.
        const int64_t relabel = env_int("UPR_RELABEL", 1);
        if (p->nnz > 0 &&
            (relabel == 2 || (relabel == 1 && !batch && g.n >= kRelabelMinNodes))) {
            if (dalloc(&p->adj_r, p->nnz) == hipSuccess && dalloc(&p->perm, g.n) == hipSuccess &&
                dalloc(&p->order, g.n) == hipSuccess) {
                if (launch_degree_relabel(g, p->nnz, p->order, p->perm, p->adj_r, s) != hipSuccess)
                    return bail(UPR_E_HIP, "relabelling the adjacency failed");
            } else {
                (void)hipGetLastError();
                dfree(p->adj_r);
                dfree(p->perm);
                dfree(p->order);
                p->adj_r = p->perm = p->order = nullptr;
            }
        }
    }
    *out = p;
    return UPR_OK;
}

void upr_plan_destroy(upr_plan *p)
{
    if (!p) return;
    (void)hipSetDevice(p->device);
    (void)hipDeviceSynchronize();
    dfree(p->wdeg);
    dfree(p->hub_ids);
    dfree(p->chunks);
    dfree(p->gacc);
    dfree(p->hub_ticket);
    dfree(p->hub_bits);
    dfree(p->adj_r);
    dfree(p->perm);
    dfree(p->order);
    delete p;
}

int upr_plan_info(const upr_plan *p, int64_t *n, int64_t *nnz, int64_t *total, int64_t *maxdeg,
                  int64_t *nh)
{
    if (!p) return UPR_E_ARG;
    if (n) *n = p->g.n;
    if (nnz) *nnz = p->nnz;
    if (total) *total = p->total;
    if (maxdeg) *maxdeg = p->maxdeg;
    if (nh) *nh = p->nh;
    return UPR_OK;
}

int upr_gain_table(upr_ctx *c, const upr_plan *p, int32_t k, const int32_t *part, int32_t *conn,
                   hipStream_t s)
{
    int rc = check_plan(c, p);
    if (rc) return rc;
    if (k < 2 || k > UPR_MAX_K) return fail(c, UPR_E_ARG, "k=%d outside [2, %d]", k, UPR_MAX_K);
    if (p->g.n > 0 && (!part || !conn)) return fail(c, UPR_E_ARG, "part/conn NULL");
    HIP_TRY(c, hipSetDevice(c->device));
    HIP_TRY(c, hipMemsetAsync(c->counters, 0, sizeof(unsigned long long) * kCntWords, s));
    HIP_TRY(c, launch_check_part(p->g.n, k, part, c->counters, s));
    rc = sync_counters(c, s);
    if (rc) return rc;
    if (c->cnt[CNT_BAD_INPUT]) return fail(c, UPR_E_ARG, "part holds values outside [0, k)");
    PhaseTimer t(c, 0, s);
    const PartView pv{part, 4};
    HIP_TRY(c, launch_zero_hub_rows(p->hubs(), conn, k, s));
    HIP_TRY(c, launch_gain_table(p->g, k, pv, conn, p->hub_t, p->hubs(), s));
    return UPR_OK;
}

int upr_block_weights(upr_ctx *c, const upr_plan *p, int32_t k, const int32_t *part, int64_t *W,
                      hipStream_t s)
{
    int rc = check_plan(c, p);
    if (rc) return rc;
    if (k < 2 || k > UPR_MAX_K) return fail(c, UPR_E_ARG, "k=%d outside [2, %d]", k, UPR_MAX_K);
    if (!W || (p->g.n > 0 && !part)) return fail(c, UPR_E_ARG, "part/block_w NULL");
    HIP_TRY(c, hipSetDevice(c->device));
    HIP_TRY(c, hipMemsetAsync(c->counters, 0, sizeof(unsigned long long) * kCntWords, s));
    HIP_TRY(c, launch_check_part(p->g.n, k, part, c->counters, s));
    rc = sync_counters(c, s);
    if (rc) return rc;
    if (c->cnt[CNT_BAD_INPUT]) return fail(c, UPR_E_ARG, "part holds values outside [0, k)");
    HIP_TRY(c, launch_fill_i64(W, k, 0, s));
    HIP_TRY(c, launch_block_weights(p->g, k, part, W, c->counters, s));
    return UPR_OK;
}

int upr_edge_cut(upr_ctx *c, const upr_plan *p, const int32_t *part, int64_t *cut, hipStream_t s)
{
    int rc = check_plan(c, p);
    if (rc) return rc;
    if (!cut || (p->g.n > 0 && !part)) return fail(c, UPR_E_ARG, "part/cut NULL");
    HIP_TRY(c, hipSetDevice(c->device));
    PhaseTimer t(c, 6, s);
    HIP_TRY(c, hipMemsetAsync(c->counters, 0, sizeof(unsigned long long) * kCntWords, s));
    HIP_TRY(c, launch_cut_edges(p->g, part, c->counters, CNT_TMP, s));
    HIP_TRY(c, launch_store_half(c->counters, CNT_TMP, cut, s));
    return UPR_OK;
}

int upr_edge_cut_noalloc(upr_ctx *c, const upr_graph *graph, const int32_t *part, int64_t *cut,
                         hipStream_t s)
{
    if (!c) return UPR_E_ARG;
    if (!graph || !cut) return fail(c, UPR_E_ARG, "graph/cut NULL");
    if (graph->n < 0 || graph->n > UPR_NOALLOC_MAX_NODES)
        return fail(c, UPR_E_ARG, "n=%lld outside [0, %lld], the no-allocation scratch limit",
                    (long long)graph->n, (long long)UPR_NOALLOC_MAX_NODES);
    if (graph->n > 0 && (!graph->xadj || !part)) return fail(c, UPR_E_ARG, "xadj/part NULL");
    if (!c->noalloc) return fail(c, UPR_E_HIP, "the no-allocation scratch of device %d is unavailable", c->device);
    HIP_TRY(c, hipSetDevice(c->device));
    const GraphView g{graph->n, graph->xadj, graph->adjncy, graph->adjwgt, graph->vwgt};
    HIP_TRY(c, launch_cut_noalloc(g, part, cut, c->noalloc, s));
    return UPR_OK;
}

// Enqueue `span` on s as a HIP graph: replayed when a graph with this key was
// captured before, else captured on the context's own stream (nothing runs
// while capturing), instantiated, kept (at most kCaptureMax, the oldest
// dropped) and launched.
static int run_captured(upr_ctx *c, const uint64_t (&key)[kCaptureKey],
                        const std::function<int(hipStream_t)> &span, hipStream_t s)
{
    for (auto &g : c->captured)
        if (std::equal(key, key + kCaptureKey, g.key)) {
            HIP_TRY(c, hipGraphLaunch(g.exec, s));
            return UPR_OK;
        }
    HIP_TRY(c, hipStreamBeginCapture(c->cap_stream, hipStreamCaptureModeThreadLocal));
    const int rc = span(c->cap_stream);
    hipGraph_t graph = nullptr;
    const hipError_t e = hipStreamEndCapture(c->cap_stream, &graph);
    if (rc || e != hipSuccess) {
        if (graph) (void)hipGraphDestroy(graph);
        (void)hipGetLastError();
        return rc ? rc : fail(c, UPR_E_HIP, "capturing the move phases failed: %s",
                              hipGetErrorString(e));
    }
    hipGraphExec_t exec = nullptr;
    const hipError_t ei = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
    (void)hipGraphDestroy(graph);
    if (ei != hipSuccess) {
        (void)hipGetLastError();
        return fail(c, UPR_E_HIP, "instantiating the move phases failed: %s", hipGetErrorString(ei));
    }
    if (c->captured.size() >= kCaptureMax) {
        (void)hipGraphExecDestroy(c->captured.front().exec);
        c->captured.erase(c->captured.begin());
    }
    upr_ctx::Captured g;
    std::copy(key, key + kCaptureKey, g.key);
    g.exec = exec;
    c->captured.push_back(g);
    HIP_TRY(c, hipGraphLaunch(exec, s));
    return UPR_OK;
}

// One round (moves = true) or a standalone rebalancing (moves = false) of a
// single graph (b == null) or of every graph of a batch.
static int round_core(upr_ctx *c, const upr_plan *p, upr_batch *b, const upr_params *q,
                      int32_t *part, int32_t *conn, int64_t *W, int64_t *stats, hipStream_t s,
                      bool moves, const uint8_t *active = nullptr)
{
    const int64_t n = p->g.n;
    const int32_t k = q->k;
    const int32_t ng = b ? b->ng : 1;
    int64_t lmax = 0;
    Blocks bk;
    bk.k = k;
    bk.ng = ng;
    if (b) {
        bk.lmax = b->lmax_d;
        bk.src_lmax = b->srcl_d;
        bk.penq = b->penq_d;
    } else {
        lmax = upr_lmax(p->total, k, q->eps_num, q->eps_den);
        if (p->maxvw > lmax)
            return fail(c, UPR_E_INFEASIBLE, "node weight %lld exceeds L_max %lld",
                        (long long)p->maxvw, (long long)lmax);
        bk.lmax = c->lmax1;
        bk.src_lmax = c->srcl1;
        bk.penq = c->penq;
    }
    if (q->mode == 3) {
        bk.alpha_num = q->alpha_num;
        bk.alpha_den = q->alpha_den;
    }
    const int optimistic = (q->variant & UPR_VAR_OPTIMISTIC) ? 1 : 0;
    const int plain = (q->variant & UPR_VAR_PLAIN_PRIORITY) ? 1 : 0;
    // the interleaved best prefix: single graphs, rounds with moves
    const bool prefix = moves && !b && (q->variant & UPR_VAR_BEST_PREFIX) && n > 0;
    // one graph without the best prefix: the applies sum their change of the
    // cut, and the cut statistics after them are a sum unless an apply
    // rebuilt tiles
    const bool cut_delta = !b && !prefix;
    const int32_t K = bk.total();
    int64_t *gstat = b ? b->gstat_d : nullptr;
    StatsGeom sg;
    if (b) {
        sg.goff = b->goff_d;
        sg.span = b->stats_span;
        sg.window = b->stats_window;
    }
    HIP_TRY(c, hipSetDevice(c->device));
    int rc = ensure_workspace(c, n, K);
    if (rc) return rc;
    if (prefix && (rc = ensure_bp(c, n, K))) return rc;
    set_chunking(c->rb, b ? b->max_n : n, K);
    c->rb.goff = b ? b->goff_d : nullptr;
    const HubView h = p->hubs();
    PhaseTimer whole(c, 7, s);

    PenTable pq;
    if (!b) host_penq(q->tau_num, q->tau_den, pq.q);
    // the segment path's counters start at zero
    const bool seg = moves && q->seq_penalty && seq_segments_fit(seq_score_bits(p->maxwdeg), n);
    HIP_TRY(c, launch_round_init(bk, c->bucket, W, pq, lmax, b ? 0 : 1, c->counters,
                                 q->rebuild_table, seg ? c->seg_cur : nullptr,
                                 seg ? seq_counter_words(K) : 0, s, h,
                                 q->rebuild_table ? conn : nullptr, k));
    // compact partition copy for the neighbour gathers (kept in step by the apply)
    const PartView pv{c->pc, k <= 256 ? 1 : 2, k <= 128 ? 1 : 0};
    // and the same in the plan's label order for the table build
    const PartView tpv = table_part(c, p, pv);
    bool moved = false;
    // everything from here to the rebalancing: enqueued on s, or captured
    // once per configuration and replayed (upr_capture_enable)
    const std::function<int(hipStream_t)> span = [&](hipStream_t s) -> int {
    if (b) HIP_TRY(c, launch_fill_i64(gstat, (int64_t)GS_COUNT * ng, 0, s));
    HIP_TRY(c, launch_pack_part(n, bk, b ? b->goff_d : nullptr, part, c->pc, pv.bytes, c->counters, s,
                                p->order, p->order ? c->pc2 : nullptr));
    if (q->rebuild_table) {
        const GraphView tg = p->table_graph();
        {
            PhaseTimer t(c, 0, s);
            // the hub rows were cleared by the round's init
            HIP_TRY(c, launch_gain_table(tg, k, tpv, conn, p->hub_t, h, s, c->inner, pv));
        }
    }
    // one graph with moves and without the best prefix: the statistics pass
    // adds into copies that the bucket prefix pass, its first reader, sums
    const bool spread = moves && !b && !prefix && c->stat_copies > 1;
    int64_t *wsp = spread ? c->stat_wsp : nullptr, *bsp = spread ? c->stat_bsp : nullptr;
    {
        PhaseTimer t(c, 1, s);
        // the rebuilt table's own entries come from the tile build
        HIP_TRY(c, launch_node_stats(p->g, bk, sg, part, conn, p->wdeg, q->rebuild_table ? W : nullptr,
                                     moves ? c->bucket : nullptr, q->t_num, q->t_den, c->counters,
                                     CNT_CUT2_BEFORE, moves && q->seq_penalty ? c->avail : nullptr,
                                     gstat, GS_CUT2_BEFORE, s, q->rebuild_table ? c->inner : nullptr,
                                     p->nh > 0 ? p->hub_bits : nullptr, false, wsp, bsp,
                                     c->stat_copies));
    }
    if (prefix) HIP_TRY(c, launch_bp_record_start(n, K, part, W, c->bp, s));
    if (moves) {
        {
            PhaseTimer t(c, 2, s);
            HIP_TRY(c, launch_cb_prefix(bk, c->bucket, W, q->mode, c->pen1, s, wsp, bsp,
                                        c->stat_copies));
            // with the degree order, the flags and keys also in label order
            const bool rl = pv.flagged && pv.bytes == 1 && p->order;
            PhaseTimer tk(c, 8, s);
            HIP_TRY(c, launch_best_move(p->g, bk, part, conn, W, c->bucket, c->pen1, q->mode,
                                        active, c->key, c->pen, c->counters,
                                        pv.flagged ? (uint8_t *)c->pc : nullptr, s,
                                        rl ? (uint8_t *)c->pc2 : nullptr, rl ? c->key2 : nullptr,
                                        p->perm, pv, best_move_adj_deg(k, pv.bytes, p->maxdeg), p->maxdeg));
        }
        // no host decision here: with no candidates the filter and the apply
        // find nothing to do; a bad part value is reported at the next
        // synchronisation (every kernel range-checks it)
        moved = true;
        {
            PhaseTimer t(c, 3, s);
            int64_t *gp_out = q->seq_penalty ? c->gp : nullptr;
            const bool rl = pv.flagged && pv.bytes == 1 && p->order;
            {
                PhaseTimer tk(c, 9, s);
                HIP_TRY(c, launch_filter(p->g, bk, optimistic, part, pv, c->key, c->pen, p->hub_t,
                                         c->mvto, c->accflag, c->counters, gp_out, s,
                                         rl ? p->adj_r : nullptr, rl ? tpv : PartView{},
                                         rl ? c->key2 : nullptr, rl ? p->order : nullptr));
            }
            HIP_TRY(c, launch_filter_hub(p->g, bk, optimistic, part, pv, c->key, c->pen, h,
                                         c->mvto, c->accflag, c->counters, gp_out, s));
            if (q->seq_penalty) {
                const int sb = seq_score_bits(p->maxwdeg);
                if (seq_segments_fit(sb, n)) {
                    const SegWs ws{c->seg_cur,    c->seg_off,    c->seg_boff,  c->seg_cpre,
                                   c->seg_slist,  c->seg_meta,   c->seg_bblk,  c->seg_bpos,
                                   c->seg_bsize,  c->seg_bdel,   c->seg_bcnt,  c->seg_scan_c,
                                   c->seg_scan_d, c->seg_spl,    c->ev_key,    c->ev_key2,
                                   c->seq_bucket_avg};
                    HIP_TRY(c, launch_seq_segments(p->g, bk, b ? b->goff_d : nullptr, c->key,
                                                   c->gp, part, c->avail, sb, ws, W, c->bucket,
                                                   q->mode, p->hub_t, c->mvto, c->accflag,
                                                   c->counters, s));
                } else {
                    // eligible candidates in id order; their number sizes the sort
                    HIP_TRY(c, launch_seq_select(n, c->key, c->gp, c->cand, c->counters + CNT_ELIG,
                                                 c->seq_temp, c->seq_temp_size, s));
                    const int rs = sync_counters(c, s);
                    if (rs) return rs;
                    if (c->cnt[CNT_BAD_INPUT])
                        return fail(c, UPR_E_ARG, b ? "part holds a block outside its graph's range"
                                                    : "part holds values outside [0, k)");
                    const int64_t ne = (int64_t)c->cnt[CNT_ELIG];
                    HIP_TRY(c, launch_seq_net(ne, c->cand, c->key, part, p->g.vwgt, c->avail, bk, sb,
                                              c->ev_key, c->ev_key2, c->ev_val, c->ev_val2,
                                              c->ev_prefix, c->netpre, c->seq_temp,
                                              c->seq_temp_size, s));
                    HIP_TRY(c, launch_filter_seq(p->g, bk, part, c->cand, ne, c->key, c->gp,
                                                 c->netpre, W, c->bucket, q->mode, p->hub_t,
                                                 c->mvto, c->accflag, c->counters, s));
                }
            }
            if (b) HIP_TRY(c, launch_batch_move_stats(n, b->stats_span, bk, b->goff_d, part, c->key, c->accflag,
                                                       gstat, s));
        }
        {
            PhaseTimer t(c, 4, s);
            HIP_TRY(c, apply_moves(c, p, bk, part, pv, conn, W, s, cut_delta));
        }
        {
            PhaseTimer t(c, 6, s);
            HIP_TRY(c, launch_node_stats(p->g, bk, sg, part, conn, p->wdeg, nullptr, nullptr, 0, 1,
                                         c->counters, CNT_CUT2_MOVES, nullptr, gstat,
                                         GS_CUT2_MOVES, s, nullptr, nullptr, cut_delta));
        }
    }
    return UPR_OK;
    };
    // captured: a graph or a batch (its own plan), no driver activity mask,
    // no best prefix, no phase timing, and no host synchronisation inside the
    // span (the segment path of the sequence-aware price)
    const bool cap = c->capture && c->cap_stream && !active && !prefix && moves &&
                     c->timing.mask == 0 && (!q->seq_penalty || seg);
    if (cap) {
        const uint64_t key[kCaptureKey] = {
            p->serial, c->ws_gen, (uint64_t)k, (uint64_t)(uint32_t)q->eps_num,
            (uint64_t)(uint32_t)q->eps_den, (uint64_t)(uint32_t)q->t_num, (uint64_t)(uint32_t)q->t_den,
            (uint64_t)(uint32_t)q->mode, (uint64_t)(uint32_t)q->rebuild_table,
            (uint64_t)(uint32_t)q->seq_penalty, (uint64_t)(uint32_t)q->variant,
            q->mode == 3 ? ((uint64_t)(uint32_t)q->alpha_num << 32 | (uint32_t)q->alpha_den) : 0,
            (uint64_t)(uintptr_t)part, (uint64_t)(uintptr_t)conn, (uint64_t)(uintptr_t)W, 0};
        rc = run_captured(c, key, span, s);
        moved = true;
    } else {
        rc = span(s);
    }
    if (rc) return rc;
    int64_t iters = 0, status = 0;
    // the cut after rebalancing and the statistics (iters < 0: derived on the device)
    const auto cut_after = [&]() -> int {
        PhaseTimer t(c, 6, s);
        HIP_TRY(c, launch_node_stats(p->g, bk, sg, part, conn, p->wdeg, nullptr, nullptr, 0, 1,
                                     c->counters, CNT_CUT2_AFTER, nullptr, gstat, GS_CUT2_AFTER, s,
                                     nullptr, nullptr, cut_delta));
        return UPR_OK;
    };
    const std::function<int()> tail = [&]() -> int {
        const int r = cut_after();
        if (r) return r;
        HIP_TRY(c, launch_stats_final(stats, c->counters, lmax, -1, -1, s));
        return UPR_OK;
    };
    bool early = false, tail_kept = false;
    {
        PhaseTimer t(c, 5, s);
        if (b) {
            rc = rebalance_loop_batch(c, p, b, bk, plain, part, pv, conn, W, q->max_rebalance_iters, s);
        } else {
            const int64_t it_max =
                q->max_rebalance_iters > 0 ? q->max_rebalance_iters : default_iters(p, k);
            // moves can overload a block except in constrained rounds. Their
            // speculative first sub-iteration is usually the only one: the
            // round's closing kernels are then enqueued before the host waits
            // for its counts, so that the device runs them while the host
            // turns round (not while the rebalancing or cut phase is timed)
            const bool spec = moves && q->mode != 1;
            early = spec && !prefix && (c->timing.mask & (3u << 5)) == 0;
            rc = rebalance_loop(c, p, bk, plain, part, pv, conn, W, it_max, &iters, &status, s,
                                spec, prefix ? c->bp.rbrec : nullptr, cut_delta,
                                early ? &tail : nullptr, &tail_kept);
        }
        if (rc) return rc;
    }
    if (tail_kept) {
        // what the device derived, from the counts the host decided on
        if (iters == (c->cnt[CNT_OVER0] != 0 ? 1 : 0) && status == (c->cnt[CNT_OVER] != 0 ? 1 : 0))
            return UPR_OK;
    }
    if (prefix) {
        PhaseTimer t(c, 5, s);
        const BpApply ap{bk, p->hub_t, h, p->dirty_threshold, c->dirty, p->table_graph(), tpv,
                         p->order ? (void *)c->pc2 : nullptr, p->perm, p->all_threshold};
        int its = 0;
        const hipError_t e = run_best_prefix(p->g, K, lmax, part, pv, conn, W, c->accflag, c->key,
                                             c->mvto, c->counters, c->bp, ap, stats, &its, s);
        if (e != hipSuccess) {
            (void)hipGetLastError();
            return fail(c, UPR_E_HIP, "best prefix failed: %s", hipGetErrorString(e));
        }
    }
    // an early tail that did not stand: its recount (if any) is undone
    if (early) HIP_TRY(c, launch_cnt_set(c->counters, CNT_CUT2_AFTER, 0, s));
    if ((rc = cut_after())) return rc;
    if (b) {
        HIP_TRY(c, hipMemcpyAsync(b->host3_d, b->host3_h, sizeof(int64_t) * 3 * ng,
                                  hipMemcpyHostToDevice, s));
        HIP_TRY(c, launch_batch_stats_final(ng, gstat, b->lmax_d, b->host3_d, moved ? 1 : 0, stats, s));
        return UPR_OK;
    }
    if (!moves) {
        // standalone rebalancing: nothing moved before it
        HIP_TRY(c, launch_cnt_copy(c->counters, CNT_CUT2_MOVES, CNT_CUT2_BEFORE, s));
    }
    HIP_TRY(c, launch_stats_final(stats, c->counters, lmax, iters, status, s));
    if (prefix) HIP_TRY(c, launch_bp_stats(c->bp, stats, s));
    return UPR_OK;
}

static int round_common(upr_ctx *c, const upr_plan *p, const upr_params *q, int32_t *part,
                        int32_t *conn, int64_t *W, int64_t *stats, hipStream_t s, bool moves)
{
    int rc = check_plan(c, p);
    if (rc) return rc;
    rc = check_params(c, p, q);
    if (rc) return rc;
    if (!W || !stats || (p->g.n > 0 && (!part || !conn)))
        return fail(c, UPR_E_ARG, "part/conn/block_w/stats NULL");
    return round_core(c, p, nullptr, q, part, conn, W, stats, s, moves);
}

int upr_refine_round(upr_ctx *c, const upr_plan *p, const upr_params *q, int32_t *part,
                     int32_t *conn, int64_t *W, int64_t *stats, hipStream_t s)
{
    return round_common(c, p, q, part, conn, W, stats, s, true);
}

int upr_refine_rounds(upr_ctx *c, const upr_plan *p, const upr_params *q, int32_t rounds,
                      int32_t *part, int32_t *conn, int64_t *W, int64_t *stats, hipStream_t s)
{
    if (!c) return UPR_E_ARG;
    if (rounds < 0) return fail(c, UPR_E_ARG, "rounds=%d is negative", rounds);
    if (rounds > 0 && (!q || !stats)) return fail(c, UPR_E_ARG, "params/stats NULL");
    for (int32_t r = 0; r < rounds; ++r) {
        const int rc = round_common(c, p, q + r, part, conn, W, stats + (int64_t)r * UPR_STATS_LEN,
                                    s, true);
        if (rc) return rc;
    }
    return UPR_OK;
}

int upr_rebalance(upr_ctx *c, const upr_plan *p, const upr_params *q, int32_t *part, int32_t *conn,
                  int64_t *W, int64_t *stats, hipStream_t s)
{
    return round_common(c, p, q, part, conn, W, stats, s, false);
}

// ------------------------------------------------------------- batches --

void upr_batch_destroy(upr_batch *b)
{
    if (!b) return;
    (void)hipSetDevice(b->device);
    (void)hipDeviceSynchronize();
    if (b->plan) upr_plan_destroy(b->plan);
    dfree(b->xadj);
    dfree(b->adjncy);
    dfree(b->adjwgt);
    dfree(b->vwgt);
    dfree(b->goff_d);
    dfree(b->lmax_d);
    dfree(b->srcl_d);
    dfree(b->penq_d);
    dfree(b->gstat_d);
    dfree(b->host3_d);
    delete b;
}

int upr_batch_create(upr_ctx *c, const upr_graph *graphs, const int64_t *nnz_host, int32_t ng,
                     int32_t k, int32_t eps_num, int32_t eps_den, int32_t flags,
                     const upr_plan_opts *opts, upr_batch **out, hipStream_t s)
{
    if (!c) return UPR_E_ARG;
    if (!out) return fail(c, UPR_E_ARG, "out is NULL");
    *out = nullptr;
    if (!graphs || ng < 1) return fail(c, UPR_E_ARG, "need at least one graph");
    if (k < 2 || k > UPR_MAX_K) return fail(c, UPR_E_ARG, "k=%d outside [2, %d]", k, UPR_MAX_K);
    if ((int64_t)ng * k > UPR_MAX_BATCH_BLOCKS)
        return fail(c, UPR_E_ARG, "ng*k = %lld blocks exceeds %d", (long long)ng * k,
                    UPR_MAX_BATCH_BLOCKS);
    if (eps_num <= 0 || eps_den <= 0) return fail(c, UPR_E_ARG, "eps must be > 0");
    if (flags & ~UPR_BATCH_TRUSTED) return fail(c, UPR_E_ARG, "unknown batch flags 0x%x", flags);
    const bool trusted = (flags & UPR_BATCH_TRUSTED) != 0;
    HIP_TRY(c, hipSetDevice(c->device));
    upr_batch *b = new upr_batch();
    b->ctx = c;
    b->device = c->device;
    b->ng = ng;
    b->k = k;
    b->eps_num = eps_num;
    b->eps_den = eps_den;
    auto bail = [&](int code, const char *msg) {
        upr_batch_destroy(b);
        return fail(c, code, "%s", msg);
    };
    // sizes and offsets
    std::vector<int64_t> eoff(ng + 1, 0);
    b->off.assign(ng + 1, 0);
    b->weighted.assign(ng, 0);
    bool any_ew = false, any_vw = false;
    for (int32_t g = 0; g < ng; ++g) {
        const upr_graph &G = graphs[g];
        if (G.n < 0 || (G.n > 0 && !G.xadj)) return bail(UPR_E_ARG, "a graph has n < 0 or xadj NULL");
        int64_t nnz = 0;
        if (nnz_host) nnz = G.n > 0 ? nnz_host[g] : 0;
        else if (G.n > 0 && hipMemcpy(&nnz, G.xadj + G.n, sizeof nnz, hipMemcpyDeviceToHost) != hipSuccess)
            return bail(UPR_E_HIP, "reading xadj[n] failed");
        if (nnz < 0 || (nnz > 0 && !G.adjncy)) return bail(UPR_E_GRAPH, "a graph has xadj[n] < 0 or adjncy NULL");
        b->off[g + 1] = b->off[g] + G.n;
        eoff[g + 1] = eoff[g] + nnz;
        b->max_n = std::max<int64_t>(b->max_n, G.n);
        any_ew |= G.adjwgt != nullptr;
        any_vw |= G.vwgt != nullptr;
        b->weighted[g] = G.vwgt != nullptr;
    }
    b->n = b->off[ng];
    b->nnz = eoff[ng];
    if (b->n >= ((int64_t)1 << 31) - 1) return bail(UPR_E_ARG, "the batch has 2^31 nodes or more");
    {
        // statistics pass: ranges no longer than the smallest graph meet at
        // most two graphs
        int64_t min_n = 0;
        for (int32_t g = 0; g < ng; ++g) {
            const int64_t gn = b->off[g + 1] - b->off[g];
            if (gn > 0 && (min_n == 0 || gn < min_n)) min_n = gn;
        }
        b->stats_span = stats_span(b->n, min_n);
        auto graph_of = [&](int64_t v) {
            return (int32_t)(std::upper_bound(b->off.begin(), b->off.end(), v) - b->off.begin()) - 1;
        };
        int32_t most = 1;
        for (int64_t lo = 0; lo < b->n; lo += b->stats_span) {
            const int64_t hi = std::min(lo + b->stats_span, b->n);
            most = std::max(most, graph_of(hi - 1) - graph_of(lo) + 1);
        }
        b->stats_window = most * k;
    }
    // the union CSR
    if (dalloc(&b->xadj, b->n + 1) != hipSuccess || dalloc(&b->adjncy, b->nnz) != hipSuccess ||
        (any_ew && dalloc(&b->adjwgt, b->nnz) != hipSuccess) ||
        (any_vw && dalloc(&b->vwgt, b->n) != hipSuccess) || dalloc(&b->goff_d, ng + 1) != hipSuccess ||
        dalloc(&b->lmax_d, ng) != hipSuccess || dalloc(&b->srcl_d, ng) != hipSuccess ||
        dalloc(&b->penq_d, (int64_t)ng * kSlots) != hipSuccess ||
        dalloc(&b->gstat_d, (int64_t)ng * GS_COUNT) != hipSuccess ||
        dalloc(&b->host3_d, 3 * (int64_t)ng) != hipSuccess)
        return bail(UPR_E_NOMEM, "batch allocation failed");
    if (bind_batch_pinned(c, b) != UPR_OK) return bail(UPR_E_NOMEM, "pinned batch allocation failed");
    // every graph: rows well formed (xadj from 0, nondecreasing; positive node
    // weights) before anything reads its adjacency, then neighbour ids inside
    // the graph and positive edge weights
    unsigned long long init[4] = {~0ull, ~0ull, ~0ull, ~0ull}, got[4];
    HIP_TRY(c, hipMemcpyAsync(c->flags, init, sizeof init, hipMemcpyHostToDevice, s));
    if (!trusted) {
        for (int32_t g = 0; g < ng; ++g) {
            const upr_graph &G = graphs[g];
            if (G.n > 0)
                HIP_TRY(c, launch_validate(GraphView{G.n, G.xadj, G.adjncy, G.adjwgt, G.vwgt}, c->flags, 0, s));
        }
        HIP_TRY(c, hipMemcpyAsync(got, c->flags, sizeof got, hipMemcpyDeviceToHost, s));
        HIP_TRY(c, hipStreamSynchronize(s));
        if (got[0] != ~0ull) return bail(UPR_E_GRAPH, "a graph's xadj does not start at 0 or decreases");
        if (got[3] != ~0ull) return bail(UPR_E_GRAPH, "a graph has a non-positive node weight");
    }
    for (int32_t g = 0; g < ng; ++g) {
        const upr_graph &G = graphs[g];
        const GraphView src{G.n, G.xadj, G.adjncy, G.adjwgt, G.vwgt};
        if (G.n == 0) continue;
        if (!trusted) HIP_TRY(c, launch_validate(src, c->flags, 1, s));
        if (launch_batch_copy(src, b->off[g], eoff[g], eoff[g + 1] - eoff[g], b->xadj, b->adjncy,
                              b->adjwgt, b->vwgt, 0, s) != hipSuccess)
            return bail(UPR_E_HIP, "copying a graph into the batch failed");
    }
    // the closing offset xadj[n] (from pageable memory: the copy completes before returning)
    HIP_TRY(c, hipMemcpyAsync(b->xadj + b->n, &eoff[ng], sizeof(int64_t), hipMemcpyHostToDevice, s));
    HIP_TRY(c, hipMemcpyAsync(got, c->flags, sizeof got, hipMemcpyDeviceToHost, s));
    HIP_TRY(c, hipStreamSynchronize(s));
    if (got[1] != ~0ull) return bail(UPR_E_GRAPH, "a graph names a neighbour outside its own nodes");
    if (got[3] != ~0ull) return bail(UPR_E_GRAPH, "a graph has a non-positive edge weight");
    const upr_graph ug{b->n, b->xadj, b->adjncy, b->adjwgt, b->vwgt};
    int rc = plan_create(c, &ug, &b->plan, s, !trusted, b->nnz, opts, true);
    if (rc) {
        const std::string msg(c->err);
        upr_batch_destroy(b);
        return fail(c, rc, "batch plan: %s", msg.c_str());
    }
    // per-graph L_max from the graphs' total node weights
    std::vector<int64_t> tot(2 * (size_t)ng);
    int64_t *d_tot = nullptr;
    if (dalloc(&d_tot, 2 * (int64_t)ng) != hipSuccess) return bail(UPR_E_NOMEM, "batch allocation failed");
    bool ok = hipMemcpy(b->goff_d, b->off.data(), sizeof(int64_t) * (ng + 1), hipMemcpyHostToDevice) == hipSuccess &&
              launch_batch_totals(b->goff_d, ng, b->vwgt, d_tot, s) == hipSuccess &&
              hipStreamSynchronize(s) == hipSuccess &&
              hipMemcpy(tot.data(), d_tot, sizeof(int64_t) * 2 * ng, hipMemcpyDeviceToHost) == hipSuccess;
    dfree(d_tot);
    if (!ok) return bail(UPR_E_HIP, "batch totals failed");
    b->lmax.resize(ng);
    b->maxvw.resize(ng);
    for (int32_t g = 0; g < ng; ++g) {
        b->lmax[g] = upr_lmax(tot[2 * g], k, eps_num, eps_den);
        b->maxvw[g] = tot[2 * g + 1];
        if (b->maxvw[g] > b->lmax[g]) {
            upr_batch_destroy(b);
            return fail(c, UPR_E_INFEASIBLE, "graph %d: node weight %lld exceeds L_max %lld", g,
                        (long long)tot[2 * g + 1], (long long)b->lmax[g]);
        }
    }
    if (hipMemcpy(b->lmax_d, b->lmax.data(), sizeof(int64_t) * ng, hipMemcpyHostToDevice) != hipSuccess)
        return bail(UPR_E_HIP, "batch upload failed");
    *out = b;
    return UPR_OK;
}

int upr_batch_info(const upr_batch *b, int64_t *n_total, int64_t *nnz_total, int64_t *node_off,
                   int64_t *lmax)
{
    if (!b) return UPR_E_ARG;
    if (n_total) *n_total = b->n;
    if (nnz_total) *nnz_total = b->nnz;
    if (node_off) std::copy(b->off.begin(), b->off.end(), node_off);
    if (lmax) std::copy(b->lmax.begin(), b->lmax.end(), lmax);
    return UPR_OK;
}

static int batch_common(upr_ctx *c, upr_batch *b, const upr_params *q, const int32_t *tau_num,
                        const int32_t *tau_den, int32_t *part, int32_t *conn, int64_t *W,
                        int64_t *stats, hipStream_t s, bool moves)
{
    if (!c) return UPR_E_ARG;
    if (!b) return fail(c, UPR_E_ARG, "batch is NULL");
    if (b->ctx != c) return fail(c, UPR_E_ARG, "batch belongs to another context");
    int rc = check_params(c, b->plan, q);
    if (rc) return rc;
    if (q->k != b->k) return fail(c, UPR_E_ARG, "k=%d but the batch was built for k=%d", q->k, b->k);
    if ((int64_t)q->eps_num * b->eps_den != (int64_t)b->eps_num * q->eps_den)
        return fail(c, UPR_E_ARG, "eps differs from the batch's");
    if (!W || !stats || (b->n > 0 && (!part || !conn)))
        return fail(c, UPR_E_ARG, "part/conn/block_w/stats NULL");
    if ((tau_num == nullptr) != (tau_den == nullptr))
        return fail(c, UPR_E_ARG, "give both tau arrays or neither");
    if (q->variant & UPR_VAR_BEST_PREFIX)
        return fail(c, UPR_E_ARG, "the best-prefix variant is for single-graph rounds");
    HIP_TRY(c, hipSetDevice(c->device));
    // the host mirrors live in the context's pinned area, shared by its
    // batches: the previous call's last copy out of it must have completed
    HIP_TRY(c, hipStreamSynchronize(s));
    if (bind_batch_pinned(c, b) != UPR_OK) return fail(c, UPR_E_NOMEM, "pinned batch allocation failed");
    if (moves) {
        // per-graph penalty tables; graphs in the same round share one
        int64_t last_num = -1, last_den = -1;
        for (int32_t g = 0; g < b->ng; ++g) {
            const int32_t tn = tau_num ? tau_num[g] : q->tau_num;
            const int32_t td = tau_den ? tau_den[g] : q->tau_den;
            if (td <= 0 || tn < 0 || tn > td) return fail(c, UPR_E_ARG, "graph %d: tau must be in [0, 1]", g);
            int64_t *row = b->penq_h + (int64_t)g * kSlots;
            if (g > 0 && tn == last_num && td == last_den) {
                std::copy(row - kSlots, row, row);
            } else {
                host_penq(tn, td, row);
                last_num = tn;
                last_den = td;
            }
        }
        HIP_TRY(c, hipMemcpyAsync(b->penq_d, b->penq_h, sizeof(int64_t) * kSlots * b->ng,
                                  hipMemcpyHostToDevice, s));
    }
    return round_core(c, b->plan, b, q, part, conn, W, stats, s, moves);
}

int upr_batch_carry(upr_ctx *c, const upr_batch *src, const int32_t *src_part,
                    const int32_t *src_conn, const int64_t *src_W, const upr_batch *dst,
                    const int32_t *src_index, int32_t *dst_part, int32_t *dst_conn, int64_t *dst_W,
                    hipStream_t s)
{
    if (!c) return UPR_E_ARG;
    if (!src || !dst || !src_index) return fail(c, UPR_E_ARG, "batch or index NULL");
    if (src->ctx != c || dst->ctx != c) return fail(c, UPR_E_ARG, "batch belongs to another context");
    if (src->k != dst->k) return fail(c, UPR_E_ARG, "k differs (%d and %d)", src->k, dst->k);
    std::vector<int64_t> rec;
    int64_t max_cells = 0;
    for (int32_t g = 0; g < dst->ng; ++g) {
        const int32_t o = src_index[g];
        if (o < 0) continue;
        if (o >= src->ng) return fail(c, UPR_E_ARG, "graph %d: source index %d out of range", g, o);
        const int64_t n = dst->off[g + 1] - dst->off[g];
        if (src->off[o + 1] - src->off[o] != n)
            return fail(c, UPR_E_ARG, "graph %d: %lld nodes, source graph %d has %lld", g, (long long)n,
                        o, (long long)(src->off[o + 1] - src->off[o]));
        rec.insert(rec.end(), {src->off[o], dst->off[g], n, (int64_t)o, (int64_t)g});
        max_cells = std::max<int64_t>(max_cells, std::max<int64_t>(n * src->k, src->k));
    }
    const int32_t nrec = (int32_t)(rec.size() / 5);
    if (nrec == 0) return UPR_OK;
    if ((!src_part || !src_conn || !src_W || !dst_part || !dst_conn || !dst_W))
        return fail(c, UPR_E_ARG, "state array NULL");
    HIP_TRY(c, hipSetDevice(c->device));
    if ((int64_t)rec.size() > c->carry_cap) {
        HIP_TRY(c, hipStreamSynchronize(s));
        dfree(c->carry);
        c->carry_cap = 0;
        const int64_t cap = std::max<int64_t>((int64_t)rec.size(), 5 * 1024);
        if (dalloc(&c->carry, cap) != hipSuccess) {
            (void)hipGetLastError();
            return fail(c, UPR_E_NOMEM, "carry records allocation failed");
        }
        c->carry_cap = cap;
    }
    // the records go through pageable memory: the copy completes before the
    // call returns, so the host vector may go
    HIP_TRY(c, hipMemcpyAsync(c->carry, rec.data(), sizeof(int64_t) * rec.size(), hipMemcpyHostToDevice, s));
    HIP_TRY(c, launch_batch_carry(c->carry, nrec, max_cells, src->k, src_part, src_conn, src_W, dst_part,
                                  dst_conn, dst_W, s));
    return UPR_OK;
}

int upr_batch_refine_round(upr_ctx *c, upr_batch *b, const upr_params *q, const int32_t *tau_num,
                           const int32_t *tau_den, int32_t *part, int32_t *conn, int64_t *W,
                           int64_t *stats, hipStream_t s)
{
    return batch_common(c, b, q, tau_num, tau_den, part, conn, W, stats, s, true);
}

int upr_batch_rebalance(upr_ctx *c, upr_batch *b, const upr_params *q, int32_t *part,
                        int32_t *conn, int64_t *W, int64_t *stats, hipStream_t s)
{
    return batch_common(c, b, q, nullptr, nullptr, part, conn, W, stats, s, false);
}

// --------------------------------------------------------------- driver --

namespace {

// (x) < (num / den) * y for nonnegative integers, exactly.
bool below(int64_t x, int32_t num, int32_t den, int64_t y)
{
    return (__int128)x * den < (__int128)num * y;
}

// tau_1 + (1 - tau_1) (i - 1) / (rounds - 1), reduced to num / den.
void tau_linear(int64_t i, int64_t rounds, int32_t t1n, int32_t t1d, int32_t *num, int32_t *den)
{
    int64_t n, d;
    if (rounds <= 1) {
        n = t1n;
        d = t1d;
    } else {
        // (t1n (R-1) + (t1d - t1n)(i-1)) / (t1d (R-1))
        n = (int64_t)t1n * (rounds - 1) + (int64_t)(t1d - t1n) * (i - 1);
        d = (int64_t)t1d * (rounds - 1);
    }
    int64_t a = n, b = d;
    while (b) {
        const int64_t t = a % b;
        a = b;
        b = t;
    }
    if (a == 0) a = 1;
    *num = (int32_t)(n / a);
    *den = (int32_t)(d / a);
}

}  // namespace

int upr_refine(upr_ctx *c, const upr_plan *p, const upr_driver *d, int32_t *part, int32_t *conn,
               int64_t *W, int64_t *log_stats, int32_t *log_kind, int32_t *n_log, hipStream_t s)
{
    int rc = check_plan(c, p);
    if (rc) return rc;
    if (!d || !n_log || !log_kind || !log_stats) return fail(c, UPR_E_ARG, "driver/log NULL");
    if (d->lp_rounds < 0 || d->fm_rounds < 0 || d->lp_min_den <= 0 || d->lp_min_num < 0 ||
        d->fm_switch_den <= 0 || d->fm_switch_num < 0 || d->tau1_den <= 0 || d->tau1_num < 0 ||
        d->tau1_num > d->tau1_den)
        return fail(c, UPR_E_ARG, "driver parameters out of range");
    upr_params q{};
    q.k = d->k;
    q.eps_num = d->eps_num;
    q.eps_den = d->eps_den;
    q.t_num = d->t_num;
    q.t_den = d->t_den;
    q.tau_num = 1;
    q.tau_den = 1;
    q.rebuild_table = 1;
    q.seq_penalty = d->seq_penalty;
    q.alpha_num = q.alpha_den = 1;
    rc = check_params(c, p, &q);
    if (rc) return rc;
    const int64_t n = p->g.n;
    if (!W || (n > 0 && (!part || !conn))) return fail(c, UPR_E_ARG, "part/conn/block_w NULL");
    HIP_TRY(c, hipSetDevice(c->device));
    int32_t nl = 0;  // log entries: at most lp_rounds + 1 + fm_rounds
    int64_t st[UPR_STATS_LEN];
    uint8_t *active = nullptr;
    int32_t *start = nullptr;
    if (dalloc(&active, n) != hipSuccess || dalloc(&start, n) != hipSuccess) {
        dfree(active);
        dfree(start);
        return fail(c, UPR_E_NOMEM, "driver allocation failed");
    }
    auto done = [&](int code) {
        (void)hipStreamSynchronize(s);
        dfree(active);
        dfree(start);
        *n_log = nl;
        return code;
    };
    auto read_stats = [&](int32_t i) -> int {
        HIP_TRY(c, hipMemcpyAsync(st, log_stats + (int64_t)i * UPR_STATS_LEN, sizeof st,
                                  hipMemcpyDeviceToHost, s));
        HIP_TRY(c, hipStreamSynchronize(s));
        return UPR_OK;
    };
    // label propagation (Section 6): penalty-free rounds on the active set,
    // rollback and stop when a round does not improve
    if (d->lp_rounds > 0 && n > 0) HIP_TRY(c, launch_boundary(p->g, part, active, s));
    for (int32_t r = 0; r < d->lp_rounds && n > 0; ++r) {
        // an empty active set ends the phase
        HIP_TRY(c, launch_count_u8(active, n, (int64_t *)(c->counters + CNT_TMP), s));
        int64_t nact = 0;
        HIP_TRY(c, hipMemcpyAsync(&nact, c->counters + CNT_TMP, sizeof nact, hipMemcpyDeviceToHost, s));
        HIP_TRY(c, hipStreamSynchronize(s));
        if (nact == 0) break;
        HIP_TRY(c, hipMemcpyAsync(start, part, sizeof(int32_t) * n, hipMemcpyDeviceToDevice, s));
        upr_params ql = q;
        ql.mode = 2;
        rc = round_core(c, p, nullptr, &ql, part, conn, W, log_stats + (int64_t)nl * UPR_STATS_LEN, s,
                        true, active);
        if (rc) return done(rc);
        if ((rc = read_stats(nl)) != UPR_OK) return done(rc);
        log_kind[nl++] = UPR_LOG_LP;
        const int64_t before = st[UPR_ST_CUT_BEFORE], after = st[UPR_ST_CUT_AFTER];
        if (after >= before) {
            // no net improvement: restore the round's starting partition
            HIP_TRY(c, hipMemcpyAsync(part, start, sizeof(int32_t) * n, hipMemcpyDeviceToDevice, s));
            HIP_TRY(c, hipMemcpyAsync(log_stats + (int64_t)nl * UPR_STATS_LEN,
                                      log_stats + (int64_t)(nl - 1) * UPR_STATS_LEN,
                                      sizeof(int64_t) * UPR_STATS_LEN, hipMemcpyDeviceToDevice, s));
            log_kind[nl++] = UPR_LOG_ROLLBACK;
            break;
        }
        HIP_TRY(c, launch_next_active(p->g, start, part, active, s));
        if (below(before - after, d->lp_min_num, d->lp_min_den, before)) break;
    }
    // FM rounds (Section 5.5): penalised rounds with tau rising linearly from
    // tau_1, a switch to constrained rounds once a round improves the cut by
    // less than the threshold, and a constrained round at the end
    bool unconstrained = true;
    const int64_t n_unc = std::max<int64_t>(d->fm_rounds - 1, 1);
    int64_t i_unc = 0;
    for (int32_t r = 0; r < d->fm_rounds; ++r) {
        const bool last = r == d->fm_rounds - 1;
        upr_params qf = q;
        int32_t kind;
        if (unconstrained && !last) {
            ++i_unc;
            qf.mode = 0;
            tau_linear(i_unc, n_unc, d->tau1_num, d->tau1_den, &qf.tau_num, &qf.tau_den);
            kind = UPR_LOG_UNCONSTRAINED;
        } else {
            unconstrained = false;
            qf.mode = 1;
            kind = UPR_LOG_CONSTRAINED;
        }
        rc = round_core(c, p, nullptr, &qf, part, conn, W, log_stats + (int64_t)nl * UPR_STATS_LEN,
                        s, true);
        if (rc) return done(rc);
        if ((rc = read_stats(nl)) != UPR_OK) return done(rc);
        log_kind[nl++] = kind;
        const int64_t before = st[UPR_ST_CUT_BEFORE], after = st[UPR_ST_CUT_AFTER];
        const bool small = below(before - after, d->fm_switch_num, d->fm_switch_den, std::max<int64_t>(before, 1));
        if (kind == UPR_LOG_UNCONSTRAINED && small) unconstrained = false;
        else if (kind == UPR_LOG_CONSTRAINED && small) break;
    }
    if (d->fm_rounds == 0 && n > 0) {
        // the table and block weights of the final partition
        HIP_TRY(c, launch_zero_hub_rows(p->hubs(), conn, d->k, s));
        HIP_TRY(c, launch_gain_table(p->g, d->k, PartView{part, 4}, conn, p->hub_t, p->hubs(), s));
        HIP_TRY(c, launch_fill_i64(W, d->k, 0, s));
        HIP_TRY(c, launch_block_weights(p->g, d->k, part, W, c->counters, s));
    }
    return done(UPR_OK);
}

int upr_last_moves(upr_ctx *c, int64_t n, int32_t *target, int64_t *score, int64_t *pen,
                   uint8_t *accept, hipStream_t s)
{
    if (!c) return UPR_E_ARG;
    if (n < 0 || n > c->cap_n) return fail(c, UPR_E_ARG, "n=%lld exceeds the last round's size", (long long)n);
    HIP_TRY(c, hipSetDevice(c->device));
    HIP_TRY(c, launch_export_moves(n, c->key, c->pen, c->accflag, target, score, pen, accept, s));
    return UPR_OK;
}

int upr_capture_enable(upr_ctx *c, int enable)
{
    if (!c) return UPR_E_ARG;
    if (enable && !c->cap_stream) {
        HIP_TRY(c, hipSetDevice(c->device));
        HIP_TRY(c, hipStreamCreateWithFlags(&c->cap_stream, hipStreamNonBlocking));
    }
    if (!enable) {
        HIP_TRY(c, hipSetDevice(c->device));
        HIP_TRY(c, hipDeviceSynchronize());
        drop_captured(c);
    }
    c->capture = enable != 0;
    return UPR_OK;
}

int upr_timing_enable(upr_ctx *c, int enable)
{
    if (!c) return UPR_E_ARG;
    c->timing.mask = (uint32_t)enable & ((1u << UPR_NUM_PHASES) - 1u);
    return UPR_OK;
}

int upr_timing_read(upr_ctx *c, double *ms, int64_t *counts, int reset)
{
    if (!c) return UPR_E_ARG;
    for (auto &pd : c->timing.pending) {
        float x = 0.f;
        (void)hipEventSynchronize(pd.b);
        if (hipEventElapsedTime(&x, pd.a, pd.b) == hipSuccess) {
            c->timing.ms[pd.phase] += x;
            c->timing.counts[pd.phase] += 1;
        }
        c->timing.pool.push_back(pd.a);
        c->timing.pool.push_back(pd.b);
    }
    c->timing.pending.clear();
    for (int i = 0; i < UPR_NUM_PHASES; ++i) {
        if (ms) ms[i] = c->timing.ms[i];
        if (counts) counts[i] = c->timing.counts[i];
        if (reset) {
            c->timing.ms[i] = 0;
            c->timing.counts[i] = 0;
        }
    }
    return UPR_OK;
}

}  // extern "C"
