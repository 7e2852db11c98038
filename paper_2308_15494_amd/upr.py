"""Python binding of libupr (include/upr.h): argument marshalling only.

Every computation runs in the HIP kernels of libupr.so; this module passes
device pointers of torch ROCm tensors and the current HIP stream through the
C ABI. If the library is not built, loading fails with an error: there is no
fallback.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libupr.so")

UPR_OK = 0
ERRORS = {-1: "UPR_E_ARG", -2: "UPR_E_GRAPH", -3: "UPR_E_INFEASIBLE", -4: "UPR_E_NOMEM",
          -5: "UPR_E_HIP"}
STATS_LEN = 12
MAX_BATCH_BLOCKS = 65536  # UPR_MAX_BATCH_BLOCKS: graphs times k of one batch
STAT_NAMES = ["l_max", "cut_before", "cut_after_moves", "cut_after", "candidates",
              "accepted", "rebalance_moves", "rebalance_iters", "status", "prefix_steps",
              "reverted"]
PHASES = ["gain_tile", "stats", "best_move", "filter", "apply", "rebalance", "cut", "call",
          "best_move_kernel", "filter_kernel"]
MODES = {"penalised": 0, "constrained": 1, "free": 2, "limited": 3}


class UprError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"{ERRORS.get(code, code)}: {msg}")
        self.code = code


class _Graph(C.Structure):
    _fields_ = [("n", C.c_int64), ("xadj", C.c_void_p), ("adjncy", C.c_void_p),
                ("adjwgt", C.c_void_p), ("vwgt", C.c_void_p)]


class Params(C.Structure):
    """upr_params: k, eps, t, tau (rationals), mode, rebuild_table, max_rebalance_iters,
    seq_penalty, alpha (rational, mode 3), variant (bit flags)."""
    _fields_ = [("k", C.c_int32), ("eps_num", C.c_int32), ("eps_den", C.c_int32),
                ("t_num", C.c_int32), ("t_den", C.c_int32), ("tau_num", C.c_int32),
                ("tau_den", C.c_int32), ("mode", C.c_int32), ("rebuild_table", C.c_int32),
                ("max_rebalance_iters", C.c_int32), ("seq_penalty", C.c_int32),
                ("alpha_num", C.c_int32), ("alpha_den", C.c_int32), ("variant", C.c_int32)]


VAR_OPTIMISTIC = 1
VAR_PLAIN_PRIORITY = 2
VAR_BEST_PREFIX = 4


def params(k, eps=(3, 100), t=(7, 10), tau=(1, 1), mode=0, rebuild_table=1,
           max_rebalance_iters=0, seq_penalty=1, alpha=(1, 1), variant=0) -> Params:
    if isinstance(mode, str):
        mode = MODES[mode]
    return Params(k, eps[0], eps[1], t[0], t[1], tau[0], tau[1], mode, rebuild_table,
                  max_rebalance_iters, seq_penalty, alpha[0], alpha[1], variant)


_lib = None

# (name, restype, argtypes) of every exported function of include/upr.h
_SIGS = [
    ("upr_create", C.c_int, [C.POINTER(C.c_void_p), C.c_int]),
    ("upr_destroy", None, [C.c_void_p]),
    ("upr_last_error", C.c_char_p, [C.c_void_p]),
    ("upr_plan_create", C.c_int, [C.c_void_p, C.POINTER(_Graph), C.POINTER(C.c_void_p), C.c_void_p]),
    ("upr_plan_destroy", None, [C.c_void_p]),
    ("upr_plan_info", C.c_int, [C.c_void_p] + [C.POINTER(C.c_int64)] * 5),
    ("upr_validate_graph", C.c_int, [C.c_void_p, C.POINTER(_Graph), C.c_void_p]),
    ("upr_gain_table", C.c_int, [C.c_void_p, C.c_void_p, C.c_int32, C.c_void_p, C.c_void_p,
                                 C.c_void_p]),
    ("upr_block_weights", C.c_int, [C.c_void_p, C.c_void_p, C.c_int32, C.c_void_p, C.c_void_p,
                                    C.c_void_p]),
    ("upr_edge_cut", C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p]),
    ("upr_edge_cut_noalloc", C.c_int, [C.c_void_p, C.POINTER(_Graph), C.c_void_p, C.c_void_p,
                                       C.c_void_p]),
    ("upr_refine_round", C.c_int, [C.c_void_p, C.c_void_p, C.POINTER(Params), C.c_void_p,
                                   C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p]),
    ("upr_refine_rounds", C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_int32, C.c_void_p,
                                    C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p]),
    ("upr_rebalance", C.c_int, [C.c_void_p, C.c_void_p, C.POINTER(Params), C.c_void_p,
                                C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p]),
    ("upr_last_moves", C.c_int, [C.c_void_p, C.c_int64, C.c_void_p, C.c_void_p, C.c_void_p,
                                 C.c_void_p, C.c_void_p]),
    ("upr_lmax", C.c_int64, [C.c_int64, C.c_int32, C.c_int32, C.c_int32]),
    ("upr_penalty_table", C.c_int, [C.c_int32, C.c_int32, C.c_void_p]),
    ("upr_best_move_adjacency_degree", C.c_int32, [C.c_int32, C.c_int64]),
    ("upr_batch_create", C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_int32, C.c_int32,
                                   C.c_int32, C.c_int32, C.c_int32, C.c_void_p,
                                   C.POINTER(C.c_void_p), C.c_void_p]),
    ("upr_plan_create_opts", C.c_int, [C.c_void_p, C.POINTER(_Graph), C.c_void_p,
                                       C.POINTER(C.c_void_p), C.c_void_p]),
    ("upr_batch_destroy", None, [C.c_void_p]),
    ("upr_batch_info", C.c_int, [C.c_void_p, C.POINTER(C.c_int64), C.POINTER(C.c_int64),
                                 C.c_void_p, C.c_void_p]),
    ("upr_batch_refine_round", C.c_int, [C.c_void_p, C.c_void_p, C.POINTER(Params), C.c_void_p,
                                         C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p,
                                         C.c_void_p, C.c_void_p]),
    ("upr_batch_carry", C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p,
                                  C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p,
                                  C.c_void_p]),
    ("upr_batch_rebalance", C.c_int, [C.c_void_p, C.c_void_p, C.POINTER(Params), C.c_void_p,
                                      C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p]),
    ("upr_refine", C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p,
                             C.c_void_p, C.c_void_p, C.c_void_p, C.POINTER(C.c_int32),
                             C.c_void_p]),
    ("upr_capture_enable", C.c_int, [C.c_void_p, C.c_int]),
    ("upr_timing_enable", C.c_int, [C.c_void_p, C.c_int]),
    ("upr_timing_read", C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_int]),
]


def lib():
    """Load libupr.so (built by paper_2308_15494_amd.build); raise if absent."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is not built; run __graft_entry__.build() or "
                               "python -m paper_2308_15494_amd.build")
        L = C.CDLL(LIB_PATH)
        for name, res, args in _SIGS:
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


class Driver(C.Structure):
    """upr_driver: label propagation then FM rounds (Sections 5.5 and 6)."""
    _fields_ = [("k", C.c_int32), ("eps_num", C.c_int32), ("eps_den", C.c_int32),
                ("t_num", C.c_int32), ("t_den", C.c_int32), ("lp_rounds", C.c_int32),
                ("lp_min_num", C.c_int32), ("lp_min_den", C.c_int32), ("fm_rounds", C.c_int32),
                ("tau1_num", C.c_int32), ("tau1_den", C.c_int32), ("fm_switch_num", C.c_int32),
                ("fm_switch_den", C.c_int32), ("seq_penalty", C.c_int32)]


LOG_KINDS = {0: "lp", 1: "rollback", 2: "unconstrained", 3: "constrained"}


def driver(k, eps=(3, 100), t=(7, 10), lp_rounds=5, lp_min=(1, 1000), fm_rounds=10,
           tau1=(1, 2), fm_switch=(2, 1000), seq_penalty=1) -> Driver:
    return Driver(k, eps[0], eps[1], t[0], t[1], lp_rounds, lp_min[0], lp_min[1], fm_rounds,
                  tau1[0], tau1[1], fm_switch[0], fm_switch[1], seq_penalty)


def refine(ctx, plan, d: Driver, part, conn, W, stream=None):
    """Run the driver in place; returns [(kind, stats ndarray)] per round."""
    import torch
    cap = d.lp_rounds + 1 + d.fm_rounds
    log = torch.zeros(max(cap, 1) * STATS_LEN, dtype=torch.int64, device=part.device)
    kinds = np.zeros(max(cap, 1), np.int32)
    nl = C.c_int32(0)
    ctx.check(lib().upr_refine(ctx.handle, plan.handle, C.byref(d), _ptr(part), _ptr(conn),
                               _ptr(W), _ptr(log), kinds.ctypes.data, C.byref(nl),
                               _stream(stream)))
    st = log.cpu().numpy().reshape(-1, STATS_LEN)
    return [(LOG_KINDS[int(kinds[i])], st[i].copy()) for i in range(nl.value)]


def lmax(total, k, eps=(3, 100)) -> int:
    return int(lib().upr_lmax(total, k, eps[0], eps[1]))


def best_move_adjacency_degree(k, max_degree) -> int:
    return int(lib().upr_best_move_adjacency_degree(k, max_degree))


def penalty_table(tau) -> np.ndarray:
    out = np.zeros(54, dtype=np.int64)
    rc = lib().upr_penalty_table(tau[0], tau[1], out.ctypes.data)
    if rc != UPR_OK:
        raise UprError(rc, "bad tau")
    return out


def _stream(stream):
    import torch
    if stream is None:
        stream = torch.cuda.current_stream()
    return C.c_void_p(stream.cuda_stream)


def _ptr(t):
    return None if t is None else C.c_void_p(t.data_ptr())


class Context:
    """upr_ctx on one device; owns the device workspace."""

    def __init__(self, device: int = 0):
        self.handle = C.c_void_p()
        rc = lib().upr_create(C.byref(self.handle), device)
        if rc != UPR_OK:
            raise UprError(rc, f"upr_create(device={device}) failed")
        self.device = device

    def check(self, rc):
        if rc != UPR_OK:
            raise UprError(rc, lib().upr_last_error(self.handle).decode())

    def close(self):
        if self.handle:
            lib().upr_destroy(self.handle)
            self.handle = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def capture(self, enable: bool):
        """Replay the move phases of repeated round configurations from HIP
        graphs (upr_capture_enable)."""
        self.check(lib().upr_capture_enable(self.handle, 1 if enable else 0))

    def timing(self, enable: bool, phases=None):
        """Time every phase (enable, phases None), only the listed phases
        (names or indices into PHASES), or nothing."""
        mask = 0
        if enable:
            if phases is None:
                mask = (1 << len(PHASES)) - 1
            else:
                for ph in phases:
                    mask |= 1 << (PHASES.index(ph) if isinstance(ph, str) else int(ph))
        self.check(lib().upr_timing_enable(self.handle, mask))

    def timing_read(self, reset=True) -> dict:
        ms = np.zeros(len(PHASES), np.float64)
        cnt = np.zeros(len(PHASES), np.int64)
        self.check(lib().upr_timing_read(self.handle, ms.ctypes.data, cnt.ctypes.data, int(reset)))
        return {name: (float(ms[i]), int(cnt[i])) for i, name in enumerate(PHASES)}


class DeviceGraph:
    """A graphgen.Graph uploaded to device memory (torch tensors)."""

    def __init__(self, g, device="cuda"):
        import torch
        self.n = int(g.n)
        self.nnz = int(g.xadj[-1]) if g.n > 0 else 0
        self.m = self.nnz // 2
        self.xadj = torch.from_numpy(np.ascontiguousarray(g.xadj, np.int64)).to(device)
        self.adjncy = torch.from_numpy(np.ascontiguousarray(g.adjncy, np.int32)).to(device)
        self.adjwgt = None if g.adjwgt is None else torch.from_numpy(
            np.ascontiguousarray(g.adjwgt, np.int32)).to(device)
        self.vwgt = None if g.vwgt is None else torch.from_numpy(
            np.ascontiguousarray(g.vwgt, np.int32)).to(device)
        self.c = _Graph(self.n, self.xadj.data_ptr(), self.adjncy.data_ptr(),
                        _ptr(self.adjwgt), _ptr(self.vwgt))


class PlanOpts(C.Structure):
    """upr_plan_opts: traversal thresholds (0 = default; low_threshold is
    ignored by the library)."""
    _fields_ = [("hub_threshold", C.c_int64), ("low_threshold", C.c_int64),
                ("dirty_div", C.c_int64)]


def plan_opts(hub_threshold=0, dirty_div=0) -> PlanOpts:
    return PlanOpts(hub_threshold, 0, dirty_div)


class Plan:
    """upr_plan: a prepared graph (degrees, hub chunks). Keeps the graph alive."""

    def __init__(self, ctx: Context, dg: DeviceGraph, stream=None, opts: PlanOpts = None):
        self.ctx = ctx
        self.graph = dg
        self.handle = C.c_void_p()
        self.opts = opts
        if opts is None:
            ctx.check(lib().upr_plan_create(ctx.handle, C.byref(dg.c), C.byref(self.handle),
                                            _stream(stream)))
        else:
            ctx.check(lib().upr_plan_create_opts(ctx.handle, C.byref(dg.c), C.byref(opts),
                                                 C.byref(self.handle), _stream(stream)))

    def info(self) -> dict:
        vals = [C.c_int64() for _ in range(5)]
        self.ctx.check(lib().upr_plan_info(self.handle, *[C.byref(v) for v in vals]))
        return dict(zip(["n", "nnz", "total_weight", "max_degree", "num_hubs"],
                        [v.value for v in vals]))

    def close(self):
        if self.handle:
            lib().upr_plan_destroy(self.handle)
            self.handle = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def validate_graph(ctx: Context, dg: DeviceGraph, stream=None):
    ctx.check(lib().upr_validate_graph(ctx.handle, C.byref(dg.c), _stream(stream)))


def gain_table(ctx, plan, k, part, conn=None, stream=None):
    import torch
    if conn is None:
        conn = torch.empty(plan.graph.n * k, dtype=torch.int32, device=part.device)
    ctx.check(lib().upr_gain_table(ctx.handle, plan.handle, k, _ptr(part), _ptr(conn),
                                   _stream(stream)))
    return conn


def block_weights(ctx, plan, k, part, W=None, stream=None):
    import torch
    if W is None:
        W = torch.empty(k, dtype=torch.int64, device=part.device)
    ctx.check(lib().upr_block_weights(ctx.handle, plan.handle, k, _ptr(part), _ptr(W),
                                      _stream(stream)))
    return W


def edge_cut(ctx, plan, part, out=None, stream=None):
    import torch
    if out is None:
        out = torch.empty(1, dtype=torch.int64, device=part.device)
    ctx.check(lib().upr_edge_cut(ctx.handle, plan.handle, _ptr(part), _ptr(out), _stream(stream)))
    return out


NOALLOC_MAX_NODES = 1 << 28


def edge_cut_noalloc(ctx, dg, part, out, stream=None):
    """upr_edge_cut_noalloc: the cut of part on DeviceGraph dg into the
    caller's device int64 tensor out (nothing is allocated)."""
    ctx.check(lib().upr_edge_cut_noalloc(ctx.handle, C.byref(dg.c), _ptr(part), _ptr(out),
                                         _stream(stream)))
    return out


def refine_round(ctx, plan, p: Params, part, conn, W, stats=None, stream=None):
    """One round in place on (part, conn, W); returns the device stats tensor."""
    import torch
    if stats is None:
        stats = torch.empty(STATS_LEN, dtype=torch.int64, device=part.device)
    ctx.check(lib().upr_refine_round(ctx.handle, plan.handle, C.byref(p), _ptr(part), _ptr(conn),
                                     _ptr(W), _ptr(stats), _stream(stream)))
    return stats


def refine_rounds(ctx, plan, ps, part, conn, W, stats=None, stream=None):
    """Rounds with the Params of the sequence ps, one after another, in one
    call (upr_refine_rounds); returns the device stats tensor [len(ps),
    STATS_LEN]."""
    import torch
    arr = (Params * len(ps))(*ps)
    if stats is None:
        stats = torch.empty((max(len(ps), 1), STATS_LEN), dtype=torch.int64, device=part.device)
    ctx.check(lib().upr_refine_rounds(ctx.handle, plan.handle, C.cast(arr, C.c_void_p), len(ps),
                                      _ptr(part), _ptr(conn), _ptr(W), _ptr(stats),
                                      _stream(stream)))
    return stats


def rebalance(ctx, plan, p: Params, part, conn, W, stats=None, stream=None):
    import torch
    if stats is None:
        stats = torch.empty(STATS_LEN, dtype=torch.int64, device=part.device)
    ctx.check(lib().upr_rebalance(ctx.handle, plan.handle, C.byref(p), _ptr(part), _ptr(conn),
                                  _ptr(W), _ptr(stats), _stream(stream)))
    return stats


def last_moves(ctx, n, device="cuda", stream=None) -> dict:
    import torch
    out = dict(target=torch.empty(n, dtype=torch.int32, device=device),
               score=torch.empty(n, dtype=torch.int64, device=device),
               pen=torch.empty(n, dtype=torch.int64, device=device),
               accept=torch.empty(n, dtype=torch.uint8, device=device))
    ctx.check(lib().upr_last_moves(ctx.handle, n, _ptr(out["target"]), _ptr(out["score"]),
                                   _ptr(out["pen"]), _ptr(out["accept"]), _stream(stream)))
    return out


def stats_dict(stats) -> dict:
    s = stats.cpu().numpy() if hasattr(stats, "cpu") else np.asarray(stats)
    return {name: int(s[i]) for i, name in enumerate(STAT_NAMES)}


class Refiner:
    """Convenience holder: graph on device, plan, and (part, conn, W) state."""

    def __init__(self, g, k, device=0, ctx=None, opts: PlanOpts = None):
        import torch
        self.ctx = ctx or Context(device)
        self.dev = torch.device("cuda", device)
        self.dg = DeviceGraph(g, self.dev)
        self.plan = Plan(self.ctx, self.dg, opts=opts)
        self.k = k
        self.conn = torch.zeros(max(self.dg.n * k, 1), dtype=torch.int32, device=self.dev)
        self.W = torch.zeros(k, dtype=torch.int64, device=self.dev)
        self.stats = torch.zeros(STATS_LEN, dtype=torch.int64, device=self.dev)
        self.part = None

    def set_partition(self, part):
        import torch
        self.part = torch.from_numpy(np.ascontiguousarray(part, np.int32)).to(self.dev)

    def round(self, p: Params):
        refine_round(self.ctx, self.plan, p, self.part, self.conn, self.W, self.stats)
        return self.stats

    def rounds(self, ps, stats=None):
        """The rounds of ps in one call; returns their stats [len(ps), STATS_LEN]."""
        return refine_rounds(self.ctx, self.plan, ps, self.part, self.conn, self.W, stats)

    def rebalance(self, p: Params):
        rebalance(self.ctx, self.plan, p, self.part, self.conn, self.W, self.stats)
        return self.stats


class Batch:
    """upr_batch: graphs with a common k and eps refined by the same launches.

    The library copies the graphs into one union (graph g's nodes at
    off[g]..off[g+1]); part holds global block ids g*k + j, W is [ng * k],
    stats [ng, STATS_LEN]. The input DeviceGraphs may be dropped after
    construction."""

    def __init__(self, ctx: Context, graphs, k, eps=(3, 100), stream=None, trusted=False,
                 opts: PlanOpts = None):
        """trusted: every graph was validated before (UPR_BATCH_TRUSTED);
        opts: the union's plan thresholds."""
        import torch
        self.ctx, self.k, self.eps = ctx, k, eps
        self.ng = len(graphs)
        dgs = [g if isinstance(g, DeviceGraph) else DeviceGraph(g) for g in graphs]
        arr = (_Graph * self.ng)(*[d.c for d in dgs])
        nnz = np.ascontiguousarray([d.nnz for d in dgs], np.int64)
        self.handle = C.c_void_p()
        ctx.check(lib().upr_batch_create(ctx.handle, C.cast(arr, C.c_void_p), nnz.ctypes.data,
                                         self.ng, k, eps[0], eps[1], 1 if trusted else 0,
                                         None if opts is None else C.byref(opts),
                                         C.byref(self.handle), _stream(stream)))
        torch.cuda.synchronize()
        n, nnz = C.c_int64(), C.c_int64()
        self.off = np.zeros(self.ng + 1, np.int64)
        self.lmax = np.zeros(self.ng, np.int64)
        ctx.check(lib().upr_batch_info(self.handle, C.byref(n), C.byref(nnz),
                                       self.off.ctypes.data, self.lmax.ctypes.data))
        self.n, self.nnz = n.value, nnz.value
        dev = torch.device("cuda", ctx.device)
        self.dev = dev
        self.conn = torch.zeros(max(self.n * k, 1), dtype=torch.int32, device=dev)
        self.W = torch.zeros(self.ng * k, dtype=torch.int64, device=dev)
        self.stats = torch.zeros(self.ng * STATS_LEN, dtype=torch.int64, device=dev)
        self.part = None

    def set_partitions(self, parts):
        """parts: one local partition (values in [0, k)) per graph, or None for
        a graph whose slice is filled on the device afterwards (carry_from);
        then only the given slices are uploaded."""
        import torch
        if any(p is None for p in parts):
            self.part = torch.zeros(self.n, dtype=torch.int32, device=self.dev)
            for g, p in enumerate(parts):
                if p is None or self.off[g + 1] == self.off[g]:
                    continue
                glob = (np.asarray(p, np.int64) + g * self.k).astype(np.int32)
                self.part[self.off[g]:self.off[g + 1]].copy_(torch.from_numpy(glob))
            return
        glob = np.zeros(max(self.n, 1), np.int32)
        for g, p in enumerate(parts):
            glob[self.off[g]:self.off[g + 1]] = np.asarray(p, np.int64) + g * self.k
        self.part = torch.from_numpy(glob[: self.n] if self.n else glob[:0]).to(self.dev)

    def local_partitions(self, graphs=None):
        """Local partitions of every graph, or only of the graphs listed (in
        that order, each slice downloaded by itself)."""
        if graphs is not None:
            return [(self.part[self.off[g]:self.off[g + 1]].cpu().numpy().astype(np.int64)
                     - g * self.k).astype(np.int32) for g in graphs]
        p = self.part.cpu().numpy().astype(np.int64)
        return [(p[self.off[g]:self.off[g + 1]] - g * self.k).astype(np.int32)
                for g in range(self.ng)]

    def graph_stats(self) -> list:
        st = self.stats.cpu().numpy().reshape(self.ng, STATS_LEN)
        return [stats_dict(st[g]) for g in range(self.ng)]

    def round(self, p: Params, taus=None, stream=None):
        """taus: one (num, den) per graph, or None for p's tau everywhere."""
        tn = td = None
        if taus is not None:
            tn = np.ascontiguousarray([t[0] for t in taus], np.int32)
            td = np.ascontiguousarray([t[1] for t in taus], np.int32)
        self.ctx.check(lib().upr_batch_refine_round(
            self.ctx.handle, self.handle, C.byref(p),
            None if tn is None else tn.ctypes.data, None if td is None else td.ctypes.data,
            _ptr(self.part), _ptr(self.conn), _ptr(self.W), _ptr(self.stats), _stream(stream)))
        return self.stats

    def rebalance(self, p: Params, stream=None):
        self.ctx.check(lib().upr_batch_rebalance(self.ctx.handle, self.handle, C.byref(p),
                                                 _ptr(self.part), _ptr(self.conn), _ptr(self.W),
                                                 _ptr(self.stats), _stream(stream)))
        return self.stats

    def carry_from(self, src: "Batch", src_index, stream=None):
        """upr_batch_carry: graphs of this batch with src_index[g] >= 0 take
        the partition, table rows and block weights of graph src_index[g] of
        src (device to device)."""
        idx = np.ascontiguousarray(src_index, np.int32)
        if self.part is None:
            raise ValueError("set_partitions first (the carried graphs' slices are overwritten)")
        self.ctx.check(lib().upr_batch_carry(
            self.ctx.handle, src.handle, _ptr(src.part), _ptr(src.conn), _ptr(src.W), self.handle,
            idx.ctypes.data, _ptr(self.part), _ptr(self.conn), _ptr(self.W), _stream(stream)))

    def close(self):
        if self.handle:
            lib().upr_batch_destroy(self.handle)
            self.handle = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
