"""ctypes binding of the CPU oracle (upr_oracle.c).

TEST INFRASTRUCTURE ONLY: the tests, the smoke check and the CPU-baseline leg
of the benchmark use it; the product path never imports it. All arrays are
host numpy arrays; the oracle works in place like the round it models.

Statistics slots (int64[12]):
    0 l_max, 1 cut_before, 2 cut_after_moves, 3 cut_after, 4 candidates,
    5 accepted, 6 rebalance_moves, 7 rebalance_iters, 8 status (0 balanced,
    1 rebalancing stuck or out of iterations), 9 prefix_steps and
    10 reverted (best-prefix rounds: filtered moves kept, -1 if no boundary
    was balanced; nodes returned to their round-start block), 11 unused.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "upr_oracle.c")
LIB = os.path.join(HERE, "liborc.so")
SLOTS = 54
STATS = 12
STAT_NAMES = ["l_max", "cut_before", "cut_after_moves", "cut_after", "candidates",
              "accepted", "rebalance_moves", "rebalance_iters", "status", "prefix_steps",
              "reverted"]


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (single-threaded, -O2)."""
    if force or not os.path.exists(LIB) or os.path.getmtime(LIB) < os.path.getmtime(SRC):
        tmp = LIB + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-std=c11", "-Wall", "-Wextra", "-fPIC", "-shared",
                               SRC, "-o", tmp])
        os.replace(tmp, LIB)
    return LIB


class _Graph(C.Structure):
    _fields_ = [("n", C.c_int64), ("xadj", C.c_void_p), ("adjncy", C.c_void_p),
                ("adjwgt", C.c_void_p), ("vwgt", C.c_void_p)]


class _Params(C.Structure):
    _fields_ = [("k", C.c_int32), ("eps_num", C.c_int32), ("eps_den", C.c_int32),
                ("t_num", C.c_int32), ("t_den", C.c_int32), ("tau_num", C.c_int32),
                ("tau_den", C.c_int32), ("mode", C.c_int32), ("rebuild_table", C.c_int32),
                ("max_rebalance_iters", C.c_int32), ("seq_penalty", C.c_int32),
                ("alpha_num", C.c_int32), ("alpha_den", C.c_int32), ("variant", C.c_int32)]


class _Debug(C.Structure):
    _fields_ = [("target", C.c_void_p), ("score", C.c_void_p), ("pen", C.c_void_p),
                ("accept", C.c_void_p), ("pen_seq", C.c_void_p), ("gp", C.c_void_p),
                ("seq", C.c_void_p), ("bgain", C.c_void_p), ("bbal", C.c_void_p),
                ("pref", C.c_void_p), ("rrec", C.c_void_p)]


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB) or os.path.getmtime(LIB) < os.path.getmtime(SRC):
            build(force=True)
        L = C.CDLL(LIB)
        L.orc_lmax.restype = C.c_int64
        L.orc_lmax.argtypes = [C.c_int64, C.c_int32, C.c_int32, C.c_int32]
        L.orc_slot.restype = C.c_int32
        L.orc_slot.argtypes = [C.c_int64, C.c_int64]
        L.orc_penq.restype = None
        L.orc_penq.argtypes = [C.c_int32, C.c_int32, C.c_void_p]
        L.orc_total_weight.restype = C.c_int64
        L.orc_total_weight.argtypes = [C.POINTER(_Graph)]
        L.orc_gain_table.restype = None
        L.orc_gain_table.argtypes = [C.POINTER(_Graph), C.c_int32, C.c_void_p, C.c_void_p]
        L.orc_block_weights.restype = None
        L.orc_block_weights.argtypes = [C.POINTER(_Graph), C.c_int32, C.c_void_p, C.c_void_p]
        L.orc_cut_edges.restype = C.c_int64
        L.orc_cut_edges.argtypes = [C.POINTER(_Graph), C.c_void_p]
        L.orc_cut_table.restype = C.c_int64
        L.orc_cut_table.argtypes = [C.POINTER(_Graph), C.c_int32, C.c_void_p, C.c_void_p]
        L.orc_penalty_buckets.restype = None
        L.orc_penalty_buckets.argtypes = [C.POINTER(_Graph), C.c_int32, C.c_void_p, C.c_void_p,
                                          C.c_int32, C.c_int32, C.c_void_p, C.c_void_p]
        L.orc_refine_round.restype = C.c_int
        L.orc_refine_round.argtypes = [C.POINTER(_Graph), C.POINTER(_Params), C.c_void_p,
                                       C.c_void_p, C.c_void_p, C.c_void_p, C.POINTER(_Debug)]
        L.orc_refine_round_active.restype = C.c_int
        L.orc_refine_round_active.argtypes = [C.POINTER(_Graph), C.POINTER(_Params), C.c_void_p,
                                              C.c_void_p, C.c_void_p, C.c_void_p,
                                              C.POINTER(_Debug), C.c_void_p]
        L.orc_rebalance.restype = C.c_int
        L.orc_rebalance.argtypes = [C.POINTER(_Graph), C.POINTER(_Params), C.c_void_p,
                                    C.c_void_p, C.c_void_p, C.c_void_p]
        _lib = L
    return _lib


def _ptr(a):
    return None if a is None else a.ctypes.data


def _check(a, dtype, size, name):
    if a is None:
        return
    if a.dtype != dtype or not a.flags.c_contiguous or a.size < size:
        raise ValueError(f"{name}: need contiguous {dtype} of size >= {size}")


class Graph:
    """Keeps the numpy arrays alive while the C struct points into them."""

    def __init__(self, g):
        self.n = int(g.n)
        self.xadj = np.ascontiguousarray(g.xadj, dtype=np.int64)
        self.adjncy = np.ascontiguousarray(g.adjncy, dtype=np.int32)
        self.adjwgt = None if g.adjwgt is None else np.ascontiguousarray(g.adjwgt, dtype=np.int32)
        self.vwgt = None if g.vwgt is None else np.ascontiguousarray(g.vwgt, dtype=np.int32)
        self.c = _Graph(self.n, _ptr(self.xadj), _ptr(self.adjncy), _ptr(self.adjwgt),
                        _ptr(self.vwgt))


OPTIMISTIC = 1        # variant bit: optimistic conflict filter
PLAIN_PRIORITY = 2    # variant bit: rebalancing priority by the plain gain
BEST_PREFIX = 4       # variant bit: interleaved move sequence and best prefix


def params(k, eps=(3, 100), t=(7, 10), tau=(1, 1), mode=0, rebuild_table=1,
           max_rebalance_iters=0, seq_penalty=1, alpha=(1, 1), variant=0) -> _Params:
    return _Params(k, eps[0], eps[1], t[0], t[1], tau[0], tau[1], mode, rebuild_table,
                   max_rebalance_iters, seq_penalty, alpha[0], alpha[1], variant)


def lmax(total, k, eps=(3, 100)):
    return int(lib().orc_lmax(total, k, eps[0], eps[1]))


def slot(w, c):
    return int(lib().orc_slot(w, c))


def penq(tau):
    out = np.zeros(SLOTS, dtype=np.int64)
    lib().orc_penq(tau[0], tau[1], out.ctypes.data)
    return out


def total_weight(g):
    G = g if isinstance(g, Graph) else Graph(g)
    return int(lib().orc_total_weight(C.byref(G.c)))


def gain_table(g, k, part):
    G = g if isinstance(g, Graph) else Graph(g)
    part = np.ascontiguousarray(part, dtype=np.int32)
    conn = np.zeros(G.n * k, dtype=np.int32)
    lib().orc_gain_table(C.byref(G.c), k, part.ctypes.data, conn.ctypes.data)
    return conn.reshape(G.n, k)


def block_weights(g, k, part):
    G = g if isinstance(g, Graph) else Graph(g)
    part = np.ascontiguousarray(part, dtype=np.int32)
    W = np.zeros(k, dtype=np.int64)
    lib().orc_block_weights(C.byref(G.c), k, part.ctypes.data, W.ctypes.data)
    return W


def cut_edges(g, part):
    G = g if isinstance(g, Graph) else Graph(g)
    part = np.ascontiguousarray(part, dtype=np.int32)
    return int(lib().orc_cut_edges(C.byref(G.c), part.ctypes.data))


def cut_table(g, k, part, conn):
    G = g if isinstance(g, Graph) else Graph(g)
    part = np.ascontiguousarray(part, dtype=np.int32)
    conn = np.ascontiguousarray(conn, dtype=np.int32)
    return int(lib().orc_cut_table(C.byref(G.c), k, part.ctypes.data, conn.ctypes.data))


def penalty_buckets(g, k, part, conn, t=(7, 10)):
    """Bucket weights c(B_{l,j}) as int64[k, 54] and per-node 1+slot (0 if the
    node is not available for rebalancing)."""
    G = g if isinstance(g, Graph) else Graph(g)
    part = np.ascontiguousarray(part, dtype=np.int32)
    conn = np.ascontiguousarray(conn, dtype=np.int32).reshape(-1)
    bucket = np.zeros(k * SLOTS, dtype=np.int64)
    avail = np.zeros(G.n, dtype=np.int32)
    lib().orc_penalty_buckets(C.byref(G.c), k, part.ctypes.data, conn.ctypes.data, t[0], t[1],
                              bucket.ctypes.data, avail.ctypes.data)
    return bucket.reshape(k, SLOTS), avail


def refine_round(g, p: _Params, part, conn=None, W=None, debug=False, active=None):
    """Run one round in place on (part, conn, W). Returns (stats, dbg) where dbg
    is a dict of per-node arrays (target, score, pen, accept, pen_seq, gp) or None. active:
    optional uint8 mask of the nodes that may look for a move."""
    G = g if isinstance(g, Graph) else Graph(g)
    k = p.k
    _check(part, np.int32, G.n, "part")
    if conn is None:
        conn = np.zeros(G.n * k, dtype=np.int32)
    if W is None:
        W = np.zeros(k, dtype=np.int64)
    _check(conn.reshape(-1), np.int32, G.n * k, "conn")
    _check(W, np.int64, k, "W")
    stats = np.zeros(STATS, dtype=np.int64)
    dbg = None
    dstruct = None
    if debug:
        dbg = dict(target=np.zeros(G.n, np.int32), score=np.zeros(G.n, np.int64),
                   pen=np.zeros(G.n, np.int64), accept=np.zeros(G.n, np.uint8),
                   pen_seq=np.zeros(G.n, np.int64), gp=np.zeros(G.n, np.int64),
                   seq=np.zeros(4 * max(G.n, 1), np.int64),
                   bgain=np.zeros(G.n + 1, np.int64), bbal=np.zeros(G.n + 1, np.uint8),
                   pref=np.full(4, -2, np.int64), rrec=np.zeros(max(G.n, 1), np.int64))
        dstruct = _Debug(*[dbg[f].ctypes.data for f, _ in _Debug._fields_])
    if active is not None:
        _check(active, np.uint8, G.n, "active")
    rc = lib().orc_refine_round_active(C.byref(G.c), C.byref(p), part.ctypes.data,
                                       conn.ctypes.data, W.ctypes.data, stats.ctypes.data,
                                       C.byref(dstruct) if dstruct is not None else None,
                                       None if active is None else active.ctypes.data)
    if rc != 0:
        raise ValueError(f"oracle refine_round rejected its arguments (rc={rc})")
    if dbg is not None and dbg["pref"][0] >= 0:
        # best-prefix round: trim the sequence and boundary arrays to size
        ln, nm = int(dbg["pref"][0]), int(dbg["pref"][1])
        dbg["seq"] = dbg["seq"][: 4 * ln].reshape(ln, 4)
        dbg["bgain"] = dbg["bgain"][: nm + 1]
        dbg["bbal"] = dbg["bbal"][: nm + 1]
    return stats, dbg


def rebalance(g, p: _Params, part, conn=None, W=None):
    G = g if isinstance(g, Graph) else Graph(g)
    k = p.k
    _check(part, np.int32, G.n, "part")
    if conn is None:
        conn = np.zeros(G.n * k, dtype=np.int32)
    if W is None:
        W = np.zeros(k, dtype=np.int64)
    stats = np.zeros(STATS, dtype=np.int64)
    rc = lib().orc_rebalance(C.byref(G.c), C.byref(p), part.ctypes.data, conn.ctypes.data,
                             W.ctypes.data, stats.ctypes.data)
    if rc != 0:
        raise ValueError(f"oracle rebalance rejected its arguments (rc={rc})")
    return stats


def stats_dict(stats) -> dict:
    return {name: int(stats[i]) for i, name in enumerate(STAT_NAMES)}
