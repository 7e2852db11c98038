"""Slow, definition-level reference computations used to pin the oracle.

Everything here is written from the problem statement of Section 2 and the
penalty definitions of Section 5.3 with Python integers and Fractions, on
tiny inputs: edge lists instead of tables, sets instead of histograms, cut
differences instead of table lookups.
"""
from __future__ import annotations

import itertools
from fractions import Fraction

import numpy as np


def edges(g):
    """Undirected edge list [(u, v, w)] with u < v."""
    out = []
    for v in range(g.n):
        for e in range(int(g.xadj[v]), int(g.xadj[v + 1])):
            u = int(g.adjncy[e])
            if v < u:
                out.append((v, u, 1 if g.adjwgt is None else int(g.adjwgt[e])))
    return out


def node_w(g, v):
    return 1 if g.vwgt is None else int(g.vwgt[v])


def cut(g, part):
    return sum(w for u, v, w in edges(g) if part[u] != part[v])


def omega(g, v, block, part):
    """omega(v, V_block): edge weight from v into the block."""
    s = 0
    for e in range(int(g.xadj[v]), int(g.xadj[v + 1])):
        if part[int(g.adjncy[e])] == block:
            s += 1 if g.adjwgt is None else int(g.adjwgt[e])
    return s


def wdeg(g, v):
    return sum(1 if g.adjwgt is None else int(g.adjwgt[e])
               for e in range(int(g.xadj[v]), int(g.xadj[v + 1])))


def block_weight(g, part, j):
    return sum(node_w(g, v) for v in range(g.n) if part[v] == j)


def move_gain(g, part, v, j):
    """gain(m) = cut(Pi) - cut(Pi o m), by recomputing the cut."""
    after = list(part)
    after[v] = j
    return cut(g, part) - cut(g, after)


def lmax_exact(total, k, eps):
    """L_max = (1 + eps) * ceil(c(V)/k), rounded down to an integer weight."""
    per = -(-total // k)
    return int((1 + Fraction(*eps)) * per // 1)


def slot_exact(w, c, slots=54):
    """ceil(log_{3/2}(w/c)) as the least integer l with (3/2)^l >= w/c,
    clamped to [0, slots-1]."""
    if w <= 0:
        return 0
    r = Fraction(w, c)
    l = 0
    while Fraction(3, 2) ** l < r:
        l += 1
    return min(max(l, 0), slots - 1)


def available_sets(g, k, part, t):
    """B[j][l] as Python sets of nodes available for rebalancing."""
    B = [[set() for _ in range(54)] for _ in range(k)]
    for v in range(g.n):
        a = part[v]
        inner = omega(g, v, a, part)
        if Fraction(inner) >= Fraction(*t) * wdeg(g, v):
            B[a][slot_exact(inner, node_w(g, v))].add(v)
    return B


def penalty_q16(g, k, part, t, tau, v, j, lmax):
    """Penalty of moving v into V_j in Q16 (None = forbidden).

    No penalty when V_j + v stays within L_max; otherwise l is the least slot
    whose cumulative bucket weight covers c(V_j + v) - L_max and the penalty is
    tau * (3/2)^l * c(v), the per-unit factor rounded down to Q16 first.
    """
    need = block_weight(g, part, j) + node_w(g, v) - lmax
    if need <= 0:
        return 0
    B = available_sets(g, k, part, t)
    acc = 0
    for l in range(54):
        acc += sum(node_w(g, u) for u in B[j][l])
        if acc >= need:
            per_unit = (Fraction(*tau) * Fraction(3, 2) ** l * 65536) // 1
            return min(int(per_unit) * node_w(g, v), 1 << 62)
    return None


def move_cap(L, mode, alpha):
    """Largest weight a move may bring its target to without penalty:
    L_max, or floor(alpha * L_max) in the limited-imbalance variant."""
    return int(Fraction(*alpha) * L // 1) if mode == 3 else L


def best_moves(g, k, part, t, tau, eps, mode=0, alpha=(1, 1)):
    """S2 by brute force: for each v, argmax over blocks j != Pi(v) of
    gain * 2^16 - penalty (ties to the smaller j); candidate iff > 0.
    Mode 3 (limited imbalance): no penalty, and only targets that stay within
    floor(alpha * L_max). Returns dict v -> (target, score, pen)."""
    total = sum(node_w(g, v) for v in range(g.n))
    L = lmax_exact(total, k, eps)
    cap = move_cap(L, mode, alpha)
    out = {}
    for v in range(g.n):
        best = None
        for j in range(k):
            if j == part[v]:
                continue
            if omega(g, v, j, part) == 0:
                continue
            fits = block_weight(g, part, j) + node_w(g, v) <= cap
            if mode in (1, 3) and not fits:
                continue
            P = 0 if mode in (2, 3) else penalty_q16(g, k, part, t, tau, v, j, L)
            if P is None:
                continue
            s = move_gain(g, part, v, j) * 65536 - P
            if best is None or s > best[1]:
                best = (j, s, P)
        if best is not None and best[1] > 0:
            out[v] = best
    return out


def all_partitions(n, k):
    """Every assignment of n nodes to k blocks as an int8 array [k^n, n]."""
    idx = np.arange(k ** n, dtype=np.int64)
    digits = np.empty((k ** n, n), dtype=np.int8)
    for i in range(n):
        digits[:, i] = idx % k
        idx //= k
    return digits


def optimum(g, k, eps):
    """Minimum cut over all balanced k-way partitions (exhaustive)."""
    P = all_partitions(g.n, k)
    vw = np.ones(g.n, np.int64) if g.vwgt is None else g.vwgt.astype(np.int64)
    total = int(vw.sum())
    L = lmax_exact(total, k, eps)
    ok = np.ones(P.shape[0], dtype=bool)
    for j in range(k):
        ok &= ((P == j).astype(np.int64) @ vw) <= L
    best = None
    E = edges(g)
    cutv = np.zeros(P.shape[0], dtype=np.int64)
    for u, v, w in E:
        cutv += w * (P[:, u] != P[:, v])
    cutv = np.where(ok, cutv, np.iinfo(np.int64).max)
    i = int(np.argmin(cutv))
    best = int(cutv[i])
    return best, P[i].astype(np.int32), L


def graph_from_edges(n, edge_list, vwgt=None, wts=None):
    from paper_2308_15494_amd import graphgen as gg
    e = np.asarray(edge_list, dtype=np.int64).reshape(-1, 2)
    w = None if wts is None else np.asarray(wts, dtype=np.int32)
    xadj, adjncy, adjwgt = gg.csr_from_undirected(n, e[:, 0], e[:, 1], w)
    vw = None if vwgt is None else np.asarray(vwgt, dtype=np.int32)
    return gg.Graph(n, xadj, adjncy, adjwgt, vw, name="fixture")


def load_golden(name):
    import json
    import os
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", name)
    with open(path) as f:
        return json.load(f)


def rebalance_bucket(gain, c, slots=54):
    """Monotone bucket of the rebalancing priority of Section 7.1 (lower
    first): gain*c for gain >= 0, gain/c for gain < 0, bucketed by
    ceil(log_{3/2}) of the magnitude."""
    if gain > 0:
        return slots - 1 - slot_exact(gain * c, 1, slots)
    if gain == 0:
        return slots
    return slots + 1 + slot_exact(-gain, c, slots)


def rebalance_one_iteration(g, k, part, L, plain=False):
    """One synchronous rebalancing sub-iteration, from the rules of Section 7.1
    on Python lists: nodes of overloaded blocks take their best-gain move into
    a block that stays balanced (or, unconnected to any, the lightest such
    block, smaller id on ties); each target takes the offers aimed at it in
    (priority bucket, id) order while they fit; each overloaded block keeps,
    in the same order, its accepted nodes until its excess is covered. With
    plain, the priority is the gain itself (node weights left out).
    Returns the new partition (a list)."""
    part = list(part)
    W = [block_weight(g, part, j) for j in range(k)]
    info = {}
    for v in range(g.n):
        a = part[v]
        if W[a] <= L:
            continue
        cv = node_w(g, v)
        valid = [j for j in range(k) if j != a and W[j] + cv <= L]
        if not valid:
            continue
        conn = {j: omega(g, v, j, part) for j in valid}
        connected = [j for j in valid if conn[j] > 0]
        if connected:
            tgt = max(connected, key=lambda j: (conn[j], -j))
        else:
            tgt = min(valid, key=lambda j: (W[j], j))
        gain = move_gain(g, part, v, tgt)
        info[v] = (tgt, rebalance_bucket(gain, 1 if plain else cv))
    accepted = []
    for j in range(k):
        nodes = sorted((v for v in info if info[v][0] == j), key=lambda v: (info[v][1], v))
        room = L - W[j]
        for v in nodes:
            if node_w(g, v) > room:
                break
            room -= node_w(g, v)
            accepted.append(v)
    out = list(part)
    for a in range(k):
        if W[a] <= L:
            continue
        nodes = sorted((v for v in accepted if part[v] == a), key=lambda v: (info[v][1], v))
        got = 0
        for v in nodes:
            if got >= W[a] - L:
                break
            got += node_w(g, v)
            out[v] = info[v][0]
    return out


def pessimistic_gain(g, part, v, target, earlier):
    """Worst true gain of moving v to `target` over every subset of the
    earlier candidate neighbours `earlier` (dict u -> target_u) that may have
    moved first; each subset's gain is a recomputed cut difference."""
    nbrs = [u for u in earlier]
    worst = None
    for mask in range(1 << len(nbrs)):
        cur = list(part)
        for i, u in enumerate(nbrs):
            if mask >> i & 1:
                cur[u] = earlier[u]
        gain = move_gain(g, cur, v, target)
        worst = gain if worst is None else min(worst, gain)
    return worst


def penalty_for_excess(g, k, part, t, tau, j, X, cv, mode):
    """Section 5.3 penalty (Q16) of a node of weight cv whose move leaves
    block j with excess X over L_max (over the cap in mode 3); None if
    forbidden."""
    if X <= 0 or mode == 2:
        return 0
    if mode in (1, 3):
        return None
    B = available_sets(g, k, part, t)
    acc = 0
    for l in range(54):
        acc += sum(node_w(g, u) for u in B[j][l])
        if acc >= X:
            per_unit = (Fraction(*tau) * Fraction(3, 2) ** l * 65536) // 1
            return min(int(per_unit) * cv, 1 << 62)
    return None


def optimistic_gain(g, part, v, target, earlier):
    """True gain of moving v to `target` once every earlier candidate
    neighbour (dict u -> target_u) has made its move."""
    cur = list(part)
    for u, tu in earlier.items():
        cur[u] = tu
    return move_gain(g, cur, v, target)


def filter_decisions(g, k, part, t, tau, eps, mode=0, seq=True, alpha=(1, 1), optimistic=False):
    """S3 by brute force. Candidates from best_moves, in (score desc, id asc)
    order; pessimistic gain as the worst true gain over the moves earlier
    candidate neighbours may make; with seq, each block's weight is tracked
    along the order (eligible candidates, i.e. positive pessimistic gain, add
    their weight to their target and, unless available for rebalancing,
    remove it from their block) and every move is priced against it.
    Returns {v: (accepted, pen_seq)} with pen_seq None when forbidden."""
    total = sum(node_w(g, v) for v in range(g.n))
    L = lmax_exact(total, k, eps)
    cap = move_cap(L, mode, alpha)
    moves = best_moves(g, k, part, t, tau, eps, mode, alpha)
    order = sorted(moves, key=lambda v: (-moves[v][1], v))
    W = [block_weight(g, part, j) for j in range(k)]
    B = available_sets(g, k, part, t)
    avail = {u for j in range(k) for l in range(54) for u in B[j][l]}
    net = [0] * k
    out = {}
    pos = {v: i for i, v in enumerate(order)}
    for v in order:
        b, _, pen = moves[v]
        nb = set(int(u) for u in g.adjncy[g.xadj[v]:g.xadj[v + 1]])
        earlier = {u: moves[u][0] for u in nb if u in moves and pos[u] < pos[v]}
        if optimistic:
            gp = optimistic_gain(g, list(part), v, b, earlier)
        else:
            gp = pessimistic_gain(g, list(part), v, b, earlier)
        cv = node_w(g, v)
        P = pen
        if seq:
            P = penalty_for_excess(g, k, part, t, tau, b, W[b] + net[b] + cv - cap, cv, mode)
            if gp > 0:
                net[b] += cv
                if v not in avail:
                    net[part[v]] -= cv
        acc = P is not None and gp > 0 and gp * 65536 - P > 0
        out[v] = (acc, P)
    return out


def rebalance_all(g, k, part, L, plain=False):
    """Sub-iterations with the rules of rebalance_one_iteration until no block
    is overloaded, nothing moved, or the iteration cap (k + 1 for unit node
    weights, 4k otherwise). Returns the partition and the moves in the order
    they were made: (node, from, to) per sub-iteration, each source's nodes
    in (priority bucket, id) order, grouped by source block."""
    part = list(part)
    cap = k + 1 if g.vwgt is None else 4 * k
    moves = []
    for it in range(1, cap + 1):
        W = [block_weight(g, part, j) for j in range(k)]
        if all(w <= L for w in W):
            break
        new = rebalance_one_iteration(g, k, part, L, plain)
        moved = [v for v in range(g.n) if new[v] != part[v]]
        if not moved:
            break
        # the order of the rebalancer: per source, by (bucket, id), with the
        # bucket of the move from the sub-iteration's starting partition
        def bucket(v):
            gain = move_gain(g, part, v, new[v])
            return rebalance_bucket(gain, 1 if plain else node_w(g, v))
        moved.sort(key=lambda v: (part[v], bucket(v), v))
        moves += [(v, part[v], new[v]) for v in moved]
        part = new
    return part, moves


def interleaved_best_prefix(g, k, part0, filtered, L, plain=False):
    """Section 5.4 from its rules, on lists: `filtered` are the filtered moves
    (node, target) in the filter's order, applied together to part0; the
    rebalancer then runs; a node moved by both is one move from its start to
    its end (dropped if it ends where it started); each filtered move is
    followed by the fewest unused rebalancing moves out of its target block
    (in the rebalancer's order) that leave that block at most L; exact gains
    are cut differences. Returns (final partition, best boundary or -1,
    cumulative gains per boundary, balanced flags per boundary)."""
    after = list(part0)
    for v, t in filtered:
        after[v] = t
    final, rmoves = rebalance_all(g, k, after, L, plain)
    fset = {v for v, _ in filtered}
    seq_m = [(v, part0[v], final[v]) for v, _ in filtered if final[v] != part0[v]]
    rlists = {}
    for v, a, b in rmoves:
        if v not in fset:
            rlists.setdefault(a, []).append((v, a, b))
    used = {j: 0 for j in range(k)}
    cur = list(part0)

    def balanced(p):
        return all(block_weight(g, p, j) <= L for j in range(k))

    cut0 = cut(g, part0)
    gains, bal, steps = [0], [balanced(cur)], []
    for v, a, b in seq_m:
        step = [(v, a, b)]
        cur[v] = b
        lst = rlists.get(b, [])
        while block_weight(g, cur, b) > L and used[b] < len(lst):
            r = lst[used[b]]
            used[b] += 1
            cur[r[0]] = r[2]
            step.append(r)
        steps.append(step)
        gains.append(cut0 - cut(g, cur))
        bal.append(balanced(cur))
    best = -1
    for j in range(len(gains)):
        if bal[j] and (best < 0 or gains[j] > gains[best]):
            best = j
    if best < 0:
        return final, best, gains, bal
    out = list(part0)
    for step in steps[:best]:
        for v, a, b in step:
            out[v] = b
    return out, best, gains, bal
