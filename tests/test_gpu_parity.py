"""GPU parity: the HIP path through the C ABI against the CPU oracle, element
by element on the same seeded inputs. Everything is integer arithmetic, so
the bar is bit-exact: gain table, block weights, partition, cut and
statistics after every round, and the per-node move decisions."""
import os
import sys

import numpy as np
import pytest

from oracle import oracle as O
from paper_2308_15494_amd import graphgen as gg

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def upr():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2308_15494_amd import upr as U
    U.lib()
    return U


@pytest.fixture(scope="module")
def ctx(upr):
    c = upr.Context(0)
    yield c
    c.close()


def skewed_partition(n, k, seed, heavy=0.5):
    rng = np.random.default_rng(seed)
    p = np.full(k, (1 - heavy) / (k - 1))
    p[0] = heavy
    return rng.choice(k, size=n, p=p).astype(np.int32)


def to_dev(a, torch_dtype=None):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda")


class Pair:
    """The same round state on the GPU and in the oracle."""

    def __init__(self, upr, ctx, g, k, part0):
        import torch
        self.upr, self.ctx, self.g, self.k = upr, ctx, g, k
        self.dg = upr.DeviceGraph(g)
        self.plan = upr.Plan(ctx, self.dg)
        self.part = to_dev(part0.astype(np.int32))
        self.conn = torch.zeros(max(g.n * k, 1), dtype=torch.int32, device="cuda")
        self.W = torch.zeros(k, dtype=torch.int64, device="cuda")
        self.stats = torch.zeros(12, dtype=torch.int64, device="cuda")
        self.G = O.Graph(g)
        self.opart = part0.astype(np.int32).copy()
        self.oconn = np.zeros(max(g.n * k, 1), np.int32)
        self.oW = np.zeros(k, np.int64)

    def round(self, **kw):
        p = self.upr.params(self.k, **kw)
        self.upr.refine_round(self.ctx, self.plan, p, self.part, self.conn, self.W, self.stats)
        ost, odbg = O.refine_round(self.G, O.params(self.k, **kw), self.opart, self.oconn, self.oW,
                                   debug=True)
        return ost, odbg

    def rebalance(self, **kw):
        p = self.upr.params(self.k, **kw)
        self.upr.rebalance(self.ctx, self.plan, p, self.part, self.conn, self.W, self.stats)
        return O.rebalance(self.G, O.params(self.k, **kw), self.opart, self.oconn, self.oW)

    def compare(self, ost, odbg=None, what=""):
        import torch
        torch.cuda.synchronize()
        st = self.stats.cpu().numpy()
        assert O.stats_dict(st) == O.stats_dict(ost), f"{what}: stats differ"
        assert np.array_equal(self.part.cpu().numpy(), self.opart), f"{what}: part differs"
        assert np.array_equal(self.W.cpu().numpy(), self.oW), f"{what}: block weights differ"
        if self.g.n:
            assert np.array_equal(self.conn.cpu().numpy()[: self.g.n * self.k],
                                  self.oconn[: self.g.n * self.k]), f"{what}: gain table differs"
        if odbg is not None and self.g.n:
            mv = self.upr.last_moves(self.ctx, self.g.n)
            torch.cuda.synchronize()
            assert np.array_equal(mv["target"].cpu().numpy(), odbg["target"]), f"{what}: targets"
            assert np.array_equal(mv["score"].cpu().numpy(), odbg["score"]), f"{what}: scores"
            assert np.array_equal(mv["pen"].cpu().numpy(), odbg["pen"]), f"{what}: penalties"
            assert np.array_equal(mv["accept"].cpu().numpy(), odbg["accept"]), f"{what}: accept"


# ------------------------------------------------------------ S1 / cut --

@pytest.mark.parametrize("case", [
    ("er", lambda: gg.random_small(300, 0.05, seed=1), 2),
    ("er_w", lambda: gg.random_small(400, 0.04, seed=2, wmax=9, vmax=5), 5),
    ("cl", lambda: gg.chung_lu(5000, 10.0, 2.3, seed=3), 8),
    ("cl_w", lambda: gg.chung_lu(3000, 12.0, 2.1, seed=4, wmax=16), 64),
    ("grid", lambda: gg.grid2d(61, 77), 64),
    ("rmat", lambda: gg.rmat(13, 16, seed=5), 256),
    ("bigk", lambda: gg.chung_lu(700, 6.0, 2.5, seed=6), 3000),
    ("kmax", lambda: gg.random_small(40, 0.2, seed=7), 8192),
])
def test_gain_table_and_cut(upr, ctx, case):
    import torch
    name, make, k = case
    g = make()
    say(f"gain table case={name} n={g.n} nnz={g.nnz} k={k}")
    part = gg.random_partition(g.n, k, 3)
    dg = upr.DeviceGraph(g)
    plan = upr.Plan(ctx, dg)
    dpart = to_dev(part)
    conn = upr.gain_table(ctx, plan, k, dpart)
    W = upr.block_weights(ctx, plan, k, dpart)
    cut = upr.edge_cut(ctx, plan, dpart)
    torch.cuda.synchronize()
    assert np.array_equal(conn.cpu().numpy().reshape(g.n, k), O.gain_table(g, k, part))
    assert np.array_equal(W.cpu().numpy(), O.block_weights(g, k, part))
    assert int(cut.item()) == O.cut_edges(g, part)


def star_graph(n, centers, total, seed):
    """Random light edges (weights 1..50) away from the centers plus, at each
    center, a star of 16 leaves whose edge weights add up to exactly `total`."""
    rng = np.random.default_rng(seed)
    u = rng.integers(0, n, size=4 * n)
    v = rng.integers(0, n, size=4 * n)
    w = rng.integers(1, 51, size=4 * n)
    keep = ~(np.isin(u, centers) | np.isin(v, centers))
    u, v, w = u[keep], v[keep], w[keep]
    nr = u.size
    eu, ev, ew = [u], [v], [w]
    nxt = max(centers) + 1
    for c in centers:
        leaves = 16
        wt = np.full(leaves, total // leaves, np.int64)
        wt[: total % leaves] += 1
        eu.append(np.full(leaves, c))
        ev.append(np.arange(nxt, nxt + leaves))
        ew.append(wt)
        nxt += leaves
    u, v, w = np.concatenate(eu), np.concatenate(ev), np.concatenate(ew)
    # star edges first so that duplicates keep the star weight
    order = np.r_[np.arange(nr, u.size), np.arange(nr)]
    xadj, adjncy, adjwgt = gg.csr_from_undirected(n, u[order], v[order], w[order])
    return gg._finish(gg.Graph(n, xadj, adjncy, adjwgt, None, name=f"star{total}"))


@pytest.mark.parametrize("total", [65535, 65536, 200000])
def test_gain_table_counter_width(upr, ctx, total):
    """Tiled rows count in 16-bit LDS halves while every weighted degree is
    below 2^16 and in 32-bit words otherwise. Stars whose weights add up to
    2^16 - 1 (the largest packed count, no carry into the neighbour entry),
    2^16 and more, with their leaves all in one block, then rounds."""
    import torch
    n = 3000
    centers = [0, 1001, 1502]
    g = star_graph(n, centers, total, seed=total % 97)
    for k in (2, 3, 64):
        part = gg.random_partition(g.n, k, 5)
        nxt = max(centers) + 1
        for i, c in enumerate(centers):
            part[nxt + 16 * i: nxt + 16 * (i + 1)] = (i + 1) % k
        wdeg = np.bincount(np.repeat(np.arange(g.n), g.degrees()), weights=g.adjwgt, minlength=g.n)
        say(f"counter width total={total} k={k} max_wdeg={int(wdeg.max())}")
        dg = upr.DeviceGraph(g)
        plan = upr.Plan(ctx, dg)
        conn = upr.gain_table(ctx, plan, k, to_dev(part))
        torch.cuda.synchronize()
        ref = O.gain_table(g, k, part)
        for i, c in enumerate(centers):
            assert ref[c, (i + 1) % k] == total
        assert np.array_equal(conn.cpu().numpy().reshape(g.n, k), ref)
        pr = Pair(upr, ctx, g, k, part)
        for r in range(1, 4):
            ost, odbg = pr.round(tau=gg.tau_schedule(r, 3))
            pr.compare(ost, odbg, f"total {total} k {k} round {r}")


def test_gain_table_hub_rows(upr, ctx, monkeypatch):
    """The standalone table build with hubs of several edge chunks, twice into
    the same buffer: the hub rows are cleared before the chunks add into them,
    so the second partition's table holds no counts of the first."""
    import torch
    monkeypatch.setenv("UPR_HUB_THRESHOLD", "40")
    for seed, k in ((1, 64), (2, 5)):
        g = gg.rmat(16, 16, seed=seed)  # largest degrees near 10^4: hubs of up to 3 chunks
        if seed == 2:
            g = gg.with_weights(g, seed, wmax=7)
        say(f"hub table case seed={seed} n={g.n} max_deg={g.meta['max_degree']} k={k}")
        dg = upr.DeviceGraph(g)
        plan = upr.Plan(ctx, dg)
        assert plan.info()["num_hubs"] > 0
        assert g.meta["max_degree"] > 4096  # a hub of more than one chunk
        conn = None
        for rep in range(2):
            part = gg.random_partition(g.n, k, 10 * seed + rep)
            conn = upr.gain_table(ctx, plan, k, to_dev(part), conn)
            torch.cuda.synchronize()
            assert np.array_equal(conn.cpu().numpy().reshape(g.n, k), O.gain_table(g, k, part)), rep


def test_hub_paths(upr, ctx, monkeypatch):
    """Force a low hub threshold so the hub kernels (one workgroup per edge
    chunk) carry real rows through whole rounds; these hubs fit one chunk
    each, the table test above has hubs of several."""
    import torch
    monkeypatch.setenv("UPR_HUB_THRESHOLD", "40")
    for seed in range(3):
        g = gg.with_weights(gg.chung_lu(6000, 12.0, 2.05, seed=seed, d_max=5000), seed, wmax=7,
                            vmax=3 if seed == 2 else 0)
        k = [8, 64, 5][seed]
        say(f"hub case seed={seed} n={g.n} max_deg={g.meta['max_degree']} k={k}")
        part = gg.random_partition(g.n, k, seed)
        pr = Pair(upr, ctx, g, k, part)
        assert pr.plan.info()["num_hubs"] > 0
        for r in range(1, 5):
            ost, odbg = pr.round(tau=gg.tau_schedule(r, 4))
            pr.compare(ost, odbg, f"seed {seed} round {r}")


# ------------------------------------------------------------ rounds --

SMALL = [
    ("er", lambda s: gg.random_small(60, 0.08, seed=s), 3),
    ("er_w", lambda s: gg.random_small(80, 0.07, seed=s, wmax=6, vmax=4), 4),
    ("cl", lambda s: gg.chung_lu(1500, 6.0, 2.3, seed=s), 8),
    ("cl_w", lambda s: gg.with_weights(gg.chung_lu(2500, 8.0, 2.2, seed=s), s, wmax=9, vmax=3), 16),
    ("grid", lambda s: gg.grid2d(40, 50), 64),
    ("rgg", lambda s: gg.rgg2d(3000, seed=s), 32),
    ("rmat", lambda s: gg.rmat(11, 16, seed=s), 64),
]


@pytest.mark.parametrize("case", SMALL, ids=[c[0] for c in SMALL])
@pytest.mark.parametrize("mode", [0, 1, 2])
@pytest.mark.parametrize("seq", [1, 0])
def test_round_parity_small(upr, ctx, case, mode, seq):
    name, make, k = case
    for seed in range(2):
        g = make(seed + 1)
        for pname, part0 in [("random", gg.random_partition(g.n, k, seed)),
                             ("skewed", skewed_partition(g.n, k, seed, 0.4))]:
            say(f"round parity case={name} mode={mode} seq={seq} seed={seed} start={pname} "
                f"n={g.n} k={k}")
            pr = Pair(upr, ctx, g, k, part0)
            for r in range(1, 5):
                ost, odbg = pr.round(tau=gg.tau_schedule(r, 4), mode=mode, seq_penalty=seq)
                pr.compare(ost, odbg, f"{name} mode {mode} seq {seq} seed {seed} {pname} round {r}")


@pytest.mark.parametrize("k", [100, 126, 130, 200, 300, 1100])
@pytest.mark.parametrize("seq", [1, 0])
def test_round_parity_large_k(upr, ctx, k, seq):
    """Rounds at k beyond the small cases: the candidate flag in the one-byte
    partition copy (k <= 128, with both best-move kernels: k = 100 is a
    multiple of 4, k = 126 is not), the one-byte copy without it (k = 130,
    200), the two-byte copy (k = 300) and rows longer than a wave (k = 1100)."""
    g = gg.chung_lu(6000, 10.0, 2.2, seed=k)
    for pname, part0 in [("random", gg.random_partition(g.n, k, 1)),
                         ("skewed", skewed_partition(g.n, k, 2, 0.3))]:
        say(f"large k={k} seq={seq} start={pname} n={g.n}")
        pr = Pair(upr, ctx, g, k, part0)
        for r in range(1, 4):
            ost, odbg = pr.round(tau=gg.tau_schedule(r, 3), seq_penalty=seq)
            pr.compare(ost, odbg, f"k {k} seq {seq} {pname} round {r}")


VARIANTS = [
    ("limited", dict(mode=3), True),
    ("optimistic", dict(variant=1), False),
    ("plain_priority", dict(variant=2), False),
    ("optimistic_plain_limited", dict(mode=3, variant=3), True),
]


@pytest.mark.parametrize("case", SMALL[:5] + SMALL[6:], ids=[c[0] for c in SMALL[:5] + SMALL[6:]])
@pytest.mark.parametrize("var", VARIANTS, ids=[v[0] for v in VARIANTS])
@pytest.mark.parametrize("seq", [1, 0])
def test_round_parity_variants(upr, ctx, case, var, seq):
    """The Section 8.2 variants: limited imbalance (alpha from 2 down to 1.1),
    optimistic filter, plain-gain rebalancing priority."""
    name, make, k = case
    vname, kw, uses_alpha = var
    for seed in range(2):
        g = make(seed + 11)
        part0 = skewed_partition(g.n, k, seed, 0.4)
        say(f"variant {vname} case={name} seq={seq} seed={seed} n={g.n} k={k}")
        pr = Pair(upr, ctx, g, k, part0)
        for r in range(1, 5):
            extra = dict(kw)
            if uses_alpha:
                extra["alpha"] = gg.alpha_schedule(r, 4)
            ost, odbg = pr.round(tau=gg.tau_schedule(r, 4), seq_penalty=seq, **extra)
            pr.compare(ost, odbg, f"{vname} {name} seq {seq} seed {seed} round {r}")


@pytest.mark.parametrize("t", [(7, 10), (2, 5), (0, 1), (1, 1)])
def test_round_parity_threshold(upr, ctx, t):
    g = gg.chung_lu(4000, 8.0, 2.2, seed=9)
    k = 16
    pr = Pair(upr, ctx, g, k, skewed_partition(g.n, k, 1, 0.3))
    say(f"threshold t={t}")
    for r in range(1, 4):
        ost, odbg = pr.round(t=t, tau=(1, 1))
        pr.compare(ost, odbg, f"t {t} round {r}")


def test_round_parity_chunglu10k(upr, ctx):
    """The 10k-node Chung-Lu workload: 10 rounds with tau (8+r)/18 and a
    final rebalance, bit-exact after every round."""
    g, k, eps, rounds, seed = gg.workload("chunglu10k")
    pr = Pair(upr, ctx, g, k, gg.random_partition(g.n, k, seed))
    for r in range(1, rounds + 1):
        say(f"chunglu10k round {r}")
        ost, odbg = pr.round(eps=eps, tau=gg.tau_schedule(r, rounds))
        pr.compare(ost, odbg, f"round {r}")
    ost = pr.rebalance(eps=eps)
    pr.compare(ost, None, "final rebalance")


def test_resident_equals_rebuild(upr, ctx):
    g = gg.with_weights(gg.chung_lu(5000, 8.0, 2.3, seed=12), 3, wmax=5, vmax=2)
    k = 12
    part0 = gg.random_partition(g.n, k, 4)
    a = Pair(upr, ctx, g, k, part0)
    b = Pair(upr, ctx, g, k, part0)
    for r in range(1, 6):
        say(f"resident round {r}")
        tau = gg.tau_schedule(r, 5)
        ost, odbg = a.round(tau=tau, rebuild_table=1)
        a.compare(ost, odbg, f"rebuild round {r}")
        ost, odbg = b.round(tau=tau, rebuild_table=0 if r > 1 else 1)
        b.compare(ost, odbg, f"resident round {r}")


def test_rebalance_parity(upr, ctx):
    for seed in range(4):
        g = gg.with_weights(gg.chung_lu(3000, 6.0, 2.4, seed=seed), seed,
                            wmax=4 if seed % 2 else 0, vmax=5 if seed >= 2 else 0)
        k = [2, 7, 16, 64][seed]
        say(f"rebalance seed={seed} k={k}")
        pr = Pair(upr, ctx, g, k, skewed_partition(g.n, k, seed, 0.6))
        ost = pr.rebalance()
        pr.compare(ost, None, f"rebalance seed {seed}")
        ost = pr.rebalance(max_rebalance_iters=1)
        pr.compare(ost, None, f"rebalance again seed {seed}")


def test_rebalance_iteration_cap_and_stuck(upr, ctx):
    g = gg.chung_lu(2000, 5.0, 2.3, seed=4)
    k = 6
    part0 = skewed_partition(g.n, k, 4, heavy=0.7)
    pr = Pair(upr, ctx, g, k, part0)
    ost = pr.rebalance(max_rebalance_iters=1)
    pr.compare(ost, None, "cap 1")
    # stuck: two heavy nodes that fit nowhere
    from tests import bruteforce as bf
    g2 = bf.graph_from_edges(5, [[0, 1], [1, 2], [2, 3], [3, 4]], vwgt=[4, 4, 1, 1, 1])
    pr2 = Pair(upr, ctx, g2, 2, np.array([0, 0, 1, 1, 1], np.int32))
    ost = pr2.rebalance(eps=(1, 10))
    pr2.compare(ost, None, "stuck")
    assert ost[8] == 1


def test_determinism_across_streams(upr, ctx):
    import torch
    g = gg.rmat(12, 16, seed=21)
    k = 32
    outs = []
    for i in range(3):
        s = torch.cuda.Stream() if i else torch.cuda.current_stream()
        with torch.cuda.stream(s):
            r = upr.Refiner(g, k, ctx=ctx)
            r.set_partition(gg.random_partition(g.n, k, 1))
            for rr in range(1, 4):
                r.round(upr.params(k, tau=gg.tau_schedule(rr, 3)))
            s.synchronize()
            outs.append((r.part.cpu().numpy(), r.stats.cpu().numpy(), r.conn.cpu().numpy()))
    for o in outs[1:]:
        for x, y in zip(outs[0], o):
            assert np.array_equal(x, y)


# ------------------------------------------------------------ edge cases --

def test_edge_cases(upr, ctx):
    from tests import bruteforce as bf
    cases = [
        ("no edges", gg.Graph(50, np.zeros(51, np.int64), np.zeros(0, np.int32)), 4),
        ("single node", gg.Graph(1, np.zeros(2, np.int64), np.zeros(0, np.int32)), 2),
        ("one edge", bf.graph_from_edges(2, [[0, 1]]), 2),
        ("k>n", gg.random_small(10, 0.4, seed=3), 17),
        ("golden escape", bf.graph_from_edges(10, bf.load_golden("full_block_escape.json")["edges"]), 2),
    ]
    for name, g, k in cases:
        say(f"edge case {name}")
        for part0 in [gg.random_partition(g.n, k, 1), np.zeros(g.n, np.int32)]:
            pr = Pair(upr, ctx, g, k, part0)
            for r in range(1, 3):
                ost, odbg = pr.round(tau=(1, r))
                pr.compare(ost, odbg, f"{name} round {r}")


def test_golden_fixtures_on_gpu(upr, ctx):
    from tests import bruteforce as bf
    for fname in ["full_block_escape.json", "filter_conflict.json"]:
        fx = bf.load_golden(fname)
        g = bf.graph_from_edges(fx["n"], fx["edges"])
        for case in fx["cases"]:
            say(f"golden {fname} mode={case['mode']} tau={case['tau']}")
            pr = Pair(upr, ctx, g, fx["k"], np.array(fx["part_in"], np.int32))
            ost, odbg = pr.round(eps=tuple(fx["eps"]), t=tuple(fx["t"]), tau=tuple(case["tau"]),
                                 mode=case["mode"])
            pr.compare(ost, odbg, fname)
            got = upr.stats_dict(pr.stats)
            assert {key: got[key] for key in case["stats"]} == case["stats"]
            assert pr.part.cpu().numpy().tolist() == case["part_out"]


def test_empty_graph(upr, ctx):
    import torch
    g = gg.Graph(0, np.zeros(1, np.int64), np.zeros(0, np.int32))
    dg = upr.DeviceGraph(g)
    plan = upr.Plan(ctx, dg)
    part = torch.zeros(0, dtype=torch.int32, device="cuda")
    conn = torch.zeros(0, dtype=torch.int32, device="cuda")
    W = torch.zeros(4, dtype=torch.int64, device="cuda")
    st = upr.refine_round(ctx, plan, upr.params(4), part, conn, W)
    torch.cuda.synchronize()
    assert upr.stats_dict(st) == {"l_max": 0, "cut_before": 0, "cut_after_moves": 0,
                                  "cut_after": 0, "candidates": 0, "accepted": 0,
                                  "rebalance_moves": 0, "rebalance_iters": 0, "status": 0,
                                  "prefix_steps": 0, "reverted": 0}


def test_errors(upr, ctx):
    import torch
    g = gg.random_small(30, 0.2, seed=1)
    dg = upr.DeviceGraph(g)
    plan = upr.Plan(ctx, dg)
    k = 4
    conn = torch.zeros(g.n * k, dtype=torch.int32, device="cuda")
    W = torch.zeros(k, dtype=torch.int64, device="cuda")
    good = to_dev(gg.random_partition(g.n, k, 1))
    for bad in [dict(k=1), dict(k=8193), dict(k=4, eps=(0, 1)), dict(k=4, tau=(3, 2)), dict(k=4, t=(2, 1)),
                dict(k=4, mode=7), dict(k=4, mode=3, alpha=(9, 10)), dict(k=4, mode=3, alpha=(1, 0)),
                dict(k=4, variant=8)]:
        kk = bad.pop("k")
        with pytest.raises(upr.UprError) as ei:
            upr.refine_round(ctx, plan, upr.params(kk, **bad), good, conn, W)
        assert ei.value.code == -1
    badpart = good.clone()
    badpart[3] = 9
    with pytest.raises(upr.UprError) as ei:
        upr.refine_round(ctx, plan, upr.params(k), badpart, conn, W)
    assert ei.value.code == -1
    with pytest.raises(upr.UprError) as ei:
        upr.gain_table(ctx, plan, k, badpart, conn)
    assert ei.value.code == -1
    # infeasible: a node heavier than L_max
    gw = gg.Graph(g.n, g.xadj, g.adjncy, None, np.full(g.n, 1, np.int32))
    gw.vwgt[0] = 1000
    planw = upr.Plan(ctx, upr.DeviceGraph(gw))
    with pytest.raises(upr.UprError) as ei:
        upr.refine_round(ctx, planw, upr.params(k), good, conn, W)
    assert ei.value.code == -3
    # malformed graph: neighbour id out of range is caught at plan creation
    adj = g.adjncy.copy()
    adj[5] = g.n + 3
    with pytest.raises(upr.UprError) as ei:
        upr.Plan(ctx, upr.DeviceGraph(gg.Graph(g.n, g.xadj, adj)))
    assert ei.value.code == -2
    # asymmetric structure is caught by validation
    adj = g.adjncy.copy()
    row = int(np.argmax(np.diff(g.xadj) >= 2))
    e = int(g.xadj[row])
    cand = [u for u in range(g.n) if u != row and u not in set(adj[g.xadj[row]:g.xadj[row + 1]].tolist())]
    adj[e] = min(cand)
    adj[g.xadj[row]:g.xadj[row + 1]].sort()
    with pytest.raises(upr.UprError) as ei:
        upr.validate_graph(ctx, upr.DeviceGraph(gg.Graph(g.n, g.xadj, adj)))
    assert ei.value.code == -2
    upr.validate_graph(ctx, dg)  # the generator's graph is valid
    # the context still works after errors
    pr = Pair(upr, ctx, g, k, gg.random_partition(g.n, k, 1))
    ost, odbg = pr.round()
    pr.compare(ost, odbg, "after errors")


# ------------------------------------------------------------ apply modes --
# (the full-size workloads are compared in test_gpu_fullsize.py)

@pytest.mark.parametrize("div,all_div", [("1", "0"), ("100000000", "1"), ("100000000", "0"),
                                         ("1", "100000000"), ("16", "32")],
                         ids=["delta", "rebuild_marked", "rebuild_all", "all_below_marking",
                              "all_div_above_dirty_div"])
def test_apply_modes(upr, ctx, monkeypatch, div, all_div):
    """The ways of updating the table after moves (integer-atomic deltas,
    marking and rebuilding the tiles of the movers' neighbours, or rebuilding
    every tile) give the oracle's table. The last two cases ask for a
    whole-table threshold below the marking one (it is raised to the marking
    threshold, so hub rows get their deltas whenever tiles are not marked)."""
    monkeypatch.setenv("UPR_DIRTY_DIV", div)
    monkeypatch.setenv("UPR_REBUILD_ALL_DIV", all_div)
    monkeypatch.setenv("UPR_HUB_THRESHOLD", "64")
    for name, g, k in [("rmat", gg.rmat(12, 16, seed=31), 32),
                       ("cl_w", gg.with_weights(gg.chung_lu(4000, 8.0, 2.1, seed=5), 5, 6, 3), 8),
                       ("grid", gg.grid2d(50, 60), 16)]:
        say(f"apply mode div={div} case={name}")
        pr = Pair(upr, ctx, g, k, skewed_partition(g.n, k, 3, 0.35))
        for r in range(1, 5):
            ost, odbg = pr.round(tau=gg.tau_schedule(r, 4))
            pr.compare(ost, odbg, f"{name} round {r}")


@pytest.mark.parametrize("div", ["1", "100000000"], ids=["delta", "rebuild"])
@pytest.mark.parametrize("relabel", ["2", "0"], ids=["relabelled", "as_given"])
def test_table_relabelling(upr, ctx, monkeypatch, relabel, div):
    """The table build reads a copy of the adjacency whose neighbour ids are
    renumbered by descending degree, with the partition copy in that order
    (forced here below the default size limit, and switched off): tables,
    partitions and statistics equal the oracle's in both apply modes, with
    hubs, and with the one- and two-byte partition copies (k = 300)."""
    monkeypatch.setenv("UPR_RELABEL", relabel)
    monkeypatch.setenv("UPR_DIRTY_DIV", div)
    monkeypatch.setenv("UPR_HUB_THRESHOLD", "64")
    for name, g, k in [("rmat", gg.rmat(12, 16, seed=41), 32),
                       ("cl_w", gg.with_weights(gg.chung_lu(4000, 8.0, 2.1, seed=6), 6, 6, 3), 8),
                       ("cl_k300", gg.chung_lu(3000, 12.0, 2.2, seed=7), 300),
                       ("grid", gg.grid2d(40, 50), 16)]:
        say(f"relabel={relabel} div={div} case={name}")
        pr = Pair(upr, ctx, g, k, skewed_partition(g.n, k, 4, 0.35))
        for r in range(1, 5):
            ost, odbg = pr.round(tau=gg.tau_schedule(r, 4))
            pr.compare(ost, odbg, f"{name} round {r}")


def hub_star_on_grid(rows, cols, leaves):
    """A rows x cols grid plus one hub joined to `leaves` leaves (ids after
    the grid: the hub, then its leaves)."""
    n0 = rows * cols
    ids = np.arange(n0, dtype=np.int64).reshape(rows, cols)
    u = np.r_[ids[:, :-1].ravel(), ids[:-1, :].ravel(), np.full(leaves, n0)]
    v = np.r_[ids[:, 1:].ravel(), ids[1:, :].ravel(), n0 + 1 + np.arange(leaves)]
    n = n0 + 1 + leaves
    xadj, adjncy, _ = gg.csr_from_undirected(n, u, v)
    return gg._finish(gg.Graph(n, xadj, adjncy, None, None, name="hub_star_grid"))


def test_cut_from_apply_deltas(upr, ctx, monkeypatch):
    """The cut after the moves and after rebalancing is summed from the
    movers' edges while the moving degrees stay small, else recounted. A hub
    (above a forced threshold of 64) whose 300 leaves sit in the other block
    is the only node with a positive pessimistic gain: its move is summed by
    the hub-chunk walk; later rounds and a skewed start move ordinary nodes
    (the tile walk) and, in the first rounds, enough to be recounted. Their
    rebalancing ends after its first sub-iteration in some rounds (the closing
    statistics enqueued before the host's wait stand) and needs more in
    others (they are taken again), with and without a recount. Every
    statistic equals the oracle's."""
    monkeypatch.setenv("UPR_HUB_THRESHOLD", "64")
    monkeypatch.setenv("UPR_DIRTY_DIV", "1")
    g = hub_star_on_grid(60, 70, 300)
    n0 = 60 * 70
    part = np.zeros(g.n, np.int32)
    part[2300:n0] = 1
    part[n0 + 1:] = 1  # the leaves; the hub stays in block 0
    pr = Pair(upr, ctx, g, 2, part)
    assert pr.plan.info()["num_hubs"] == 1
    ost, odbg = pr.round(tau=(1, 2))
    pr.compare(ost, odbg, "hub round")
    assert int(ost[5]) == 1 and odbg["accept"][n0] == 1  # the hub alone moved
    for r in range(2, 4):
        ost, odbg = pr.round(tau=(1, 1))
        pr.compare(ost, odbg, f"round {r}")
    # ordinary movers, many at first
    for name, g2, k in [("cl", gg.chung_lu(6000, 8.0, 2.3, seed=3), 8),
                        ("rmat_w", gg.with_weights(gg.rmat(12, 16, seed=4), 4, wmax=5), 16)]:
        pr = Pair(upr, ctx, g2, k, skewed_partition(g2.n, k, 5, 0.4))
        iters = set()
        for r in range(1, 7):
            ost, odbg = pr.round(tau=gg.tau_schedule(r, 6))
            pr.compare(ost, odbg, f"{name} round {r}")
            iters.add(int(O.stats_dict(ost)["rebalance_iters"]))
        assert 1 in iters and max(iters) >= 2, iters
        ost = pr.rebalance()
        pr.compare(ost, None, f"{name} standalone rebalance")


def test_rounds_with_one_rebalancing_iteration(upr, ctx):
    """Rounds with moves whose rebalancing may run one sub-iteration: it is
    the speculative one, so the round's closing statistics enqueued before
    the host's wait stand, with the status derived on the device (1 while
    blocks stay overloaded, 0 once balanced). Every statistic, the
    partition, W and the table equal the oracle's."""
    for name, g2, k in [("cl", gg.chung_lu(6000, 8.0, 2.3, seed=3), 8),
                        ("rmat_w", gg.with_weights(gg.rmat(12, 16, seed=4), 4, wmax=5), 16)]:
        say(f"one rebalancing iteration case={name} n={g2.n} k={k}")
        pr = Pair(upr, ctx, g2, k, skewed_partition(g2.n, k, 5, 0.4))
        seen = set()
        for r in range(1, 5):
            ost, odbg = pr.round(tau=gg.tau_schedule(r, 4), max_rebalance_iters=1)
            pr.compare(ost, odbg, f"{name} round {r}")
            st = O.stats_dict(ost)
            seen.add((int(st["rebalance_iters"]), int(st["status"])))
        if name == "cl":
            assert {(1, 0), (1, 1)} <= seen, seen


# ------------------------------------------------------------ driver --

@pytest.mark.parametrize("case", [("cl", 8), ("rgg", 16), ("rmat", 8), ("cl_w", 4)])
def test_driver_parity(upr, ctx, case):
    """The refinement driver (label propagation with rollback and active
    sets, then FM rounds with the tau schedule and the switch to constrained
    rounds): every round's statistics, its kind and the final partition,
    table and block weights equal the oracle driver's."""
    import torch
    from oracle import driver as D
    name, k = case
    g = {"cl": lambda: gg.chung_lu(3000, 8.0, 2.3, seed=5),
         "rgg": lambda: gg.rgg2d(3000, seed=6),
         "rmat": lambda: gg.rmat(11, 16, seed=7),
         "cl_w": lambda: gg.with_weights(gg.chung_lu(2000, 8.0, 2.2, seed=8), 8, wmax=9, vmax=3)}[name]()
    for start in (gg.random_partition(g.n, k, 1), skewed_partition(g.n, k, 2, 0.3)):
        say(f"driver case={name} n={g.n} k={k}")
        opart = start.copy()
        olog = D.refine(g, k, opart)
        dg = upr.DeviceGraph(g)
        plan = upr.Plan(ctx, dg)
        part = to_dev(start)
        conn = torch.zeros(g.n * k, dtype=torch.int32, device="cuda")
        W = torch.zeros(k, dtype=torch.int64, device="cuda")
        glog = upr.refine(ctx, plan, upr.driver(k), part, conn, W)
        assert [x[0] for x in glog] == [x[1] for x in olog], "round kinds"
        for i, ((gk, gst), (_, ok, ost)) in enumerate(zip(glog, olog)):
            assert O.stats_dict(gst) == O.stats_dict(ost), f"round {i} ({gk}) stats"
        torch.cuda.synchronize()
        assert np.array_equal(part.cpu().numpy(), opart)
        assert np.array_equal(conn.cpu().numpy().reshape(g.n, k), O.gain_table(g, k, opart))
        assert np.array_equal(W.cpu().numpy(), O.block_weights(g, k, opart))


def test_plan_and_batch_outlive_context(upr, ctx):
    """A plan and a batch destroyed after their context leave no error
    behind: the next call on another context succeeds."""
    g = gg.chung_lu(2000, 8.0, 2.3, seed=31)
    c2 = upr.Context(0)
    dg = upr.DeviceGraph(g)
    plan = upr.Plan(c2, dg)
    b = upr.Batch(c2, [g, gg.rgg2d(800, seed=32)], 4)
    c2.close()
    plan.close()
    b.close()
    pr = Pair(upr, ctx, g, 4, gg.random_partition(g.n, 4, 1))
    ost, odbg = pr.round(tau=(1, 2))
    pr.compare(ost, odbg, "after a closed context")


# ------------------------------------------------------ best-move forms --

@pytest.mark.parametrize("adj", ["0", "4", "16"], ids=["row", "adj4", "adj16"])
def test_best_move_forms(upr, ctx, monkeypatch, adj):
    """Best move from the table row (UPR_ADJ_DEG=0) or, for nodes of degree
    up to the bound, from the adjacency with the compact partition copy (one
    and two bytes, flagged and not): the same targets, scores, penalties and
    rounds as the oracle, in every mode, weighted, resident, and in a batch."""
    monkeypatch.setenv("UPR_ADJ_DEG", adj)
    for name, g, k in [("grid", gg.grid2d(70, 90), 64),
                       ("cl_w", gg.with_weights(gg.chung_lu(4000, 6.0, 2.3, seed=61), 62, 7, 4), 8),
                       ("er", gg.random_small(600, 0.01, seed=63), 3),
                       ("cl_k300", gg.chung_lu(3000, 8.0, 2.4, seed=64), 300),
                       ("rgg", gg.rgg2d(5000, seed=65), 130)]:
        for mode in (0, 1, 2):
            say(f"best move adj={adj} case={name} mode={mode}")
            pr = Pair(upr, ctx, g, k, skewed_partition(g.n, k, 5, 0.3))
            for r in range(1, 4):
                ost, odbg = pr.round(tau=gg.tau_schedule(r, 3), mode=mode,
                                     rebuild_table=1 if r == 1 else 0)
                pr.compare(ost, odbg, f"{name} mode {mode} round {r}")
    # a batch (global block ids, local rows)
    import torch
    from oracle import oracle as O
    graphs = [gg.grid2d(30, 40), gg.chung_lu(2000, 5.0, 2.4, seed=66)]
    k = 16
    parts = [gg.random_partition(g.n, k, 70 + i) for i, g in enumerate(graphs)]
    b = upr.Batch(ctx, graphs, k)
    b.set_partitions(parts)
    b.round(upr.params(k, tau=(1, 2)))
    torch.cuda.synchronize()
    got, loc = b.graph_stats(), b.local_partitions()
    for i, g in enumerate(graphs):
        ref = parts[i].copy()
        st, _ = O.refine_round(g, O.params(k, tau=(1, 2)), ref)
        assert got[i] == O.stats_dict(st) and np.array_equal(loc[i], ref), i
    b.close()
