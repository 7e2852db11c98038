"""GPU parity of batches: many graphs refined by the same launches must give,
graph by graph, exactly what the oracle gives for that graph alone (part,
gain table, block weights and statistics after every round)."""
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


def mixed_graphs(seed):
    """Uneven graphs of every family, some weighted, one empty, one edgeless."""
    return [
        gg.chung_lu(3000, 8.0, 2.2, seed=seed),
        gg.random_small(400, 0.02, seed=seed + 1, wmax=7, vmax=3),
        gg.grid2d(31, 29),
        gg.with_weights(gg.chung_lu(2000, 10.0, 2.1, seed=seed + 2), seed, wmax=9),
        gg.rmat(10, 12, seed=seed + 3),
        gg.Graph(0, np.zeros(1, np.int64), np.zeros(0, np.int32), None, None, name="empty"),
        gg.random_small(40, 0.0, seed=seed + 4),  # no edges
        gg.rgg2d(1500, seed=seed + 5),
    ]


class Oracles:
    def __init__(self, graphs, k, parts):
        self.G = [O.Graph(g) for g in graphs]
        self.part = [p.astype(np.int32).copy() for p in parts]
        self.conn = [np.zeros(max(g.n * k, 1), np.int32) for g in graphs]
        self.W = [np.zeros(k, np.int64) for _ in graphs]
        self.k = k

    def round(self, i, **kw):
        return O.refine_round(self.G[i], O.params(self.k, **kw), self.part[i], self.conn[i],
                              self.W[i])[0]

    def rebalance(self, i, **kw):
        return O.rebalance(self.G[i], O.params(self.k, **kw), self.part[i], self.conn[i], self.W[i])


def compare(b, orc, graphs, ost, what):
    import torch
    torch.cuda.synchronize()
    k = b.k
    part = b.part.cpu().numpy()
    conn = b.conn.cpu().numpy()
    W = b.W.cpu().numpy()
    st = b.stats.cpu().numpy().reshape(b.ng, -1)
    for g, gr in enumerate(graphs):
        o0, o1 = b.off[g], b.off[g + 1]
        assert O.stats_dict(st[g]) == O.stats_dict(ost[g]), f"{what}: graph {g} stats"
        assert np.array_equal(part[o0:o1] - g * k, orc.part[g]), f"{what}: graph {g} part"
        assert np.array_equal(W[g * k:(g + 1) * k], orc.W[g]), f"{what}: graph {g} W"
        assert np.array_equal(conn[o0 * k:o1 * k], orc.conn[g][: gr.n * k]), f"{what}: graph {g} conn"


@pytest.mark.parametrize("k", [2, 8, 64])
@pytest.mark.parametrize("seq", [1, 0])
def test_batch_equals_each_graph_alone(upr, ctx, k, seq):
    graphs = mixed_graphs(7 + k)
    parts = [skewed_partition(g.n, k, i, 0.35) if i % 2 else gg.random_partition(g.n, k, i)
             for i, g in enumerate(graphs)]
    say(f"batch k={k} seq={seq} graphs={[g.n for g in graphs]}")
    b = upr.Batch(ctx, graphs, k)
    b.set_partitions(parts)
    orc = Oracles(graphs, k, parts)
    rounds = 4
    for r in range(1, rounds + 1):
        # graphs at different rounds of their schedules: tau differs per graph
        taus = [gg.tau_schedule(min(r + g % 3, rounds), rounds) for g in range(b.ng)]
        b.round(upr.params(k, tau=(1, 1), seq_penalty=seq), taus=taus)
        ost = [orc.round(g, tau=taus[g], seq_penalty=seq) for g in range(b.ng)]
        compare(b, orc, graphs, ost, f"k {k} seq {seq} round {r}")
    b.rebalance(upr.params(k))
    ost = [orc.rebalance(g) for g in range(b.ng)]
    compare(b, orc, graphs, ost, f"k {k} final rebalance")
    b.close()


def test_batch_modes_and_resident_table(upr, ctx):
    k = 16
    graphs = mixed_graphs(3)[:5]
    parts = [skewed_partition(g.n, k, i, 0.5) for i, g in enumerate(graphs)]
    for mode in (0, 1, 2):
        say(f"batch mode={mode}")
        b = upr.Batch(ctx, graphs, k)
        b.set_partitions(parts)
        orc = Oracles(graphs, k, parts)
        for r in range(1, 4):
            p = upr.params(k, tau=gg.tau_schedule(r, 3), mode=mode, rebuild_table=1 if r == 1 else 0)
            b.round(p)
            ost = [orc.round(g, tau=gg.tau_schedule(r, 3), mode=mode) for g in range(b.ng)]
            compare(b, orc, graphs, ost, f"mode {mode} round {r}")
        b.close()


def test_batch_of_one_equals_plain_call(upr, ctx):
    import torch
    g, k, eps, rounds, seed = gg.workload("chunglu10k")
    part0 = gg.random_partition(g.n, k, seed)
    b = upr.Batch(ctx, [g], k, eps)
    b.set_partitions([part0])
    r = upr.Refiner(g, k, ctx=ctx)
    r.set_partition(part0)
    for i in range(1, rounds + 1):
        p = upr.params(k, eps, tau=gg.tau_schedule(i, rounds))
        b.round(p)
        r.round(p)
        torch.cuda.synchronize()
        assert np.array_equal(b.part.cpu().numpy(), r.part.cpu().numpy()), f"round {i}"
        assert np.array_equal(b.stats.cpu().numpy(), r.stats.cpu().numpy()), f"round {i}"
        assert np.array_equal(b.conn.cpu().numpy(), r.conn.cpu().numpy()), f"round {i}"
    b.close()


def test_batch_rebalance_caps_per_graph(upr, ctx):
    """Unit-weight and node-weighted graphs in one batch keep their own
    iteration caps (k+1 and 4k) and their own stuck status."""
    k = 4
    graphs = [gg.chung_lu(800, 6.0, 2.3, seed=1),
              gg.with_weights(gg.chung_lu(900, 6.0, 2.3, seed=2), 2, vmax=9),
              gg.grid2d(20, 20)]
    parts = [np.zeros(g.n, np.int32) for g in graphs]  # everything in block 0
    for cap in (0, 1, 2):
        say(f"batch rebalance cap={cap}")
        b = upr.Batch(ctx, graphs, k)
        b.set_partitions(parts)
        orc = Oracles(graphs, k, parts)
        b.rebalance(upr.params(k, max_rebalance_iters=cap))
        ost = [orc.rebalance(g, max_rebalance_iters=cap) for g in range(b.ng)]
        compare(b, orc, graphs, ost, f"cap {cap}")
        b.close()


def test_batch_errors(upr, ctx):
    import torch
    k = 4
    graphs = [gg.random_small(30, 0.2, seed=1), gg.random_small(20, 0.2, seed=2)]
    b = upr.Batch(ctx, graphs, k)
    # a node holding a block of the other graph
    parts = [np.zeros(30, np.int32), np.zeros(20, np.int32)]
    b.set_partitions(parts)
    p = b.part.cpu().numpy()
    p[3] = k + 1  # graph 0 node in graph 1's block range
    b.part = torch.from_numpy(p).cuda()
    with pytest.raises(upr.UprError) as e:
        b.round(upr.params(k))
    assert "UPR_E_ARG" in str(e.value)
    # k and eps must match the batch
    b.set_partitions(parts)
    with pytest.raises(upr.UprError):
        b.round(upr.params(k + 1))
    with pytest.raises(upr.UprError):
        b.round(upr.params(k, eps=(5, 100)))
    b.close()
    # a graph naming a node outside itself
    bad = gg.random_small(10, 0.3, seed=3)
    adj = bad.adjncy.copy()
    adj[0] = 15
    badg = gg.Graph(bad.n, bad.xadj, adj, None, None, name="bad")
    with pytest.raises(upr.UprError) as e:
        upr.Batch(ctx, [graphs[0], badg], k)
    assert "UPR_E_GRAPH" in str(e.value)
    # too many blocks
    with pytest.raises(upr.UprError):
        upr.Batch(ctx, [graphs[0]] * 9, 8192)


def test_batch_carry_state(upr, ctx):
    """upr_batch_carry: graphs carried from one batch into a rebuilt one keep
    their partition (block ids renumbered to the new range), table rows and
    block weights, device to device; a resident round of the new batch then
    equals each graph's oracle round from the same state."""
    import torch
    k = 8
    graphs = [gg.chung_lu(3000, 8.0, 2.2, seed=81), gg.grid2d(31, 29),
              gg.with_weights(gg.chung_lu(2000, 10.0, 2.1, seed=82), 83, wmax=9),
              gg.rmat(10, 12, seed=84)]
    parts = [gg.random_partition(g.n, k, 90 + i) for i, g in enumerate(graphs)]
    a = upr.Batch(ctx, graphs, k)
    a.set_partitions(parts)
    for r in range(1, 3):
        a.round(upr.params(k, tau=gg.tau_schedule(r, 4)))
    torch.cuda.synchronize()
    a_parts = a.local_partitions()
    a_conn = a.conn.cpu().numpy()
    a_W = a.W.cpu().numpy().reshape(len(graphs), k)
    # the new union: graph 3, a newcomer, graph 0, graph 2 (graph 1 left)
    newcomer = gg.rgg2d(1200, seed=85)
    order = [3, None, 0, 2]
    b = upr.Batch(ctx, [graphs[i] if i is not None else newcomer for i in order], k)
    start = gg.random_partition(newcomer.n, k, 99)
    # carried slices: None (filled on the device by the carry, only the
    # newcomer's slice is uploaded)
    b.set_partitions([start if i is None else None for i in order])
    b.carry_from(a, [i if i is not None else -1 for i in order])
    torch.cuda.synchronize()
    got = b.local_partitions()
    # single slices, in the order asked
    assert all(np.array_equal(x, got[g]) for x, g in zip(b.local_partitions([2, 0, 3]), [2, 0, 3]))
    b_conn = b.conn.cpu().numpy()
    b_W = b.W.cpu().numpy().reshape(len(order), k)
    for g, i in enumerate(order):
        n = graphs[i].n if i is not None else newcomer.n
        rows = b_conn[b.off[g] * k:(b.off[g] + n) * k]
        if i is None:
            assert np.array_equal(got[g], start)
            assert not rows.any() and not b_W[g].any()  # untouched
            continue
        assert np.array_equal(got[g], a_parts[i]), g
        assert np.array_equal(rows, a_conn[a.off[i] * k:(a.off[i] + n) * k]), g
        assert np.array_equal(b_W[g], a_W[i]), g
        assert np.array_equal(b.part.cpu().numpy()[b.off[g]:b.off[g + 1]] // k, np.full(n, g))
    a.close()
    b.close()
    # resident round after a carry without newcomers
    c = upr.Batch(ctx, [graphs[2], graphs[0]], k)
    c.set_partitions([np.zeros(graphs[2].n, np.int32), np.zeros(graphs[0].n, np.int32)])
    a = upr.Batch(ctx, graphs, k)
    a.set_partitions(parts)
    a.round(upr.params(k, tau=gg.tau_schedule(1, 4)))
    c.carry_from(a, [2, 0])
    c.round(upr.params(k, tau=gg.tau_schedule(2, 4), rebuild_table=0))
    torch.cuda.synchronize()
    st = c.graph_stats()
    loc = c.local_partitions()
    for g, i in enumerate([2, 0]):
        ref = parts[i].copy()
        conn = np.zeros(graphs[i].n * k, np.int32)
        W = np.zeros(k, np.int64)
        O.refine_round(graphs[i], O.params(k, tau=gg.tau_schedule(1, 4)), ref, conn, W)
        ost, _ = O.refine_round(graphs[i], O.params(k, tau=gg.tau_schedule(2, 4), rebuild_table=0),
                                ref, conn, W)
        assert st[g] == O.stats_dict(ost), g
        assert np.array_equal(loc[g], ref), g
        n = graphs[i].n
        assert np.array_equal(c.conn.cpu().numpy()[c.off[g] * k:(c.off[g] + n) * k], conn), g
    a.close()
    c.close()


def test_concurrent_batches_in_threads(upr, ctx):
    """Batches with different k, each on a context and stream of its own and
    refined from host threads of their own at the same time, give what the
    same batches give one after the other on one context."""
    import threading
    import torch
    groups = {k: [gg.chung_lu(2500 + 300 * i, 8.0, 2.3, seed=40 + k + i) if i % 2 == 0 else
                  gg.rmat(10, 12, seed=50 + k + i) for i in range(4)] for k in (4, 8, 16)}
    parts = {k: [skewed_partition(g.n, k, i, 0.3) for i, g in enumerate(gs)] for k, gs in groups.items()}
    R = 5

    def run(b, k, stream=None):
        for r in range(1, R + 1):
            b.round(upr.params(k, tau=gg.tau_schedule(r, R)), stream=stream)

    # one after the other, one context
    seq = {}
    for k, gs in groups.items():
        b = upr.Batch(ctx, gs, k)
        b.set_partitions(parts[k])
        run(b, k)
        seq[k] = (b.local_partitions(), b.stats.cpu().numpy().copy(), b.W.cpu().numpy().copy())
        b.close()
    # concurrently: a context, stream and thread per batch
    conc = {k: upr.Batch(upr.Context(0), gs, k) for k, gs in groups.items()}
    streams = {k: torch.cuda.Stream() for k in conc}
    for k, b in conc.items():
        b.set_partitions(parts[k])
    torch.cuda.synchronize()
    errors = []

    def work(k, b):
        try:
            run(b, k, streams[k])
        except Exception as e:
            errors.append(e)

    say("concurrent batches k=" + ",".join(str(k) for k in conc))
    threads = [threading.Thread(target=work, args=(k, b)) for k, b in conc.items()]
    for t in threads:
        t.start()
    for t in threads:
        t.join()
    torch.cuda.synchronize()
    assert not errors, errors
    for k, b in conc.items():
        p_seq, st_seq, w_seq = seq[k]
        for j, (x, y) in enumerate(zip(b.local_partitions(), p_seq)):
            assert np.array_equal(x, y), f"k={k} graph {j}: partition"
        assert np.array_equal(b.stats.cpu().numpy(), st_seq), f"k={k}: statistics"
        assert np.array_equal(b.W.cpu().numpy(), w_seq), f"k={k}: block weights"
        c = b.ctx
        b.close()
        c.close()
