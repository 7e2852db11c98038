"""GPU: the captured move phases (upr_capture_enable) against eager rounds,
round by round, with eager work between the graph replays (every replay is
checked: statistics, partition, block weights and table), across the
configurations a graph is keyed by, and with more configurations than the
context keeps."""
import numpy as np
import pytest

from paper_2308_15494_amd import graphgen as gg
from tests.test_gpu_parity import say, skewed_partition, to_dev, upr  # noqa: F401

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx2(upr):
    """An eager context and one that captures."""
    eager, cap = upr.Context(0), upr.Context(0)
    cap.capture(True)
    yield eager, cap
    cap.capture(False)
    eager.close()
    cap.close()


class Run:
    def __init__(self, upr, ctx, g, k, part0):
        import torch
        self.upr, self.ctx, self.k = upr, ctx, k
        self.dg = upr.DeviceGraph(g)
        self.plan = upr.Plan(ctx, self.dg)
        self.part = to_dev(part0.astype(np.int32))
        self.conn = torch.zeros(max(g.n * k, 1), dtype=torch.int32, device="cuda")
        self.W = torch.zeros(k, dtype=torch.int64, device="cuda")

    def round(self, **kw):
        return self.upr.refine_round(self.ctx, self.plan, self.upr.params(self.k, **kw), self.part,
                                     self.conn, self.W).cpu().numpy()

    def state(self):
        return self.part.cpu().numpy(), self.W.cpu().numpy(), self.conn.cpu().numpy()


def _compare(a, b, what):
    sa, sb = a.state(), b.state()
    for name, x, y in zip(("part", "W", "conn"), sa, sb):
        assert np.array_equal(x, y), f"{what}: {name}"


CASES = [
    ("cl", lambda: gg.chung_lu(6000, 8.0, 2.3, seed=5), 16, {}),
    ("cl_w", lambda: gg.chung_lu(5000, 10.0, 2.2, seed=6, wmax=9), 8, {}),
    ("rmat16_relabelled", lambda: gg.rmat(16, 16, seed=7), 64, {}),
    ("grid_adjacency_form", lambda: gg.grid2d(60, 70), 32, {}),
    ("k300", lambda: gg.chung_lu(6000, 10.0, 2.2, seed=8), 300, {}),
    ("seq_off_mode2", lambda: gg.chung_lu(5000, 8.0, 2.3, seed=9), 16, dict(seq_penalty=0, mode=2)),
    ("optimistic_limited", lambda: gg.chung_lu(5000, 8.0, 2.3, seed=10), 16,
     dict(variant=1, mode=3, alpha=(3, 2))),
]


@pytest.mark.parametrize("case", CASES, ids=[c[0] for c in CASES])
@pytest.mark.parametrize("form", ["rebuild", "resident"])
def test_captured_rounds_equal_eager(upr, ctx2, case, form):
    eager, cap = ctx2
    name, make, k, kw = case
    g = make()
    part0 = skewed_partition(g.n, k, 2, 0.3)
    a, b = Run(upr, eager, g, k, part0), Run(upr, cap, g, k, part0)
    R = 6
    say(f"capture {name} {form} n={g.n} k={k}")
    for r in range(1, R + 1):
        p = dict(kw, tau=gg.tau_schedule(r, R), rebuild_table=1 if form == "rebuild" or r == 1 else 0)
        sa, sb = a.round(**p), b.round(**p)
        assert np.array_equal(sa, sb), f"{name} {form} round {r}: stats"
        _compare(a, b, f"{name} {form} round {r}")
        # eager work on the capturing context between replays
        cut = upr.edge_cut(cap, b.plan, b.part).cpu().numpy()
        assert int(cut.reshape(-1)[0]) == int(sb[3])
    a.plan.close()
    b.plan.close()


def test_capture_keys_and_eviction(upr, ctx2):
    """More configurations than the context keeps (16), revisited in another
    order, and a new partition array (a new key): always the eager result."""
    eager, cap = ctx2
    g = gg.chung_lu(4000, 8.0, 2.3, seed=12)
    k = 8
    part0 = gg.random_partition(g.n, k, 3)
    a, b = Run(upr, eager, g, k, part0), Run(upr, cap, g, k, part0)
    confs = [dict(t=(t, 10), mode=m) for t in (3, 5, 7, 9, 10) for m in (0, 1, 2, 3)]
    order = confs + confs[::-1] + confs[::3]
    for i, c in enumerate(order):
        extra = dict(alpha=(3, 2)) if c["mode"] == 3 else {}
        assert np.array_equal(a.round(tau=(1, 2), **c, **extra), b.round(tau=(1, 2), **c, **extra)), i
    _compare(a, b, "after the configurations")
    # new arrays for the same graph: a new key
    b.part = b.part.clone()
    b.conn = b.conn.clone()
    b.W = b.W.clone()
    for r in range(3):
        assert np.array_equal(a.round(tau=(1, 1)), b.round(tau=(1, 1))), r
    _compare(a, b, "after new arrays")
    a.plan.close()
    b.plan.close()


def test_captured_batch_rounds_equal_eager(upr, ctx2):
    """A batch (its own plan, per-graph penalty factors uploaded eagerly every
    round): captured and eager rounds agree on every graph after every round."""
    eager, cap = ctx2
    graphs = [gg.chung_lu(3000 + 500 * i, 8.0, 2.3, seed=20 + i) if i % 2 == 0 else
              gg.rgg2d(2500 + 400 * i, seed=30 + i) for i in range(6)]
    k = 8
    parts = [skewed_partition(g.n, k, i, 0.3) for i, g in enumerate(graphs)]
    ba, bb = upr.Batch(eager, graphs, k), upr.Batch(cap, graphs, k)
    ba.set_partitions(parts)
    bb.set_partitions(parts)
    R = 6
    for r in range(1, R + 1):
        taus = [gg.tau_schedule(min(r + g, R), R) for g in range(len(graphs))]
        p = upr.params(k, tau=(1, 1))
        sa = ba.round(p, taus=taus).cpu().numpy()
        sb = bb.round(p, taus=taus).cpu().numpy()
        assert np.array_equal(sa, sb), f"round {r}: stats"
        for name in ("part", "W", "conn"):
            assert np.array_equal(getattr(ba, name).cpu().numpy(), getattr(bb, name).cpu().numpy()), \
                f"round {r}: {name}"
        # eager work on the capturing context between replays
        g0 = upr.DeviceGraph(graphs[0])
        pl = upr.Plan(cap, g0)
        upr.gain_table(cap, pl, k, to_dev(parts[0].astype(np.int32)))
        pl.close()
    ba.close()
    bb.close()
