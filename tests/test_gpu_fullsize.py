"""GPU parity at full size: the three single-graph workloads in the
configuration the benchmark times, against the oracle, element by element
after every round compared.

* rmat20: R-MAT scale 20 (irregular), k = 64, all 20 rounds of its schedule.
* grid2048: the 2048 x 2048 4-neighbour grid (regular), k = 64, 3 rounds.
* chunglu8m: the 8M-node Chung-Lu graph with exponent 2.1 (hubs above 10^5
  edges, split into dozens of edge chunks), edge weights in [1, 16], k = 256:
  the n x k table is 8.2 GB, so its byte offsets pass 4 GiB; 2 rounds.

Compared after each round: the statistics, the partition, the block
weights, every node's target, score, penalty and filter decision, and the
whole gain table (in row chunks for the 8.2 GB one). Each round is its own
test, so that progress shows while the oracle works through the large
graphs (about half a minute per 8M-node round on one core)."""
import sys

import numpy as np
import pytest

from oracle import oracle as O
from paper_2308_15494_amd import graphgen as gg
from tests.test_gpu_parity import ctx, upr  # noqa: F401  (fixtures)

# the 8M-node rounds take half a minute each in the oracle, after a minute of
# generation
pytestmark = [pytest.mark.gpu, pytest.mark.timeout(900)]


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


class FullPair:
    """The same round state on the GPU and in the oracle, compared with the
    table in row chunks (no full host copy of the device table)."""

    def __init__(self, upr, ctx, name):
        import torch
        g, k, eps, rounds, seed = gg.workload(name)
        self.upr, self.ctx, self.g, self.k = upr, ctx, g, k
        self.eps, self.rounds = eps, rounds
        part0 = gg.random_partition(g.n, k, seed)
        self.dg = upr.DeviceGraph(g)
        self.plan = upr.Plan(ctx, self.dg)
        self.part = torch.from_numpy(part0.copy()).to("cuda")
        self.conn = torch.zeros(g.n * k, dtype=torch.int32, device="cuda")
        self.W = torch.zeros(k, dtype=torch.int64, device="cuda")
        self.stats = torch.zeros(12, dtype=torch.int64, device="cuda")
        self.G = O.Graph(g)
        self.opart = part0.copy()
        self.oconn = np.zeros(g.n * k, np.int32)
        self.oW = np.zeros(k, np.int64)
        self.done = 0

    def round(self, r):
        assert r == self.done + 1, "rounds run in order"
        kw = dict(eps=self.eps, tau=gg.tau_schedule(r, self.rounds))
        self.upr.refine_round(self.ctx, self.plan, self.upr.params(self.k, **kw), self.part,
                              self.conn, self.W, self.stats)
        ost, odbg = O.refine_round(self.G, O.params(self.k, **kw), self.opart, self.oconn,
                                   self.oW, debug=True)
        self.done = r
        return ost, odbg

    def compare(self, ost, odbg, what, rows=1 << 20):
        import torch
        torch.cuda.synchronize()
        assert O.stats_dict(self.stats.cpu().numpy()) == O.stats_dict(ost), f"{what}: stats"
        assert np.array_equal(self.part.cpu().numpy(), self.opart), f"{what}: partition"
        assert np.array_equal(self.W.cpu().numpy(), self.oW), f"{what}: block weights"
        mv = self.upr.last_moves(self.ctx, self.g.n)
        for key in ("target", "score", "pen", "accept"):
            assert np.array_equal(mv[key].cpu().numpy(), odbg[key]), f"{what}: {key}"
        del mv
        n, k = self.g.n, self.k
        for v0 in range(0, n, rows):
            v1 = min(v0 + rows, n)
            got = self.conn[v0 * k:v1 * k].cpu().numpy()
            assert np.array_equal(got, self.oconn[v0 * k:v1 * k]), f"{what}: table rows {v0}.."

    def close(self):
        self.plan.close()


@pytest.fixture(scope="module")
def rmat20(upr, ctx):
    pr = FullPair(upr, ctx, "rmat20")
    say(f"rmat20 n={pr.g.n} m={pr.g.m}")
    yield pr
    pr.close()


@pytest.fixture(scope="module")
def grid(upr, ctx):
    pr = FullPair(upr, ctx, "grid2048")
    say(f"grid2048 n={pr.g.n} m={pr.g.m}")
    yield pr
    pr.close()


@pytest.fixture(scope="module")
def cl8m(upr, ctx):
    say("chunglu8m: generating")
    pr = FullPair(upr, ctx, "chunglu8m")
    say(f"chunglu8m n={pr.g.n} m={pr.g.m} max degree {pr.g.meta['max_degree']}")
    yield pr
    pr.close()
    del pr
    import torch
    torch.cuda.empty_cache()


@pytest.mark.parametrize("r", range(1, 21))
def test_rmat20_round(rmat20, r):
    """R-MAT scale 20, k = 64: the benchmark's workload, every round."""
    ost, odbg = rmat20.round(r)
    rmat20.compare(ost, odbg, f"rmat20 round {r}")


def test_grid2048_shape(grid):
    g = grid.g
    assert g.n == 4_194_304 and g.m == 8_384_512 and grid.k == 64
    assert g.meta["max_degree"] == 4 and g.irregularity() < 0.1


@pytest.mark.parametrize("r", [1, 2, 3])
def test_grid2048_round(grid, r):
    """The regular contrast: 2048 x 2048 grid at k = 64."""
    say(f"grid2048 round {r}")
    ost, odbg = grid.round(r)
    grid.compare(ost, odbg, f"grid2048 round {r}")
    if r == 1:
        # a random start moves many nodes: the filter and the apply are busy
        assert ost[5] > 100_000


def test_chunglu8m_shape(cl8m):
    """The paths only this workload reaches: a table beyond 4 GiB, hubs of
    more than 10^5 edges (dozens of 4096-edge chunks) and weighted degrees
    that need 32-bit table counters."""
    g = cl8m.g
    assert g.n == 8_000_000 and cl8m.k == 256 and g.adjwgt is not None
    assert g.meta["max_degree"] > 100_000
    assert g.n * cl8m.k * 4 > (1 << 32)
    info = cl8m.plan.info()
    assert info["num_hubs"] > 0 and info["max_degree"] // 4096 >= 25
    wdeg = np.add.reduceat(g.adjwgt.astype(np.int64), g.xadj[:-1])
    assert int(wdeg.max()) >= 1 << 16


@pytest.mark.parametrize("r", [1, 2])
def test_chunglu8m_round(cl8m, r):
    """8M-node weighted Chung-Lu at k = 256."""
    say(f"chunglu8m round {r}")
    ost, odbg = cl8m.round(r)
    cl8m.compare(ost, odbg, f"chunglu8m round {r}")
