"""The threshold autotuner: every candidate gives the same result (checked by
the tuner itself), and the chosen plan reproduces the oracle."""
import sys

import numpy as np
import pytest

from oracle import oracle as O
from paper_2308_15494_amd import graphgen as gg

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def env():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2308_15494_amd import tune, upr
    upr.lib()
    ctx = upr.Context(0)
    yield upr, tune, ctx
    ctx.close()


def test_tune_graph(env):
    upr, tune, ctx = env
    g = gg.chung_lu(20000, 10.0, 2.1, seed=3)
    k = 16
    part0 = gg.random_partition(g.n, k, 4)
    opts, rep = tune.tune_graph(ctx, g, k, part0, rounds=2, repeats=1)
    print(rep["chosen"], flush=True)
    assert all(t["same_result"] for t in rep["trials"])
    assert rep["chosen"]["hub_threshold"] in tune.HUB
    # the tuned plan against the oracle over a few rounds
    r = upr.Refiner(g, k, ctx=ctx, opts=opts)
    r.set_partition(part0)
    op = part0.copy()
    G = O.Graph(g)
    for i in range(1, 4):
        r.round(upr.params(k, tau=gg.tau_schedule(i, 3)))
        st, _ = O.refine_round(G, O.params(k, tau=gg.tau_schedule(i, 3)), op)
        assert upr.stats_dict(r.stats) == O.stats_dict(st)
    assert np.array_equal(r.part.cpu().numpy(), op)


def test_tune_batch(env):
    upr, tune, ctx = env
    k = 8
    graphs = [gg.chung_lu(3000, 8.0, 2.3, seed=s) for s in range(3)] + [gg.rgg2d(2000, seed=9)]
    parts = [gg.random_partition(g.n, k, i) for i, g in enumerate(graphs)]
    opts, rep = tune.tune_batch(ctx, graphs, k, parts, rounds=2, repeats=1)
    assert all(t["same_result"] for t in rep["trials"])
    assert len(rep["trials"]) >= 10
