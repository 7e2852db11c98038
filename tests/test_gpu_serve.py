"""Serving with continuous batching: every request's result (final partition
and per-round statistics) is the same in the mix as alone, and the same as
the oracle's, also when the server's context replays its move phases from
captured HIP graphs and when its groups run concurrently."""
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
def env():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2308_15494_amd import serve, upr
    upr.lib()
    ctx = upr.Context(0)
    yield upr, serve, ctx
    ctx.close()


@pytest.fixture(scope="module")
def cap_ctx(env):
    upr = env[0]
    c = upr.Context(0)
    c.capture(True)
    yield c
    c.capture(False)
    c.close()


def make_requests(serve, count, seed, rate):
    rng = np.random.default_rng(seed)
    arr = serve.poisson_arrivals(count, rate, seed)
    reqs = []
    for i in range(count):
        m = int(np.exp(rng.uniform(np.log(2e3), np.log(6e4))))
        if i % 2:
            g = gg.chung_lu(max(m // 8, 50), 16.0, float(rng.uniform(2.1, 2.8)), seed=seed + i)
        else:
            g = gg.rmat(max(int(np.ceil(np.log2(max(m / 16, 16)))), 4), 16, seed=seed + i)
        k = int(rng.choice([4, 8, 16]))
        reqs.append(serve.Request(i, g, k, (3, 100), rounds=int(rng.integers(2, 6)),
                                  arrival=float(arr[i]), part_seed=seed + 1000 + i))
    return reqs


@pytest.mark.parametrize("mode", ["plain", "captured", "concurrent", "uploads_ahead"])
@pytest.mark.parametrize("budget_mb", [1, 4096])
def test_serve_results_same_alone_and_in_mix(env, cap_ctx, budget_mb, mode):
    upr, serve, ctx = env
    reqs = make_requests(serve, 14, 5, rate=400.0)
    say(f"serve budget={budget_mb}MB mode={mode} sizes={[r.graph.n for r in reqs]} "
        f"k={[r.k for r in reqs]}")
    # requests refined alone run on the eager context; the concurrent server
    # gives every (k, eps) group a context, stream and thread of its own, and
    # may upload the arrived requests' graphs from a thread of its own
    srv = serve.Server(cap_ctx if mode == "captured" else ctx, budget_mb << 20,
                       concurrent=mode in ("concurrent", "uploads_ahead"),
                       uploads_ahead=4 if mode == "uploads_ahead" else 0)
    res = srv.run(reqs)
    # the contexts of the groups and of the upload thread are reused
    res2 = srv.run(reqs) if mode in ("concurrent", "uploads_ahead") else res
    srv.close()
    assert [(r.rid, r.stats) for r in res2] == [(r.rid, r.stats) for r in res]
    assert all(np.array_equal(a.part, b.part) for a, b in zip(res, res2))
    assert [r.rid for r in res] == list(range(len(reqs)))
    for req, r in zip(reqs, res):
        part, stats = serve.refine_alone(ctx, req)
        assert np.array_equal(r.part, part), f"request {req.rid}: partition differs from alone"
        assert r.stats == stats, f"request {req.rid}: statistics differ from alone"
        assert r.latency >= 0 and r.done >= r.admitted >= r.arrival - 1e-9
    # the oracle agrees with a few of them
    for req, r in list(zip(reqs, res))[:4]:
        G = O.Graph(req.graph)
        p = gg.random_partition(req.graph.n, req.k, req.part_seed)
        conn = np.zeros(req.graph.n * req.k, np.int32)
        W = np.zeros(req.k, np.int64)
        for i in range(1, req.rounds + 1):
            st, _ = O.refine_round(G, O.params(req.k, req.eps, tau=gg.tau_schedule(i, req.rounds)),
                                   p, conn, W)
            assert O.stats_dict(st) == O.stats_dict(np.array(
                [r.stats[i - 1][n] for n in upr.STAT_NAMES] + [0, 0, 0])), f"request {req.rid} round {i}"
        assert np.array_equal(p, r.part)


@pytest.mark.parametrize("uploads", [0, 3])
def test_serve_admission_respects_budget(env, uploads):
    upr, serve, ctx = env
    reqs = make_requests(serve, 8, 9, rate=1e4)
    budget = max(r.footprint() for r in reqs) + 1
    seen = []
    srv = serve.Server(ctx, budget, uploads_ahead=uploads)
    res = srv.run(reqs, on_done=lambda r: seen.append(r.rid))
    srv.close()
    assert sorted(seen) == list(range(len(reqs)))
    by_id = {r.rid: r for r in res}
    # at every admission, the requests then in the server fit the budget
    for r in res:
        t = r.admitted
        live = [q for q in reqs if by_id[q.rid].admitted <= t < by_id[q.rid].done]
        assert len(live) <= 1 or sum(q.footprint() for q in live) <= budget
