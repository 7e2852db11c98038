"""Autotuner of the traversal thresholds (upr_plan_opts) for one graph or one
batch.

The thresholds decide how work is spread over lanes and workgroups (hub
threshold: degree above which a node's edges are split into whole-workgroup
chunks; dirty divisor: when the apply rebuilds table tiles instead of sending atomic
deltas). None of them changes a result, so the tuner may pick any of them:
it times a few rounds of the real workload per candidate, coordinate by
coordinate, and keeps the fastest. It also checks that every candidate gives
the same statistics, which is the property that makes tuning safe.
"""
from __future__ import annotations

import time

import numpy as np

from . import graphgen as gg
from . import upr

HUB = (1024, 2048, 4096, 8192, 16384)
DIRTY = (2, 4, 8, 16, 32)


def _time_rounds(make_runner, rounds, repeats):
    run, reset, stats = make_runner()
    best = float("inf")
    out = None
    for _ in range(repeats):
        reset()
        import torch
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for i in range(1, rounds + 1):
            run(i)
        torch.cuda.synchronize()
        best = min(best, time.perf_counter() - t0)
        out = stats()
    return best, out


def tune_graph(ctx, g, k, part0, eps=(3, 100), rounds=3, repeats=2, total_rounds=20):
    """Pick upr_plan_opts for one graph from timed trial rounds (the first
    `rounds` rounds of its schedule from part0). Returns (opts, report)."""
    import torch
    dg = upr.DeviceGraph(g)

    def runner_for(opts):
        def make():
            plan = upr.Plan(ctx, dg, opts=opts)
            part = torch.empty(g.n, dtype=torch.int32, device="cuda")
            conn = torch.zeros(max(g.n * k, 1), dtype=torch.int32, device="cuda")
            W = torch.zeros(k, dtype=torch.int64, device="cuda")
            stats = torch.zeros(upr.STATS_LEN, dtype=torch.int64, device="cuda")
            p0 = torch.from_numpy(np.ascontiguousarray(part0, np.int32)).cuda()

            def reset():
                part.copy_(p0)

            def run(i):
                upr.refine_round(ctx, plan, upr.params(k, eps, tau=gg.tau_schedule(i, total_rounds)),
                                 part, conn, W, stats)

            def result():
                return stats.cpu().numpy().copy(), part.cpu().numpy().copy()
            make.plan = plan
            return run, reset, result
        return make

    return _coordinate_search(runner_for, rounds, repeats)


def tune_batch(ctx, graphs, k, parts, eps=(3, 100), rounds=3, repeats=2, total_rounds=10):
    """Pick upr_plan_opts for a batch (the union's plan) from timed trial
    rounds. Returns (opts, report)."""
    dgs = [upr.DeviceGraph(g) for g in graphs]

    def runner_for(opts):
        def make():
            b = upr.Batch(ctx, dgs, k, eps, opts=opts)

            def reset():
                b.set_partitions(parts)

            def run(i):
                b.round(upr.params(k, eps, tau=gg.tau_schedule(i, total_rounds)))

            def result():
                return b.stats.cpu().numpy().copy(), b.part.cpu().numpy().copy()
            return run, reset, result
        return make

    return _coordinate_search(runner_for, rounds, repeats)


def _coordinate_search(runner_for, rounds, repeats):
    cur = dict(hub_threshold=4096, dirty_div=16)
    report = []
    ref = None
    best_t = None
    for name, values in (("hub_threshold", HUB), ("dirty_div", DIRTY)):
        best_v = cur[name]
        for v in values:
            trial = dict(cur)
            trial[name] = v
            t, res = _time_rounds(runner_for(upr.plan_opts(**trial)), rounds, repeats)
            if ref is None:
                ref = res
            same = bool(np.array_equal(ref[0], res[0]) and np.array_equal(ref[1], res[1]))
            report.append(dict(trial, seconds=t, same_result=same))
            if not same:
                raise RuntimeError(f"thresholds {trial} changed the result")
            if best_t is None or t < best_t:
                best_t, best_v = t, v
        cur[name] = best_v
    return upr.plan_opts(**cur), dict(chosen=cur, best_seconds=best_t, trials=report)
