"""GPU parity of the interleaved move sequence and best prefix (Section 5.4):
the round with the best-prefix variant against the oracle, element by
element after every round (statistics including the kept boundary and the
undone nodes, partition, block weights, table, per-node moves)."""
import numpy as np
import pytest

from paper_2308_15494_amd import graphgen as gg
from tests.test_gpu_parity import Pair, ctx, say, skewed_partition, upr  # noqa: F401

pytestmark = pytest.mark.gpu

BEST_PREFIX = 4


@pytest.mark.parametrize("case", [
    ("er_w", lambda: gg.random_small(400, 0.04, seed=2, wmax=9, vmax=5), 5),
    ("cl", lambda: gg.chung_lu(5000, 10.0, 2.3, seed=3), 8),
    ("cl_w", lambda: gg.chung_lu(4000, 12.0, 2.1, seed=4, wmax=16), 32),
    ("grid", lambda: gg.grid2d(61, 77), 16),
    ("rgg", lambda: gg.rgg2d(6000, seed=5), 4),
    ("rmat", lambda: gg.rmat(13, 16, seed=5), 64),
], ids=lambda c: c[0] if isinstance(c, tuple) else str(c))
@pytest.mark.parametrize("mode", [0, 2])
def test_prefix_rounds(upr, ctx, case, mode):
    name, make, k = case
    g = make()
    for start in ("random", "skewed"):
        part0 = gg.random_partition(g.n, k, 7) if start == "random" else \
            skewed_partition(g.n, k, 8, 0.4)
        pr = Pair(upr, ctx, g, k, part0)
        kept = []
        for r in range(1, 5):
            say(f"prefix {name} mode {mode} {start} round {r}")
            ost, odbg = pr.round(tau=gg.tau_schedule(r, 4), mode=mode, variant=BEST_PREFIX)
            pr.compare(ost, odbg, f"{name} {start} round {r}")
            kept.append((int(ost[9]), int(odbg["pref"][1])))
        say(f"  kept/steps per round: {kept}")


def test_prefix_seq_off_and_resident(upr, ctx):
    """With the round-start price (seq_penalty 0) and the resident table."""
    g = gg.chung_lu(6000, 8.0, 2.3, seed=21)
    k = 16
    pr = Pair(upr, ctx, g, k, skewed_partition(g.n, k, 2, 0.3))
    for r in range(1, 5):
        ost, odbg = pr.round(tau=gg.tau_schedule(r, 4), seq_penalty=0, variant=BEST_PREFIX,
                             rebuild_table=1 if r == 1 else 0)
        pr.compare(ost, odbg, f"round {r}")


def test_prefix_proper_prefixes_occur(upr, ctx):
    """Penalty-free rounds from skewed starts on a power-law graph: some
    rounds keep a proper prefix (the GPU undoes moves) and match the oracle."""
    g = gg.chung_lu(20000, 8.0, 2.2, seed=31)
    k = 8
    proper = 0
    for seed in range(3):
        pr = Pair(upr, ctx, g, k, skewed_partition(g.n, k, seed, 0.35))
        for r in range(1, 4):
            ost, odbg = pr.round(mode=2, variant=BEST_PREFIX)
            pr.compare(ost, odbg, f"seed {seed} round {r}")
            proper += 0 <= ost[9] < odbg["pref"][1]
    say(f"proper prefixes: {proper}")
    assert proper >= 1


def test_prefix_rmat20(upr, ctx):
    """The benchmark graph (R-MAT scale 20, k = 64) with the best prefix,
    first four rounds."""
    g, k, eps, rounds, seed = gg.workload("rmat20")
    pr = Pair(upr, ctx, g, k, gg.random_partition(g.n, k, seed))
    for r in range(1, 5):
        say(f"prefix rmat20 round {r}")
        ost, odbg = pr.round(eps=eps, tau=gg.tau_schedule(r, rounds), variant=BEST_PREFIX)
        pr.compare(ost, odbg, f"rmat20 round {r}")
        say(f"  kept {int(ost[9])} of {int(odbg['pref'][1])} steps, undone {int(ost[10])}")


def test_prefix_batch_rejected(upr, ctx):
    g = gg.chung_lu(2000, 8.0, 2.3, seed=3)
    b = upr.Batch(ctx, [g, gg.rgg2d(1000, seed=4)], 4)
    b.set_partitions([gg.random_partition(g.n, 4, 1), gg.random_partition(1000, 4, 2)])
    with pytest.raises(upr.UprError) as ei:
        b.round(upr.params(4, variant=BEST_PREFIX))
    assert ei.value.code == -1
    b.close()
