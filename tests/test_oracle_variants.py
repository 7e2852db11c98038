"""Pins of the oracle's variants of Section 8.2: limited imbalance (no
penalty, targets capped at alpha * L_max, alpha shrinking over the rounds),
the optimistic conflict filter (an earlier candidate neighbour counts as
moved), and rebalancing by the plain gain (no node weight in the priority)."""
import numpy as np
import pytest

from paper_2308_15494_amd import graphgen as gg
from tests import bruteforce as bf
from tests.test_oracle_round import SMALL, skewed_partition


def run(orc, g, k, part0, **kw):
    part = part0.copy()
    st, dbg = orc.refine_round(g, orc.params(k, **kw), part, debug=True)
    return st, dbg, part


# ------------------------------------------------- limited imbalance --

def test_alpha_schedule():
    """alpha_1 = 2, alpha_R = 1.1, linear in between (Section 8.2)."""
    from fractions import Fraction
    R = 10
    vals = [Fraction(*gg.alpha_schedule(r, R)) for r in range(1, R + 1)]
    assert vals[0] == 2 and vals[-1] == Fraction(11, 10)
    steps = {vals[i] - vals[i + 1] for i in range(R - 1)}
    assert steps == {Fraction(1, 10)}
    assert gg.alpha_schedule(1, 1) == (11, 10)


@pytest.mark.parametrize("name,make", SMALL)
@pytest.mark.parametrize("k", [2, 3, 5])
@pytest.mark.parametrize("alpha", [(1, 1), (11, 10), (3, 2), (2, 1)])
def test_limited_imbalance_best_moves_bruteforce(orc, name, make, k, alpha):
    for seed in range(3):
        g = make(seed + 7 * k)
        for part0 in [gg.random_partition(g.n, k, seed), skewed_partition(g.n, k, seed)]:
            _, dbg, _ = run(orc, g, k, part0, mode=3, alpha=alpha)
            expect = bf.best_moves(g, k, list(part0), (7, 10), (1, 1), (3, 100), 3, alpha)
            got = {v: (int(dbg["target"][v]), int(dbg["score"][v]), int(dbg["pen"][v]))
                   for v in range(g.n) if dbg["target"][v] >= 0}
            assert got == expect


@pytest.mark.parametrize("name,make", SMALL)
@pytest.mark.parametrize("seq", [0, 1])
@pytest.mark.parametrize("alpha", [(11, 10), (2, 1)])
def test_limited_imbalance_filter_bruteforce(orc, name, make, seq, alpha):
    k = 3
    for seed in range(3):
        g = make(300 + seed)
        if g.n > 40:
            continue
        part0 = skewed_partition(g.n, k, seed, heavy=0.45)
        _, dbg, _ = run(orc, g, k, part0, mode=3, alpha=alpha, seq_penalty=seq)
        expect = bf.filter_decisions(g, k, list(part0), (7, 10), (1, 1), (3, 100), 3, bool(seq),
                                     alpha=alpha)
        got = {int(v): (bool(dbg["accept"][v]), None if dbg["pen_seq"][v] < 0 else int(dbg["pen_seq"][v]))
               for v in np.nonzero(dbg["target"] >= 0)[0]}
        assert got == expect


@pytest.mark.parametrize("seq", [0, 1])
def test_limited_imbalance_special_cases(orc, seq):
    """alpha = 1 is the constrained round; an alpha large enough that no
    block can exceed alpha * L_max is the penalty-free round."""
    g = gg.chung_lu(3000, 8.0, 2.3, seed=3)
    k = 8
    for start in (gg.random_partition(g.n, k, 1), skewed_partition(g.n, k, 1, 0.4)):
        a = run(orc, g, k, start, mode=3, alpha=(1, 1), seq_penalty=seq)
        b = run(orc, g, k, start, mode=1, seq_penalty=seq)
        assert np.array_equal(a[0], b[0]) and np.array_equal(a[2], b[2])
        a = run(orc, g, k, start, mode=3, alpha=(k, 1), seq_penalty=seq)
        b = run(orc, g, k, start, mode=2, seq_penalty=seq)
        assert np.array_equal(a[0], b[0]) and np.array_equal(a[2], b[2])


# ------------------------------------------------ optimistic filter --

@pytest.mark.parametrize("name,make", SMALL)
@pytest.mark.parametrize("seq", [0, 1])
@pytest.mark.parametrize("mode", [0, 2])
def test_optimistic_filter_bruteforce(orc, name, make, seq, mode):
    k = 3
    for seed in range(3):
        g = make(400 + seed)
        if g.n > 40:
            continue
        part0 = skewed_partition(g.n, k, seed, heavy=0.45)
        _, dbg, _ = run(orc, g, k, part0, mode=mode, seq_penalty=seq, variant=orc.OPTIMISTIC)
        expect = bf.filter_decisions(g, k, list(part0), (7, 10), (1, 1), (3, 100), mode, bool(seq),
                                     optimistic=True)
        got = {int(v): (bool(dbg["accept"][v]), None if dbg["pen_seq"][v] < 0 else int(dbg["pen_seq"][v]))
               for v in np.nonzero(dbg["target"] >= 0)[0]}
        assert got == expect


def test_optimistic_and_pessimistic_on_a_matching(orc):
    """A perfect matching with every pair split: both ends want to join the
    other, the earlier one moves and the later one must not follow (either
    way the later move would cut its edge again). With every pair in one
    block nobody is a candidate."""
    n = 40
    edges = [(2 * i, 2 * i + 1) for i in range(n // 2)]
    g = bf.graph_from_edges(n, edges)
    k = 4
    # partner pairs split across blocks: both are candidates of each other,
    # so the order matters; same block: no candidates at all
    part0 = np.array([i % 2 for i in range(n)], np.int32)
    a = run(orc, g, k, part0, mode=2)
    b = run(orc, g, k, part0, mode=2, variant=orc.OPTIMISTIC)
    # the pair (u, v): u is earlier and targets v's block. Pessimistically u
    # counts in the worse of its blocks for v (v's own block: gain -1);
    # optimistically u has already joined v's block (gain -1 again). Only the
    # earlier end of every pair moves.
    assert a[0][5] == b[0][5] == n // 2
    part1 = np.zeros(n, np.int32)
    a = run(orc, g, k, part1, mode=2)
    b = run(orc, g, k, part1, mode=2, variant=orc.OPTIMISTIC)
    assert np.array_equal(a[0], b[0]) and a[0][4] == 0


# ------------------------------------------ plain-gain rebalancing --

@pytest.mark.parametrize("k", [2, 3, 5])
def test_plain_priority_one_iteration_bruteforce(orc, k):
    from tests.test_oracle_round import with_isolated
    for seed in range(8):
        base = gg.random_small(26, 0.12, seed=seed, wmax=4, vmax=5)
        g = with_isolated(base, 4, seed)
        part0 = skewed_partition(g.n, k, seed, heavy=0.55)
        L = orc.lmax(orc.total_weight(g), k)
        part = part0.copy()
        orc.rebalance(g, orc.params(k, max_rebalance_iters=1, variant=orc.PLAIN_PRIORITY), part)
        assert part.tolist() == bf.rebalance_one_iteration(g, k, list(part0), L, plain=True)


def test_plain_priority_unit_weights_unchanged(orc):
    """With unit node weights g*c(u) = g and g/c(u) = g: the variant is the
    main rebalancer."""
    g = gg.chung_lu(3000, 8.0, 2.3, seed=8)
    k = 8
    for start in (skewed_partition(g.n, k, 3, 0.5), np.zeros(g.n, np.int32)):
        pa, pb = start.copy(), start.copy()
        sa = orc.rebalance(g, orc.params(k), pa)
        sb = orc.rebalance(g, orc.params(k, variant=orc.PLAIN_PRIORITY), pb)
        assert np.array_equal(sa, sb) and np.array_equal(pa, pb)


def test_variant_params_checked(orc):
    g = gg.random_small(10, 0.3, seed=1)
    part = np.zeros(10, np.int32)
    with pytest.raises(Exception):
        orc.refine_round(g, orc.params(2, mode=3, alpha=(9, 10)), part)
    with pytest.raises(Exception):
        orc.refine_round(g, orc.params(2, variant=8), part)
