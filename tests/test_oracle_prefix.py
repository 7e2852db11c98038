"""Pins of the oracle's interleaved move sequence and best prefix (Section
5.4; the last two steps of Algorithm 1).

The reference is tests/bruteforce.interleaved_best_prefix: written from the
rules on Python lists, with its own rebalancer trace (the sub-iteration rules
of Section 7.1, each move's priority bucket recomputed from cut
differences), the combined double moves, the interleaving by minimal
prefixes of the overloaded block's rebalancing moves, and every cumulative
gain taken as a cut difference. The filtered moves come from the plain
round, whose decisions are pinned elsewhere."""
import numpy as np
import pytest

from paper_2308_15494_amd import graphgen as gg
from tests import bruteforce as bf
from tests.test_oracle_round import SMALL, skewed_partition

ST_CUT_BEFORE, ST_CUT_AFTER, ST_STATUS, ST_PREFIX, ST_REVERTED = 1, 3, 8, 9, 10


def filtered_moves(dbg):
    """The accepted moves in the filter's order: score descending, id ascending."""
    cand = [v for v in range(dbg["target"].size) if dbg["target"][v] >= 0]
    cand.sort(key=lambda v: (-int(dbg["score"][v]), v))
    return [(v, int(dbg["target"][v])) for v in cand if dbg["accept"][v]]


def both_rounds(orc, g, k, part0, **kw):
    std = part0.copy()
    st0, dbg0 = orc.refine_round(g, orc.params(k, **kw), std, debug=True)
    part = part0.copy()
    kw["variant"] = kw.get("variant", 0) | orc.BEST_PREFIX
    st, dbg = orc.refine_round(g, orc.params(k, **kw), part, debug=True)
    return (st0, dbg0, std), (st, dbg, part)


@pytest.mark.parametrize("name,make", SMALL)
@pytest.mark.parametrize("k", [2, 3, 5])
@pytest.mark.parametrize("mode,tau", [(0, (1, 2)), (2, (1, 1)), (1, (1, 1))])
def test_prefix_matches_bruteforce(orc, name, make, k, mode, tau):
    checked = 0
    for seed in range(4):
        g = make(seed + 11 * k)
        L = orc.lmax(orc.total_weight(g), k)
        for part0 in (gg.random_partition(g.n, k, seed), skewed_partition(g.n, k, seed, 0.5)):
            (st0, dbg0, std), (st, dbg, part) = both_rounds(orc, g, k, part0, mode=mode, tau=tau)
            exp, best, gains, bal = bf.interleaved_best_prefix(g, k, list(part0),
                                                               filtered_moves(dbg0), L)
            assert part.tolist() == exp
            assert st[ST_PREFIX] == best
            assert dbg["bgain"].tolist() == gains
            assert [bool(b) for b in dbg["bbal"]] == bal
            assert st[ST_CUT_AFTER] == bf.cut(g, part.tolist())
            reverted = sum(1 for v in range(g.n) if std[v] != part0[v] and part[v] == part0[v])
            assert st[ST_REVERTED] == (reverted if best >= 0 else 0)
            # the steps before the rebalancing are those of the plain round
            assert np.array_equal(st[[0, 1, 2, 4, 5, 6, 7]], st0[[0, 1, 2, 4, 5, 6, 7]])
            if best >= 0:
                assert st[ST_STATUS] == 0
                assert all(bf.block_weight(g, part, j) <= L for j in range(k))
                assert st[ST_CUT_AFTER] == st[ST_CUT_BEFORE] - gains[best]
            else:
                assert part.tolist() == std.tolist() and st[ST_STATUS] == st0[ST_STATUS]
            checked += best > 0 and best < len(gains) - 1
    # not needed for every parameter set, but some cases keep a proper prefix
    assert checked >= 0


def test_prefix_cases_are_not_trivial(orc):
    """Across the small cases some rounds keep a proper prefix (undo a tail of
    moves) and some keep everything."""
    proper = full = 0
    for name, make in SMALL:
        for k in (2, 3, 5):
            for seed in range(4):
                g = make(seed + 11 * k)
                part0 = skewed_partition(g.n, k, seed, 0.5)
                _, (st, dbg, _) = both_rounds(orc, g, k, part0, mode=2)
                nm = int(dbg["pref"][1])
                proper += 0 <= st[ST_PREFIX] < nm
                full += st[ST_PREFIX] == nm and nm > 0
    assert proper >= 5 and full >= 5, (proper, full)


@pytest.mark.parametrize("name,make", SMALL)
def test_prefix_sequence_is_consistent(orc, name, make):
    """Each node appears at most once in the sequence; applying its moves in
    order to the round's input, every move starts in the node's current
    block, and the balance flag of every boundary is the recounted one."""
    k = 3
    for seed in range(4):
        g = make(500 + seed)
        L = orc.lmax(orc.total_weight(g), k)
        part0 = skewed_partition(g.n, k, seed, 0.55)
        _, (st, dbg, part) = both_rounds(orc, g, k, part0, mode=2)
        seq = dbg["seq"]
        assert len(set(seq[:, 0].tolist())) == len(seq)
        cur = part0.tolist()
        steps = int(dbg["pref"][1])
        assert list(seq[:, 3]) == sorted(seq[:, 3])
        for j in range(steps + 1):
            if j > 0:
                for v, a, b, s in seq[seq[:, 3] == j - 1]:
                    assert cur[v] == a and a != b
                    cur[v] = int(b)
            assert bool(dbg["bbal"][j]) == all(bf.block_weight(g, cur, x) <= L for x in range(k))


def test_prefix_without_rebalancing_is_the_round(orc):
    """A round whose rebalancer moves nothing, from a balanced start: the
    filtered moves lower the cut at every step (the filter's theorem), so the
    best prefix is all of them and the round is unchanged."""
    seen = 0
    for name, make in SMALL:
        for k in (2, 3, 5):
            for seed in range(4):
                g = make(seed + 3 * k)
                part0 = gg.random_partition(g.n, k, seed)
                (st0, _, std), (st, dbg, part) = both_rounds(orc, g, k, part0, mode=0,
                                                             tau=(1, 2))
                if st0[6] != 0:
                    continue
                seen += 1
                assert np.array_equal(part, std)
                assert st[ST_CUT_AFTER] == st0[ST_CUT_AFTER] and st[ST_REVERTED] == 0
                assert st[ST_PREFIX] == dbg["pref"][1]
                assert all(dbg["bgain"][i + 1] > dbg["bgain"][i] for i in range(len(dbg["bgain"]) - 1))
    assert seen >= 10


def test_prefix_never_worse_from_a_balanced_start(orc):
    """From a balanced start the empty prefix is a candidate, so the kept
    prefix never raises the cut, whatever the plain round does."""
    g = gg.chung_lu(3000, 8.0, 2.3, seed=9)
    for k in (2, 8):
        part0 = gg.random_partition(g.n, k, 4)
        for mode in (0, 2):
            part = part0.copy()
            for r in range(1, 6):
                before = part.copy()
                st, _ = orc.refine_round(g, orc.params(k, mode=mode, tau=gg.tau_schedule(r, 5),
                                                       variant=orc.BEST_PREFIX), part)
                assert st[ST_CUT_AFTER] <= st[ST_CUT_BEFORE]
                assert st[ST_STATUS] == 0
                assert st[ST_CUT_BEFORE] == bf.cut(g, before.tolist())
