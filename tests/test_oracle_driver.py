"""Pins of the oracle's refinement driver (Sections 5.5 and 6): the active
sets against their definitions, the rollback rule, the order of the round
kinds and the switching thresholds, read back from the per-round stats."""
from fractions import Fraction

import numpy as np
import pytest

from oracle import driver as D
from paper_2308_15494_amd import graphgen as gg
from tests.test_oracle_round import skewed_partition


def np_boundary(g, part):
    src = np.repeat(np.arange(g.n), np.diff(g.xadj))
    diff = part[src] != part[g.adjncy]
    out = np.zeros(g.n, np.uint8)
    np.maximum.at(out, src[diff], 1)
    return out


def np_next_active(g, before, after):
    moved = before != after
    src = np.repeat(np.arange(g.n), np.diff(g.xadj))
    hit = moved[g.adjncy]
    out = np.zeros(g.n, np.uint8)
    np.maximum.at(out, src[hit], 1)
    out[moved] = 0
    return out


@pytest.mark.parametrize("seed", range(4))
def test_active_sets(seed):
    g = gg.chung_lu(400, 6.0, 2.3, seed=seed)
    a = gg.random_partition(g.n, 4, seed)
    b = a.copy()
    rng = np.random.default_rng(seed)
    idx = rng.choice(g.n, 30, replace=False)
    b[idx] = (b[idx] + 1) % 4
    assert np.array_equal(D.boundary(g, a), np_boundary(g, a))
    assert np.array_equal(D.next_active(g, a, b), np_next_active(g, a, b))
    assert not D.next_active(g, a, a).any()


def test_tau_linear():
    assert D.tau_linear(1, 9, (1, 2)) == (1, 2)
    assert D.tau_linear(9, 9, (1, 2)) == (1, 1)
    assert Fraction(*D.tau_linear(5, 9, (1, 2))) == Fraction(3, 4)
    assert D.tau_linear(1, 1, (1, 2)) == (1, 2)


@pytest.mark.parametrize("case", [("cl", 8), ("rgg", 16), ("rmat", 8)])
def test_driver_rules(orc, case):
    name, k = case
    g = {"cl": lambda: gg.chung_lu(3000, 8.0, 2.3, seed=5),
         "rgg": lambda: gg.rgg2d(3000, seed=6),
         "rmat": lambda: gg.rmat(11, 16, seed=7)}[name]()
    for start in (gg.random_partition(g.n, k, 1), skewed_partition(g.n, k, 2, 0.3)):
        part = start.copy()
        log = D.refine(g, k, part)
        kinds = [x[1] for x in log]
        lp = [x for x in log if x[0] == "lp"]
        fm = [x for x in log if x[0] == "fm"]
        # LP: at most 5 rounds plus a rollback, which ends the phase
        assert len([x for x in lp if x[1] == "lp"]) <= 5
        for i, (_, kind, st) in enumerate(lp):
            if kind == "lp" and st[3] >= st[1]:
                assert i + 1 < len(lp) and lp[i + 1][1] == "rollback"
        if lp and lp[-1][1] == "rollback":
            assert np.array_equal(lp[-1][2], lp[-2][2])
        # FM: unconstrained rounds, then constrained ones; the last is
        # constrained; a switch happens only after a small improvement
        fk = [x[1] for x in fm]
        assert fk and fk[-1] == "constrained"
        first_c = fk.index("constrained")
        assert all(x == "unconstrained" for x in fk[:first_c])
        assert all(x == "constrained" for x in fk[first_c:])
        def small(st):
            return Fraction(int(st[1] - st[3])) < Fraction(2, 1000) * max(int(st[1]), 1)
        for i in range(first_c):
            # an unconstrained round is followed by another one unless it was
            # small or the next round is the budget's last
            if i < first_c - 1:
                assert not small(fm[i][2])
            else:
                assert small(fm[i][2]) or first_c == 9
        # constrained rounds stop at the first small one
        for i in range(first_c, len(fk) - 1):
            assert not small(fm[i][2])
        assert len(fm) == 10 or small(fm[-1][2])
        # the final partition is the last round's and is balanced
        assert int(fm[-1][2][8]) == 0
        assert int(orc.cut_edges(g, part)) == int(fm[-1][2][3])
