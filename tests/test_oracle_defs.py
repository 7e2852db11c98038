"""Pins of the oracle's definitional pieces against Section 2 and Section 5.3.

Each check compares the oracle with an independent computation: exact
rationals, edge-list brute force, or identities that follow from the
definitions.
"""
import math
from fractions import Fraction

import numpy as np
import pytest

from paper_2308_15494_amd import graphgen as gg
from tests import bruteforce as bf


# ---------------------------------------------------------------- L_max --

@pytest.mark.parametrize("total,k,eps,expected", [
    (10_000, 8, (3, 100), 1287),          # Chung-Lu 10k, k=8
    (1_048_576, 64, (3, 100), 16875),     # R-MAT scale 20, k=64
    (4_194_304, 64, (3, 100), 67502),     # 2048^2 grid, k=64
    (8_000_000, 256, (3, 100), 32187),    # Chung-Lu 8M, k=256
    (10, 2, (3, 100), 5),                 # eps * ceil(C/k) < 1: no slack at all
    (101, 4, (1, 10), 28),                # ceil(101/4) = 26 -> 28.6
])
def test_lmax_values(orc, total, k, eps, expected):
    assert orc.lmax(total, k, eps) == expected
    assert bf.lmax_exact(total, k, eps) == expected


def test_lmax_random(orc):
    rng = np.random.default_rng(0)
    for _ in range(2000):
        total = int(rng.integers(0, 1 << 40))
        k = int(rng.integers(2, 70000))
        eps = (int(rng.integers(1, 1000)), int(rng.integers(1, 1000)))
        assert orc.lmax(total, k, eps) == bf.lmax_exact(total, k, eps)


# ----------------------------------------------------------------- slots --

@pytest.mark.parametrize("w,c,expected", [
    (0, 1, 0), (1, 1, 0), (1, 5, 0),       # ratio <= 1: slot 0
    (3, 2, 1),                             # exactly 3/2
    (2, 1, 2),                             # 1.5 < 2 <= 2.25
    (9, 4, 2), (10, 4, 3),                 # 9/4 = 1.5^2 exactly; just above
    (27, 8, 3), (28, 8, 4),                # 1.5^3 exactly; just above
    (81, 16, 4),
    (2**31 - 1, 1, 53),                    # largest int32 ratio fits slot 53
])
def test_slot_values(orc, w, c, expected):
    assert orc.slot(w, c) == expected
    assert bf.slot_exact(w, c) == expected


def test_slot_random(orc):
    rng = np.random.default_rng(1)
    for _ in range(3000):
        c = int(rng.integers(1, 1 << int(rng.integers(1, 31))))
        w = int(rng.integers(0, 1 << int(rng.integers(1, 31))))
        s = orc.slot(w, c)
        assert s == bf.slot_exact(w, c)
        # ceil(log_{3/2}(w/c)) away from exact powers
        if w > c:
            x = math.log(w / c) / math.log(1.5)
            if abs(x - round(x)) > 1e-9:
                assert s == min(53, math.ceil(x))


# ------------------------------------------------------------- penalties --

@pytest.mark.parametrize("tau", [(0, 1), (1, 2), (9, 18), (13, 18), (1, 1), (19, 38), (7, 9)])
def test_penq_exact(orc, tau):
    q = orc.penq(tau)
    for l in range(54):
        exact = Fraction(*tau) * Fraction(3, 2) ** l * 65536
        assert q[l] == math.floor(exact)
    if tau[0] == tau[1]:
        assert q[0] == 65536 and q[1] == 98304 and q[2] == 147456


def test_penq_monotone_in_tau(orc):
    prev = orc.penq((0, 1))
    assert not prev.any()
    for r in range(1, 11):
        cur = orc.penq(gg.tau_schedule(r, 10))
        assert np.all(cur >= prev)
        prev = cur


# ----------------------------------------------------- gain table and cut --

GRAPHS = [
    lambda: gg.random_small(25, 0.2, seed=1),
    lambda: gg.random_small(30, 0.15, seed=2, wmax=7, vmax=4),
    lambda: gg.chung_lu(200, 6.0, 2.3, seed=3),
    lambda: gg.grid2d(7, 9),
    lambda: gg.with_weights(gg.rmat(7, 4, seed=4), seed=5, wmax=11, vmax=3),
]


@pytest.mark.parametrize("make", GRAPHS)
@pytest.mark.parametrize("k", [2, 3, 8])
def test_gain_table_bruteforce(orc, make, k):
    g = make()
    part = gg.random_partition(g.n, k, seed=k)
    conn = orc.gain_table(g, k, part)
    for v in range(g.n):
        for j in range(k):
            assert conn[v, j] == bf.omega(g, v, j, part)
    # row sums are the weighted degrees
    assert all(conn[v].sum() == bf.wdeg(g, v) for v in range(g.n))


@pytest.mark.parametrize("make", GRAPHS)
@pytest.mark.parametrize("k", [2, 5])
def test_cut_and_weights(orc, make, k):
    g = make()
    rng = np.random.default_rng(k)
    part = rng.integers(0, k, size=g.n).astype(np.int32)
    c = bf.cut(g, part)
    assert orc.cut_edges(g, part) == c
    conn = orc.gain_table(g, k, part)
    assert orc.cut_table(g, k, part, conn) == c
    W = orc.block_weights(g, k, part)
    for j in range(k):
        assert W[j] == bf.block_weight(g, part, j)
    assert W.sum() == orc.total_weight(g)


def test_cut_extremes(orc):
    g = gg.random_small(20, 0.3, seed=7, wmax=4)
    assert orc.cut_edges(g, np.zeros(g.n, np.int32)) == 0
    alt = np.arange(g.n, dtype=np.int32)  # every node its own block: all edges cut
    total = sum(w for _, _, w in bf.edges(g))
    assert orc.cut_edges(g, alt) == total


# ------------------------------------------------------ penalty buckets --

@pytest.mark.parametrize("make", GRAPHS)
@pytest.mark.parametrize("t", [(7, 10), (2, 5), (1, 1), (0, 1)])
def test_penalty_buckets_sets(orc, make, t):
    g = make()
    k = 3
    part = gg.random_partition(g.n, k, seed=3)
    conn = orc.gain_table(g, k, part)
    bucket, avail = orc.penalty_buckets(g, k, part, conn, t)
    B = bf.available_sets(g, k, part, t)
    for j in range(k):
        for l in range(54):
            assert bucket[j, l] == sum(bf.node_w(g, u) for u in B[j][l])
    members = {u for j in range(k) for l in range(54) for u in B[j][l]}
    assert set(np.nonzero(avail)[0].tolist()) == members
    if t == (0, 1):
        assert avail.all()  # t = 0: every node is available


def test_lemma1_inequality_per_node(orc):
    """Lemma 1's chain for one rebalancing node b of block V_1:
    omega(I(b)) <= (1/t) omega(b, V_1) <= (1/t) (3/2)^slot(b) c(b)."""
    for seed in range(6):
        g = gg.with_weights(gg.chung_lu(300, 6.0, 2.4, seed=seed), seed=seed, wmax=5, vmax=3)
        k = 4
        part = gg.random_partition(g.n, k, seed)
        conn = orc.gain_table(g, k, part)
        for t in [(7, 10), (2, 5), (1, 1)]:
            _, avail = orc.penalty_buckets(g, k, part, conn, t)
            for b in np.nonzero(avail)[0]:
                s = int(avail[b]) - 1
                inner = int(conn[b, part[b]])
                deg = bf.wdeg(g, int(b))
                assert Fraction(*t) * deg <= inner
                assert inner <= Fraction(3, 2) ** s * bf.node_w(g, int(b))
