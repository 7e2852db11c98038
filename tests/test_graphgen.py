"""Input generators: CSR invariants, determinism, workload shapes."""
import numpy as np
import pytest

from paper_2308_15494_amd import graphgen as gg


def check_csr(g):
    n = g.n
    assert g.xadj.dtype == np.int64 and g.adjncy.dtype == np.int32
    assert g.xadj[0] == 0 and np.all(np.diff(g.xadj) >= 0)
    assert g.xadj[-1] == g.adjncy.size
    src = np.repeat(np.arange(n), np.diff(g.xadj))
    dst = g.adjncy.astype(np.int64)
    assert np.all((dst >= 0) & (dst < n))
    assert not np.any(src == dst), "self-loop"
    # rows strictly increasing -> no duplicates
    same_row = src[1:] == src[:-1]
    assert np.all(dst[1:][same_row] > dst[:-1][same_row])
    # symmetric, with symmetric weights
    fwd = src * n + dst
    rev = dst * n + src
    order_f = np.argsort(fwd)
    order_r = np.argsort(rev)
    assert np.array_equal(fwd[order_f], rev[order_r])
    if g.adjwgt is not None:
        assert np.all(g.adjwgt > 0)
        assert np.array_equal(g.adjwgt[order_f], g.adjwgt[order_r])
    if g.vwgt is not None:
        assert np.all(g.vwgt > 0)


@pytest.mark.parametrize("make", [
    lambda: gg.chung_lu(3000, 10.0, 2.5, seed=5),
    lambda: gg.chung_lu(2000, 8.0, 2.1, seed=6, wmax=16),
    lambda: gg.rmat(12, 8, seed=7),
    lambda: gg.grid2d(17, 23),
    lambda: gg.rgg2d(3000, seed=8),
    lambda: gg.random_small(40, 0.2, seed=9, wmax=5, vmax=3),
    lambda: gg.with_weights(gg.rmat(10, 8, seed=1), seed=2, wmax=9, vmax=4),
])
def test_csr_invariants(make):
    check_csr(make())


def test_determinism():
    a = gg.rmat(12, 8, seed=11)
    b = gg.rmat(12, 8, seed=11)
    c = gg.rmat(12, 8, seed=12)
    assert np.array_equal(a.xadj, b.xadj) and np.array_equal(a.adjncy, b.adjncy)
    assert not (a.xadj.size == c.xadj.size and np.array_equal(a.adjncy, c.adjncy))
    p1 = gg.random_partition(1000, 7, 3)
    p2 = gg.random_partition(1000, 7, 3)
    assert np.array_equal(p1, p2)


def test_random_partition_balanced():
    for n, k in [(10, 3), (1000, 8), (12345, 64), (5, 8)]:
        p = gg.random_partition(n, k, 1)
        cnt = np.bincount(p, minlength=k)
        assert cnt.max() - cnt.min() <= 1
        assert p.dtype == np.int32 and p.min() >= 0 and p.max() < k


def test_grid_counts():
    g = gg.grid2d(2048, 2048)
    assert g.n == 4_194_304 and g.m == 8_384_512


def test_chunglu10k_shape():
    g, k, eps, rounds, seed = gg.workload("chunglu10k")
    assert g.n == 10_000 and k == 8 and eps == (3, 100) and rounds == 10
    # 50,000 endpoint pairs minus self-loops and duplicates
    assert 45_000 < g.m <= 50_000
    # power law: irregular by the paper's std/mean degree statistic
    assert g.irregularity() > 1.0


def test_rgg_is_regular():
    g = gg.rgg2d(20000, seed=3)
    assert g.irregularity() < 0.6
    assert 6.0 < 2 * g.m / g.n < 8.5


def test_tau_schedule():
    from fractions import Fraction
    R = 10
    vals = [Fraction(*gg.tau_schedule(r, R)) for r in range(1, R + 1)]
    assert vals[0] == Fraction(1, 2) and vals[-1] == 1
    diffs = {vals[i + 1] - vals[i] for i in range(R - 1)}
    assert diffs == {Fraction(1, 18)}
    assert Fraction(*gg.tau_schedule(3, 20)) == Fraction(21, 38)
