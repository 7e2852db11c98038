"""Seeded synthetic graph and partition generators.

This module produces the *inputs* of a refinement round: an undirected graph
G = (V, E, c, omega) with positive integer node weights c and edge weights
omega (Section 2, Preliminaries), stored as a symmetric CSR, and an initial
k-way partition. It holds none of the refinement arithmetic; both the CPU
oracle and the HIP path consume what it produces.

The paper evaluates on real graphs (Section 8.1, Table 1) split by the ratio of
the standard deviation to the mean of the node degree: irregular graphs
(social, web, power-law generators) and regular graphs (meshes, road networks,
geometric graphs). Those datasets are stood in for by seeded generators with
the same structure classes:

* Chung-Lu expected-degree graphs with a power-law weight sequence
  (irregular, like the paper's artificial power-law instances),
* R-MAT (Chakrabarti, Zhan, Faloutsos 2004) with a seeded id permutation,
* 2D 4-neighbour grids and 2D random geometric graphs (regular).

CSR layout (all host numpy arrays):
    xadj   int64[n+1], xadj[0] = 0, nondecreasing
    adjncy int32[nnz], rows sorted ascending, symmetric, no self-loops,
           no duplicates
    adjwgt int32[nnz] or None (None = every edge weight 1)
    vwgt   int32[n]   or None (None = every node weight 1)
"""
from __future__ import annotations

import dataclasses
import math
import os
from concurrent.futures import ThreadPoolExecutor

import numpy as np


@dataclasses.dataclass
class Graph:
    n: int
    xadj: np.ndarray
    adjncy: np.ndarray
    adjwgt: np.ndarray | None = None
    vwgt: np.ndarray | None = None
    name: str = ""
    meta: dict = dataclasses.field(default_factory=dict)

    @property
    def nnz(self) -> int:
        return int(self.xadj[-1])

    @property
    def m(self) -> int:
        """Number of undirected edges."""
        return self.nnz // 2

    def degrees(self) -> np.ndarray:
        return np.diff(self.xadj)

    def irregularity(self) -> float:
        """Standard deviation over mean of the node degree (Section 8.1)."""
        d = self.degrees().astype(np.float64)
        mu = d.mean() if d.size else 0.0
        return float(d.std() / mu) if mu > 0 else 0.0

    def total_node_weight(self) -> int:
        return int(self.n if self.vwgt is None else int(self.vwgt.astype(np.int64).sum()))


def _workers() -> int:
    return max(1, min(16, os.cpu_count() or 1))


def _threaded(fn, arr, out_dtype, chunk=1 << 22):
    """fn applied to consecutive chunks of arr on a thread pool (numpy's
    searching and sorting routines release the GIL), concatenated."""
    if arr.size <= chunk or _workers() == 1:
        return fn(arr).astype(out_dtype, copy=False)
    out = np.empty(arr.size, dtype=out_dtype)

    def run(i):
        out[i:i + chunk] = fn(arr[i:i + chunk])

    with ThreadPoolExecutor(_workers()) as ex:
        list(ex.map(run, range(0, arr.size, chunk)))
    return out


def _argsort(key: np.ndarray) -> np.ndarray:
    """An ordering of key by value (equal keys in any order). Large inputs
    are split by value into buckets at sampled splitters, and the buckets
    are sorted on a thread pool."""
    if key.size < (1 << 23) or _workers() == 1:
        return np.argsort(key, kind="stable")
    nb = 4 * _workers()
    sample = np.sort(key[:: max(key.size // 65536, 1)])
    spl = sample[np.linspace(0, sample.size - 1, nb + 1)[1:-1].astype(np.int64)]
    bucket = _threaded(lambda x: np.searchsorted(spl, x, side="right"), key, np.int16)
    counts = np.bincount(bucket, minlength=nb)
    by_bucket = np.argsort(bucket, kind="stable")
    del bucket
    starts = np.concatenate([[0], np.cumsum(counts)])
    out = np.empty(key.size, dtype=np.int64)

    def run(b):
        idx = by_bucket[starts[b]:starts[b + 1]]
        out[starts[b]:starts[b + 1]] = idx[np.argsort(key[idx], kind="stable")]

    with ThreadPoolExecutor(_workers()) as ex:
        list(ex.map(run, range(nb)))
    return out


def searchsorted_right(cdf: np.ndarray, x: np.ndarray) -> np.ndarray:
    """np.searchsorted(cdf, x, side="right"), on a thread pool for large x."""
    return _threaded(lambda c: np.searchsorted(cdf, c, side="right"), x, np.int64)


def csr_from_undirected(n: int, u: np.ndarray, v: np.ndarray,
                        w: np.ndarray | None = None) -> tuple:
    """Symmetric CSR from undirected pairs.

    Self-loops are dropped; duplicate pairs (in either orientation) are merged,
    keeping the weight of the first occurrence. Rows come out sorted: row x
    lists its smaller neighbours, then its larger ones, each ascending.
    """
    u = np.asarray(u, dtype=np.int64)
    v = np.asarray(v, dtype=np.int64)
    keep = u != v
    u, v = u[keep], v[keep]
    if w is not None:
        w = np.asarray(w)[keep]
    key = np.minimum(u, v) * n + np.maximum(u, v)
    del u, v, keep
    if w is None:
        key = np.unique(key)
    else:
        # sorted distinct keys, each with the weight of its first draw
        order = _argsort(key)
        ks = key[order]
        first = np.ones(ks.size, dtype=bool)
        first[1:] = ks[1:] != ks[:-1]
        starts = np.flatnonzero(first)
        key = ks[starts]
        del ks, first
        if starts.size:
            w = w[np.minimum.reduceat(order, starts)].astype(np.int32)
        else:
            w = w[:0].astype(np.int32)
        del order, starts
    lo = key // n
    hi = key - lo * n
    del key
    below = np.bincount(hi, minlength=n) if n > 0 else np.zeros(0, np.int64)
    above = np.bincount(lo, minlength=n) if n > 0 else np.zeros(0, np.int64)
    xadj = np.zeros(n + 1, dtype=np.int64)
    np.cumsum(below + above, out=xadj[1:])
    nnz = int(xadj[-1])
    adjncy = np.empty(nnz, dtype=np.int32)
    adjwgt = None if w is None else np.empty(nnz, dtype=np.int32)
    m = lo.size
    rank = np.arange(m, dtype=np.int64)
    # larger neighbours: the pairs are sorted by (lo, hi) already
    first_above = np.cumsum(above) - above
    pos = xadj[lo] + below[lo] + (rank - first_above[lo])
    adjncy[pos] = hi
    if w is not None:
        adjwgt[pos] = w
    # smaller neighbours: the pairs sorted by (hi, lo)
    if w is None:
        kb = np.sort(hi * n + lo)
        row = kb // n
        col = kb - row * n
        wb = None
    else:
        ob = _argsort(hi * n + lo)
        row, col, wb = hi[ob], lo[ob], w[ob]
        del ob
    first_below = np.cumsum(below) - below
    pos = xadj[row] + (rank - first_below[row])
    adjncy[pos] = col
    if wb is not None:
        adjwgt[pos] = wb
    return xadj, adjncy, adjwgt


def _finish(g: Graph) -> Graph:
    d = g.degrees()
    g.meta.setdefault("n", g.n)
    g.meta["m"] = g.m
    g.meta["nnz"] = g.nnz
    g.meta["max_degree"] = int(d.max()) if d.size else 0
    g.meta["irregularity"] = g.irregularity()
    return g


def _chung_lu_weights(n: int, avg_deg: float, beta: float, d_max: float) -> np.ndarray:
    """Power-law weight sequence w_i = d_max * (i0 / (i + i0))^(1/(beta-1)).

    i0 is found by bisection so that the mean weight equals avg_deg.
    """
    i = np.arange(n, dtype=np.float64)
    gamma = 1.0 / (beta - 1.0)
    buf = np.empty(n, dtype=np.float64)

    def fill(i0: float, lo: int, hi: int):
        buf[lo:hi] = d_max * (i0 / (i[lo:hi] + i0)) ** gamma

    def mean_for(i0: float) -> float:
        # the elementwise values on a thread pool, the mean over the whole array
        if n < (1 << 20) or _workers() == 1:
            fill(i0, 0, n)
        else:
            step = (n + _workers() - 1) // _workers()
            with ThreadPoolExecutor(_workers()) as ex:
                list(ex.map(lambda lo: fill(i0, lo, min(lo + step, n)), range(0, n, step)))
        return float(buf.mean())

    lo, hi = 1e-9, float(n) * 1e6
    for _ in range(200):
        mid = math.sqrt(lo * hi)
        if mean_for(mid) < avg_deg:
            lo = mid
        else:
            hi = mid
    i0 = math.sqrt(lo * hi)
    return d_max * (i0 / (i + i0)) ** gamma


def chung_lu(n: int, avg_deg: float, beta: float, seed: int, d_max: float | None = None,
             wmax: int = 0) -> Graph:
    """Chung-Lu expected-degree graph in edge-sampling form.

    floor(n*avg_deg/2) endpoint pairs are drawn with probability proportional
    to the weight sequence; self-loops and duplicates are dropped. With
    wmax > 0 every undirected edge gets a weight uniform in [1, wmax].
    """
    rng = np.random.default_rng(seed)
    if d_max is None:
        d_max = math.sqrt(n * avg_deg)
    w = _chung_lu_weights(n, avg_deg, beta, d_max)
    cdf = np.cumsum(w)
    cdf /= cdf[-1]
    pairs = int(n * avg_deg // 2)
    a = searchsorted_right(cdf, rng.random(pairs))
    b = searchsorted_right(cdf, rng.random(pairs))
    np.minimum(a, n - 1, out=a)
    np.minimum(b, n - 1, out=b)
    ew = rng.integers(1, wmax + 1, size=pairs, dtype=np.int32) if wmax > 0 else None
    xadj, adjncy, adjwgt = csr_from_undirected(n, a, b, ew)
    g = Graph(n, xadj, adjncy, adjwgt, None, name=f"chunglu_n{n}_d{avg_deg}_b{beta}_s{seed}")
    g.meta.update(dict(kind="chung_lu", avg_deg=avg_deg, beta=beta, seed=seed,
                       d_max=d_max, wmax=wmax, pairs=pairs))
    return _finish(g)


def rmat(scale: int, edge_factor: int, seed: int, a: float = 0.57, b: float = 0.19,
         c: float = 0.19, permute: bool = True) -> Graph:
    """R-MAT graph with 2^scale nodes and edge_factor * 2^scale draws.

    Each draw descends scale levels of the adjacency matrix choosing the
    quadrant with probabilities (a, b, c, d = 1 - a - b - c). Node ids are
    passed through a seeded permutation so that hubs are not clustered at
    small ids. Self-loops and duplicates are dropped.
    """
    rng = np.random.default_rng(seed)
    n = 1 << scale
    draws = edge_factor * n
    src = np.zeros(draws, dtype=np.int64)
    dst = np.zeros(draws, dtype=np.int64)
    ab = a + b
    abc = a + b + c
    for lvl in range(scale):
        r = rng.random(draws, dtype=np.float32)
        bit = np.int64(1) << (scale - 1 - lvl)
        row = r >= ab
        col = ((r >= a) & (r < ab)) | (r >= abc)
        src += row * bit
        dst += col * bit
    if permute:
        perm = rng.permutation(n).astype(np.int64)
        src = perm[src]
        dst = perm[dst]
    xadj, adjncy, _ = csr_from_undirected(n, src, dst)
    g = Graph(n, xadj, adjncy, None, None, name=f"rmat_s{scale}_ef{edge_factor}_s{seed}")
    g.meta.update(dict(kind="rmat", scale=scale, edge_factor=edge_factor, seed=seed,
                       abcd=(a, b, c, 1 - a - b - c), draws=draws))
    return _finish(g)


def grid2d(rows: int, cols: int) -> Graph:
    """4-neighbour grid, row-major ids."""
    n = rows * cols
    ids = np.arange(n, dtype=np.int64).reshape(rows, cols)
    hu = ids[:, :-1].ravel()
    hv = ids[:, 1:].ravel()
    vu = ids[:-1, :].ravel()
    vv = ids[1:, :].ravel()
    xadj, adjncy, _ = csr_from_undirected(n, np.concatenate([hu, vu]), np.concatenate([hv, vv]))
    g = Graph(n, xadj, adjncy, None, None, name=f"grid_{rows}x{cols}")
    g.meta.update(dict(kind="grid2d", rows=rows, cols=cols))
    return _finish(g)


def rgg2d(n: int, seed: int, avg_deg: float = 8.0) -> Graph:
    """2D random geometric graph in the unit square (no torus).

    Radius r = sqrt(avg_deg / (pi * n)); the realised average degree is
    slightly below avg_deg because of the boundary.
    """
    from scipy.spatial import cKDTree

    rng = np.random.default_rng(seed)
    pts = rng.random((n, 2))
    r = math.sqrt(avg_deg / (math.pi * n))
    pairs = cKDTree(pts).query_pairs(r, output_type="ndarray")
    xadj, adjncy, _ = csr_from_undirected(n, pairs[:, 0], pairs[:, 1])
    g = Graph(n, xadj, adjncy, None, None, name=f"rgg_n{n}_s{seed}")
    g.meta.update(dict(kind="rgg2d", seed=seed, radius=r, target_avg_deg=avg_deg))
    return _finish(g)


def random_small(n: int, p: float, seed: int, wmax: int = 0, vmax: int = 0) -> Graph:
    """Erdos-Renyi G(n, p) with optional uniform edge/node weights (for tests)."""
    rng = np.random.default_rng(seed)
    iu, ju = np.triu_indices(n, 1)
    keep = rng.random(iu.size) < p
    u, v = iu[keep], ju[keep]
    ew = rng.integers(1, wmax + 1, size=u.size, dtype=np.int32) if wmax > 0 else None
    xadj, adjncy, adjwgt = csr_from_undirected(n, u, v, ew)
    vw = rng.integers(1, vmax + 1, size=n, dtype=np.int32) if vmax > 0 else None
    g = Graph(n, xadj, adjncy, adjwgt, vw, name=f"er_n{n}_p{p}_s{seed}")
    g.meta.update(dict(kind="erdos_renyi", p=p, seed=seed, wmax=wmax, vmax=vmax))
    return _finish(g)


def random_partition(n: int, k: int, seed: int) -> np.ndarray:
    """Seeded uniform-random balanced assignment: part[perm[i]] = i mod k."""
    rng = np.random.default_rng(seed)
    perm = rng.permutation(n)
    part = np.empty(n, dtype=np.int32)
    part[perm] = (np.arange(n) % k).astype(np.int32)
    return part


def with_weights(g: Graph, seed: int, wmax: int = 0, vmax: int = 0) -> Graph:
    """Copy of g with uniform random edge weights in [1, wmax] (symmetric) and
    node weights in [1, vmax]; 0 keeps unit weights."""
    rng = np.random.default_rng(seed)
    adjwgt = g.adjwgt
    if wmax > 0:
        src = np.repeat(np.arange(g.n, dtype=np.int64), g.degrees())
        dst = g.adjncy.astype(np.int64)
        lo = np.minimum(src, dst)
        hi = np.maximum(src, dst)
        key = lo * g.n + hi
        uk, inv = np.unique(key, return_inverse=True)
        wu = rng.integers(1, wmax + 1, size=uk.size, dtype=np.int32)
        adjwgt = wu[inv].astype(np.int32)
    vwgt = g.vwgt
    if vmax > 0:
        vwgt = rng.integers(1, vmax + 1, size=g.n, dtype=np.int32)
    h = Graph(g.n, g.xadj, g.adjncy, adjwgt, vwgt, name=g.name + f"_w{wmax}_v{vmax}",
              meta=dict(g.meta))
    return _finish(h)


# ---------------------------------------------------------------------------
# Named workloads (sizes of the paper-style configurations)
# ---------------------------------------------------------------------------

def workload(name: str) -> tuple:
    """Return (graph, k, eps=(num, den), rounds, init_part_seed) for a named workload.

    chunglu10k  : Chung-Lu n=10,000, avg degree 10, exponent 2.5, seed 1; k=8
    rmat20      : R-MAT scale 20, 16 draws per node, seed 20; k=64
    grid2048    : 2048 x 2048 4-neighbour grid; k=64
    chunglu8m   : Chung-Lu n=8,000,000, avg degree 32, exponent 2.1,
                  d_max=2e5, edge weights in [1,16], seed 3; k=256
    """
    if name == "chunglu10k":
        return chung_lu(10_000, 10.0, 2.5, seed=1), 8, (3, 100), 10, 2
    if name == "rmat20":
        return rmat(20, 16, seed=20), 64, (3, 100), 20, 2
    if name == "grid2048":
        return grid2d(2048, 2048), 64, (3, 100), 20, 2
    if name == "chunglu8m":
        return chung_lu(8_000_000, 32.0, 2.1, seed=3, d_max=2e5, wmax=16), 256, (3, 100), 20, 2
    raise KeyError(name)


def batch_set(count: int = 512, seed0: int = 1000, n_min: int = 1000, n_max: int = 200_000):
    """The many-graphs workload: `count` graphs (seeds seed0 + i), sizes
    log-uniform in [n_min, n_max]; even i Chung-Lu (exponent uniform in
    [2.1, 2.8], mean degree uniform in [8, 24]), odd i 2D random geometric
    (mean degree 8); k drawn from {2, 4, 8, 16, 32, 64}; eps 3/100; 10
    rounds each. Returns a list of (graph, k, part0_seed)."""
    out = []
    ks = [2, 4, 8, 16, 32, 64]
    for i in range(count):
        rng = np.random.default_rng(seed0 + i)
        n = int(round(math.exp(rng.uniform(math.log(n_min), math.log(n_max)))))
        k = int(ks[rng.integers(0, len(ks))])
        if i % 2 == 0:
            beta = float(rng.uniform(2.1, 2.8))
            d = float(rng.uniform(8.0, 24.0))
            g = chung_lu(n, d, beta, seed=seed0 + i)
        else:
            g = rgg2d(n, seed=seed0 + i)
        out.append((g, k, seed0 + i))
    return out


def serve_set(count: int = 2000, seed0: int = 100_000, m_min: float = 1e4, m_max: float = 1e7):
    """The serving workload: `count` requests (seeds seed0 + j), edge counts
    log-uniform in [m_min, m_max]; Chung-Lu with n = m/8 (mean degree 16,
    exponent uniform in [2.1, 2.8]) or R-MAT with scale ceil(log2(m/16)) and
    16 draws per node, with equal probability; k drawn from {8, 32, 128};
    eps 3/100; 10 rounds. Returns a list of (graph, k, part0_seed)."""
    out = []
    for j in range(count):
        rng = np.random.default_rng(seed0 + j)
        m = math.exp(rng.uniform(math.log(m_min), math.log(m_max)))
        k = int([8, 32, 128][rng.integers(0, 3)])
        if rng.random() < 0.5:
            n = max(int(m / 8), 64)
            g = chung_lu(n, 16.0, float(rng.uniform(2.1, 2.8)), seed=seed0 + j)
        else:
            g = rmat(max(int(math.ceil(math.log2(max(m / 16, 16)))), 4), 16, seed=seed0 + j)
        out.append((g, k, seed0 + j))
    return out


def generate_parallel(fn, count: int, workers: int, **kw):
    """fn(count, ...) split over worker processes by index ranges (forked;
    call before any GPU use)."""
    import multiprocessing as mp
    if workers <= 1 or count < 2 * workers:
        return fn(count, **kw)
    seed_key = "seed0"
    seed0 = kw.pop(seed_key)
    chunks = [(i, min(i + (count + workers - 1) // workers, count))
              for i in range(0, count, (count + workers - 1) // workers)]
    ctx = mp.get_context("fork")
    pool = ctx.Pool(len(chunks))
    try:
        parts = pool.starmap(_gen_range, [(fn.__name__, a, b, seed0, kw) for a, b in chunks])
    except BaseException:
        pool.terminate()
        pool.join()
        raise
    # the workers exit on their own (no terminate, no signal)
    pool.close()
    pool.join()
    return [x for part in parts for x in part]


def _gen_range(name, a, b, seed0, kw):
    fn = globals()[name]
    return fn(b - a, seed0=seed0 + a, **kw)


def alpha_schedule(r: int, rounds: int) -> tuple:
    """Block-weight cap factor of round r (1-based) of the limited-imbalance
    variant, as a rational (num, den): linear from alpha_1 = 2 down to
    alpha_final = 1.1 (Section 8.2); a single round uses 1.1."""
    if rounds <= 1:
        return (11, 10)
    return (20 * (rounds - 1) - 9 * (r - 1), 10 * (rounds - 1))


def tau_schedule(r: int, rounds: int) -> tuple:
    """Penalty factor of round r (1-based) as a rational (num, den).

    The paper interpolates linearly from a small tau_1 to tau_final = 1
    (Section 5.5) without fixing tau_1; the value 1/2 is the one it uses
    elsewhere (dynamic activation, constant-penalty variant). So
    tau_r = 1/2 + (1/2)(r-1)/(R-1) = (R - 2 + r) / (2R - 2), clamped to r <= R.
    """
    if rounds <= 1:
        return (1, 1)
    r = max(1, min(r, rounds))
    num = rounds - 2 + r
    den = 2 * rounds - 2
    gcd = math.gcd(num, den)
    return (num // gcd, den // gcd)
