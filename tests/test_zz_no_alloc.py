"""The no-allocation edge cut (upr_edge_cut_noalloc, scratch in a static
device array) against upr_edge_cut, which allocates its workspace in the
context: two calls in a row on one context, the second on a smaller graph
(the scratch keeps the first call's partial sums), plus weighted and
edgeless graphs and the size limit. Results are integers: equal exactly,
and equal to the oracle's cut."""
import numpy as np
import pytest

from oracle import oracle as O
from paper_2308_15494_amd import graphgen as gg

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def upr():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2308_15494_amd import upr as U
    U.lib()
    return U


def both_cuts(upr, ctx, g, k, seed):
    import torch
    part = gg.random_partition(g.n, k, seed)
    dg = upr.DeviceGraph(g)
    plan = upr.Plan(ctx, dg)
    dpart = torch.from_numpy(part).to("cuda")
    ref = upr.edge_cut(ctx, plan, dpart)
    out = torch.full((1,), -7, dtype=torch.int64, device="cuda")
    upr.edge_cut_noalloc(ctx, dg, dpart, out)
    torch.cuda.synchronize()
    plan.close()
    return int(out.item()), int(ref.item()), O.cut_edges(g, part)


def test_noalloc_cut_matches_edge_cut(upr):
    ctx = upr.Context(0)
    try:
        # first a larger graph (1025 tiles of 1024 nodes, a ragged last tile,
        # hubs), then a smaller one: the second call reads only its own tiles
        big = gg.rmat(20, 16, seed=20)
        small = gg.chung_lu(3001, 8.0, 2.3, seed=5)
        for name, g, k in [("big", big, 64), ("small", small, 8)]:
            got, ref, orc = both_cuts(upr, ctx, g, k, 2)
            print(f"noalloc cut {name} n={g.n}: {got} {ref} {orc}", flush=True)
            assert got == ref == orc, name
        for name, g, k in [("weighted", gg.chung_lu(5000, 12.0, 2.1, seed=4, wmax=16), 64),
                           ("ragged", gg.grid2d(33, 65), 4),
                           ("edgeless", gg.random_small(50, 0.0, seed=1), 2),
                           ("one_node", gg.random_small(1, 0.0, seed=1), 2)]:
            got, ref, orc = both_cuts(upr, ctx, g, k, 3)
            assert got == ref == orc, name
    finally:
        ctx.close()


def test_noalloc_cut_rejects_oversize(upr):
    """n above the scratch capacity is refused before anything is enqueued
    (the pointers are never read)."""
    import ctypes as C
    import torch
    ctx = upr.Context(0)
    try:
        out = torch.full((1,), -7, dtype=torch.int64, device="cuda")
        fake = upr._Graph(upr.NOALLOC_MAX_NODES + 1, out.data_ptr(), out.data_ptr(), None, None)
        rc = upr.lib().upr_edge_cut_noalloc(ctx.handle, C.byref(fake), C.c_void_p(out.data_ptr()),
                                           C.c_void_p(out.data_ptr()), upr._stream(None))
        assert rc == -1
        assert b"no-allocation" in upr.lib().upr_last_error(ctx.handle)
        torch.cuda.synchronize()
        assert int(out.item()) == -7
    finally:
        ctx.close()
