"""GPU: a schedule of rounds in one call (upr_refine_rounds) against the
oracle round by round (statistics, partition, block weights, table at the
end) and against one call per round; its argument checks."""
import numpy as np
import pytest

from oracle import oracle as O
from paper_2308_15494_amd import graphgen as gg
from tests.test_gpu_parity import ctx, say, skewed_partition, to_dev, upr  # noqa: F401

pytestmark = pytest.mark.gpu


def _state(upr, g, k, part0):
    import torch
    dg = upr.DeviceGraph(g)
    return dict(dg=dg, part=to_dev(part0.astype(np.int32)),
                conn=torch.zeros(max(g.n * k, 1), dtype=torch.int32, device="cuda"),
                W=torch.zeros(k, dtype=torch.int64, device="cuda"))


@pytest.mark.parametrize("case", [
    ("cl", lambda: gg.chung_lu(6000, 8.0, 2.3, seed=5), 16, 1),
    ("cl_w", lambda: gg.chung_lu(4000, 10.0, 2.2, seed=6, wmax=9), 8, 1),
    ("rmat", lambda: gg.rmat(12, 16, seed=7), 64, 1),
    ("grid_resident", lambda: gg.grid2d(50, 60), 32, 0),
], ids=lambda c: c[0])
def test_rounds_match_oracle_and_single_calls(upr, ctx, case):
    name, make, k, rebuild = case
    g = make()
    R = 6
    part0 = skewed_partition(g.n, k, 3, 0.35)
    ps = [upr.params(k, tau=gg.tau_schedule(r, R), mode=r % 3,
                     rebuild_table=1 if (rebuild or r == 1) else 0) for r in range(1, R + 1)]
    say(f"rounds {name} n={g.n} k={k} rounds={R}")
    # one call for all rounds
    a = _state(upr, g, k, part0)
    plan_a = upr.Plan(ctx, a["dg"])
    st_a = upr.refine_rounds(ctx, plan_a, ps, a["part"], a["conn"], a["W"]).cpu().numpy()
    # one call per round
    b = _state(upr, g, k, part0)
    plan_b = upr.Plan(ctx, b["dg"])
    st_b = []
    for p in ps:
        st_b.append(upr.refine_round(ctx, plan_b, p, b["part"], b["conn"], b["W"]).cpu().numpy())
    assert np.array_equal(st_a, np.stack(st_b))
    for key in ("part", "conn", "W"):
        assert np.array_equal(a[key].cpu().numpy(), b[key].cpu().numpy()), key
    # the oracle, round by round
    G = O.Graph(g)
    opart = part0.astype(np.int32).copy()
    oconn = np.zeros(max(g.n * k, 1), np.int32)
    oW = np.zeros(k, np.int64)
    for r in range(1, R + 1):
        ost, _ = O.refine_round(G, O.params(k, tau=gg.tau_schedule(r, R), mode=r % 3,
                                            rebuild_table=1 if (rebuild or r == 1) else 0),
                                opart, oconn, oW)
        assert np.array_equal(st_a[r - 1][:len(ost)], ost), f"round {r}"
    assert np.array_equal(a["part"].cpu().numpy(), opart)
    assert np.array_equal(a["W"].cpu().numpy(), oW)
    assert np.array_equal(a["conn"].cpu().numpy(), oconn)
    plan_a.close()
    plan_b.close()


def test_rounds_arguments_and_partial_failure(upr, ctx):
    import torch
    g = gg.chung_lu(3000, 8.0, 2.3, seed=8)
    k = 8
    part0 = gg.random_partition(g.n, k, 1)
    s = _state(upr, g, k, part0)
    plan = upr.Plan(ctx, s["dg"])
    L = upr.lib()
    # zero rounds: nothing happens
    before = s["part"].clone()
    assert L.upr_refine_rounds(ctx.handle, plan.handle, None, 0, upr._ptr(s["part"]),
                               upr._ptr(s["conn"]), upr._ptr(s["W"]), None, upr._stream(None)) == 0
    torch.cuda.synchronize()
    assert torch.equal(before, s["part"])
    # a negative count is an argument error
    rc = L.upr_refine_rounds(ctx.handle, plan.handle, None, -1, upr._ptr(s["part"]),
                             upr._ptr(s["conn"]), upr._ptr(s["W"]), None, upr._stream(None))
    assert rc == -1  # UPR_E_ARG
    # round 2 of 3 has k outside the range: round 1 stands, the call fails there
    good = upr.params(k, tau=(1, 2))
    bad = upr.params(1, tau=(1, 2))
    stats = torch.full((3, upr.STATS_LEN), -7, dtype=torch.int64, device="cuda")
    with pytest.raises(upr.UprError):
        upr.refine_rounds(ctx, plan, [good, bad, good], s["part"], s["conn"], s["W"], stats)
    st = stats.cpu().numpy()
    assert (st[1:] == -7).all()  # rounds 2 and 3 wrote nothing
    G = O.Graph(g)
    opart = part0.astype(np.int32).copy()
    oconn = np.zeros(g.n * k, np.int32)
    oW = np.zeros(k, np.int64)
    ost, _ = O.refine_round(G, O.params(k, tau=(1, 2)), opart, oconn, oW)
    assert np.array_equal(st[0][:len(ost)], ost)  # round 1 ran and stands
    assert np.array_equal(s["part"].cpu().numpy(), opart)
    plan.close()
