"""RRT-Connect local planner on the GPU against the oracle (oracle/rrtc.py):
per edge the same outcome (straight line, repaired by RRT-Connect, failed),
the same iteration count and tree sizes, repaired costs within 1e-5, local
paths equal waypoint for waypoint (sampling, nearest node and steering are
FP32 with one operation order on both sides), and the plan over the
repaired graph.  Excused and counted: edges whose straight-line check or an
endpoint lies within 1e-5 of contact, and calls with an extension segment
whose minimum signed distance does."""
import numpy as np
import pytest
import torch

import oracle
import oracle.rrtc as R
import workloads as wl
from tests import parity as P

pytestmark = pytest.mark.gpu

CASES = [("2d-small", 1, 32, 4, (50, 256, 1.0, 0.1, 1.5)),
         ("2d-large", 2, 64, 5, (100, 512, 0.8, 0.05, 1.4)),
         ("arm7", 1, 32, 3, (30, 256, 0.5, 0.1, 1.3)),
         ("arm7", 2, 48, 4, (100, 512, 0.4, 0.1, 1.5)),
         ("3d-point", 1, 40, 4, (60, 256, 1.5, 0.2, 1.5))]


def _say(*a):
    print("[case]", *a, flush=True)


def _flat(t):
    return np.concatenate([np.asarray(t[0]).ravel(), np.asarray(t[1]).ravel(), np.asarray(t[2]).ravel()])


def _run(gt, orc, name, scene, N, M, lp, seed=17, stage=0):
    w = wl.make_workload(name, scene, N=N, M=M)
    o = R.LPOpts(*lp)
    stats = torch.zeros(6, device="cuda", dtype=torch.int64)
    opts = gt.make_rrtc_opts(o.budget, o.cap, o.eta, o.res, o.ell_factor, stats)
    pl = gt.Planner(w, flags=True)
    pl.sample(w["seed"], 0)
    pl.check()
    pl.repair(opts, seed, stage)
    torch.cuda.synchronize()
    g_cost = _flat((pl.C_s.cpu().numpy(), pl.C_h.cpu().numpy()[: M - 1], pl.C_l.cpu().numpy())).astype(np.float64)
    g_flag = pl.flags.cpu().numpy().astype(np.int32)
    r = orc.plan(w)
    c0, f0, sd0 = _flat(r["cost"]), _flat(r["flag"]), _flat(r["minsd"])
    cost, flag, info = R.repair(w, r["Q"], c0, f0, o, seed, stage)
    excused = np.abs(sd0) <= P.BAND
    excused[info["vertex_band"]] = True
    excused[info["ids"][info["near_band"]]] = True
    return dict(w=w, o=o, opts=opts, pl=pl, stats=stats.cpu().numpy(), g_cost=g_cost, g_flag=g_flag, cost=cost,
                flag=flag, info=info, excused=excused, r=r)


@pytest.mark.parametrize("name,scene,N,M,lp", CASES)
def test_repair_matches_oracle(gt, orc, name, scene, N, M, lp):
    _say("rrtc repair", name, "scene", scene, "N", N, "M", M, "lp", lp)
    c = _run(gt, orc, name, scene, N, M, lp)
    ex = c["excused"]
    _say("candidates", len(c["info"]["ids"]), "repaired", int((c["flag"] == 2).sum()), "excused", int(ex.sum()),
         "gpu stats", c["stats"])
    bad = (c["g_flag"] != c["flag"]) & ~ex
    assert not bad.any(), (np.flatnonzero(bad)[:8], c["g_flag"][bad][:8], c["flag"][bad][:8])
    keep = ~ex
    np.testing.assert_allclose(c["g_cost"][keep], c["cost"][keep], rtol=P.REL)
    # counters: calls and successes over the non-excused candidates agree
    info = c["info"]
    assert c["stats"][0] == len(info["ids"]) or ex.any()
    assert c["stats"][1] == int(info["ok"].sum()) or ex.any()
    if not ex.any():
        assert c["stats"][2] == int(info["iters"].sum())
        assert c["stats"][3] == int(info["sizes"].sum())


@pytest.mark.parametrize("name,scene,N,M,lp", [CASES[0], CASES[2]])
def test_local_paths_equal_oracle_paths(gt, orc, name, scene, N, M, lp):
    c = _run(gt, orc, name, scene, N, M, lp)
    info, pl, w, o = c["info"], c["pl"], c["w"], c["o"]
    model = oracle.Model(w)
    ids = info["ids"][info["ok"] & ~info["near_band"]]
    picked = ids[:: max(1, len(ids) // 12)][:12]
    failed = info["ids"][~info["ok"] & ~info["near_band"]][:3]
    _say("local paths", name, "edges", list(picked), "failed", list(failed))
    for e in list(picked) + list(failed):
        e = int(e)
        path, cost = pl.local_path(e, c["opts"], 17, 0)
        x, y = R.edge_endpoints(w, c["r"]["Q"], e)
        want = R.call(model, w, x, y, o, 17, 0, e)
        if not want["ok"]:
            assert path.shape[0] == 0 and cost == np.inf
            continue
        got = path.cpu().numpy()
        assert np.array_equal(got, want["path"]), e  # bit for bit
        assert cost == np.float32(c["g_cost"][e])  # the same computation as the repair's
        assert cost == pytest.approx(want["cost"], rel=P.REL)


def test_plan_over_the_repaired_graph(gt, orc):
    name, scene, N, M, lp = CASES[2]
    c = _run(gt, orc, name, scene, N, M, lp)
    pl = c["pl"]
    pl.sweep()
    pl.extract()
    torch.cuda.synchronize()
    w = c["w"]
    cost3 = oracle.split_edges(c["cost"], M, N, 1)
    V, A, Vs, a_s = oracle.minplus(*cost3)
    _say("plan over repaired graph: gpu", float(pl.cost.item()), "oracle", Vs, "straight-line only",
         c["r"]["path_cost"])
    if not c["excused"].any():
        assert float(pl.cost.item()) == pytest.approx(Vs, rel=P.REL)
    assert float(pl.cost.item()) <= c["r"]["path_cost"] * (1 + P.REL)  # repair only lowers costs


@pytest.mark.parametrize("lp", [(1, 64, 1.0, 0.1, 1.5), (40, 2, 1.0, 0.1, 1.5), (40, 128, 1.0, 0.1, 1.0),
                                (40, 128, 3.0, 0.5, 3.0)])
def test_degenerate_budgets_match_oracle(gt, orc, lp):
    """budget 1; trees of two nodes; ell_factor 1 (a segment-shaped ellipsoid:
    no detour exists); long steps with a wide ellipsoid."""
    c = _run(gt, orc, "2d-small", 3, 24, 3, lp)
    ex = c["excused"]
    _say("degenerate", lp, "repaired", int((c["flag"] == 2).sum()), "excused", int(ex.sum()))
    assert not ((c["g_flag"] != c["flag"]) & ~ex).any()
    np.testing.assert_allclose(c["g_cost"][~ex], c["cost"][~ex], rtol=P.REL)
    if lp[4] == 1.0:
        assert (c["flag"] != 2).all()


def test_free_scene_has_no_candidates(gt):
    w = wl.make_workload("2d-small", 0, N=16, M=3)
    w["circles"] = np.zeros((0, 3), np.float32)
    w["boxes"] = np.zeros((0, 4), np.float32)
    stats = torch.zeros(6, device="cuda", dtype=torch.int64)
    pl = gt.Planner(w, flags=True)
    pl.sample(w["seed"], 0)
    pl.check()
    before = pl.C_h.clone()
    pl.repair(gt.make_rrtc_opts(20, 64, 1.0, 0.1, 1.5, stats), 1, 0)
    torch.cuda.synchronize()
    assert int(stats[0].item()) == 0 and torch.equal(before, pl.C_h) and int(pl.flags.max().item()) == 0


def test_large_trees_match_oracle(gt, orc):
    """Trees of up to 2048 nodes (the LDS holds both): a wall of circles
    across x = 0 whose only gap lies far outside the query ellipsoids, so the
    calls on crossing edges run their whole budget and fill their trees."""
    import oracle.rrtc as R
    ys = np.arange(-12.0, 12.01, 0.4)
    ys = ys[(ys < 7.7) | (ys > 9.8)]
    wall = np.stack([np.zeros_like(ys), ys, np.full_like(ys, 0.3)], 1).astype(np.float32)
    w = wl.make_workload("2d-small", 0, N=12, M=2)
    w["circles"], w["boxes"] = wall, np.zeros((0, 4), np.float32)
    o = R.LPOpts(2500, 2048, 0.4, 0.05, 1.3)
    opts = gt.make_rrtc_opts(o.budget, o.cap, o.eta, o.res, o.ell_factor)
    pl = gt.Planner(w, flags=True)
    pl.sample(w["seed"], 0)
    pl.check()
    pl.repair(opts, 17, 0)
    torch.cuda.synchronize()
    g_cost = _flat((pl.C_s.cpu().numpy(), pl.C_h.cpu().numpy()[:1], pl.C_l.cpu().numpy())).astype(np.float64)
    g_flag = pl.flags.cpu().numpy().astype(np.int32)
    r = orc.plan(w)
    c0, f0, sd0 = _flat(r["cost"]), _flat(r["flag"]), _flat(r["minsd"])
    cost, flag, info = R.repair(w, r["Q"], c0, f0, o, 17, 0)
    ex = np.abs(sd0) <= P.BAND
    ex[info["vertex_band"]] = True
    ex[info["ids"][info["near_band"]]] = True
    _say("large trees: calls", len(info["ids"]), "repaired", int((flag == 2).sum()), "largest tree",
         int(info["sizes"].max()), "excused", int(ex.sum()))
    assert not ((g_flag != flag) & ~ex).any()
    np.testing.assert_allclose(g_cost[~ex], cost[~ex], rtol=P.REL)
    assert info["sizes"].max() > 512
