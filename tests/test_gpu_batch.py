"""Batched plans (persistent per-group edge launches over the tiles of every
plan) give, plan by plan, exactly the results of the single-plan calls with
the same seed, with and without hipGraph capture."""
import numpy as np
import pytest
import torch

import workloads as wl

pytestmark = pytest.mark.gpu


def _say(*a):
    print("[case]", *a, flush=True)


def mixed_specs(gt):
    R, G = gt.GTMP_ANYTIME_RESTART, gt.GTMP_ANYTIME_GROWING
    return [
        dict(w=wl.make_workload("2d-small", 0), mode=R, stages=1),
        dict(w=wl.make_workload("arm7", 0, N=64, M=3), mode=R, stages=2),
        dict(w=wl.make_workload("2d-large", 1, N=128, M=5, H=16), mode=R, stages=3),
        dict(w=wl.make_workload("2d-small", 3), mode=G, stages=6, M_min=2, N_min=16),
        dict(w=wl.make_workload("arm7", 2, N=48, M=4, H=16), mode=G, stages=4, M_min=3, N_min=12),
        dict(w=wl.make_workload("arm7", 1, N=100, M=2, H=12), mode=R, stages=1),
        dict(w=wl.make_workload("2d-large", 2, N=300, M=4, H=16), mode=G, stages=3, M_min=3, N_min=75),
        dict(w=wl.make_workload("2d-small", 4, H=2), mode=R, stages=2),
    ]


def single(gt, sp):
    w = sp["w"]
    if sp["mode"] == gt.GTMP_ANYTIME_GROWING:
        ap = gt.AnytimePlanner(w, sp["mode"], sp["stages"], M_min=sp["M_min"], N_min=sp["N_min"])
    else:
        ap = gt.AnytimePlanner(w, sp["mode"], sp["stages"])
    ap.run(w["seed"])
    torch.cuda.synchronize()
    return ap


@pytest.mark.parametrize("graph", [False, True])
def test_batch_equals_single_plans(gt, graph):
    specs = mixed_specs(gt)
    _say("batch", len(specs), "graph", graph)
    bp = gt.BatchPlanner(specs, use_graph=graph)
    bp.run()
    torch.cuda.synchronize()
    for i, sp in enumerate(specs):
        ap = single(gt, sp)
        S = sp["stages"]
        meta_b = bp.best_meta[i].cpu().numpy()
        meta_s = ap.best_meta.cpu().numpy()
        _say("plan", i, sp["w"]["name"], "mode", sp["mode"], "meta", meta_b, meta_s)
        assert np.array_equal(meta_b, meta_s)
        n_st = int(meta_s[3])
        assert torch.equal(bp.stage_costs[i, :n_st], ap.stage_costs[:n_st])
        assert float(bp.best_cost[i].item()) == float(ap.best_cost.item())
        Mb = int(meta_s[1])
        assert torch.equal(bp.plan_idx(i)[:Mb + 1], ap.best_idx[:Mb + 1])


def _same_chains(a, b):
    """best_idx holds each plan's best chain in its first M + 1 entries (M of
    the best stage); the rest is not written."""
    ma, mb = a.best_meta.cpu().numpy(), b.best_meta.cpu().numpy()
    assert np.array_equal(ma, mb)
    for i in range(len(a.specs)):
        M = int(ma[i, 1])
        assert torch.equal(a.plan_idx(i)[:M + 1], b.plan_idx(i)[:M + 1]), i


def test_batch_graph_equals_eager_repeatedly(gt):
    """Every policy, growing plans included, captured: the kept graph is
    launched again by later calls (with eager work and synchronisations in
    between) and matches the eager batch each time."""
    specs = mixed_specs(gt)
    _say("batch graph repeat", len(specs))
    eager = gt.BatchPlanner(specs, use_graph=False)
    eager.run()
    torch.cuda.synchronize()
    g = gt.BatchPlanner(specs, use_graph=True)
    for rep in range(3):
        g.run()
        torch.cuda.synchronize()
        assert torch.equal(g.best_cost, eager.best_cost), rep
        _same_chains(g, eager)
        assert torch.equal(g.stage_costs.nan_to_num(-1), eager.stage_costs.nan_to_num(-1)), rep
        x = torch.randn(4096, device="cuda").sum()  # eager work between launches
        torch.cuda.synchronize()
        del x


def test_batch_graph_after_another_batch_on_its_workspace(gt):
    """A kept graph launched after another batch wrote the same workspace:
    its tables are uploaded again first, and its results stay those of the
    eager batch.  The two batches alternate on one workspace, results
    checked after every call."""
    specs_a = mixed_specs(gt)
    specs_b = [sp for sp in specs_a if sp["mode"] == gt.GTMP_ANYTIME_RESTART][::-1]
    _say("alternating batches on one workspace")
    ref_a = gt.BatchPlanner(specs_a, use_graph=False)
    ref_b = gt.BatchPlanner(specs_b, use_graph=False)
    ref_a.run()
    ref_b.run()
    torch.cuda.synchronize()
    a = gt.BatchPlanner(specs_a, use_graph=True)
    b = gt.BatchPlanner(specs_b, use_graph=True)
    assert b.workspace.numel() <= a.workspace.numel()
    b.workspace = a.workspace[: b.workspace.numel()]
    for rep in range(2):
        for bp, ref in ((a, ref_a), (b, ref_b)):
            bp.run()
            torch.cuda.synchronize()
            assert torch.equal(bp.best_cost, ref.best_cost), rep
            _same_chains(bp, ref)


def test_batch_same_robot_many_plans(gt):
    """Many arm plans share the persistent launch: waves switch plans."""
    R = gt.GTMP_ANYTIME_RESTART
    specs = [dict(w=wl.make_workload("arm7", s % 5, N=32 + 16 * (s % 4), M=3 + s % 3), mode=R, stages=1,
                  seed=100 + s) for s in range(24)]
    _say("24 arm plans")
    bp = gt.BatchPlanner(specs)
    bp.run()
    torch.cuda.synchronize()
    for i in (0, 5, 11, 17, 23):
        sp = specs[i]
        ap = gt.AnytimePlanner(sp["w"], R, 1)
        ap.run(sp["seed"])
        torch.cuda.synchronize()
        assert float(bp.best_cost[i].item()) == float(ap.best_cost.item())
        assert torch.equal(bp.stage_costs[i, :1], ap.stage_costs[:1])


def test_batch_plain_plan_equals_oracle(gt, orc):
    """A one-stage restart plan of a batch is the plain planner (Alg. 1):
    its cost is the oracle's on the samples of key (seed, stage 0)."""
    specs = mixed_specs(gt)
    bp = gt.BatchPlanner(specs)
    bp.run()
    torch.cuda.synchronize()
    for i in (0, 5):
        w = specs[i]["w"]
        r = orc.plan(w, stage=0)
        c = float(bp.best_cost[i].item())
        _say("oracle plan", i, w["name"], c, r["path_cost"])
        if np.isfinite(r["path_cost"]):
            assert c == pytest.approx(r["path_cost"], rel=1e-5)
        else:
            assert not np.isfinite(c)
