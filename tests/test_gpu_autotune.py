"""Autotuner: every launch-shape candidate gives bit-identical edge costs,
flags and batch results (tile invariance), and the tuner returns one of the
candidates and caches it."""
import json

import pytest
import torch

import workloads as wl
from paper_2608_25830_amd import autotune as AT

pytestmark = pytest.mark.gpu


def _say(*a):
    print("[case]", *a, flush=True)


@pytest.mark.parametrize("name,kw", [("2d-large", dict(N=200, M=4, H=16)), ("arm7", dict(N=96, M=3))])
def test_edge_results_invariant_over_candidates(gt, name, kw):
    w = wl.make_workload(name, 1, **kw)
    pl = gt.Planner(w, flags=True)
    pl.sample(w["seed"], 0)
    ref = None
    for c in AT.candidates(w):
        _say(name, c)
        AT.apply(pl.opts, c)
        pl.check()
        torch.cuda.synchronize()
        got = [t.clone() for t in (pl.C_s, pl.C_h, pl.C_l, pl.flags)]
        if ref is None:
            ref = got
            continue
        for a, b in zip(ref, got):
            assert torch.equal(a, b), c


def test_batch_results_invariant_over_candidates(gt):
    specs = wl.batch_specs(n=10, seed=3, N_choices=(64, 96, 128), M_range=(3, 5))
    ref = None
    for c in ({}, dict(states_per_iter=1, sphere_chunks=1, blocks_per_cu=1),
              dict(states_per_iter=8, sphere_chunks=2, blocks_per_cu=4)):
        _say("batch", c)
        bp = gt.BatchPlanner(specs, opts=c)
        bp.run()
        torch.cuda.synchronize()
        meta = bp.best_meta.cpu()
        # the defined part of each plan's best chain: M + 1 entries of the best stage
        chains = torch.cat([bp.plan_idx(i)[:int(meta[i, 1]) + 1] for i in range(len(specs))])
        got = [bp.best_cost.clone(), chains, bp.stage_costs.nan_to_num(-1).clone(), bp.best_meta.clone()]
        if ref is None:
            ref = got
            continue
        for a, b in zip(ref, got):
            assert torch.equal(a, b), c


def test_tuner_picks_a_candidate_and_caches(gt, tmp_path):
    w = wl.make_workload("2d-large", 0, N=128, M=3, H=16)
    path = str(tmp_path / "tune.json")
    e = AT.tune_edge(w, cache_path=path, reps=1, force=True)
    keys = ("states_per_iter", "sphere_chunks", "blocks_per_cu")
    assert {k: e[k] for k in keys} in AT.candidates(w)
    assert e["ms"] == min(r["ms"] for r in e["table"])
    with open(path) as f:
        table = json.load(f)
    assert table[AT.problem_key(w)]["ms"] == e["ms"]
    _say("tuned", {k: e[k] for k in keys}, e["ms"])
