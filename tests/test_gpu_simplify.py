"""Path shortcutting on the GPU against the oracle (oracle/simplify.py): the
table of passing shortcuts element by element (pairs whose oracle signed
distance lies within 1e-5 of zero excused and counted), the simplified
length within 1e-5 relative of the oracle optimum, the returned chain valid
in the oracle's table, and the invariant that a plan's simplified length is
never above its own cost."""
import math

import numpy as np
import pytest
import torch

import oracle
import oracle.simplify as OSI
import workloads as wl
from tests import parity as P

pytestmark = pytest.mark.gpu


def _say(*a):
    print("[case]", *a, flush=True)


def _check(model, wp, H, out):
    """Compare one batch of shortcut results with the oracle.  Returns the
    number of excused pairs."""
    wp = np.asarray(wp, np.float32)
    B, K, d = wp.shape
    valid = out["valid"].cpu().numpy().astype(bool)
    idx = out["idx"].cpu().numpy()
    count = out["count"].cpu().numpy()
    cost = out["cost"].cpu().numpy()
    owp = out["wp"].cpu().numpy()
    upper = np.triu(np.ones((K, K), bool), 1)
    excused = 0
    for b in range(B):
        v_or, minsd = OSI.shortcut_table(model, wp[b], H)
        band = upper & (np.abs(minsd) <= P.BAND)
        excused += int(band.sum())
        assert not valid[b][~upper].any()
        bad = upper & ~band & (valid[b] != v_or)
        assert not bad.any(), (b, np.argwhere(bad)[:5], minsd[bad][:5])
        n = int(count[b])
        assert (idx[b][n:] == -1).all() and np.isnan(owp[b][n:]).all()
        if n == 0:
            assert math.isinf(cost[b])
            if not band.any():
                assert OSI.shortest_over(v_or, wp[b])[0] is None
            continue
        chain = idx[b][:n]
        assert chain[0] == 0 and chain[-1] == K - 1 and (np.diff(chain) > 0).all()
        assert all(valid[b][i, j] for i, j in zip(chain[:-1], chain[1:]))
        np.testing.assert_array_equal(owp[b][:n], wp[b][chain])
        L64 = sum(np.linalg.norm(wp[b][j].astype(np.float64) - wp[b][i]) for i, j in zip(chain[:-1], chain[1:]))
        assert cost[b] == pytest.approx(L64, rel=P.REL)
        if not band.any():
            assert all(v_or[i, j] for i, j in zip(chain[:-1], chain[1:]))
            _, c_or = OSI.shortest_over(v_or, wp[b])
            assert cost[b] == pytest.approx(c_or, rel=P.REL)
    return excused


def _thin(w, keep):
    """The workload with only its first `keep` circles and no boxes (so that
    random paths keep feasible chains)."""
    if keep is not None:
        w["circles"] = w["circles"][:keep]
        w["boxes"] = w["boxes"][:0]
    return w


@pytest.mark.parametrize("name,scene,K,spread,keep", [("2d-small", 0, 6, 1.0, None), ("2d-small", 3, 6, 0.3, 4),
                                                      ("2d-small", 1, 8, 0.5, 5), ("2d-large", 2, 18, 0.1, 30),
                                                      ("2d-large", 1, 18, 0.15, 25), ("2d-small", 4, 2, 1.0, None)])
def test_random_paths_match_oracle(gt, orc, name, scene, K, spread, keep):
    w = _thin(wl.make_workload(name, scene, N=64), keep)
    H = int(w["H"])
    wp = wl.random_paths(w, 24, K, seed=scene, spread=spread)
    _say(name, "scene", scene, "K", K, "H", H, "spread", spread, "circles", len(w["circles"]))
    pl = gt.Planner(w)
    out = gt.simplify_paths(pl.robot, pl.scene, 2, H, torch.from_numpy(wp).cuda())
    torch.cuda.synchronize()
    _say("excused pairs", _check(orc.Model(w), wp, H, out), "kept", out["count"].cpu().numpy()[:12])


@pytest.mark.parametrize("scene,spread", [(0, 0.05), (2, 0.2)])
def test_arm_random_paths_match_oracle(gt, orc, scene, spread):
    w = wl.make_workload("arm7", scene, N=64)
    K, H = int(w["M"]) + 2, int(w["H"])
    wp = wl.random_paths(w, 12, K, seed=10 + scene, spread=spread)
    _say("arm7 scene", scene, "K", K, "spread", spread)
    pl = gt.Planner(w)
    out = pl.simplify(torch.from_numpy(wp).cuda())
    torch.cuda.synchronize()
    _say("excused pairs", _check(orc.Model(w), wp, H, out), "kept", out["count"].cpu().numpy())


@pytest.mark.parametrize("name,scene,N,M", [("2d-small", 1, 64, None), ("2d-large", 0, 256, None), ("3d-point", 0, 96, None),
                                            ("2d-large", 2, 64, 62), ("arm7", 1, 64, None), ("arm7", 3, 64, None)])
def test_oracle_planned_paths_match(gt, orc, name, scene, N, M):
    """The oracle's own plan (M + 2 waypoints, up to the 64-waypoint limit)
    shortcut on both sides."""
    w = wl.make_workload(name, scene, N=N, M=M)
    r = orc.plan(w)
    wp = np.asarray(r["wp"], np.float32)[None]
    _say(name, "scene", scene, "N", N, "K", wp.shape[1], "oracle plan cost", r["path_cost"])
    pl = gt.Planner(w)
    out = pl.simplify(torch.from_numpy(wp).cuda())
    torch.cuda.synchronize()
    _say("excused pairs", _check(orc.Model(w), wp, int(w["H"]), out), "kept", int(out["count"].item()),
         "simplified", float(out["cost"].item()))


@pytest.mark.parametrize("name,scene,N", [("2d-small", 1, 64), ("2d-large", 0, 256), ("arm7", 1, 256),
                                          ("arm7", 3, 512), ("arm7", 0, 2048), ("2d-large", 1, 1024)])
def test_gpu_plan_never_lengthens(gt, name, scene, N):
    """Invariant without the oracle: the plan's own chain is a candidate of
    the shortcut recursion (same FP32 edge lengths, same summation order as
    the value iteration), so the simplified length never exceeds the plan's
    cost, bit for bit."""
    w = wl.make_workload(name, scene, N=N)
    pl = gt.Planner(w)
    pl.plan(w["seed"], 0)
    out = pl.simplify()
    torch.cuda.synchronize()
    plan_cost = float(pl.cost.item())
    _say(name, "scene", scene, "N", N, "plan cost", plan_cost, "simplified", float(out["cost"].item()),
         "kept", int(out["count"].item()))
    assert plan_cost < w["penalty"]
    v = out["valid"].cpu().numpy()[0]
    K = v.shape[0]
    if all(v[i, i + 1] for i in range(K - 1)):
        assert 2 <= int(out["count"].item()) <= K
        assert float(out["cost"].item()) <= plan_cost
    else:  # a plan edge decided within rounding of contact by the two state tests
        _say("a consecutive pair failed the re-check")


def test_free_space_and_degenerate_inputs(gt, orc):
    w = wl.make_workload("2d-small", 0)
    w["circles"] = np.zeros((0, 3), np.float32)
    w["boxes"] = np.zeros((0, 4), np.float32)
    pl = gt.Planner(w)
    wp = wl.random_paths(w, 3, 7, seed=5, spread=0.8)
    wp[2, 3] = np.nan  # a NaN waypoint: every shortcut touching it fails
    out = gt.simplify_paths(pl.robot, pl.scene, 2, 8, torch.from_numpy(wp).cuda())
    torch.cuda.synchronize()
    count = out["count"].cpu().numpy()
    idx = out["idx"].cpu().numpy()
    assert list(count[:2]) == [2, 2] and (idx[:2, :2] == [0, 6]).all()
    L = np.linalg.norm(wp[0, -1].astype(np.float64) - wp[0, 0])
    assert float(out["cost"][0]) == pytest.approx(L, rel=1e-6)
    v = out["valid"].cpu().numpy()[2].astype(bool)
    assert not v[:, 3].any() and not v[3, :].any()
    assert count[2] == 2 and v[0, 6]  # the straight line skips the NaN waypoint
    # empty batch: nothing enqueued, no error
    gt.gtmp_simplify_paths(pl.robot, pl.scene, 2, 8, torch.empty((0, 4, 2), device="cuda"),
                           torch.empty((0,), device="cuda", dtype=torch.uint8),
                           torch.empty((0,), device="cuda", dtype=torch.int32),
                           torch.empty((0,), device="cuda", dtype=torch.int32),
                           torch.empty((0,), device="cuda"))
