"""Parity of the anytime policies and the growing-budget sampler (HIP path
through the C ABI) with the oracle (Alg. 1 anytime-gtmp / ao-gtmp /
expand-samples; Sec. IV-C..E)."""
import math

import numpy as np
import pytest
import torch

import oracle
import oracle.anytime as OA
import workloads as wl
from tests import parity as P

pytestmark = pytest.mark.gpu


def _say(*a):
    print("[case]", *a, flush=True)


def _dev(a, dtype=None):
    t = torch.from_numpy(np.ascontiguousarray(a))
    return t.cuda() if dtype is None else t.to("cuda", dtype)


@pytest.mark.parametrize("name,scale,scene", [("2d-small", 1.02, 0), ("2d-small", 1.3, 0), ("2d-small", 2.0, 0),
                                              ("2d-small", 4.0, 0), ("arm7", 1.05, 0), ("arm7", 1.5, 1),
                                              ("arm7", 2.0, 0), ("arm7", 3.0, 1), ("arm7", 4.0, 2),
                                              ("3d-point", 1.05, 0), ("3d-point", 2.5, 1), ("2d-small", None, 0)])
def test_informed_draws_bit_exact(gt, name, scale, scene):
    """Both proposal regions (frame box at thin bounds, clipped bounding box
    once the hyperspheroid reaches beyond the box): same points, same attempt
    counts as the oracle."""
    w = wl.make_workload(name, scene)
    _say("informed", name, scale)
    d = w["d"]
    q0, qg = w["q0"].astype(np.float64), w["goals"][0].astype(np.float64)
    c = np.float32(np.inf) if scale is None else np.float32(np.linalg.norm(qg - q0) * scale)
    prob = gt.make_problem(d, 3, 64, 1, 8, w["lo"], w["hi"], w["penalty"])
    X = torch.empty((300, d), device="cuda")
    att = torch.empty((300,), device="cuda", dtype=torch.int32)
    gt.gtmp_sample_informed(prob, _dev(w["q0"]), _dev(w["goals"]), _dev(np.array([c], np.float32)), 21, 5, 2, X, att)
    torch.cuda.synchronize()
    Xg, Ag = X.cpu().numpy(), att.cpu().numpy()
    for n in range(300):
        x, a = OA.informed_draw(w, None if scale is None else c, 21, 5, 2, n)
        assert a == Ag[n], (n, a, Ag[n])
        assert np.array_equal(x.view(np.uint32), Xg[n].view(np.uint32)), (n, x, Xg[n])


@pytest.mark.parametrize("name,M,N,n_old,cscale,dup", [("2d-small", 4, 64, 32, 1.3, 0), ("2d-small", 3, 40, 0, 1.5, 0),
                                                       ("arm7", 3, 48, 24, 1.5, 0), ("2d-large", 5, 256, 128, 1.2, 0),
                                                       ("2d-small", 4, 64, 32, None, 0),
                                                       ("2d-small", 4, 96, 48, 1.3, 6), ("arm7", 3, 64, 32, 2.0, 4),
                                                       ("arm7", 3, 2048, 1024, 1.5, 0), ("2d-large", 3, 1024, 700, 1.1, 0)])
def test_expand_samples_bit_exact(gt, name, M, N, n_old, cscale, dup):
    """Expansion against the oracle, bit for bit: closest-pair ranks from the
    device pair ranking (with exact ties from repeated samples when dup > 0:
    each old sample repeated dup times, ties broken by pair index) and the
    uniform half."""
    w = wl.make_workload(name, 1, M=M, N=N)
    _say("expand", name, M, N, n_old, cscale, dup)
    d = w["d"]
    q0, qg = w["q0"].astype(np.float64), w["goals"][0].astype(np.float64)
    c = np.float32(np.inf) if cscale is None else np.float32(np.linalg.norm(qg - q0) * cscale)
    Q_old = oracle.sample_layers(M, max(n_old, 1), d, w["lo"], w["hi"], 3, 1)[:, :n_old]
    if dup:
        Q_old = np.ascontiguousarray(np.repeat(Q_old[:, : (n_old + dup - 1) // dup], dup, axis=1)[:, :n_old])
    want = OA.expand_samples(w, [Q_old[m] for m in range(M)], M, N, None if cscale is None else c, 13, 6)
    prob = gt.make_problem(d, M, N, 1, w["H"], w["lo"], w["hi"], w["penalty"])
    ws = gt._aligned_workspace(gt.gtmp_expand_workspace_size(prob))
    Qn = torch.empty((M, N, d), device="cuda")
    Qo = _dev(Q_old) if n_old > 0 else None
    gt.gtmp_expand_samples(prob, _dev(w["q0"]), _dev(w["goals"]), Qo, n_old, Qn, _dev(np.array([c], np.float32)),
                           13, 6, ws)
    torch.cuda.synchronize()
    got = Qn.cpu().numpy()
    assert np.array_equal(got.view(np.uint32), np.stack(want).view(np.uint32))


def _anytime(gt, w, mode, stages, **kw):
    ap = gt.AnytimePlanner(w, mode, stages, **kw)
    ap.run(w["seed"])
    torch.cuda.synchronize()
    return ap


@pytest.mark.parametrize("name,kw", [("2d-small", {}), ("arm7", dict(N=96, M=3)), ("2d-large", dict(N=128, M=4))])
@pytest.mark.parametrize("graph", [False, True])
def test_restart_matches_oracle(gt, name, kw, graph):
    w = wl.make_workload(name, 0, **kw)
    _say("restart", name, kw, "graph", graph)
    S = 5
    ap = _anytime(gt, w, gt.GTMP_ANYTIME_RESTART, S, use_graph=graph)
    best, costs = OA.plan_restart(w, S, w["seed"])
    got = ap.stage_costs.cpu().numpy().astype(np.float64)
    np.testing.assert_allclose(got, costs, rtol=P.REL)
    meta = ap.best_meta.cpu().numpy()
    assert meta[3] == S
    assert float(ap.best_cost.item()) == pytest.approx(best["cost"], rel=P.REL)
    srt = np.sort(costs)
    if srt[1] - srt[0] > P.REL * srt[0]:
        assert meta[0] == best["stage"]
        assert list(ap.best_idx.cpu().numpy()) == list(best["idx"])


def test_restart_graph_replays_match_eager(gt):
    """The captured stage replayed several times, with eager work and
    synchronisations between the calls, gives the eager results each time."""
    w = wl.make_workload("2d-small", 2)
    _say("graph replays")
    eager = _anytime(gt, w, gt.GTMP_ANYTIME_RESTART, 6, use_graph=False)
    ref = eager.stage_costs.clone()
    g = gt.AnytimePlanner(w, gt.GTMP_ANYTIME_RESTART, 6, use_graph=True)
    for rep in range(3):
        g.run(w["seed"])
        torch.cuda.synchronize()
        assert torch.equal(g.stage_costs, ref), rep
        assert torch.equal(g.best_idx, eager.best_idx)
        x = torch.randn(1000, device="cuda").sum()  # eager work in between
        torch.cuda.synchronize()
        del x


@pytest.mark.parametrize("name,sched,kw", [("2d-small", (3, 5, 16, 64, 8), {}), ("2d-large", (4, 5, 64, 256, 6), {}),
                                           ("arm7", (3, 4, 32, 64, 5), {})])
def test_growing_matches_oracle(gt, name, sched, kw):
    w = wl.make_workload(name, 1, **kw)
    M_min, M_max, N_min, N_max, S = sched
    _say("growing", name, sched)
    ap = gt.AnytimePlanner(w, gt.GTMP_ANYTIME_GROWING, S, M_min=M_min, M_max=M_max, N_min=N_min, N_max=N_max)
    ap.run(w["seed"])
    torch.cuda.synchronize()
    best, costs, stages = OA.plan_growing(w, M_min, M_max, N_min, N_max, S, w["seed"])
    got = ap.stage_costs.cpu().numpy().astype(np.float64)[:len(costs)]
    # both sides run their own trajectory: FP32 and FP64 bounds give
    # informed draws that agree to rounding, so stage costs agree to 1e-5
    np.testing.assert_allclose(got, costs, rtol=P.REL)
    meta = ap.best_meta.cpu().numpy()
    assert meta[3] == len(costs)
    assert float(ap.best_cost.item()) == pytest.approx(best["cost"], rel=P.REL)
    assert (meta[1], meta[2]) == (best["M"], best["N"]) or abs(sorted(costs)[1] - sorted(costs)[0]) <= P.REL * best["cost"]


def _best_wp_rows(ap):
    wp = ap.best_wp.cpu().numpy()
    keep = ~np.isnan(wp).any(1)
    n = int(keep.sum())
    assert keep[:n].all() and not keep[n:].any()  # kept waypoints, then NaN rows
    return wp[:n]


@pytest.mark.parametrize("name,kw,graph", [("2d-small", {}, False), ("2d-small", {}, True),
                                           ("arm7", dict(N=96, M=3), False), ("2d-large", dict(N=128, M=4), True)])
def test_restart_with_shortcuts_matches_oracle(gt, name, kw, graph):
    w = wl.make_workload(name, 1, **kw)
    _say("restart + simp", name, kw, "graph", graph)
    S = 5
    ap = _anytime(gt, w, gt.GTMP_ANYTIME_RESTART, S, use_graph=graph, simplify=True)
    best, costs = OA.plan_restart(w, S, w["seed"], simplify=True)
    got = ap.stage_costs.cpu().numpy().astype(np.float64)
    np.testing.assert_allclose(got, costs, rtol=P.REL)  # stage paths themselves
    meta = ap.best_meta.cpu().numpy()
    _say("oracle best", best["cost"], "stage", best["stage"], "gpu", float(ap.best_cost.item()), "stage", meta[0])
    assert float(ap.best_cost.item()) == pytest.approx(best["cost"], rel=P.REL)
    srt = np.sort(costs)
    if srt[1] - srt[0] > P.REL * srt[0] and meta[0] == best["stage"]:
        np.testing.assert_array_equal(_best_wp_rows(ap), best["wp"])


@pytest.mark.parametrize("name,sched", [("2d-small", (3, 5, 16, 64, 8)), ("arm7", (3, 4, 32, 64, 5))])
def test_growing_with_shortcuts_matches_oracle(gt, name, sched):
    w = wl.make_workload(name, 1)
    M_min, M_max, N_min, N_max, S = sched
    _say("growing + simp", name, sched)
    ap = gt.AnytimePlanner(w, gt.GTMP_ANYTIME_GROWING, S, M_min=M_min, M_max=M_max, N_min=N_min, N_max=N_max,
                           simplify=True)
    ap.run(w["seed"])
    torch.cuda.synchronize()
    best, costs, _ = OA.plan_growing(w, M_min, M_max, N_min, N_max, S, w["seed"], simplify=True)
    got = ap.stage_costs.cpu().numpy().astype(np.float64)[:len(costs)]
    _say("stage shortcut lengths gpu", got, "oracle", costs)
    np.testing.assert_allclose(got, costs, rtol=P.REL)
    assert float(ap.best_cost.item()) == pytest.approx(best["cost"], rel=P.REL)
    wp = _best_wp_rows(ap)
    assert np.array_equal(wp[0], w["q0"]) and np.array_equal(wp[-1], w["goals"][0])
    L = sum(np.linalg.norm(b.astype(np.float64) - a) for a, b in zip(wp[:-1], wp[1:]))
    assert L == pytest.approx(float(ap.best_cost.item()), rel=P.REL)


def _oracle_lp_stage(w, Q, o, seed, s):
    r = OA._plan_on(w, Q, o, seed, s)
    info = r["lp_info"]
    sd = np.concatenate([np.asarray(x).ravel() for x in r["minsd"]])
    excused = bool((np.abs(sd) <= P.BAND).any() or info["near_band"].any() or len(info["vertex_band"]))
    return r["path_cost"], excused


@pytest.mark.parametrize("name,kw,lp", [("2d-small", dict(N=24, M=3), (40, 128, 1.0, 0.1, 1.5)),
                                        ("arm7", dict(N=32, M=3), (30, 256, 0.5, 0.1, 1.3))])
def test_restart_with_rrt_connect_matches_oracle(gt, name, kw, lp):
    import oracle.rrtc as R
    w = wl.make_workload(name, 1, **kw)
    o = R.LPOpts(*lp)
    S = 4
    _say("restart + rrtc", name, kw, lp)
    ap = gt.AnytimePlanner(w, gt.GTMP_ANYTIME_RESTART, S, use_graph=True,
                           lp=gt.make_rrtc_opts(o.budget, o.cap, o.eta, o.res, o.ell_factor))
    ap.run(w["seed"])
    torch.cuda.synchronize()
    got = ap.stage_costs.cpu().numpy().astype(np.float64)
    checked = 0
    for s in range(S):
        Q = oracle.sample_layers(w["M"], w["N"], w["d"], w["lo"], w["hi"], w["seed"], s)
        c, excused = _oracle_lp_stage(w, Q, o, w["seed"], s)
        _say("stage", s, "gpu", got[s], "oracle", c, "excused", excused)
        if abs(got[s] - c) <= P.REL * abs(c):
            checked += 1
        else:  # only a decision within the band of contact may move a stage's cost
            assert excused, (s, got[s], c)
    assert checked >= 2
    assert (got < w["penalty"]).all()  # the repair connects every stage on these scenes
    assert float(ap.best_cost.item()) == pytest.approx(np.min(got), rel=1e-7)


def test_growing_with_rrt_connect_matches_oracle(gt):
    import oracle.rrtc as R
    w = wl.make_workload("2d-small", 2)
    o = R.LPOpts(40, 128, 1.0, 0.1, 1.5)
    sched = (2, 3, 8, 32, 5)
    M_min, M_max, N_min, N_max, S = sched
    ap = gt.AnytimePlanner(w, gt.GTMP_ANYTIME_GROWING, S, M_min=M_min, M_max=M_max, N_min=N_min, N_max=N_max,
                           lp=gt.make_rrtc_opts(o.budget, o.cap, o.eta, o.res, o.ell_factor))
    ap.run(w["seed"])
    torch.cuda.synchronize()
    best, costs, _ = OA.plan_growing(w, M_min, M_max, N_min, N_max, S, w["seed"], lp=o)
    got = ap.stage_costs.cpu().numpy().astype(np.float64)[:len(costs)]
    _say("growing + rrtc gpu", got, "oracle", costs)
    np.testing.assert_allclose(got, costs, rtol=P.REL)
    assert float(ap.best_cost.item()) == pytest.approx(best["cost"], rel=P.REL)
