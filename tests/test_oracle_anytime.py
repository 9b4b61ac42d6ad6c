"""Pins of the oracle's anytime policies (Alg. 1 anytime-gtmp / ao-gtmp;
Sec. IV-C..E) and of the growing-budget sampler (Alg. 1 expand-samples):
informed-set membership (Sec. IV-E), uniformity of the ellipsoid draws
(radial law of a uniform d-ball), the Householder frame against NumPy, the
d-ball acceptance rate, the mixture coin, the closest-pair property of the
midpoints, monotone archives and the free-space convergence of Thm. 3."""
import math

import numpy as np
import pytest
from scipy import stats
from scipy.special import gamma

import oracle
import oracle.anytime as OA
import workloads as wl


def ellipsoid_coords(w, c, X):
    """Map draws back to the unit ball with an independently built frame:
    a1 = (q_g - q0)/|q_g - q0|, any orthonormal completion."""
    q0 = w["q0"].astype(np.float64)
    qg = np.asarray(w["goals"], np.float64)[0]
    d = q0.size
    cmin = np.linalg.norm(qg - q0)
    a1 = (qg - q0) / cmin
    Qm, _ = np.linalg.qr(np.column_stack([a1, np.eye(d)[:, :d - 1] + 1e-3]))
    Qm[:, 0] = a1
    r = np.array([c / 2] + [math.sqrt(c * c - cmin * cmin) / 2] * (d - 1))
    Y = ((X.astype(np.float64) - (q0 + qg) / 2) @ Qm) / r
    return Y


def test_householder_frame():
    w = wl.make_workload("arm7", 0)
    centre, H, r1, r2, cmin = OA.informed_params(7, w["q0"], w["goals"][0], 9.0)
    a1 = (w["goals"][0].astype(np.float64) - w["q0"]) / np.linalg.norm(w["goals"][0].astype(np.float64) - w["q0"])
    np.testing.assert_allclose(H @ H.T, np.eye(7), atol=1e-6)
    np.testing.assert_allclose(H[:, 0], a1, atol=1e-6)
    assert r1 == pytest.approx(4.5) and r2 == pytest.approx(math.sqrt(81 - cmin ** 2) / 2, rel=1e-6)


def test_informed_draws_in_set_and_uniform_2d():
    w = wl.make_workload("2d-small", 0)
    c = 26.0  # c_min = 25.456; the ellipse stays inside the box
    X = np.stack([OA.informed_draw(w, np.float32(c), 7, 3, 1, n)[0] for n in range(3000)])
    q0, qg = w["q0"].astype(np.float64), w["goals"][0].astype(np.float64)
    s = np.linalg.norm(X - q0, axis=1) + np.linalg.norm(X - qg, axis=1)
    assert np.all(s <= c * (1 + 1e-6))
    Y = ellipsoid_coords(w, c, X)
    rad = np.linalg.norm(Y, axis=1)
    assert rad.max() <= 1 + 1e-5
    # uniform in the d-ball: |y|^d ~ U(0, 1), angle ~ U(-pi, pi)
    assert stats.kstest(rad ** 2, "uniform").pvalue > 1e-3
    ang = np.arctan2(Y[:, 1], Y[:, 0])
    assert stats.kstest(ang, stats.uniform(loc=-np.pi, scale=2 * np.pi).cdf).pvalue > 1e-3


def test_informed_draws_arm_in_set_box_and_acceptance():
    w = wl.make_workload("arm7", 0)
    q0, qg = w["q0"].astype(np.float64), w["goals"][0].astype(np.float64)
    cmin = np.linalg.norm(qg - q0)
    c = float(np.float32(cmin * 1.05))
    draws = [OA.informed_draw(w, np.float32(c), 11, 0, 2, n) for n in range(400)]
    X = np.stack([x for x, _ in draws])
    att = np.array([a for _, a in draws])
    assert np.all(att > 0)
    s = np.linalg.norm(X - q0, axis=1) + np.linalg.norm(X - qg, axis=1)
    assert np.all(s <= c * (1 + 1e-6))
    assert np.all(X >= w["lo"]) and np.all(X <= w["hi"])
    # acceptance of the cube -> ball rejection: volume ratio of the 7-ball
    p_ball = math.pi ** 3.5 / gamma(4.5) / 2 ** 7
    rate = len(att) / att.sum()
    assert rate <= p_ball * 1.3  # box rejections can only lower it


def _ref_informed(w, c, n, seed):
    """Uniform points of X_f(c) n box drawn by two constructions that share
    nothing with the oracle's sampler: a uniform point of the hyperspheroid
    (Gaussian direction, radius u^(1/d), an orthonormal frame from a QR
    factorisation) kept when inside the box, or a uniform point of the box
    kept when inside X_f(c); whichever accepts more often."""
    g = np.random.default_rng(seed)
    q0 = w["q0"].astype(np.float64)
    qg = np.asarray(w["goals"], np.float64)[0]
    lo, hi = w["lo"].astype(np.float64), w["hi"].astype(np.float64)
    d = q0.size
    cmin = np.linalg.norm(qg - q0)
    a1 = (qg - q0) / cmin
    F, _ = np.linalg.qr(np.column_stack([a1, g.normal(size=(d, d - 1))]))
    F[:, 0] = a1
    r = np.array([c / 2] + [math.sqrt(max(c * c - cmin * cmin, 0.0)) / 2] * (d - 1))

    def ell(k):
        z = g.normal(size=(k, d))
        z /= np.linalg.norm(z, axis=1, keepdims=True)
        z *= g.uniform(size=(k, 1)) ** (1.0 / d)
        x = (q0 + qg) / 2 + (z * r) @ F.T
        return x[np.all((x >= lo) & (x <= hi), axis=1)]

    def box(k):
        x = g.uniform(lo, hi, size=(k, d))
        return x[np.linalg.norm(x - q0, axis=1) + np.linalg.norm(x - qg, axis=1) <= c]

    gen = max((ell, box), key=lambda f: f(4000).shape[0])
    out, have = [], 0
    while have < n:
        x = gen(200000)
        out.append(x)
        have += x.shape[0]
    return np.concatenate(out)[:n]


@pytest.mark.parametrize("name,scene", [("arm7", 0), ("arm7", 1), ("2d-small", 0)])
@pytest.mark.parametrize("factor", [1.05, 2.0, 3.0, 4.0])
def test_informed_draws_exact_uniform_in_both_regimes(name, scene, factor):
    """The uniform half is exactly uniform on X_f(c) n box at every bound:
    thin hyperspheroids inside the box (frame-box proposal) and ones reaching
    far beyond it (clipped bounding box): every draw inside the set and the
    box, no draw reaching the attempt cap, and the same law as an
    independent construction (two-sample KS on each coordinate, on
    |x - q0| + |x - q_g| and on the radius in the hyperspheroid's frame)."""
    w = wl.make_workload(name, scene)
    q0, qg = w["q0"].astype(np.float64), w["goals"][0].astype(np.float64)
    cmin = np.linalg.norm(qg - q0)
    c = np.float32(cmin * factor)
    n = 2500
    draws = [OA.informed_draw(w, c, 13, 2, 3, k) for k in range(n)]
    X = np.stack([x for x, _ in draws]).astype(np.float64)
    att = np.array([a for _, a in draws])
    assert np.all(att >= 1), "a draw reached the attempt cap"
    assert att.mean() < 40  # at least ~3 % of the proposals accepted
    s = np.linalg.norm(X - q0, axis=1) + np.linalg.norm(X - qg, axis=1)
    assert np.all(s <= float(c) * (1 + 1e-6))
    assert np.all(X >= w["lo"]) and np.all(X <= w["hi"])
    clipped, _, _ = OA.informed_proposal(w, c)
    assert clipped == (factor > 1.5)  # the regimes the workloads reach
    R = _ref_informed(w, float(c), 20000, 1000 + scene)
    Y = ellipsoid_coords(w, float(c), X)
    Yr = ellipsoid_coords(w, float(c), R)
    sr = np.linalg.norm(R - q0, axis=1) + np.linalg.norm(R - qg, axis=1)
    pv = [stats.ks_2samp(X[:, i], R[:, i]).pvalue for i in range(X.shape[1])]
    pv.append(stats.ks_2samp(s, sr).pvalue)
    pv.append(stats.ks_2samp(np.linalg.norm(Y, axis=1), np.linalg.norm(Yr, axis=1)).pvalue)
    assert min(pv) > 1e-4, pv


def test_informed_radius_law_inside_the_box():
    """A hyperspheroid inside the box: the draws are uniform in it, so the
    radius in its frame follows |y|^d ~ U(0, 1) (one-sample KS)."""
    w = wl.make_workload("2d-small", 1)
    c = np.float32(26.0)  # c_min = 25.456; the ellipse stays inside the box
    clipped, c_lo, c_hi = OA.informed_proposal(w, c)
    assert not clipped
    X = np.stack([OA.informed_draw(w, c, 21, 0, 0, k)[0] for k in range(3000)])
    rad = np.linalg.norm(ellipsoid_coords(w, float(c), X), axis=1)
    assert rad.max() <= 1 + 1e-5
    assert stats.kstest(rad ** 2, "uniform").pvalue > 1e-3


def test_informed_clipped_box_covers_the_set():
    """The clipped bounding box holds every point of X_f(c) n box: the
    extreme points of the hyperspheroid along each axis (closed form:
    centre_i +- sqrt(sum_j F_ij^2 r_j^2)) clipped to the box lie inside it."""
    for name, scene, f in (("arm7", 0, 1.5), ("arm7", 2, 1.2), ("2d-small", 0, 1.3), ("3d-point", 1, 1.1)):
        w = wl.make_workload(name, scene)
        q0, qg = w["q0"].astype(np.float64), w["goals"][0].astype(np.float64)
        cmin = np.linalg.norm(qg - q0)
        c = float(np.float32(cmin * f))
        _, c_lo, c_hi = OA.informed_proposal(w, np.float32(c))
        d = q0.size
        r = np.array([c / 2] + [math.sqrt(c * c - cmin * cmin) / 2] * (d - 1))
        a1 = (qg - q0) / cmin
        F, _ = np.linalg.qr(np.column_stack([a1, np.eye(d)[:, :d - 1] + 1e-3]))
        F[:, 0] = a1
        e = np.sqrt(((F * r) ** 2).sum(axis=1))
        lo = np.maximum(w["lo"], (q0 + qg) / 2 - e)
        hi = np.minimum(w["hi"], (q0 + qg) / 2 + e)
        assert np.all(c_lo <= lo) and np.all(c_hi >= hi)
        assert np.all(c_lo >= w["lo"]) and np.all(c_hi <= w["hi"])


def test_informed_attempt_cap_returns_the_centre():
    """Past the attempt cap the draw is the hyperspheroid's centre (a point
    of the set) with the count -1; with one allowed attempt at a thin bound
    in 7 dimensions the first ball test fails for most slots."""
    w = wl.make_workload("arm7", 0)
    d = 7
    q0, qg = oracle._f32(w["q0"]), oracle._f32(w["goals"][0])
    lo, hi = oracle._f32(w["lo"]), oracle._f32(w["hi"])
    cmin = float(np.linalg.norm(qg.astype(np.float64) - q0))
    c = float(np.float32(cmin * 1.05))
    capped = 0
    for n in range(40):
        out = np.zeros(d, np.float32)
        a = oracle.lib().or_sample_informed(d, oracle._ptr(lo, oracle._fp), oracle._ptr(hi, oracle._fp),
                                            oracle._ptr(q0, oracle._fp), oracle._ptr(qg, oracle._fp), c, 1e3, 3, 0,
                                            0, n, 1, oracle._ptr(out, oracle._fp))
        if a == -1:
            capped += 1
            np.testing.assert_array_equal(out, (q0 + qg) * np.float32(0.5))
        else:
            assert a == 1
    assert capped > 20


def test_unbounded_draw_is_box_sample():
    w = wl.make_workload("2d-small", 0)
    x, a = OA.informed_draw(w, None, 5, 2, 1, 9)
    assert a == 0
    words = oracle.sample_words(5, 2, 1, 9, 1, 0)
    want = np.array([np.float32(-10 + ((int(words[i]) >> 8) * 2.0 ** -24) * 20) for i in range(2)], np.float32)
    np.testing.assert_array_equal(x, want)


def test_coin_is_fair():
    n = sum(OA.coin_heuristic(3, 1, 2, k) for k in range(4000))
    assert stats.binomtest(n, 4000, 0.5).pvalue > 1e-3


def test_expand_midpoints_are_the_closest_pairs():
    w = wl.make_workload("2d-small", 0, M=3, N=40)
    d = 2
    Q0 = oracle.sample_layers(3, 20, d, w["lo"], w["hi"], 9, 0)
    c = np.float32(40.0)
    Q = OA.expand_samples(w, list(Q0), 3, 40, c, 9, 4)
    assert all(q.shape == (40, d) for q in Q)
    for m in range(3):
        np.testing.assert_array_equal(Q[m][:20], Q0[m])  # old samples kept
    # layer 1: neighbours = expanded layer 0 (40) and old layer 2 (20)
    prev, nxt = Q[0].astype(np.float64), Q0[2].astype(np.float64)
    heur = [n for n in range(20, 40) if OA.coin_heuristic(9, 4, 1, n)]
    assert len(heur) > 3
    D = np.linalg.norm(prev[:, None, :] - nxt[None, :, :], axis=-1)
    used = []
    for n in heur:
        x = Q[1][n].astype(np.float64)
        mid = (prev[:, None, :] + nxt[None, :, :]) / 2
        a, b = np.unravel_index(np.argmin(np.linalg.norm(mid - x, axis=-1)), D.shape)
        assert np.linalg.norm(mid[a, b] - x) < 1e-5
        used.append(D[a, b])
    # the used pairs are the k closest ones
    k = len(used)
    assert max(used) <= np.sort(D.ravel())[k - 1] + 1e-5
    assert sorted(used) == pytest.approx(list(np.sort(D.ravel())[:k]), abs=1e-5)


def test_growing_schedule_rule():
    s = OA.growing_schedule(2, 4, 16, 64, 20)
    assert s == [(2, 16, 0), (2, 32, 16), (2, 64, 32), (3, 64, 0), (4, 64, 0)]
    assert OA.growing_schedule(8, 8, 512, 2048, 10) == [(8, 512, 0), (8, 1024, 512), (8, 2048, 1024)]
    assert len(OA.growing_schedule(1, 50, 8, 8, 5)) == 5


def test_restart_archive_monotone_and_min():
    w = wl.make_workload("2d-small", 1)
    best, costs = OA.plan_restart(w, 6, w["seed"])
    assert best["cost"] == min(costs)
    assert best["stage"] == int(np.argmin(costs))
    running = np.minimum.accumulate(costs)
    assert np.all(np.diff(running) <= 0)
    # a stage is the plain planner on the samples of key (seed, stage)
    r = oracle.plan(w, stage=3)
    assert costs[3] == r["path_cost"]


def test_growing_bounds_and_informed_membership():
    w = wl.make_workload("2d-small", 2)
    best, costs, stages = OA.plan_growing(w, 3, 5, 16, 64, 8, 77)
    bounds = [st["bound"] for st in stages]
    assert all(b2 <= b1 for b1, b2 in zip(bounds, bounds[1:]))  # c_min never increases
    q0, qg = w["q0"].astype(np.float64), w["goals"][0].astype(np.float64)
    sched = OA.growing_schedule(3, 5, 16, 64, 8)
    checked = 0
    for si, (st, (M, N, n_old)) in enumerate(zip(stages, sched)):
        if not (np.isfinite(st["bound"]) and st["bound"] < w["penalty"]):
            continue
        # the new uniform-half draws of this stage lie in X_f(c_min)
        for m in range(M):
            for n in range(n_old, N):
                if OA.coin_heuristic(77, si, m, n):
                    continue
                x = st["Q"][m, n].astype(np.float64)
                assert np.linalg.norm(x - q0) + np.linalg.norm(x - qg) <= np.float32(st["bound"]) * (1 + 1e-5)
                checked += 1
    assert checked > 50


def test_growing_free_space_converges_to_straight_line():
    """Thm. 3: in free space the best cost tends to |q_g - q0|."""
    w = wl.make_workload("2d-small", 0)
    w["circles"] = np.zeros((0, 3), np.float32)
    direct = float(np.linalg.norm(w["goals"][0].astype(np.float64) - w["q0"]))
    best, costs, _ = OA.plan_growing(w, 2, 4, 8, 64, 10, 5)
    running = np.minimum.accumulate(costs)
    assert running[-1] >= direct
    assert (running[-1] - direct) < 0.5 * (running[0] - direct) + 1e-9
    assert (running[-1] - direct) / direct < 0.01


def test_biased_heuristic_half_takes_closest_predicted_free_pairs():
    """Surrogate bias with a selector network whose logit is the closed form
    3 relu(x_0 / pi) - 1: with tau = 0 a midpoint counts as free iff
    x_0 <= pi / 3.  The heuristic draws must be, in order, the candidate pairs
    (the BIAS_CANDIDATES * n_new closest) whose midpoint passes that test."""
    import oracle.surrogate as S
    w = wl.make_workload("2d-small", 0, M=3, N=40)
    d = 2
    P = {k: np.zeros(s) for k, s in S.shapes().items()}
    P["W1"][0, 0] = 1.0
    for l in (2, 3, 4):
        P[f"W{l}"][0, 0] = 1.0
    P["w5"][0] = 3.0
    P["b5"][0] = -1.0
    _, Bf = wl.surrogate_init(0, d)
    Q0 = oracle.sample_layers(3, 20, d, w["lo"], w["hi"], 9, 0)
    c = np.float32(40.0)
    Q = OA.expand_samples(w, list(Q0), 3, 40, c, 9, 4, bias=(P, Bf, 0.0))
    prev, nxt = Q[0], Q0[2]
    order = OA.pair_order(prev, nxt)[:OA.BIAS_CANDIDATES * 20]
    mids = [(prev[a] + nxt[b]) * np.float32(0.5) for a, b in (divmod(int(p), nxt.shape[0]) for p in order)]
    free = [x for x in mids if float(x[0]) / np.pi <= 1 / 3]
    heur = [n for n in range(20, 40) if OA.coin_heuristic(9, 4, 1, n)]
    assert 3 < len(heur) <= len(free)
    for h, n in enumerate(heur):
        np.testing.assert_array_equal(Q[1][n], free[h])
    assert all(float(Q[1][n][0]) <= np.pi / 3 for n in heur)


def _polyline_ok(w, wp):
    """Every segment of wp passes the straight-line check at the plan's
    state spacing (H states per segment), first and last waypoints are the
    start and the goal; returns the FP64 length."""
    model = oracle.Model(w)
    assert np.array_equal(wp[0], np.asarray(w["q0"], np.float32))
    assert np.array_equal(wp[-1], np.asarray(w["goals"], np.float32)[0])
    L = 0.0
    for a, b in zip(wp[:-1], wp[1:]):
        c, sd, f = oracle.edge(model, int(w["H"]), a, b)
        assert f == 0
        L += np.linalg.norm(b.astype(np.float64) - a)
    return L


def test_restart_with_shortcuts_stores_shorter_free_paths():
    """Alg. 1 anytime-gtmp with simp(): the stored path is a shortcut of the
    winning stage's path, no longer than it, and the archive never exceeds
    the archive of the loop without shortcuts."""
    w = wl.make_workload("2d-small", 1)
    plain, costs = OA.plan_restart(w, 6, w["seed"])
    best, costs2 = OA.plan_restart(w, 6, w["seed"], simplify=True)
    assert costs2 == costs  # stage paths do not depend on the archive
    assert best["cost"] <= plain["cost"]
    r = oracle.plan(w, stage=best["stage"])
    assert best["cost"] <= r["path_cost"]
    assert best["cost"] == pytest.approx(_polyline_ok(w, best["wp"]), rel=1e-12)
    # waypoints are a subsequence of the stage path
    wp = np.asarray(r["wp"], np.float32)
    pos = [int(np.flatnonzero((wp == x).all(1))[0]) for x in best["wp"]]
    assert pos == sorted(pos) and pos[0] == 0 and pos[-1] == len(wp) - 1


def test_growing_with_shortcuts_bounds_by_the_shortcut_length():
    w = wl.make_workload("2d-small", 2)
    best, costs, stages = OA.plan_growing(w, 3, 5, 16, 64, 8, 77, simplify=True)
    plain, costs0, _ = OA.plan_growing(w, 3, 5, 16, 64, 8, 77)
    # the first stage runs unbounded on both: its shortcut is no longer, and
    # a path through a failed edge has none
    if costs0[0] < w["penalty"]:
        assert costs[0] <= costs0[0]
    else:
        assert costs[0] == np.inf
    assert np.isfinite(best["cost"])
    bounds = [st["bound"] for st in stages]
    run = np.minimum.accumulate(costs)
    assert bounds[1:] == list(run[:-1])  # c_min is the best shortcut length so far
    assert best["cost"] == run[-1]
    ww = dict(w)
    ww["M"], ww["N"] = best["M"], best["N"]
    assert best["cost"] == pytest.approx(_polyline_ok(ww, best["wp"]), rel=1e-12)


def test_restart_with_rrt_connect_lowers_every_stage():
    """The RRT-Connect repair only replaces failed costs by local path
    lengths, so each stage's optimum can only drop; a stage whose straight-
    line plan needs a failed edge is solved when the repair connects one."""
    import oracle.rrtc as R
    w = wl.make_workload("2d-small", 1, N=24, M=3)
    lp = R.LPOpts(budget=40, cap=128, eta=1.0, res=0.1, ell_factor=1.5)
    plain, c0 = OA.plan_restart(w, 4, w["seed"])
    best, c1 = OA.plan_restart(w, 4, w["seed"], lp=lp)
    assert all(b <= a * (1 + 1e-12) for a, b in zip(c0, c1))
    assert best["cost"] <= plain["cost"]
    assert any(b < a for a, b in zip(c0, c1))
    assert all(c < w["penalty"] for c in c1)
