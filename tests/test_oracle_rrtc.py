"""Pins of the RRT-Connect local-planner oracle (oracle/rrtc.py, or_rrtc in
gtmp_oracle.c): one-iteration connection in free space with the closed-form
path, samples uniform in the query ellipsoid, tree invariants (step bound,
ellipsoid, segments clear of every circle up to the discretisation bound),
a wall whose only gap lies outside the ellipsoid (no call may succeed) or
inside it (paths cross the wall only through the gap), and the repair pass
over a sampled graph."""
import numpy as np
import pytest
from scipy import stats

import oracle
import oracle.rrtc as R
import workloads as wl


def _w2(circles):
    w = wl.make_workload("2d-small", 0)
    w["circles"] = np.asarray(circles, np.float32).reshape(-1, 3)
    w["boxes"] = np.zeros((0, 4), np.float32)
    return w


def _seg_point_dist(a, b, c):
    a, b, c = (np.asarray(v, np.float64) for v in (a, b, c))
    ab = b - a
    t = np.clip(np.dot(c - a, ab) / max(np.dot(ab, ab), 1e-300), 0.0, 1.0)
    return np.linalg.norm(a + t * ab - c)


def test_free_space_connects_in_one_iteration():
    w = _w2(np.zeros((0, 3)))
    m = oracle.Model(w)
    x, y = np.array([-5, -3], np.float32), np.array([5, 2], np.float32)
    o = R.LPOpts(budget=10, cap=256, eta=1.0, res=0.1, ell_factor=1.5)
    r = R.call(m, w, x, y, o, 7, 0, 123)
    assert r["ok"] and r["iters"] == 1
    P = r["path"].astype(np.float64)
    assert np.array_equal(r["path"][0], x) and np.array_equal(r["path"][-1], y)
    # x -> one step towards the first sample -> straight back to y
    q = R.sample(w, x, y, 1.5, 7, 0, 123, 0)
    step = np.linalg.norm(q.astype(np.float64) - x)
    assert np.linalg.norm(P[1] - P[0]) == pytest.approx(min(step, 1.0), rel=1e-5)
    u = (P[-1] - P[1]) / np.linalg.norm(P[-1] - P[1])
    for p in P[2:-1]:
        v = p - P[1]
        assert abs(v[0] * u[1] - v[1] * u[0]) < 1e-4  # on the line q_new -> y
    L = np.linalg.norm(P[1] - P[0]) + np.linalg.norm(P[-1] - P[1])
    assert r["cost"] == pytest.approx(L, rel=1e-6)
    ell = 1.5 * np.linalg.norm(y.astype(np.float64) - x)
    assert r["cost"] <= ell * (1 + 1e-6)
    assert r["sizes"][0] == 2 and r["sizes"][1] == len(P) - 1


def test_samples_uniform_in_query_ellipsoid():
    w = _w2(np.zeros((0, 3)))
    x, y = np.array([-2, 1], np.float32), np.array([3, -1], np.float32)
    centre, H, r1, r2, ell = R.ellipsoid(x, y, 1.4)
    Z = []
    for i in range(3000):
        q = R.sample(w, x, y, 1.4, 11, 2, 5, i).astype(np.float64)
        assert np.linalg.norm(q - x) + np.linalg.norm(q - y) <= ell * (1 + 1e-5)
        z = H.astype(np.float64).T @ (q - centre)  # H is a symmetric reflection
        Z.append([z[0] / r1, z[1] / r2])
    Z = np.asarray(Z)
    r2s = (Z ** 2).sum(1)
    assert stats.kstest(r2s, "uniform").pvalue > 1e-3  # |y|^2 of a uniform disk draw is U(0, 1)
    ang = np.arctan2(Z[:, 1], Z[:, 0])
    assert stats.kstest((ang + np.pi) / (2 * np.pi), "uniform").pvalue > 1e-3


@pytest.mark.parametrize("seed", range(3))
def test_tree_invariants_in_clutter(seed):
    rng = np.random.default_rng(seed)
    circles = np.concatenate([rng.uniform(-4, 4, (12, 2)), rng.uniform(0.4, 1.0, (12, 1))], 1)
    w = _w2(circles)
    m = oracle.Model(w)
    o = R.LPOpts(budget=200, cap=400, eta=0.6, res=0.05, ell_factor=1.6)
    done = 0
    for k in range(20):
        x, y = rng.uniform(-6, 6, 2).astype(np.float32), rng.uniform(-6, 6, 2).astype(np.float32)
        if (oracle.state_sd(m, np.stack([x, y])) <= 0).any():
            continue
        r = R.call(m, w, x, y, o, 3, 1, k)
        _, _, _, _, ell = R.ellipsoid(x, y, o.ell_factor)
        for t in range(2):
            n = r["sizes"][t]
            T, par = r["trees"][t][:n].astype(np.float64), r["parents"][t][:n]
            assert par[0] == -1 and (par[1:] >= 0).all() and (par[1:] < np.arange(1, n)).all()
            for j in range(1, n):
                a, b = T[par[j]], T[j]
                assert np.linalg.norm(b - a) <= o.eta * (1 + 1e-6)
                assert np.linalg.norm(b - x) + np.linalg.norm(b - y) <= ell * (1 + 1e-5)
                for c in circles:  # discrete check: penetration at most res^2 / (8 r)
                    assert _seg_point_dist(a, b, c[:2]) > c[2] - o.res ** 2 / (4 * c[2])
        if r["ok"]:
            P = r["path"].astype(np.float64)
            assert np.array_equal(r["path"][0], x) and np.array_equal(r["path"][-1], y)
            assert r["cost"] == pytest.approx(np.linalg.norm(np.diff(P, axis=0), axis=1).sum(), rel=1e-12)
            done += 1
    assert done >= 3


def _wall(gap_lo, gap_hi):
    ys = np.arange(-12.0, 12.01, 0.4)
    ys = ys[(ys < gap_lo - 0.3) | (ys > gap_hi + 0.3)]
    return np.stack([np.zeros_like(ys), ys, np.full_like(ys, 0.3)], 1)


def test_gap_outside_the_ellipsoid_never_connects():
    w = _w2(_wall(8.0, 9.5))  # semi-minor axis of E(x, y; 9) is 3.35: the gap lies outside
    m = oracle.Model(w)
    x, y = np.array([-3, 0], np.float32), np.array([3, 0], np.float32)
    o = R.LPOpts(budget=400, cap=1024, eta=0.5, res=0.05, ell_factor=1.5)
    out = R.batch(m, w, np.tile(x, (6, 1)), np.tile(y, (6, 1)), np.arange(6), o, 9, 0)
    assert not out["ok"].any()
    assert (out["iters"] == o.budget).all()


def test_gap_inside_the_ellipsoid_is_the_only_crossing():
    gap = (1.0, 2.6)
    w = _w2(_wall(*gap))
    m = oracle.Model(w)
    x, y = np.array([-3, 0], np.float32), np.array([3, 0], np.float32)
    o = R.LPOpts(budget=400, cap=1024, eta=0.5, res=0.05, ell_factor=1.5)
    hits = 0
    for e in range(6):
        r = R.call(m, w, x, y, o, 9, 0, e)
        if not r["ok"]:
            continue
        hits += 1
        P = r["path"].astype(np.float64)
        for a, b in zip(P[:-1], P[1:]):
            if (a[0] < 0) != (b[0] < 0):
                yc = a[1] + (b[1] - a[1]) * (0 - a[0]) / (b[0] - a[0])
                assert gap[0] - 0.3 < yc < gap[1] + 0.3
    assert hits >= 3


def test_repair_pass_on_a_sampled_graph():
    w = wl.make_workload("2d-small", 1, N=24, M=3)
    r = oracle.plan(w)
    flat = lambda t: np.concatenate([t[0].ravel(), t[1].ravel(), t[2].ravel()])
    cost0, flag0 = flat(r["cost"]), flat(r["flag"])
    o = R.LPOpts(budget=60, cap=256, eta=1.0, res=0.1, ell_factor=1.5)
    cost, flag, info = R.repair(w, r["Q"], cost0, flag0, o, 5, 0)
    assert set(np.flatnonzero(flag == 2)) <= set(info["ids"]) <= set(np.flatnonzero(flag0 == 1))
    assert (flag[flag0 == 0] == 0).all() and np.array_equal(cost[flag0 == 0], cost0[flag0 == 0])
    rep = flag == 2
    assert rep.sum() > 0
    L = cost0[rep] - w["penalty"]  # straight-line length of the repaired edges
    assert (cost[rep] >= L * (1 - 1e-12)).all()
    # batch results equal single calls
    model = oracle.Model(w)
    for k in range(0, len(info["ids"]), max(1, len(info["ids"]) // 8)):
        e = int(info["ids"][k])
        x, y = R.edge_endpoints(w, r["Q"], e)
        one = R.call(model, w, x, y, o, 5, 0, e)
        assert one["ok"] == info["ok"][k] and one["iters"] == info["iters"][k]
        assert tuple(one["sizes"]) == tuple(info["sizes"][k])
        if one["ok"]:
            assert one["cost"] == info["cost"][k]
