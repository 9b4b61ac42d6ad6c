"""Parity of the HIP path (through the C ABI) with the FP64 oracle on the same
seeded inputs.  Bars: samples bit-exact; edge flags exact outside the 1e-5
signed-distance band; costs, values and path cost within 1e-5 relative; path
indices equal up to the first near-tie; minimisers bit-exact on tie-free rows."""
import math

import numpy as np
import pytest
import torch

import workloads as wl
from tests import parity as P

pytestmark = pytest.mark.gpu


def _say(*a):
    print("[case]", *a, flush=True)


def gpu_plan(gt, w, seed_stage=0, flags=True, minsd=False, mode=None, spi=0):
    pl = gt.Planner(w, flags=flags, minsd=minsd)
    if mode is not None:
        pl.opts.mode = mode
    pl.opts.states_per_iter = spi
    pl.plan(w["seed"], seed_stage)
    torch.cuda.synchronize()
    return pl


def oracle_all(orc, w, Q):
    m = orc.Model(w)
    return orc.edge_costs(m, w["M"], w["N"], w["G"], w["H"], w["q0"], w["goals"], Q, w["penalty"])


# ----------------------------------------------------------------- a1 sampler
@pytest.mark.parametrize("name", ["2d-small", "2d-large", "arm7", "arm7-n4096"])
def test_sampler_bit_exact(gt, orc, name):
    w = wl.make_workload(name, 0)
    _say("sampler", name)
    pl = gt.Planner(w, flags=False)
    for stage in (0, 3):
        pl.sample(w["seed"], stage)
        torch.cuda.synchronize()
        want = orc.sample_layers(w["M"], w["N"], w["d"], w["lo"], w["hi"], w["seed"], stage)
        got = pl.Q.cpu().numpy()
        assert np.array_equal(got.view(np.uint32), want.view(np.uint32))


# ----------------------------------------------------------------- a5 sweep
@pytest.mark.parametrize("M,N,G,p_inf,p_tie", [(4, 64, 1, 0, 0), (4, 64, 1, 0.3, 0.5), (16, 1024, 1, 0, 0.3),
                                               (8, 2048, 1, 0, 0), (8, 2048, 1, 0.1, 0.2), (5, 1000, 3, 0.2, 0.3),
                                               (3, 333, 2, 0.5, 0), (1, 50, 4, 0, 0), (6, 1, 1, 0, 0),
                                               (3, 4096, 1, 0, 0.1), (2, 7, 1, 1.0, 0),
                                               (1, 2048, 1, 0, 0), (1, 4096, 3, 0.1, 0.2), (1, 1025, 2, 0, 0.3)])
def test_minplus_matches_oracle(gt, orc, M, N, G, p_inf, p_tie):
    _say("minplus", M, N, G, p_inf, p_tie)
    Cs, Ch, Cl = wl.random_costs(M * 1000 + N, M, N, G, p_inf=p_inf, p_tie=p_tie)
    dev = lambda a: torch.from_numpy(np.ascontiguousarray(a)).cuda()
    tCs, tCh, tCl = dev(Cs), dev(Ch.reshape(max(M - 1, 1), N, N) if M > 1 else np.zeros((1, N, N), np.float32)), dev(Cl)
    V = torch.empty((M, N), device="cuda")
    A = torch.empty((M, N), device="cuda", dtype=torch.int32)
    Vs = torch.empty(1, device="cuda")
    a_s = torch.empty(1, device="cuda", dtype=torch.int32)
    gt.gtmp_minplus_sweep(M, N, G, tCs, tCh if M > 1 else None, tCl, V, A, Vs, a_s)
    torch.cuda.synchronize()
    V_or, A_or, Vs_or, as_or = orc.minplus(Cs, Ch, Cl)
    Vg, Ag = V.cpu().numpy().astype(np.float64), A.cpu().numpy()
    fin = np.isfinite(V_or)
    assert np.array_equal(np.isfinite(Vg), fin)
    np.testing.assert_allclose(Vg[fin], V_or[fin], rtol=P.REL, atol=0)
    # minimisers: identical wherever the oracle's runner-up is clearly worse
    Ch64, Cl64 = Ch.astype(np.float64), Cl.astype(np.float64)
    checked = 0
    for m in range(M):
        rows = Cl64 if m == M - 1 else Ch64[m] + V_or[m + 1][None, :]
        srt = np.sort(rows, axis=1)
        best = srt[:, 0]
        second = srt[:, 1] if rows.shape[1] > 1 else np.full(rows.shape[0], np.inf)
        with np.errstate(invalid="ignore"):
            clear = (second - best > P.REL * np.maximum(np.abs(best), 1.0)) | ~np.isfinite(best)
        assert np.array_equal(Ag[m][clear], A_or[m][clear]), m
        checked += int(clear.sum())
    assert checked > 0
    if np.isfinite(Vs_or):
        assert float(Vs.item()) == pytest.approx(Vs_or, rel=P.REL)
    else:
        assert math.isinf(Vs.item()) and int(a_s.item()) == -1


@pytest.mark.parametrize("M,N", [(3, 96), (3, 48), (4, 33), (2, 300), (5, 7)])
def test_minplus_exact_ties_lowest_index(gt, orc, M, N):
    # integer costs and a zero goal layer: every sum is exact on both sides,
    # so equal values are genuine ties and both sides keep the lowest index
    # (sizes cover the LDS-staged small sweep, with one or several threads
    # per row, and the streamed one)
    G = 1
    g = np.random.default_rng(3)
    Cs = g.integers(0, 3, N).astype(np.float32)
    Ch = g.integers(0, 3, (M - 1, N, N)).astype(np.float32)
    Cl = np.zeros((N, G), np.float32)
    dev = lambda a: torch.from_numpy(np.ascontiguousarray(a)).cuda()
    V = torch.empty((M, N), device="cuda")
    A = torch.empty((M, N), device="cuda", dtype=torch.int32)
    Vs = torch.empty(1, device="cuda")
    a_s = torch.empty(1, device="cuda", dtype=torch.int32)
    gt.gtmp_minplus_sweep(M, N, G, dev(Cs), dev(Ch), dev(Cl), V, A, Vs, a_s)
    torch.cuda.synchronize()
    V_or, A_or, Vs_or, as_or = orc.minplus(Cs, Ch, Cl)
    assert np.array_equal(A.cpu().numpy(), A_or)
    assert np.array_equal(V.cpu().numpy().astype(np.float64), V_or)
    assert int(a_s.item()) == as_or and float(Vs.item()) == Vs_or


# ----------------------------------------------------------------- a2-a4 edges
EDGE_CASES = [("2d-small", 0, {}), ("2d-small", 3, {}), ("2d-large", 0, dict(N=300, M=3)),
              ("2d-large", 1, dict(N=128, M=4)), ("arm7", 0, dict(N=96, M=3)), ("arm7", 1, dict(N=300, M=2)),
              ("arm7", 2, dict(N=40, M=4, H=9)), ("3d-point", 0, dict(N=96, M=4)), ("3d-point", 2, dict(N=64, M=3, H=7))]


@pytest.mark.parametrize("name,scene,kw", EDGE_CASES)
@pytest.mark.parametrize("mode", [0, 1])
def test_edges_match_oracle(gt, orc, name, scene, kw, mode):
    w = wl.make_workload(name, scene, **kw)
    _say("edges", name, scene, kw, "mode", mode)
    pl = gpu_plan(gt, w, mode=mode, minsd=(mode == 1))
    Q = orc.sample_layers(w["M"], w["N"], w["d"], w["lo"], w["hi"], w["seed"], 0)
    assert np.array_equal(pl.Q.cpu().numpy(), Q)
    cost, minsd, flag = oracle_all(orc, w, Q)
    got = P.flat(pl.C_s.cpu().numpy(), pl.C_h.cpu().numpy()[: w["M"] - 1], pl.C_l.cpu().numpy())
    rep = P.compare_edges(got, pl.flags.cpu().numpy(), P.flat(*cost), P.flat(*minsd), P.flat(*flag))
    _say("edges report", rep)
    if mode == 1:
        ms = pl.minsd.cpu().numpy().astype(np.float64)
        ref = P.flat(*minsd)
        fin = np.isfinite(ref)
        np.testing.assert_allclose(ms[fin], ref[fin], atol=2e-5, rtol=1e-5)


# Graphs of at least 4,096 pre-pass tiles, whose pre-pass blocks take eight
# consecutive rows: blocks spanning two or three layers (N < 8), layer
# boundaries at every offset within a block with a ragged last column segment
# (N = 300), last blocks holding several goal rows (G = 3, whose source
# vertex varies along the row), one sample per layer (every block spans
# eight layers), and a 3-D point robot (M = 17, N = 256: 4,098 tiles).  The plan's path and waypoints check the extraction on chains
# of about a thousand vertices (staged in LDS) and of 4,101 (past the staged
# length: one thread walks the chain).
PREPASS_ROW_CASES = [("2d-large", 0, dict(N=4, M=1100, H=8), 1), ("2d-large", 1, dict(N=300, M=9, H=8), 3),
                     ("arm7", 0, dict(N=5, M=900, H=6), 3), ("2d-large", 2, dict(N=1, M=4100, H=8), 1),
                     ("3d-point", 1, dict(N=256, M=17), 1)]


@pytest.mark.parametrize("name,scene,kw,G", PREPASS_ROW_CASES)
def test_eight_row_prepass_blocks_match_oracle(gt, orc, name, scene, kw, G):
    w = wl.make_workload(name, scene, **kw)
    if G > 1:
        rng = np.random.default_rng(11)
        lo, hi = np.asarray(w["lo"], np.float64), np.asarray(w["hi"], np.float64)
        extra = (lo + (hi - lo) * rng.random((G - 1, w["d"]))).astype(np.float32)
        w["goals"] = np.concatenate([w["goals"], extra]).astype(np.float32)
        w["G"] = G
    M, N = w["M"], w["N"]
    assert (1 + (M - 1) * N + G) * -(-N // 256) >= 4096  # eight rows per pre-pass block
    _say("eight-row pre-pass", name, scene, kw, "G", G)
    pl = gpu_plan(gt, w)
    ref = orc.plan(w)
    got = P.flat(pl.C_s.cpu().numpy(), pl.C_h.cpu().numpy()[: M - 1], pl.C_l.cpu().numpy())
    rep = P.compare_edges(got, pl.flags.cpu().numpy(), P.flat(*ref["cost"]), P.flat(*ref["minsd"]),
                          P.flat(*ref["flag"]))
    _say("report", rep)
    c_gpu = float(pl.cost.item())
    idx_gpu = pl.idx.cpu().numpy()
    # The sweep sums a path's M + 1 positive edge costs one layer at a time in
    # FP32: besides the costs' own 1e-5, the sum may drift by (M + 1) 2^-24
    # relative (the recursive-summation bound), 6.6e-5 at M = 1100.
    rel = P.REL + (M + 1) * 2.0 ** -24
    if rep["excused"] == 0:
        assert c_gpu == pytest.approx(ref["path_cost"], rel=rel)
        n = P.check_path_indices(ref["cost"], ref["V"], ref["idx"], idx_gpu, ref["path_cost"], rel=rel)
        _say("indices compared", n, "of", M + 1)
        # past the first near-tie: the returned chain is one whose oracle
        # edge costs sum to the returned cost
        assert P.path_cost_from_oracle(ref["cost"], idx_gpu) == pytest.approx(c_gpu, rel=rel)
    if np.isfinite(c_gpu):
        wp = pl.wp.cpu().numpy()
        assert np.array_equal(wp[0], w["q0"]) and np.array_equal(wp[-1], w["goals"][idx_gpu[-1]])
        for m in range(M):
            assert np.array_equal(wp[m + 1], ref["Q"][m, idx_gpu[m]])


@pytest.mark.parametrize("twists", ["general", "quarter-plus-ulp", "quarter-minus-ulp"])
@pytest.mark.parametrize("mode", [0, 1])
def test_edges_match_oracle_twists(gt, orc, twists, mode):
    """DH twists other than the workloads' 0 / +-pi/2 (which the GPU applies
    as exact quarter turns): arbitrary angles, and the floats one step above
    or below +-pi/2 (beyond the 1e-7 rad snapping tolerance: the general frame
    update with a cosine near 0).  Flags and costs against the oracle under
    the same rules as every edge test."""
    w = wl.make_workload("arm7", 1, N=96, M=3)
    g = np.random.default_rng(7)
    dh = np.array(w["dh"], dtype=np.float32)
    if twists == "general":
        dh[:, 1] = g.uniform(-np.pi, np.pi, dh.shape[0]).astype(np.float32)
    else:
        q = np.float32(np.pi / 2)
        step = np.nextafter(q, np.float32(4)) if twists == "quarter-plus-ulp" else np.nextafter(q, np.float32(0))
        dh[:, 1] = np.where(np.arange(dh.shape[0]) % 2 == 0, step, -step).astype(np.float32)
    w["dh"] = dh
    _say("edges twists", twists, "mode", mode)
    pl = gpu_plan(gt, w, mode=mode, minsd=(mode == 1))
    Q = orc.sample_layers(w["M"], w["N"], w["d"], w["lo"], w["hi"], w["seed"], 0)
    cost, minsd, flag = oracle_all(orc, w, Q)
    got = P.flat(pl.C_s.cpu().numpy(), pl.C_h.cpu().numpy()[: w["M"] - 1], pl.C_l.cpu().numpy())
    rep = P.compare_edges(got, pl.flags.cpu().numpy(), P.flat(*cost), P.flat(*minsd), P.flat(*flag))
    _say("edges report", rep)
    assert rep["failed"] < rep["edges"]  # the scene leaves some edges free


@pytest.mark.parametrize("spi", [1, 2, 4, 8])
def test_states_per_iter_invariance(gt, orc, spi):
    w = wl.make_workload("2d-large", 2, N=200, M=3)
    _say("spi", spi)
    a = gpu_plan(gt, w, spi=spi)
    b = gpu_plan(gt, w, spi=4)
    for x, y in ((a.C_s, b.C_s), (a.C_h, b.C_h), (a.C_l, b.C_l), (a.flags, b.flags)):
        assert torch.equal(x, y)


def test_fast_equals_full_flags_arm(gt, orc):
    w = wl.make_workload("arm7", 3, N=128, M=3)
    _say("fast-vs-full arm")
    a = gpu_plan(gt, w, mode=0)
    b = gpu_plan(gt, w, mode=1, minsd=True)
    fa, fb = a.flags.cpu().numpy(), b.flags.cpu().numpy()
    ms = b.minsd.cpu().numpy()
    diff = fa != fb
    assert np.all(np.abs(ms[diff]) <= 1e-5)


# ----------------------------------------------------------------- end to end
PLAN_CASES = [("2d-small", s, {}) for s in range(5)] + [
    ("2d-large", 0, dict(N=256, M=6)), ("2d-large", 3, dict(N=160, M=8, H=20)),
    ("arm7", 0, dict(N=128, M=4)), ("arm7", 1, dict(N=64, M=6)), ("arm7", 4, dict(N=200, M=3)),
    ("arm7", 2, dict(N=256, M=5)),
    ("3d-point", 1, dict(N=128, M=5)), ("3d-point", 3, {})]


@pytest.mark.parametrize("name,scene,kw", PLAN_CASES)
def test_plan_matches_oracle(gt, orc, name, scene, kw):
    w = wl.make_workload(name, scene, **kw)
    _say("plan", name, scene, kw)
    pl = gpu_plan(gt, w)
    ref = orc.plan(w)
    cost3, minsd3, flag3 = ref["cost"], ref["minsd"], ref["flag"]
    got = P.flat(pl.C_s.cpu().numpy(), pl.C_h.cpu().numpy()[: w["M"] - 1], pl.C_l.cpu().numpy())
    gflag = pl.flags.cpu().numpy()
    rep = P.compare_edges(got, gflag, P.flat(*cost3), P.flat(*minsd3), P.flat(*flag3))
    c_gpu = float(pl.cost.item())
    idx_gpu = pl.idx.cpu().numpy()
    c_or = ref["path_cost"]
    if rep["excused"] == 0:
        assert c_gpu == pytest.approx(c_or, rel=P.REL)
        n = P.check_path_indices(cost3, ref["V"], ref["idx"], idx_gpu, c_or)
        _say("indices compared", n, "of", w["M"] + 1)
    else:
        ex = (gflag != P.flat(*flag3))
        ex3 = [ex[: w["N"]], ex[w["N"]: w["N"] + (w["M"] - 1) * w["N"] ** 2].reshape(w["M"] - 1, w["N"], w["N"]),
               ex[w["N"] + (w["M"] - 1) * w["N"] ** 2:].reshape(w["N"], 1)]
        len3 = [np.where(f == 1, c - w["penalty"], c) for c, f in zip(cost3, flag3)]
        lo, hi = P.excused_bounds(orc, cost3, len3, ex3, w["penalty"])
        assert lo * (1 - P.REL) <= c_gpu <= hi * (1 + P.REL)
    # the returned chain re-summed with oracle edge costs gives the returned cost
    resum = P.path_cost_from_oracle(cost3, idx_gpu)
    if rep["excused"] == 0:
        assert resum == pytest.approx(c_gpu, rel=P.REL)
    # waypoints are the chosen samples
    wp = pl.wp.cpu().numpy()
    Q = ref["Q"]
    assert np.array_equal(wp[0], w["q0"]) and np.array_equal(wp[-1], w["goals"][idx_gpu[-1]])
    for m in range(w["M"]):
        assert np.array_equal(wp[m + 1], Q[m, idx_gpu[m]])
    _say("plan report", rep, "cost", c_gpu, c_or)


def test_plan_deterministic(gt, orc):
    w = wl.make_workload("arm7", 0, N=256, M=4)
    _say("determinism")
    a = gpu_plan(gt, w)
    C1 = [t.clone() for t in (a.C_s, a.C_h, a.C_l, a.V, a.A, a.idx, a.flags)]
    a.plan(w["seed"], 0)
    torch.cuda.synchronize()
    for x, y in zip(C1, (a.C_s, a.C_h, a.C_l, a.V, a.A, a.idx, a.flags)):
        assert torch.equal(x, y)


# ----------------------------------------------------------------- edge cases
def test_empty_scene_costs_are_lengths(gt, orc):
    w = wl.make_workload("2d-small", 0)
    w["circles"] = np.zeros((0, 3), np.float32)
    _say("empty scene")
    pl = gpu_plan(gt, w)
    Q = pl.Q.cpu().numpy().astype(np.float64)
    assert pl.flags.cpu().numpy().sum() == 0
    L = np.linalg.norm(Q[1][None, :, :] - Q[0][:, None, :], axis=-1)
    np.testing.assert_allclose(pl.C_h.cpu().numpy()[0], L, rtol=1e-6)
    assert float(pl.cost.item()) >= math.dist(w["q0"], w["goals"][0]) * (1 - 1e-6)


def test_h2_and_penalty_inf_and_no_path(gt, orc):
    # H = 2: endpoints only; penalty +inf: failed edges absent
    w = wl.make_workload("2d-small", 1, H=2, penalty=math.inf)
    _say("H=2, penalty inf")
    pl = gpu_plan(gt, w)
    ref = orc.plan(w)
    got = P.flat(pl.C_s.cpu().numpy(), pl.C_h.cpu().numpy()[: w["M"] - 1], pl.C_l.cpu().numpy())
    P.compare_edges(got, pl.flags.cpu().numpy(), P.flat(*ref["cost"]), P.flat(*ref["minsd"]), P.flat(*ref["flag"]))
    # a start inside an obstacle: every start edge fails, no path with +inf penalty
    w2 = wl.make_workload("2d-small", 1, penalty=math.inf)
    w2["circles"] = np.concatenate([w2["circles"], [[-9.0, -9.0, 0.5]]]).astype(np.float32)
    _say("walled start")
    pl2 = gpu_plan(gt, w2)
    assert math.isinf(pl2.cost.item()) and np.all(pl2.idx.cpu().numpy() == -1)
    assert np.all(pl2.flags.cpu().numpy()[: w2["N"]] == 1)


def test_multi_goal_single_layer_and_length_limit(gt, orc):
    w = wl.make_workload("2d-small", 2, M=1, N=37, H=5)
    w["goals"] = np.array([[9.0, 9.0], [8.5, -9.0], [-9.0, 8.0]], np.float32)
    w["G"] = 3
    _say("M=1 G=3")
    pl = gpu_plan(gt, w)
    ref = orc.plan(w)
    got = P.flat(pl.C_s.cpu().numpy(), np.zeros(0), pl.C_l.cpu().numpy())
    P.compare_edges(got, pl.flags.cpu().numpy(), P.flat(*ref["cost"]), P.flat(*ref["minsd"]), P.flat(*ref["flag"]))
    assert float(pl.cost.item()) == pytest.approx(ref["path_cost"], rel=P.REL)
    # length limit: edges longer than ell fail
    pl3 = gt.Planner(wl.make_workload("2d-small", 0), flags=True, max_edge_len=6.0)
    pl3.plan(0)
    torch.cuda.synchronize()
    Q = pl3.Q.cpu().numpy().astype(np.float64)
    L = np.linalg.norm(Q[1][None, :, :] - Q[0][:, None, :], axis=-1)
    E0 = pl3.flags.cpu().numpy()[64: 64 + 64 * 64].reshape(64, 64)
    assert np.all(E0[L > 6.0 + 1e-4] == 1)


def test_single_layer_many_samples(gt, orc):
    # M = 1 with N beyond the one-block sweep's value buffers (1024): the
    # goal layer and the start reduction must take the per-layer launches
    w = wl.make_workload("2d-small", 4, M=1, N=2048, H=8)
    _say("M=1 N=2048")
    pl = gpu_plan(gt, w)
    ref = orc.plan(w)
    got = P.flat(pl.C_s.cpu().numpy(), np.zeros(0), pl.C_l.cpu().numpy())
    rep = P.compare_edges(got, pl.flags.cpu().numpy(), P.flat(*ref["cost"]), P.flat(*ref["minsd"]),
                          P.flat(*ref["flag"]))
    assert rep["excused"] == 0
    assert float(pl.cost.item()) == pytest.approx(ref["path_cost"], rel=P.REL)
    P.check_path_indices(ref["cost"], ref["V"], ref["idx"], pl.idx.cpu().numpy(), ref["path_cost"])


def test_single_sample_layers(gt, orc):
    w = wl.make_workload("arm7", 0, N=1, M=5)
    _say("N=1")
    pl = gpu_plan(gt, w)
    ref = orc.plan(w)
    assert float(pl.cost.item()) == pytest.approx(ref["path_cost"], rel=P.REL)
    assert list(pl.idx.cpu().numpy()) == [0] * 5 + [0]


def _bisection_order(H):
    """Interior grid points 1..H-2 of an edge breadth-first by bisection of
    [0, H-1] (the order the interior kernel checks them in)."""
    out, queue = [], [(0, H - 1)]
    while queue:
        a, b = queue.pop(0)
        if b - a < 2:
            continue
        mid = (a + b) // 2
        out.append(mid)
        queue += [(a, mid), (mid, b)]
    return out


def test_stats_counters(gt, orc):
    """The kernel's counters against the oracle: edges taken = edges with both
    endpoints free; states = those a walk in bisection order with early exit
    evaluates (up to and including the first state in contact), whatever the
    kernel's spreading of its last edges over the lanes.  States and endpoints
    within the 1e-5 band may fall either way: the counts are bracketed."""
    w = wl.make_workload("arm7", 0, N=128, M=3)
    pl = gpu_plan(gt, w)
    s = pl.stats.cpu().numpy()
    E = pl.E
    assert 0 < s[1] <= E and s[0] >= s[1]
    assert s[0] <= s[1] * (w["H"] - 2)
    M, N, H, d = w["M"], w["N"], w["H"], w["d"]
    Q = pl.Q.cpu().numpy().astype(np.float32)
    q0 = np.asarray(w["q0"], np.float32)[None]
    goals = np.asarray(w["goals"], np.float32).reshape(-1, d)
    U = [np.repeat(q0, N, 0)]  # C_s | C_h | C_l edge order
    V = [Q[0]]
    for m in range(M - 1):
        U.append(np.repeat(Q[m], N, 0))
        V.append(np.tile(Q[m + 1], (N, 1)))
    U.append(np.repeat(Q[M - 1], len(goals), 0))
    V.append(np.tile(goals, (N, 1)))
    U, V = np.concatenate(U), np.concatenate(V)
    assert len(U) == E
    model = orc.Model(w)
    sdu, sdv = orc.state_sd(model, U), orc.state_sd(model, V)
    sure = (sdu > P.BAND) & (sdv > P.BAND)
    maybe = (sdu >= -P.BAND) & (sdv >= -P.BAND)
    order = _bisection_order(H)
    t = (np.asarray(order, np.float32) / np.float32(H - 1))[None, :, None]
    ce = np.flatnonzero(maybe)
    X = (U[ce, None, :] + t * (V[ce, None, :] - U[ce, None, :])).astype(np.float32)
    sd = orc.state_sd(model, X.reshape(-1, d)).reshape(len(ce), len(order))
    n = len(order)

    def first(mask):  # states walked: up to the first flagged one, else all
        hit = mask.any(1)
        return np.where(hit, mask.argmax(1) + 1, n)

    lo, hi = first(sd <= P.BAND), first(sd < -P.BAND)
    only_maybe = ~sure[ce]  # endpoints in the band: taken or not
    states_lo = int(lo[~only_maybe].sum())
    states_hi = int(hi.sum())
    _say("stats", "edges", int(s[1]), "in", int(sure.sum()), "..", int(maybe.sum()),
         "states", int(s[0]), "in", states_lo, "..", states_hi)
    assert sure.sum() <= s[1] <= maybe.sum()
    assert states_lo <= s[0] <= states_hi
