"""Benchmark: edge-states checked per second and plans per second of the
layered-graph planner on one MI355X.

One step = one whole plan on the 7-DoF arm workload (M=8 layers of N=2048
samples, H=16 states per edge, 40 collision spheres, 15 sphere + 15 box
obstacles): sample the layers, realise and cost all 29,364,224 edges, run the
min-plus sweep, extract the path.  Inputs (scene, robot) are resident in HBM
before timing starts; each step draws fresh samples (stage = step index).

Prints one JSON line with the throughput, a roofline entry for the dominant
kernel (the early-exit interior edge checker) measured with HIP events on the
stream it runs on, and the FP64 oracle timed on the host cores on a bounded
sample of the same workload.

    python bench.py [--gpus 1] [--steps 50] [--warmup 5] [--workload arm7]
    python bench.py --form batch [--steps 2] [--warmup 1]

``--form batch`` times the batched form instead: 512 independent plans
(2D point robot and 7-DoF arm mixed, N in {128..2048}, M in 4..16, H = 16,
plain / restart / growing policies) through gtmp_plan_batch, one step = the
whole batch, next to the same plans run one by one through the single-plan
entry point; every plan's result must be bit-identical between the two.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_FP32_TFLOPS = 157.3  # MI355X FP32 vector peak (published)

# HBM bytes per launch of the interior checker on each workload, from the
# FETCH_SIZE / WRITE_SIZE counter runs summarised in profiles/ (scaled by the
# plain-copy calibration).  A value is only reported while the kernel sources
# still hash to the fingerprint it was measured on.
MEASURED_TRAFFIC = {"arm7": (7.982e+07, "7fb879ce13ee603a", "profiles/k_interior_arm7.md")}
KERNEL_SOURCES = ["paper_2608_25830_amd/csrc/edge.hip", "paper_2608_25830_amd/csrc/edge_common.hpp",
                  "paper_2608_25830_amd/csrc/gtmp_device.hpp"]


def kernel_fingerprint():
    import hashlib
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def arm_state_flops(n_joints, n_spheres, n_obs_sph, n_obs_box, d):
    """Algorithmic FP32 operations of one state evaluation in the interior
    checker (FMA = 2, any other arithmetic op = 1):
      lerp                 2 d
      DH FK per joint      48 (frame update and origin) + 1 (angle) + 2 (sin, cos)
      sphere centres       K * 3 * (sub + fma) = 9 K
      sphere obstacles     per obstacle 2 + per (sphere) 3 sub + 3 fma + 1 min = 10
      box obstacles        per obstacle 6 + per (sphere) 3 med3 + 3 sub + 3 fma + 1 min = 13"""
    K = n_spheres
    return (2 * d + 51 * n_joints + 9 * K + n_obs_sph * (2 + 10 * K) + n_obs_box * (6 + 13 * K))


def arm_grid_state_flops(n_joints, n_spheres, d):
    """Algorithmic FP32 operations of one arm state behind the obstacle bins,
    apart from the exact tests (FMA = 2, any other arithmetic op = 1):
      lerp                 2 d
      DH FK per joint      48 + 1 + 2 as above, and the link vector 3 sub
      per sphere           centre 3 fma + bin coordinates 3 fma + 3 clamps = 15
    Each exact sphere-obstacle test (counted by the kernel) adds
      GRID_TEST_FLOPS      R add + R^2 mul + 3 (med3 + sub + fma) + compare = 15"""
    return 2 * d + 54 * n_joints + 15 * n_spheres


GRID_TEST_FLOPS = 15
GRID_MAX_OBS = 64  # obstacles the bin masks hold (the filter's automatic range)


POINT_GRID_MAX_OBS = 96     # obstacles the point kernels' bin masks hold
POINT_GRID_MIN_TILES = 1024  # 256-edge tiles from which the point kernels take the bins


def point_grid_state_flops(d):
    """Point state in R^d behind the obstacle bins, apart from the exact tests
    (GRID_TEST_FLOPS each): lerp 2d, bin coordinates d fma, d saturating
    conversions = 5d."""
    return 5 * d


def point_uses_bins(w, opts):
    n_obs = sum(len(w[k]) for k in (("circles", "boxes") if w["kind"] == "point2d" else ("obs_spheres", "obs_boxes")))
    rows = 1 + (w["M"] - 1) * w["N"] + w["G"]
    tiles = rows * ((w["N"] + 255) // 256)
    return int(opts.sphere_chunks) == 0 and 0 < n_obs <= POINT_GRID_MAX_OBS and tiles >= POINT_GRID_MIN_TILES


def point_state_flops(n_circ, n_box, d):
    """Point robot in R^d: lerp 2d; per circle/sphere d sub + d fma (2 FLOP) + min; per box d med3 + d sub +
    d fma + min (7 and 9 FLOP in 2D)."""
    return 2 * d + n_circ * (d + 2 * d + 1) + n_box * (2 * d + 2 * d + 1) + 0


def cpu_baseline(w, min_seconds=10.0, max_seconds=30.0):
    """FP64 oracle on a bounded sample of the workload's edges (all H states
    of each sampled edge, every sphere against every obstacle)."""
    import oracle
    M, N, G, H, d = w["M"], w["N"], w["G"], w["H"], w["d"]
    Q = oracle.sample_layers(M, N, d, w["lo"], w["hi"], w["seed"], 0)
    model = oracle.Model(w)
    E = oracle.n_edges(M, N, G)
    rng = np.random.default_rng(0)
    chunk = 16384
    done = 0
    t0 = time.perf_counter()
    while True:
        ids = rng.integers(0, E, chunk)
        oracle.edge_subset(model, M, N, G, H, w["q0"], w["goals"], Q, ids, w["penalty"])
        done += chunk
        el = time.perf_counter() - t0
        if el >= min_seconds or el >= max_seconds:
            break
    rate = done * H / el
    return dict(value=rate, unit="edge-states/s", cores=oracle.threads(), kind="oracle",
                sample=f"{done} uniformly drawn edges of the {w['name']} plan (seed {w['seed']}, stage 0), "
                       f"all {H} states each, {el:.1f} s wall", plans_per_s=rate / (E * H))


def bench_classes(args, torch, wl, gtmp):
    """Anytime-GTMP with the class-indexed archive on the small 2D scene:
    one step = one restart stage (sample, edge check, class-augmented sweep,
    archive update); reports the classes archived after all stages next to
    the plain restart policy on the same stages."""
    w = wl.make_workload("2d-small", args.scene, N=args.classes_n)
    reps = w["circles"][:, :2]
    S = args.steps
    cp = gtmp.ClassPlanner(w, reps, S, L=64, cap=4096)
    cp.run(w["seed"])
    torch.cuda.synchronize()
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    a.record()
    cp.run(w["seed"])
    b.record()
    b.synchronize()
    ms = a.elapsed_time(b) / S
    arch = cp.archive()
    rp = gtmp.AnytimePlanner(w, gtmp.GTMP_ANYTIME_RESTART, S)
    rp.run(w["seed"])
    torch.cuda.synchronize()
    a.record()
    rp.run(w["seed"])
    b.record()
    b.synchronize()
    ms_plain = a.elapsed_time(b) / S
    costs = sorted(c for c, _, _ in arch.values())
    out = {
        "metric": "restart stages/s with the class-augmented sweep and class archive (2D)",
        "value": 1e3 / ms,
        "unit": "stages/s",
        "n_gpus": 1,
        "steps": S,
        "warmup": 1,
        "ms_per_step": ms,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": f"2d-small scene seed {w['seed']}: M={w['M']}, N={w['N']}, H={w['H']}, "
                               f"{len(reps)} class-defining circles, L=64 labels per vertex"},
        "classes_archived": len(arch),
        "overflow": int(cp.overflow.item()),
        "best_cost": costs[0] if costs else None,
        "median_class_cost": costs[len(costs) // 2] if costs else None,
        "plain_restart_ms_per_stage": ms_plain,
    }
    print(json.dumps(out), flush=True)


def bench_restart(args, torch, wl, gtmp):
    """Random-restart policy: one step = one stage = one whole plan on fresh
    samples (sample, edge check, sweep, extract, archive), the stage captured
    once as a hipGraph and replayed (no host work between plans)."""
    w = wl.make_workload(args.workload, args.scene)
    S = args.steps
    ap = gtmp.AnytimePlanner(w, gtmp.GTMP_ANYTIME_RESTART, S, use_graph=not args.no_graph)
    for _ in range(max(args.warmup, 1)):
        ap.run(w["seed"])  # first call captures and instantiates the graph
    torch.cuda.synchronize()
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    a.record()
    ap.run(w["seed"])
    b.record()
    b.synchronize()
    ms = a.elapsed_time(b) / S
    E = w["N"] + (w["M"] - 1) * w["N"] ** 2 + w["N"] * w["G"]
    costs = ap.stage_costs.cpu().numpy()
    out = {
        "metric": "plans/s (random-restart stages, one hipGraph replay per plan)",
        "value": 1e3 / ms,
        "unit": "plans/s",
        "n_gpus": 1,
        "steps": S,
        "warmup": args.warmup,
        "ms_per_step": ms,
        "edge_states_per_s": E * w["H"] / (ms / 1e3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": f"{args.workload}: {w['kind']} d={w['d']}, M={w['M']}, N={w['N']}, H={w['H']}, "
                               f"scene seed {w['seed']}", "graph": not args.no_graph, "edges": E},
        "best_cost": float(np.nanmin(costs)),
    }
    print(json.dumps(out), flush=True)


def bench_lazy(args, torch, wl, gtmp):
    """Lazy edge realisation against the full check on the same plans: one
    step = one whole plan (sample, then rounds of sweep / extract / check of
    the selected edges), per band; the full plan beside it.  Every lazy cost
    must equal the full plan's bit for bit."""
    w = wl.make_workload(args.workload, args.scene)
    bands = [float(b) for b in args.lazy_bands.split(",")]
    full = gtmp.Planner(w, flags=True)
    lazy = gtmp.Planner(w, flags=True)
    stats = torch.zeros(2, device="cuda", dtype=torch.int64)

    def timed(fn):
        for i in range(args.warmup):
            fn(1_000_000 + i)
        torch.cuda.synchronize()
        out, ms = [], []
        for i in range(args.steps):
            a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            t0 = time.perf_counter()
            a.record()
            extra = fn(i)
            b.record()
            b.synchronize()
            ms.append((a.elapsed_time(b), (time.perf_counter() - t0) * 1e3))
            out.append((float(full.cost.item()) if extra is None else float(lazy.cost.item()), extra))
        return out, ms

    def run_full(i):
        full.plan(w["seed"], i)
        return None

    full_out, full_ms = timed(run_full)
    rows = []
    for band in bands:
        def run(i):
            stats.zero_()
            st, r = lazy.plan_lazy(w["seed"], i, band=band, max_rounds=args.lazy_rounds, stats=stats)
            known = int((lazy.flags != 0xFF).sum().item())
            return (st, r, int(stats[1].item()), known)
        out, ms = timed(run)
        same = all(o[0] == f[0] for o, f in zip(out, full_out))
        rows.append({"band": band, "ms_per_plan_host": float(np.mean([m[1] for m in ms])),
                     "rounds": float(np.mean([o[1][1] for o in out])),
                     "checked_frac": float(np.mean([o[1][2] for o in out])) / full.E,
                     "known_frac": float(np.mean([o[1][3] for o in out])) / full.E,
                     "complete": all(o[1][0] == gtmp.GTMP_OK for o in out), "cost_equals_full": same})
        print(f"[lazy] band {band}: {rows[-1]['ms_per_plan_host']:.2f} ms, rounds {rows[-1]['rounds']:.1f}, "
              f"checked {rows[-1]['checked_frac']:.4f}, same cost {same}", file=sys.stderr, flush=True)
    best = min(rows, key=lambda r: r["ms_per_plan_host"])
    full_host = float(np.mean([m[1] for m in full_ms]))
    out = {
        "metric": f"plans/s, lazy edge realisation ({args.workload}, best band {best['band']})",
        "value": 1e3 / best["ms_per_plan_host"],
        "unit": "plans/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": best["ms_per_plan_host"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": f"{args.workload}: {w['kind']} d={w['d']}, M={w['M']}, N={w['N']}, H={w['H']}, "
                               f"scene seed {w['seed']}", "edges": full.E},
        "full_check_ms_per_plan": full_host,
        "full_check_ms_per_plan_gpu": float(np.mean([m[0] for m in full_ms])),
        "bands": rows,
    }
    print(json.dumps(out), flush=True)


RRTC_LP = dict(tree_cap=512, step=0.4, resolution=0.1, ell_factor=1.5)


def bench_rrtc(args, torch, wl, gtmp):
    """RRT-Connect local planner (the paper's LP budget sweep setting: the
    7-DoF arm at M = 6 layers of N = 100 samples).  One step = one whole plan:
    sample, straight-line edge check, RRT-Connect on every edge whose straight
    line failed between free endpoints, sweep, extract.  Each budget in the
    sweep is timed over the same stages; budget 1 is the straight line alone
    (no repair).  The main line reports the budget given by --rrtc-budget."""
    budgets = [int(b) for b in args.rrtc_budgets.split(",")]
    if args.rrtc_budget not in budgets:
        budgets.append(args.rrtc_budget)
    lp = dict(RRTC_LP, tree_cap=args.rrtc_cap)
    w = wl.make_workload("arm7", args.scene, M=6, N=100)
    pl = gtmp.Planner(w, flags=True)
    d, M, N, H = pl.d, pl.M, pl.N, pl.H
    f_state = arm_state_flops(d, len(w["sph_link"]), w["obs_spheres"].shape[0], w["obs_boxes"].shape[0], d)
    stats = torch.zeros(6, device="cuda", dtype=torch.int64)
    rows = []
    for B in budgets:
        opts = gtmp.make_rrtc_opts(B, stats=stats, **lp)

        def one(stage):
            pl.sample(w["seed"], stage)
            pl.check()
            if B > 1:
                rb.record()
                pl.repair(opts, w["seed"], stage)
                re.record()
            pl.sweep()
            pl.extract()

        rb, re = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        for i in range(args.warmup):
            one(1_000_000 + i)
        torch.cuda.synchronize()
        stats.zero_()
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        costs, rep_ms = [], []
        t0 = time.perf_counter()
        a.record()
        for i in range(args.steps):
            one(i)
            if B > 1:
                re.synchronize()
                rep_ms.append(rb.elapsed_time(re))
            costs.append(pl.cost[0].clone())
        b.record()
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        ms = a.elapsed_time(b) / args.steps
        st = stats.cpu().numpy().astype(np.float64) / args.steps
        c = torch.stack(costs).cpu().numpy().astype(np.float64)
        solved = c < w["penalty"]
        rows.append({"budget": B, "ms_per_plan": ms, "plans_per_s": 1e3 / ms, "wall_s": wall,
                     "rrtc_ms": float(np.mean(rep_ms)) if rep_ms else 0.0,
                     "solved": int(solved.sum()), "mean_cost_solved": float(c[solved].mean()) if solved.any() else None,
                     "calls": st[0], "repaired": st[1], "iterations": st[2], "tree_nodes": st[3],
                     "states_checked": st[4], "nn_distances": st[5]})
        print(f"[rrtc] budget {B}: {ms:.2f} ms/plan, solved {int(solved.sum())}/{args.steps}", file=sys.stderr,
              flush=True)
    main = next(r for r in rows if r["budget"] == args.rrtc_budget)
    flop = main["states_checked"] * f_state + main["nn_distances"] * 3 * d
    achieved = flop / (main["rrtc_ms"] / 1e3) / 1e12 if main["rrtc_ms"] > 0 else None
    out = {
        "metric": f"plans/s with the RRT-Connect local planner (7-DoF, M=6, N=100, budget {args.rrtc_budget})",
        "value": main["plans_per_s"],
        "unit": "plans/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": main["ms_per_plan"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": f"arm7 (M=6, N=100, H={H}, scene seed {w['seed']}), RRT-Connect step "
                               f"{lp['step']}, resolution {lp['resolution']}, ell "
                               f"{lp['ell_factor']} |y - x|, tree cap {lp['tree_cap']}",
                   "M": M, "N": N, "H": H, "d": d, "edges": pl.E},
        "sweep": rows,
        "roofline": {"bound": "alu", "achieved": achieved, "peak": PEAK_FP32_TFLOPS, "unit": "TFLOP/s",
                     "frac": achieved / PEAK_FP32_TFLOPS if achieved else None, "traffic": None,
                     "kernel": "k_rrtc (one wave per RRT-Connect call; repair time incl. candidate collection)",
                     "flop_per_state": f_state, "kernel_ms": main["rrtc_ms"]},
    }
    if not args.no_cpu:
        out["cpu_baseline"] = rrtc_cpu_baseline(w, args.rrtc_budget, main["calls"], args.cpu_seconds, lp)
    print(json.dumps(out), flush=True)


def rrtc_cpu_baseline(w, budget, calls_per_plan, min_seconds, lp):
    """The oracle on the same workload: its straight-line plan timed whole,
    then RRT-Connect calls on the candidate edges of that plan, in chunks
    until min_seconds have passed; plans/s = 1 / (plan time + calls per plan
    / calls per second)."""
    import oracle
    import oracle.rrtc as R
    t0 = time.perf_counter()
    r = oracle.plan(w)
    t_plan = time.perf_counter() - t0
    flat = lambda t: np.concatenate([np.asarray(x).ravel() for x in t])
    c0, f0 = flat(r["cost"]), flat(r["flag"])
    o = R.LPOpts(budget, lp["tree_cap"], lp["step"], lp["resolution"], lp["ell_factor"])
    model = oracle.Model(w)
    ids = [e for e in np.flatnonzero(f0 == 1)]
    rng = np.random.default_rng(0)
    rng.shuffle(ids)
    X, Y, I = [], [], []
    for e in ids:
        x, y = R.edge_endpoints(w, r["Q"], int(e))
        if (oracle.state_sd(model, np.stack([x, y])) > 0).all():
            X.append(x)
            Y.append(y)
            I.append(int(e))
        if len(I) >= 20000:
            break
    done, t_calls, k = 0, 0.0, 0
    while t_calls < min_seconds and k < len(I):
        n = min(256, len(I) - k)
        t0 = time.perf_counter()
        R.batch(model, w, np.asarray(X[k:k + n]), np.asarray(Y[k:k + n]), np.asarray(I[k:k + n]), o, w["seed"], 0)
        t_calls += time.perf_counter() - t0
        done += n
        k += n
    cps = done / t_calls
    t = t_plan + calls_per_plan / cps
    return {"value": 1.0 / t, "unit": "plans/s", "cores": oracle.threads(), "kind": "oracle",
            "sample": f"one straight-line plan ({t_plan:.2f} s) plus {done} RRT-Connect calls at budget {budget} "
                      f"on uniformly drawn candidate edges of it ({t_calls:.1f} s, {cps:.0f} calls/s), scaled to "
                      f"{calls_per_plan:.0f} calls per plan", "calls_per_s": cps}


def bench_batch(args, torch, wl, gtmp):
    specs = wl.batch_specs(n=args.batch_plans)
    opts = {}
    if args.tune:
        from paper_2608_25830_amd import autotune
        opts = autotune.tune_batch(specs)
    print(f"[bench] batch of {len(specs)} plans, opts {opts}", file=sys.stderr, flush=True)
    # captured as one graph on the first call, launched again by the others
    bp = gtmp.BatchPlanner(specs, opts=opts, use_graph=not args.no_graph)
    for _ in range(max(args.warmup, 1)):
        bp.run()
    torch.cuda.synchronize()
    start, stop = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    t0 = time.perf_counter()
    start.record()
    for _ in range(args.steps):
        bp.run()
    stop.record()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ms_batch = start.elapsed_time(stop) / args.steps
    print(f"[bench] batch {ms_batch:.1f} ms/step", file=sys.stderr, flush=True)
    best_b = bp.best_cost.cpu().numpy()
    stages_b = bp.best_meta[:, 3].cpu().numpy()
    # the same plans, one single-plan call each (each warmed once, then timed)
    ms_single = 0.0
    same = 0
    for i, sp in enumerate(specs):
        ap = gtmp.single_planner(sp)
        seed = int(sp.get("seed", sp["w"]["seed"]))
        ap.run(seed)
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record()
        ap.run(seed)
        b.record()
        b.synchronize()
        ms_single += a.elapsed_time(b)
        same += int(float(ap.best_cost.item()) == float(best_b[i]) or
                    (not np.isfinite(best_b[i]) and not np.isfinite(float(ap.best_cost.item()))))
        del ap
    print(f"[bench] single-plan calls {ms_single:.1f} ms", file=sys.stderr, flush=True)
    n = len(specs)
    n_arm = sum(sp["w"]["kind"] != "point2d" for sp in specs)
    out = {
        "metric": "plans/s (batched, mixed 2D / 7-DoF plans)",
        "value": n / (ms_batch / 1e3),
        "unit": "plans/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_batch,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": f"batch of {n} plans ({n_arm} arm, {n - n_arm} 2D point), N in 128..2048, "
                               f"M in 4..16, H=16, plain / restart(4) / growing policies",
                   "plans": n, "stages_run": int(stages_b.sum())},
        "single_plan_calls": {"ms": ms_single, "plans_per_s": n / (ms_single / 1e3)},
        "speedup_vs_single": ms_single / ms_batch,
        "equal_cost_frac": same / n,
        "batch_opts": opts,
        "wall_s": wall,
    }
    print(json.dumps(out), flush=True)


def _train_surrogate(args, torch, wl, gtmp, w):
    P0, Bf = wl.surrogate_init(7, w["d"])
    S = wl.SURROGATE
    net = gtmp.Surrogate(P0, Bf, batch=S["batch"])
    t0 = time.perf_counter()
    X, y = gtmp.make_labels(w, args.labels, seed=101, stage=0)
    losses = net.train(X, y, epochs=args.epochs, lr=S["lr"])
    torch.cuda.synchronize()
    train_s = time.perf_counter() - t0
    del X, y
    Xh, yh = gtmp.make_labels(w, 1 << 16, seed=101, stage=1)
    acc = float(((net.infer(Xh) > 0) == (yh == 1)).float().mean().item())
    return net, losses, train_s, acc


def _growing_series(torch, gtmp, w, seed, net, stages=6):
    """Best cost after each stage of the growing loop (M 6 -> 8, N 256 ->
    2048) and the time to finish stages 1..s, each prefix run on its own
    (the loop is deterministic, so prefix s repeats the first s stages)."""
    ap = gtmp.AnytimePlanner(w, gtmp.GTMP_ANYTIME_GROWING, stages, M_min=6, M_max=8, N_min=256, N_max=2048,
                             bias=net, bias_tau=0.0)
    ap.run(seed)  # warm-up
    torch.cuda.synchronize()
    sc = ap.stage_costs.cpu().numpy().astype(float)
    best = np.minimum.accumulate(np.where(np.isnan(sc), np.inf, sc))
    ms = []
    for s in range(1, stages + 1):
        ap.opts.max_stages = s
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record()
        ap.run(seed)
        b.record()
        b.synchronize()
        ms.append(a.elapsed_time(b))
    return [float(x) for x in best], ms


def bench_surrogate(args, torch, wl, gtmp):
    """7-DoF arm at N = 4096, M = 8: plain plans against surrogate-pruned
    plans on the same samples (only edges with two free endpoints inferred),
    and the growing loop with and without the surrogate bias of the heuristic
    half over 16 (scene, seed) pairs as cost against time."""
    w = wl.make_workload("arm7", args.scene, N=4096)
    S = wl.SURROGATE
    net, losses, train_s, acc = _train_surrogate(args, torch, wl, gtmp, w)
    print(f"[bench] trained in {train_s:.2f} s, held-out accuracy {acc:.4f}", file=sys.stderr, flush=True)
    pl = gtmp.Planner(w, flags=True)
    robot, scene = gtmp.model_of(w)
    M, N, d = int(w["M"]), int(w["N"]), int(w["d"])
    coll = torch.empty(M * N, device="cuda", dtype=torch.uint8)
    prune = torch.empty(pl.E, device="cuda", dtype=torch.uint8)
    logits = torch.empty(pl.E, device="cuda")
    # threshold: free-edge recall on a held-out plan (stage 999), every edge inferred
    pl.plan(w["seed"], 999)
    net.prune(pl.prob, pl.q0, pl.goals, pl.Q, math.inf, prune, logits)
    tau_dev = torch.empty(1, device="cuda")
    gtmp.gtmp_surrogate_threshold(logits, pl.flags, S["recall"], tau_dev)
    tau = float(tau_dev.item())
    print(f"[bench] tau {tau:.4f}", file=sys.stderr, flush=True)

    def ev():
        return torch.cuda.Event(enable_timing=True)

    res = dict(plain=[], pruned=[], prune_ms=[], same=0, false_prune=[], pruned_frac=[], cand=[])
    for i in range(args.warmup + args.steps):
        a, b, c, e = ev(), ev(), ev(), ev()
        a.record()
        pl.plan(w["seed"], i)
        b.record()
        b.synchronize()
        c_plain = float(pl.cost.item())
        flags_plain = pl.flags.clone()
        c.record()
        gtmp.gtmp_state_check(robot, scene, d, pl.Q.reshape(M * N, d), None, coll)
        net.prune(pl.prob, pl.q0, pl.goals, pl.Q, tau, prune, vcoll=coll)
        e.record()
        pl.check(prune=prune)
        pl.sweep()
        pl.extract()
        f = ev()
        f.record()
        f.synchronize()
        if i < args.warmup:
            continue
        res["plain"].append(a.elapsed_time(b))
        res["pruned"].append(c.elapsed_time(f))
        res["prune_ms"].append(c.elapsed_time(e))
        c_pr = float(pl.cost.item())
        res["same"] += int(abs(c_pr - c_plain) <= 1e-5 * abs(c_plain))
        free = flags_plain == 0
        res["false_prune"].append(float((prune.bool() & free).sum().item()) / max(1, int(free.sum().item())))
        res["pruned_frac"].append(float(prune.float().mean().item()))
        nf = (coll.reshape(M, N) == 0).sum(dim=1).cpu().numpy().astype(np.int64)
        res["cand"].append(int(nf[0] + (nf[:-1] * nf[1:]).sum() + nf[-1] * int(w["G"])))
    ms_plain = float(np.mean(res["plain"]))
    ms_pruned = float(np.mean(res["pruned"]))
    ms_prune = float(np.mean(res["prune_ms"]))
    cand = float(np.mean(res["cand"]))
    mlp_flop = 2 * (64 * 256 + 3 * 256 * 256 + 256)
    achieved = cand * mlp_flop / (ms_prune / 1e3) / 1e12

    # growing loop, plain against biased, 4 scenes x 4 seeds: cost against time
    pairs = []
    for sc_i in range(4):
        ws = wl.make_workload("arm7", sc_i, N=4096)
        net_s = net if sc_i == args.scene else _train_surrogate(args, torch, wl, gtmp, ws)[0]
        for k in range(4):
            seed = int(ws["seed"]) + 1000 * k
            bp, tp = _growing_series(torch, gtmp, ws, seed, None)
            bb, tb = _growing_series(torch, gtmp, ws, seed, net_s)
            target = bp[-1]
            s_p = next(i for i, c in enumerate(bp) if c <= target * (1 + 1e-5))
            s_b = next((i for i, c in enumerate(bb) if c <= target * (1 + 1e-5)), None)
            pairs.append(dict(scene=sc_i, seed=seed, plain_best=bp, plain_ms=tp, biased_best=bb, biased_ms=tb,
                              plain_time_to_cost_ms=tp[s_p],
                              biased_time_to_cost_ms=None if s_b is None else tb[s_b]))
            print(f"[bench] growing scene {sc_i} seed {seed}: plain {bp[-1]:.3f} in {tp[-1]:.1f} ms, "
                  f"biased {bb[-1]:.3f} in {tb[-1]:.1f} ms", file=sys.stderr, flush=True)
    reached = [p for p in pairs if p["biased_time_to_cost_ms"] is not None]
    ratio = [p["biased_time_to_cost_ms"] / p["plain_time_to_cost_ms"] for p in reached]
    grow = {
        "pairs": len(pairs),
        "biased_reaches_plain_final_cost": len(reached),
        "median_time_ratio_biased_over_plain": float(np.median(ratio)) if ratio else None,
        "biased_better_final": sum(1 for p in pairs if p["biased_best"][-1] < p["plain_best"][-1] * (1 - 1e-5)),
        "plain_better_final": sum(1 for p in pairs if p["plain_best"][-1] < p["biased_best"][-1] * (1 - 1e-5)),
        "mean_final_cost": {"plain": float(np.mean([p["plain_best"][-1] for p in pairs])),
                            "biased": float(np.mean([p["biased_best"][-1] for p in pairs]))},
        "mean_loop_ms": {"plain": float(np.mean([p["plain_ms"][-1] for p in pairs])),
                         "biased": float(np.mean([p["biased_ms"][-1] for p in pairs]))},
        "series": pairs,
    }
    out = {
        "metric": "plans/s (7-DoF, N=4096): surrogate-pruned vs plain at equal cost",
        "value": 1e3 / ms_pruned,
        "unit": "plans/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_pruned,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "bf16 mlp / f32 check",
        "data": "synthetic",
        "config": {"workload": f"arm7 d=7, M=8, N=4096, H=16, scene seed {w['seed']}; surrogate 64-256x4-1 "
                               f"BF16, {2 * args.labels} labels, {args.epochs} epochs", "edges": pl.E},
        "plain": {"plans_per_s": 1e3 / ms_plain, "ms": ms_plain},
        "pruned": {"plans_per_s": 1e3 / ms_pruned, "ms": ms_pruned, "prune_ms": ms_prune,
                   "ratio_pruned_over_plain": ms_pruned / ms_plain,
                   "candidate_edges": cand, "candidate_frac": cand / pl.E,
                   "pruned_frac": float(np.mean(res["pruned_frac"])),
                   "false_prune_frac": float(np.mean(res["false_prune"])),
                   "equal_cost_frac": res["same"] / args.steps, "tau_logit": tau},
        "roofline": {"bound": "mfma", "achieved": achieved, "peak": 2500.0, "unit": "TFLOP/s",
                     "frac": achieved / 2500.0, "traffic": None,
                     "kernel": "surrogate inference at candidate-edge midpoints (sample check, lists, k_mlp_prune)"},
        "training": {"seconds": train_s, "steps": int(losses.numel()), "final_loss": float(losses[-20:].mean()),
                     "heldout_accuracy": acc},
        "growing_bias": grow,
    }
    print(json.dumps(out), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=None,
                    help="timed steps (default 50 for the plain form, whose step is about a millisecond, so that "
                         "one late host enqueue barely moves the mean; 10 for the others)")
    ap.add_argument("--warmup", type=int, default=None, help="untimed steps first (default 5 plain, 2 others)")
    ap.add_argument("--workload", default="arm7")
    ap.add_argument("--form", default="plain", choices=["plain", "batch", "surrogate", "restart", "classes", "rrtc",
                                                              "lazy"])
    ap.add_argument("--rrtc-budgets", default="1,100,400,1000", help="rrtc form: budgets of the sweep")
    ap.add_argument("--lazy-bands", default="0.1,0.5,2", help="lazy form: selection bands")
    ap.add_argument("--lazy-rounds", type=int, default=100000, help="lazy form: round limit")
    ap.add_argument("--rrtc-budget", type=int, default=400, help="rrtc form: budget of the main line")
    ap.add_argument("--rrtc-cap", type=int, default=RRTC_LP["tree_cap"], help="rrtc form: nodes per tree")
    ap.add_argument("--classes-n", type=int, default=64, help="classes form: samples per layer")
    ap.add_argument("--no-graph", action="store_true",
                    help="restart and batch forms: enqueue stages instead of replaying a graph")
    ap.add_argument("--labels", type=int, default=1 << 20, help="surrogate: label pairs (2x states)")
    ap.add_argument("--epochs", type=int, default=5, help="surrogate: training epochs")
    ap.add_argument("--batch-plans", type=int, default=512)
    ap.add_argument("--tune", action="store_true", help="batch: pick launch shapes with the autotuner first")
    ap.add_argument("--scene", type=int, default=0)
    ap.add_argument("--no-cpu", action="store_true", help="skip the oracle CPU baseline")
    ap.add_argument("--cpu-seconds", type=float, default=10.0)
    ap.add_argument("--opt", action="append", default=[],
                    help="edge-check option as field=value (fields of gtmp_edge_opts, e.g. sphere_chunks=1)")
    ap.add_argument("--copy-calib-mib", type=int, default=0,
                    help="before the plans, copy a buffer of this many MiB once (reference kernel for the "
                         "FETCH_SIZE / WRITE_SIZE counters)")
    args = ap.parse_args()
    if args.steps is None:
        args.steps = 50 if args.form == "plain" else 10
    if args.warmup is None:
        args.warmup = 5 if args.form == "plain" else 2
    if args.gpus != 1:
        print(f"bench.py measures one GPU only (asked for {args.gpus}); the planner is not built for "
              f"several GPUs.", file=sys.stderr)
        sys.exit(2)

    import torch
    import workloads as wl
    from paper_2608_25830_amd import gtmp

    if not torch.cuda.is_available():
        print("no GPU visible", file=sys.stderr)
        sys.exit(1)
    if args.copy_calib_mib > 0:
        n = args.copy_calib_mib * (1 << 20) // 4
        src = torch.ones(n, device="cuda")
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    if args.form == "batch":
        return bench_batch(args, torch, wl, gtmp)
    if args.form == "surrogate":
        return bench_surrogate(args, torch, wl, gtmp)
    if args.form == "restart":
        return bench_restart(args, torch, wl, gtmp)
    if args.form == "classes":
        return bench_classes(args, torch, wl, gtmp)
    if args.form == "rrtc":
        return bench_rrtc(args, torch, wl, gtmp)
    if args.form == "lazy":
        return bench_lazy(args, torch, wl, gtmp)
    w = wl.make_workload(args.workload, args.scene)
    pl = gtmp.Planner(w)
    for kv in args.opt:
        k, v = kv.split("=")
        setattr(pl.opts, k, int(v))
    M, N, G, H, d = pl.M, pl.N, pl.G, pl.H, pl.d
    E = pl.E
    def make_events(n):
        evs = [torch.cuda.Event(enable_timing=True) for _ in range(n)]
        for e in evs:
            e.record()
        return evs

    for i in range(args.warmup):
        pl.plan(w["seed"], 1_000_000 + i)
    torch.cuda.synchronize()

    # per-step kernel events and counter snapshots stay on the device until the end
    kb, ke = make_events(args.steps), make_events(args.steps)
    sb = make_events(args.steps + 1)  # step boundaries
    stats_hist = torch.zeros((args.steps + 1, 4), device="cuda", dtype=torch.int64)
    cost_hist = torch.zeros((args.steps,), device="cuda")
    start = torch.cuda.Event(enable_timing=True)
    stop = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t_start = time.perf_counter()
    start.record()
    stats_hist[0].copy_(pl.stats)
    for i in range(args.steps):
        sb[i].record()
        pl.opts.ev_begin = kb[i].cuda_event
        pl.opts.ev_end = ke[i].cuda_event
        pl.plan(w["seed"], i)
        stats_hist[i + 1].copy_(pl.stats)
        cost_hist[i].copy_(pl.cost[0])
    sb[args.steps].record()
    stop.record()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t_start
    total_ms = start.elapsed_time(stop)
    ms_per_step = total_ms / args.steps
    kernel_ms = [kb[i].elapsed_time(ke[i]) for i in range(args.steps)]
    step_ms = np.array([sb[i].elapsed_time(sb[i + 1]) for i in range(args.steps)])
    states = torch.diff(stats_hist[:, 0]).cpu().numpy().astype(np.float64)
    tests = torch.diff(stats_hist[:, 2]).cpu().numpy().astype(np.float64)
    costs = cost_hist.cpu().numpy()

    value = E * H / (ms_per_step / 1e3)
    k_ms = float(np.mean(kernel_ms))
    st = float(np.mean(states))
    grid = None
    if w["kind"] == "arm":
        n_obs = w["obs_spheres"].shape[0] + w["obs_boxes"].shape[0]
        f_dense = arm_state_flops(d, len(w["sph_link"]), w["obs_spheres"].shape[0], w["obs_boxes"].shape[0], d)
        if int(pl.opts.sphere_chunks) == 0 and n_obs <= GRID_MAX_OBS:
            # the bin filter: per-state work plus the exact tests it made
            f_state = arm_grid_state_flops(d, len(w["sph_link"]), d)
            t_mean = float(np.mean(tests))
            flop = st * f_state + t_mean * GRID_TEST_FLOPS
            grid = {"exact_tests_per_launch": t_mean, "exact_tests_per_state": t_mean / st,
                    "test_flops": GRID_TEST_FLOPS,
                    "full_test_flop_per_state": f_dense,
                    "full_test_equivalent_tflops": st * f_dense / (k_ms / 1e3) / 1e12}
        else:
            f_state = f_dense
            flop = st * f_state
    else:
        sph, box = (w["circles"], w["boxes"]) if w["kind"] == "point2d" else (w["obs_spheres"], w["obs_boxes"])
        f_dense = point_state_flops(sph.shape[0], box.shape[0], d)
        if point_uses_bins(w, pl.opts):
            f_state = point_grid_state_flops(d)
            t_mean = float(np.mean(tests))
            flop = st * f_state + t_mean * GRID_TEST_FLOPS
            grid = {"exact_tests_per_launch": t_mean, "exact_tests_per_state": t_mean / st,
                    "test_flops": GRID_TEST_FLOPS,
                    "full_test_flop_per_state": f_dense,
                    "full_test_equivalent_tflops": st * f_dense / (k_ms / 1e3) / 1e12}
        else:
            f_state = f_dense
            flop = st * f_state
    achieved = flop / (k_ms / 1e3) / 1e12
    traffic, traffic_src = None, None
    if args.workload in MEASURED_TRAFFIC and not args.opt:
        tb, fp, src = MEASURED_TRAFFIC[args.workload]
        if fp == kernel_fingerprint():
            traffic, traffic_src = tb, src
    out = {
        "metric": "edge-states checked/sec (7-DoF, N=2048)" if args.workload == "arm7" else
                  f"edge-states checked/sec ({args.workload})",
        "value": value,
        "unit": "edge-states/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "plans_per_s": 1e3 / ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": f"{args.workload}: {w['kind']} d={d}, M={M}, N={N}, H={H}, G={G}, scene seed "
                               f"{w['seed']}", "M": M, "N": N, "H": H, "d": d, "edges": E,
                   "edge_states": E * H},
        "roofline": {"bound": "alu", "achieved": achieved, "peak": PEAK_FP32_TFLOPS, "unit": "TFLOP/s",
                     "frac": achieved / PEAK_FP32_TFLOPS, "traffic": traffic, "traffic_unit": "bytes/launch",
                     "traffic_source": traffic_src,
                     "kernel": "k_interior (early-exit interior edge checker)" + (", obstacle-bin filter" if grid else ""),
                     "kernel_ms": k_ms, "states_evaluated_per_launch": st, "flop_per_state": f_state,
                     "states_evaluated_frac": st / (E * H),
                     "obstacle_bins": grid},
        "edge_opts": {k: int(getattr(pl.opts, k)) for k in ("mode", "states_per_iter", "blocks_per_cu",
                                                               "sphere_chunks")},
        "mean_path_cost": float(np.mean(costs)),
        "step_ms_median": float(np.median(step_ms)),
        "step_ms_iqr": [float(np.percentile(step_ms, 25)), float(np.percentile(step_ms, 75))],
        "wall_s": wall,
    }
    out["sweep_roofline"] = sweep_report(torch, pl)
    if not args.opt:
        out["roofline_full_test"] = full_test_report(torch, w, pl)
    out["simplify"] = simplify_report(args, torch, gtmp, w, pl)
    out["lazy"] = lazy_report(args, torch, gtmp, w, costs)
    if not args.no_cpu:
        out["cpu_baseline"] = cpu_baseline(w, min_seconds=args.cpu_seconds)
    print(json.dumps(out), flush=True)


def sweep_report(torch, pl, reps=20):
    """Outside the timed region: the min-plus sweep of the last plan's costs
    alone, HIP events around each call; algorithmic bytes = every cost read
    once plus V and A written: 4 ((M-1) N^2 + N + N G) + 8 M N."""
    M, N, G = pl.M, pl.N, pl.G
    nbytes = 4 * ((M - 1) * N * N + N + N * G) + 8 * M * N
    pl.sweep()
    torch.cuda.synchronize()
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(reps)]
    for a, b in ev:
        a.record()
        pl.sweep()
        b.record()
    torch.cuda.synchronize()
    ms = float(np.median([a.elapsed_time(b) for a, b in ev]))
    gbs = nbytes / (ms / 1e3) / 1e9
    return {"bound": "hbm", "achieved": gbs, "peak": 8000.0, "unit": "GB/s", "frac": gbs / 8000.0,
            "bytes_per_sweep": nbytes, "ms_per_sweep": ms, "layers": M - 1}


def lazy_report(args, torch, gtmp, w, costs, band=0.2):
    """Outside the timed region: the same stages planned lazily (checks
    only near the optimum, reading back one flag per round), timed on the
    host clock; every cost must equal the timed plans' bit for bit."""
    lz = gtmp.Planner(w, flags=True)
    lz.plan_lazy(w["seed"], 1_000_000, band=band)  # warm-up
    torch.cuda.synchronize()
    ms, same, rounds = [], True, []
    for i in range(args.steps):
        t0 = time.perf_counter()
        st, r = lz.plan_lazy(w["seed"], i, band=band)
        c = float(lz.cost.item())
        ms.append((time.perf_counter() - t0) * 1e3)
        same = same and st == gtmp.GTMP_OK and c == float(costs[i])
        rounds.append(r)
    return {"band": band, "ms_per_plan": float(np.mean(ms)), "plans_per_s": 1e3 / float(np.mean(ms)),
            "rounds_mean": float(np.mean(rounds)), "costs_equal_full_check": bool(same)}


def simplify_report(args, torch, gtmp, w, pl):
    """Outside the timed region: the timed steps' paths (re-planned, the
    stages are deterministic) shortcut in one batched call, timed with HIP
    events; mean path length before and after (the paper's simplified path
    length)."""
    K = pl.M + 2
    paths = torch.empty((args.steps, K, pl.d), device="cuda")
    raw = torch.empty((args.steps,), device="cuda")
    for i in range(args.steps):
        pl.plan(w["seed"], i)
        paths[i].copy_(pl.wp)
        raw[i].copy_(pl.cost[0])
    pl.simplify(paths)  # warm-up
    torch.cuda.synchronize()
    b, e = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    b.record()
    out = pl.simplify(paths)
    e.record()
    torch.cuda.synchronize()
    raw = raw.cpu().numpy().astype(np.float64)
    sc = out["cost"].cpu().numpy().astype(np.float64)
    ok = np.isfinite(sc) & (raw < w["penalty"])
    return {"paths": int(args.steps), "waypoints": K, "ms_per_call": b.elapsed_time(e),
            "mean_path_cost": float(raw[ok].mean()) if ok.any() else None,
            "mean_simplified_cost": float(sc[ok].mean()) if ok.any() else None,
            "mean_waypoints_kept": float(out["count"].cpu().numpy()[ok].mean()) if ok.any() else None}


def full_test_report(torch, w, pl, reps=3):
    """Outside the timed region: the same plans with the unfiltered test
    (sphere_chunks 2: every robot sphere against every obstacle at each
    evaluated state; early exit along an edge and the vertex pre-pass stay
    on), its interior kernel timed with HIP events on the plan's stream.
    Algorithmic FLOP = states evaluated (kernel counter) x the full test's
    FP32 operations per state."""
    if w["kind"] != "arm":
        return None
    saved = {k: int(getattr(pl.opts, k)) for k in ("sphere_chunks", "states_per_iter", "blocks_per_cu")}
    pl.opts.sphere_chunks, pl.opts.states_per_iter, pl.opts.blocks_per_cu = 2, 0, 0
    f_dense = arm_state_flops(pl.d, len(w["sph_link"]), w["obs_spheres"].shape[0], w["obs_boxes"].shape[0], pl.d)
    ms, states = [], []
    try:
        for i in range(reps + 1):
            kb, ke = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            kb.record()  # torch creates the HIP event on its first record
            ke.record()
            s0 = pl.stats.clone()
            pl.opts.ev_begin, pl.opts.ev_end = kb.cuda_event, ke.cuda_event
            pl.plan(w["seed"], i)
            torch.cuda.synchronize()
            if i > 0:
                ms.append(kb.elapsed_time(ke))
                states.append(float((pl.stats[0] - s0[0]).item()))
    finally:
        pl.opts.ev_begin, pl.opts.ev_end = None, None
        for k, v in saved.items():
            setattr(pl.opts, k, v)
    k_ms, st = float(np.mean(ms)), float(np.mean(states))
    achieved = st * f_dense / (k_ms / 1e3) / 1e12
    return {"bound": "alu", "achieved": achieved, "peak": PEAK_FP32_TFLOPS, "unit": "TFLOP/s",
            "frac": achieved / PEAK_FP32_TFLOPS, "kernel": "k_interior, unfiltered test (sphere_chunks 2)",
            "kernel_ms": k_ms, "states_evaluated_per_launch": st, "flop_per_state": f_dense,
            "early_exit": True, "plans": reps}


if __name__ == "__main__":
    main()
