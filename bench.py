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

    python bench.py [--gpus 1] [--steps 10] [--warmup 2] [--workload arm7]
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
MEASURED_TRAFFIC = {"arm7": (52.38e6, "183f662d58bceb9f", "profiles/k_interior_arm7.md")}
KERNEL_SOURCES = ["paper_2608_25830_amd/csrc/edge.hip", "paper_2608_25830_amd/csrc/gtmp_device.hpp",
                  "paper_2608_25830_amd/csrc/gtmp_launch.hpp"]


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


def point_state_flops(n_circ, n_box, d):
    """Point robot: lerp 2d, circle 2 sub + 2 fma + min = 7 (2D), box 2 med3 + 2 sub + 2 fma + min = 9."""
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


def bench_batch(args, torch, wl, gtmp):
    specs = wl.batch_specs(n=args.batch_plans)
    opts = {}
    if args.tune:
        from paper_2608_25830_amd import autotune
        opts = autotune.tune_batch(specs)
    print(f"[bench] batch of {len(specs)} plans, opts {opts}", file=sys.stderr, flush=True)
    bp = gtmp.BatchPlanner(specs, opts=opts)
    for _ in range(args.warmup):
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


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="arm7")
    ap.add_argument("--form", default="plain", choices=["plain", "batch"])
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
    stats_hist = torch.zeros((args.steps + 1, 4), device="cuda", dtype=torch.int64)
    cost_hist = torch.zeros((args.steps,), device="cuda")
    start = torch.cuda.Event(enable_timing=True)
    stop = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t_start = time.perf_counter()
    start.record()
    stats_hist[0].copy_(pl.stats)
    for i in range(args.steps):
        pl.opts.ev_begin = kb[i].cuda_event
        pl.opts.ev_end = ke[i].cuda_event
        pl.plan(w["seed"], i)
        stats_hist[i + 1].copy_(pl.stats)
        cost_hist[i].copy_(pl.cost[0])
    stop.record()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t_start
    total_ms = start.elapsed_time(stop)
    ms_per_step = total_ms / args.steps
    kernel_ms = [kb[i].elapsed_time(ke[i]) for i in range(args.steps)]
    states = torch.diff(stats_hist[:, 0]).cpu().numpy().astype(np.float64)
    costs = cost_hist.cpu().numpy()

    value = E * H / (ms_per_step / 1e3)
    if w["kind"] == "arm":
        f_state = arm_state_flops(d, len(w["sph_link"]), w["obs_spheres"].shape[0], w["obs_boxes"].shape[0], d)
    else:
        f_state = point_state_flops(w["circles"].shape[0], w["boxes"].shape[0], d)
    k_ms = float(np.mean(kernel_ms))
    st = float(np.mean(states))
    achieved = st * f_state / (k_ms / 1e3) / 1e12
    traffic, traffic_src = None, None
    if args.workload in MEASURED_TRAFFIC and not args.opt:
        tb, fp, src = MEASURED_TRAFFIC[args.workload]
        if fp == kernel_fingerprint():
            traffic, traffic_src = tb, src
    out = {
        "metric": "edge-states checked/sec (7-DoF, N=2048)",
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
                     "kernel": "k_interior (early-exit interior edge checker)",
                     "kernel_ms": k_ms, "states_evaluated_per_launch": st, "flop_per_state": f_state,
                     "states_evaluated_frac": st / (E * H)},
        "edge_opts": {k: int(getattr(pl.opts, k)) for k in ("mode", "states_per_iter", "blocks_per_cu",
                                                               "sphere_chunks")},
        "mean_path_cost": float(np.mean(costs)),
        "wall_s": wall,
    }
    if not args.no_cpu:
        out["cpu_baseline"] = cpu_baseline(w, min_seconds=args.cpu_seconds)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
