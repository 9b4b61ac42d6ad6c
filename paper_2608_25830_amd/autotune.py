"""Launch-shape autotuner for the edge checker and the batched planner.

The knobs only change how the work is spread over the chip, never what is
computed: every candidate gives bit-identical costs and flags (the interior
check of an edge stops at its first colliding state in any order, and a free
edge's cost is its length either way).  The tuner times each candidate on the
caller's own problem with HIP events around the edge check and keeps the
fastest; results are cached in memory and, when a path is given, in a JSON
file keyed by robot group, problem sizes and a hash of the library (entries
of another build of the kernels never match).

Knobs:
  point robots: sphere_chunks 0 (the obstacle bins, on graphs of at least
                1024 tiles whose scene has at most 96 obstacles) with
                blocks_per_cu in {0, 1, 2, 4}, or 2 (every state against every
                obstacle) with states_per_iter in {1, 2, 4, 8} (interior states
                per lane and iteration) and blocks_per_cu in {0 (auto), 1, 2, 4, 8}
  arms:         sphere_chunks 0 (the obstacle-bin filter, when the scene has
                at most 64 obstacles) with blocks_per_cu in {0, 2, 4, 6}, or
                {1, 2, 4} (every robot sphere against every obstacle in one
                pass at 128+ VGPRs, or in chunks at fewer registers and higher
                occupancy) with blocks_per_cu in {0, 1, 2, 3, 4}
"""
from __future__ import annotations

import json
import os
import statistics
import threading

import torch

from . import gtmp as gt

_LOCK = threading.Lock()
_MEM: dict[str, dict] = {}


def _pow2_bucket(n: int) -> int:
    b = 1
    while b < n:
        b <<= 1
    return b


_LIB_TAG: list[str] = []


def library_tag() -> str:
    """First 12 hex digits of the SHA-256 of the loaded libgtmp.so: a cached
    timing is only reused by the kernels it was measured on."""
    if not _LIB_TAG:
        import hashlib
        with open(gt.LIB_PATH, "rb") as f:
            _LIB_TAG.append(hashlib.sha256(f.read()).hexdigest()[:12])
    return _LIB_TAG[0]


def problem_key(w) -> str:
    """Robot group, DoF, robot spheres, obstacles, H, M and the power-of-two
    bucket of N (the quantities that decide which launch shape wins), and
    the library the timings belong to."""
    if w["kind"] in ("point2d", "point"):
        grp = f"point{int(w['d'])}"
        sph, box = (w["circles"], w["boxes"]) if w["kind"] == "point2d" else (w["obs_spheres"], w["obs_boxes"])
        nob = f"{len(sph)}+{len(box)}"
        ks = 1
    else:
        grp = f"arm{int(w['d'])}"
        nob = f"{len(w['obs_spheres'])}+{len(w['obs_boxes'])}"
        ks = len(w["sph_r"])
    return (f"{grp}:K{ks}:obs{nob}:H{int(w['H'])}:M{int(w['M'])}:N{_pow2_bucket(int(w['N']))}"
            f":lib{library_tag()}")


def candidates(w) -> list[dict]:
    if w["kind"] in ("point2d", "point"):
        bins = [dict(states_per_iter=0, sphere_chunks=0, blocks_per_cu=b) for b in (0, 1, 2, 4)]
        return bins + [dict(states_per_iter=s, sphere_chunks=2, blocks_per_cu=b) for s in (1, 2, 4, 8)
                       for b in (0, 1, 2, 4, 8)]
    bins = [dict(states_per_iter=0, sphere_chunks=0, blocks_per_cu=b) for b in (0, 2, 4, 6)]
    return bins + [dict(states_per_iter=0, sphere_chunks=c, blocks_per_cu=b) for c in (1, 2, 4)
                   for b in (0, 1, 2, 3, 4)]


def apply(opts, cand: dict):
    """Copy a candidate into a gtmp_edge_opts or gtmp_batch_opts struct."""
    opts.states_per_iter = int(cand["states_per_iter"])
    opts.sphere_chunks = int(cand["sphere_chunks"])
    opts.blocks_per_cu = int(cand["blocks_per_cu"])
    return opts


def _load(path):
    if path and os.path.exists(path):
        with open(path) as f:
            return json.load(f)
    return {}


def _save(path, table):
    if not path:
        return
    tmp = path + ".tmp"
    with open(tmp, "w") as f:
        json.dump(table, f, indent=1, sort_keys=True)
    os.replace(tmp, path)


def time_edge_check(pl: "gt.Planner", cand: dict, reps: int = 3, warmup: int = 1) -> float:
    """Median milliseconds of gtmp_edge_check_cost for one candidate on the
    planner's current samples."""
    apply(pl.opts, cand)
    t0, t1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    times = []
    for r in range(warmup + reps):
        t0.record()
        pl.check()
        t1.record()
        t1.synchronize()
        if r >= warmup:
            times.append(t0.elapsed_time(t1))
    return statistics.median(times)


def tune_edge(w, cache_path: str | None = None, reps: int = 3, cands: list[dict] | None = None,
              planner: "gt.Planner | None" = None, force: bool = False) -> dict:
    """Best launch shape for the edge check of workload ``w``: returns the
    candidate dict plus its time (``ms``) and the whole timing table."""
    key = problem_key(w)
    with _LOCK:
        if not force:
            if key in _MEM:
                return _MEM[key]
            table = _load(cache_path)
            if key in table:
                _MEM[key] = table[key]
                return table[key]
    pl = planner or gt.Planner(w)
    pl.sample(int(w["seed"]), 0)
    res = []
    for c in cands or candidates(w):
        res.append((time_edge_check(pl, c, reps), c))
    ms, best = min(res, key=lambda x: x[0])
    entry = dict(best, ms=ms, table=[dict(c, ms=t) for t, c in res])
    with _LOCK:
        _MEM[key] = entry
        if cache_path:
            table = _load(cache_path)
            table[key] = entry
            _save(cache_path, table)
    return entry


def tune_batch(specs, cache_path: str | None = None, reps: int = 2) -> dict:
    """Batch options from per-group tuning: the arm group (the dominant cost
    when present) sets sphere_chunks and blocks_per_cu, the 2D point group
    sets states_per_iter.  Each group is tuned on its largest plan."""
    best = dict(states_per_iter=0, sphere_chunks=0, blocks_per_cu=0)
    groups: dict[str, dict] = {}
    for sp in specs:
        w = sp["w"]
        g = "arm" if w["kind"] == "arm" else "point"
        size = int(w["M"]) * int(w["N"]) ** 2
        if g not in groups or size > groups[g][0]:
            groups[g] = (size, w)
    if "point" in groups:
        e = tune_edge(groups["point"][1], cache_path, reps)
        best["states_per_iter"] = e["states_per_iter"]
        best["blocks_per_cu"] = e["blocks_per_cu"]
    if "arm" in groups:
        e = tune_edge(groups["arm"][1], cache_path, reps)
        best["sphere_chunks"] = e["sphere_chunks"]
        best["blocks_per_cu"] = e["blocks_per_cu"]
    return best
