"""Pick the scene seeds used by the tests and the benchmark.

A scene seed is accepted when the start and the goal are collision-free with
some clearance, which needs the collision model; the generators in
``workloads`` hold none of it, so the choice is made here with the FP64 oracle
only and written to ``workloads/valid_scenes.json``.

Rules (readings, the paper leaves the synthetic scenes open):
* Point-robot workloads (2D and 3D): signed distance of start and goal to
  the obstacles > 0.1.
* Arm: no obstacle within 0.2 m of the base (signed distance of the base
  point > 0.2); for the k-th candidate (start, goal) pair the first k whose
  configurations both have signed distance > 0.01 m and whose joint-space
  distance is at least pi.

Run:  python -m oracle.select_scenes
"""
from __future__ import annotations

import json
import math

import numpy as np

import oracle
import workloads as wl

N_SCENES = 5


def _valid_2d(name, n_want=N_SCENES, max_seed=1000):
    out = []
    for seed in range(max_seed):
        w = wl.make_workload(name, seed=seed)
        m = oracle.Model(w)
        sd = oracle.state_sd(m, np.stack([w["q0"], w["goals"][0]]))
        if sd.min() > 0.1:
            out.append({"seed": seed})
        if len(out) == n_want:
            break
    return out


def _valid_arm(n_want=N_SCENES, max_seed=1000, max_k=200):
    out = []
    for seed in range(max_seed):
        w = wl.make_workload("arm7", seed=seed, sg=0)
        pt = dict(kind="point", d=3, obs_spheres=w["obs_spheres"], obs_boxes=w["obs_boxes"])
        if oracle.state_sd(oracle.Model(pt), np.zeros((1, 3), np.float32))[0] <= 0.2:
            continue
        m = oracle.Model(w)
        for k in range(max_k):
            q0, qg = wl.arm_start_goal(seed, k)
            if np.linalg.norm(qg.astype(np.float64) - q0.astype(np.float64)) < math.pi:
                continue
            sd = oracle.state_sd(m, np.stack([q0, qg]))
            if sd.min() > 0.01:
                out.append({"seed": seed, "sg": k})
                break
        if len(out) == n_want:
            break
    return out


def main():
    res = {"2d-small": _valid_2d("2d-small"), "2d-large": _valid_2d("2d-large"), "arm7": _valid_arm(),
           "3d-point": _valid_2d("3d-point")}
    with open(wl.VALID_SCENES_PATH, "w") as f:
        json.dump(res, f, indent=1)
    print(json.dumps(res))


if __name__ == "__main__":
    main()
