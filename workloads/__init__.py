"""Seeded synthetic workloads for the layered-graph planner.

This module only draws inputs: obstacle scenes, serial-arm models, start and
goal configurations and random cost tensors.  It holds none of the planner's
arithmetic (no sampling of waypoints, no interpolation, no collision test, no
value iteration), so both the FP64 reference in ``oracle/`` and the HIP path
can take their inputs from here without sharing any of the computation.

The paper evaluates on MotionBenchMaker and on Sturtevant's 2D street maps;
neither dataset is available, so the scenes below stand in for them with the
shapes given by the five workloads:

* ``2d-small``  : 2D point robot in [-10,10]^2, 15 circles (centres uniform,
  radius U(1,2)), start (-9,-9), goal (9,9), M=4, N=64, H=8.
* ``2d-large``  : 2D point robot, 50 circles (radius U(0.5,1.0), a reading:
  the workload gives no circle radius) + 20 axis-aligned boxes (half-extents
  U(0.3,1.5) per axis), M=16, N=1024, H=32.
* ``arm7``      : 7-DoF serial arm with seeded standard-DH parameters (link
  lengths a_i ~ U(0.1,0.4) m, offsets d_i ~ U(0,0.1) m, twists drawn from
  {-pi/2, 0, +pi/2}), 40 collision spheres of radius 0.05 m spread over the
  links in proportion to link length, 15 sphere + 15 box obstacles with sizes
  U(0.05,0.2) m and centres uniform in [-1,1]^3, joint box [-pi,pi]^7,
  M=8, N=2048, H=16.
* ``arm7-n4096``: the arm7 scene at N=4096 (surrogate workload).
* ``3d-point``  : 3D point robot in [-10,10]^3, 40 spheres (radius U(1,2))
  + 10 axis-aligned boxes (half-extents U(0.5,1.5)), start (-9,-9,-9), goal
  (9,9,9), M=6, N=256, H=16 (the three-dimensional point case of the
  collision kernels).

Every array is float32 (int32 for indices), the precision the planner stores.
A scene is identified by an integer seed; which seeds give a collision-free
start and goal is decided by ``oracle/select_scenes.py`` (it needs the
collision model, which does not belong here) and stored in
``valid_scenes.json`` next to this file.
"""
from __future__ import annotations

import json
import math
import os

import numpy as np

PI32 = float(np.float32(math.pi))

# Edge penalty: edge cost = length + PENALTY * collision flag.
PENALTY = 1.0e3

_HERE = os.path.dirname(os.path.abspath(__file__))
VALID_SCENES_PATH = os.path.join(_HERE, "valid_scenes.json")


def _rng(*key: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(list(key)))


# --------------------------------------------------------------------------- #
# problem shapes
# --------------------------------------------------------------------------- #
WORKLOADS = {
    "2d-small": dict(kind="point2d", d=2, M=4, N=64, H=8, n_circles=15, r_circ=(1.0, 2.0),
                     n_boxes=0, h_box=(0.3, 1.5)),
    "2d-large": dict(kind="point2d", d=2, M=16, N=1024, H=32, n_circles=50, r_circ=(0.5, 1.0),
                     n_boxes=20, h_box=(0.3, 1.5)),
    "3d-point": dict(kind="point", d=3, M=6, N=256, H=16, n_spheres=40, r_sph=(1.0, 2.0), n_boxes=10,
                     h_box=(0.5, 1.5)),
    "arm7": dict(kind="arm", d=7, M=8, N=2048, H=16, n_obs_spheres=15, n_obs_boxes=15),
    "arm7-n4096": dict(kind="arm", d=7, M=8, N=4096, H=16, n_obs_spheres=15, n_obs_boxes=15),
}


def box_limits(kind: str, d: int):
    """Sampling box (lo, hi) as float32 arrays."""
    if kind in ("point2d", "point"):
        lo = np.full(d, -10.0, np.float32)
        hi = np.full(d, 10.0, np.float32)
    else:
        lo = np.full(d, -PI32, np.float32)
        hi = np.full(d, PI32, np.float32)
    return lo, hi


# --------------------------------------------------------------------------- #
# 2D scenes
# --------------------------------------------------------------------------- #
def scene_2d(seed: int, n_circles: int, r_circ=(1.0, 2.0), n_boxes: int = 0,
             h_box=(0.3, 1.5), extent: float = 10.0):
    """Circles [n,3] = (cx, cy, r) and boxes [n,4] = (cx, cy, hx, hy), centres
    uniform in [-extent, extent]^2."""
    g = _rng(seed, 2)
    cc = g.uniform(-extent, extent, size=(n_circles, 2))
    rr = g.uniform(r_circ[0], r_circ[1], size=(n_circles, 1))
    circles = np.concatenate([cc, rr], axis=1).astype(np.float32)
    bc = g.uniform(-extent, extent, size=(n_boxes, 2))
    bh = g.uniform(h_box[0], h_box[1], size=(n_boxes, 2))
    boxes = np.concatenate([bc, bh], axis=1).astype(np.float32).reshape(n_boxes, 4)
    return circles, boxes


START_2D = np.array([-9.0, -9.0], np.float32)
GOAL_2D = np.array([9.0, 9.0], np.float32)


def scene_3d(seed: int, n_spheres: int, r_sph=(1.0, 2.0), n_boxes: int = 0, h_box=(0.5, 1.5),
             extent: float = 10.0):
    """Spheres [n,4] = (c, r) and boxes [n,6] = (c, h), centres uniform in
    [-extent, extent]^3."""
    g = _rng(seed, 3)
    sc = g.uniform(-extent, extent, size=(n_spheres, 3))
    sr = g.uniform(r_sph[0], r_sph[1], size=(n_spheres, 1))
    spheres = np.concatenate([sc, sr], axis=1).astype(np.float32)
    bc = g.uniform(-extent, extent, size=(n_boxes, 3))
    bh = g.uniform(h_box[0], h_box[1], size=(n_boxes, 3))
    boxes = np.concatenate([bc, bh], axis=1).astype(np.float32).reshape(n_boxes, 6)
    return spheres, boxes


START_3D = np.array([-9.0, -9.0, -9.0], np.float32)
GOAL_3D = np.array([9.0, 9.0, 9.0], np.float32)


# --------------------------------------------------------------------------- #
# 7-DoF arm
# --------------------------------------------------------------------------- #
def arm_robot(seed: int, n_joints: int = 7, n_spheres: int = 40, sphere_r: float = 0.05):
    """Standard-DH arm: dh[J,4] = (a, alpha, d, theta_offset); collision spheres
    given by (link index 1..J, fraction t along the link from frame origin
    o_{i-1} to o_i, radius)."""
    g = _rng(seed, 7)
    a = g.uniform(0.1, 0.4, size=n_joints)
    dd = g.uniform(0.0, 0.1, size=n_joints)
    alpha = g.choice(np.array([-math.pi / 2, 0.0, math.pi / 2]), size=n_joints)
    theta0 = np.zeros(n_joints)
    dh = np.stack([a, alpha, dd, theta0], axis=1).astype(np.float32)
    # spheres per link in proportion to link length, largest-remainder rounding
    length = np.hypot(dh[:, 0].astype(np.float64), dh[:, 2].astype(np.float64))
    quota = n_spheres * length / length.sum()
    count = np.floor(quota).astype(np.int64)
    order = np.argsort(-(quota - count), kind="stable")
    for i in order[: n_spheres - int(count.sum())]:
        count[i] += 1
    link, tt = [], []
    for i in range(n_joints):
        for j in range(count[i]):
            link.append(i + 1)
            tt.append((j + 0.5) / count[i])
    sph_link = np.array(link, np.int32)
    sph_t = np.array(tt, np.float32)
    sph_r = np.full(n_spheres, sphere_r, np.float32)
    return dh, sph_link, sph_t, sph_r


def arm_obstacles(seed: int, n_spheres: int = 15, n_boxes: int = 15, extent: float = 1.0):
    """Sphere obstacles [n,4] = (cx, cy, cz, r) and boxes [n,6] = (cx, cy, cz,
    hx, hy, hz), centres uniform in [-extent, extent]^3, sizes U(0.05, 0.2)."""
    g = _rng(seed, 3)
    sc = g.uniform(-extent, extent, size=(n_spheres, 3))
    sr = g.uniform(0.05, 0.2, size=(n_spheres, 1))
    bc = g.uniform(-extent, extent, size=(n_boxes, 3))
    bh = g.uniform(0.05, 0.2, size=(n_boxes, 3))
    spheres = np.concatenate([sc, sr], axis=1).astype(np.float32)
    boxes = np.concatenate([bc, bh], axis=1).astype(np.float32)
    return spheres, boxes


def arm_start_goal(seed: int, k: int, d: int = 7):
    """k-th candidate (start, goal) pair of joint configurations, uniform in
    [-pi, pi]^d."""
    g = _rng(seed, 1000 + k)
    q = g.uniform(-math.pi, math.pi, size=(2, d)).astype(np.float32)
    return q[0].copy(), q[1].copy()


# --------------------------------------------------------------------------- #
# random cost tensors (min-plus sweep tests)
# --------------------------------------------------------------------------- #
def random_costs(seed: int, M: int, N: int, G: int = 1, p_inf: float = 0.0,
                 p_tie: float = 0.0, lo: float = 0.0, hi: float = 10.0):
    """C_s[N], C_h[M-1,N,N], C_l[N,G] float32.  ``p_inf`` of the entries are
    +inf (absent edges); ``p_tie`` of them are snapped to a coarse grid so that
    exact ties occur."""
    g = _rng(seed, 11)

    def draw(shape):
        x = g.uniform(lo, hi, size=shape)
        if p_tie > 0:
            snap = g.random(size=shape) < p_tie
            x = np.where(snap, np.round(x), x)
        if p_inf > 0:
            x = np.where(g.random(size=shape) < p_inf, np.inf, x)
        return x.astype(np.float32)

    return draw((N,)), draw((max(M - 1, 0), N, N)), draw((N, G))


# --------------------------------------------------------------------------- #
# assembled workloads
# --------------------------------------------------------------------------- #
def load_valid_scenes():
    with open(VALID_SCENES_PATH) as f:
        return json.load(f)


def make_workload(name: str, scene: int = 0, *, seed: int | None = None, sg: int | None = None,
                  M: int | None = None, N: int | None = None, H: int | None = None,
                  penalty: float = PENALTY):
    """Assemble a workload as a dict of numpy arrays and scalars.

    ``scene`` indexes the list of validated scene seeds for the workload (see
    ``valid_scenes.json``); ``seed`` / ``sg`` bypass that list.  M, N, H
    override the workload's sizes (used for smaller parity cases)."""
    spec = dict(WORKLOADS[name])
    if seed is None:
        key = "arm7" if spec["kind"] == "arm" else name
        entry = load_valid_scenes()[key][scene]
        seed = int(entry["seed"])
        if sg is None:
            sg = int(entry.get("sg", 0))
    sg = 0 if sg is None else sg
    for k, v in (("M", M), ("N", N), ("H", H)):
        if v is not None:
            spec[k] = v
    d = spec["d"]
    lo, hi = box_limits(spec["kind"], d)
    w = dict(name=name, kind=spec["kind"], seed=int(seed), sg=int(sg), d=d, M=spec["M"], N=spec["N"],
             H=spec["H"], G=1, lo=lo, hi=hi, penalty=float(penalty))
    if spec["kind"] == "point2d":
        circles, boxes = scene_2d(seed, spec["n_circles"], spec["r_circ"], spec["n_boxes"], spec["h_box"])
        w.update(circles=circles, boxes=boxes, q0=START_2D.copy(), goals=GOAL_2D.reshape(1, 2).copy())
    elif spec["kind"] == "point":
        spheres, boxes = scene_3d(seed, spec["n_spheres"], spec["r_sph"], spec["n_boxes"], spec["h_box"])
        w.update(obs_spheres=spheres, obs_boxes=boxes, q0=START_3D.copy(), goals=GOAL_3D.reshape(1, 3).copy())
    else:
        dh, sl, st, sr = arm_robot(seed)
        spheres, boxes = arm_obstacles(seed, spec["n_obs_spheres"], spec["n_obs_boxes"])
        q0, qg = arm_start_goal(seed, sg, d)
        w.update(dh=dh, sph_link=sl, sph_t=st, sph_r=sr, obs_spheres=spheres, obs_boxes=boxes,
                 q0=q0, goals=qg.reshape(1, d))
    return w



# --------------------------------------------------------------------------- #
# batches of independent plans
# --------------------------------------------------------------------------- #
BATCH = dict(n=512, N=(128, 256, 512, 1024, 2048), M=(4, 16), H=16, restart_stages=4)


def batch_specs(n: int = BATCH["n"], seed: int = 0, N_choices=BATCH["N"], M_range=BATCH["M"], H: int = BATCH["H"],
                restart_stages: int = BATCH["restart_stages"]):
    """A seeded batch of independent plans: robot by a fair coin (2D point
    robot on the large 2D scenes, or the 7-DoF arm on its scenes), scene
    uniform over the five validated ones, N uniform over ``N_choices``, M
    uniform over ``M_range`` (inclusive), and the policy uniform over
    ``plain`` (one stage), ``restart`` (``restart_stages`` stages) and
    ``growing`` (from (M-2, N/4) to (M, N): the stages at N/4, N/2 and N,
    then M-1 and M).  Each plan draws its samples with its own key
    (``seed`` field)."""
    rng = np.random.default_rng(np.random.SeedSequence([0x6A7C, seed]))
    specs = []
    for i in range(n):
        arm = bool(rng.integers(0, 2))
        scene = int(rng.integers(0, 5))
        N = int(N_choices[int(rng.integers(0, len(N_choices)))])
        M = int(rng.integers(M_range[0], M_range[1] + 1))
        mode = ("plain", "restart", "growing")[int(rng.integers(0, 3))]
        w = make_workload("arm7" if arm else "2d-large", scene, M=M, N=N, H=H)
        sp = dict(w=w, mode=mode, seed=1000003 * (seed + 1) + i)
        if mode == "plain":
            sp["stages"] = 1
        elif mode == "restart":
            sp["stages"] = restart_stages
        else:
            sp.update(M_min=max(1, M - 2), N_min=max(1, N // 4), stages=5)
        specs.append(sp)
    return specs


# --------------------------------------------------------------------------- #
# paths to shortcut
# --------------------------------------------------------------------------- #
def random_paths(w, B: int, K: int, seed: int = 0, spread: float = 1.0):
    """B seeded paths of K waypoints from the workload's start to its first
    goal: waypoint k is the point k/(K-1) of the way along the straight line
    plus a perturbation uniform in +-spread/2 of the box width per axis,
    clipped to the box (spread 1 gives waypoints anywhere in the box).
    float32 [B][K][d]."""
    rng = np.random.default_rng(np.random.SeedSequence([0x5137, seed]))
    d = int(w["d"])
    lo, hi = np.asarray(w["lo"], np.float64)[:d], np.asarray(w["hi"], np.float64)[:d]
    q0 = np.asarray(w["q0"], np.float64).reshape(d)
    qg = np.asarray(w["goals"], np.float64).reshape(-1, d)[0]
    t = np.linspace(0.0, 1.0, K)[None, :, None]
    base = q0 + t * (qg - q0)
    noise = rng.uniform(-0.5, 0.5, (B, K, d)) * spread * (hi - lo)
    P = np.clip(base + noise, lo, hi)
    P[:, 0], P[:, -1] = q0, qg
    return P.astype(np.float32)


# --------------------------------------------------------------------------- #
# learned collision surrogate: initial parameters and Fourier frequencies
# --------------------------------------------------------------------------- #
SURROGATE = dict(width=256, depth=4, n_freq=16, in_pad=64, batch=8192, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8,
                 n_labels=2_000_000, recall=0.999)


def surrogate_init(seed: int, d: int = 7):
    """Seeded initial parameters of the surrogate MLP (He-normal hidden
    weights, N(0, 1/width) output weights, zero biases) as float32 arrays
    keyed W1, b1, ..., W4, b4, w5, b5, and the Fourier frequency matrix
    B [n_freq][d] ~ N(0, 1)."""
    S = SURROGATE
    rng = _rng(0x5AE, seed)
    W, D, F, I = S["width"], S["depth"], S["n_freq"], S["in_pad"]
    P = {}
    fan = I
    for l in range(1, D + 1):
        P[f"W{l}"] = (rng.standard_normal((W, fan)) * np.sqrt(2.0 / fan)).astype(np.float32)
        P[f"b{l}"] = np.zeros(W, np.float32)
        fan = W
    P["w5"] = (rng.standard_normal(W) * np.sqrt(1.0 / W)).astype(np.float32)
    P["b5"] = np.zeros(1, np.float32)
    Bf = rng.standard_normal((F, d)).astype(np.float32)
    return P, Bf
