"""Oracle of the RRT-Connect local planner (Sec. III, LP(x, y; s, ell) with
the query ellipsoid; the construction in the proof of the local-planner reach
proposition of the appendix) and of the repair pass that runs it on the edges
whose straight line failed.

TEST INFRASTRUCTURE (see the package docstring).  The planner itself is
``or_rrtc`` in gtmp_oracle.c (its header states every decision); this module
wraps it and applies it to a sampled graph.
"""
from __future__ import annotations

import ctypes as C
from dataclasses import dataclass

import numpy as np

import oracle as O
import oracle.anytime as OA

BAND = 1e-5


@dataclass
class LPOpts:
    budget: int = 100       # s: iterations (samples) per call
    cap: int = 512          # nodes per tree
    eta: float = 0.5        # extension step
    res: float = 0.1        # collision states every res along an extension
    ell_factor: float = 1.5  # query ellipsoid major axis = ell_factor |y - x|


def ellipsoid(x, y, ell_factor):
    """(centre, H, r1, r2, ell) of the query ellipsoid E(x, y; ell) as FP32."""
    x, y = O._f32(x), O._f32(y)
    d = x.size
    acc = np.float32(0)
    for i in range(d):
        t = np.float32(y[i] - x[i])
        acc = np.float32(acc + np.float32(t * t))
    ell = np.float32(np.float32(ell_factor) * np.sqrt(acc, dtype=np.float32))
    centre, H, r1, r2, _ = OA.informed_params(d, x, y, ell)
    return centre, H, r1, r2, float(ell)


def sample(w, x, y, ell_factor, seed, stage, e, i):
    """The draw of iteration i of call e (None when no attempt passes)."""
    d = int(w["d"])
    centre, H, r1, r2, _ = ellipsoid(x, y, ell_factor)
    lo, hi = O._f32(w["lo"])[:d], O._f32(w["hi"])[:d]
    q = np.zeros(d, np.float32)
    H = O._f32(H).ravel()
    ok = O.lib().or_rrtc_sample(d, O._ptr(lo, O._fp), O._ptr(hi, O._fp), O._ptr(O._f32(centre), O._fp),
                                O._ptr(H, O._fp), r1, r2, seed, stage, e, i, O._ptr(q, O._fp))
    return q if ok else None


def call(model, w, x, y, opts: LPOpts, seed, stage, e, band=BAND):
    """One call.  Returns a dict: ok, cost, path [n][d], iters, sizes (x tree,
    y tree), near_band, trees [2][cap][d], parents [2][cap]."""
    d = int(w["d"])
    x, y = O._f32(x), O._f32(y)
    lo, hi = O._f32(w["lo"])[:d], O._f32(w["hi"])[:d]
    cap = int(opts.cap)
    path = np.zeros((2 * cap, d), np.float32)
    trees = np.zeros((2, cap, d), np.float32)
    parents = np.full((2, cap), -2, np.int32)
    n_path, iters, near = C.c_int(), C.c_int(), C.c_int()
    sizes = np.zeros(2, np.int32)
    cost = np.zeros(1, np.float64)
    ok = O.lib().or_rrtc(model.ref(), O._ptr(x, O._fp), O._ptr(y, O._fp), O._ptr(lo, O._fp), O._ptr(hi, O._fp),
                         int(opts.budget), cap, float(opts.eta), float(opts.res), float(opts.ell_factor), seed, stage,
                         int(e), band, O._ptr(path, O._fp), C.byref(n_path), O._ptr(cost, O._dp), C.byref(iters),
                         O._ptr(sizes, O._ip), C.byref(near), O._ptr(trees, O._fp), O._ptr(parents, O._ip))
    return dict(ok=bool(ok), cost=float(cost[0]), path=path[:n_path.value].copy(), iters=iters.value,
                sizes=(int(sizes[0]), int(sizes[1])), near_band=bool(near.value), trees=trees, parents=parents)


def batch(model, w, X, Y, ids, opts: LPOpts, seed, stage, band=BAND):
    """Calls over endpoint pairs X[k] -> Y[k] keyed by ids[k] (OpenMP)."""
    d = int(w["d"])
    X, Y = O._f32(X).reshape(-1, d), O._f32(Y).reshape(-1, d)
    n = X.shape[0]
    ids = np.ascontiguousarray(ids, dtype=np.uint32)
    lo, hi = O._f32(w["lo"])[:d], O._f32(w["hi"])[:d]
    ok = np.zeros(n, np.int32)
    cost = np.zeros(n, np.float64)
    iters = np.zeros(n, np.int32)
    sizes = np.zeros((n, 2), np.int32)
    near = np.zeros(n, np.int32)
    npath = np.zeros(n, np.int32)
    if n:
        O.lib().or_rrtc_batch(model.ref(), n, O._ptr(X, O._fp), O._ptr(Y, O._fp), O._ptr(ids, O._up),
                              O._ptr(lo, O._fp), O._ptr(hi, O._fp), int(opts.budget), int(opts.cap), float(opts.eta),
                              float(opts.res), float(opts.ell_factor), seed, stage, band, O._ptr(ok, O._ip),
                              O._ptr(cost, O._dp), O._ptr(iters, O._ip), O._ptr(sizes, O._ip), O._ptr(near, O._ip),
                              O._ptr(npath, O._ip))
    return dict(ok=ok.astype(bool), cost=cost, iters=iters, sizes=sizes, near_band=near.astype(bool), n_path=npath)


def edge_endpoints(w, Q, e):
    """Endpoints of flat edge e (C_s | C_h row-major | C_l)."""
    M, N = Q.shape[0], Q.shape[1]
    goals = O._f32(w["goals"]).reshape(-1, Q.shape[2])
    G = goals.shape[0]
    if e < N:
        return O._f32(w["q0"]), Q[0, e]
    r = e - N
    if r < (M - 1) * N * N:
        m, uv = divmod(r, N * N)
        u, v = divmod(uv, N)
        return Q[m, u], Q[m + 1, v]
    r -= (M - 1) * N * N
    u, g = divmod(r, G)
    return Q[M - 1, u], goals[g]


def repair(w, Q, flat_cost, flat_flag, opts: LPOpts, seed, stage, max_len=np.inf, band=BAND):
    """The repair pass over one sampled graph: every edge whose straight line
    failed (flag 1) with both endpoints collision-free and |y - x| <= max_len
    gets one call; a success replaces its cost by the local path's length
    and its flag by 2.  Returns (cost, flag, info) with info = dict of the
    candidate ids and the per-call outputs, and the ids of candidate edges
    whose endpoint signed distance lies within `band` of zero."""
    model = O.Model(w)
    d = int(w["d"])
    Q = O._f32(Q)
    M, N = Q.shape[0], Q.shape[1]
    goals = O._f32(w["goals"]).reshape(-1, d)
    G = goals.shape[0]
    verts = np.concatenate([O._f32(w["q0"]).reshape(1, d), Q.reshape(-1, d), goals])
    vsd = O.state_sd(model, verts)

    def vid(layer, i):  # -1 = start, M = goals
        return 0 if layer < 0 else (1 + M * N + i if layer == M else 1 + layer * N + i)

    E = flat_cost.size
    ids, X, Y, vband = [], [], [], []
    for e in np.flatnonzero(np.asarray(flat_flag) == 1):
        e = int(e)
        if e < N:
            a, b = vid(-1, 0), vid(0, e)
        elif e < N + (M - 1) * N * N:
            m, uv = divmod(e - N, N * N)
            a, b = vid(m, uv // N), vid(m + 1, uv % N)
        else:
            u, g = divmod(e - N - (M - 1) * N * N, G)
            a, b = vid(M - 1, u), vid(M, g)
        x, y = verts[a], verts[b]
        if abs(vsd[a]) <= band or abs(vsd[b]) <= band:
            vband.append(e)
        if not (vsd[a] > 0 and vsd[b] > 0):
            continue
        if np.sqrt(np.sum((y.astype(np.float64) - x) ** 2)) > max_len:
            continue
        ids.append(e)
        X.append(x)
        Y.append(y)
    ids = np.asarray(ids, np.int64)
    out = batch(model, w, np.asarray(X, np.float32).reshape(-1, d), np.asarray(Y, np.float32).reshape(-1, d),
                ids.astype(np.uint32), opts, seed, stage, band)
    cost = np.array(flat_cost, np.float64, copy=True)
    flag = np.array(flat_flag, np.int32, copy=True)
    cost[ids[out["ok"]]] = out["cost"][out["ok"]]
    flag[ids[out["ok"]]] = 2
    out.update(ids=ids, vertex_band=np.asarray(vband, np.int64))
    assert E == cost.size
    return cost, flag, out
