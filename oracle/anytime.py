"""Oracle of the two anytime policies (Alg. 1 anytime-gtmp and ao-gtmp;
Sec. IV-C..E) with one homotopy class (|K| = 1), and of the growing-budget
sampler (Alg. 1 expand-samples).

TEST INFRASTRUCTURE (see the package docstring).  Plain Python loops over
stages, layers and slots; the arithmetic of each step is the C oracle's.
"""
from __future__ import annotations

import numpy as np

import oracle as O
import oracle.simplify as OSI

MAX_ATTEMPTS = 16384
# biased heuristic half: the closest pairs scored by the surrogate per new
# slot of a layer
BIAS_CANDIDATES = 4


def _bound(c, penalty):
    """The cost bound of the informed set as the FP32 value the sampler uses;
    None when there is no bound yet (no path, or only paths through a failed
    edge)."""
    c32 = np.float32(c)
    if not np.isfinite(c32) or c32 >= np.float32(penalty):
        return None
    return c32


def informed_draw(w, c, seed, stage, m, n):
    """One draw of the uniform half for slot (m, n): the informed set
    X_f(c) (Sec. IV-E) intersected with the box; uniform in the box without a
    bound.  Returns (x float32[d], attempts); attempts is 0 for an unbounded
    draw and -1 when the attempt cap was reached (x is then the centre)."""
    d = w["d"]
    out = np.zeros(d, np.float32)
    lo, hi = O._f32(w["lo"]), O._f32(w["hi"])
    q0, qg = O._f32(w["q0"]), O._f32(np.asarray(w["goals"])[0])
    cc = np.inf if c is None else float(c)
    a = O.lib().or_sample_informed(d, O._ptr(lo, O._fp), O._ptr(hi, O._fp), O._ptr(q0, O._fp), O._ptr(qg, O._fp),
                                   cc, float(w["penalty"]), seed, stage, m, n, MAX_ATTEMPTS, O._ptr(out, O._fp))
    return out, a


def informed_params(d, q0, qg, c):
    centre = np.zeros(d, np.float32)
    H = np.zeros(d * d, np.float32)
    r1, r2, cmin = (np.zeros(1, np.float32) for _ in range(3))
    q0, qg = O._f32(q0), O._f32(qg)
    O.lib().or_informed_params(d, O._ptr(q0, O._fp), O._ptr(qg, O._fp), float(c), O._ptr(centre, O._fp),
                               O._ptr(H, O._fp), O._ptr(r1, O._fp), O._ptr(r2, O._fp), O._ptr(cmin, O._fp))
    return centre, H.reshape(d, d), float(r1[0]), float(r2[0]), float(cmin[0])


def informed_proposal(w, c):
    """Proposal region of the uniform half for the bound c: (clipped, c_lo,
    c_hi) with clipped = True for the hyperspheroid's bounding box clipped to
    the sampling box (bounds c_lo, c_hi), False for its own frame box."""
    d = w["d"]
    centre, H, r1, r2, _ = informed_params(d, w["q0"], np.asarray(w["goals"])[0], c)
    lo, hi = O._f32(w["lo"]), O._f32(w["hi"])
    c_lo, c_hi = np.zeros(d, np.float32), np.zeros(d, np.float32)
    H = np.ascontiguousarray(H.ravel(), np.float32)
    k = O.lib().or_informed_proposal(d, O._ptr(lo, O._fp), O._ptr(hi, O._fp), O._ptr(centre, O._fp),
                                     O._ptr(H, O._fp), r1, r2, O._ptr(c_lo, O._fp), O._ptr(c_hi, O._fp))
    return bool(k), c_lo, c_hi


def coin_heuristic(seed, stage, m, n):
    return bool(O.lib().or_coin_heuristic(seed, stage, m, n))


def pair_order(prev, nxt):
    """Pairs (a, b) of prev x nxt ranked by FP32 squared distance, ties by
    (a, b): indices a * len(nxt) + b in rank order."""
    prev, nxt = O._f32(prev), O._f32(nxt)
    nu, nv = prev.shape[0], nxt.shape[0]
    d2 = np.zeros((nu, nv), np.float32)
    O.lib().or_pair_d2_all(prev.shape[1], nu, O._ptr(prev, O._fp), nv, O._ptr(nxt, O._fp), O._ptr(d2, O._fp))
    return np.argsort(d2.ravel(), kind="stable")


def _free_candidates(order, prev, nxt, n_new, bias, trace=None):
    """Biased heuristic half: of the BIAS_CANDIDATES * n_new closest pairs,
    the ones whose FP32 midpoint the surrogate scores at or below the
    threshold (logit <= tau), in rank order."""
    import oracle.surrogate as S
    P, Bf, tau = bias
    nv = nxt.shape[0]
    k = min(order.size, BIAS_CANDIDATES * n_new)
    ab = [divmod(int(order[r]), nv) for r in range(k)]
    X = np.stack([(prev[a] + nxt[b]) * np.float32(0.5) for a, b in ab]) if ab else np.zeros((0, prev.shape[1]))
    z = S.logits_of_states(P, Bf, X.astype(np.float64)) if ab else np.zeros(0)
    if trace is not None:
        trace.append(z)
    return [int(order[r]) for r in range(k) if z[r] <= tau]


def expand_samples(w, Q, M, N, c_best, seed, stage, bias=None, trace=None):
    """Alg. 1 expand-samples.  Q is a list of M float32 arrays [n_m][d]
    (layers may be empty); returns the list grown to N samples per layer,
    layers processed in increasing m.  ``bias`` = (params, fourier, tau):
    the heuristic half takes, in rank order, only pairs whose midpoint the
    surrogate predicts free (see _free_candidates); ``trace`` (a list)
    collects the candidates' logits of each layer."""
    d = w["d"]
    q0 = O._f32(w["q0"]).reshape(1, d)
    goals = O._f32(w["goals"]).reshape(-1, d)
    c = _bound(c_best, w["penalty"])
    Q = [np.asarray(q, np.float32).reshape(-1, d).copy() for q in Q]
    for m in range(M):
        prev = q0 if m == 0 else Q[m - 1]
        nxt = goals if m == M - 1 else Q[m + 1]
        heuristic_ok = c is not None and prev.shape[0] > 0 and nxt.shape[0] > 0
        order = pair_order(prev, nxt) if heuristic_ok else None
        nv = nxt.shape[0]
        n_old = Q[m].shape[0]
        if heuristic_ok and bias is not None:
            order = np.asarray(_free_candidates(order, prev, nxt, N - n_old, bias, trace), np.int64)
        new = []
        h = 0
        for n in range(n_old, N):
            heur = heuristic_ok and coin_heuristic(seed, stage, m, n)
            if heur:
                rank = h
                h += 1
                if rank < order.size:
                    a, b = divmod(int(order[rank]), nv)
                    new.append((prev[a] + nxt[b]) * np.float32(0.5))
                    continue
            x, _ = informed_draw(w, c, seed, stage, m, n)
            new.append(x)
        if new:
            Q[m] = np.concatenate([Q[m], np.stack(new).astype(np.float32)], axis=0)
    return Q


def _plan_on(w, Qarr, lp=None, seed=0, stage=0):
    """The plain plan on samples Qarr; with ``lp`` (oracle.rrtc.LPOpts) the
    RRT-Connect repair (keyed by seed and stage) runs on the straight-line
    costs before the sweep."""
    ww = dict(w)
    ww["M"], ww["N"] = Qarr.shape[0], Qarr.shape[1]
    r = O.plan(ww, Q=Qarr)
    if lp is None:
        return r
    import oracle.rrtc as RR
    M, N = Qarr.shape[0], Qarr.shape[1]
    G = np.asarray(ww["goals"]).reshape(-1, ww["d"]).shape[0]
    flat = np.concatenate([np.asarray(x).ravel() for x in r["cost"]])
    fflag = np.concatenate([np.asarray(x).ravel() for x in r["flag"]])
    cost, flag, info = RR.repair(ww, Qarr, flat, fflag, lp, seed, stage)
    cost3 = O.split_edges(cost, M, N, G)
    V, A, Vs, a_s = O.minplus(*cost3)
    idx, wp, c, rc = O.extract(A, a_s, Vs, Qarr, ww["q0"], ww["goals"])
    r.update(cost=cost3, flag=O.split_edges(flag, M, N, G), V=V, A=A, Vs=Vs, a_s=a_s, idx=idx, wp=wp,
             path_cost=c, no_path=rc, lp_info=info)
    return r


def _shortcut(w, r):
    """simp() of the stage path r (oracle/simplify.py): (kept waypoints or
    None, shortcut length, +inf when no chain passes)."""
    wp = np.asarray(r["wp"], np.float32)
    kept, c, _, _ = OSI.simplify(O.Model(w), wp, int(w["H"]))
    return (None, np.inf) if kept is None else (wp[kept], c)


def plan_restart(w, stages, seed, simplify=False, lp=None):
    """Anytime-GTMP (Alg. 1; Sec. IV-D) with |K| = 1: stage s plans on the
    samples of key (seed, s); the archive keeps the lowest cost (strictly
    lower replaces, so ties keep the earlier stage).  With ``simplify`` a
    stage path whose cost is below the archived cost is stored shortcut
    (Alg. 1: the archive entry becomes simp() of the path), and only when a
    shortcut chain exists."""
    best = dict(cost=np.inf, stage=-1, idx=None)
    per_stage = []
    for s in range(stages):
        Q = O.sample_layers(w["M"], w["N"], w["d"], w["lo"], w["hi"], seed, s)
        r = _plan_on(w, Q, lp, seed, s)
        per_stage.append(r["path_cost"])
        if r["path_cost"] < best["cost"]:
            if not simplify:
                best = dict(cost=r["path_cost"], stage=s, idx=r["idx"].copy(), M=w["M"], N=w["N"])
                continue
            wp, c = _shortcut(w, r)
            if wp is not None:
                best = dict(cost=c, stage=s, idx=r["idx"].copy(), M=w["M"], N=w["N"], wp=wp)
    return best, per_stage


def growing_schedule(M_min, M_max, N_min, N_max, max_stages):
    """(M, N, n_old) of each stage: N doubles (capped) while N < N_max, then M
    grows by one per stage with a fresh epoch (n_old = 0); the loop ends after
    the stage at (M_max, N_max) or at the stage cap."""
    out = []
    M, N, n_old = M_min, N_min, 0
    for _ in range(max_stages):
        out.append((M, N, n_old))
        if M >= M_max and N >= N_max:
            break
        if N < N_max:
            n_old, N = N, min(2 * N, N_max)
        else:
            M, n_old = M + 1, 0
    return out


def plan_growing(w, M_min, M_max, N_min, N_max, max_stages, seed, bias=None, trace=None, simplify=False, lp=None):
    """AO-GTMP (Alg. 1; Sec. IV-E): expand the samples under the current
    cost bound, plan, keep the best, grow the budget (``bias`` as in
    expand_samples).  With ``simplify`` every stage path is shortcut first
    (Alg. 1: P_i = simp(gtmp(...))) and the shortcut lengths are compared,
    so the best shortcut length bounds the informed sampler.  ``lp`` runs the
    RRT-Connect repair in every stage (see _plan_on)."""
    d = w["d"]
    best = dict(cost=np.inf, stage=-1, idx=None)
    per_stage, stages = [], []
    Q = None
    for s, (M, N, n_old) in enumerate(growing_schedule(M_min, M_max, N_min, N_max, max_stages)):
        if n_old == 0:
            Q = [np.zeros((0, d), np.float32) for _ in range(M)]
        Q = expand_samples(w, Q, M, N, best["cost"], seed, s, bias, trace)
        Qarr = np.stack(Q).astype(np.float32)
        r = _plan_on(w, Qarr, lp, seed, s)
        c, wp = r["path_cost"], None
        if simplify:
            ww = dict(w)
            ww["M"], ww["N"] = M, N
            wp, c = _shortcut(ww, r)
        per_stage.append(c)
        stages.append(dict(M=M, N=N, Q=Qarr, cost=c, bound=best["cost"]))
        if c < best["cost"]:
            best = dict(cost=c, stage=s, idx=r["idx"].copy(), M=M, N=N, wp=wp)
    return best, per_stage, stages
