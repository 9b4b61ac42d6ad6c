"""Comparison rules between the HIP path and the FP64 oracle.

* Edge flags must match exactly, except on edges whose oracle minimum signed
  distance over the edge's states is within BAND of zero (counted).
* Costs of edges whose flags match agree within REL relative.
* Path cost: within REL of the oracle optimum.  When excused edges exist the
  optimum is bracketed by two oracle runs (every excused edge free / every
  excused edge failed), both computed from oracle values only.
* Path indices: equal at every step up to the first near-tie, i.e. where the
  oracle's runner-up exceeds its minimum by more than REL * |cost|.
"""
from __future__ import annotations

import numpy as np

BAND = 1e-5
REL = 1e-5

# figures recorded by tests, printed at the end of the run (tests/conftest.py)
NOTES: list = []


def note(*a):
    NOTES.append(" ".join(str(x) for x in a))


def flat(Cs, Ch, Cl):
    return np.concatenate([np.ravel(Cs), np.ravel(Ch), np.ravel(Cl)])


def compare_edges(gpu_cost, gpu_flag, or_cost, or_minsd, or_flag, band=BAND, rel=REL):
    """All arguments flat [E].  Returns a dict with counts; asserts the rules."""
    gpu_cost = np.asarray(gpu_cost, np.float64)
    or_cost = np.asarray(or_cost, np.float64)
    gpu_flag = np.asarray(gpu_flag).astype(np.int64)
    or_flag = np.asarray(or_flag).astype(np.int64)
    mism = gpu_flag != or_flag
    near = np.abs(np.asarray(or_minsd)) <= band
    bad = mism & ~near
    assert not bad.any(), f"{bad.sum()} flag mismatches outside the band, first at {np.flatnonzero(bad)[:10]}"
    ok = ~mism
    fin = ok & np.isfinite(or_cost)
    err = np.abs(gpu_cost[fin] - or_cost[fin])
    lim = rel * np.maximum(np.abs(or_cost[fin]), 1e-30)
    assert np.all(err <= lim), f"cost mismatch: worst rel {np.max(err / np.maximum(np.abs(or_cost[fin]), 1e-30))}"
    inf = ok & ~np.isfinite(or_cost)
    assert np.all(~np.isfinite(gpu_cost[inf]))
    return dict(edges=int(gpu_cost.size), excused=int(mism.sum()), near_band=int(near.sum()),
                failed=int(or_flag.sum()))


def excused_bounds(orc, or_cost3, or_len3, excused3, penalty):
    """Oracle optimum with every excused edge set free (low) and failed (high)."""
    lo, hi = [], []
    for c, ln, ex in zip(or_cost3, or_len3, excused3):
        c_lo = np.where(ex, ln, c)
        c_hi = np.where(ex, ln + penalty, c)
        lo.append(c_lo)
        hi.append(c_hi)
    return orc.minplus(*lo)[2], orc.minplus(*hi)[2]


def path_cost_from_oracle(or_cost3, idx):
    Cs, Ch, Cl = or_cost3
    M = Ch.shape[0] + 1
    c = Cs[idx[0]]
    for m in range(M - 1):
        c += Ch[m, idx[m], idx[m + 1]]
    c += Cl[idx[M - 1], idx[M]]
    return c


def check_path_indices(or_cost3, V, idx_or, idx_gpu, cost, rel=REL):
    """Indices must agree until the first near-tie of the oracle's choice."""
    Cs, Ch, Cl = or_cost3
    M = Ch.shape[0] + 1
    tol = rel * max(abs(cost), 1.0)
    rows = [Cs + V[0]]
    for m in range(M):
        if m < M - 1:
            rows.append(Ch[m, idx_or[m]] + V[m + 1])
        else:
            rows.append(Cl[idx_or[m]])
    compared = 0
    for step, r in enumerate(rows):
        r = np.asarray(r, np.float64)
        best = r[idx_or[step]]
        others = np.delete(r, idx_or[step])
        if others.size and np.min(others) - best <= tol:
            break
        assert idx_gpu[step] == idx_or[step], f"index mismatch at step {step}: {idx_gpu[step]} vs {idx_or[step]}"
        compared += 1
    return compared


# Surrogate logits (BF16 network, FP32 accumulation) against the FP64 oracle
# with the same BF16 rounding points: see tests/test_gpu_surrogate.py for how
# these bounds follow from the arithmetic.
Z_TOL = 1e-4
Z_LOOSE = 1e-2


def check_logits(z, z_or):
    scale = np.maximum(1.0, np.abs(z_or))
    err = np.abs(np.asarray(z, np.float64) - z_or) / scale
    assert np.all(err <= Z_LOOSE), err.max()
    assert np.mean(err <= Z_TOL) >= 0.97, np.mean(err <= Z_TOL)
    return err
