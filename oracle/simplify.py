"""Oracle of path simplification (simp() of Alg. 1 ao-gtmp; Sec. IV-E).

TEST INFRASTRUCTURE (see the package docstring).

The paper leaves simp() undefined.  Reading used on both sides: for a path
with waypoints w_0 .. w_{K-1}, the shortcut i -> j (j > i) is valid iff the
straight segment w_i -> w_j passes the discrete straight-line check with
H_ij = (j - i)(H - 1) + 1 states at t = h / (H_ij - 1), h = 0 .. H_ij - 1
(the spacing of the plan's own edges; a consecutive pair is checked with H
states, as the plan checked it), a state colliding iff its signed distance is
<= 0.  The simplified path is the shortest chain from w_0 to w_{K-1} over
valid shortcuts (Euclidean lengths; ties to the lowest next index).
"""
from __future__ import annotations

import numpy as np

import oracle as O


def shortcut_table(model, wp, H):
    """valid [K][K] (upper triangle), minsd [K][K] of every shortcut."""
    wp = np.asarray(wp, np.float32)
    K = wp.shape[0]
    valid = np.zeros((K, K), bool)
    minsd = np.full((K, K), np.inf)
    for i in range(K):
        for j in range(i + 1, K):
            Hij = (j - i) * (H - 1) + 1
            _, sd, f = O.edge(model, Hij, wp[i], wp[j])
            valid[i, j] = f == 0
            minsd[i, j] = sd
    return valid, minsd


def shortest_over(valid, wp):
    """Shortest chain 0 -> K-1 using valid shortcuts: (indices, length)."""
    wp = np.asarray(wp, np.float64)
    K = wp.shape[0]
    best = np.full(K, np.inf)
    nxt = np.full(K, -1)
    best[K - 1] = 0.0
    for i in range(K - 2, -1, -1):
        for j in range(i + 1, K):
            if not valid[i, j] or not np.isfinite(best[j]):
                continue
            c = np.linalg.norm(wp[j] - wp[i]) + best[j]
            if c < best[i]:
                best[i], nxt[i] = c, j
    if not np.isfinite(best[0]):
        return None, np.inf
    idx = [0]
    while idx[-1] != K - 1:
        idx.append(int(nxt[idx[-1]]))
    return idx, float(best[0])


def simplify(model, wp, H):
    valid, minsd = shortcut_table(model, wp, H)
    idx, cost = shortest_over(valid, wp)
    return idx, cost, valid, minsd
