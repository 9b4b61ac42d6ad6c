"""Pins of the path-simplification oracle (oracle/simplify.py): straight line
in free space, a shortcut blocked by an obstacle, enumeration of every
subsequence of waypoints, and the shortcut checks against the textbook
segment-to-circle distance (one-way invariants of a discrete check)."""
import itertools

import numpy as np
import pytest

import oracle
import oracle.simplify as OSI
import workloads as wl


def _model(circles, boxes=None):
    w = wl.make_workload("2d-small", 0)
    w["circles"] = np.asarray(circles, np.float32).reshape(-1, 3)
    w["boxes"] = np.zeros((0, 4), np.float32) if boxes is None else np.asarray(boxes, np.float32).reshape(-1, 4)
    return oracle.Model(w)


def test_free_space_becomes_the_straight_line():
    m = _model(np.zeros((0, 3)))
    wp = np.array([[-5, -5], [-1, 3], [2, -4], [4, 4], [6, 5]], np.float32)
    idx, cost, valid, _ = OSI.simplify(m, wp, 8)
    assert idx == [0, 4]
    assert cost == pytest.approx(np.linalg.norm(wp[4].astype(np.float64) - wp[0]), rel=1e-12)
    assert valid[np.triu_indices(5, 1)].all()


def test_blocked_shortcut_keeps_the_detour():
    m = _model([[0.0, 0.0, 2.0]])
    wp = np.array([[-5, 0], [0, 3], [5, 0]], np.float32)
    idx, cost, valid, minsd = OSI.simplify(m, wp, 8)
    assert not valid[0, 2] and valid[0, 1] and valid[1, 2]
    assert idx == [0, 1, 2]
    assert minsd[0, 2] == pytest.approx(-2.0)  # the segment passes through the centre
    assert cost == pytest.approx(2 * np.hypot(5, 3), rel=1e-12)


def _seg_circle_dist(a, b, c):
    a, b, c = (np.asarray(x, np.float64) for x in (a, b, c))
    ab = b - a
    t = np.clip(np.dot(c - a, ab) / max(np.dot(ab, ab), 1e-300), 0, 1)
    return np.linalg.norm(a + t * ab - c)


@pytest.mark.parametrize("seed", range(4))
def test_dp_equals_enumeration_and_checks_are_one_way_sound(seed):
    rng = np.random.default_rng(seed)
    circles = np.concatenate([rng.uniform(-6, 6, (5, 2)), rng.uniform(0.5, 1.5, (5, 1))], 1)
    m = _model(circles)
    K = 7
    wp = rng.uniform(-8, 8, (K, 2)).astype(np.float32)
    idx, cost, valid, minsd = OSI.simplify(m, wp, 6)
    # one-way invariants of the discrete check against the continuous segment
    for i, j in zip(*np.triu_indices(K, 1)):
        clear = all(_seg_circle_dist(wp[i], wp[j], c[:2]) > c[2] + 1e-9 for c in circles)
        if clear:
            assert valid[i, j]
        if not valid[i, j]:
            assert not clear
    # enumeration of every subsequence 0 < ... < K-1
    best = np.inf
    for r in range(0, K - 1):
        for mid in itertools.combinations(range(1, K - 1), r):
            seq = (0,) + mid + (K - 1,)
            if all(valid[a, b] for a, b in zip(seq[:-1], seq[1:])):
                best = min(best, sum(np.linalg.norm(wp[b].astype(np.float64) - wp[a]) for a, b in zip(seq[:-1], seq[1:])))
    assert cost == pytest.approx(best, rel=1e-12) if np.isfinite(best) else not np.isfinite(cost)
