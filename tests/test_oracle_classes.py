"""Pins of the class-augmented sweep oracle (oracle/classes.py): ray-crossing
labels against the angle-sum winding number of closed polygons, the two sides
of an obstacle, and the sweep against enumeration of every chain."""
import numpy as np
import pytest

import oracle.classes as OC


def _loop_label(poly, reps):
    lab = (0,) * len(reps)
    for a, b in zip(poly, np.roll(poly, -1, axis=0)):
        lab = OC.add(lab, OC.edge_label(a, b, reps))
    return lab


def test_closed_loops_label_is_minus_the_winding_number():
    """An upward ray is crossed in -x by a counter-clockwise loop around its
    point: the summed crossings of a closed polygon are minus its winding
    number about each representative point (angle sum, FP64)."""
    rng = np.random.default_rng(0)
    reps = rng.uniform(-3, 3, (6, 2)).astype(np.float32)
    checked = 0
    for _ in range(300):
        k = int(rng.integers(3, 9))
        if rng.uniform() < 0.5:  # star-shaped loops around a random point, sometimes twice
            c = rng.uniform(-3, 3, 2)
            turns = int(rng.integers(1, 3))
            ang = np.sort(rng.uniform(0, 2 * np.pi * turns, k * turns)) * (1 if rng.uniform() < 0.5 else -1)
            rad = rng.uniform(0.5, 4, ang.size)
            poly = (c + np.stack([rad * np.cos(ang), rad * np.sin(ang)], 1)).astype(np.float32)
        else:
            poly = rng.uniform(-5, 5, (k, 2)).astype(np.float32)
        lab = _loop_label(poly, reps)
        for i, z in enumerate(reps):
            d = np.linalg.norm(poly.astype(np.float64) - z, axis=1).min()
            if d < 1e-3:
                continue
            assert lab[i] == -OC.winding_number(poly, z), (poly, z)
            checked += 1
    assert checked > 1000


def test_two_sides_of_an_obstacle_differ_by_one():
    reps = np.array([[0.0, 0.0], [5.0, 5.0]], np.float32)
    start, goal = np.array([-2.0, 0.1], np.float32), np.array([2.0, -0.1], np.float32)
    over = [start, np.array([0.0, 1.0], np.float32), goal]
    under = [start, np.array([0.0, -1.0], np.float32), goal]

    def lab(path):
        out = (0, 0)
        for a, b in zip(path[:-1], path[1:]):
            out = OC.add(out, OC.edge_label(a, b, reps))
        return out
    a, b = lab(over), lab(under)
    assert a == (1, 0) and b == (0, 0)
    # a detour far away around no representative point keeps the label
    far = [start, np.array([-2.0, 3.0], np.float32), np.array([-1.0, 3.0], np.float32), goal]
    assert lab(far) == a


@pytest.mark.parametrize("seed,M,N,G,k", [(0, 3, 4, 1, 2), (1, 2, 5, 2, 3), (2, 4, 3, 1, 3), (6, 3, 4, 2, 1)])
def test_sweep_equals_enumeration(seed, M, N, G, k):
    rng = np.random.default_rng(seed)
    Q = rng.uniform(-4, 4, (M, N, 2)).astype(np.float32)
    q0 = np.array([-4.5, -4.5], np.float32)
    goals = rng.uniform(3.5, 4.5, (G, 2)).astype(np.float32)
    reps = rng.uniform(-3, 3, (k, 2)).astype(np.float32)
    pen = 1e3
    Cs = rng.uniform(1, 5, N)
    Ch = rng.uniform(1, 5, (max(M - 1, 1), N, N))
    Cl = rng.uniform(1, 5, (N, G))
    # some failed edges (cost >= penalty are absent)
    Ch[rng.uniform(size=Ch.shape) < 0.2] += pen
    Cs[0] += pen
    got, _ = OC.class_sweep(Cs, Ch, Cl, Q, q0, goals, reps, pen)
    want = OC.brute_force_classes(Cs, Ch, Cl, Q, q0, goals, reps, pen)
    assert set(got) == set(want)
    assert len(want) >= 2
    for lab, (cost, chain) in got.items():
        assert cost == pytest.approx(want[lab], rel=1e-12)
        lab2, cost2 = OC.chain_label_cost(Cs, Ch, Cl, Q, q0, goals, reps, chain)
        assert lab2 == lab and cost2 == pytest.approx(cost, rel=1e-12)


def test_archive_keeps_the_lowest_cost_per_class():
    a = {}
    OC.archive_update(a, {(1,): (5.0, [0]), (0,): (3.0, [1])}, 0)
    OC.archive_update(a, {(1,): (5.0, [2]), (0,): (2.0, [3]), (2,): (9.0, [4])}, 1)
    assert a[(1,)] == (5.0, [0], 0)  # tie keeps the earlier stage
    assert a[(0,)] == (2.0, [3], 1)
    assert a[(2,)] == (9.0, [4], 1)
