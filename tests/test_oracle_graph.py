"""Pins of the oracle's edge realisation (Sec. III-B; straight-line LP) and of
its value iteration / extraction (Sec. IV-B; Alg. 1): closed forms in
obstacle-free space, one-way invariants against the textbook segment-to-circle
distance, brute-force enumeration of every chain, SciPy's graph shortest
path, and the cost re-summed along the returned chain."""
import itertools
import math

import numpy as np
import pytest
from scipy.sparse import csr_matrix
from scipy.sparse.csgraph import shortest_path

import workloads as wl


def free_model(orc, d):
    return orc.Model(dict(kind="point", d=d, obs_spheres=np.zeros((0, d + 1), np.float32),
                          obs_boxes=np.zeros((0, 2 * d), np.float32)))


def seg_point_dist(a, b, c):
    """Textbook distance from point c to segment [a, b]: project, clamp."""
    a, b, c = (np.asarray(x, np.float64) for x in (a, b, c))
    ab = b - a
    t = np.clip(np.dot(c - a, ab) / np.dot(ab, ab), 0.0, 1.0)
    return np.linalg.norm(a + t * ab - c)


# ----------------------------------------------------------------- edges
def test_free_edges_cost_length(orc):
    m = free_model(orc, 3)
    g = np.random.default_rng(0)
    for _ in range(20):
        u, v = g.uniform(-5, 5, 3).astype(np.float32), g.uniform(-5, 5, 3).astype(np.float32)
        c, s, f = orc.edge(m, 9, u, v)
        assert f == 0 and np.isinf(s)
        assert c == pytest.approx(np.linalg.norm(v.astype(np.float64) - u), rel=1e-15)


def test_boundary_state_is_collision(orc):
    # the middle state (1, 0) of this edge lies exactly on the unit circle
    m = orc.Model(dict(kind="point", d=2, obs_spheres=np.array([[0, 0, 1]], np.float32),
                       obs_boxes=np.zeros((0, 4), np.float32)))
    c, s, f = orc.edge(m, 3, np.array([1, -1], np.float32), np.array([1, 1], np.float32), penalty=1e3)
    assert s == 0.0 and f == 1 and c == pytest.approx(2.0 + 1e3)
    # the same edge with H = 2 checks only the endpoints (distance sqrt(2) - 1)
    c, s, f = orc.edge(m, 2, np.array([1, -1], np.float32), np.array([1, 1], np.float32))
    assert f == 0 and s == pytest.approx(math.sqrt(2) - 1) and c == pytest.approx(2.0)


def test_penalty_inf_and_length_limit(orc):
    m = orc.Model(dict(kind="point", d=2, obs_spheres=np.array([[0, 0, 1]], np.float32),
                       obs_boxes=np.zeros((0, 4), np.float32)))
    c, _, f = orc.edge(m, 8, np.array([-2, 0], np.float32), np.array([2, 0], np.float32), penalty=np.inf)
    assert f == 1 and np.isinf(c)
    # a free edge longer than the LP length limit fails
    c, _, f = orc.edge(m, 8, np.array([-3, 2], np.float32), np.array([3, 2], np.float32), penalty=5.0, max_len=5.9)
    assert f == 1 and c == pytest.approx(11.0)
    c, _, f = orc.edge(m, 8, np.array([-3, 2], np.float32), np.array([3, 2], np.float32), penalty=5.0, max_len=6.1)
    assert f == 0 and c == pytest.approx(6.0)


def test_discrete_vs_continuous_segment_invariants(orc):
    """Continuous segment clear => every discrete state clear; a discrete state
    inside a circle => the segment meets that circle."""
    w = wl.make_workload("2d-small", seed=0)
    m = orc.Model(w)
    circ = w["circles"].astype(np.float64)
    g = np.random.default_rng(4)
    n_flag = n_clear = 0
    for _ in range(600):
        u, v = g.uniform(-10, 10, 2).astype(np.float32), g.uniform(-10, 10, 2).astype(np.float32)
        _, s, f = orc.edge(m, 8, u, v)
        dseg = min(seg_point_dist(u, v, c[:2]) - c[2] for c in circ)
        if dseg > 0:
            assert f == 0
            n_clear += 1
        if f == 1:
            assert dseg <= 0
            n_flag += 1
        assert s >= dseg - 1e-12  # a discrete state is never closer than the segment
    assert n_flag > 50 and n_clear > 50


def test_edge_costs_layout(orc):
    w = wl.make_workload("2d-small", scene=0, N=6, M=3, H=5)
    Q = orc.sample_layers(3, 6, 2, w["lo"], w["hi"], w["seed"])
    m = orc.Model(w)
    (Cs, Ch, Cl), (Ss, Sh, Sl), (Fs, Fh, Fl) = orc.edge_costs(m, 3, 6, 1, 5, w["q0"], w["goals"], Q)
    assert Cs.shape == (6,) and Ch.shape == (2, 6, 6) and Cl.shape == (6, 1)
    assert orc.n_edges(3, 6) == 2 * 6 + 2 * 36  # 2N + (M-1) N^2 edges
    # spot-check against single-edge evaluations
    assert orc.edge(m, 5, w["q0"], Q[0, 4])[0] == Cs[4]
    assert orc.edge(m, 5, Q[1, 2], Q[2, 5])[0] == Ch[1, 2, 5]
    assert orc.edge(m, 5, Q[2, 3], w["goals"][0])[0] == Cl[3, 0]
    ids = np.array([4, 6 + 36 + 2 * 6 + 5, 6 + 72 + 3])
    c, _, _ = orc.edge_subset(m, 3, 6, 1, 5, w["q0"], w["goals"], Q, ids)
    np.testing.assert_array_equal(c, [Cs[4], Ch[1, 2, 5], Cl[3, 0]])


# ----------------------------------------------------------------- value iteration
def _random_costs(seed, M, N, G, p_inf=0.0, integer=False):
    g = np.random.default_rng(seed)
    x = lambda *s: (g.integers(0, 5, size=s).astype(np.float64) if integer else g.uniform(0, 10, s))
    Cs, Ch, Cl = x(N), x(M - 1, N, N), x(N, G)
    if p_inf:
        for a in (Cs, Ch, Cl):
            a[g.random(a.shape) < p_inf] = np.inf
    return Cs, Ch, Cl


@pytest.mark.parametrize("M,N,G,p_inf,integer", [(1, 5, 1, 0, False), (2, 4, 2, 0, False), (3, 5, 1, 0.3, False),
                                                 (4, 4, 2, 0, True), (4, 5, 1, 0.2, True), (3, 3, 3, 0.5, True)])
def test_dp_equals_brute_force(orc, M, N, G, p_inf, integer):
    for seed in range(6):
        Cs, Ch, Cl = _random_costs(seed, M, N, G, p_inf, integer)
        V, A, Vs, a_s = orc.minplus(Cs, Ch, Cl)
        best, chain = orc.brute_force(Cs, Ch, Cl)
        if np.isinf(best):
            assert np.isinf(Vs) and a_s == -1
            continue
        assert Vs == pytest.approx(best, rel=1e-12)
        Q = np.zeros((M, N, 1), np.float32)
        idx, _, c, rc = orc.extract(A, a_s, Vs, Q, np.zeros(1, np.float32), np.zeros((G, 1), np.float32))
        assert rc == 0
        # lowest index at every step = lexicographically first optimal chain
        assert tuple(idx) == chain
        resum = Cs[idx[0]] + sum(Ch[m, idx[m], idx[m + 1]] for m in range(M - 1)) + Cl[idx[M - 1], idx[M]]
        assert resum == pytest.approx(Vs, rel=1e-12)


def test_dp_equals_scipy_shortest_path(orc):
    for seed in range(5):
        M, N, G = 5, 7, 2
        Cs, Ch, Cl = _random_costs(100 + seed, M, N, G, 0.25)
        # vertex 0 = q0, 1 + m N + u = layer vertices, then goals
        nv = 1 + M * N + G
        rows, cols, vals = [], [], []
        def add(a, b, c):
            if np.isfinite(c):
                rows.append(a); cols.append(b); vals.append(c)
        for u in range(N):
            add(0, 1 + u, Cs[u])
        for m in range(M - 1):
            for u in range(N):
                for v in range(N):
                    add(1 + m * N + u, 1 + (m + 1) * N + v, Ch[m, u, v])
        for u in range(N):
            for gg in range(G):
                add(1 + (M - 1) * N + u, 1 + M * N + gg, Cl[u, gg])
        D = shortest_path(csr_matrix((vals, (rows, cols)), shape=(nv, nv)), directed=True, indices=0)
        want = D[1 + M * N:].min()
        Vs = orc.minplus(Cs, Ch, Cl)[2]
        if np.isinf(want):
            assert np.isinf(Vs)
        else:
            assert Vs == pytest.approx(want, rel=1e-12)


def test_dp_all_infinite_has_no_path(orc):
    Cs, Ch, Cl = np.full(3, np.inf), np.full((1, 3, 3), np.inf), np.full((3, 1), np.inf)
    V, A, Vs, a_s = orc.minplus(Cs, Ch, Cl)
    assert np.isinf(Vs) and a_s == -1 and np.all(A == -1)
    idx, wp, c, rc = orc.extract(A, a_s, Vs, np.zeros((2, 3, 2), np.float32), np.zeros(2, np.float32),
                                 np.zeros((1, 2), np.float32))
    assert rc == 1 and np.all(idx == -1) and np.isinf(c)


def test_dp_terminal_values(orc):
    # V_g shifts the goal choice: J at the goals is V_g (default 0)
    Cs, Ch, Cl = np.array([1.0, 2.0]), np.zeros((0, 2, 2)), np.array([[1.0, 3.0], [1.0, 1.0]])
    assert orc.minplus(Cs, Ch, Cl)[2:] == (2.0, 0)
    V, A, Vs, a_s = orc.minplus(Cs, Ch, Cl, Vg=np.array([5.0, 0.0]))
    assert (Vs, a_s) == (3.0, 1) and A[0, 1] == 1


def test_free_space_collinear_closed_form(orc):
    """Obstacle-free: the chain through one on-segment point per layer costs
    exactly |q_g - q0|, every other chain costs more (triangle inequality)."""
    g = np.random.default_rng(7)
    M, N, d = 4, 9, 3
    q0 = np.array([-4.0, -2.0, 1.0], np.float32)
    qg = np.array([4.0, 2.0, -1.0], np.float32)
    Q = g.uniform(-5, 5, (M, N, d)).astype(np.float32)
    pick = g.integers(0, N, M)
    for m in range(M):
        t = (m + 1) / (M + 1)  # exact in binary for M = 4 only where representable; use float32 points
        Q[m, pick[m]] = (q0 + np.float32(t) * (qg - q0)).astype(np.float32)
    m_ = free_model(orc, d)
    (Cs, Ch, Cl), _, _ = orc.edge_costs(m_, M, N, 1, 6, q0, qg.reshape(1, d), Q)
    V, A, Vs, a_s = orc.minplus(Cs, Ch, Cl)
    idx, wp, c, rc = orc.extract(A, a_s, Vs, Q, q0, qg.reshape(1, d))
    direct = np.linalg.norm(qg.astype(np.float64) - q0)
    assert Vs == pytest.approx(direct, rel=1e-6)  # points are float32 roundings of on-segment points
    assert list(idx[:M]) == list(pick)
    # any chain costs at least the straight distance
    for chain in itertools.islice(itertools.product(range(N), repeat=M), 200):
        cc = Cs[chain[0]] + sum(Ch[m, chain[m], chain[m + 1]] for m in range(M - 1)) + Cl[chain[-1], 0]
        assert cc >= direct * (1 - 1e-7)


def test_single_layer_special_case(orc):
    w = wl.make_workload("2d-small", scene=1, N=16, M=1, H=6)
    Q = orc.sample_layers(1, 16, 2, w["lo"], w["hi"], w["seed"])
    m = orc.Model(w)
    (Cs, Ch, Cl), _, _ = orc.edge_costs(m, 1, 16, 1, 6, w["q0"], w["goals"], Q)
    Vs = orc.minplus(Cs, Ch, Cl)[2]
    assert Vs == pytest.approx(min(Cs[u] + Cl[u, 0] for u in range(16)), rel=1e-15)
