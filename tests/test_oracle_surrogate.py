"""Pins of the surrogate oracle (oracle/surrogate.py) against things other
than itself: PyTorch's float32 -> bfloat16 conversion (round to nearest even)
and hand-computed ties, closed forms of the features, of a selector network
and of the BCE loss, central finite differences of the FP64 network, the
closed form of Adam's first steps, and brute-force enumeration of the edge
midpoints."""
import math

import numpy as np
import pytest
import torch

import oracle.surrogate as S
import workloads as wl


# --------------------------------------------------------------------- BF16
def test_bf16_matches_torch_round_to_nearest_even():
    rng = np.random.default_rng(1)
    x = np.concatenate([
        rng.standard_normal(20000) * 10.0 ** rng.integers(-30, 30, 20000),
        rng.uniform(-4, 4, 20000),
        np.float32(2.0) ** rng.integers(-140, -120, 200) * rng.uniform(1, 2, 200),  # near / below normals
    ]).astype(np.float32)
    want = torch.from_numpy(x).to(torch.bfloat16).to(torch.float64).numpy()
    np.testing.assert_array_equal(S.bf16(x.astype(np.float64)), want)


@pytest.mark.parametrize("x,want", [
    (1 + 2 ** -8, 1.0),                  # tie, even neighbour below
    (1 + 3 * 2 ** -8, 1 + 2 ** -6),      # tie, even neighbour above
    (-(1 + 2 ** -8), -1.0),
    (1 + 2 ** -8 + 2 ** -20, 1 + 2 ** -7),  # just above the tie
    (255.5, 256.0),                      # 8 significant bits: 255 | 256, tie to even 256
    (257.0, 256.0),                      # spacing 2 above 256: tie 256 | 258 -> 256
    (0.0, 0.0),
])
def test_bf16_hand_ties(x, want):
    assert S.bf16(np.array([x]))[0] == want


# ----------------------------------------------------------------- features
def test_features_closed_forms():
    _, Bf = wl.surrogate_init(0, 7)
    f0 = S.features(np.zeros((1, 7)), Bf, bf16_round=False)[0]
    assert np.all(f0[:7] == 0) and np.all(f0[7:23] == 0) and np.all(f0[23:39] == 1) and np.all(f0[39:] == 0)
    for j in range(7):
        q = np.zeros((1, 7))
        q[0, j] = np.pi
        f = S.features(q, Bf, bf16_round=False)[0]
        assert f[j] == pytest.approx(1.0)
        np.testing.assert_allclose(f[7:23], np.sin(2 * np.pi * Bf[:, j].astype(np.float64)), atol=1e-12)
        np.testing.assert_allclose(f[23:39], np.cos(2 * np.pi * Bf[:, j].astype(np.float64)), atol=1e-12)
    assert f.shape == (64,)


def _zero_net():
    return {k: np.zeros(s) for k, s in S.shapes().items()}


def test_selector_network_closed_form():
    """W1 routes feature 0 (q_0 / pi) into unit 0, the hidden layers pass unit
    0 through, w5[0] = 3, b5 = -1: logit = 3 relu(q_0 / pi) - 1."""
    P = _zero_net()
    P["W1"][0, 0] = 1.0
    for l in (2, 3, 4):
        P[f"W{l}"][0, 0] = 1.0
    P["w5"][0] = 3.0
    P["b5"][0] = -1.0
    _, Bf = wl.surrogate_init(0, 7)
    X = np.random.default_rng(2).uniform(-np.pi, np.pi, (50, 7))
    z = S.logits_of_states(P, Bf, X, bf16_round=False)
    np.testing.assert_allclose(z, 3 * np.maximum(X[:, 0] / np.pi, 0) - 1, atol=1e-14)


def test_bce_closed_forms():
    assert S.bce_with_logits([0.0, 0.0], [0, 1]) == pytest.approx(math.log(2))
    assert S.bce_with_logits([1000.0], [1]) == pytest.approx(0.0, abs=1e-300)
    assert S.bce_with_logits([-1000.0], [1]) == pytest.approx(1000.0)
    assert S.bce_with_logits([2.0], [0]) == pytest.approx(math.log1p(math.exp(2.0)))
    z = np.linspace(-30, 30, 61)
    np.testing.assert_allclose(S.sigmoid(z), 1 / (1 + np.exp(-z)), rtol=1e-13)


# ----------------------------------------------------------------- backward
def test_gradients_match_central_differences():
    """FP64 network (no BF16 rounding): every gradient block against central
    differences at random coordinates."""
    P, Bf = wl.surrogate_init(3, 7)
    P = {k: v.astype(np.float64) for k, v in P.items()}
    rng = np.random.default_rng(4)
    for k in P:  # non-zero biases so that their gradients are exercised off zero
        if k.startswith("b"):
            P[k] = rng.standard_normal(P[k].shape) * 0.1
    X = rng.uniform(-np.pi, np.pi, (24, 7))
    y = (rng.uniform(size=24) < 0.4).astype(np.float64)
    X0 = S.features(X, Bf, bf16_round=False)
    _, G = S.loss_and_grad(P, X0, y, bf16_round=False)
    h = 1e-6
    checked = 0
    for k in S.LAYERS:
        flat = P[k].reshape(-1)
        for idx in rng.choice(flat.size, size=min(6, flat.size), replace=False):
            old = flat[idx]
            flat[idx] = old + h
            lp, _ = S.loss_and_grad(P, X0, y, bf16_round=False)
            flat[idx] = old - h
            lm, _ = S.loss_and_grad(P, X0, y, bf16_round=False)
            flat[idx] = old
            fd = (lp - lm) / (2 * h)
            g = G[k].reshape(-1)[idx]
            assert abs(fd - g) <= 1e-6 * max(abs(g), 1e-3), (k, idx, fd, g)
            checked += 1
    assert checked >= 40


def test_bias_gradient_of_output_at_zero_logit():
    """With all weights zero the logit is b5 = 0: dL/db5 = mean(1/2 - y)."""
    P = _zero_net()
    y = np.array([1, 0, 1, 1], np.float64)
    _, G = S.loss_and_grad(P, np.zeros((4, 64)), y, bf16_round=True)
    assert G["b5"][0] == pytest.approx(np.mean(0.5 - y))
    assert np.all(G["W4"] == 0) and np.all(G["w5"] == 0)


# --------------------------------------------------------------------- Adam
def test_adam_first_steps_closed_form():
    rng = np.random.default_rng(5)
    P = {k: rng.standard_normal(s) for k, s in S.shapes().items()}
    G = {k: rng.standard_normal(s) for k, s in S.shapes().items()}
    z = {k: np.zeros(s) for k, s in S.shapes().items()}
    lr, eps = 1e-3, 1e-8
    P1, m1, v1 = S.adam(P, G, z, z, 1, lr=lr, eps=eps)
    for k in S.LAYERS:
        np.testing.assert_allclose(P1[k], P[k] - lr * G[k] / (np.abs(G[k]) + eps), rtol=0, atol=1e-15)
    # a constant gradient keeps m_hat = g and v_hat = g^2: the same step again
    P2, _, _ = S.adam(P1, G, m1, v1, 2, lr=lr, eps=eps)
    for k in S.LAYERS:
        np.testing.assert_allclose(P2[k] - P1[k], -lr * G[k] / (np.abs(G[k]) + eps),
                                   rtol=1e-9, atol=1e-15)


# ----------------------------------------------------------------- the uses
def test_edge_midpoints_enumerated():
    rng = np.random.default_rng(6)
    M, N, d, G = 3, 4, 2, 2
    Q = rng.uniform(-1, 1, (M, N, d)).astype(np.float32)
    q0 = rng.uniform(-1, 1, d).astype(np.float32)
    goals = rng.uniform(-1, 1, (G, d)).astype(np.float32)
    mids = S.edge_midpoints(q0, goals, Q)
    want = [(q0.astype(np.float64) + Q[0, v]) / 2 for v in range(N)]
    for m in range(M - 1):
        for u in range(N):
            for v in range(N):
                want.append((Q[m, u].astype(np.float64) + Q[m + 1, v]) / 2)
    for u in range(N):
        for g in range(G):
            want.append((Q[M - 1, u].astype(np.float64) + goals[g]) / 2)
    np.testing.assert_array_equal(mids, np.array(want))


def test_free_recall_threshold_is_the_smallest_that_keeps_the_recall():
    rng = np.random.default_rng(7)
    z = rng.standard_normal(5000)
    flags = (rng.uniform(size=5000) < 0.3).astype(np.uint8)
    tau = S.free_recall_threshold(z, flags, 0.999)
    free = z[flags == 0]
    assert np.mean(free <= tau) >= 0.999
    below = np.max(free[free < tau])
    assert np.mean(free <= below) < 0.999
