"""FP64 oracle of the learned collision surrogate and of its two uses.

TEST INFRASTRUCTURE (see the package docstring): only tests, the smoke run and
the CPU baseline may import this module; it shares no code with the HIP path.

The paper has no network of its own.  The surrogate fills two slots the paper
leaves open: the heuristic half of the per-sample fair-coin mixture, which may
be any sampler that depends on the history (Sec. III, Layered Sampling Model),
and learned functions in the role of a local planner (Sec. II, Related Work).
It only prunes edges and biases heuristic samples; every edge it does not
prune is still checked exactly.

Network (FP32 parameters, BF16 weights and activations between layers):
  features  x = [q/pi, sin(2 pi B q/pi), cos(2 pi B q/pi)], B in R^{16 x d},
            rounded to BF16 and zero-padded to 64
  hidden    a_l = bf16(relu(bf16(W_l) a_{l-1} + b_l)),  l = 1..4, width 256
  logit     z = bf16(w_5) . a_4 + b_5
  loss      mean over the batch of softplus(z) - y z   (BCE with logits)
Backward, with the same rounding points: dz = (sigmoid(z) - y) / n;
dA_4 = dz w_5; dZ_l = bf16(dA_l * [a_l > 0]); dW_l = dZ_l^T a_{l-1};
db_l = sum_b dZ_l; dA_{l-1} = dZ_l bf16(W_l).  Adam (Kingma and Ba 2015) on the
FP32 parameters.

Here every product and sum is FP64; ``bf16=True`` applies the BF16 rounding
(round to nearest, ties to even) at exactly the points listed above, so that
the only differences from a FP32-accumulating implementation are the order
and precision of the sums.  ``bf16=False`` is the plain FP64 network, used to
pin the backward pass with central finite differences.
"""
from __future__ import annotations

import numpy as np

WIDTH = 256
DEPTH = 4
N_FREQ = 16
IN_PAD = 64
LAYERS = ("W1", "b1", "W2", "b2", "W3", "b3", "W4", "b4", "w5", "b5")


def shapes(d_in: int = IN_PAD):
    s = {"W1": (WIDTH, d_in), "b1": (WIDTH,)}
    for l in range(2, DEPTH + 1):
        s[f"W{l}"] = (WIDTH, WIDTH)
        s[f"b{l}"] = (WIDTH,)
    s["w5"] = (WIDTH,)
    s["b5"] = (1,)
    return s


# --------------------------------------------------------------------- BF16
def bf16(x):
    """Round to the nearest BF16 value (8 significant bits, FP32 exponent
    range), ties to even.  Written from the format's definition: scale so
    that the 8 kept bits form the integer part, round half to even, scale
    back.  Values below the smallest normal keep the subnormal spacing."""
    x = np.asarray(x, np.float64)
    out = np.zeros_like(x)
    nz = (x != 0) & np.isfinite(x)
    m, e = np.frexp(x[nz])               # x = m 2^e, 0.5 <= |m| < 1
    step_exp = np.maximum(e - 8, -133)   # spacing of BF16 values near x
    step = np.ldexp(1.0, step_exp)
    out[nz] = np.round(x[nz] / step) * step  # np.round: half to even
    out[~nz] = x[~nz]
    return out


def _r(x, on):
    return bf16(x) if on else np.asarray(x, np.float64)


# ----------------------------------------------------------------- features
def features(X, Bf, bf16_round=True):
    """[n][d] joint vectors -> [n][64] network inputs."""
    X = np.asarray(X, np.float64)
    n, d = X.shape
    qh = X / np.pi
    s = 2.0 * np.pi * (qh @ np.asarray(Bf, np.float64).T)
    f = np.zeros((n, IN_PAD))
    f[:, :d] = qh
    f[:, d:d + N_FREQ] = np.sin(s)
    f[:, d + N_FREQ:d + 2 * N_FREQ] = np.cos(s)
    return _r(f, bf16_round)


# ------------------------------------------------------------------ forward
def forward(P, X0, bf16_round=True):
    """Returns (logits [n], activations [a0 = X0, a1..a4])."""
    acts = [np.asarray(X0, np.float64)]
    a = acts[0]
    for l in range(1, DEPTH + 1):
        W = _r(P[f"W{l}"], bf16_round)
        z = a @ W.T + np.asarray(P[f"b{l}"], np.float64)
        a = _r(np.maximum(z, 0.0), bf16_round)
        acts.append(a)
    z = a @ _r(P["w5"], bf16_round) + float(np.asarray(P["b5"]).reshape(-1)[0])
    return z, acts


def bce_with_logits(z, y):
    """Mean of softplus(z) - y z, in the overflow-free form
    max(z, 0) - y z + log1p(exp(-|z|))."""
    z = np.asarray(z, np.float64)
    y = np.asarray(y, np.float64)
    return float(np.mean(np.maximum(z, 0) - y * z + np.log1p(np.exp(-np.abs(z)))))


def sigmoid(z):
    z = np.asarray(z, np.float64)
    return np.where(z >= 0, 1.0 / (1.0 + np.exp(-np.abs(z))), np.exp(-np.abs(z)) / (1.0 + np.exp(-np.abs(z))))


# ----------------------------------------------------------------- backward
def loss_and_grad(P, X0, y, bf16_round=True):
    """Loss and gradients (dict with the parameter names) of the mean BCE."""
    z, acts = forward(P, X0, bf16_round)
    n = z.shape[0]
    y = np.asarray(y, np.float64)
    loss = bce_with_logits(z, y)
    dz = (sigmoid(z) - y) / n
    G = {}
    a4 = acts[DEPTH]
    G["w5"] = a4.T @ dz
    G["b5"] = np.array([dz.sum()])
    dA = np.outer(dz, _r(P["w5"], bf16_round))
    for l in range(DEPTH, 0, -1):
        dZ = _r(dA * (acts[l] > 0), bf16_round)
        G[f"W{l}"] = dZ.T @ acts[l - 1]
        G[f"b{l}"] = dZ.sum(axis=0)
        if l > 1:
            dA = dZ @ _r(P[f"W{l}"], bf16_round)
    return loss, G


# --------------------------------------------------------------------- Adam
def adam(P, G, m, v, t, lr=1e-3, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam step (t counts from 1): returns new (P, m, v) dicts."""
    Pn, mn, vn = {}, {}, {}
    for k in LAYERS:
        g = np.asarray(G[k], np.float64)
        mk = b1 * np.asarray(m[k], np.float64) + (1 - b1) * g
        vk = b2 * np.asarray(v[k], np.float64) + (1 - b2) * g * g
        mhat = mk / (1 - b1 ** t)
        vhat = vk / (1 - b2 ** t)
        Pn[k] = np.asarray(P[k], np.float64) - lr * mhat / (np.sqrt(vhat) + eps)
        mn[k], vn[k] = mk, vk
    return Pn, mn, vn


# ----------------------------------------------------------------- the uses
def logits_of_states(P, Bf, X, bf16_round=True):
    return forward(P, features(X, Bf, bf16_round), bf16_round)[0]


def edge_midpoints(q0, goals, Q):
    """Midpoint (u + v) / 2 of every edge in the flat edge order
    C_s | C_h[m][u][v] | C_l[u][g] (FP64 from the FP32 vertices)."""
    Q = np.asarray(Q, np.float64)
    M, N, d = Q.shape
    q0 = np.asarray(q0, np.float64).reshape(1, d)
    goals = np.asarray(goals, np.float64).reshape(-1, d)
    parts = [(q0 + Q[0]) / 2]
    for m in range(M - 1):
        parts.append(((Q[m][:, None, :] + Q[m + 1][None, :, :]) / 2).reshape(-1, d))
    parts.append(((Q[M - 1][:, None, :] + goals[None, :, :]) / 2).reshape(-1, d))
    return np.concatenate(parts, axis=0)


def prune_decisions(P, Bf, q0, goals, Q, tau_logit, bf16_round=True):
    """Edge e is pruned iff the logit at its midpoint exceeds tau_logit.
    Returns (mask uint8 [E], logits [E])."""
    z = logits_of_states(P, Bf, edge_midpoints(q0, goals, Q), bf16_round)
    return (z > tau_logit).astype(np.uint8), z


def free_recall_threshold(logits, flags, recall=0.999):
    """The smallest logit threshold that keeps at least ``recall`` of the free
    edges (flag 0) unpruned: pruning is z > tau."""
    zf = np.sort(np.asarray(logits, np.float64)[np.asarray(flags) == 0])
    if zf.size == 0:
        return np.inf
    k = int(np.ceil(recall * zf.size)) - 1
    return float(zf[min(max(k, 0), zf.size - 1)])
