"""Parity at the full sizes the benchmarks run, in the launch configuration
bench.py times (default options): the oracle computes a million sampled
edges one by one (every state of each; the arm at N = 2048 is compared edge
for edge in test_gpu_fullsize_arm7.py), the returned path is re-summed from the oracle's
edge costs, and the sweep is checked row by row on sampled rows against its
defining recursion evaluated on the host in FP32.  Also the full 512-plan
batch distribution (a seeded subset of its plans) against single-plan calls,
and surrogate pruning at N = 4096."""
import numpy as np
import pytest
import torch

import oracle.surrogate as OS
import workloads as wl
from tests import parity as P

pytestmark = pytest.mark.gpu


def _say(*a):
    print("[case]", *a, flush=True)


def _edge_ends(w, Q, ids):
    """(u, v) of flat edge ids in the order C_s | C_h | C_l."""
    M, N, G = w["M"], w["N"], w["G"]
    q0 = np.asarray(w["q0"], np.float32)
    goals = np.asarray(w["goals"], np.float32).reshape(G, -1)
    nh = (M - 1) * N * N
    U, V = [], []
    for e in ids:
        e = int(e)
        if e < N:
            U.append(q0); V.append(Q[0, e])
        elif e < N + nh:
            r = e - N
            m, uv = divmod(r, N * N)
            U.append(Q[m, uv // N]); V.append(Q[m + 1, uv % N])
        else:
            r = e - N - nh
            U.append(Q[M - 1, r // G]); V.append(goals[r % G])
    return np.array(U), np.array(V)


def _path_edges(w, idx):
    M, N, G = w["M"], w["N"], w["G"]
    e = [int(idx[0])]
    for m in range(M - 1):
        e.append(N + m * N * N + int(idx[m]) * N + int(idx[m + 1]))
    e.append(N + (M - 1) * N * N + int(idx[M - 1]) * G + int(idx[M]))
    return e


@pytest.mark.parametrize("name,n_sample", [("arm7-n4096", 1_000_000), ("2d-large", 1_000_000)])
def test_full_size_plan(gt, orc, name, n_sample):
    w = wl.make_workload(name, 0)
    M, N, G, H = w["M"], w["N"], w["G"], w["H"]
    _say("full size", name, "M", M, "N", N, "H", H)
    pl = gt.Planner(w, flags=True)
    pl.plan(w["seed"], 0)
    torch.cuda.synchronize()
    Q = orc.sample_layers(M, N, w["d"], w["lo"], w["hi"], w["seed"], 0)
    assert np.array_equal(pl.Q.cpu().numpy(), Q)
    E = pl.E
    idx = pl.idx.cpu().numpy()
    rng = np.random.default_rng(20)
    ids = np.unique(np.concatenate([rng.integers(0, E, n_sample), _path_edges(w, idx)]))
    flat = torch.cat([pl.C_s.reshape(-1), pl.C_h[: M - 1].reshape(-1), pl.C_l.reshape(-1)])
    t_ids = torch.from_numpy(ids).cuda()
    got_c = flat[t_ids].cpu().numpy()
    got_f = pl.flags[t_ids].cpu().numpy()
    model = orc.Model(w)
    c_or, sd_or, f_or = orc.edge_subset(model, M, N, G, H, w["q0"], w["goals"], Q, ids, w["penalty"])
    rep = P.compare_edges(got_c, got_f, c_or, sd_or, f_or)
    _say("sampled edges", rep)
    P.note(f"{name} sampled edges: {rep}")
    # the returned path re-summed from the oracle's costs of its edges
    pe = _path_edges(w, idx)
    pos = np.searchsorted(ids, pe)
    c_gpu = float(pl.cost.item())
    assert c_gpu < w["penalty"]
    if not np.any(np.abs(sd_or[pos]) <= P.BAND):
        assert float(np.sum(c_or[pos])) == pytest.approx(c_gpu, rel=P.REL)
    # the sweep's recursion on sampled rows, in FP32 as the kernel adds
    V = pl.V.cpu().numpy()
    A = pl.A.cpu().numpy()
    for m in rng.choice(M - 1, size=min(3, M - 1), replace=False):
        rows = rng.choice(N, size=64, replace=False)
        C = pl.C_h[int(m)][torch.from_numpy(rows).cuda()].cpu().numpy()
        s = (C + V[m + 1][None, :]).astype(np.float32)
        np.testing.assert_array_equal(V[m][rows], s.min(axis=1))
        np.testing.assert_array_equal(A[m][rows], s.argmin(axis=1))


def test_full_batch_distribution_equals_single(gt):
    specs = wl.batch_specs(n=32, seed=11)
    _say("batch of", len(specs), "from the full distribution, largest N", max(sp["w"]["N"] for sp in specs))
    bp = gt.BatchPlanner(specs)
    bp.run()
    torch.cuda.synchronize()
    best = bp.best_cost.cpu().numpy()
    meta = bp.best_meta.cpu().numpy()
    for i, sp in enumerate(specs):
        ap = gt.single_planner(sp)
        ap.run(int(sp["seed"]))
        torch.cuda.synchronize()
        assert np.array_equal(meta[i], ap.best_meta.cpu().numpy()), i
        c = float(ap.best_cost.item())
        assert best[i] == c or (not np.isfinite(best[i]) and not np.isfinite(c)), (i, best[i], c)
        del ap


def test_full_size_surrogate_prune(gt, orc):
    """arm7 at N = 4096 (117 M edges): logits at sampled edge midpoints against
    the oracle, decisions outside the band, and the exact check of every
    unpruned edge identical to the plain check."""
    w = wl.make_workload("arm7", 0, N=4096)
    M, N, G = w["M"], w["N"], w["G"]
    P0, Bf = wl.surrogate_init(7, 7)
    net = gt.Surrogate(P0, Bf, batch=256)
    pl = gt.Planner(w, flags=True)
    pl.sample(w["seed"], 0)
    pl.check()
    torch.cuda.synchronize()
    plain_f = pl.flags.clone()
    plain_c = torch.cat([pl.C_s.reshape(-1), pl.C_h[: M - 1].reshape(-1), pl.C_l.reshape(-1)])
    prune = torch.empty(pl.E, device="cuda", dtype=torch.uint8)
    logits = torch.empty(pl.E, device="cuda")
    net.workspace = gt._aligned_workspace(gt.gtmp_surrogate_workspace_size(1 << 21))
    tau = 0.0
    net.prune(pl.prob, pl.q0, pl.goals, pl.Q, tau, prune, logits)
    torch.cuda.synchronize()
    _say("pruned fraction", float(prune.float().mean().item()))
    rng = np.random.default_rng(3)
    ids = rng.integers(0, pl.E, 4000)
    Q = orc.sample_layers(M, N, 7, w["lo"], w["hi"], w["seed"], 0)
    U, V = _edge_ends(w, Q, ids)
    mids = (U.astype(np.float64) + V.astype(np.float64)) / 2
    P64 = {k: v.astype(np.float64) for k, v in P0.items()}
    z_or = OS.logits_of_states(P64, Bf, mids)
    t_ids = torch.from_numpy(ids).cuda()
    z = logits[t_ids].cpu().numpy().astype(np.float64)
    P.check_logits(z, z_or)
    m = prune[t_ids].cpu().numpy()
    clear = np.abs(z_or - tau) > P.Z_LOOSE * max(1.0, abs(tau))
    assert np.array_equal(m[clear], (z_or[clear] > tau).astype(np.uint8))
    # exact check of the survivors
    pl.check(prune=prune)
    torch.cuda.synchronize()
    keep = prune == 0
    pr_c = torch.cat([pl.C_s.reshape(-1), pl.C_h[: M - 1].reshape(-1), pl.C_l.reshape(-1)])
    assert torch.equal(pl.flags[keep], plain_f[keep])
    assert torch.equal(pr_c[keep], plain_c[keep])
    assert bool((pl.flags[~keep] == 1).all())
