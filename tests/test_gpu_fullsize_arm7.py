"""Complete parity of the 7-DoF arm plan at its benchmark size (M = 8,
N = 2048, H = 16: 29,364,224 edges, 469,827,584 states) in the launch
configuration bench.py times: every edge's flag and cost against the FP64
oracle (every state of every edge), then the oracle's own value iteration
(Sec. IV-B recursion) and extraction (Alg. 1) on its own costs against the
GPU's path: cost within 1e-5 relative, indices equal up to the first near-tie.

The oracle's edges are computed one block at a time (the start edges with
the goal edges, then each C_h[m]), one test per block, so that each step
reports as it ends; the blocks are kept for the value-iteration test."""
import numpy as np
import pytest
import torch

import workloads as wl
from tests import parity as P

pytestmark = pytest.mark.gpu

BLOCKS = ["ends"] + [f"h{m}" for m in range(7)]
_oracle = {}


def _say(*a):
    print("[case]", *a, flush=True)


@pytest.fixture(scope="module")
def arm7_gpu(gt, orc):
    w = wl.make_workload("arm7", 0)
    assert (w["M"], w["N"], w["H"]) == (8, 2048, 16)
    _say("arm7 full plan on the GPU")
    pl = gt.Planner(w, flags=True)
    pl.plan(w["seed"], 0)
    torch.cuda.synchronize()
    M = w["M"]
    Q = orc.sample_layers(M, w["N"], w["d"], w["lo"], w["hi"], w["seed"], 0)
    assert np.array_equal(pl.Q.cpu().numpy(), Q)
    out = dict(w=w, Q=Q, Cs=pl.C_s.cpu().numpy(), Ch=pl.C_h[: M - 1].cpu().numpy(), Cl=pl.C_l.cpu().numpy(),
               flags=pl.flags.cpu().numpy(), idx=pl.idx.cpu().numpy(), cost=float(pl.cost.item()),
               model=orc.Model(w))
    del pl
    torch.cuda.empty_cache()
    return out


def _block_ids(w, block):
    M, N, G = w["M"], w["N"], w["G"]
    nh = (M - 1) * N * N
    if block == "ends":
        return np.concatenate([np.arange(N), N + nh + np.arange(N * G)]).astype(np.int64)
    m = int(block[1:])
    return (N + m * N * N + np.arange(N * N)).astype(np.int64)


@pytest.mark.parametrize("block", BLOCKS)
def test_arm7_full_edges(gt, orc, arm7_gpu, block):
    g = arm7_gpu
    w = g["w"]
    M, N, G, H = w["M"], w["N"], w["G"], w["H"]
    ids = _block_ids(w, block)
    _say("oracle edges", block, ids.size)
    c_or, sd_or, f_or = orc.edge_subset(g["model"], M, N, G, H, w["q0"], w["goals"], g["Q"], ids, w["penalty"])
    if block == "ends":
        got_c = np.concatenate([g["Cs"], g["Cl"].ravel()])
        got_f = np.concatenate([g["flags"][:N], g["flags"][N + (M - 1) * N * N:]])
    else:
        m = int(block[1:])
        got_c = g["Ch"][m].ravel()
        got_f = g["flags"][ids]
    rep = P.compare_edges(got_c, got_f, c_or, sd_or, f_or)
    _say("block", block, rep)
    P.note(f"arm7 N=2048 block {block}: {rep}")
    _oracle[block] = (c_or, sd_or, f_or, got_f != f_or)


def test_arm7_full_value_iteration(gt, orc, arm7_gpu):
    """The oracle's own value iteration and extraction on its own FP64 edge
    costs (all 29.4 M) against the GPU's returned path."""
    g = arm7_gpu
    w = g["w"]
    M, N, G = w["M"], w["N"], w["G"]
    missing = [b for b in BLOCKS if b not in _oracle]
    assert not missing, f"oracle blocks not computed: {missing}"
    ce, sde, fe, xe = _oracle["ends"]
    Cs, Cl = ce[:N], ce[N:].reshape(N, G)
    Ch = np.stack([_oracle[f"h{m}"][0].reshape(N, N) for m in range(M - 1)])
    excused = sum(int(_oracle[b][3].sum()) for b in BLOCKS)
    near = sum(int((np.abs(_oracle[b][1]) <= P.BAND).sum()) for b in BLOCKS)
    failed = sum(int(_oracle[b][2].sum()) for b in BLOCKS)
    _say("all edges", N + (M - 1) * N * N + N * G, "failed", failed, "excused", excused, "in band", near)
    P.note(f"arm7 N=2048 all {N + (M - 1) * N * N + N * G} edges: failed {failed}, excused {excused}, "
           f"oracle |minsd| <= 1e-5 on {near}")
    V, A, Vs, a_s = orc.minplus(Cs, Ch, Cl)
    idx_or, _, c_or, rc = orc.extract(A, a_s, Vs, g["Q"], w["q0"], w["goals"])
    assert rc == 0 and np.isfinite(c_or) and c_or < w["penalty"]
    c_gpu = g["cost"]
    if excused == 0:
        assert c_gpu == pytest.approx(c_or, rel=P.REL)
        k = P.check_path_indices((Cs, Ch, Cl), V, idx_or, g["idx"], c_or)
        _say("cost", c_gpu, "oracle", c_or, "indices equal up to the first near-tie:", k, "of", M + 1)
        P.note(f"arm7 N=2048 path cost {c_gpu} (oracle DP {c_or}), indices equal at {k} of {M + 1} steps "
               f"before the first near-tie")
    else:
        ex_s, ex_l = xe[:N], xe[N:].reshape(N, G)
        ex_h = np.stack([_oracle[f"h{m}"][3].reshape(N, N) for m in range(M - 1)])
        fs, fl = fe[:N], fe[N:].reshape(N, G)
        fh = np.stack([_oracle[f"h{m}"][2].reshape(N, N) for m in range(M - 1)])
        lens = [np.where(f == 1, c - w["penalty"], c) for c, f in ((Cs, fs), (Ch, fh), (Cl, fl))]
        lo, hi = P.excused_bounds(orc, (Cs, Ch, Cl), lens, (ex_s, ex_h, ex_l), w["penalty"])
        _say("cost", c_gpu, "oracle", c_or, "bracket", lo, hi)
        P.note(f"arm7 N=2048 path cost {c_gpu} (oracle DP {c_or}, bracket {lo}..{hi} over excused edges)")
        assert lo * (1 - P.REL) <= c_gpu <= hi * (1 + P.REL)
    # the GPU's chain re-summed with the oracle's edge costs is its cost
    # (when no excused edge lies on it)
    resum = P.path_cost_from_oracle((Cs, Ch, Cl), g["idx"])
    if excused == 0:
        assert resum == pytest.approx(c_gpu, rel=P.REL)
    _oracle.clear()
