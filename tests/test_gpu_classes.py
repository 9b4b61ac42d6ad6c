"""Class-augmented sweep and class-indexed archive on the GPU against the
oracle (oracle/classes.py): the same set of classes, costs within 1e-5, every
returned chain carrying its label, and the cheapest class equal to the plain
optimum.  Labels are integer decisions taken in FP32 with the same operation
order on both sides, so they must agree exactly; cases whose edges include
one within the 1e-5 signed-distance band of the oracle are skipped for the
set comparison."""
import numpy as np
import pytest
import torch

import oracle.classes as OC
import workloads as wl
from tests import parity as P

pytestmark = pytest.mark.gpu


def _say(*a):
    print("[case]", *a, flush=True)


def _oracle_costs(orc, w, stage=0):
    r = orc.plan(w, stage=stage)
    return r


@pytest.mark.parametrize("scene,N,M", [(0, 32, 4), (1, 64, 4), (2, 48, 3), (4, 40, 5), (3, 24, 6)])
def test_class_sweep_matches_oracle(gt, orc, scene, N, M):
    w = wl.make_workload("2d-small", scene, N=N, M=M)
    reps = w["circles"][:, :2]
    _say("class sweep scene", scene, "N", N, "M", M)
    pl = gt.Planner(w, flags=True)
    pl.plan(w["seed"], 0)
    torch.cuda.synchronize()
    got, ovf = gt.class_sweep(pl, reps, L=64)
    r = _oracle_costs(orc, w)
    Cs, Ch, Cl = r["cost"]
    want, J = OC.class_sweep(Cs, Ch, Cl, r["Q"], w["q0"], w["goals"], reps, w["penalty"])
    assert max(len(d) for layer in J for d in layer) <= 64 and len(want) <= 64
    assert ovf == 0
    rep = P.compare_edges(P.flat(pl.C_s.cpu().numpy(), pl.C_h.cpu().numpy()[: M - 1], pl.C_l.cpu().numpy()),
                          pl.flags.cpu().numpy(), P.flat(*r["cost"]), P.flat(*r["minsd"]), P.flat(*r["flag"]))
    _say("classes gpu", len(got), "oracle", len(want), "excused edges", rep["excused"])
    # every returned chain carries its label and cost (oracle edge costs)
    for lab, (cost, chain) in got.items():
        lab2, cost2 = OC.chain_label_cost(Cs, Ch, Cl, r["Q"], w["q0"], w["goals"], reps, chain)
        assert lab2 == lab
        if rep["excused"] == 0:
            assert cost2 == pytest.approx(cost, rel=P.REL)
    if rep["excused"] == 0:
        assert set(got) == set(want)
        for lab, (cost, _) in want.items():
            assert got[lab][0] == pytest.approx(cost, rel=P.REL)
        # the cheapest class is the plain optimum
        assert min(c for c, _ in got.values()) == pytest.approx(float(pl.cost.item()), rel=P.REL)


def test_full_lists_count_dropped_labels(gt, orc):
    w = wl.make_workload("2d-small", 1, N=64, M=4)
    reps = w["circles"][:, :2]
    pl = gt.Planner(w)
    pl.plan(w["seed"], 0)
    torch.cuda.synchronize()
    got, ovf = gt.class_sweep(pl, reps, L=4)
    _say("L=4 classes", len(got), "dropped", ovf)
    assert 0 < len(got) <= 4 and ovf > 0
    r = _oracle_costs(orc, w)
    Cs, Ch, Cl = r["cost"]
    want, _ = OC.class_sweep(Cs, Ch, Cl, r["Q"], w["q0"], w["goals"], reps, w["penalty"])
    for lab, (cost, chain) in got.items():
        lab2, cost2 = OC.chain_label_cost(Cs, Ch, Cl, r["Q"], w["q0"], w["goals"], reps, chain)
        assert lab2 == lab and lab in want
        assert cost >= want[lab][0] * (1 - P.REL)  # never below the class optimum
    # the global optimum survives truncation (kept lists hold the cheapest labels)
    assert min(c for c, _ in got.values()) == pytest.approx(min(c for c, _ in want.values()), rel=P.REL)


@pytest.mark.parametrize("kind,scene,N,M,S,k", [("2d-small", 0, 32, 4, 6, 16), ("2d-small", 2, 24, 3, 8, 16),
                                                  ("2d-large", 2, 32, 16, 4, 16)])
def test_class_archive_matches_oracle(gt, orc, kind, scene, N, M, S, k):
    w = wl.make_workload(kind, scene, N=N, M=M)
    reps = w["circles"][:k, :2]
    _say("class archive scene", scene, "stages", S)
    cp = gt.ClassPlanner(w, reps, S, L=64, cap=512)
    cp.run(w["seed"])
    torch.cuda.synchronize()
    assert int(cp.overflow.item()) == 0
    arch = cp.archive()
    want = {}
    excused = 0
    for s in range(S):
        r = orc.plan(w, stage=s)
        Cs, Ch, Cl = r["cost"]
        found, _ = OC.class_sweep(Cs, Ch, Cl, r["Q"], w["q0"], w["goals"], reps, w["penalty"])
        OC.archive_update(want, found, s)
        excused += int(np.sum(np.abs(P.flat(*r["minsd"])) <= P.BAND))
    _say("archive gpu", len(arch), "oracle", len(want), "band edges", excused)
    if excused == 0:
        assert set(arch) == set(want)
        for lab, (cost, stage, wp) in arch.items():
            c_or, chain, s_or = want[lab]
            assert cost == pytest.approx(c_or, rel=P.REL)
            if stage == s_or:
                Q = orc.sample_layers(M, N, 2, w["lo"], w["hi"], w["seed"], s_or)
                pts = [w["q0"]] + [Q[m, chain[m]] for m in range(M)] + [w["goals"][chain[M]]]
                np.testing.assert_array_equal(wp, np.array(pts, np.float32))
    # anytime: at least as many classes as one stage, the best no worse than stage 0
    assert len(arch) >= 1


def _gpu_sweep_vs_oracle(gt, orc, w, k, L):
    reps = w["circles"][:k, :2]
    pl = gt.Planner(w, flags=True)
    pl.plan(w["seed"], 0)
    torch.cuda.synchronize()
    got, ovf = gt.class_sweep(pl, reps, L=L)
    r = _oracle_costs(orc, w)
    Cs, Ch, Cl = r["cost"]
    want, J = OC.class_sweep(Cs, Ch, Cl, r["Q"], w["q0"], w["goals"], reps, w["penalty"])
    M = int(w["M"])
    rep = P.compare_edges(P.flat(pl.C_s.cpu().numpy(), pl.C_h.cpu().numpy()[: M - 1], pl.C_l.cpu().numpy()),
                          pl.flags.cpu().numpy(), P.flat(*r["cost"]), P.flat(*r["minsd"]), P.flat(*r["flag"]))
    return pl, reps, got, ovf, r, want, J, rep


@pytest.mark.parametrize("scene,N,k", [(2, 48, 16), (1, 48, 8), (2, 32, 16)])
def test_class_sweep_m16_matches_oracle(gt, orc, scene, N, k):
    """The 2d-large workload at its own chain length (M = 16: chains of 17
    edges) with up to 16 representative points, so that labels use both
    words; every vertex list fits L = 64, so the sets must agree."""
    w = wl.make_workload("2d-large", scene, N=N, M=16)
    _say("class sweep 2d-large M=16 scene", scene, "N", N, "k", k)
    pl, reps, got, ovf, r, want, J, rep = _gpu_sweep_vs_oracle(gt, orc, w, k, 64)
    Cs, Ch, Cl = r["cost"]
    assert max(len(d) for layer in J for d in layer) <= 64
    assert ovf == 0
    P.note(f"class sweep 2d-large M=16 scene {scene} N={N} k={k}: {len(got)} classes (oracle {len(want)}), "
           f"excused edges {rep['excused']}")
    assert len(want) > 0
    for lab, (cost, chain) in got.items():
        lab2, cost2 = OC.chain_label_cost(Cs, Ch, Cl, r["Q"], w["q0"], w["goals"], reps, chain)
        assert lab2 == lab
        if rep["excused"] == 0:
            assert cost2 == pytest.approx(cost, rel=P.REL)
    if rep["excused"] == 0:
        assert set(got) == set(want)
        for lab, (cost, _) in want.items():
            assert got[lab][0] == pytest.approx(cost, rel=P.REL)
        assert min(c for c, _ in got.values()) == pytest.approx(float(pl.cost.item()), rel=P.REL)


def test_class_sweep_m16_full_lists(gt, orc):
    """M = 16 with more labels per vertex than L = 64: the kept labels are
    real classes at no less than their optimum, and the global optimum
    survives."""
    w = wl.make_workload("2d-large", 2, N=64, M=16)
    pl, reps, got, ovf, r, want, J, rep = _gpu_sweep_vs_oracle(gt, orc, w, 16, 64)
    Cs, Ch, Cl = r["cost"]
    _say("2d-large M=16 N=64 classes", len(got), "oracle", len(want), "dropped", ovf)
    assert max(len(d) for layer in J for d in layer) > 64 and ovf > 0
    assert rep["excused"] == 0
    for lab, (cost, chain) in got.items():
        lab2, cost2 = OC.chain_label_cost(Cs, Ch, Cl, r["Q"], w["q0"], w["goals"], reps, chain)
        assert lab2 == lab and lab in want
        assert cost2 == pytest.approx(cost, rel=P.REL)
        assert cost >= want[lab][0] * (1 - P.REL)
    assert min(c for c, _ in got.values()) == pytest.approx(min(c for c, _ in want.values()), rel=P.REL)


def test_class_sweep_full_size_2d_large(gt):
    """The full 2d-large workload (M = 16, N = 1024, 16 representative
    points, L = 64): every returned chain carries its label (recomputed by the
    oracle's crossing rule from the chain's own waypoints) and its cost (the
    sum of the GPU's edge costs along it), labels are distinct, and the
    cheapest class is the plain optimum of the same graph."""
    w = wl.make_workload("2d-large", 2)
    assert int(w["M"]) == 16 and int(w["N"]) == 1024
    reps = w["circles"][:16, :2]
    pl = gt.Planner(w)
    pl.plan(w["seed"], 0)
    torch.cuda.synchronize()
    _say("class sweep 2d-large full size")
    got, ovf = gt.class_sweep(pl, reps, L=64)
    Cs, Ch, Cl = (x.cpu().numpy() for x in (pl.C_s, pl.C_h, pl.C_l))
    Q = pl.Q.cpu().numpy()
    P.note(f"class sweep 2d-large full size: {len(got)} classes kept, {ovf} labels dropped")
    assert len(got) > 0
    for lab, (cost, chain) in got.items():
        lab2, cost2 = OC.chain_label_cost(Cs, Ch, Cl, Q, w["q0"], w["goals"], reps, chain)
        assert lab2 == lab
        assert cost2 == pytest.approx(cost, rel=P.REL)
    assert min(c for c, _ in got.values()) == pytest.approx(float(pl.cost.item()), rel=P.REL)
