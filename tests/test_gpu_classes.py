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


@pytest.mark.parametrize("scene,N,M,S", [(0, 32, 4, 6), (2, 24, 3, 8)])
def test_class_archive_matches_oracle(gt, orc, scene, N, M, S):
    w = wl.make_workload("2d-small", scene, N=N, M=M)
    reps = w["circles"][:, :2]
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
