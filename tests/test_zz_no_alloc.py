"""The edge check that allocates nothing (gtmp_edge_check_cost_noalloc,
scratch in a static device array) against gtmp_edge_check_cost with a
caller workspace: bit-identical costs, flags and minimum signed distances,
on two calls in a row, the second with a smaller problem (the array keeps
the first call's contents), and the size limit rejected on the host."""
import pytest
import torch

import workloads as wl

pytestmark = pytest.mark.gpu


def _say(*a):
    print("[case]", *a, flush=True)


def _both(gt, w, minsd=False):
    """Costs, flags (and minsd) of one sampled plan through both entry
    points: the allocating one first, then the static-scratch one into fresh
    outputs."""
    pl = gt.Planner(w, flags=True, minsd=minsd)
    pl.sample(w["seed"], 0)
    pl.check()
    torch.cuda.synchronize()
    ref = [pl.C_s.clone(), pl.C_h.clone(), pl.C_l.clone(), pl.flags.clone()]
    if minsd:
        ref.append(pl.minsd.clone())
    C_s, C_h, C_l = torch.full_like(pl.C_s, -1.0), torch.full_like(pl.C_h, -1.0), torch.full_like(pl.C_l, -1.0)
    flags = torch.full_like(pl.flags, 7)
    ms = torch.full_like(pl.minsd, -1.0) if minsd else None
    gt.gtmp_edge_check_cost_noalloc(pl.prob, pl.robot, pl.scene, pl.q0, pl.goals, pl.Q, C_s,
                                    C_h if pl.M > 1 else None, C_l, ms, flags, None, pl.opts)
    torch.cuda.synchronize()
    got = [C_s, C_h, C_l, flags] + ([ms] if minsd else [])
    M = pl.M
    for k, (a, b) in enumerate(zip(ref, got)):
        if k == 1:
            a, b = a[: max(M - 1, 0)], b[: max(M - 1, 0)]
        assert torch.equal(a, b), k
    return pl


@pytest.mark.parametrize("first,second", [(("arm7", 0, {}), ("arm7", 1, dict(N=300, M=4))),
                                          (("2d-large", 0, dict(N=700, M=6)), ("2d-small", 2, {}))])
def test_noalloc_equals_workspace_entry_twice(gt, first, second):
    for name, scene, kw in (first, second):
        w = wl.make_workload(name, scene, **kw)
        _say("noalloc", name, scene, kw)
        _both(gt, w)
    # full mode (every state, minimum signed distances) on a small arm plan
    _both(gt, wl.make_workload("arm7", 3, N=96, M=3), minsd=True)


def test_noalloc_rejects_problems_beyond_the_scratch(gt):
    w = wl.make_workload("arm7", 0, N=4096)
    prob = gt.make_problem(w["d"], w["M"], w["N"], w["G"], w["H"], w["lo"], w["hi"], w["penalty"])
    assert gt.gtmp_edge_check_workspace_size(prob) > gt.NOALLOC_SCRATCH_BYTES
    robot, scene = gt.model_of(w, "cuda")
    x = torch.empty(16, device="cuda")
    with pytest.raises(gt.GtmpError) as e:
        gt.gtmp_edge_check_cost_noalloc(prob, robot, scene, x, x, x, x, x, x)
    assert "scratch" in str(e.value)
