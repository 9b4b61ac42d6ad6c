"""Learned collision surrogate on the GPU against the FP64 oracle with BF16
rounding at the same points (oracle/surrogate.py).

Tolerances.  Features are computed in FP64 on both sides and rounded once to
BF16, so the network inputs agree.  The hidden layers accumulate in FP32 on
the GPU (MFMA order) and in FP64 in the oracle; a pre-activation whose two
sums fall on opposite sides of a BF16 rounding boundary rounds to adjacent
BF16 values (one step, 2^-8 relative), and that flip propagates to the logit.
With 1024 rounding points per state such flips are common but small: on 1024
arm states the FP32 emulation of the same network (numpy float32 products,
BF16 rounding at the same points) differs from the FP64 oracle by a median
1.5e-8 and at most 1.4e-3, with 98.6 % of the states within 1e-4; the GPU
differs by at most 2.4e-3 with 98.9 % within 1e-4.  Bounds: 97 % of the
states within 1e-4 max(1, |z|) (Z_TOL) and every state within
1e-2 max(1, |z|) (Z_LOOSE); decisions (prune, bias) are compared outside a
band of Z_LOOSE around the threshold.  Gradient blocks: 1e-3 normwise
relative (measured 1.1e-4).  The loss, a mean of terms whose derivative in
the logit is at most 1 in size, may differ by the mean logit error."""
import numpy as np
import pytest
import torch

import oracle
import oracle.surrogate as OS
import workloads as wl

pytestmark = pytest.mark.gpu

from tests.parity import Z_LOOSE, Z_TOL, check_logits as _check_logits  # noqa: E402

G_TOL = 1e-3


def _say(*a):
    print("[case]", *a, flush=True)


@pytest.fixture(scope="module")
def arm():
    return wl.make_workload("arm7", 0)


def _net(gt, seed=0, d=7, batch=512):
    P, Bf = wl.surrogate_init(seed, d)
    return gt.Surrogate(P, Bf, batch=batch), {k: v.astype(np.float64) for k, v in P.items()}, Bf


def test_layout_matches_the_parameter_shapes(gt):
    off = gt.gtmp_surrogate_layout()
    sizes = [int(np.prod(s)) for s in OS.shapes().values()]
    assert off[0] == 0
    assert [b - a for a, b in zip(off[:10], off[1:11])] == sizes


def test_label_states_and_labels(gt, orc, arm):
    n, H = 1000, arm["H"]
    _say("label states", n)
    X, y = gt.make_labels(arm, n, seed=5, stage=77)
    Xc = X.cpu().numpy()
    Q = orc.sample_layers(3, n, 7, arm["lo"], arm["hi"], 5, 77)
    np.testing.assert_array_equal(Xc[:n], Q[0])
    h = 1 + np.arange(n) % (H - 2)
    t = (h.astype(np.float32) / np.float32(H - 1)).astype(np.float64)[:, None]
    u, v = Q[1].astype(np.float64), Q[2].astype(np.float64)
    want = (t * (v.astype(np.float32) - u.astype(np.float32)).astype(np.float64) + u).astype(np.float32)
    np.testing.assert_array_max_ulp(Xc[n:], want, maxulp=1)
    sd = orc.state_sd(orc.Model(arm), Xc)
    yc = y.cpu().numpy()
    sure = np.abs(sd) > 1e-5
    assert np.array_equal(yc[sure], (sd[sure] <= 0).astype(np.uint8))
    assert 0.05 < yc.mean() < 0.95


def test_forward_logits_match_oracle(gt, orc, arm):
    net, P, Bf = _net(gt)
    X, _ = gt.make_labels(arm, 512, seed=5, stage=78)
    z = net.infer(X).cpu().numpy().astype(np.float64)
    z_or = OS.logits_of_states(P, Bf, X.cpu().numpy().astype(np.float64))
    err = _check_logits(z, z_or)
    _say("logits max err", err.max(), "median", np.median(err), "within Z_TOL", np.mean(err <= Z_TOL))


def test_forward_ragged_sizes_and_chunks(gt, orc, arm):
    """Row counts that are not tile multiples, and more rows than one chunk of
    the workspace holds: same logits as one call per row block."""
    net, P, Bf = _net(gt, batch=256)
    X, _ = gt.make_labels(arm, 700, seed=9, stage=1)  # 1400 rows > 256-row chunks
    z = net.infer(X).cpu().numpy()
    z_or = OS.logits_of_states(P, Bf, X.cpu().numpy().astype(np.float64))
    _check_logits(z, z_or)
    for n in (1, 37, 129):
        zi = net.infer(X[:n].contiguous()).cpu().numpy()
        np.testing.assert_array_equal(zi, z[:n])
    assert net.infer(X[:0].contiguous()).numel() == 0


def test_gradients_match_oracle(gt, orc, arm):
    net, P, Bf = _net(gt)
    X, y = gt.make_labels(arm, 256, seed=5, stage=79)
    zbuf = torch.empty(X.shape[0], device="cuda")
    loss = float(net.grad(X, y, logits=zbuf).item())
    g = net.grad_buf.cpu().numpy().astype(np.float64)
    Xc, yc = X.cpu().numpy().astype(np.float64), y.cpu().numpy().astype(np.float64)
    l_or, G = OS.loss_and_grad(P, OS.features(Xc, Bf), yc)
    z_or = OS.logits_of_states(P, Bf, Xc)
    dz = np.abs(zbuf.cpu().numpy() - z_or)
    _check_logits(zbuf.cpu().numpy(), z_or)
    assert abs(loss - l_or) <= dz.mean() + 1e-6 * l_or
    off = net.offsets
    for i, k in enumerate(gt.SUR_NAMES):
        end = off[i + 1] if i + 1 < 10 else net.total
        a, b = g[off[i]:end], G[k].reshape(-1)
        rel = np.linalg.norm(a - b) / np.linalg.norm(b)
        _say("grad", k, rel)
        assert rel <= G_TOL, k


def test_gradients_deterministic(gt, arm):
    net, _, _ = _net(gt, batch=1024)
    X, y = gt.make_labels(arm, 512, seed=3, stage=3)
    net.grad(X, y)
    g1 = net.grad_buf.clone()
    net.grad(X, y)
    assert torch.equal(g1, net.grad_buf)


def test_adam_matches_oracle_and_refreshes_bf16(gt, arm):
    net, P, Bf = _net(gt)
    rng = np.random.default_rng(11)
    grads = [{k: rng.standard_normal(np.shape(v)) * 1e-2 for k, v in P.items()} for _ in range(3)]
    m = {k: np.zeros(np.shape(v)) for k, v in P.items()}
    v = {k: np.zeros(np.shape(v)) for k, v in P.items()}
    Pr = P
    for t, G in enumerate(grads, start=1):
        flat = np.zeros(net.total, np.float32)
        for i, k in enumerate(gt.SUR_NAMES):
            end = net.offsets[i + 1] if i + 1 < 10 else net.total
            flat[net.offsets[i]:end] = G[k].reshape(-1).astype(np.float32)
        net.adam(torch.from_numpy(flat).cuda())
        Gr = {k: G[k].astype(np.float32).astype(np.float64) for k in G}
        Pr, m, v = OS.adam(Pr, Gr, m, v, t)
    got = net.to_dict()
    for k in gt.SUR_NAMES:
        np.testing.assert_allclose(got[k].astype(np.float64), Pr[k].reshape(got[k].shape), rtol=1e-6, atol=1e-8)
    # the BF16 copy is the round-to-nearest-even image of the FP32 values
    want = net.params.to(torch.bfloat16).view(torch.int16)
    assert torch.equal(net.params_bf16, want)


def test_training_lowers_the_loss_and_beats_the_majority_class(gt, arm):
    net, _, _ = _net(gt, seed=1, batch=8192)
    Xt, yt = gt.make_labels(arm, 1 << 17, seed=6, stage=1)
    Xh, yh = gt.make_labels(arm, 1 << 13, seed=6, stage=2)
    losses = net.train(Xt, yt, epochs=4).cpu().numpy()
    zh = net.infer(Xh).cpu().numpy()
    yhc = yh.cpu().numpy()
    acc = np.mean((zh > 0) == (yhc == 1))
    base = max(yhc.mean(), 1 - yhc.mean())
    _say("loss", losses[0], losses[-8:].mean(), "acc", acc, "majority", base)
    assert losses[-8:].mean() < 0.9 * losses[:4].mean()
    assert acc > base + 0.1


# ----------------------------------------------------------------- pruning
def _small_plan(gt, w):
    pl = gt.Planner(w, flags=True)
    pl.sample(w["seed"], 0)
    return pl


def test_prune_decisions_match_oracle(gt, orc):
    w = wl.make_workload("arm7", 1, N=48, M=3)
    net, P, Bf = _net(gt, seed=2)
    pl = _small_plan(gt, w)
    prune = torch.empty(pl.E, device="cuda", dtype=torch.uint8)
    logits = torch.empty(pl.E, device="cuda")
    Q = orc.sample_layers(w["M"], w["N"], w["d"], w["lo"], w["hi"], w["seed"], 0)
    z_or = OS.edge_midpoints(w["q0"], w["goals"], Q)
    z_or = OS.logits_of_states(P, Bf, z_or)
    tau = float(np.median(z_or))
    net.prune(pl.prob, pl.q0, pl.goals, pl.Q, tau, prune, logits)
    mask = prune.cpu().numpy()
    z = logits.cpu().numpy().astype(np.float64)
    _check_logits(z, z_or)
    clear = np.abs(z_or - tau) > Z_LOOSE * np.maximum(1.0, abs(tau))
    assert np.array_equal(mask[clear], (z_or[clear] > tau).astype(np.uint8))
    _say("pruned", mask.mean(), "excused", (~clear).sum())
    assert 0.3 < mask.mean() < 0.7


def test_pruned_check_is_exact_on_survivors(gt, orc):
    """Survivors carry the plain checker's flags and costs; pruned edges cost
    length + penalty; the pruned plan is never cheaper than the plain one and
    equal when no edge of the plain optimum was pruned."""
    w = wl.make_workload("arm7", 1, N=64, M=3)
    net, _, _ = _net(gt, seed=2)
    pl = _small_plan(gt, w)
    pl.check()
    pl.sweep()
    pl.extract()
    plain = [t.clone() for t in (pl.C_s, pl.C_h, pl.C_l, pl.flags)]
    c_plain = float(pl.cost.item())
    idx_plain = pl.idx.cpu().numpy()
    prune = torch.empty(pl.E, device="cuda", dtype=torch.uint8)
    logits = torch.empty(pl.E, device="cuda")
    net.prune(pl.prob, pl.q0, pl.goals, pl.Q, 0.0, prune, logits)
    pl.check(prune=prune)
    pl.sweep()
    pl.extract()
    flat = lambda Cs, Ch, Cl: torch.cat([Cs.reshape(-1), Ch[: w["M"] - 1].reshape(-1), Cl.reshape(-1)])
    c0 = flat(*plain[:3]).cpu().numpy()
    c1 = flat(pl.C_s, pl.C_h, pl.C_l).cpu().numpy()
    f0, f1 = plain[3].cpu().numpy(), pl.flags.cpu().numpy()
    m = prune.cpu().numpy().astype(bool)
    assert np.array_equal(f1[~m], f0[~m]) and np.array_equal(c1[~m], c0[~m])
    assert np.all(f1[m] == 1)
    length = np.where(f0 == 1, c0 - w["penalty"], c0)
    np.testing.assert_allclose(c1[m], length[m] + w["penalty"], rtol=1e-6)
    c_pr = float(pl.cost.item())
    assert c_pr >= c_plain
    # edges of the plain optimum
    N = w["N"]
    path_edges = [idx_plain[0]]
    for k in range(w["M"] - 1):
        path_edges.append(N + k * N * N + idx_plain[k] * N + idx_plain[k + 1])
    path_edges.append(N + (w["M"] - 1) * N * N + idx_plain[w["M"] - 1])
    hit = bool(m[path_edges].any())
    _say("plain", c_plain, "pruned", c_pr, "optimum pruned", hit, "pruned frac", m.mean())
    if not hit:
        assert c_pr == c_plain


def _vertex_coll(gt, w, pl):
    robot, scene = gt.model_of(w)
    coll = torch.empty(w["M"] * w["N"], device="cuda", dtype=torch.uint8)
    gt.gtmp_state_check(robot, scene, w["d"], pl.Q.reshape(-1, w["d"]).contiguous(), None, coll)
    return coll


def _candidates(free, N, G):
    """Edges whose sample endpoints are free (q0 and goals count as free),
    in edge order C_s | C_h | C_l, from the vertex flags."""
    M = free.shape[0]
    parts = [free[0]]
    for m in range(M - 1):
        parts.append((free[m][:, None] & free[m + 1][None, :]).reshape(-1))
    parts.append(np.repeat(free[M - 1], G))
    return np.concatenate(parts)


@pytest.mark.parametrize("scene,N,M", [(1, 64, 3), (0, 100, 4), (2, 37, 1)])
def test_prune_infers_only_candidate_edges(gt, scene, N, M):
    """With the sample flags, only edges whose endpoints are free are
    inferred: their logits and decisions are bit-identical to those of the
    all-edge call, every other edge is unpruned with a NaN logit; the exact
    check of the mask leaves the plain optimum's cost when no edge of it is
    pruned."""
    w = wl.make_workload("arm7", scene, N=N, M=M)
    net, _, _ = _net(gt, seed=2)
    pl = _small_plan(gt, w)
    pl.check()
    pl.sweep()
    pl.extract()
    c_plain = float(pl.cost.item())
    flags_plain = pl.flags.clone()
    coll = _vertex_coll(gt, w, pl)
    E = pl.E
    pa, za = torch.empty(E, device="cuda", dtype=torch.uint8), torch.empty(E, device="cuda")
    pc, zc = torch.full((E,), 7, device="cuda", dtype=torch.uint8), torch.zeros(E, device="cuda")
    net.prune(pl.prob, pl.q0, pl.goals, pl.Q, 0.0, pa, za)
    net.prune(pl.prob, pl.q0, pl.goals, pl.Q, 0.0, pc, zc, vcoll=coll)
    free = coll.cpu().numpy().reshape(M, N) == 0
    cand = _candidates(free, N, w["G"])
    assert cand.shape[0] == E
    pa_, za_, pc_, zc_ = (t.cpu().numpy() for t in (pa, za, pc, zc))
    _say("candidates", cand.mean(), "pruned among them", pc_[cand].mean() if cand.any() else 0)
    assert np.array_equal(zc_[cand].view(np.uint32), za_[cand].view(np.uint32))
    assert np.array_equal(pc_[cand], pa_[cand])
    assert np.all(np.isnan(zc_[~cand])) and np.all(pc_[~cand] == 0)
    # non-candidate edges fail the exact check
    assert np.all(flags_plain.cpu().numpy()[~cand] == 1)
    pl.check(prune=pc)
    pl.sweep()
    pl.extract()
    m = pc_.astype(bool)
    f1 = pl.flags.cpu().numpy()
    assert np.array_equal(f1[~m], flags_plain.cpu().numpy()[~m])
    assert float(pl.cost.item()) >= c_plain * (1 - 1e-6)


def test_prune_with_every_sample_colliding_or_free(gt):
    """Edge cases of the candidate lists: every sample colliding (no edge is
    inferred) and every sample free (the all-edge result)."""
    w = wl.make_workload("arm7", 1, N=40, M=3)
    net, _, _ = _net(gt, seed=2)
    pl = _small_plan(gt, w)
    E = pl.E
    pa, za = torch.empty(E, device="cuda", dtype=torch.uint8), torch.empty(E, device="cuda")
    net.prune(pl.prob, pl.q0, pl.goals, pl.Q, 0.0, pa, za)
    p1, z1 = torch.full((E,), 3, device="cuda", dtype=torch.uint8), torch.zeros(E, device="cuda")
    net.prune(pl.prob, pl.q0, pl.goals, pl.Q, 0.0, p1, z1,
              vcoll=torch.ones(w["M"] * w["N"], device="cuda", dtype=torch.uint8))
    assert int(p1.sum().item()) == 0 and bool(torch.isnan(z1).all().item())
    p0, z0 = torch.empty(E, device="cuda", dtype=torch.uint8), torch.empty(E, device="cuda")
    net.prune(pl.prob, pl.q0, pl.goals, pl.Q, 0.0, p0, z0,
              vcoll=torch.zeros(w["M"] * w["N"], device="cuda", dtype=torch.uint8))
    assert torch.equal(p0, pa) and torch.equal(z0.view(torch.int32), za.view(torch.int32))


# ------------------------------------------------- pruning threshold
@pytest.mark.parametrize("E,p_free,recall,kind", [(0, 0.5, 0.999, "normal"), (1000, 0.0, 0.999, "normal"),
                                                  (1, 1.0, 0.999, "normal"), (5000, 0.3, 0.999, "normal"),
                                                  (5000, 0.3, 1.0, "normal"), (5000, 0.3, 0.5, "ties"),
                                                  (100_003, 0.04, 0.999, "ties"), (4_000_000, 0.05, 0.999, "normal"),
                                                  (20_000, 0.5, 0.9, "signed-zero"), (20_000, 0.5, 0.999, "nan")])
def test_threshold_matches_oracle(gt, E, p_free, recall, kind):
    """gtmp_surrogate_threshold against the oracle's definition: the same
    logit (the k-th smallest free-edge logit), +inf without a free edge."""
    _say("threshold", E, p_free, recall, kind)
    g = np.random.default_rng(E + 7)
    z = (g.normal(size=E) * 3).astype(np.float32)
    if kind == "ties":
        z = np.round(z * 4).astype(np.float32) / 4
    elif kind == "signed-zero":
        z[g.random(E) < 0.3] = 0.0
        z[g.random(E) < 0.3] = -0.0
    elif kind == "nan":
        z[g.random(E) < 0.01] = np.nan
    flags = (g.random(E) >= p_free).astype(np.uint8)
    want = OS.free_recall_threshold(z.astype(np.float64), flags, recall)
    tau = torch.empty(1, device="cuda")
    gt.gtmp_surrogate_threshold(torch.from_numpy(z).cuda(), torch.from_numpy(flags).cuda(), recall, tau)
    got = float(tau.item())
    if np.isnan(want):
        assert np.isnan(got)
    else:
        assert got == want, (got, want)
    # the recall it promises
    if (flags == 0).any() and np.isfinite(got):
        zf = z[flags == 0].astype(np.float64)
        assert np.mean(zf <= got) >= recall - 1e-12


# ------------------------------------------------- biased heuristic half
def _clear_tau(zs):
    """The middle of the widest gap between sorted candidate logits in their
    central 90 %: a threshold whose decisions no logit error within Z_LOOSE
    can change."""
    z = np.sort(np.concatenate([np.asarray(a, np.float64) for a in zs]))
    lo, hi = int(0.05 * z.size), int(0.95 * z.size)
    gaps = z[lo + 1:hi + 1] - z[lo:hi]
    k = int(np.argmax(gaps))
    tau = 0.5 * (z[lo + k] + z[lo + k + 1])
    assert gaps[k] > 2 * Z_LOOSE * max(1.0, abs(tau)), gaps[k]
    return tau


@pytest.mark.parametrize("name,M,N,n_old,cscale", [("arm7", 3, 48, 24, 1.5), ("2d-small", 4, 64, 0, 1.3)])
def test_biased_expansion_bit_exact(gt, orc, name, M, N, n_old, cscale):
    import oracle.anytime as OA
    w = wl.make_workload(name, 1, M=M, N=N)
    d = w["d"]
    net, P, Bf = _net(gt, seed=4, d=d)
    q0, qg = w["q0"].astype(np.float64), w["goals"][0].astype(np.float64)
    c = np.float32(np.linalg.norm(qg - q0) * cscale)
    Q_old = orc.sample_layers(M, max(n_old, 1), d, w["lo"], w["hi"], 3, 1)[:, :n_old]
    # the candidates of a layer depend on the decisions of the layers before
    # it: iterate until the threshold is clear of every candidate it meets
    tau = 0.0
    for _ in range(6):
        trace = []
        want = OA.expand_samples(w, [Q_old[m] for m in range(M)], M, N, c, 13, 6, bias=(P, Bf, tau), trace=trace)
        z = np.concatenate(trace)
        if np.min(np.abs(z - tau)) > Z_LOOSE * max(1.0, abs(tau)):
            break
        tau = _clear_tau(trace)
    else:
        raise AssertionError("no clear threshold")
    kept = sum(int((z <= tau).sum()) for z in trace)
    _say("biased expand", name, "tau", tau, "candidates", sum(z.size for z in trace), "kept", kept)
    prob = gt.make_problem(d, M, N, 1, w["H"], w["lo"], w["hi"], w["penalty"])
    ws = gt._aligned_workspace(gt.gtmp_expand_biased_workspace_size(prob))
    Qn = torch.empty((M, N, d), device="cuda")
    dev = lambda a: torch.from_numpy(np.ascontiguousarray(a, np.float32)).cuda()
    Qo = dev(Q_old) if n_old > 0 else None
    gt.gtmp_expand_samples_biased(prob, dev(w["q0"]), dev(w["goals"]), Qo, n_old, Qn, dev(np.array([c])), 13, 6, net,
                                  tau, ws)
    got = Qn.cpu().numpy()
    assert np.array_equal(got.view(np.uint32), np.stack(want).view(np.uint32))
    assert 0 < kept < sum(z.size for z in trace)


def _selector_net(gt, d):
    """Closed-form surrogate: logit = 3 relu(q_0 / pi) - 1.  One weight per
    layer is non-zero and every product and sum is exact in FP32, so the GPU
    and the oracle compute the same logits and take the same decisions."""
    P = {k: np.zeros(s) for k, s in OS.shapes().items()}
    P["W1"][0, 0] = 1.0
    for l in (2, 3, 4):
        P[f"W{l}"][0, 0] = 1.0
    P["w5"][0] = 3.0
    P["b5"][0] = -1.0
    _, Bf = wl.surrogate_init(0, d)
    return gt.Surrogate({k: v.astype(np.float32) for k, v in P.items()}, Bf, batch=256), P, Bf


@pytest.mark.parametrize("name,sched,kw", [("2d-small", (2, 4, 16, 64, 6), {}),
                                           ("arm7", (2, 3, 16, 48, 4), dict(H=12))])
def test_biased_growing_plan_matches_oracle(gt, name, sched, kw):
    import oracle.anytime as OA
    import parity as PR
    w = wl.make_workload(name, 1, **kw)
    M_min, M_max, N_min, N_max, S = sched
    net, P, Bf = _selector_net(gt, w["d"])
    _say("biased growing", name, sched)
    ap = gt.AnytimePlanner(w, gt.GTMP_ANYTIME_GROWING, S, M_min=M_min, M_max=M_max, N_min=N_min, N_max=N_max,
                           bias=net, bias_tau=0.0)
    ap.run(w["seed"])
    torch.cuda.synchronize()
    best, costs, stages = OA.plan_growing(w, M_min, M_max, N_min, N_max, S, w["seed"], bias=(P, Bf, 0.0))
    got = ap.stage_costs.cpu().numpy().astype(np.float64)[:len(costs)]
    np.testing.assert_allclose(got, costs, rtol=PR.REL)
    assert float(ap.best_cost.item()) == pytest.approx(best["cost"], rel=PR.REL)
    # the biased run differs from the unbiased one once a bound exists
    plain = OA.plan_growing(w, M_min, M_max, N_min, N_max, S, w["seed"])[1]
    _say("costs biased", costs, "plain", plain)


# ----------------------------------------------------------------- gain
@pytest.fixture(scope="module")
def trained(gt):
    """Surrogate trained on the arm scene: 1 M uniform + 1 M edge states with
    exact labels, 4 epochs of Adam at batch 8192."""
    w = wl.make_workload("arm7", 0)
    P, Bf = wl.surrogate_init(7, 7)
    net = gt.Surrogate(P, Bf, batch=8192)
    X, y = gt.make_labels(w, 1 << 20, seed=101, stage=0)
    losses = net.train(X, y, epochs=4).cpu().numpy()
    Xh, yh = gt.make_labels(w, 1 << 14, seed=101, stage=1)
    acc = float(np.mean((net.infer(Xh).cpu().numpy() > 0) == (yh.cpu().numpy() == 1)))
    _say("trained: loss", losses[:3].mean(), "->", losses[-20:].mean(), "held-out accuracy", acc)
    return w, net, acc


def test_bias_gain_more_free_heuristic_samples(gt, orc, trained):
    """What the trained network gains for the sampler: with the bias, the
    heuristic half of an expansion holds more collision-free samples than
    without it (same key, same bound, same old samples)."""
    import oracle.anytime as OA
    w, net, acc = trained
    M, N, n_old, seed, stage = 8, 512, 256, 31, 2
    d = 7
    q0, qg = w["q0"].astype(np.float64), w["goals"][0].astype(np.float64)
    c = np.float32(1.3 * np.linalg.norm(qg - q0))
    Q_old = orc.sample_layers(M, n_old, d, w["lo"], w["hi"], 21, 0)
    prob = gt.make_problem(d, M, N, 1, w["H"], w["lo"], w["hi"], w["penalty"])
    dev = lambda a: torch.from_numpy(np.ascontiguousarray(a, np.float32)).cuda()
    heur = np.array([[OA.coin_heuristic(seed, stage, m, n) for n in range(n_old, N)] for m in range(M)])
    robot = gt.make_arm_robot(w["dh"], w["sph_link"], w["sph_t"], w["sph_r"])
    scene = gt.Scene(3, w["obs_spheres"], w["obs_boxes"])
    free = {}
    for biased in (False, True):
        Qn = torch.empty((M, N, d), device="cuda")
        if biased:
            ws = gt._aligned_workspace(gt.gtmp_expand_biased_workspace_size(prob))
            gt.gtmp_expand_samples_biased(prob, dev(w["q0"]), dev(w["goals"]), dev(Q_old), n_old, Qn,
                                          dev(np.array([c])), seed, stage, net, 0.0, ws)
        else:
            ws = gt._aligned_workspace(gt.gtmp_expand_workspace_size(prob))
            gt.gtmp_expand_samples(prob, dev(w["q0"]), dev(w["goals"]), dev(Q_old), n_old, Qn, dev(np.array([c])),
                                   seed, stage, ws)
        X = Qn[:, n_old:].reshape(-1, d).contiguous()
        coll = torch.empty(X.shape[0], device="cuda", dtype=torch.uint8)
        gt.gtmp_state_check(robot, scene, d, X, None, coll)
        cc = coll.cpu().numpy().reshape(M, N - n_old)
        free[biased] = float(1.0 - cc[heur].mean())
    _say("free heuristic samples: plain", free[False], "biased", free[True], "(net accuracy", acc, ")")
    assert free[True] > free[False] + 0.05
