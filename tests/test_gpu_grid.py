"""The obstacle-bin filter of the edge check (the automatic choice for arm
scenes of at most 64 obstacles and for point-robot graphs of at least 1024
tiles whose scene has at most 96) against the test of every robot sphere or
point state against every obstacle (sphere_chunks = 2): both decide each
state by the same FP32 difference-form gaps, so every edge cost and flag must
agree bit for bit.  Cases: the arm7 scenes, per-sphere radii, one and two mask
words (32 / 33 / 60 obstacles), the fallback above 64, no obstacles,
degenerate obstacles and robot spheres of radius 0, a scene scaled by 50, and
the lazy rounds' compacted-tile kernel.  Agreement with the oracle is checked
by the parity tests, which run the automatic choice."""
import numpy as np
import pytest
import torch

import workloads as wl

pytestmark = pytest.mark.gpu


def _say(*a):
    print("[case]", *a, flush=True)


def _flat(pl):
    M = pl.M
    parts = [pl.C_s.cpu().numpy().ravel()]
    if M > 1:
        parts.append(pl.C_h.cpu().numpy()[: M - 1].ravel())
    parts.append(pl.C_l.cpu().numpy().ravel())
    return np.concatenate(parts)


def _both(gt, w, seed=None):
    """Edge costs and flags of one sample set under both tests (point robots:
    four states per lane and evaluation on both sides, as the bin kernel
    takes them, so that the same states are evaluated)."""
    out = []
    for chunks in (0, 2):
        pl = gt.Planner(w, flags=True)
        pl.opts.sphere_chunks = chunks
        pl.opts.states_per_iter = 4
        pl.sample(w["seed"] if seed is None else seed, 0)
        pl.check()
        torch.cuda.synchronize()
        out.append((_flat(pl), pl.flags.cpu().numpy().copy(), int(pl.stats[0].item())))
    return out


def _assert_same(res, label):
    (cg, fg, sg), (cd, fd, sd) = res
    n_free = int((fg == 0).sum())
    _say(label, "edges", fg.size, "free", n_free, "states grid", sg, "dense", sd)
    assert np.array_equal(fg, fd), f"{label}: flags differ at {np.flatnonzero(fg != fd)[:10]}"
    assert np.array_equal(cg.view(np.uint32), cd.view(np.uint32)), label
    assert sg == sd  # the same states are evaluated (same early exits)
    return n_free


def _obstacles(seed, n_sph, n_box, extent=1.0):
    g = np.random.default_rng(seed)
    sp = np.concatenate([g.uniform(-extent, extent, (n_sph, 3)), g.uniform(0.05, 0.2, (n_sph, 1))], 1)
    bx = np.concatenate([g.uniform(-extent, extent, (n_box, 3)), g.uniform(0.05, 0.2, (n_box, 3))], 1)
    return sp.astype(np.float32).reshape(n_sph, 4), bx.astype(np.float32).reshape(n_box, 6)


@pytest.mark.parametrize("scene", [0, 1, 2])
def test_grid_matches_full_test_arm7(gt, scene):
    w = wl.make_workload("arm7", scene, M=4, N=256)
    n_free = _assert_same(_both(gt, w), f"arm7 scene {scene}")
    assert 0 < n_free < w["N"] * (w["N"] * 3 + 2)


def test_grid_per_sphere_radii(gt):
    w = wl.make_workload("arm7", 0, M=3, N=256)
    g = np.random.default_rng(7)
    w["sph_r"] = g.uniform(0.02, 0.09, w["sph_r"].shape).astype(np.float32)
    _assert_same(_both(gt, w), "per-sphere radii")


@pytest.mark.parametrize("n_sph,n_box", [(16, 16), (17, 16), (30, 30), (0, 40), (40, 0), (40, 30)])
def test_grid_obstacle_counts(gt, n_sph, n_box):
    """32 obstacles fill one mask word, 33 and 60 take two, 70 fall back to the
    full test for both settings."""
    w = wl.make_workload("arm7", 1, M=3, N=192)
    w["obs_spheres"], w["obs_boxes"] = _obstacles(n_sph * 100 + n_box, n_sph, n_box)
    _assert_same(_both(gt, w), f"{n_sph} spheres + {n_box} boxes")


def test_grid_no_obstacles(gt):
    w = wl.make_workload("arm7", 0, M=3, N=128)
    w["obs_spheres"] = np.zeros((0, 4), np.float32)
    w["obs_boxes"] = np.zeros((0, 6), np.float32)
    res = _both(gt, w)
    _assert_same(res, "no obstacles")
    assert (res[0][1] == 0).all()


def test_grid_degenerate_obstacles_and_radius(gt):
    """Flat boxes (one half-extent 0), point boxes, sphere obstacles of radius
    0 and robot spheres of radius 0: the bins still list every contact."""
    w = wl.make_workload("arm7", 2, M=3, N=192)
    sp, bx = _obstacles(5, 12, 14)
    sp[:4, 3] = 0.0
    bx[np.arange(5), 3 + np.arange(5) % 3] = 0.0
    bx[5:8, 3:] = 0.0
    w["obs_spheres"], w["obs_boxes"] = sp, bx
    _assert_same(_both(gt, w), "degenerate obstacles")
    w["sph_r"] = np.zeros_like(w["sph_r"])
    _assert_same(_both(gt, w), "robot radius 0")


def test_grid_scaled_scene(gt):
    """Arm and obstacles scaled by 50: the bin maps follow the scene's extent."""
    w = wl.make_workload("arm7", 0, M=3, N=192)
    w["dh"] = w["dh"].copy()
    w["dh"][:, 0] *= 50.0
    w["dh"][:, 2] *= 50.0
    w["sph_r"] = w["sph_r"] * 50.0
    w["obs_spheres"] = w["obs_spheres"] * 50.0
    w["obs_boxes"] = w["obs_boxes"] * 50.0
    _assert_same(_both(gt, w), "scaled by 50")


@pytest.mark.parametrize("band", [0.0, 0.5])
def test_grid_lazy_rounds(gt, band):
    """Lazy rounds run the compacted-tile kernel: the filtered and the full
    test give the same rounds, checked edges and plan."""
    w = wl.make_workload("arm7", 1, M=4, N=256)
    res = []
    for chunks in (0, 2):
        pl = gt.Planner(w, flags=True)
        pl.opts.sphere_chunks = chunks
        stats = torch.zeros(2, device="cuda", dtype=torch.int64)
        st, rounds = pl.plan_lazy(w["seed"], 0, band=band, max_rounds=20000, stats=stats)
        torch.cuda.synchronize()
        res.append((st, rounds, stats.cpu().numpy().copy(), pl.flags.cpu().numpy().copy(), _flat(pl),
                    float(pl.V_s.item())))
    _say("lazy band", band, "rounds", res[0][1], res[1][1], "V_s", res[0][5], res[1][5])
    assert res[0][0] == res[1][0] == gt.GTMP_OK
    assert res[0][1] == res[1][1]
    assert np.array_equal(res[0][2], res[1][2])
    assert np.array_equal(res[0][3], res[1][3])
    assert np.array_equal(res[0][4].view(np.uint32), res[1][4].view(np.uint32))
    assert res[0][5] == res[1][5]


# ---------------------------------------------------------------- against the oracle
@pytest.mark.parametrize("variant", ["radii", "two_words", "radii_two_words"])
@pytest.mark.parametrize("chunks", [0, 2])
def test_arm_variants_match_oracle(gt, orc, variant, chunks):
    """Per-sphere radii and scenes needing two mask words, through the bins
    and through the chunked test, against the FP64 oracle (flags exact
    outside the 1e-5 signed-distance band, costs within 1e-5 relative)."""
    from tests import parity as P
    w = wl.make_workload("arm7", 3, M=3, N=96)
    g = np.random.default_rng(11)
    if "radii" in variant:
        w["sph_r"] = g.uniform(0.02, 0.09, w["sph_r"].shape).astype(np.float32)
    if "two_words" in variant:
        w["obs_spheres"], w["obs_boxes"] = _obstacles(23, 26, 22)
    pl = gt.Planner(w, flags=True)
    pl.opts.sphere_chunks = chunks
    pl.plan(w["seed"], 0)
    torch.cuda.synchronize()
    Q = orc.sample_layers(w["M"], w["N"], w["d"], w["lo"], w["hi"], w["seed"], 0)
    assert np.array_equal(pl.Q.cpu().numpy(), Q)
    cost, minsd, flag = orc.edge_costs(orc.Model(w), w["M"], w["N"], w["G"], w["H"], w["q0"], w["goals"], Q,
                                       w["penalty"])
    got = P.flat(pl.C_s.cpu().numpy(), pl.C_h.cpu().numpy()[: w["M"] - 1], pl.C_l.cpu().numpy())
    rep = P.compare_edges(got, pl.flags.cpu().numpy(), P.flat(*cost), P.flat(*minsd), P.flat(*flag))
    _say("arm variant", variant, "chunks", chunks, rep)
    assert 0 < rep["failed"] < rep["edges"]


# ---------------------------------------------------------------- point robots
def _scene_2d(seed, n_circ, n_box):
    g = np.random.default_rng(seed)
    circ = np.concatenate([g.uniform(-10, 10, (n_circ, 2)), g.uniform(0.5, 1.0, (n_circ, 1))], 1)
    box = np.concatenate([g.uniform(-10, 10, (n_box, 2)), g.uniform(0.3, 1.5, (n_box, 2))], 1)
    return circ.astype(np.float32).reshape(n_circ, 3), box.astype(np.float32).reshape(n_box, 4)


@pytest.mark.parametrize("name", ["2d-large", "3d-point"])
@pytest.mark.parametrize("scene", [0, 1])
def test_point_grid_matches_full_test(gt, name, scene):
    """Point robots: the bins (automatic for a graph of at least 1024 tiles)
    against every state tested against every obstacle."""
    w = wl.make_workload(name, scene, M=5, N=256)  # 1026 tiles of 256 edges
    n_free = _assert_same(_both(gt, w), f"{name} scene {scene}")
    assert 0 < n_free < w["N"] * (w["N"] * 3 + 2)


@pytest.mark.parametrize("n_circ,n_box", [(20, 10), (40, 20), (60, 30), (70, 30), (0, 1)])
def test_point_grid_obstacle_counts(gt, n_circ, n_box):
    """One, two and three mask words (30 / 60 / 90 obstacles), the full test
    above 96 for both settings, and a single box."""
    w = wl.make_workload("2d-large", 0, M=3, N=320)
    w["circles"], w["boxes"] = _scene_2d(n_circ * 100 + n_box, n_circ, n_box)
    _assert_same(_both(gt, w), f"2d {n_circ} circles + {n_box} boxes")


def test_point_grid_degenerate(gt):
    """Circles of radius 0, flat and point boxes, every state in one bin
    column (a scene of obstacles stacked at one x)."""
    w = wl.make_workload("2d-large", 1, M=3, N=320)
    circ, box = _scene_2d(9, 30, 20)
    circ[:6, 2] = 0.0
    box[:5, 2] = 0.0
    box[5:9, 2:] = 0.0
    circ[10:20, 0] = 3.0
    w["circles"], w["boxes"] = circ, box
    _assert_same(_both(gt, w), "2d degenerate")


def test_point_grid_matches_oracle(gt, orc):
    """The automatic (bin) path of the 3D point robot against the FP64 oracle."""
    from tests import parity as P
    w = wl.make_workload("3d-point", 2, M=3, N=320)  # 1284 tiles
    pl = gt.Planner(w, flags=True)
    pl.plan(w["seed"], 0)
    torch.cuda.synchronize()
    Q = orc.sample_layers(w["M"], w["N"], w["d"], w["lo"], w["hi"], w["seed"], 0)
    assert np.array_equal(pl.Q.cpu().numpy(), Q)
    cost, minsd, flag = orc.edge_costs(orc.Model(w), w["M"], w["N"], w["G"], w["H"], w["q0"], w["goals"], Q,
                                       w["penalty"])
    got = P.flat(pl.C_s.cpu().numpy(), pl.C_h.cpu().numpy()[: w["M"] - 1], pl.C_l.cpu().numpy())
    rep = P.compare_edges(got, pl.flags.cpu().numpy(), P.flat(*cost), P.flat(*minsd), P.flat(*flag))
    _say("3d point oracle", rep)
    assert 0 < rep["failed"] < rep["edges"]
