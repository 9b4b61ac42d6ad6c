"""The C-ABI library loads, exports every entry point declared in
include/gtmp.h, and rejects invalid arguments on the host before any launch
(no GPU needed: validation precedes every HIP call)."""
import ctypes as C
import math
import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "gtmp.h")
LIB = os.path.join(ROOT, "paper_2608_25830_amd", "libgtmp.so")


def declared_functions():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(gtmp_[a-z0-9_]+)\s*\(", src)))


def test_header_declares_the_entry_points():
    names = declared_functions()
    for n in ["gtmp_sample_layers", "gtmp_edge_check_cost", "gtmp_minplus_sweep", "gtmp_extract_path",
              "gtmp_status_string", "gtmp_last_error"]:
        assert n in names


def test_library_exports_every_declared_symbol():
    lib = C.CDLL(LIB)
    missing = [n for n in declared_functions() if not hasattr(lib, n)]
    assert not missing, missing


@pytest.fixture(scope="module")
def g():
    from paper_2608_25830_amd import gtmp
    return gtmp


def _prob(g, **kw):
    a = dict(d=2, M=3, N=8, G=1, H=6, lo=[-1, -1], hi=[1, 1], penalty=1e3, max_edge_len=math.inf)
    a.update(kw)
    return g.make_problem(**a)


@pytest.mark.parametrize("kw", [dict(d=0), dict(d=9, lo=[0] * 9, hi=[1] * 9), dict(M=0), dict(N=0), dict(G=0),
                                dict(H=1), dict(H=257), dict(lo=[1, -1], hi=[0, 1]), dict(penalty=-1.0),
                                dict(penalty=float("nan")), dict(max_edge_len=0.0), dict(N=70000, M=3)])
def test_invalid_problem_rejected(g, kw):
    p = _prob(g, **kw)
    n = C.c_size_t()
    assert g._lib.gtmp_edge_check_workspace_size(C.byref(p), C.byref(n)) == g.GTMP_EINVAL
    assert g._lib.gtmp_last_error().decode() != ""
    assert g._lib.gtmp_sample_layers(C.byref(p), 1, 0, C.c_void_p(16), None) == g.GTMP_EINVAL


def test_workspace_size_is_positive_and_monotone(g):
    a = g.gtmp_edge_check_workspace_size(_prob(g, N=64))
    b = g.gtmp_edge_check_workspace_size(_prob(g, N=256))
    assert 0 < a < b and a % 256 == 0


def test_null_buffers_rejected(g):
    p = _prob(g)
    assert g._lib.gtmp_sample_layers(C.byref(p), 1, 0, None, None) == g.GTMP_EINVAL
    assert g._lib.gtmp_minplus_sweep(3, 8, 1, None, None, None, None, None, None, None, None, None) == g.GTMP_EINVAL
    assert g._lib.gtmp_minplus_sweep(0, 8, 1, *([C.c_void_p(16)] * 8), None) == g.GTMP_EINVAL
    assert g._lib.gtmp_extract_path(3, 8, 1, 9, *([C.c_void_p(16)] * 9), None) == g.GTMP_EINVAL


def test_bad_models_rejected(g):
    p = _prob(g)
    scene = g.gtmp_scene()
    scene.wdim = 2
    robot = g.make_point_robot()
    ws = C.c_void_p(256)
    args = lambda: (C.byref(p), C.byref(robot), C.byref(scene), *([C.c_void_p(256)] * 9), ws, C.c_size_t(1 << 30),
                    None, None)
    # obstacle count without a pointer
    scene.n_spheres = 3
    assert g._lib.gtmp_edge_check_cost(*args()) == g.GTMP_EINVAL
    scene.n_spheres = 0
    # 3D scene for a 2D point robot
    scene.wdim = 3
    assert g._lib.gtmp_edge_check_cost(*args()) == g.GTMP_EINVAL
    scene.wdim = 2
    # unknown robot kind
    robot.kind = 7
    assert g._lib.gtmp_edge_check_cost(*args()) == g.GTMP_EINVAL
    # arm with a joint count different from d, or spheres out of link order
    arm = g.make_arm_robot(np.zeros((2, 4), np.float32) + [0.2, 0, 0, 0], [2, 1], [0.5, 0.5], [0.05, 0.05])
    scene.wdim = 3
    p3 = _prob(g, d=2)
    assert g._lib.gtmp_edge_check_cost(C.byref(p3), C.byref(arm), C.byref(scene), *([C.c_void_p(256)] * 9), ws,
                                       C.c_size_t(1 << 30), None, None) == g.GTMP_EINVAL
    assert "link order" in g._lib.gtmp_last_error().decode()
    # workspace too small
    robot = g.make_point_robot()
    scene.wdim = 2
    assert g._lib.gtmp_edge_check_cost(C.byref(p), C.byref(robot), C.byref(scene), *([C.c_void_p(256)] * 9), ws,
                                       C.c_size_t(16), None, None) == g.GTMP_EWORKSPACE


# ------------------------------------------------------------ anytime / batch / surrogate validation
def _net(g, d=7, params=256, p16=256, fourier=256):
    return g.gtmp_surrogate(d, C.c_void_p(fourier) if fourier else None, C.c_void_p(params) if params else None,
                            C.c_void_p(p16) if p16 else None)


def test_surrogate_layout_and_workspace(g):
    off = g.gtmp_surrogate_layout()
    assert off[0] == 0 and off[10] == 64 * 256 + 256 + 3 * (256 * 256 + 256) + 256 + 1
    assert all(o % 64 == 0 for o in off[:9])  # every weight block 16-byte aligned in both precisions
    n = C.c_size_t()
    assert g._lib.gtmp_surrogate_workspace_size(0, C.byref(n)) == g.GTMP_EINVAL
    assert g.gtmp_surrogate_workspace_size(256) < g.gtmp_surrogate_workspace_size(8192)


@pytest.mark.parametrize("bad", [dict(d=0), dict(d=9), dict(params=0), dict(p16=0), dict(fourier=0),
                                 dict(p16=258), dict(params=260)])
def test_surrogate_bad_net_rejected(g, bad):
    net = _net(g, **bad)
    ws = C.c_void_p(1 << 20)
    assert g._lib.gtmp_surrogate_infer(C.byref(net), 10, C.c_void_p(256), C.c_void_p(256), ws, 1 << 30,
                                       None) == g.GTMP_EINVAL
    assert g._lib.gtmp_surrogate_refresh_bf16(C.byref(net), None) == g.GTMP_EINVAL


def test_surrogate_calls_validate_sizes(g):
    net = _net(g)
    ws = C.c_void_p(1 << 20)
    big = C.c_size_t(1 << 40)
    # training batches are positive multiples of 256
    for n in (0, 100, 300):
        assert g._lib.gtmp_surrogate_grad(C.byref(net), n, *([C.c_void_p(256)] * 5), ws, big, None) == g.GTMP_EINVAL
    # workspace too small / misaligned
    assert g._lib.gtmp_surrogate_grad(C.byref(net), 256, *([C.c_void_p(256)] * 5), ws, C.c_size_t(1024),
                                      None) == g.GTMP_EWORKSPACE
    assert g._lib.gtmp_surrogate_infer(C.byref(net), 10, C.c_void_p(256), C.c_void_p(256), C.c_void_p(1 << 20 | 8),
                                       big, None) == g.GTMP_EINVAL
    # Adam hyper-parameters
    for t, lr, b1, b2, eps in ((0, 1e-3, .9, .999, 1e-8), (1, -1.0, .9, .999, 1e-8), (1, 1e-3, 1.0, .999, 1e-8),
                               (1, 1e-3, .9, .999, 0.0)):
        assert g._lib.gtmp_surrogate_adam(C.byref(net), *([C.c_void_p(256)] * 3), t, lr, b1, b2, eps,
                                          None) == g.GTMP_EINVAL
    # label states need interior states; prune needs matching d
    p = _prob(g, H=2)
    assert g._lib.gtmp_surrogate_label_states(C.byref(p), 1, 0, 10, C.c_void_p(256), None) == g.GTMP_EINVAL
    p = _prob(g)
    assert g._lib.gtmp_surrogate_prune(C.byref(p), C.byref(net), *([C.c_void_p(256)] * 3), None, 0.0,
                                       C.c_void_p(256), None, ws, big, None) == g.GTMP_EINVAL  # net d = 7, problem d = 2
    p7 = g.make_problem(7, 3, 16, 1, 8, [-3] * 7, [3] * 7, 1e3)
    n = C.c_size_t()
    assert g._lib.gtmp_surrogate_prune_workspace_size(C.byref(p7), C.byref(n)) == g.GTMP_OK and n.value > 0
    assert g._lib.gtmp_surrogate_prune(C.byref(p7), C.byref(net), *([C.c_void_p(256)] * 3), None, float("nan"),
                                       C.c_void_p(256), None, ws, big, None) == g.GTMP_EINVAL  # NaN threshold
    assert g._lib.gtmp_surrogate_prune(C.byref(p7), C.byref(net), *([C.c_void_p(256)] * 3), None, 0.0,
                                       C.c_void_p(256), None, ws, n.value - 1, None) == g.GTMP_EWORKSPACE


def test_noalloc_edge_check_validates(g):
    """The static-scratch edge check rejects, on the host, invalid problems
    and problems whose scratch exceeds the static array."""
    p = C.c_void_p(256)
    f = g._lib.gtmp_edge_check_cost_noalloc
    bad = _prob(g, N=0)
    assert f(C.byref(bad), None, None, *([p] * 9), None, None) == g.GTMP_EINVAL
    big = _prob(g, d=7, M=8, N=4096, lo=[-3] * 7, hi=[3] * 7)
    assert g.gtmp_edge_check_workspace_size(big) > g.NOALLOC_SCRATCH_BYTES
    assert f(C.byref(big), None, None, *([p] * 9), None, None) == g.GTMP_EINVAL
    assert "scratch" in g._lib.gtmp_last_error().decode()


def test_surrogate_threshold_validates(g):
    n = C.c_size_t()
    assert g._lib.gtmp_surrogate_threshold_workspace_size(C.byref(n)) == 0 and n.value >= 256
    ws, big, p = C.c_void_p(1 << 20), C.c_size_t(1 << 20), C.c_void_p(256)
    f = g._lib.gtmp_surrogate_threshold
    assert f(p, p, -1, 0.999, p, ws, big, None) == g.GTMP_EINVAL  # negative E
    for r in (0.0, -0.5, 1.5, float("nan")):
        assert f(p, p, 10, r, p, ws, big, None) == g.GTMP_EINVAL
    assert f(None, p, 10, 0.999, p, ws, big, None) == g.GTMP_EINVAL
    assert f(p, p, 10, 0.999, None, ws, big, None) == g.GTMP_EINVAL
    assert f(p, p, 10, 0.999, p, C.c_void_p((1 << 20) | 8), big, None) == g.GTMP_EINVAL
    assert f(p, p, 10, 0.999, p, ws, C.c_size_t(16), None) == g.GTMP_EWORKSPACE


def test_biased_expansion_validates(g):
    p = _prob(g)
    net = _net(g, d=2)
    need = g.gtmp_expand_biased_workspace_size(p)
    assert need > g.gtmp_expand_workspace_size(p)
    args = lambda n_old, ws_bytes, netp: (C.byref(p), C.c_void_p(256), C.c_void_p(256), C.c_void_p(1 << 20), n_old,
                                          C.c_void_p(2 << 20), C.c_void_p(256), 1, 0, netp, 0.0, C.c_void_p(1 << 24),
                                          C.c_size_t(ws_bytes), None)
    assert g._lib.gtmp_expand_samples_biased(*args(-1, need, C.byref(net))) == g.GTMP_EINVAL
    assert g._lib.gtmp_expand_samples_biased(*args(9, need, C.byref(net))) == g.GTMP_EINVAL
    assert g._lib.gtmp_expand_samples_biased(*args(4, need - 1, C.byref(net))) == g.GTMP_EWORKSPACE
    bad = _net(g, d=3)
    assert g._lib.gtmp_expand_samples_biased(*args(4, need, C.byref(bad))) == g.GTMP_EINVAL


def test_anytime_and_batch_options_validate(g):
    p = _prob(g)
    o = g.gtmp_anytime_opts()
    o.mode, o.max_stages = g.GTMP_ANYTIME_GROWING, 4
    o.M_min, o.M_max, o.N_min, o.N_max = 2, 1, 4, 8  # M_min > M_max
    n = C.c_size_t()
    assert g._lib.gtmp_anytime_workspace_size(C.byref(p), C.byref(o), C.byref(n)) == g.GTMP_EINVAL
    o.M_min, o.M_max = 1, 3
    assert g._lib.gtmp_anytime_workspace_size(C.byref(p), C.byref(o), C.byref(n)) == g.GTMP_OK
    o.max_stages = 0
    assert g._lib.gtmp_anytime_workspace_size(C.byref(p), C.byref(o), C.byref(n)) == g.GTMP_EINVAL
    o.max_stages, o.mode = 4, 7
    assert g._lib.gtmp_anytime_workspace_size(C.byref(p), C.byref(o), C.byref(n)) == g.GTMP_EINVAL
    # shortcutting: at most 64 waypoints, and it costs workspace
    o.mode, o.M_max = g.GTMP_ANYTIME_GROWING, 62
    assert g._lib.gtmp_anytime_workspace_size(C.byref(p), C.byref(o), C.byref(n)) == g.GTMP_OK
    n0 = n.value
    o.simplify = 1
    assert g._lib.gtmp_anytime_workspace_size(C.byref(p), C.byref(o), C.byref(n)) == g.GTMP_OK and n.value > n0
    o.M_max = 63
    assert g._lib.gtmp_anytime_workspace_size(C.byref(p), C.byref(o), C.byref(n)) == g.GTMP_EINVAL
    o.mode, o.simplify, o.M_max = g.GTMP_ANYTIME_RESTART, 1, 3
    assert g._lib.gtmp_anytime_workspace_size(C.byref(_prob(g, M=63)), C.byref(o), C.byref(n)) == g.GTMP_EINVAL
    # batch: empty, bad options, bad plan
    descs = (g.gtmp_plan_desc * 1)()
    D = descs[0]
    D.problem = p
    D.robot = g.make_point_robot()
    D.scene.wdim, D.scene.n_spheres, D.scene.spheres = 2, 1, 256
    D.q0, D.goals, D.seed, D.mode, D.stages, D.M_min, D.N_min = 256, 256, 1, g.GTMP_ANYTIME_RESTART, 2, 3, 8
    bo = g.gtmp_batch_opts()
    assert g._lib.gtmp_batch_workspace_size(descs, 0, C.byref(bo), C.byref(n)) == g.GTMP_EINVAL
    assert g._lib.gtmp_batch_workspace_size(descs, 1, C.byref(bo), C.byref(n)) == g.GTMP_OK and n.value > 0
    for field, val in (("sphere_chunks", 3), ("states_per_iter", 9), ("blocks_per_cu", 40)):
        bo2 = g.gtmp_batch_opts()
        setattr(bo2, field, val)
        assert g._lib.gtmp_batch_workspace_size(descs, 1, C.byref(bo2), C.byref(n)) == g.GTMP_EINVAL, field
    D.stages = 0
    assert g._lib.gtmp_batch_workspace_size(descs, 1, C.byref(bo), C.byref(n)) == g.GTMP_EINVAL


def test_class_entry_points_validate(g):
    n = C.c_size_t()
    assert g._lib.gtmp_class_sweep_workspace_size(127, 16, 8, C.byref(n)) == g.GTMP_EINVAL  # M > 126
    assert g._lib.gtmp_class_sweep_workspace_size(16, 16, 8, C.byref(n)) == g.GTMP_OK
    assert g._lib.gtmp_class_sweep_workspace_size(3, 16, 65, C.byref(n)) == g.GTMP_EINVAL  # L > 64
    assert g._lib.gtmp_class_sweep_workspace_size(3, 16, 8, C.byref(n)) == g.GTMP_OK and n.value > 0
    bufs = [C.c_void_p(256)] * 6
    outs = [C.c_void_p(256)] * 5
    assert g._lib.gtmp_class_sweep(3, 16, 1, 8, *bufs, 1e3, C.c_void_p(256), 17, *outs, C.c_void_p(1 << 20),
                                   1 << 30, None) == g.GTMP_EINVAL  # k > 16
    assert g._lib.gtmp_class_sweep(3, 16, 1, 8, *bufs, 1e3, C.c_void_p(256), 4, *outs, C.c_void_p(1 << 20),
                                   16, None) == g.GTMP_EWORKSPACE
    p3 = g.make_problem(3, 3, 8, 1, 6, [-1] * 3, [1] * 3, 1e3)
    assert g._lib.gtmp_class_anytime_workspace_size(C.byref(p3), 8, C.byref(n)) == g.GTMP_EINVAL  # d != 2
    p2 = _prob(g)
    assert g._lib.gtmp_class_anytime_workspace_size(C.byref(p2), 8, C.byref(n)) == g.GTMP_OK


def test_simplify_validates(g):
    scene = g.gtmp_scene()
    scene.wdim = 2
    robot = g.make_point_robot()
    bufs = [C.c_void_p(256)] * 4  # valid, idx, count, cost
    call = lambda d, B, K, H, wp=C.c_void_p(256), b=bufs: g._lib.gtmp_simplify_paths(
        C.byref(robot), C.byref(scene), d, B, K, H, wp, *b, None, None)
    assert call(2, 4, 1, 8) == g.GTMP_EINVAL  # K < 2
    assert call(2, 4, 65, 8) == g.GTMP_EINVAL  # K > 64
    assert call(2, 4, 8, 1) == g.GTMP_EINVAL  # H < 2
    assert call(2, 4, 8, 257) == g.GTMP_EINVAL  # H > max
    assert call(2, -1, 8, 8) == g.GTMP_EINVAL
    assert call(2, 1 << 30, 8, 8) == g.GTMP_EINVAL  # B K^2 too large
    assert call(3, 4, 8, 8) == g.GTMP_EINVAL  # point robot needs d == wdim
    assert call(2, 4, 8, 8, wp=None) == g.GTMP_EINVAL
    assert call(2, 4, 8, 8, b=[C.c_void_p(256)] * 3 + [None]) == g.GTMP_EINVAL  # cost NULL
    assert call(2, 0, 8, 8, wp=None, b=[None] * 4) == g.GTMP_OK  # nothing to do


def test_rrtc_validates(g):
    p = _prob(g)
    scene = g.gtmp_scene()
    scene.wdim = 2
    robot = g.make_point_robot()
    n = C.c_size_t()
    assert g._lib.gtmp_rrtc_workspace_size(C.byref(p), C.byref(n)) == g.GTMP_OK and n.value > 0
    ok = dict(budget=10, tree_cap=64, step=0.5, resolution=0.1, ell_factor=1.5)
    bufs = [C.c_void_p(256)] * 7

    def repair(o, ws=C.c_void_p(1 << 20), nbytes=1 << 30, b=bufs):
        return g._lib.gtmp_rrtc_repair(C.byref(p), C.byref(robot), C.byref(scene), *b, 1, 0, C.byref(o), ws,
                                       nbytes, None)
    for k, v in (("budget", 0), ("tree_cap", 1), ("tree_cap", 5000), ("step", 0.0), ("step", float("inf")),
                 ("resolution", -1.0), ("ell_factor", 0.9), ("ell_factor", float("nan"))):
        kw = dict(ok)
        kw[k] = v
        assert repair(g.make_rrtc_opts(**kw)) == g.GTMP_EINVAL, (k, v)
    kw = dict(ok, step=100.0, resolution=0.01)  # more than 4096 states per extension
    assert repair(g.make_rrtc_opts(**kw)) == g.GTMP_EINVAL
    p3 = _prob(g, d=8, lo=[-1] * 8, hi=[1] * 8)
    assert g._lib.gtmp_rrtc_repair(C.byref(p3), C.byref(g.make_point_robot()), C.byref(scene), *bufs, 1, 0,
                                   C.byref(g.make_rrtc_opts(**dict(ok, tree_cap=4096))), C.c_void_p(1 << 20),
                                   1 << 30, None) == g.GTMP_EINVAL  # LDS limit at d = 8
    o = g.make_rrtc_opts(**ok)
    assert repair(o, b=bufs[:6] + [None]) == g.GTMP_EINVAL  # flags NULL
    assert repair(o, nbytes=16) == g.GTMP_EWORKSPACE
    assert repair(o, ws=C.c_void_p((1 << 20) + 8)) == g.GTMP_EINVAL  # alignment
    E = 8 + 2 * 64 + 8
    assert g._lib.gtmp_rrtc_local_path(C.byref(p), C.byref(robot), C.byref(scene), *bufs[:3], E, 1, 0, C.byref(o),
                                       *bufs[:3], None) == g.GTMP_EINVAL  # edge out of range


def test_lazy_validates(g):
    p = _prob(g)
    scene = g.gtmp_scene()
    scene.wdim = 2
    robot = g.make_point_robot()
    n = C.c_size_t()
    assert g._lib.gtmp_lazy_workspace_size(C.byref(p), C.byref(n)) == g.GTMP_OK and n.value > 0
    bufs = [C.c_void_p(256)] * 14
    r = C.c_int32(0)

    def call(band=0.1, rounds=10, b=bufs, ws=C.c_void_p(1 << 20), nbytes=1 << 30):
        return g._lib.gtmp_plan_lazy(C.byref(p), C.byref(robot), C.byref(scene), *b, band, rounds, None,
                                     C.byref(r), ws, nbytes, None, None)
    assert call(band=-0.1) == g.GTMP_EINVAL
    assert call(band=float("inf")) == g.GTMP_EINVAL
    assert call(rounds=0) == g.GTMP_EINVAL
    assert call(b=bufs[:6] + [None] + bufs[7:]) == g.GTMP_EINVAL  # flags NULL
    assert call(nbytes=16) == g.GTMP_EWORKSPACE
    assert call(ws=C.c_void_p((1 << 20) + 4)) == g.GTMP_EINVAL
    assert g._lib.gtmp_status_string(g.GTMP_INCOMPLETE) == b"GTMP_INCOMPLETE"


def test_anytime_lp_option_validates(g):
    p = _prob(g)
    o = g.gtmp_anytime_opts()
    o.mode, o.max_stages = g.GTMP_ANYTIME_RESTART, 3
    n = C.c_size_t()
    assert g._lib.gtmp_anytime_workspace_size(C.byref(p), C.byref(o), C.byref(n)) == g.GTMP_OK
    n0 = n.value
    lp = g.make_rrtc_opts(20, 64, 0.5, 0.1, 1.5)
    o.lp = C.cast(C.pointer(lp), C.c_void_p).value
    assert g._lib.gtmp_anytime_workspace_size(C.byref(p), C.byref(o), C.byref(n)) == g.GTMP_OK and n.value > n0
    bad = g.make_rrtc_opts(0, 64, 0.5, 0.1, 1.5)  # budget 0
    o.lp = C.cast(C.pointer(bad), C.c_void_p).value
    assert g._lib.gtmp_anytime_workspace_size(C.byref(p), C.byref(o), C.byref(n)) == g.GTMP_EINVAL
