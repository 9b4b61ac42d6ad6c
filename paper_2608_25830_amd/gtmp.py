"""Python binding of libgtmp.so (include/gtmp.h).

Argument marshalling only: every step of the planner runs in the library's
HIP kernels.  PyTorch provides device memory and the current HIP stream.  The
functions named ``gtmp_*`` map one to one onto the C entry points; ``Planner``
strings them together for one plan (sample -> edge check -> min-plus sweep ->
extraction) without any host synchronisation until results are read.

If the shared library is missing, importing this module raises: there is no
fallback path.
"""
from __future__ import annotations

import ctypes as C
import math
import os
from dataclasses import dataclass

import numpy as np
import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libgtmp.so")

if not os.path.exists(LIB_PATH):
    raise ImportError(f"{LIB_PATH} is not built; run `python -m paper_2608_25830_amd.build`")

_lib = C.CDLL(LIB_PATH)

GTMP_OK, GTMP_ENOPATH, GTMP_INCOMPLETE, GTMP_EINVAL, GTMP_EHIP, GTMP_EWORKSPACE = 0, 1, 2, -1, -2, -3
GTMP_MAX_DOF, GTMP_MAX_JOINTS, GTMP_MAX_ROBOT_SPHERES, GTMP_MAX_H = 8, 8, 64, 256
GTMP_ROBOT_POINT, GTMP_ROBOT_DH_ARM = 0, 1
GTMP_CHECK_FAST, GTMP_CHECK_FULL = 0, 1


class GtmpError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"{_lib.gtmp_status_string(status).decode()}: {msg}")
        self.status = status


class gtmp_problem(C.Structure):
    _fields_ = [("d", C.c_int32), ("M", C.c_int32), ("N", C.c_int32), ("G", C.c_int32), ("H", C.c_int32),
                ("lo", C.c_float * GTMP_MAX_DOF), ("hi", C.c_float * GTMP_MAX_DOF),
                ("penalty", C.c_float), ("max_edge_len", C.c_float)]


class gtmp_robot(C.Structure):
    _fields_ = [("kind", C.c_int32), ("n_joints", C.c_int32), ("n_spheres", C.c_int32), ("reserved", C.c_int32),
                ("dh", (C.c_float * 4) * GTMP_MAX_JOINTS),
                ("sph_link", C.c_int32 * GTMP_MAX_ROBOT_SPHERES),
                ("sph_t", C.c_float * GTMP_MAX_ROBOT_SPHERES),
                ("sph_r", C.c_float * GTMP_MAX_ROBOT_SPHERES)]


class gtmp_scene(C.Structure):
    _fields_ = [("wdim", C.c_int32), ("n_spheres", C.c_int32), ("spheres", C.c_void_p),
                ("n_boxes", C.c_int32), ("boxes", C.c_void_p)]


class gtmp_edge_opts(C.Structure):
    _fields_ = [("mode", C.c_int32), ("states_per_iter", C.c_int32), ("block", C.c_int32),
                ("blocks_per_cu", C.c_int32), ("sphere_chunks", C.c_int32), ("reserved", C.c_int32 * 3),
                ("stats", C.c_void_p), ("ev_begin", C.c_void_p), ("ev_end", C.c_void_p)]


_vp = C.c_void_p
_lib.gtmp_status_string.restype = C.c_char_p
_lib.gtmp_status_string.argtypes = [C.c_int]
_lib.gtmp_last_error.restype = C.c_char_p
_lib.gtmp_version.restype = C.c_char_p
_lib.gtmp_sample_layers.argtypes = [C.POINTER(gtmp_problem), C.c_uint64, C.c_uint64, _vp, _vp]
_lib.gtmp_edge_check_workspace_size.argtypes = [C.POINTER(gtmp_problem), C.POINTER(C.c_size_t)]
_lib.gtmp_edge_check_cost.argtypes = [C.POINTER(gtmp_problem), C.POINTER(gtmp_robot), C.POINTER(gtmp_scene),
                                      _vp, _vp, _vp, _vp, _vp, _vp, _vp, _vp, _vp, _vp, C.c_size_t,
                                      C.POINTER(gtmp_edge_opts), _vp]
_lib.gtmp_edge_check_cost_noalloc.argtypes = [C.POINTER(gtmp_problem), C.POINTER(gtmp_robot),
                                              C.POINTER(gtmp_scene)] + [_vp] * 9 + [C.POINTER(gtmp_edge_opts), _vp]
NOALLOC_SCRATCH_BYTES = 32 << 20
_lib.gtmp_state_check.argtypes = [C.POINTER(gtmp_robot), C.POINTER(gtmp_scene), C.c_int32, C.c_int64, _vp, _vp,
                                  _vp, _vp]
class gtmp_rrtc_opts(C.Structure):
    _fields_ = [("budget", C.c_int32), ("tree_cap", C.c_int32), ("step", C.c_float), ("resolution", C.c_float),
                ("ell_factor", C.c_float), ("reserved", C.c_int32), ("stats", C.c_void_p)]


_lib.gtmp_rrtc_workspace_size.argtypes = [C.POINTER(gtmp_problem), C.POINTER(C.c_size_t)]
_lib.gtmp_rrtc_repair.argtypes = [C.POINTER(gtmp_problem), C.POINTER(gtmp_robot), C.POINTER(gtmp_scene)] + \
    [_vp] * 7 + [C.c_uint64, C.c_uint64, C.POINTER(gtmp_rrtc_opts), _vp, C.c_size_t, _vp]
_lib.gtmp_rrtc_local_path.argtypes = [C.POINTER(gtmp_problem), C.POINTER(gtmp_robot), C.POINTER(gtmp_scene)] + \
    [_vp] * 3 + [C.c_uint64, C.c_uint64, C.c_uint64, C.POINTER(gtmp_rrtc_opts), _vp, _vp, _vp, _vp]
_lib.gtmp_lazy_workspace_size.argtypes = [C.POINTER(gtmp_problem), C.POINTER(C.c_size_t)]
_lib.gtmp_plan_lazy.argtypes = [C.POINTER(gtmp_problem), C.POINTER(gtmp_robot), C.POINTER(gtmp_scene)] + \
    [_vp] * 14 + [C.c_float, C.c_int32, _vp, C.POINTER(C.c_int32), _vp, C.c_size_t, C.POINTER(gtmp_edge_opts), _vp]
_lib.gtmp_simplify_paths.argtypes = [C.POINTER(gtmp_robot), C.POINTER(gtmp_scene), C.c_int32, C.c_int32, C.c_int32,
                                     C.c_int32] + [_vp] * 7
_lib.gtmp_minplus_sweep.argtypes = [C.c_int32, C.c_int32, C.c_int32, _vp, _vp, _vp, _vp, _vp, _vp, _vp, _vp, _vp]
_lib.gtmp_extract_path.argtypes = [C.c_int32, C.c_int32, C.c_int32, C.c_int32, _vp, _vp, _vp, _vp, _vp, _vp, _vp,
                                   _vp, _vp, _vp]

class gtmp_anytime_opts(C.Structure):
    _fields_ = [("mode", C.c_int32), ("max_stages", C.c_int32), ("M_min", C.c_int32), ("M_max", C.c_int32),
                ("N_min", C.c_int32), ("N_max", C.c_int32), ("use_graph", C.c_int32), ("bias_tau", C.c_float),
                ("bias_net", C.c_void_p), ("simplify", C.c_int32), ("lp", C.c_void_p)]


GTMP_ANYTIME_RESTART, GTMP_ANYTIME_GROWING = 0, 1


class gtmp_plan_desc(C.Structure):
    _fields_ = [("problem", gtmp_problem), ("robot", gtmp_robot), ("scene", gtmp_scene), ("q0", C.c_void_p),
                ("goals", C.c_void_p), ("seed", C.c_uint64), ("mode", C.c_int32), ("stages", C.c_int32),
                ("M_min", C.c_int32), ("N_min", C.c_int32)]


class gtmp_batch_opts(C.Structure):
    _fields_ = [("use_graph", C.c_int32), ("states_per_iter", C.c_int32), ("sphere_chunks", C.c_int32),
                ("blocks_per_cu", C.c_int32), ("stats", C.c_void_p)]


_lib.gtmp_batch_workspace_size.argtypes = [C.POINTER(gtmp_plan_desc), C.c_int32, C.POINTER(gtmp_batch_opts),
                                           C.POINTER(C.c_size_t)]
_lib.gtmp_plan_batch.argtypes = [C.POINTER(gtmp_plan_desc), C.c_int32, C.POINTER(gtmp_batch_opts), _vp, _vp, _vp,
                                 _vp, _vp, C.c_int32, _vp, C.c_size_t, _vp]

_lib.gtmp_expand_workspace_size.argtypes = [C.POINTER(gtmp_problem), C.POINTER(C.c_size_t)]
_lib.gtmp_expand_samples.argtypes = [C.POINTER(gtmp_problem), _vp, _vp, _vp, C.c_int32, _vp, _vp, C.c_uint64,
                                     C.c_uint64, _vp, C.c_size_t, _vp]
_lib.gtmp_expand_biased_workspace_size.argtypes = [C.POINTER(gtmp_problem), C.POINTER(C.c_size_t)]
_lib.gtmp_expand_samples_biased.argtypes = [C.POINTER(gtmp_problem), _vp, _vp, _vp, C.c_int32, _vp, _vp, C.c_uint64,
                                            C.c_uint64, _vp, C.c_float, _vp, C.c_size_t, _vp]
_lib.gtmp_sample_informed.argtypes = [C.POINTER(gtmp_problem), _vp, _vp, _vp, C.c_uint64, C.c_uint64, C.c_int32,
                                      C.c_int32, _vp, _vp, _vp, _vp]
_lib.gtmp_anytime_workspace_size.argtypes = [C.POINTER(gtmp_problem), C.POINTER(gtmp_anytime_opts),
                                             C.POINTER(C.c_size_t)]
_lib.gtmp_plan_anytime.argtypes = [C.POINTER(gtmp_problem), C.POINTER(gtmp_robot), C.POINTER(gtmp_scene), _vp, _vp,
                                   C.c_uint64, C.POINTER(gtmp_anytime_opts), _vp, _vp, _vp, _vp, _vp, _vp, C.c_size_t,
                                   C.POINTER(gtmp_edge_opts), _vp]

class gtmp_surrogate(C.Structure):
    _fields_ = [("d", C.c_int32), ("fourier", C.c_void_p), ("params", C.c_void_p), ("params_bf16", C.c_void_p)]


_lib.gtmp_surrogate_layout.argtypes = [C.POINTER(C.c_int32)]
_lib.gtmp_surrogate_refresh_bf16.argtypes = [C.POINTER(gtmp_surrogate), _vp]
_lib.gtmp_surrogate_workspace_size.argtypes = [C.c_int64, C.POINTER(C.c_size_t)]
_lib.gtmp_surrogate_infer.argtypes = [C.POINTER(gtmp_surrogate), C.c_int64, _vp, _vp, _vp, C.c_size_t, _vp]
_lib.gtmp_surrogate_grad.argtypes = [C.POINTER(gtmp_surrogate), C.c_int32, _vp, _vp, _vp, _vp, _vp, _vp, C.c_size_t,
                                     _vp]
_lib.gtmp_surrogate_adam.argtypes = [C.POINTER(gtmp_surrogate), _vp, _vp, _vp, C.c_int32, C.c_float, C.c_float,
                                     C.c_float, C.c_float, _vp]
_lib.gtmp_surrogate_label_states.argtypes = [C.POINTER(gtmp_problem), C.c_uint64, C.c_uint64, C.c_int64, _vp, _vp]
_lib.gtmp_surrogate_prune_workspace_size.argtypes = [C.POINTER(gtmp_problem), C.POINTER(C.c_size_t)]
_lib.gtmp_surrogate_prune.argtypes = [C.POINTER(gtmp_problem), C.POINTER(gtmp_surrogate), _vp, _vp, _vp, _vp,
                                      C.c_float, _vp, _vp, _vp, C.c_size_t, _vp]
_lib.gtmp_surrogate_threshold_workspace_size.argtypes = [C.POINTER(C.c_size_t)]
_lib.gtmp_surrogate_threshold.argtypes = [_vp, _vp, C.c_int64, C.c_double, _vp, _vp, C.c_size_t, _vp]

_lib.gtmp_class_sweep_workspace_size.argtypes = [C.c_int32, C.c_int32, C.c_int32, C.POINTER(C.c_size_t)]
_lib.gtmp_class_sweep.argtypes = [C.c_int32] * 4 + [_vp] * 6 + [C.c_float, _vp, C.c_int32] + [_vp] * 5 + \
    [_vp, C.c_size_t, _vp]
_lib.gtmp_class_anytime_workspace_size.argtypes = [C.POINTER(gtmp_problem), C.c_int32, C.POINTER(C.c_size_t)]
_lib.gtmp_plan_classes.argtypes = [C.POINTER(gtmp_problem), C.POINTER(gtmp_scene), _vp, _vp, C.c_uint64, C.c_int32,
                                   _vp, C.c_int32, C.c_int32, C.c_int32] + [_vp] * 7 + [C.c_size_t, _vp, _vp]

EXPORTS = ["gtmp_status_string", "gtmp_last_error", "gtmp_version", "gtmp_sample_layers",
           "gtmp_edge_check_workspace_size", "gtmp_edge_check_cost", "gtmp_edge_check_cost_noalloc",
           "gtmp_state_check", "gtmp_minplus_sweep",
           "gtmp_extract_path", "gtmp_expand_workspace_size", "gtmp_expand_samples", "gtmp_sample_informed",
           "gtmp_anytime_workspace_size", "gtmp_plan_anytime", "gtmp_batch_workspace_size", "gtmp_plan_batch",
           "gtmp_surrogate_layout", "gtmp_surrogate_refresh_bf16", "gtmp_surrogate_workspace_size",
           "gtmp_surrogate_infer", "gtmp_surrogate_grad", "gtmp_surrogate_adam", "gtmp_surrogate_label_states",
           "gtmp_surrogate_prune_workspace_size", "gtmp_surrogate_prune", "gtmp_surrogate_threshold_workspace_size", "gtmp_surrogate_threshold",
           "gtmp_expand_biased_workspace_size", "gtmp_expand_samples_biased",
           "gtmp_class_sweep_workspace_size", "gtmp_class_sweep", "gtmp_class_anytime_workspace_size",
           "gtmp_plan_classes", "gtmp_simplify_paths", "gtmp_rrtc_workspace_size", "gtmp_rrtc_repair",
           "gtmp_rrtc_local_path", "gtmp_lazy_workspace_size", "gtmp_plan_lazy"]


def _check(st):
    if st < 0:
        raise GtmpError(st, _lib.gtmp_last_error().decode())
    return st


def _p(t):
    """Device pointer of a tensor (None -> NULL)."""
    if t is None:
        return None
    if not t.is_cuda:
        raise ValueError("expected a device tensor")
    if not t.is_contiguous():
        raise ValueError("expected a contiguous tensor")
    return t.data_ptr()


def _stream(stream):
    if stream is None:
        return torch.cuda.current_stream().cuda_stream
    return stream.cuda_stream if hasattr(stream, "cuda_stream") else stream


def model_of(w, device="cuda"):
    """(robot, scene) of a workload dict: a point robot in the plane
    (kind point2d), a point robot in space (kind point) or a DH arm."""
    if w["kind"] == "point2d":
        return make_point_robot(), Scene(2, w["circles"], w["boxes"], device)
    if w["kind"] == "point":
        return make_point_robot(), Scene(3, w["obs_spheres"], w["obs_boxes"], device)
    return make_arm_robot(w["dh"], w["sph_link"], w["sph_t"], w["sph_r"]), \
        Scene(3, w["obs_spheres"], w["obs_boxes"], device)


def version() -> str:
    return _lib.gtmp_version().decode()


# --------------------------------------------------------------------------- #
# struct builders
# --------------------------------------------------------------------------- #
def make_problem(d, M, N, G, H, lo, hi, penalty=1e3, max_edge_len=math.inf) -> gtmp_problem:
    p = gtmp_problem()
    p.d, p.M, p.N, p.G, p.H = int(d), int(M), int(N), int(G), int(H)
    for j in range(min(int(d), GTMP_MAX_DOF)):
        p.lo[j] = float(lo[j])
        p.hi[j] = float(hi[j])
    p.penalty = float(penalty)
    p.max_edge_len = float(max_edge_len)
    return p


def make_point_robot() -> gtmp_robot:
    r = gtmp_robot()
    r.kind = GTMP_ROBOT_POINT
    return r


def make_arm_robot(dh, sph_link, sph_t, sph_r) -> gtmp_robot:
    r = gtmp_robot()
    r.kind = GTMP_ROBOT_DH_ARM
    dh = np.asarray(dh, np.float32)
    r.n_joints = dh.shape[0]
    r.n_spheres = len(sph_link)
    for i in range(dh.shape[0]):
        for c in range(4):
            r.dh[i][c] = float(dh[i, c])
    for k in range(len(sph_link)):
        r.sph_link[k] = int(sph_link[k])
        r.sph_t[k] = float(sph_t[k])
        r.sph_r[k] = float(sph_r[k])
    return r


class Scene:
    """Obstacles resident on the device (keeps the tensors alive)."""

    def __init__(self, wdim, spheres, boxes, device="cuda"):
        self.wdim = int(wdim)
        sp = np.ascontiguousarray(spheres, np.float32).reshape(-1, self.wdim + 1)
        bx = np.ascontiguousarray(boxes, np.float32).reshape(-1, 2 * self.wdim)
        # one extra element keeps a valid pointer for empty sets
        self.spheres = torch.from_numpy(np.concatenate([sp.ravel(), np.zeros(4, np.float32)])).to(device)
        self.boxes = torch.from_numpy(np.concatenate([bx.ravel(), np.zeros(4, np.float32)])).to(device)
        self.c = gtmp_scene()
        self.c.wdim = self.wdim
        self.c.n_spheres = sp.shape[0]
        self.c.spheres = self.spheres.data_ptr()
        self.c.n_boxes = bx.shape[0]
        self.c.boxes = self.boxes.data_ptr()


# --------------------------------------------------------------------------- #
# entry points (same names as the C ABI)
# --------------------------------------------------------------------------- #
def gtmp_sample_layers(prob: gtmp_problem, seed: int, stage: int, Q: torch.Tensor, stream=None):
    return _check(_lib.gtmp_sample_layers(C.byref(prob), seed, stage, _p(Q), _stream(stream)))


def gtmp_edge_check_workspace_size(prob: gtmp_problem) -> int:
    n = C.c_size_t()
    _check(_lib.gtmp_edge_check_workspace_size(C.byref(prob), C.byref(n)))
    return n.value


def gtmp_edge_check_cost(prob, robot, scene: Scene, q0, goals, Q, C_s, C_h, C_l, workspace, minsd=None, flags=None,
                         prune=None, opts: gtmp_edge_opts | None = None, stream=None):
    return _check(_lib.gtmp_edge_check_cost(
        C.byref(prob), C.byref(robot), C.byref(scene.c), _p(q0), _p(goals), _p(Q), _p(C_s), _p(C_h), _p(C_l),
        _p(minsd), _p(flags), _p(prune), _p(workspace), workspace.numel() * workspace.element_size(),
        C.byref(opts) if opts is not None else None, _stream(stream)))


def gtmp_edge_check_cost_noalloc(prob, robot, scene: Scene, q0, goals, Q, C_s, C_h, C_l, minsd=None, flags=None,
                                 prune=None, opts: gtmp_edge_opts | None = None, stream=None):
    return _check(_lib.gtmp_edge_check_cost_noalloc(
        C.byref(prob), C.byref(robot), C.byref(scene.c), _p(q0), _p(goals), _p(Q), _p(C_s), _p(C_h), _p(C_l),
        _p(minsd), _p(flags), _p(prune), C.byref(opts) if opts is not None else None, _stream(stream)))


def gtmp_state_check(robot, scene: Scene, d, X, sd=None, coll=None, stream=None):
    n = X.shape[0] if X is not None else 0
    return _check(_lib.gtmp_state_check(C.byref(robot), C.byref(scene.c), int(d), int(n), _p(X), _p(sd), _p(coll),
                                        _stream(stream)))


def make_rrtc_opts(budget, tree_cap, step, resolution, ell_factor, stats=None) -> gtmp_rrtc_opts:
    o = gtmp_rrtc_opts()
    o.budget, o.tree_cap, o.step, o.resolution, o.ell_factor = int(budget), int(tree_cap), step, resolution, ell_factor
    if stats is not None:
        o.stats = stats.data_ptr()
    return o


def gtmp_rrtc_workspace_size(prob) -> int:
    n = C.c_size_t()
    _check(_lib.gtmp_rrtc_workspace_size(C.byref(prob), C.byref(n)))
    return n.value


def gtmp_rrtc_repair(prob, robot, scene: Scene, q0, goals, Q, C_s, C_h, C_l, flags, seed, stage, opts, workspace,
                     stream=None):
    return _check(_lib.gtmp_rrtc_repair(C.byref(prob), C.byref(robot), C.byref(scene.c), _p(q0), _p(goals), _p(Q),
                                        _p(C_s), _p(C_h), _p(C_l), _p(flags), seed, stage, C.byref(opts),
                                        _p(workspace), workspace.numel() * workspace.element_size(), _stream(stream)))


def gtmp_rrtc_local_path(prob, robot, scene: Scene, q0, goals, Q, edge, seed, stage, opts, path, count, cost,
                         stream=None):
    return _check(_lib.gtmp_rrtc_local_path(C.byref(prob), C.byref(robot), C.byref(scene.c), _p(q0), _p(goals),
                                            _p(Q), int(edge), seed, stage, C.byref(opts), _p(path), _p(count),
                                            _p(cost), _stream(stream)))


def gtmp_lazy_workspace_size(prob) -> int:
    n = C.c_size_t()
    _check(_lib.gtmp_lazy_workspace_size(C.byref(prob), C.byref(n)))
    return n.value


def gtmp_plan_lazy(prob, robot, scene: Scene, q0, goals, Q, C_s, C_h, C_l, flags, V, A, V_s, a_s, idx, wp, cost,
                   band, max_rounds, workspace, stats=None, edge_opts=None, stream=None):
    """Returns (status, rounds): status GTMP_OK, or GTMP_INCOMPLETE at the round limit."""
    r = C.c_int32(0)
    st = _check(_lib.gtmp_plan_lazy(C.byref(prob), C.byref(robot), C.byref(scene.c), _p(q0), _p(goals), _p(Q),
                                    _p(C_s), _p(C_h), _p(C_l), _p(flags), _p(V), _p(A), _p(V_s), _p(a_s), _p(idx),
                                    _p(wp), _p(cost), float(band), int(max_rounds), _p(stats), C.byref(r),
                                    _p(workspace), workspace.numel() * workspace.element_size(),
                                    C.byref(edge_opts) if edge_opts is not None else None, _stream(stream)))
    return st, r.value


def gtmp_simplify_paths(robot, scene: Scene, d, H, wp, valid, idx, count, cost, out_wp=None, stream=None):
    B, K = (int(wp.shape[0]), int(wp.shape[1])) if wp is not None else (0, 2)
    return _check(_lib.gtmp_simplify_paths(C.byref(robot), C.byref(scene.c), int(d), B, K, int(H), _p(wp), _p(valid),
                                           _p(idx), _p(count), _p(cost), _p(out_wp), _stream(stream)))


def simplify_paths(robot, scene: Scene, d, H, wp, stream=None):
    """Shortcut B paths (wp [B][K][d] on the device).  Returns a dict of
    device tensors: valid [B][K][K], idx [B][K], count [B], cost [B], wp [B][K][d]."""
    wp = wp.contiguous()
    B, K = wp.shape[0], wp.shape[1]
    dev = wp.device
    out = dict(valid=torch.empty((B, K, K), device=dev, dtype=torch.uint8),
               idx=torch.empty((B, K), device=dev, dtype=torch.int32),
               count=torch.empty((B,), device=dev, dtype=torch.int32),
               cost=torch.empty((B,), device=dev, dtype=torch.float32),
               wp=torch.empty((B, K, d), device=dev, dtype=torch.float32))
    gtmp_simplify_paths(robot, scene, d, H, wp, out["valid"], out["idx"], out["count"], out["cost"], out["wp"], stream)
    return out


def gtmp_minplus_sweep(M, N, G, C_s, C_h, C_l, V, A, V_s, a_s, Vg=None, stream=None):
    return _check(_lib.gtmp_minplus_sweep(int(M), int(N), int(G), _p(C_s), _p(C_h), _p(C_l), _p(Vg), _p(V), _p(A),
                                          _p(V_s), _p(a_s), _stream(stream)))


def gtmp_extract_path(M, N, G, d, a_s, A, V_s, Q, q0, goals, idx, wp, cost, stream=None):
    return _check(_lib.gtmp_extract_path(int(M), int(N), int(G), int(d), _p(a_s), _p(A), _p(V_s), _p(Q), _p(q0),
                                         _p(goals), _p(idx), _p(wp), _p(cost), _stream(stream)))


def _aligned_workspace(nbytes, device="cuda"):
    buf = torch.empty((nbytes + 256,), device=device, dtype=torch.uint8)
    off = (-buf.data_ptr()) % 256
    return buf[off:off + nbytes]


def gtmp_expand_workspace_size(prob) -> int:
    n = C.c_size_t()
    _check(_lib.gtmp_expand_workspace_size(C.byref(prob), C.byref(n)))
    return n.value


def gtmp_expand_samples(prob, q0, goals, Q_old, n_old, Q_new, c_best, seed, stage, workspace, stream=None):
    return _check(_lib.gtmp_expand_samples(C.byref(prob), _p(q0), _p(goals), _p(Q_old), int(n_old), _p(Q_new),
                                           _p(c_best), seed, stage, _p(workspace),
                                           workspace.numel() * workspace.element_size(), _stream(stream)))


def gtmp_sample_informed(prob, q0, goals, c_best, seed, stage, m, X, attempts=None, workspace=None, stream=None):
    if workspace is None:
        workspace = _aligned_workspace(1024)
    count = X.shape[0]
    return _check(_lib.gtmp_sample_informed(C.byref(prob), _p(q0), _p(goals), _p(c_best), seed, stage, int(m),
                                            int(count), _p(X), _p(attempts), _p(workspace), _stream(stream)))


def gtmp_anytime_workspace_size(prob, opts) -> int:
    n = C.c_size_t()
    _check(_lib.gtmp_anytime_workspace_size(C.byref(prob), C.byref(opts), C.byref(n)))
    return n.value


def gtmp_plan_anytime(prob, robot, scene: Scene, q0, goals, seed, opts, best_cost, best_idx, best_wp, best_meta,
                      stage_costs, workspace, edge_opts=None, stream=None):
    return _check(_lib.gtmp_plan_anytime(
        C.byref(prob), C.byref(robot), C.byref(scene.c), _p(q0), _p(goals), seed, C.byref(opts), _p(best_cost),
        _p(best_idx), _p(best_wp), _p(best_meta), _p(stage_costs), _p(workspace),
        workspace.numel() * workspace.element_size(), C.byref(edge_opts) if edge_opts is not None else None,
        _stream(stream)))


# --------------------------------------------------------------------------- #
# one plan
# --------------------------------------------------------------------------- #
@dataclass
class PlanResult:
    Q: torch.Tensor
    C_s: torch.Tensor
    C_h: torch.Tensor
    C_l: torch.Tensor
    V: torch.Tensor
    A: torch.Tensor
    V_s: torch.Tensor
    a_s: torch.Tensor
    idx: torch.Tensor
    wp: torch.Tensor
    cost: torch.Tensor
    flags: torch.Tensor | None = None
    minsd: torch.Tensor | None = None


class Planner:
    """Device buffers and structs for repeated plans on one workload.

    ``w`` is a workload dict (see ``workloads.make_workload``): sizes, box,
    penalty, start/goals and either 2D obstacles or an arm model with 3D
    obstacles."""

    def __init__(self, w, device="cuda", flags=False, minsd=False, max_edge_len=math.inf):
        self.w = w
        d, M, N, G, H = (int(w[k]) for k in ("d", "M", "N", "G", "H"))
        self.d, self.M, self.N, self.G, self.H = d, M, N, G, H
        self.prob = make_problem(d, M, N, G, H, w["lo"], w["hi"], w["penalty"], max_edge_len)
        self.robot, self.scene = model_of(w, device)
        f32 = dict(device=device, dtype=torch.float32)
        self.q0 = torch.from_numpy(np.asarray(w["q0"], np.float32)).to(device)
        self.goals = torch.from_numpy(np.asarray(w["goals"], np.float32).reshape(G, d)).to(device)
        self.Q = torch.empty((M, N, d), **f32)
        self.C_s = torch.empty((N,), **f32)
        self.C_h = torch.empty((max(M - 1, 1), N, N), **f32)
        self.C_l = torch.empty((N, G), **f32)
        self.V = torch.empty((M, N), **f32)
        self.A = torch.empty((M, N), device=device, dtype=torch.int32)
        self.V_s = torch.empty((1,), **f32)
        self.a_s = torch.empty((1,), device=device, dtype=torch.int32)
        self.idx = torch.empty((M + 1,), device=device, dtype=torch.int32)
        self.wp = torch.empty((M + 2, d), **f32)
        self.cost = torch.empty((1,), **f32)
        E = N + (M - 1) * N * N + N * G
        self.E = E
        self.flags = torch.empty((E,), device=device, dtype=torch.uint8) if flags else None
        self.minsd = torch.empty((E,), **f32) if minsd else None
        self.workspace = _aligned_workspace(gtmp_edge_check_workspace_size(self.prob), device)
        self.stats = torch.zeros((4,), device=device, dtype=torch.int64)
        self.opts = gtmp_edge_opts()
        self.opts.stats = self.stats.data_ptr()

    def sample(self, seed, stage=0, stream=None):
        gtmp_sample_layers(self.prob, seed, stage, self.Q, stream)

    def check(self, stream=None, prune=None):
        gtmp_edge_check_cost(self.prob, self.robot, self.scene, self.q0, self.goals, self.Q, self.C_s,
                             self.C_h if self.M > 1 else None, self.C_l, self.workspace, self.minsd, self.flags,
                             prune, self.opts, stream)

    def sweep(self, stream=None):
        gtmp_minplus_sweep(self.M, self.N, self.G, self.C_s, self.C_h if self.M > 1 else None, self.C_l, self.V,
                           self.A, self.V_s, self.a_s, None, stream)

    def extract(self, stream=None):
        gtmp_extract_path(self.M, self.N, self.G, self.d, self.a_s, self.A, self.V_s, self.Q, self.q0, self.goals,
                          self.idx, self.wp, self.cost, stream)

    def plan(self, seed, stage=0, Q=None, stream=None):
        """One whole plan; with ``Q`` given the samples are copied in instead
        of drawn (warm-start samples, Alg. 1 optional input)."""
        if Q is None:
            self.sample(seed, stage, stream)
        else:
            self.Q.copy_(Q)
        self.check(stream)
        self.sweep(stream)
        self.extract(stream)
        return self.result()

    def repair(self, opts, seed, stage=0, stream=None):
        """RRT-Connect on the edges whose straight line failed (needs flags)."""
        if self.flags is None:
            raise ValueError("repair needs a Planner built with flags=True")
        if getattr(self, "rrtc_ws", None) is None:
            self.rrtc_ws = _aligned_workspace(gtmp_rrtc_workspace_size(self.prob), self.Q.device)
        gtmp_rrtc_repair(self.prob, self.robot, self.scene, self.q0, self.goals, self.Q, self.C_s,
                         self.C_h if self.M > 1 else None, self.C_l, self.flags, seed, stage, opts, self.rrtc_ws, stream)

    def local_path(self, edge, opts, seed, stage=0, stream=None):
        """The RRT-Connect path of one edge: (waypoints [n][d] device tensor, cost)."""
        path = torch.empty((2 * opts.tree_cap, self.d), device=self.Q.device)
        count = torch.empty((1,), device=self.Q.device, dtype=torch.int32)
        cost = torch.empty((1,), device=self.Q.device)
        gtmp_rrtc_local_path(self.prob, self.robot, self.scene, self.q0, self.goals, self.Q, edge, seed, stage, opts,
                             path, count, cost, stream)
        n = int(count.item())
        return path[:n], float(cost.item())

    def plan_lazy(self, seed, stage=0, band=0.0, max_rounds=1000, stats=None, stream=None):
        """Sample, then the lazy plan (needs flags): (status, rounds)."""
        if self.flags is None:
            raise ValueError("plan_lazy needs a Planner built with flags=True")
        if getattr(self, "lazy_ws", None) is None:
            self.lazy_ws = _aligned_workspace(gtmp_lazy_workspace_size(self.prob), self.Q.device)
        self.sample(seed, stage, stream)
        return gtmp_plan_lazy(self.prob, self.robot, self.scene, self.q0, self.goals, self.Q, self.C_s,
                              self.C_h if self.M > 1 else None, self.C_l, self.flags, self.V, self.A, self.V_s,
                              self.a_s, self.idx, self.wp, self.cost, band, max_rounds, self.lazy_ws, stats,
                              self.opts, stream)

    def simplify(self, wp=None, stream=None):
        """Shortcut the extracted path (or the paths wp [B][M+2][d])."""
        wp = self.wp.unsqueeze(0) if wp is None else wp
        return simplify_paths(self.robot, self.scene, self.d, self.H, wp, stream)

    def result(self) -> PlanResult:
        return PlanResult(self.Q, self.C_s, self.C_h, self.C_l, self.V, self.A, self.V_s, self.a_s, self.idx, self.wp,
                          self.cost, self.flags, self.minsd)


class AnytimePlanner:
    """Device buffers for the anytime policies on one workload (restart:
    the workload's M, N; growing: the schedule's maxima)."""

    def __init__(self, w, mode, max_stages, M_min=None, M_max=None, N_min=None, N_max=None, use_graph=False,
                 device="cuda", bias=None, bias_tau=0.0, simplify=False, lp=None):
        self.w = w
        d, M, N, G, H = (int(w[k]) for k in ("d", "M", "N", "G", "H"))
        self.d = d
        self.opts = gtmp_anytime_opts()
        self.opts.mode = mode
        self.opts.max_stages = max_stages
        self.opts.M_min, self.opts.M_max = M_min or M, M_max or M
        self.opts.N_min, self.opts.N_max = N_min or N, N_max or N
        self.opts.use_graph = int(use_graph)
        self.opts.simplify = int(simplify)
        self.lp = lp  # a gtmp_rrtc_opts (kept alive for the struct's pointer)
        if lp is not None:
            self.opts.lp = C.cast(C.pointer(lp), C.c_void_p).value
        self.bias = bias  # a Surrogate (kept alive for the struct's pointer)
        if bias is not None:
            self.opts.bias_net = C.cast(C.pointer(bias.c), C.c_void_p).value
            self.opts.bias_tau = float(bias_tau)
        self.prob = make_problem(d, M, N, G, H, w["lo"], w["hi"], w["penalty"])
        self.robot, self.scene = model_of(w, device)
        self.q0 = torch.from_numpy(np.asarray(w["q0"], np.float32)).to(device)
        self.goals = torch.from_numpy(np.asarray(w["goals"], np.float32).reshape(G, d)).to(device)
        Mx = self.opts.M_max if mode == GTMP_ANYTIME_GROWING else M
        self.best_cost = torch.empty((1,), device=device)
        self.best_idx = torch.empty((Mx + 1,), device=device, dtype=torch.int32)
        self.best_wp = torch.empty((Mx + 2, d), device=device)
        self.best_meta = torch.empty((4,), device=device, dtype=torch.int32)
        self.stage_costs = torch.full((max_stages,), float("nan"), device=device)
        self.workspace = _aligned_workspace(gtmp_anytime_workspace_size(self.prob, self.opts), device)
        self.edge_opts = gtmp_edge_opts()

    def run(self, seed, stream=None):
        gtmp_plan_anytime(self.prob, self.robot, self.scene, self.q0, self.goals, seed, self.opts, self.best_cost,
                          self.best_idx, self.best_wp, self.best_meta, self.stage_costs, self.workspace,
                          self.edge_opts, stream)


def gtmp_batch_workspace_size(descs, opts) -> int:
    n = C.c_size_t()
    _check(_lib.gtmp_batch_workspace_size(descs, len(descs), C.byref(opts), C.byref(n)))
    return n.value


def gtmp_plan_batch(descs, opts, best_cost, best_idx, best_wp, best_meta, stage_costs, stage_stride, workspace,
                    stream=None):
    return _check(_lib.gtmp_plan_batch(descs, len(descs), C.byref(opts), _p(best_cost), _p(best_idx), _p(best_wp),
                                       _p(best_meta), _p(stage_costs), int(stage_stride), _p(workspace),
                                       workspace.numel() * workspace.element_size(), _stream(stream)))


_MODES = {"plain": GTMP_ANYTIME_RESTART, "restart": GTMP_ANYTIME_RESTART, "growing": GTMP_ANYTIME_GROWING}


def spec_mode(sp) -> int:
    m = sp.get("mode", GTMP_ANYTIME_RESTART)
    return _MODES[m] if isinstance(m, str) else int(m)


def single_planner(sp, device="cuda", use_graph=False) -> "AnytimePlanner":
    """The single-plan equivalent of one batch entry (same policy and sizes)."""
    w = sp["w"]
    if spec_mode(sp) == GTMP_ANYTIME_GROWING:
        return AnytimePlanner(w, GTMP_ANYTIME_GROWING, int(sp["stages"]), M_min=int(sp["M_min"]),
                              N_min=int(sp["N_min"]), use_graph=use_graph, device=device)
    return AnytimePlanner(w, GTMP_ANYTIME_RESTART, int(sp.get("stages", 1)), use_graph=use_graph, device=device)


class BatchPlanner:
    """A batch of independent plans.  ``specs`` is a list of dicts with keys
    ``w`` (workload dict), ``mode`` (GTMP_ANYTIME_RESTART / GROWING, or one of
    "plain", "restart", "growing"), ``stages``, optionally ``seed`` (default:
    the workload's) and, for growing plans, ``M_min`` / ``N_min`` (the
    workload's M, N are the maxima)."""

    def __init__(self, specs, use_graph=False, device="cuda", opts=None):
        self.specs = specs
        n = len(specs)
        self.descs = (gtmp_plan_desc * n)()
        self.keep = []
        idx_off, wp_off = [], []
        io = wo = 0
        for i, sp in enumerate(specs):
            w = sp["w"]
            d, M, N, G, H = (int(w[k]) for k in ("d", "M", "N", "G", "H"))
            D = self.descs[i]
            D.problem = make_problem(d, M, N, G, H, w["lo"], w["hi"], w["penalty"])
            D.robot, scene = model_of(w, device)
            q0 = torch.from_numpy(np.asarray(w["q0"], np.float32)).to(device)
            goals = torch.from_numpy(np.asarray(w["goals"], np.float32).reshape(G, d)).to(device)
            self.keep += [scene, q0, goals]
            D.scene = scene.c
            D.q0, D.goals = q0.data_ptr(), goals.data_ptr()
            D.seed = int(sp.get("seed", w["seed"]))
            D.mode = spec_mode(sp)
            D.stages = int(sp.get("stages", 1))
            D.M_min = int(sp.get("M_min", M))
            D.N_min = int(sp.get("N_min", N))
            idx_off.append(io)
            wp_off.append(wo)
            io += M + 1
            wo += (M + 2) * d
        self.idx_off, self.wp_off = idx_off, wp_off
        self.opts = gtmp_batch_opts()
        self.opts.use_graph = int(use_graph)
        if opts:
            for k in ("states_per_iter", "sphere_chunks", "blocks_per_cu"):
                if k in opts:
                    setattr(self.opts, k, int(opts[k]))
        self.stats = torch.zeros((4,), device=device, dtype=torch.int64)
        self.opts.stats = self.stats.data_ptr()
        self.stage_stride = max(int(sp.get("stages", 1)) for sp in specs)
        self.best_cost = torch.empty((n,), device=device)
        self.best_idx = torch.empty((io,), device=device, dtype=torch.int32)
        self.best_wp = torch.empty((wo,), device=device)
        self.best_meta = torch.empty((n, 4), device=device, dtype=torch.int32)
        self.stage_costs = torch.full((n, self.stage_stride), float("nan"), device=device)
        self.workspace = _aligned_workspace(gtmp_batch_workspace_size(self.descs, self.opts), device)

    def run(self, stream=None):
        gtmp_plan_batch(self.descs, self.opts, self.best_cost, self.best_idx, self.best_wp, self.best_meta,
                        self.stage_costs, self.stage_stride, self.workspace, stream)

    def plan_idx(self, i):
        M = self.descs[i].problem.M
        return self.best_idx[self.idx_off[i]:self.idx_off[i] + M + 1]


# --------------------------------------------------------------------------- #
# learned collision surrogate
# --------------------------------------------------------------------------- #
SUR_NAMES = ("W1", "b1", "W2", "b2", "W3", "b3", "W4", "b4", "w5", "b5")


def gtmp_surrogate_layout():
    off = (C.c_int32 * 11)()
    _check(_lib.gtmp_surrogate_layout(off))
    return list(off)


def gtmp_surrogate_workspace_size(n) -> int:
    b = C.c_size_t()
    _check(_lib.gtmp_surrogate_workspace_size(int(n), C.byref(b)))
    return b.value


def _nbytes(t):
    return t.numel() * t.element_size()


class Surrogate:
    """Device parameters, Adam moments and workspace of the collision
    surrogate.  ``P`` maps W1, b1, ..., w5, b5 to arrays (float32) and ``Bf``
    is the Fourier matrix [16][d]."""

    def __init__(self, P, Bf, batch=8192, device="cuda"):
        self.d = int(np.asarray(Bf).shape[1])
        self.offsets = gtmp_surrogate_layout()
        self.total = self.offsets[10]
        flat = np.zeros(self.total, np.float32)
        for i, k in enumerate(SUR_NAMES):
            a = np.asarray(P[k], np.float32).reshape(-1)
            end = self.offsets[i + 1] if i + 1 < 10 else self.total
            assert a.size == end - self.offsets[i], k
            flat[self.offsets[i]:end] = a
        self.params = torch.from_numpy(flat).to(device)
        self.params_bf16 = torch.zeros(self.total, device=device, dtype=torch.int16)
        self.fourier = torch.from_numpy(np.asarray(Bf, np.float32).copy()).to(device)
        self.c = gtmp_surrogate(self.d, self.fourier.data_ptr(), self.params.data_ptr(), self.params_bf16.data_ptr())
        self.m = torch.zeros_like(self.params)
        self.v = torch.zeros_like(self.params)
        self.grad_buf = torch.zeros_like(self.params)
        self.loss_buf = torch.zeros(1, device=device)
        self.t = 0
        self.batch = int(batch)
        self.workspace = _aligned_workspace(gtmp_surrogate_workspace_size(self.batch), device)
        _check(_lib.gtmp_surrogate_refresh_bf16(C.byref(self.c), _stream(None)))

    def to_dict(self):
        flat = self.params.cpu().numpy()
        out = {}
        for i, k in enumerate(SUR_NAMES):
            end = self.offsets[i + 1] if i + 1 < 10 else self.total
            out[k] = flat[self.offsets[i]:end].copy()
        shapes = {"W1": (256, 64), "W2": (256, 256), "W3": (256, 256), "W4": (256, 256)}
        for k, sh in shapes.items():
            out[k] = out[k].reshape(sh)
        return out

    def infer(self, X, logits=None, stream=None):
        n = X.shape[0]
        if logits is None:
            logits = torch.empty(n, device=X.device)
        _check(_lib.gtmp_surrogate_infer(C.byref(self.c), n, _p(X), _p(logits), _p(self.workspace),
                                         _nbytes(self.workspace), _stream(stream)))
        return logits

    def grad(self, X, y, logits=None, stream=None):
        """Loss and gradient of one batch (rows a multiple of 256): fills
        ``grad_buf`` and ``loss_buf``."""
        n = X.shape[0]
        _check(_lib.gtmp_surrogate_grad(C.byref(self.c), n, _p(X), _p(y), _p(self.grad_buf), _p(self.loss_buf),
                                        _p(logits), _p(self.workspace), _nbytes(self.workspace), _stream(stream)))
        return self.loss_buf

    def adam(self, grad=None, lr=1e-3, b1=0.9, b2=0.999, eps=1e-8, stream=None):
        self.t += 1
        g = self.grad_buf if grad is None else grad
        _check(_lib.gtmp_surrogate_adam(C.byref(self.c), _p(g), _p(self.m), _p(self.v), self.t, lr, b1, b2, eps,
                                        _stream(stream)))

    def train(self, X, y, epochs=1, lr=1e-3, seed=0, stream=None):
        """Mini-batch Adam over (X, y) for some epochs; batches of
        ``self.batch`` rows in a seeded order (the tail that does not fill a
        batch is left out of that epoch).  Returns the per-step losses (device)."""
        n = X.shape[0]
        steps = n // self.batch
        g = torch.Generator(device="cpu")
        g.manual_seed(seed)
        losses = torch.empty(epochs * steps, device=X.device)
        for ep in range(epochs):
            perm = torch.randperm(n, generator=g).to(X.device)
            Xs, ys = X[perm].contiguous(), y[perm].contiguous()
            for s in range(steps):
                lo = s * self.batch
                self.grad(Xs[lo:lo + self.batch], ys[lo:lo + self.batch], stream=stream)
                self.adam(lr=lr, stream=stream)
                losses[ep * steps + s].copy_(self.loss_buf[0])
        return losses

    def prune(self, prob, q0, goals, Q, tau_logit, prune, logits=None, vcoll=None, stream=None):
        """Prune mask of every edge (and the logits, when given).  ``vcoll``
        (uint8 [M][N], nonzero = colliding sample) restricts inference to the
        edges whose endpoints are free."""
        n = C.c_size_t()
        _check(_lib.gtmp_surrogate_prune_workspace_size(C.byref(prob), C.byref(n)))
        ws = getattr(self, "_prune_ws", None)
        if ws is None or _nbytes(ws) < n.value:
            ws = self._prune_ws = _aligned_workspace(n.value, Q.device)
        _check(_lib.gtmp_surrogate_prune(C.byref(prob), C.byref(self.c), _p(q0), _p(goals), _p(Q), _p(vcoll),
                                         float(tau_logit), _p(prune), _p(logits), _p(ws), _nbytes(ws),
                                         _stream(stream)))


def gtmp_surrogate_label_states(prob, seed, stage, n, X, stream=None):
    _check(_lib.gtmp_surrogate_label_states(C.byref(prob), seed, stage, int(n), _p(X), _stream(stream)))


def make_labels(w, n, seed, stage, device="cuda"):
    """2n training states of workload ``w`` and their exact collision labels
    (uniform half, then interior states of random edges)."""
    d = int(w["d"])
    prob = make_problem(d, 3, max(int(n), 1), 1, int(w["H"]), w["lo"], w["hi"], w["penalty"])
    X = torch.empty((2 * n, d), device=device)
    gtmp_surrogate_label_states(prob, seed, stage, n, X)
    robot, scene = model_of(w, device)
    y = torch.empty(2 * n, device=device, dtype=torch.uint8)
    gtmp_state_check(robot, scene, d, X, None, y)
    return X, y


def gtmp_expand_biased_workspace_size(prob) -> int:
    n = C.c_size_t()
    _check(_lib.gtmp_expand_biased_workspace_size(C.byref(prob), C.byref(n)))
    return n.value


def gtmp_expand_samples_biased(prob, q0, goals, Q_old, n_old, Q_new, c_best, seed, stage, net: "Surrogate", tau_logit,
                               workspace, stream=None):
    return _check(_lib.gtmp_expand_samples_biased(C.byref(prob), _p(q0), _p(goals), _p(Q_old), int(n_old), _p(Q_new),
                                                  _p(c_best), seed, stage, C.byref(net.c), float(tau_logit),
                                                  _p(workspace), _nbytes(workspace), _stream(stream)))


def gtmp_surrogate_threshold(logits, flags, recall, tau, workspace=None, stream=None):
    """tau (device float32 [1]) <- the smallest logit threshold that keeps at
    least ``recall`` of the free edges (flags == 0) unpruned, computed on the
    device (see include/gtmp.h)."""
    if workspace is None:
        n = C.c_size_t()
        _check(_lib.gtmp_surrogate_threshold_workspace_size(C.byref(n)))
        workspace = _aligned_workspace(n.value, logits.device)
    return _check(_lib.gtmp_surrogate_threshold(_p(logits), _p(flags), int(logits.numel()), float(recall), _p(tau),
                                                _p(workspace), _nbytes(workspace), _stream(stream)))


# --------------------------------------------------------------------------- #
# class-augmented sweep and class archive (2D point robots)
# --------------------------------------------------------------------------- #
def unpack_label(words, k):
    """Packed class label (two 64-bit words) -> tuple of k signed crossing
    counts."""
    lab = (int(words[0]) & 0xFFFFFFFFFFFFFFFF) | ((int(words[1]) & 0xFFFFFFFFFFFFFFFF) << 64)
    return tuple(((lab >> (8 * i)) & 255) - 128 for i in range(k))


def gtmp_class_sweep_workspace_size(M, N, L) -> int:
    n = C.c_size_t()
    _check(_lib.gtmp_class_sweep_workspace_size(M, N, L, C.byref(n)))
    return n.value


def class_sweep(pl: "Planner", reps, L=64, stream=None):
    """Class-augmented sweep on a planner's current samples and costs.
    Returns (dict label -> (cost, chain), overflow)."""
    reps_t = torch.from_numpy(np.ascontiguousarray(reps, np.float32).reshape(-1, 2)).to(pl.Q.device)
    k = reps_t.shape[0]
    dev = pl.Q.device
    labels = torch.empty((L, 2), device=dev, dtype=torch.int64)
    costs = torch.empty(L, device=dev)
    chains = torch.empty((L, pl.M + 1), device=dev, dtype=torch.int32)
    count = torch.zeros(1, device=dev, dtype=torch.int32)
    overflow = torch.zeros(1, device=dev, dtype=torch.int32)
    ws = _aligned_workspace(gtmp_class_sweep_workspace_size(pl.M, pl.N, L), dev)
    _check(_lib.gtmp_class_sweep(pl.M, pl.N, pl.G, L, _p(pl.Q), _p(pl.q0), _p(pl.goals), _p(pl.C_s),
                                 _p(pl.C_h) if pl.M > 1 else None, _p(pl.C_l), float(pl.w["penalty"]), _p(reps_t), k,
                                 _p(labels), _p(costs), _p(chains), _p(count), _p(overflow), _p(ws), _nbytes(ws),
                                 _stream(stream)))
    n = int(count.item())
    lab = labels.cpu().numpy()[:n]
    cst = costs.cpu().numpy()[:n]
    ch = chains.cpu().numpy()[:n]
    out = {unpack_label(lab[i], k): (float(cst[i]), [int(x) for x in ch[i]]) for i in range(n)}
    return out, int(overflow.item())


class ClassPlanner:
    """Anytime-GTMP with the class-indexed archive for a 2D point-robot
    workload: ``stages`` restart stages, at most ``L`` labels per vertex and
    ``cap`` archived classes."""

    def __init__(self, w, reps, stages, L=64, cap=1024, device="cuda"):
        assert w["kind"] == "point2d"
        self.w = w
        d, M, N, G, H = (int(w[k]) for k in ("d", "M", "N", "G", "H"))
        self.M, self.k, self.L, self.cap, self.stages = M, len(reps), L, cap, stages
        self.prob = make_problem(d, M, N, G, H, w["lo"], w["hi"], w["penalty"])
        self.scene = Scene(2, w["circles"], w["boxes"], device)
        self.q0 = torch.from_numpy(np.asarray(w["q0"], np.float32)).to(device)
        self.goals = torch.from_numpy(np.asarray(w["goals"], np.float32).reshape(G, d)).to(device)
        self.reps = torch.from_numpy(np.ascontiguousarray(reps, np.float32).reshape(-1, 2)).to(device)
        self.a_lab = torch.zeros((cap, 2), device=device, dtype=torch.int64)
        self.a_cost = torch.zeros(cap, device=device)
        self.a_stage = torch.zeros(cap, device=device, dtype=torch.int32)
        self.a_wp = torch.zeros((cap, M + 2, 2), device=device)
        self.a_count = torch.zeros(1, device=device, dtype=torch.int32)
        self.overflow = torch.zeros(1, device=device, dtype=torch.int32)
        n = C.c_size_t()
        _check(_lib.gtmp_class_anytime_workspace_size(C.byref(self.prob), L, C.byref(n)))
        self.workspace = _aligned_workspace(n.value, device)
        self.edge_opts = gtmp_edge_opts()

    def run(self, seed, stream=None):
        _check(_lib.gtmp_plan_classes(C.byref(self.prob), C.byref(self.scene.c), _p(self.q0), _p(self.goals), seed,
                                      self.stages, _p(self.reps), self.k, self.L, self.cap, _p(self.a_lab),
                                      _p(self.a_cost), _p(self.a_stage), _p(self.a_wp), _p(self.a_count),
                                      _p(self.overflow), _p(self.workspace), _nbytes(self.workspace),
                                      C.byref(self.edge_opts), _stream(stream)))

    def archive(self):
        n = int(self.a_count.item())
        lab = self.a_lab.cpu().numpy()[:n]
        return {unpack_label(lab[i], self.k): (float(self.a_cost[i].item()), int(self.a_stage[i].item()),
                                               self.a_wp[i].cpu().numpy()) for i in range(n)}
