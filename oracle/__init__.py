"""FP64 CPU reference ("oracle") of the layered-graph planner.

TEST INFRASTRUCTURE.  Only ``tests/``, ``__graft_entry__.smoke()`` and the
CPU-baseline leg of ``bench.py`` may import this package.  It shares no code
with the HIP product path (``paper_2608_25830_amd``) and imports nothing from
it; both take their inputs from the seeded generators in ``workloads``.

The arithmetic lives in ``gtmp_oracle.c`` (plain loops in double precision,
each routine citing the passage of the paper it follows); this module loads it
with ctypes and adds the few pieces that are clearer in Python (brute-force
enumeration of every chain on tiny graphs).

Every function here is pinned by a test in ``tests/test_oracle_*.py`` against
something other than itself: published Philox known-answer vectors,
closed-form signed distances, a DH chain built from
SciPy rotations, brute-force enumeration of all chains, SciPy's graph shortest
path, and closed forms in obstacle-free space.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "gtmp_oracle.c")
_LIB_PATH = os.path.join(_HERE, "liboracle.so")
_lib = None

CFLAGS = ["-O2", "-fopenmp", "-fPIC", "-shared", "-ffp-contract=off", "-fno-fast-math", "-std=c11"]


def build(force: bool = True) -> str:
    """Compile the C oracle with gcc (plain C11, OpenMP over edges)."""
    if force or not os.path.exists(_LIB_PATH):
        tmp = _LIB_PATH + ".tmp"
        subprocess.check_call(["gcc", *CFLAGS, "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            build()
        _lib = C.CDLL(_LIB_PATH)
        _declare(_lib)
    return _lib


_fp = C.POINTER(C.c_float)
_dp = C.POINTER(C.c_double)
_ip = C.POINTER(C.c_int)
_lp = C.POINTER(C.c_long)
_up = C.POINTER(C.c_uint32)


class OrModel(C.Structure):
    _fields_ = [("kind", C.c_int), ("d", C.c_int), ("wdim", C.c_int), ("n_joints", C.c_int),
                ("dh", _fp), ("n_rsph", C.c_int), ("rsph_link", _ip), ("rsph_t", _fp), ("rsph_r", _fp),
                ("n_osph", C.c_int), ("osph", _fp), ("n_obox", C.c_int), ("obox", _fp)]


def _declare(L):
    L.or_threads.restype = C.c_int
    L.or_philox4x32_10.argtypes = [_up, _up, _up]
    L.or_words.argtypes = [C.c_uint64, C.c_uint64, C.c_uint32, C.c_uint32, C.c_uint32, C.c_uint32, _up]
    L.or_sample_layers.argtypes = [C.c_int, C.c_int, C.c_int, _fp, _fp, C.c_uint64, C.c_uint64, _fp]
    L.or_fk_origins.argtypes = [C.c_int, _fp, _dp, _dp]
    L.or_arm_spheres.argtypes = [C.POINTER(OrModel), _dp, _dp]
    L.or_state_sd.argtypes = [C.POINTER(OrModel), _dp]
    L.or_state_sd.restype = C.c_double
    L.or_state_sd_batch.argtypes = [C.POINTER(OrModel), C.c_long, _fp, _dp]
    L.or_edge.argtypes = [C.POINTER(OrModel), C.c_int, C.c_double, C.c_double, _fp, _fp, _dp, _dp, _ip]
    L.or_edge_subset.argtypes = [C.POINTER(OrModel), C.c_int, C.c_int, C.c_int, C.c_int, C.c_double,
                                 C.c_double, _fp, _fp, _fp, C.c_long, _lp, _dp, _dp, _ip]
    L.or_edge_costs.argtypes = [C.POINTER(OrModel), C.c_int, C.c_int, C.c_int, C.c_int, C.c_double,
                                C.c_double, _fp, _fp, _fp, _dp, _dp, _ip]
    L.or_minplus.argtypes = [C.c_int, C.c_int, C.c_int, _dp, _dp, _dp, _dp, _dp, _ip, _dp, _ip]
    L.or_extract.argtypes = [C.c_int, C.c_int, C.c_int, C.c_int, C.c_int, _ip, C.c_double, _fp, _fp, _fp,
                             _ip, _dp, _dp]
    L.or_extract.restype = C.c_int
    L.or_informed_params.argtypes = [C.c_int, _fp, _fp, C.c_float, _fp, _fp, _fp, _fp, _fp]
    L.or_informed_proposal.argtypes = [C.c_int, _fp, _fp, _fp, _fp, C.c_float, C.c_float, _fp, _fp]
    L.or_informed_proposal.restype = C.c_int
    L.or_sample_informed.argtypes = [C.c_int, _fp, _fp, _fp, _fp, C.c_float, C.c_float, C.c_uint64, C.c_uint64,
                                     C.c_uint32, C.c_uint32, C.c_int, _fp]
    L.or_sample_informed.restype = C.c_int
    L.or_coin_heuristic.argtypes = [C.c_uint64, C.c_uint64, C.c_uint32, C.c_uint32]
    L.or_coin_heuristic.restype = C.c_int
    L.or_pair_d2_all.argtypes = [C.c_int, C.c_int, _fp, C.c_int, _fp, _fp]
    L.or_rrtc_sample.argtypes = [C.c_int, _fp, _fp, _fp, _fp, C.c_float, C.c_float, C.c_uint64, C.c_uint64,
                                 C.c_uint32, C.c_uint32, _fp]
    L.or_rrtc_sample.restype = C.c_int
    L.or_rrtc.argtypes = [C.POINTER(OrModel), _fp, _fp, _fp, _fp, C.c_int, C.c_int, C.c_float, C.c_float,
                          C.c_float, C.c_uint64, C.c_uint64, C.c_uint32, C.c_double, _fp, _ip, _dp, _ip, _ip, _ip,
                          _fp, _ip]
    L.or_rrtc.restype = C.c_int
    L.or_rrtc_batch.argtypes = [C.POINTER(OrModel), C.c_int, _fp, _fp, _up, _fp, _fp, C.c_int, C.c_int, C.c_float,
                                C.c_float, C.c_float, C.c_uint64, C.c_uint64, C.c_double, _ip, _dp, _ip, _ip, _ip,
                                _ip]


def threads() -> int:
    return int(lib().or_threads())


def _ptr(a, t):
    return a.ctypes.data_as(t) if a is not None else None


def _f32(a):
    return np.ascontiguousarray(a, dtype=np.float32)


# --------------------------------------------------------------------------- #
# model
# --------------------------------------------------------------------------- #
class Model:
    """Collision model built from a workload dict (see ``workloads``).  Keeps
    the numpy buffers alive for the lifetime of the ctypes struct."""

    def __init__(self, w):
        self.keep = []
        m = OrModel()
        if w["kind"] == "point2d" or w["kind"] == "point":
            d = int(w["d"])
            m.kind, m.d, m.wdim, m.n_joints = 0, d, d, 0
            osph = _f32(w["circles"] if "circles" in w else w["obs_spheres"]).reshape(-1, d + 1)
            obox = _f32(w["boxes"] if "boxes" in w else w["obs_boxes"]).reshape(-1, 2 * d)
            m.n_rsph = 0
        else:
            d = int(w["d"])
            m.kind, m.d, m.wdim, m.n_joints = 1, d, 3, d
            dh = _f32(w["dh"]).reshape(d, 4)
            link = np.ascontiguousarray(w["sph_link"], dtype=np.int32)
            st, sr = _f32(w["sph_t"]), _f32(w["sph_r"])
            self.keep += [dh, link, st, sr]
            m.dh, m.n_rsph = _ptr(dh, _fp), int(link.size)
            m.rsph_link, m.rsph_t, m.rsph_r = _ptr(link, _ip), _ptr(st, _fp), _ptr(sr, _fp)
            osph = _f32(w["obs_spheres"]).reshape(-1, 4)
            obox = _f32(w["obs_boxes"]).reshape(-1, 6)
        self.keep += [osph, obox]
        m.n_osph, m.osph = int(osph.shape[0]), _ptr(osph, _fp)
        m.n_obox, m.obox = int(obox.shape[0]), _ptr(obox, _fp)
        self.c = m
        self.d = d

    def ref(self):
        return C.byref(self.c)


# --------------------------------------------------------------------------- #
# a1: sampler
# --------------------------------------------------------------------------- #
def philox4x32_10(ctr, key):
    c = np.asarray(ctr, dtype=np.uint32)
    k = np.asarray(key, dtype=np.uint32)
    out = np.zeros(4, np.uint32)
    lib().or_philox4x32_10(_ptr(c, _up), _ptr(k, _up), _ptr(out, _up))
    return out


def sample_words(seed, stage, stream, n, m, blk):
    out = np.zeros(4, np.uint32)
    lib().or_words(seed, stage, stream, n, m, blk, _ptr(out, _up))
    return out


def sample_layers(M, N, d, lo, hi, seed, stage=0):
    Q = np.zeros((M, N, d), np.float32)
    lo, hi = _f32(lo), _f32(hi)
    lib().or_sample_layers(M, N, d, _ptr(lo, _fp), _ptr(hi, _fp), seed, stage, _ptr(Q, _fp))
    return Q


# --------------------------------------------------------------------------- #
# a3: collision model
# --------------------------------------------------------------------------- #
def fk_origins(dh, q):
    dh = _f32(dh)
    J = dh.shape[0]
    qq = np.ascontiguousarray(q, dtype=np.float64)
    o = np.zeros((J + 1, 3), np.float64)
    lib().or_fk_origins(J, _ptr(dh, _fp), _ptr(qq, _dp), _ptr(o, _dp))
    return o


def arm_spheres(model: Model, q):
    qq = np.ascontiguousarray(q, dtype=np.float64)
    c = np.zeros((model.c.n_rsph, 3), np.float64)
    lib().or_arm_spheres(model.ref(), _ptr(qq, _dp), _ptr(c, _dp))
    return c


def state_sd(model: Model, X):
    X = _f32(X).reshape(-1, model.d)
    sd = np.zeros(X.shape[0], np.float64)
    lib().or_state_sd_batch(model.ref(), X.shape[0], _ptr(X, _fp), _ptr(sd, _dp))
    return sd


def state_sd64(model: Model, q):
    qq = np.ascontiguousarray(q, dtype=np.float64)
    return lib().or_state_sd(model.ref(), _ptr(qq, _dp))


# --------------------------------------------------------------------------- #
# a2-a4: edges
# --------------------------------------------------------------------------- #
def edge(model: Model, H, u, v, penalty=1e3, max_len=np.inf):
    u, v = _f32(u), _f32(v)
    c, s, f = C.c_double(), C.c_double(), C.c_int()
    lib().or_edge(model.ref(), H, penalty, max_len, _ptr(u, _fp), _ptr(v, _fp), C.byref(c), C.byref(s),
                  C.byref(f))
    return c.value, s.value, f.value


def n_edges(M, N, G=1):
    return N + (M - 1) * N * N + N * G


def edge_costs(model: Model, M, N, G, H, q0, goals, Q, penalty=1e3, max_len=np.inf):
    """All edges.  Returns (C_s[N], C_h[M-1,N,N], C_l[N,G]) for cost, minsd and
    flags, each as a dict with keys 'cost', 'minsd', 'flag' holding the three
    blocks, plus the flat arrays under 'flat_*'."""
    E = n_edges(M, N, G)
    cost = np.zeros(E, np.float64)
    minsd = np.zeros(E, np.float64)
    flag = np.zeros(E, np.int32)
    q0, goals, Q = _f32(q0), _f32(goals), _f32(Q)
    lib().or_edge_costs(model.ref(), M, N, G, H, penalty, max_len, _ptr(q0, _fp), _ptr(goals, _fp),
                        _ptr(Q, _fp), _ptr(cost, _dp), _ptr(minsd, _dp), _ptr(flag, _ip))
    return split_edges(cost, M, N, G), split_edges(minsd, M, N, G), split_edges(flag, M, N, G)


def split_edges(flat, M, N, G):
    a = N
    b = N + (M - 1) * N * N
    return flat[:a].copy(), flat[a:b].reshape(M - 1, N, N).copy(), flat[b:].reshape(N, G).copy()


def edge_subset(model: Model, M, N, G, H, q0, goals, Q, edge_ids, penalty=1e3, max_len=np.inf):
    ids = np.ascontiguousarray(edge_ids, dtype=np.int64)
    n = ids.size
    cost = np.zeros(n, np.float64)
    minsd = np.zeros(n, np.float64)
    flag = np.zeros(n, np.int32)
    q0, goals, Q = _f32(q0), _f32(goals), _f32(Q)
    lib().or_edge_subset(model.ref(), M, N, G, H, penalty, max_len, _ptr(q0, _fp), _ptr(goals, _fp),
                         _ptr(Q, _fp), n, ids.ctypes.data_as(_lp), _ptr(cost, _dp), _ptr(minsd, _dp),
                         _ptr(flag, _ip))
    return cost, minsd, flag


# --------------------------------------------------------------------------- #
# a5-a6: value iteration and extraction
# --------------------------------------------------------------------------- #
def minplus(Cs, Ch, Cl, Vg=None):
    Cs = np.ascontiguousarray(Cs, dtype=np.float64)
    Cl = np.ascontiguousarray(Cl, dtype=np.float64)
    N = Cs.shape[0]
    G = Cl.shape[1]
    Ch = np.ascontiguousarray(Ch, dtype=np.float64).reshape(-1, N, N)
    M = Ch.shape[0] + 1
    V = np.zeros((M, N), np.float64)
    A = np.zeros((M, N), np.int32)
    Vs, a_s = C.c_double(), C.c_int()
    vg = None if Vg is None else np.ascontiguousarray(Vg, dtype=np.float64)
    lib().or_minplus(M, N, G, _ptr(Cs, _dp), _ptr(Ch, _dp), _ptr(Cl, _dp), _ptr(vg, _dp) if vg is not None else None,
                     _ptr(V, _dp), _ptr(A, _ip), C.byref(Vs), C.byref(a_s))
    return V, A, Vs.value, a_s.value


def extract(A, a_s, Vs, Q, q0, goals):
    Q, q0, goals = _f32(Q), _f32(q0), _f32(goals)
    M, N, d = Q.shape
    G = goals.shape[0]
    A = np.ascontiguousarray(A, dtype=np.int32)
    idx = np.zeros(M + 1, np.int32)
    wp = np.zeros((M + 2, d), np.float64)
    cost = C.c_double()
    rc = lib().or_extract(M, N, G, d, a_s, _ptr(A, _ip), Vs, _ptr(Q, _fp), _ptr(q0, _fp), _ptr(goals, _fp),
                          _ptr(idx, _ip), _ptr(wp, _dp), C.byref(cost))
    return idx, wp, cost.value, rc


def brute_force(Cs, Ch, Cl):
    """Minimum over every chain q0 -> v_0 -> ... -> v_{M-1} -> g by explicit
    enumeration (N^M * G chains; tiny graphs only).  Returns (cost, chain)
    where chain = (v_0, ..., v_{M-1}, g) is the lexicographically first
    minimiser."""
    import itertools
    Cs = np.asarray(Cs, np.float64)
    Cl = np.asarray(Cl, np.float64)
    N, G = Cl.shape
    Ch = np.asarray(Ch, np.float64).reshape(-1, N, N)
    M = Ch.shape[0] + 1
    best, arg = np.inf, None
    for chain in itertools.product(range(N), repeat=M):
        for g in range(G):
            c = Cs[chain[0]]
            for m in range(M - 1):
                c += Ch[m, chain[m], chain[m + 1]]
            c += Cl[chain[-1], g]
            if c < best:
                best, arg = c, tuple(chain) + (g,)
    return best, arg


def plan(w, stage=0, Q=None):
    """Whole plain planner on a workload dict: sample, realise and cost every
    edge, value iteration, extraction (Alg. 1 with |K| = 1).  Returns a dict."""
    model = Model(w)
    M, N, G, H, d = w["M"], w["N"], w["G"], w["H"], w["d"]
    if Q is None:
        Q = sample_layers(M, N, d, w["lo"], w["hi"], w["seed"], stage)
    cost, minsd, flag = edge_costs(model, M, N, G, H, w["q0"], w["goals"], Q, w["penalty"])
    V, A, Vs, a_s = minplus(*cost)
    idx, wp, c, rc = extract(A, a_s, Vs, Q, w["q0"], w["goals"])
    return dict(Q=Q, cost=cost, minsd=minsd, flag=flag, V=V, A=A, Vs=Vs, a_s=a_s, idx=idx, wp=wp,
                path_cost=c, no_path=rc)
