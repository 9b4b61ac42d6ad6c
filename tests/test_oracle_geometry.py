"""Pins of the oracle's collision model (Sec. III: open free space, so a
signed distance <= 0 is a collision) and of its DH forward kinematics:
closed-form signed distances at hand-placed points, the planar-arm closed
form, a DH chain composed from SciPy rotations, link-length and base-rotation
identities."""
import math

import numpy as np
import pytest
from scipy.spatial.transform import Rotation

import workloads as wl


def point_model(orc, d, spheres, boxes):
    return orc.Model(dict(kind="point", d=d, obs_spheres=np.asarray(spheres, np.float32),
                          obs_boxes=np.asarray(boxes, np.float32)))


# ----------------------------------------------------------------- 2D / 3D SDF
def test_circle_sd_closed_form(orc):
    m = point_model(orc, 2, [[1.0, 2.0, 1.5]], np.zeros((0, 4)))
    pts = np.array([[1.0, 2.0], [1.0, 4.0], [4.0, 6.0], [2.5, 2.0], [1.0, 2.75]], np.float32)
    want = [-1.5, 0.5, 5.0 - 1.5, 0.0, -0.75]
    np.testing.assert_allclose(orc.state_sd(m, pts), want, atol=1e-12)


def test_box_sd_closed_form(orc):
    # box centred (0, 0), half extents (2, 1)
    m = point_model(orc, 2, np.zeros((0, 3)), [[0.0, 0.0, 2.0, 1.0]])
    pts = np.array([[0.0, 0.0], [1.5, 0.0], [0.0, 3.0], [5.0, 5.0], [2.0, 0.5], [-3.0, 0.0]], np.float32)
    want = [-1.0, -0.5, 2.0, 5.0, 0.0, 1.0]
    want[3] = math.hypot(3.0, 4.0)
    np.testing.assert_allclose(orc.state_sd(m, pts), want, atol=1e-12)


def test_box_sd_3d_and_union_min(orc):
    m = point_model(orc, 3, [[0, 0, 5, 1]], [[0, 0, 0, 1, 1, 1]])
    pts = np.array([[0, 0, 3.0], [2, 2, 2], [0, 0, 0.5], [0, 0, 5]], np.float32)
    want = [1.0, math.sqrt(3.0), -0.5, -1.0]
    # (0,0,3): box distance 2, sphere distance 2 - 1 = 1
    np.testing.assert_allclose(orc.state_sd(m, pts), want, atol=1e-12)


def test_empty_scene_is_free(orc):
    m = point_model(orc, 2, np.zeros((0, 3)), np.zeros((0, 4)))
    assert np.all(np.isinf(orc.state_sd(m, np.zeros((4, 2), np.float32))))


# ----------------------------------------------------------------- DH FK
def dh_chain_scipy(dh, q):
    """Frame origins from 4x4 transforms composed of SciPy elementary
    rotations: A_i = Rz(q_i + off_i) Tz(d_i) Tx(a_i) Rx(alpha_i)."""
    T = np.eye(4)
    out = [T[:3, 3].copy()]
    for (a, alpha, dz, off), qi in zip(np.asarray(dh, np.float64), q):
        Rz = np.eye(4); Rz[:3, :3] = Rotation.from_euler("z", qi + off).as_matrix()
        Tz = np.eye(4); Tz[2, 3] = dz
        Tx = np.eye(4); Tx[0, 3] = a
        Rx = np.eye(4); Rx[:3, :3] = Rotation.from_euler("x", alpha).as_matrix()
        T = T @ Rz @ Tz @ Tx @ Rx
        out.append(T[:3, 3].copy())
    return np.array(out)


@pytest.mark.parametrize("seed", [0, 1, 2, 3])
def test_fk_matches_scipy_composition(orc, seed):
    dh = wl.arm_robot(seed)[0]
    g = np.random.default_rng(seed)
    for _ in range(20):
        q = g.uniform(-math.pi, math.pi, 7)
        np.testing.assert_allclose(orc.fk_origins(dh, q), dh_chain_scipy(dh, q), atol=1e-12)


def test_fk_planar_closed_form(orc):
    g = np.random.default_rng(5)
    a = g.uniform(0.1, 0.4, 5).astype(np.float32)
    dh = np.stack([a, np.zeros(5), np.zeros(5), np.zeros(5)], 1).astype(np.float32)
    q = g.uniform(-3, 3, 5)
    o = orc.fk_origins(dh, q)
    cs = np.cumsum(q)
    x = np.cumsum(a.astype(np.float64) * np.cos(cs))
    y = np.cumsum(a.astype(np.float64) * np.sin(cs))
    np.testing.assert_allclose(o[1:, 0], x, atol=1e-12)
    np.testing.assert_allclose(o[1:, 1], y, atol=1e-12)
    np.testing.assert_allclose(o[:, 2], 0.0, atol=1e-15)


def test_fk_link_length_and_base_rotation(orc):
    dh = wl.arm_robot(7)[0].astype(np.float64)
    g = np.random.default_rng(1)
    for _ in range(10):
        q = g.uniform(-math.pi, math.pi, 7)
        o = orc.fk_origins(dh.astype(np.float32), q)
        L = np.linalg.norm(np.diff(o, axis=0), axis=1)
        np.testing.assert_allclose(L, np.hypot(dh[:, 0].astype(np.float32), dh[:, 2].astype(np.float32)), atol=1e-12)
        # turning joint 1 by delta rotates every origin about the base z axis
        delta = 0.7
        q2 = q.copy(); q2[0] += delta
        R = Rotation.from_euler("z", delta).as_matrix()
        np.testing.assert_allclose(orc.fk_origins(dh.astype(np.float32), q2), o @ R.T, atol=1e-12)


def test_arm_spheres_on_links(orc):
    w = wl.make_workload("arm7", seed=3, sg=0)
    m = orc.Model(w)
    q = np.random.default_rng(2).uniform(-3, 3, 7)
    o = orc.fk_origins(w["dh"], q)
    c = orc.arm_spheres(m, q)
    L = w["sph_link"]; t = w["sph_t"].astype(np.float64)
    want = o[L - 1] + t[:, None] * (o[L] - o[L - 1])
    np.testing.assert_allclose(c, want, atol=1e-12)
    assert len(L) == 40 and np.all(np.diff(L) >= 0)


def test_arm_sd_obstacle_on_sphere(orc):
    w = wl.make_workload("arm7", seed=3, sg=0)
    q = np.random.default_rng(9).uniform(-3, 3, 7)
    base = orc.Model(w)
    c = orc.arm_spheres(base, q)
    k = 17
    w2 = dict(w)
    w2["obs_spheres"] = np.array([[c[k, 0], c[k, 1], c[k, 2], 0.1]], np.float32)
    w2["obs_boxes"] = np.zeros((0, 6), np.float32)
    sd = orc.state_sd64(orc.Model(w2), q)
    # the obstacle centre is the float32 rounding of the sphere centre
    assert sd == pytest.approx(-(0.1 + float(np.float32(0.05))), abs=1e-6)
    assert sd <= 0


def test_arm_free_in_empty_scene(orc):
    w = wl.make_workload("arm7", seed=3, sg=0)
    w["obs_spheres"] = np.zeros((0, 4), np.float32)
    w["obs_boxes"] = np.zeros((0, 6), np.float32)
    assert np.isinf(orc.state_sd64(orc.Model(w), np.zeros(7)))
