"""Pins for the oracle's Snavely model (Section VI-A factor) and its tangent
Jacobian (Section V tangent-space linearisation)."""
import json
import os

import numpy as np
import pytest
import scipy.linalg
from scipy.spatial.transform import Rotation

from oracle import camera
from synth import scene_config

from helpers import small_scene

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "snavely_worked_examples.json")


def test_golden_worked_examples():
    cases = json.load(open(GOLDEN))["cases"]
    for c in cases:
        st = camera.State.from_bal(np.array([c["cam_bal"]]), np.array([c["point"]]))
        u = camera.project(st, np.array([0]), np.array([0]))[0]
        r = camera.residuals(st, np.array([0]), np.array([0]), np.array([c["px"]]))[0]
        np.testing.assert_allclose(u, c["u"], rtol=1e-13, atol=1e-12, err_msg=c["name"])
        np.testing.assert_allclose(r, c["residual"], rtol=1e-11, atol=1e-11, err_msg=c["name"])


def test_pinhole_special_case():
    # R = I, t = 0, k1 = k2 = 0: u = -f X_xy / X_z exactly (up to the depth epsilon)
    rng = np.random.default_rng(0)
    X = rng.uniform(-3, 3, size=(50, 3))
    X[:, 2] = -rng.uniform(1, 5, size=50)
    cams = np.zeros((1, 9))
    cams[0, 6] = 321.0
    st = camera.State.from_bal(cams, X)
    u = camera.project(st, np.zeros(50, dtype=int), np.arange(50))
    np.testing.assert_allclose(u, -321.0 * X[:, :2] / X[:, 2:3], rtol=1e-13)


def test_rodrigues_matches_scipy_and_expm():
    rng = np.random.default_rng(1)
    w = np.concatenate([rng.normal(size=(20, 3)),
                        1e-6 * rng.normal(size=(5, 3)),
                        np.array([[np.pi, 0, 0], [0, 0, 0], [0, 1e-9, 0]]),
                        (np.pi - 1e-7) * np.array([[0.6, 0.8, 0.0]])])
    R = camera.so3_exp(w)
    np.testing.assert_allclose(R, Rotation.from_rotvec(w).as_matrix(), atol=2e-15)
    for wi, Ri in zip(w, R):
        np.testing.assert_allclose(Ri, scipy.linalg.expm(camera.hat(wi)), atol=2e-15)


def test_synthetic_cameras_face_origin_with_negative_depth():
    sc = scene_config("tiny")
    st = camera.State.from_bal(sc.cams_true, sc.points_true)
    # origin in the camera frame is t: depth -10 for a circle of radius 10
    np.testing.assert_allclose(st.t, np.tile([0.0, 0.0, -10.0], (sc.n_cams, 1)), atol=1e-12)
    P = np.einsum("oij,oj->oi", st.R[sc.obs_cam], st.X[sc.obs_pt]) + st.t[sc.obs_cam]
    assert np.all(P[:, 2] < -7.0) and np.all(P[:, 2] > -13.0)
    for Ri in st.R:
        np.testing.assert_allclose(Ri @ Ri.T, np.eye(3), atol=1e-14)
        assert abs(np.linalg.det(Ri) - 1.0) < 1e-14


def _fd_jacobian(st, obs_cam, obs_pt, px, h_rel=1e-6):
    nc, npnt = st.n_cams, st.n_points
    N = 9 * nc + 3 * npnt
    cols = []
    for i in range(N):
        e = np.zeros(N)
        scale = 1.0
        if i < 9 * nc and i % 9 == 6:
            scale = st.calib[i // 9, 0]
        h = h_rel * max(1.0, scale)
        e[i] = h
        rp = camera.residuals(st.retract(e), obs_cam, obs_pt, px)
        rm = camera.residuals(st.retract(-e), obs_cam, obs_pt, px)
        cols.append(((rp - rm) / (2 * h)).ravel())
    return np.stack(cols, axis=1)


@pytest.mark.parametrize("seed", [0, 1])
def test_jacobian_matches_central_differences(seed):
    sc = small_scene(n_cams=3, n_points=8, seed=seed, k=2)
    rng = np.random.default_rng(seed)
    cams = sc.cams_init.copy()
    cams[:, 7:9] = rng.normal(0, 0.05, size=(sc.n_cams, 2))   # make distortion matter
    st = camera.State.from_bal(cams, sc.points_init)
    px = rng.normal(0, 50, size=(sc.n_obs, 2))
    r, Jc, Jp = camera.linearize(st, sc.obs_cam, sc.obs_pt, px)
    n = sc.n_obs
    J = np.zeros((2 * n, 9 * sc.n_cams + 3 * sc.n_points))
    for o in range(n):
        c, p = sc.obs_cam[o], sc.obs_pt[o]
        J[2 * o:2 * o + 2, 9 * c:9 * c + 9] = Jc[o]
        J[2 * o:2 * o + 2, 9 * sc.n_cams + 3 * p:9 * sc.n_cams + 3 * p + 3] = Jp[o]
    Jfd = _fd_jacobian(st, sc.obs_cam, sc.obs_pt, px)
    for i in range(J.shape[1]):
        denom = max(np.linalg.norm(Jfd[:, i]), 1e-3)
        assert np.linalg.norm(J[:, i] - Jfd[:, i]) / denom < 1e-6, i


def test_jacobian_near_degenerate_depth_and_large_rotation():
    # point close to the camera plane and a rotation angle near pi
    cams = np.array([[np.pi - 1e-3, 0.2, 0.1, 0.3, -0.2, 0.5, 300.0, 0.02, -0.01]])
    X = np.array([[0.3, -0.2, 0.9]])
    st = camera.State.from_bal(cams, X)
    P = st.R[0] @ X[0] + st.t[0]
    assert abs(P[2]) < 0.6
    px = np.zeros((1, 2))
    r, Jc, Jp = camera.linearize(st, np.array([0]), np.array([0]), px)
    Jfd = _fd_jacobian(st, np.array([0]), np.array([0]), px, h_rel=1e-7)
    J = np.concatenate([Jc[0], Jp[0]], axis=1)
    np.testing.assert_allclose(J, Jfd, rtol=1e-5, atol=1e-5 * np.abs(J).max())


def test_gauge_directions_are_in_the_jacobian_null_space():
    sc = small_scene(n_cams=5, n_points=40, seed=3, k=3)
    st = camera.State.from_bal(sc.cams_init, sc.points_init)
    px = np.zeros((sc.n_obs, 2))
    _, Jc, Jp = camera.linearize(st, sc.obs_cam, sc.obs_pt, px)
    from oracle import linear
    J = linear.jacobian_csr(Jc, Jp, sc.obs_cam, sc.obs_pt, sc.n_cams, sc.n_points)
    N = camera.gauge_generators(st)
    scale = abs(J).max()
    for k in range(7):
        v = J @ N[k]
        assert np.linalg.norm(v) <= 1e-10 * scale * np.linalg.norm(N[k]), k
    # a non-gauge direction is not in the null space
    assert np.linalg.norm(J @ np.random.default_rng(0).normal(size=J.shape[1])) > 1.0
