"""Pins of the pose between-factor oracle (oracle/between.py) and of the LM
oracle with between-factors added (oracle/lm.py)."""
import numpy as np
import pytest

from oracle import between, camera, lm
from synth import scene_config

from helpers import between_factors, observed_pixels, small_scene


def test_log_inverts_exp_over_the_whole_angle_range():
    rng = np.random.default_rng(0)
    angles = np.concatenate([[1e-12, 1e-6, 1e-4, 0.3, 1.9, 2.0, 2.1], np.linspace(3.0, np.pi, 9)])
    for th in angles:
        for _ in range(5):
            n = rng.normal(size=3)
            n /= np.linalg.norm(n)
            phi = th * n
            got = between.so3_log(camera.so3_exp(phi))
            err = np.linalg.norm(got - phi)
            if th > np.pi - 1e-9:            # at pi, phi and -phi are the same rotation
                err = min(err, np.linalg.norm(got + phi))
            assert err <= 4e-15, (th, err)


def test_log_of_known_rotations():
    # a quarter turn about z, and a half turn about x
    Rz = np.array([[0.0, -1.0, 0.0], [1.0, 0.0, 0.0], [0.0, 0.0, 1.0]])
    assert np.allclose(between.so3_log(Rz), [0.0, 0.0, np.pi / 2], atol=1e-15, rtol=0)
    Rx = np.diag([1.0, -1.0, -1.0])
    assert np.allclose(np.abs(between.so3_log(Rx)), [np.pi, 0.0, 0.0], atol=1e-15, rtol=0)


@pytest.mark.parametrize("th", [1e-7, 0.2, 1.5, 2.8])
def test_inverse_right_jacobian_matches_central_differences(th):
    rng = np.random.default_rng(1)
    n = rng.normal(size=3)
    phi = th * n / np.linalg.norm(n)
    R = camera.so3_exp(phi)
    h = 1e-6
    fd = np.empty((3, 3))
    for k in range(3):
        e = np.zeros(3)
        e[k] = h
        fd[:, k] = (between.so3_log(R @ camera.so3_exp(e)) - between.so3_log(R @ camera.so3_exp(-e))) / (2 * h)
    assert np.max(np.abs(fd - between.so3_jr_inv(phi))) <= 2e-9


def test_relative_pose_against_homogeneous_matrices():
    sc = small_scene(n_cams=5, n_points=10)
    st = camera.State.from_bal(sc.cams_true, sc.points_true)
    fi, fj = np.array([0, 1, 4]), np.array([3, 2, 0])
    T = np.zeros((5, 4, 4))
    T[:, :3, :3], T[:, :3, 3], T[:, 3, 3] = st.R, st.t, 1.0
    Tij = np.stack([T[j] @ np.linalg.inv(T[i]) for i, j in zip(fi, fj)])
    Z = np.concatenate([between.so3_log(Tij[:, :3, :3]), Tij[:, :3, 3]], axis=1)
    r = between.residuals(st, fi, fj, Z, np.ones((3, 2)))
    assert np.max(np.abs(r)) <= 1e-13
    # a known offset in the measured translation shows up with the weight
    Z2 = Z.copy()
    Z2[1, 4] += 0.5
    r2 = between.residuals(st, fi, fj, Z2, np.array([[1.0, 3.0]] * 3))
    assert abs(r2[1, 4] + 1.5) <= 1e-13 and np.max(np.abs(np.delete(r2.ravel(), 10))) <= 1e-13


def _perturbed(st, c, k, h):
    d = np.zeros(st.n_params)
    d[9 * c + k] = h
    return st.retract(d)


def test_blocks_match_central_differences():
    sc = small_scene(n_cams=6, n_points=20)
    fi, fj, Z, w = between_factors(sc, seed=3, n_loops=4)
    st = camera.State.from_bal(sc.cams_init, sc.points_init)
    r, Ji, Jj = between.linearize(st, fi, fj, Z, w)
    h = 1e-6
    for f in range(len(fi)):
        for side, c, Jb in ((0, fi[f], Ji), (1, fj[f], Jj)):
            for k in range(9):
                rp = between.residuals(_perturbed(st, c, k, h), fi[f:f + 1], fj[f:f + 1], Z[f:f + 1], w[f:f + 1])
                rm = between.residuals(_perturbed(st, c, k, -h), fi[f:f + 1], fj[f:f + 1], Z[f:f + 1], w[f:f + 1])
                fd = (rp - rm)[0] / (2 * h)
                scale = max(1.0, np.max(np.abs(Jb[f])))
                assert np.max(np.abs(fd - Jb[f, :, k])) <= 2e-7 * scale, (f, side, k)


def test_rigid_gauge_is_null_and_scale_is_not():
    sc = small_scene(n_cams=6, n_points=20)
    fi, fj, Z, w = between_factors(sc, seed=3, n_loops=4)
    st = camera.State.from_bal(sc.cams_init, sc.points_init)
    _, Ji, Jj = between.linearize(st, fi, fj, Z, w)
    J = between.jacobian_csr(Ji, Jj, fi, fj, st.n_cams, st.n_points).toarray()
    N = camera.gauge_generators(st)
    for k in range(6):
        assert np.max(np.abs(J @ N[k])) <= 1e-9 * np.max(np.abs(J)), k
    assert np.max(np.abs(J @ N[6])) >= 1e-3


def test_lm_with_between_factors():
    sc = scene_config("tiny")
    px = observed_pixels(sc, noise_scale=0.0)
    fi, fj, Z, w = between_factors(sc, seed=5, n_loops=4, rot_sigma=1e-3, trans_sigma=1e-2)
    _, _, Z_exact, _ = between_factors(sc, seed=5, n_loops=4, rot_sigma=1e-3, trans_sigma=1e-2, noise=False)
    st_true = camera.State.from_bal(sc.cams_true, sc.points_true)
    assert np.max(np.abs(between.residuals(st_true, fi, fj, Z_exact, w))) <= 1e-9
    st0 = camera.State.from_bal(sc.cams_init, sc.points_init)
    res = lm.solve(st0, sc.obs_cam, sc.obs_pt, px, lm.LMOptions(max_iters=30, between=(fi, fj, Z_exact, w)))
    assert res.final_cost <= 1e-12 * res.initial_cost
    # noisy pixels and measurements: accepted costs never increase, and the
    # reported cost is reprojection plus between cost of the returned state
    px_n = observed_pixels(sc)
    opts = lm.LMOptions(max_iters=20, between=(fi, fj, Z, w))
    res = lm.solve(st0, sc.obs_cam, sc.obs_pt, px_n, opts)
    costs = [res.initial_cost] + [it.cost for it in res.history]
    assert all(b <= a for a, b in zip(costs, costs[1:]))
    F = camera.cost(res.state, sc.obs_cam, sc.obs_pt, px_n) + between.cost(res.state, fi, fj, Z, w)
    assert abs(F - res.final_cost) <= 1e-12 * F
    # the between residuals at the optimum are of the size of their noise
    rb = between.residuals(res.state, fi, fj, Z, w)
    assert np.sqrt(np.mean(rb ** 2)) <= 3.0
