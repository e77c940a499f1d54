"""Pins of the robust-loss oracle (oracle/robust.py).

Each pin checks the oracle against something other than itself: central
differences of rho and of the robust cost, the plain problem in the limits
where the losses reduce to it, and the statistical effect robust losses
exist for (planted outliers move the plain optimum, not the robust one).
"""
import numpy as np
import pytest

from oracle import camera, linear, lm, robust
from synth import scene_config

from helpers import observed_pixels


@pytest.mark.parametrize("kind", ["huber", "cauchy"])
@pytest.mark.parametrize("c", [0.5, 3.0])
def test_weight_is_derivative_of_rho(kind, c):
    s = np.concatenate([np.linspace(1e-3, 4 * c * c, 57), [0.3 * c * c, 2.5 * c * c]])
    s = s[np.abs(s - c * c) > 1e-3]          # huber has a kink in rho'' at c^2
    h = 1e-6 * np.maximum(s, 1.0)
    fd = (robust.rho(kind, s + h, c) - robust.rho(kind, s - h, c)) / (2 * h)
    np.testing.assert_allclose(robust.weight(kind, s, c), fd, rtol=1e-7, atol=1e-9)


def test_closed_forms_at_special_points():
    c = 2.0
    # huber: quadratic inside, rho(c^2) continuous, linear growth in |r| outside
    assert robust.rho("huber", np.array([c * c]), c)[0] == pytest.approx(c * c)
    assert robust.rho("huber", np.array([16.0]), c)[0] == pytest.approx(2 * c * 4 - c * c)
    # cauchy: rho(c^2) = c^2 log 2, weight 1/2 there
    assert robust.rho("cauchy", np.array([c * c]), c)[0] == pytest.approx(c * c * np.log(2.0))
    assert robust.weight("cauchy", np.array([c * c]), c)[0] == pytest.approx(0.5)


@pytest.mark.parametrize("kind", ["huber", "cauchy"])
def test_scaled_gradient_matches_cost_differences(kind):
    sc = scene_config("tiny_outliers")
    px = observed_pixels(sc)
    st = camera.State.from_bal(sc.cams_init, sc.points_init)
    c = 3.0
    F, r, Jc, Jp, w = robust.linearize(st, sc.obs_cam, sc.obs_pt, px, kind, c)
    assert F == pytest.approx(robust.cost(st, sc.obs_cam, sc.obs_pt, px, kind, c), rel=1e-15)
    J = linear.jacobian_csr(Jc, Jp, sc.obs_cam, sc.obs_pt, st.n_cams, st.n_points)
    g = linear.gradient(J, r.reshape(-1))
    rng = np.random.default_rng(7)
    for j in rng.choice(st.n_params, 12, replace=False):
        e = np.zeros(st.n_params)
        h = 1e-6
        e[j] = h
        fd = (robust.cost(st.retract(e), sc.obs_cam, sc.obs_pt, px, kind, c)
              - robust.cost(st.retract(-e), sc.obs_cam, sc.obs_pt, px, kind, c)) / (2 * h)
        assert g[j] == pytest.approx(fd, rel=1e-5, abs=1e-6 * np.abs(g).max())


def test_huber_equals_plain_problem_inside_scale():
    sc = scene_config("tiny")
    px = observed_pixels(sc)
    st = camera.State.from_bal(sc.cams_init, sc.points_init)
    r = camera.residuals(st, sc.obs_cam, sc.obs_pt, px)
    c = 1.01 * np.sqrt(np.max(np.sum(r * r, axis=1)))   # every residual inside
    F, rs, Jc, Jp, w = robust.linearize(st, sc.obs_cam, sc.obs_pt, px, "huber", c)
    r0, Jc0, Jp0 = camera.linearize(st, sc.obs_cam, sc.obs_pt, px)
    assert np.all(w == 1.0)
    assert F == pytest.approx(camera.cost(st, sc.obs_cam, sc.obs_pt, px), rel=1e-15)
    np.testing.assert_array_equal(Jc, Jc0)
    np.testing.assert_array_equal(rs, r0)


def test_cauchy_tends_to_plain_cost():
    sc = scene_config("tiny")
    px = observed_pixels(sc)
    st = camera.State.from_bal(sc.cams_init, sc.points_init)
    F0 = camera.cost(st, sc.obs_cam, sc.obs_pt, px)
    errs = [abs(robust.cost(st, sc.obs_cam, sc.obs_pt, px, "cauchy", c) - F0) / F0 for c in (1e2, 1e3, 1e4)]
    assert errs[0] > errs[1] > errs[2] and errs[2] < 1e-6


def _pose_error(st, sc):
    true = camera.State.from_bal(sc.cams_true, sc.points_true)
    # gauge-free comparison: predicted pixels of the clean scene
    u = camera.project(st, sc.obs_cam, sc.obs_pt)
    u0 = camera.project(true, sc.obs_cam, sc.obs_pt)
    return float(np.sqrt(np.mean(np.sum((u - u0) ** 2, axis=1))))


@pytest.mark.slow
def test_robust_losses_resist_planted_outliers():
    sc = scene_config("tiny_outliers")
    px = observed_pixels(sc)
    st0 = camera.State.from_bal(sc.cams_init, sc.points_init)
    err = {}
    for kind in ("trivial", "huber", "cauchy"):
        res = lm.solve(st0, sc.obs_cam, sc.obs_pt, px,
                       lm.LMOptions(max_iters=40, inner="schur", loss=kind, loss_scale=3.0))
        err[kind] = _pose_error(res.state, sc)
        accepted = [h.cost for h in res.history if h.accepted]
        assert all(b <= a for a, b in zip(accepted, accepted[1:]))
    # the plain optimum is pulled by 40 px outliers; the robust ones stay at
    # the inlier noise level (1 px noise, a few observations per point)
    assert err["huber"] < 0.5 * err["trivial"]
    assert err["cauchy"] < 0.5 * err["trivial"]
