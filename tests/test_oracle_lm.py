"""Pins for the oracle LM (Section V: Levenberg-Marquardt with the gain-ratio
damping update, tangent-space retraction)."""
import numpy as np
import pytest
import scipy.optimize
import scipy.sparse as sp
from scipy.spatial.transform import Rotation

from oracle import camera, lm
from synth import scene_config

from helpers import small_scene, observed_pixels


def _solve(sc, noise_scale=1.0, **opts):
    px = observed_pixels(sc, noise_scale)
    st = camera.State.from_bal(sc.cams_init, sc.points_init)
    return lm.solve(st, sc.obs_cam, sc.obs_pt, px, lm.LMOptions(**opts)), px


def test_zero_noise_converges_to_zero_cost():
    sc = scene_config("tiny")
    res, _ = _solve(sc, noise_scale=0.0, max_iters=20)
    assert res.initial_cost > 1e3
    assert res.final_cost <= 1e-20 * res.initial_cost


@pytest.mark.parametrize("inner", ["schur", "pcg"])
def test_accepted_costs_decrease_monotonically(inner):
    sc = small_scene(n_cams=6, n_points=200, seed=11, k=4)
    res, _ = _solve(sc, max_iters=15, inner=inner)
    costs = [res.initial_cost] + [h.cost for h in res.history]
    assert all(b <= a for a, b in zip(costs, costs[1:]))
    prev = res.initial_cost
    for h in res.history:
        if h.accepted:
            assert h.rho > 0 and h.cost == h.trial_cost < prev
        else:
            assert h.cost == prev
        prev = h.cost
    assert res.final_cost < 0.2 * res.initial_cost


def test_dense_and_schur_steps_give_the_same_trajectory():
    sc = small_scene(n_cams=3, n_points=25, seed=4, k=3)
    a, _ = _solve(sc, max_iters=8, inner="dense")
    b, _ = _solve(sc, max_iters=8, inner="schur")
    for ha, hb in zip(a.history, b.history):
        assert ha.accepted == hb.accepted
        assert abs(ha.cost - hb.cost) <= 1e-9 * ha.cost


def test_noisy_optimum_matches_chi_square_expectation():
    # sigma = 1 px: E[2 F*] = 2 n_obs - (N - 7), std sqrt(2 (2 n_obs - N + 7))
    sc = scene_config("tiny")
    res, _ = _solve(sc, max_iters=20)
    dof = 2 * sc.n_obs - (9 * sc.n_cams + 3 * sc.n_points - 7)
    assert abs(2 * res.final_cost - dof) < 4 * np.sqrt(2 * dof)


def _independent_residual(x, nc, npnt, obs_cam, obs_pt, px):
    """BAL model written with scipy's rotation, additive angle-axis."""
    cams = x[: 9 * nc].reshape(nc, 9)
    X = x[9 * nc:].reshape(npnt, 3)
    rot = Rotation.from_rotvec(cams[:, 0:3])
    P = np.empty((obs_cam.size, 3))
    for c in range(nc):
        m = obs_cam == c
        P[m] = rot[c].apply(X[obs_pt[m]]) + cams[c, 3:6]
    p = -P[:, :2] / P[:, 2:3]
    n2 = np.sum(p * p, axis=1, keepdims=True)
    k1, k2, f = cams[obs_cam, 7:8], cams[obs_cam, 8:9], cams[obs_cam, 6:7]
    return (f * (1 + k1 * n2 + k2 * n2 * n2) * p - px).ravel()


@pytest.mark.slow
def test_independent_least_squares_reaches_the_same_cost():
    sc = scene_config("tiny")
    res, px = _solve(sc, max_iters=30)
    nc, npnt = sc.n_cams, sc.n_points
    x0 = np.concatenate([sc.cams_init.ravel(), sc.points_init.ravel()])
    rows = np.repeat(np.arange(2 * sc.n_obs), 12)
    cols = np.concatenate([
        (9 * sc.obs_cam[:, None] + np.arange(9)[None, :]),
        (9 * nc + 3 * sc.obs_pt[:, None] + np.arange(3)[None, :])], axis=1)
    cols = np.repeat(cols, 2, axis=0).ravel()
    S = sp.csr_matrix((np.ones(rows.size), (rows, cols)), shape=(2 * sc.n_obs, x0.size))
    out = scipy.optimize.least_squares(
        _independent_residual, x0, jac="3-point", jac_sparsity=S, method="trf",
        x_scale="jac", ftol=1e-15, xtol=1e-15, gtol=1e-15, max_nfev=200,
        tr_options={"atol": 1e-14, "btol": 1e-14},
        args=(nc, npnt, sc.obs_cam, sc.obs_pt, px))
    assert abs(out.cost - res.final_cost) <= 1e-9 * res.final_cost, (out.cost, res.final_cost)


def test_predicted_decrease_stop_ends_at_the_cost_resolution():
    """pred_tol: once the step's predicted decrease is below a few DBL_EPSILON
    of F, the gain ratio is rounding noise; the solve stops there with the
    converged cost."""
    from oracle import camera as cam_mod
    sc = small_scene(n_cams=6, n_points=200, seed=11, k=4)
    px = observed_pixels(sc)
    st = cam_mod.State.from_bal(sc.cams_init, sc.points_init)
    full = lm.solve(st, sc.obs_cam, sc.obs_pt, px, lm.LMOptions(max_iters=30, inner="schur"))
    tol = 4 * np.finfo(np.float64).eps
    stop = lm.solve(st, sc.obs_cam, sc.obs_pt, px, lm.LMOptions(max_iters=30, inner="schur", pred_tol=tol))
    assert stop.stop_reason == "pred"
    assert len(stop.history) < len(full.history)
    assert all(h.pred > tol * h_prev for h, h_prev in
               zip(stop.history, [stop.initial_cost] + [h.cost for h in stop.history]))
    assert abs(stop.final_cost - full.final_cost) <= 1e-12 * full.final_cost


# ---- gain ratio and damping update (Section V, after Madsen and Nielsen) ----

def _hard_start(seed, n_cams=6, n_points=60):
    """A small scene whose point 0 starts 90% of the way toward a camera that
    sees it: the first linear models mispredict the cost badly."""
    return small_scene(n_cams=n_cams, n_points=n_points, seed=seed, k=3, pull_first_point=0.9)


def _fd_model_decrease(state, sc, px, delta):
    """L(0) - L(delta) for L(d) = 1/2 |r + J d|^2, with J delta taken as the
    central difference of the residual along the retraction curve
    s -> state (+) s delta (whose derivative at 0 is J delta), step 1e-5
    relative to delta, and the result refined by one Richardson step."""
    r0 = camera.residuals(state, sc.obs_cam, sc.obs_pt, px).ravel()

    def jd(h):
        rp = camera.residuals(state.retract(h * delta), sc.obs_cam, sc.obs_pt, px).ravel()
        rm = camera.residuals(state.retract(-h * delta), sc.obs_cam, sc.obs_pt, px).ravel()
        return (rp - rm) / (2.0 * h)

    h = 1e-5 / max(1.0, float(np.max(np.abs(delta))))
    Jd = (4.0 * jd(h) - jd(2.0 * h)) / 3.0
    return 0.5 * float(r0 @ r0) - 0.5 * float((r0 + Jd) @ (r0 + Jd))


def _replay_states(st0, history):
    """The state each iteration started from: accepted steps are retracted."""
    out, st = [], st0
    for h in history:
        out.append(st)
        if h.accepted:
            st = st.retract(h.step)
    return out


@pytest.mark.parametrize("inner", ["schur", "pcg"])
def test_predicted_decrease_equals_the_linear_model_decrease(inner):
    """The gain ratio's denominator is L(0) - L(delta) of the linear model:
    checked for every trial of a run with rejections, with J delta from
    finite differences (not from the oracle's Jacobian), and its ratio with
    the true decrease is the reported rho."""
    sc = _hard_start(5)
    px = observed_pixels(sc)
    st0 = camera.State.from_bal(sc.cams_init, sc.points_init)
    res = lm.solve(st0, sc.obs_cam, sc.obs_pt, px,
                   lm.LMOptions(max_iters=10, lambda0=1e-6, inner=inner, pcg_tol=1e-2))
    assert not all(h.accepted for h in res.history)
    for h, st in zip(res.history, _replay_states(st0, res.history)):
        model = _fd_model_decrease(st, sc, px, h.step)
        assert abs(h.pred - model) <= 1e-6 * abs(model), (h.pred, model)
        F = camera.cost(st, sc.obs_cam, sc.obs_pt, px)
        Ft = camera.cost(st.retract(h.step), sc.obs_cam, sc.obs_pt, px)
        assert abs(h.rho - (F - Ft) / model) <= 1e-6 * max(1.0, abs(h.rho))


def test_predicted_decrease_counts_the_inner_residual():
    """For a step that is not a Galerkin solution (a random direction) the
    inner residual's term matters: the formula still gives the model decrease."""
    from oracle import linear
    sc = _hard_start(5)
    px = observed_pixels(sc)
    st = camera.State.from_bal(sc.cams_init, sc.points_init)
    r, Jc, Jp = camera.linearize(st, sc.obs_cam, sc.obs_pt, px)
    J = linear.jacobian_csr(Jc, Jp, sc.obs_cam, sc.obs_pt, sc.n_cams, sc.n_points)
    D = linear.damping_diagonal(J)
    b = -linear.gradient(J, r.ravel())
    delta = 1e-3 * np.random.default_rng(3).normal(size=b.size)
    lam = 0.7
    r_in = b - linear.matvec(J, D, lam, delta)
    model = _fd_model_decrease(st, sc, px, delta)
    assert abs(delta @ r_in) > 1e-2 * abs(model)      # the term is not negligible here
    pred = lm.predicted_decrease(b, delta, r_in, lam, D)
    assert abs(pred - model) <= 1e-6 * abs(model), (pred, model)


def test_good_steps_divide_lambda_by_three():
    """Zero noise, start near the truth: the linear model predicts every
    resolvable trial to within a percent (rho >= 0.99), and the update then
    divides lambda by exactly 3."""
    sc = scene_config("tiny", rot_std=1e-4, trans_std=5e-4, point_std=5e-4)
    px = observed_pixels(sc, noise_scale=0.0)
    st0 = camera.State.from_bal(sc.cams_init, sc.points_init)
    res = lm.solve(st0, sc.obs_cam, sc.obs_pt, px, lm.LMOptions(max_iters=4, lambda0=1e-2))
    F = res.initial_cost
    checked = 0
    for h, nxt in zip(res.history, res.history[1:]):
        if h.pred <= 1e-10 * F:
            break
        assert h.accepted and h.rho >= 0.99, h.rho
        assert nxt.lam == pytest.approx(h.lam / 3.0, rel=1e-15)
        F = h.cost
        checked += 1
    assert checked >= 2


@pytest.mark.parametrize("seed,lambda0,pattern", [(5, 1e-6, "AArrrrrA"), (3, 1e-2, "AAAAArrArA")])
def test_rejections_double_nu_and_an_accept_resets_it(seed, lambda0, pattern):
    """A run of rejected trials multiplies lambda by 2, 4, 8, 16, 32; the
    first rejection after an accepted trial multiplies it by 2 again."""
    sc = _hard_start(seed)
    px = observed_pixels(sc)
    st0 = camera.State.from_bal(sc.cams_init, sc.points_init)
    res = lm.solve(st0, sc.obs_cam, sc.obs_pt, px, lm.LMOptions(max_iters=len(pattern), lambda0=lambda0))
    got = "".join("A" if h.accepted else "r" for h in res.history)
    assert got == pattern
    factors = [nxt.lam / h.lam for h, nxt in zip(res.history, res.history[1:])]
    run = 0
    for h, f in zip(res.history, factors):
        if h.accepted:
            run = 0
            assert 1.0 / 3.0 - 1e-15 <= f < 2.0
        else:
            assert f == [2.0, 4.0, 8.0, 16.0, 32.0][run]
            run += 1
        # a decisive decision: far from the threshold rho = 0
        assert abs(h.rho) > 1e-2
