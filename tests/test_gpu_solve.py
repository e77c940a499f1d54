"""Full Levenberg-Marquardt solves on the GPU against the oracle's stored
results (tests/golden/lm_reference.json, written by make_golden.py from the
oracle only), the float32-mixed form, and the implicit adjoint."""
import json
import os

import numpy as np
import pytest
import torch

from oracle import adjoint, camera
from synth import scene_config

from gpu_helpers import handle_for, observed_pixels, rel, t32i, t64

pytestmark = pytest.mark.gpu

GOLDEN = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "lm_reference.json")))["runs"]


def _solve(name, precision=0, tol=1e-6, rj=False):
    from paper_2605_30583_amd import SolveOptions
    sc = scene_config(name)
    px = observed_pixels(sc)
    ba = handle_for(sc, px, precision, rj=rj)
    stats = ba.solve(SolveOptions(max_lm_iters=GOLDEN[name]["max_iters"], pcg_tol=tol), history=True)
    return sc, px, ba, stats


@pytest.mark.parametrize("rj", [False, True], ids=["stored", "recompute"])
@pytest.mark.parametrize("name", ["tiny", "medium", "bal1700"])
def test_fp64_final_cost_matches_oracle(name, rj):
    sc, px, ba, st = _solve(name, rj=rj)
    g = GOLDEN[name]
    assert abs(st["initial_cost"] - g["initial_cost"]) <= 1e-12 * g["initial_cost"]
    assert abs(st["final_cost"] - g["final_cost"]) <= 1e-9 * g["final_cost"], (st["final_cost"], g["final_cost"])
    # accepted costs never increase
    costs = [st["initial_cost"]] + [h["cost"] for h in st["history"]]
    assert all(b <= a for a, b in zip(costs, costs[1:]))
    # the gauge-invariant predicted pixels agree
    cams, pts = ba.get_params()
    from paper_2605_30583_amd import project
    u = project(cams, pts, t32i(sc.obs_cam[:64]), t32i(sc.obs_pt[:64])).cpu().numpy()
    assert rel(u, np.array(g["predicted_pixels_sample"])) <= 1e-6
    # the reported cost is the cost of the returned parameters
    st_o = camera.State.from_bal(cams.cpu().numpy(), pts.cpu().numpy())
    assert abs(camera.cost(st_o, sc.obs_cam, sc.obs_pt, px) - st["final_cost"]) <= 1e-10 * st["final_cost"]


@pytest.mark.parametrize("rj", [False, True], ids=["stored", "recompute"])
@pytest.mark.parametrize("name", ["tiny", "bal1700"])
def test_fp32_mixed_final_cost_error_is_small(name, rj):
    sc, px, ba, st = _solve(name, precision=1, rj=rj)
    f64 = ba.cost_fp64()
    g = GOLDEN[name]["final_cost"]
    # stated, not a parity claim: the mixed form, re-evaluated in float64,
    # lands within 1e-6 of the oracle's float64 optimum and never below it
    # by more than rounding
    err = (f64 - g) / g
    print(f"{name}: float32-mixed final cost {f64:.10e}, oracle {g:.10e}, relative error {err:.3e}")
    assert err <= 1e-6
    assert err >= -1e-9


def test_warm_restart_continues_from_set_params():
    from paper_2605_30583_amd import SolveOptions
    sc = scene_config("tiny")
    px = observed_pixels(sc)
    a = handle_for(sc, px)
    s1 = a.solve(SolveOptions(max_lm_iters=4, pcg_tol=1e-6))
    cams, pts = a.get_params()
    b = handle_for(sc, px, cams=cams.cpu().numpy(), points=pts.cpu().numpy())
    assert abs(b.linearize(outputs=False)["cost"] - s1["final_cost"]) <= 1e-10 * s1["final_cost"]
    s2 = b.solve(SolveOptions(max_lm_iters=16, pcg_tol=1e-6, lambda0=s1["final_lambda"]))
    assert abs(s2["final_cost"] - GOLDEN["tiny"]["final_cost"]) <= 1e-9 * GOLDEN["tiny"]["final_cost"]


@pytest.mark.parametrize("rj", [False, True], ids=["stored", "recompute"])
def test_adjoint_matches_oracle_implicit_gradient(rj):
    sc, px, ba, st = _solve("tiny", rj=rj)
    cams, pts = ba.get_params()
    state = camera.State.from_bal(cams.cpu().numpy(), pts.cpu().numpy())
    g = adjoint.point_norm_loss_grad(state)
    lam = 1e-4
    ref = adjoint.implicit_grad_obs(state, sc.obs_cam, sc.obs_pt, px, g, lam, "schur")
    out = ba.backward(None, 2.0 * pts, lambda_adj=lam, pcg_tol=1e-12, max_pcg_iters=5000).cpu().numpy()
    assert rel(out, ref) <= 1e-6


def test_adjoint_camera_gradient_uses_the_angle_axis_chain_rule():
    # gradient given w.r.t. the BAL angle-axis vector; the tangent gradient is
    # built here from central differences of Log(Exp(w) Exp(d)) with scipy
    from scipy.spatial.transform import Rotation
    sc, px, ba, st = _solve("tiny")
    cams, pts = ba.get_params()
    cams_np = cams.cpu().numpy()
    state = camera.State.from_bal(cams_np, pts.cpu().numpy())
    rng = np.random.default_rng(3)
    g_aa = rng.normal(size=(sc.n_cams, 9))
    g_tan = g_aa.copy()
    h = 1e-6
    for c in range(sc.n_cams):
        R0 = Rotation.from_rotvec(cams_np[c, :3])
        Jd = np.empty((3, 3))
        for k in range(3):
            e = np.zeros(3)
            e[k] = h
            wp = (R0 * Rotation.from_rotvec(e)).as_rotvec()
            wm = (R0 * Rotation.from_rotvec(-e)).as_rotvec()
            Jd[:, k] = (wp - wm) / (2 * h)
        g_tan[c, :3] = Jd.T @ g_aa[c, :3]
    g = np.concatenate([g_tan.ravel(), np.zeros(3 * sc.n_points)])
    lam = 1e-4
    ref = adjoint.implicit_grad_obs(state, sc.obs_cam, sc.obs_pt, px, g, lam, "schur")
    out = ba.backward(t64(g_aa), None, lambda_adj=lam, pcg_tol=1e-12, max_pcg_iters=5000).cpu().numpy()
    assert rel(out, ref) <= 1e-6


def test_autograd_function_backward():
    from paper_2605_30583_amd import BAFunction, SolveOptions
    sc = scene_config("tiny")
    px = t64(observed_pixels(sc)).requires_grad_(True)
    cams, pts = BAFunction.apply(px, t64(sc.cams_init), t64(sc.points_init), t32i(sc.obs_cam), t32i(sc.obs_pt),
                                 SolveOptions(max_lm_iters=20, pcg_tol=1e-6), 0, 1e-4, 1e-12, 5000)
    loss = (pts * pts).sum()
    loss.backward()
    state = camera.State.from_bal(cams.detach().cpu().numpy(), pts.detach().cpu().numpy())
    ref = adjoint.implicit_grad_obs(state, sc.obs_cam, sc.obs_pt, px.detach().cpu().numpy(),
                                    adjoint.point_norm_loss_grad(state), 1e-4, "schur")
    assert rel(px.grad.cpu().numpy(), ref) <= 1e-6


def test_autograd_function_second_backward_of_a_retained_graph():
    from paper_2605_30583_amd import BAFunction, SolveOptions
    sc = scene_config("tiny")
    px = t64(observed_pixels(sc)).requires_grad_(True)
    cams, pts = BAFunction.apply(px, t64(sc.cams_init), t64(sc.points_init), t32i(sc.obs_cam), t32i(sc.obs_pt),
                                 SolveOptions(max_lm_iters=20, pcg_tol=1e-6), 0, 1e-4, 1e-12, 5000)
    loss = (pts * pts).sum()
    loss.backward(retain_graph=True)
    first = px.grad.clone()
    loss.backward()
    assert rel(px.grad.cpu().numpy(), 2.0 * first.cpu().numpy()) <= 1e-12


def test_backward_reports_an_unconverged_adjoint_solve():
    sc, px, ba, st = _solve("tiny")
    _, pts = ba.get_params()
    with pytest.warns(RuntimeWarning, match="adjoint PCG stopped"):
        ba.backward(None, 2.0 * pts, lambda_adj=1e-4, pcg_tol=1e-12, max_pcg_iters=2)
    assert ba.last_backward_iters == 2
    assert ba.last_backward_rel_resid > 1e-12
    ba.backward(None, 2.0 * pts, lambda_adj=1e-4, pcg_tol=1e-12, max_pcg_iters=5000)
    assert ba.last_backward_rel_resid <= 1e-12
