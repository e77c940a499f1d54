"""Robust losses (Huber, Cauchy) on the GPU against the oracle
(oracle/robust.py): the IRLS-scaled linearisation, the weighted
normal-equation product, full LM solves against the oracle's stored results
on the tiny scene with 5% planted 40 px outliers, the float32-mixed form,
and the adjoint with the weights held fixed."""
import json
import os

import numpy as np
import pytest
import torch

from oracle import adjoint, camera, linear, robust
from synth import scene_config

from gpu_helpers import handle_for, observed_pixels, rel, t64

pytestmark = pytest.mark.gpu

GOLDEN = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "lm_reference.json")))["runs"]
SCALE = 3.0


@pytest.fixture(scope="module")
def scene():
    sc = scene_config("tiny_outliers")
    return sc, observed_pixels(sc)


@pytest.mark.parametrize("rj", [False, True], ids=["stored", "recompute"])
@pytest.mark.parametrize("kind", ["huber", "cauchy"])
def test_linearize_and_product_match_oracle(scene, kind, rj):
    sc, px = scene
    ba = handle_for(sc, px, 0, rj=rj)
    ba.set_loss(kind, SCALE)
    out = ba.linearize()
    st = camera.State.from_bal(sc.cams_init, sc.points_init)
    F, r, Jc, Jp, w = robust.linearize(st, sc.obs_cam, sc.obs_pt, px, kind, SCALE)
    assert 0.0 < w.min() < 1.0                       # some observations are down-weighted
    J = linear.jacobian_csr(Jc, Jp, sc.obs_cam, sc.obs_pt, st.n_cams, st.n_points)
    D = linear.damping_diagonal(J)
    assert abs(out["cost"] - F) <= 1e-12 * F
    assert rel(out["resid"].cpu(), r) <= 1e-11
    assert rel(out["jac_cam"].cpu(), Jc) <= 1e-12
    assert rel(out["jac_pt"].cpu(), Jp) <= 1e-12
    assert rel(out["grad"].cpu(), linear.gradient(J, r.ravel())) <= 1e-12
    assert rel(out["diag"].cpu(), D) <= 1e-12
    assert abs(ba.cost_fp64() - F) <= 1e-12 * F
    rng = np.random.default_rng(3)
    for lam in (1e-6, 1e-2, 1e2):
        p = rng.normal(size=st.n_params)
        wv, pap = ba.matvec(lam, t64(p))
        ref = linear.matvec(J, D, lam, p)
        assert rel(wv.cpu(), ref) <= 1e-12
        assert abs(pap - p @ ref) <= 1e-12 * abs(p @ ref)


@pytest.mark.parametrize("rj", [False, True], ids=["stored", "recompute"])
@pytest.mark.parametrize("kind", ["huber", "cauchy"])
def test_fp32_mixed_weighted_product_matches_oracle(scene, kind, rj):
    """The weighted product in the float32-mixed form, whose IRLS weights the
    recomputed-block product reads from its step-ordered copy: a wrong or
    stale weight changes J^T W J p directly (a solve could still converge to
    the same optimum by other steps).  Bar: float32 blocks and products, as
    for the unweighted mixed product."""
    sc, px = scene
    ba = handle_for(sc, px, 1, rj=rj)
    ba.set_loss(kind, SCALE)
    ba.linearize(outputs=False)
    st = camera.State.from_bal(sc.cams_init, sc.points_init)
    _, r, Jc, Jp, w = robust.linearize(st, sc.obs_cam, sc.obs_pt, px, kind, SCALE)
    J = linear.jacobian_csr(Jc, Jp, sc.obs_cam, sc.obs_pt, st.n_cams, st.n_points)
    D = linear.damping_diagonal(J)
    rng = np.random.default_rng(4)
    for lam in (1e-4, 1e-1):
        p = rng.normal(size=st.n_params)
        wv, pap = ba.matvec(lam, t64(p))
        ref = linear.matvec(J, D, lam, p)
        assert rel(wv.cpu(), ref) <= 2e-5
        assert abs(pap - p @ ref) <= 2e-5 * abs(p @ ref)


def _solve(name, precision=0, rj=False):
    from paper_2605_30583_amd import SolveOptions
    g = GOLDEN[name]
    sc = scene_config(g["scene"])
    px = observed_pixels(sc)
    ba = handle_for(sc, px, precision, rj=rj)
    ba.set_loss(g["loss"], g["loss_scale"])
    st = ba.solve(SolveOptions(max_lm_iters=g["max_iters"], pcg_tol=1e-6), history=True)
    return sc, px, ba, st, g


@pytest.mark.parametrize("rj", [False, True], ids=["stored", "recompute"])
@pytest.mark.parametrize("name", ["tiny_outliers_huber", "tiny_outliers_cauchy"])
def test_fp64_robust_solve_matches_oracle(name, rj):
    sc, px, ba, st, g = _solve(name, rj=rj)
    assert abs(st["initial_cost"] - g["initial_cost"]) <= 1e-12 * g["initial_cost"]
    assert abs(st["final_cost"] - g["final_cost"]) <= 1e-9 * g["final_cost"], (st["final_cost"], g["final_cost"])
    costs = [st["initial_cost"]] + [h["cost"] for h in st["history"]]
    assert all(b <= a for a, b in zip(costs, costs[1:]))
    # the reported cost is the robust cost of the returned parameters
    cams, pts = ba.get_params()
    st_o = camera.State.from_bal(cams.cpu().numpy(), pts.cpu().numpy())
    F = robust.cost(st_o, sc.obs_cam, sc.obs_pt, px, g["loss"], g["loss_scale"])
    assert abs(F - st["final_cost"]) <= 1e-10 * st["final_cost"]


@pytest.mark.parametrize("rj", [False, True], ids=["stored", "recompute"])
@pytest.mark.parametrize("name", ["tiny_outliers_huber", "tiny_outliers_cauchy"])
def test_fp32_mixed_robust_solve_error_is_small(name, rj):
    sc, px, ba, st, g = _solve(name, precision=1, rj=rj)
    f64 = ba.cost_fp64()
    err = (f64 - g["final_cost"]) / g["final_cost"]
    print(f"{name}: float32-mixed final robust cost {f64:.10e}, oracle {g['final_cost']:.10e}, rel error {err:.3e}")
    assert -1e-9 <= err <= 1e-6


@pytest.mark.parametrize("rj", [False, True], ids=["stored", "recompute"])
@pytest.mark.parametrize("kind", ["huber", "cauchy"])
def test_robust_adjoint_matches_oracle(kind, rj):
    from paper_2605_30583_amd import SolveOptions
    sc = scene_config("tiny_outliers")
    px = observed_pixels(sc)
    ba = handle_for(sc, px, 0, rj=rj)
    ba.set_loss(kind, SCALE)
    ba.solve(SolveOptions(max_lm_iters=20, pcg_tol=1e-10))
    cams, pts = ba.get_params()
    st = camera.State.from_bal(cams.cpu().numpy(), pts.cpu().numpy())
    lam = 1e-4
    g_theta = adjoint.point_norm_loss_grad(st)
    ref = adjoint.implicit_grad_obs(st, sc.obs_cam, sc.obs_pt, px, g_theta, lam, loss=kind, loss_scale=SCALE)
    out = ba.backward(None, 2.0 * pts, lambda_adj=lam, pcg_tol=1e-12, max_pcg_iters=5000).cpu().numpy()
    assert rel(out, ref) <= 1e-6


def test_trivial_loss_is_the_plain_problem_and_bad_losses_are_rejected():
    from paper_2605_30583_amd._native import CasparError
    sc = scene_config("tiny")
    px = observed_pixels(sc)
    a = handle_for(sc, px, 0)
    b = handle_for(sc, px, 0)
    b.set_loss("huber", SCALE)
    b.set_loss("trivial", 1.0)
    la, lb = a.linearize(), b.linearize()
    assert la["cost"] == lb["cost"]
    assert torch.equal(la["grad"], lb["grad"])
    with pytest.raises(CasparError):
        b.set_loss("huber", 0.0)
    with pytest.raises(CasparError):
        b.set_loss("cauchy", float("nan"))
    with pytest.raises(ValueError):
        b.set_loss("tukey", 1.0)
    assert b._lib.caspar_ba_set_loss(b._h, 7, 1.0) != 0     # unknown kind: an error status


@pytest.mark.parametrize("rj", [False, True], ids=["stored", "recompute"])
def test_huber_loss_with_between_factors(scene, rj):
    """Both widening rows at once: the Huber loss on the reprojection factors
    beside pose between-factors (which it leaves unweighted).  Linearisation
    and products against the oracle's stacked system; after a short solve the
    reported cost is the oracle's objective at the returned parameters."""
    from oracle import lm
    from helpers import between_factors
    from paper_2605_30583_amd import SolveOptions
    sc, px = scene
    bf = between_factors(sc, seed=21, n_loops=4)
    ba = handle_for(sc, px, 0, rj=rj)
    ba.set_loss("huber", SCALE)
    ba.set_between(*bf)
    out = ba.linearize()
    st = camera.State.from_bal(sc.cams_init, sc.points_init)
    F, J, g, D = lm._linearize(st, sc.obs_cam, sc.obs_pt, px, "huber", SCALE, bf)
    assert abs(out["cost"] - F) <= 1e-12 * F
    assert rel(out["grad"].cpu(), g) <= 1e-12
    assert rel(out["diag"].cpu(), D) <= 1e-12
    rng = np.random.default_rng(5)
    for lam in (1e-6, 1e-2, 1e2):
        p = rng.normal(size=st.n_params)
        wv, pap = ba.matvec(lam, t64(p))
        ref = linear.matvec(J, D, lam, p)
        assert rel(wv.cpu(), ref) <= 1e-12
        assert abs(pap - p @ ref) <= 1e-12 * abs(p @ ref)
    stats = ba.solve(SolveOptions(max_lm_iters=10, pcg_tol=1e-10, max_pcg_iters=2000))
    assert stats["final_cost"] < stats["initial_cost"]
    cams, pts = ba.get_params()
    st1 = camera.State.from_bal(cams.cpu().numpy(), pts.cpu().numpy())
    opts = lm.LMOptions(loss="huber", loss_scale=SCALE, between=bf)
    F1 = lm.total_cost(st1, sc.obs_cam, sc.obs_pt, px, opts)
    assert abs(stats["final_cost"] - F1) <= 1e-10 * F1, (stats["final_cost"], F1)
