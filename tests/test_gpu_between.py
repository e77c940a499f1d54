"""Pose between-factors on the GPU against the oracle (oracle/between.py and
the between-aware LM and adjoint oracles): the linearisation (cost, gradient,
damping diagonal), the product and block-Jacobi with the factors, full LM
solves against the stored oracle run (tiny scene, camera chain plus four loop
closures), the float32-mixed form, the adjoint, and the argument checks."""
import json
import os

import numpy as np
import pytest
import torch

from oracle import adjoint, between, camera, lm, linear
from synth import scene_config

from gpu_helpers import handle_for, rel, t64
from helpers import between_factors, observed_pixels

pytestmark = pytest.mark.gpu

GOLDEN = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "lm_reference.json")))["runs"]


@pytest.fixture(scope="module")
def scene():
    sc = scene_config("tiny")
    px = observed_pixels(sc)
    bf = between_factors(sc, seed=21, n_loops=4)
    return sc, px, bf


def _oracle_system(sc, px, bf, cams=None):
    st = camera.State.from_bal(sc.cams_init if cams is None else cams, sc.points_init)
    F, J, g, D = lm._linearize(st, sc.obs_cam, sc.obs_pt, px, between=bf)
    return st, F, J, g, D


@pytest.mark.parametrize("rj", [False, True], ids=["stored", "recompute"])
def test_linearize_product_and_preconditioner_match_oracle(scene, rj):
    sc, px, bf = scene
    ba = handle_for(sc, px, 0, rj=rj)
    ba.set_between(*bf)
    out = ba.linearize()
    st, F, J, g, D = _oracle_system(sc, px, bf)
    assert abs(out["cost"] - F) <= 1e-12 * F
    assert rel(out["grad"].cpu(), g) <= 1e-12
    assert rel(out["diag"].cpu(), D) <= 1e-12
    assert abs(ba.cost_fp64() - F) <= 1e-12 * F
    rng = np.random.default_rng(3)
    for lam in (1e-6, 1e-2, 1e2):
        p = rng.normal(size=st.n_params)
        w, pap = ba.matvec(lam, t64(p))
        ref = linear.matvec(J, D, lam, p)
        assert rel(w.cpu(), ref) <= 1e-12
        assert abs(pap - p @ ref) <= 1e-12 * abs(p @ ref)
        r = rng.normal(size=st.n_params)
        Mc, Mp = linear.block_jacobi_inverse(J, D, lam, st.n_cams, st.n_points)
        z = ba.block_jacobi_apply(lam, t64(r))
        assert rel(z.cpu(), linear.apply_block_jacobi(Mc, Mp, r)) <= 1e-10


@pytest.mark.parametrize("rj", [False, True], ids=["stored", "recompute"])
def test_fp64_solve_matches_oracle(scene, rj):
    from paper_2605_30583_amd import SolveOptions
    sc, px, bf = scene
    g = GOLDEN["tiny_between"]
    assert tuple(g["between"]) == (21, 4, 2e-3, 1e-2)
    ba = handle_for(sc, px, 0, rj=rj)
    ba.set_between(*bf)
    st = ba.solve(SolveOptions(max_lm_iters=g["max_iters"], pcg_tol=1e-6), history=True)
    assert abs(st["initial_cost"] - g["initial_cost"]) <= 1e-12 * g["initial_cost"]
    assert abs(st["final_cost"] - g["final_cost"]) <= 1e-9 * g["final_cost"], (st["final_cost"], g["final_cost"])
    costs = [st["initial_cost"]] + [h["cost"] for h in st["history"]]
    assert all(b <= a for a, b in zip(costs, costs[1:]))
    cams, pts = ba.get_params()
    stg = camera.State.from_bal(cams.cpu().numpy(), pts.cpu().numpy())
    F = camera.cost(stg, sc.obs_cam, sc.obs_pt, px) + between.cost(stg, *bf)
    assert abs(F - st["final_cost"]) <= 1e-10 * F


@pytest.mark.parametrize("rj", [False, True], ids=["stored", "recompute"])
def test_fp32_mixed_solve_error_is_small(scene, rj):
    from paper_2605_30583_amd import SolveOptions
    sc, px, bf = scene
    g = GOLDEN["tiny_between"]
    ba = handle_for(sc, px, 1, rj=rj)
    ba.set_between(*bf)
    ba.solve(SolveOptions(max_lm_iters=40, pcg_tol=1e-6))
    err = (ba.cost_fp64() - g["final_cost"]) / g["final_cost"]
    print(f"float32-mixed with between-factors: rel cost error {err:.3e}")
    assert -1e-9 <= err <= 1e-6


@pytest.mark.parametrize("rj", [False, True], ids=["stored", "recompute"])
def test_adjoint_matches_oracle(scene, rj):
    from paper_2605_30583_amd import SolveOptions
    sc, px, bf = scene
    ba = handle_for(sc, px, 0, rj=rj)
    ba.set_between(*bf)
    ba.solve(SolveOptions(max_lm_iters=20, pcg_tol=1e-10))
    cams, pts = ba.get_params()
    st = camera.State.from_bal(cams.cpu().numpy(), pts.cpu().numpy())
    lam = 1e-4
    ref = adjoint.implicit_grad_obs(st, sc.obs_cam, sc.obs_pt, px, adjoint.point_norm_loss_grad(st), lam, between=bf)
    out = ba.backward(None, 2.0 * pts, lambda_adj=lam, pcg_tol=1e-12, max_pcg_iters=5000).cpu().numpy()
    assert rel(out, ref) <= 1e-6


def test_removing_the_factors_restores_the_plain_problem_and_bad_input_is_refused(scene):
    from paper_2605_30583_amd._native import CasparError
    sc, px, bf = scene
    a = handle_for(sc, px, 0)
    b = handle_for(sc, px, 0)
    b.set_between(*bf)
    assert b.linearize()["cost"] > a.linearize()["cost"]
    b.set_between(np.zeros(0, np.int32), np.zeros(0, np.int32), np.zeros((0, 6)), np.zeros((0, 2)))
    la, lb = a.linearize(), b.linearize()
    assert la["cost"] == lb["cost"] and torch.equal(la["grad"], lb["grad"])
    fi, fj, Z, w = bf
    with pytest.raises(CasparError, match="out of range"):
        b.set_between(fi, np.where(np.arange(len(fj)) == 2, sc.n_cams, fj), Z, w)
    with pytest.raises(CasparError, match="same"):
        b.set_between(fi, fi, Z, w)
    w_bad = w.copy()
    w_bad[1, 1] = 0.0
    with pytest.raises(CasparError, match="positive"):
        b.set_between(fi, fj, Z, w_bad)
    Z_bad = Z.copy()
    Z_bad[0, 0] = np.inf
    with pytest.raises(CasparError, match="non-finite"):
        b.set_between(fi, fj, Z_bad, w)
    b.set_between(fi, fj, Z, w)
    with pytest.raises(CasparError, match="gauge"):
        b.backward(None, torch.zeros((sc.n_points, 3), dtype=torch.float64, device="cuda"), gauge_project=True)


@pytest.mark.parametrize("precision,tol", [(0, 1e-12), (1, 3e-6)], ids=["fp64", "fp32_mixed"])
@pytest.mark.parametrize("rj", [False, True], ids=["stored", "recompute"])
def test_ragged_scene_with_factors_on_an_unobserved_camera(precision, tol, rj):
    """Ragged degrees, a point split across tiles, an orphan point, and a
    camera seen by no observation that only its between-factors tie down."""
    from gpu_helpers import ragged_scene
    sc = ragged_scene()
    px = observed_pixels(sc)
    nc = sc.n_cams
    fi = np.array([0, 5, 79, 80, 80, 12], np.int32)
    fj = np.array([1, 80, 3, 7, 44, 13], np.int32)
    st_true = camera.State.from_bal(sc.cams_true, sc.points_true)
    rng = np.random.default_rng(8)
    Z, w = between.measurements(st_true, fi, fj, rng.normal(size=(6, 3)), rng.normal(size=(6, 3)), 3e-3, 2e-2)
    assert nc == 81 and not np.any(sc.obs_cam == 80)
    bf = (fi, fj, Z, w)
    ba = handle_for(sc, px, precision, rj=rj)
    ba.set_between(*bf)
    out = ba.linearize()
    st, F, J, g, D = _oracle_system(sc, px, bf)
    assert abs(out["cost"] - F) <= tol * F
    assert rel(out["grad"].cpu(), g) <= 10 * tol
    assert rel(out["diag"].cpu(), D) <= 10 * tol
    p = rng.normal(size=st.n_params)
    lam = 1e-2
    wv, pap = ba.matvec(lam, t64(p))
    ref = linear.matvec(J, D, lam, p)
    assert rel(wv.cpu(), ref) <= 10 * tol
    assert abs(pap - p @ ref) <= 10 * tol * abs(p @ ref)
    cam80 = slice(9 * 80, 9 * 81)
    assert rel(wv.cpu()[cam80], ref[cam80]) <= 10 * tol        # the camera the factors alone hold
