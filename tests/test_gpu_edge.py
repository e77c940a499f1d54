"""Degenerate and boundary cases of the GPU path against the oracle: PCG
with a zero right-hand side, with no iterations allowed and with exactly one
or two iterations; an LM solve allowed no iteration; a problem with a single
camera; and a pose graph with no points and no observations (between-factors
alone)."""
import json
import os

import numpy as np
import pytest
import torch

from oracle import between, camera, lm, linear, pcg as opcg
from synth import make_scene, scene_config

from gpu_helpers import handle_for, oracle_lin, rel, t64
from helpers import between_factors, observed_pixels

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def tiny():
    sc = scene_config("tiny")
    px = observed_pixels(sc)
    return sc, px, oracle_lin(sc, px)


@pytest.mark.parametrize("rj", [False, True], ids=["stored", "recompute"])
def test_pcg_zero_rhs_zero_cap_and_short_runs(tiny, rj):
    sc, px, ref = tiny
    ba = handle_for(sc, px, rj=rj)
    lam = 1e-2
    x, iters, _ = ba.pcg(lam, t64(np.zeros(ref.J.shape[1])), 1e-6, 500)
    assert iters == 0 and float(x.abs().max()) == 0.0
    b = -ref.g
    x, iters, _ = ba.pcg(lam, t64(b), 1e-6, 0)
    assert iters == 0 and float(x.abs().max()) == 0.0
    Mc, Mp = linear.block_jacobi_inverse(ref.J, ref.D, lam, sc.n_cams, sc.n_points)
    for cap in (1, 2, 5):
        x, iters, _ = ba.pcg(lam, t64(b), 1e-12, cap)
        xo, _, ko, why = opcg.pcg(ref.J, ref.D, lam, b, Mc, Mp, 1e-12, cap)
        assert why == "max_iter" and iters == ko == cap
        assert rel(x.cpu().numpy(), xo) <= 1e-11, cap


def test_solve_allowed_no_iteration(tiny):
    from paper_2605_30583_amd import SolveOptions
    sc, px, ref = tiny
    ba = handle_for(sc, px)
    st = ba.solve(SolveOptions(max_lm_iters=0))
    assert st["lm_iters"] == 0 and st["pcg_iters_total"] == 0
    assert st["final_cost"] == st["initial_cost"]
    assert abs(st["initial_cost"] - ref.cost) <= 1e-12 * ref.cost


@pytest.mark.parametrize("rj", [False, True], ids=["stored", "recompute"])
def test_single_camera_problem(rj):
    sc = make_scene(1, 64, 9, k_values=(1,), k_probs=(1.0,))
    px = observed_pixels(sc)
    ba = handle_for(sc, px, rj=rj)
    ref = oracle_lin(sc, px)
    out = ba.linearize()
    assert abs(out["cost"] - ref.cost) <= 1e-12 * ref.cost
    assert rel(out["grad"].cpu(), ref.g) <= 1e-12
    p = np.random.default_rng(2).normal(size=ref.J.shape[1])
    w, _ = ba.matvec(1e-2, t64(p))
    assert rel(w.cpu(), linear.matvec(ref.J, ref.D, 1e-2, p)) <= 1e-12


@pytest.mark.parametrize("precision", [0, 1], ids=["fp64", "fp32_mixed"])
def test_pose_graph_without_points(precision):
    """Sixteen cameras, no points, no observations: the solve minimises the
    between-factor cost alone, to the oracle's result."""
    from paper_2605_30583_amd import BundleAdjuster, SolveOptions
    sc = scene_config("tiny")
    fi, fj, Z, w = between_factors(sc, seed=21, n_loops=4)
    st0 = camera.State.from_bal(sc.cams_init, np.zeros((0, 3)))
    empty_i, empty_px = np.zeros(0, np.int32), np.zeros((0, 2))
    res = lm.solve(st0, empty_i, empty_i, empty_px, lm.LMOptions(max_iters=10, between=(fi, fj, Z, w)))
    dev = "cuda"
    ba = BundleAdjuster(t64(sc.cams_init), torch.zeros((0, 3), dtype=torch.float64, device=dev),
                        torch.zeros(0, dtype=torch.int32, device=dev), torch.zeros(0, dtype=torch.int32, device=dev),
                        torch.zeros((0, 2), dtype=torch.float64, device=dev), precision)
    ba.set_between(fi, fj, Z, w)
    st = ba.solve(SolveOptions(max_lm_iters=10, pcg_tol=1e-12, max_pcg_iters=2000))
    assert abs(st["initial_cost"] - res.initial_cost) <= 1e-12 * res.initial_cost
    tol = 1e-8 if precision == 0 else 1e-4
    assert abs(st["final_cost"] - res.final_cost) <= tol * res.final_cost, (st["final_cost"], res.final_cost)
    cams, _ = ba.get_params()
    stg = camera.State.from_bal(cams.cpu().numpy(), np.zeros((0, 3)))
    assert abs(between.cost(stg, fi, fj, Z, w) - st["final_cost"]) <= 1e-10 * st["final_cost"]


def test_product_timing_every_kth_launch(tiny):
    """Event timing of the fused product: with stride 1 every launch that did
    work is timed (one per PCG iteration); with stride 3 about a third of
    them; a negative stride is refused."""
    from paper_2605_30583_amd import SolveOptions
    sc, px, ref = tiny
    ba = handle_for(sc, px, rj=True)
    counts = {}
    for every in (1, 3):
        ba.set_params(t64(sc.cams_init), t64(sc.points_init))
        ba.set_timing(True, every=every)
        st = ba.solve(SolveOptions(max_lm_iters=5, pcg_tol=1e-6))
        tim = ba.get_timing()
        ba.set_timing(False)
        assert tim["matvec_ms"] > 0.0
        counts[every] = (tim["matvec_launches"], st["pcg_iters_total"], st["lm_iters"])
    n1, total1, _ = counts[1]
    assert n1 == total1
    n3, total3, lm3 = counts[3]
    assert abs(n3 - total3 / 3.0) <= lm3 + 1, counts
    with pytest.raises(Exception):
        ba.set_timing(True, every=-2)
