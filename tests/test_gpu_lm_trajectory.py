"""The GPU's Levenberg-Marquardt trajectory against the oracle's, iteration
by iteration (Section V: gain ratio and the quality-based damping update
after Madsen and Nielsen).

For every run stored in tests/golden/lm_reference.json (written by
make_golden.py from the oracle only, with exact Schur-complement steps) the
GPU solves the same problem with PCG at tolerance 1e-10, so its steps are
the exact ones up to that tolerance, and records each iteration.  Every
iteration whose predicted decrease the cost can resolve (pred > 1e-10 F;
below that the gain ratio is rounding noise and accepting or rejecting is
chance) must take the same decision with the same damping: the accept flag
exactly, lambda, pred, rho and the cost to the tolerances below.  The runs
cover the converging problems (lambda / 3 on every good step), the robust
losses and the between-factors, and two hard starts whose first trials are
rejected (lambda x2, x4, ... and the reset of nu on the next accepted step)."""
import json
import math
import os

import pytest

from synth import scene_config

from gpu_helpers import handle_for, observed_pixels
from helpers import between_factors

pytestmark = pytest.mark.gpu

GOLDEN = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "lm_reference.json")))["runs"]

RUNS = ["tiny", "medium", "bal1700", "tiny_outliers_huber", "tiny_outliers_cauchy", "tiny_between",
        "hard_start_a", "hard_start_b"]


def _gpu_history(name, rj):
    from paper_2605_30583_amd import SolveOptions
    g = GOLDEN[name]
    sc = scene_config(g["scene"])
    px = observed_pixels(sc)
    ba = handle_for(sc, px, 0, rj=rj)
    if g["loss"] != "trivial":
        ba.set_loss(g["loss"], g["loss_scale"])
    if g["between"]:
        seed, loops, rs, ts = g["between"]
        ba.set_between(*between_factors(sc, seed=seed, n_loops=loops, rot_sigma=rs, trans_sigma=ts))
    st = ba.solve(SolveOptions(max_lm_iters=g["max_iters"], pcg_tol=1e-10, max_pcg_iters=5000,
                               lambda0=g["lambda0"]), history=True)
    ba.close()
    return st, g


@pytest.mark.parametrize("rj", [False, True], ids=["stored", "recompute"])
@pytest.mark.parametrize("name", RUNS)
def test_lm_trajectory_matches_oracle(name, rj):
    """Bars, per compared iteration (F: the cost it starts from):
    pred to 1e-6 (the GPU's step is the exact one to PCG tolerance 1e-10);
    rho to 1e-6 max(1, |rho|) plus 2e-12 F / pred, since rho divides the
    difference of two costs, each summed to about 1e-12 of F in another order
    (the initial costs are checked at that bar);
    the cost after the iteration to 1e-9 of it plus what those two bars allow
    in F - rho pred: (|d rho| + 1e-6 |rho|) pred;
    lambda to the error the update can carry forward: the factor
    max(1/3, 1 - (2 rho - 1)^3) has slope at most 6 and value at least 1/3,
    so each accepted step with rho < 1 adds 18 |d rho| of relative error,
    and rejections (lambda * nu) add none."""
    st, g = _gpu_history(name, rj)
    hist = st["history"]
    F = g["initial_cost"]
    assert abs(st["initial_cost"] - F) <= 1e-12 * F
    compared = 0
    lam_err = 1e-12
    for i, h in enumerate(hist):
        if i >= len(g["preds"]) or g["preds"][i] <= 1e-10 * F:
            break
        where = f"{name} iteration {i}"
        pred_o, rho_o, cost_o = g["preds"][i], g["rhos"][i], g["costs"][i]
        assert bool(h["accepted"]) == g["accepted"][i], where
        assert abs(h["lam"] - g["lambdas"][i]) <= lam_err * g["lambdas"][i], (where, h["lam"], g["lambdas"][i])
        assert abs(h["pred"] - pred_o) <= 1e-6 * pred_o, (where, h["pred"], pred_o)
        assert math.isfinite(h["rho"]) == math.isfinite(rho_o), where
        d_rho = 0.0
        if math.isfinite(rho_o):
            d_rho = 1e-6 * max(1.0, abs(rho_o)) + 2e-12 * F / pred_o
            assert abs(h["rho"] - rho_o) <= d_rho, (where, h["rho"], rho_o, d_rho)
            if g["accepted"][i] and rho_o < 1.0:
                lam_err += 18.0 * d_rho
        d_cost = 1e-9 * cost_o + (d_rho + 1e-6 * abs(rho_o if math.isfinite(rho_o) else 0.0)) * pred_o
        assert abs(h["cost"] - cost_o) <= d_cost, (where, h["cost"], cost_o, d_cost)
        F = cost_o
        compared += 1
    # every run resolves several iterations; the hard starts include their
    # rejections
    assert compared >= 3
    if name.startswith("hard_start"):
        assert not all(g["accepted"][:compared])
