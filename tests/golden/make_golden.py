"""Writes tests/golden/lm_reference.json: the oracle's Levenberg-Marquardt
results on the synthetic workloads (plain least squares, the robust losses
on the tiny scene with planted outliers, and the tiny scene with pose
between-factors: a camera chain plus four loop closures).

Calls only synth/ and oracle/ (exact Schur-complement steps, float64).
Run from the repository root:
    python tests/golden/make_golden.py [workload ...]
(default: all; named workloads are recomputed and merged into the file).
"""
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

from oracle import between, camera, lm  # noqa: E402
from synth import between_draws, scene_config  # noqa: E402

# run name -> (scene, LM iterations, loss, loss scale in pixels, between-factors, lambda0)
# between-factors: (draw seed, loop closures, rotation sigma, translation sigma)
BETWEEN = (21, 4, 2e-3, 1e-2)
RUNS = {
    "tiny": ("tiny", 20, "trivial", 1.0, None, 1e-2),
    "medium": ("medium", 30, "trivial", 1.0, None, 1e-2),
    "bal1700": ("bal1700", 20, "trivial", 1.0, None, 1e-2),
    "tiny_outliers_huber": ("tiny_outliers", 40, "huber", 3.0, None, 1e-2),
    "tiny_outliers_cauchy": ("tiny_outliers", 40, "cauchy", 3.0, None, 1e-2),
    "tiny_between": ("tiny", 20, "trivial", 1.0, BETWEEN, 1e-2),
    # runs with rejected trials: the damping rule's growth and reset
    "hard_start_a": ("hard_start_a", 12, "trivial", 1.0, None, 1e-3),
    "hard_start_b": ("hard_start_b", 12, "trivial", 1.0, None, 1e-2),
}


def between_for(sc, spec):
    seed, loops, rs, ts = spec
    d = between_draws(sc.n_cams, seed, loops)
    st_true = camera.State.from_bal(sc.cams_true, sc.points_true)
    Z, w = between.measurements(st_true, d.fi, d.fj, d.rot_noise, d.trans_noise, rs, ts)
    return d.fi, d.fj, Z, w


def main():
    path = os.path.join(ROOT, "tests", "golden", "lm_reference.json")
    out = {"source": "oracle.lm.solve with exact Schur-complement steps (float64); lambda0 per run; "
                     "observed pixels = oracle.camera.project(true parameters) + the scene's noise",
           "runs": {}}
    if os.path.exists(path):
        out["runs"] = json.load(open(path))["runs"]
    names = sys.argv[1:] or list(RUNS)
    for name in names:
        scene, iters, loss, scale, bspec, lam0 = RUNS[name]
        sc = scene_config(scene)
        st_true = camera.State.from_bal(sc.cams_true, sc.points_true)
        px = camera.project(st_true, sc.obs_cam, sc.obs_pt) + sc.noise
        st = camera.State.from_bal(sc.cams_init, sc.points_init)
        t = time.time()
        bf = between_for(sc, bspec) if bspec else None
        res = lm.solve(st, sc.obs_cam, sc.obs_pt, px,
                       lm.LMOptions(max_iters=iters, inner="schur", loss=loss, loss_scale=scale, between=bf,
                                    lambda0=lam0))
        out["runs"][name] = {
            "scene": scene,
            "loss": loss,
            "loss_scale": scale,
            "max_iters": iters,
            "between": list(bspec) if bspec else None,
            "lambda0": lam0,
            "initial_cost": res.initial_cost,
            "final_cost": res.final_cost,
            "stop_reason": res.stop_reason,
            "accepted": [bool(h.accepted) for h in res.history],
            "costs": [h.cost for h in res.history],
            "lambdas": [h.lam for h in res.history],
            "preds": [h.pred for h in res.history],
            "rhos": [h.rho for h in res.history],
            "trial_costs": [h.trial_cost for h in res.history],
            "predicted_pixels_sample": camera.project(res.state, sc.obs_cam[:64], sc.obs_pt[:64]).tolist(),
            "oracle_seconds": time.time() - t,
        }
        print(name, res.initial_cost, res.final_cost, f"{time.time() - t:.1f}s", flush=True)
    json.dump(out, open(path, "w"), indent=1)
    print("wrote", path)


if __name__ == "__main__":
    main()
