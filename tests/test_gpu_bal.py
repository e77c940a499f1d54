"""A problem read from a BAL file by the native reader solves on the GPU to
the oracle's stored result (tiny scene, float64, 20 LM iterations)."""
import json
import os

import numpy as np
import pytest
import torch

from oracle import bal as obal
from oracle import camera
from synth import scene_config

pytestmark = pytest.mark.gpu

GOLDEN = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "lm_reference.json")))["runs"]


def test_solve_from_a_bal_file_matches_the_oracle(tmp_path):
    from paper_2605_30583_amd import FP64, BundleAdjuster, SolveOptions, read_bal
    sc = scene_config("tiny")
    st_true = camera.State.from_bal(sc.cams_true, sc.points_true)
    px = camera.project(st_true, sc.obs_cam, sc.obs_pt) + sc.noise
    path = tmp_path / "tiny.bal"
    obal.write(path, sc.cams_init, sc.points_init, sc.obs_cam, sc.obs_pt, px)
    p = read_bal(path)
    dev = torch.device("cuda:0")
    t = {k: torch.from_numpy(v).to(dev) for k, v in p.items()}
    ba = BundleAdjuster(t["cams"], t["points"], t["obs_cam"], t["obs_pt"], t["px"], FP64)
    g = GOLDEN["tiny"]
    st = ba.solve(SolveOptions(max_lm_iters=g["max_iters"], pcg_tol=1e-6))
    assert abs(st["initial_cost"] - g["initial_cost"]) <= 1e-12 * g["initial_cost"]
    assert abs(st["final_cost"] - g["final_cost"]) <= 1e-9 * g["final_cost"]
    ba.close()
