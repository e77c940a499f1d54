"""Shared test helpers: observed pixels for a synthetic scene, formed with the
oracle's projection (tests may call the oracle)."""
import numpy as np

from oracle import camera
from synth import make_scene


def observed_pixels(scene, noise_scale=1.0):
    st = camera.State.from_bal(scene.cams_true, scene.points_true)
    return camera.project(st, scene.obs_cam, scene.obs_pt) + noise_scale * scene.noise


def small_scene(n_cams=4, n_points=30, seed=7, k=3, **kw):
    return make_scene(n_cams, n_points, seed, k_values=(k,), k_probs=(1.0,), **kw)
