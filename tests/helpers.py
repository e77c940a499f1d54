"""Shared test helpers: observed pixels for a synthetic scene, formed with the
oracle's projection (tests may call the oracle)."""
import numpy as np

from oracle import between, camera
from synth import between_draws, make_scene


def observed_pixels(scene, noise_scale=1.0):
    st = camera.State.from_bal(scene.cams_true, scene.points_true)
    return camera.project(st, scene.obs_cam, scene.obs_pt) + noise_scale * scene.noise


def small_scene(n_cams=4, n_points=30, seed=7, k=3, **kw):
    return make_scene(n_cams, n_points, seed, k_values=(k,), k_probs=(1.0,), **kw)


def between_factors(scene, seed=21, n_loops=0, rot_sigma=2e-3, trans_sigma=1e-2, noise=True):
    """Pose between-factors for a scene: pairs and noise draws from synth,
    measurements from the true poses by the oracle (noise=False: exact
    measurements, same weights).  Returns (fi, fj, Z [n, 6], w [n, 2])."""
    d = between_draws(scene.n_cams, seed, n_loops)
    st = camera.State.from_bal(scene.cams_true, scene.points_true)
    k = 1.0 if noise else 0.0
    Z, w = between.measurements(st, d.fi, d.fj, k * d.rot_noise, k * d.trans_noise, rot_sigma, trans_sigma)
    return d.fi, d.fj, Z, w
