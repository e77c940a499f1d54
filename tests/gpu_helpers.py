"""Helpers shared by the GPU tests: scenes, tensors, oracle references."""
import dataclasses

import numpy as np
import torch

from oracle import camera, linear
from synth import Scene, make_scene

from helpers import observed_pixels

DEV = "cuda"


def t64(a):
    return torch.tensor(np.ascontiguousarray(a), dtype=torch.float64, device=DEV)


def t32i(a):
    return torch.tensor(np.ascontiguousarray(a), dtype=torch.int32, device=DEV)


def ragged_scene(seed=13):
    """80 cameras, mixed 1..8 observations per point, plus one point seen by
    every camera (more than one wave tile), one point with no observation
    and one camera with no observation."""
    sc = make_scene(80, 400, seed, k_values=(1, 2, 3, 5, 8), k_probs=(0.2, 0.2, 0.2, 0.2, 0.2))
    rng = np.random.default_rng(seed + 1000)
    big = np.array([[0.4, -0.3, 0.2]])
    orphan = np.array([[1.0, 1.0, -1.0]])
    pts = np.concatenate([sc.points_true, big, orphan])
    cams = np.concatenate([sc.cams_true, sc.cams_true[3:4]])
    oc = np.concatenate([sc.obs_cam, np.arange(80, dtype=np.int32)])
    op = np.concatenate([sc.obs_pt, np.full(80, sc.n_points, dtype=np.int32)])
    noise = np.concatenate([sc.noise, rng.normal(0, 1, size=(80, 2))])
    cams0 = np.concatenate([sc.cams_init, sc.cams_init[3:4]])
    pts0 = np.concatenate([sc.points_init, big + rng.normal(0, 0.05, (1, 3)), orphan])
    return Scene(cams, pts, oc.astype(np.int32), op.astype(np.int32), noise, cams0, pts0)


def handle_for(sc, px, precision=0, cams=None, points=None, rj=False):
    from paper_2605_30583_amd import BundleAdjuster
    return BundleAdjuster(t64(sc.cams_init if cams is None else cams),
                          t64(sc.points_init if points is None else points),
                          t32i(sc.obs_cam), t32i(sc.obs_pt), t64(px), precision, recompute_jacobian=rj)


@dataclasses.dataclass
class OracleLin:
    state: camera.State
    r: np.ndarray
    Jc: np.ndarray
    Jp: np.ndarray
    J: object
    D: np.ndarray
    g: np.ndarray
    cost: float


def oracle_lin(sc, px, cams=None, points=None):
    st = camera.State.from_bal(sc.cams_init if cams is None else cams, sc.points_init if points is None else points)
    r, Jc, Jp = camera.linearize(st, sc.obs_cam, sc.obs_pt, px)
    J = linear.jacobian_csr(Jc, Jp, sc.obs_cam, sc.obs_pt, sc.n_cams, sc.n_points)
    return OracleLin(st, r, Jc, Jp, J, linear.damping_diagonal(J), linear.gradient(J, r.ravel()),
                     0.5 * float(np.sum(r * r)))


def rel(a, b):
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


__all__ = ["DEV", "t64", "t32i", "ragged_scene", "handle_for", "oracle_lin", "rel", "observed_pixels"]
