"""Robust losses on the squared residual norm and their IRLS weighting
(oracle).

The paper notes that the residual formulation makes weighting schemes and
robust loss functions easy to try (Section VI-A) and fixes none of them.
Reading taken here, for s_o = |r_o|^2 and a loss rho with scale c > 0:

  cost      F = 1/2 sum_o rho(s_o)
  weights   w_o = rho'(s_o), frozen at each linearisation (iteratively
            reweighted least squares)
  model     the residuals and Jacobian blocks of observation o are scaled by
            sqrt(w_o): with the scaled J~, r~ the normal equations are
            (J~^T J~ + lambda D~) delta = -J~^T r~, D~ = clamp(diag J~^T J~),
            and J~^T r~ = sum_o w_o J_o^T r_o is the exact gradient of F.

Losses:
  trivial   rho(s) = s
  huber     rho(s) = s                      for s <= c^2
                   = 2 c sqrt(s) - c^2      otherwise
  cauchy    rho(s) = c^2 log(1 + s / c^2)

Pins (tests/test_oracle_robust.py): rho' against central differences of
rho; the scaled gradient against central differences of the robust cost;
huber equal to the plain problem when every residual lies inside the scale;
cauchy approaching the plain cost as the scale grows; with gross outliers
planted, the robust optimum stays near the true parameters while the plain
one moves away.
"""
from __future__ import annotations

import numpy as np

from . import camera

LOSSES = ("trivial", "huber", "cauchy")


def rho(kind: str, s: np.ndarray, c: float) -> np.ndarray:
    s = np.asarray(s, dtype=np.float64)
    if kind == "trivial":
        return s.copy()
    if kind == "huber":
        return np.where(s <= c * c, s, 2.0 * c * np.sqrt(s) - c * c)
    if kind == "cauchy":
        return c * c * np.log1p(s / (c * c))
    raise ValueError(kind)


def weight(kind: str, s: np.ndarray, c: float) -> np.ndarray:
    """rho'(s)."""
    s = np.asarray(s, dtype=np.float64)
    if kind == "trivial":
        return np.ones_like(s)
    if kind == "huber":
        return np.where(s <= c * c, 1.0, c / np.sqrt(np.maximum(s, c * c)))
    if kind == "cauchy":
        return 1.0 / (1.0 + s / (c * c))
    raise ValueError(kind)


def cost(state: camera.State, obs_cam, obs_pt, obs_px, kind: str, c: float) -> float:
    if kind == "trivial":
        return camera.cost(state, obs_cam, obs_pt, obs_px)   # the plain cost, same summation
    r = camera.residuals(state, obs_cam, obs_pt, obs_px)
    return 0.5 * float(np.sum(rho(kind, np.sum(r * r, axis=1), c)))


def linearize(state: camera.State, obs_cam, obs_pt, obs_px, kind: str, c: float):
    """Robust cost and the IRLS-scaled system of one linearisation.

    Returns F, r~ [n,2], Jc~ [n,2,9], Jp~ [n,2,3], w [n]."""
    r, Jc, Jp = camera.linearize(state, obs_cam, obs_pt, obs_px)
    s = np.sum(r * r, axis=1)
    w = weight(kind, s, c)
    sw = np.sqrt(w)
    F = 0.5 * float(np.sum(rho(kind, s, c)))
    return F, r * sw[:, None], Jc * sw[:, None, None], Jp * sw[:, None, None], w
