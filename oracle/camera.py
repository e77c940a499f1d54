"""Snavely reprojection residual and its tangent-space Jacobian (oracle).

Follows the factor of Section VI-A: a camera is a pose (R, t) plus a
calibration (f, k1, k2); the point is moved into the camera frame,
P = R X + t, the depth gets a sign-preserving epsilon, the normalised image
point is p = -P_xy / d, the radial factor is 1 + k1 |p|^2 + k2 |p|^4 and the
predicted pixel is f * radial * p; the residual is prediction minus
measurement.

Tangent space (Section V: linearisation and retraction follow SymForce's
tangent-space approach): a camera update is [dw(3), dt(3), df, dk1, dk2] with
the rotation perturbed on the right, R <- R Exp(dw); t, calibration and the
point are updated additively.

Pins (tests/test_oracle_camera.py): hand-derived worked examples with exact
binary values (tests/golden/), the R = I, t = 0, k = 0 pinhole special case,
central finite differences of every Jacobian column, the 7 similarity-gauge
null vectors, Rodrigues vs. a matrix-exponential series.
"""
from __future__ import annotations

import numpy as np

EPS_F64 = 10.0 * np.finfo(np.float64).eps


def hat(v: np.ndarray) -> np.ndarray:
    """Skew matrices [v]x of shape [..., 3, 3]."""
    v = np.asarray(v, dtype=np.float64)
    z = np.zeros(v.shape[:-1])
    return np.stack([
        np.stack([z, -v[..., 2], v[..., 1]], axis=-1),
        np.stack([v[..., 2], z, -v[..., 0]], axis=-1),
        np.stack([-v[..., 1], v[..., 0], z], axis=-1),
    ], axis=-2)


def so3_exp(w: np.ndarray) -> np.ndarray:
    """Rotation matrices Exp(w) by Rodrigues' formula, [..., 3] -> [..., 3, 3].

    Small angles use the Taylor series of sin(a)/a and (1-cos a)/a^2.
    """
    w = np.asarray(w, dtype=np.float64)
    a2 = np.sum(w * w, axis=-1)
    a = np.sqrt(a2)
    small = a < 1e-4
    safe = np.where(small, 1.0, a)
    s = np.where(small, 1.0 - a2 / 6.0 + a2 * a2 / 120.0, np.sin(safe) / safe)
    c = np.where(small, 0.5 - a2 / 24.0 + a2 * a2 / 720.0, (1.0 - np.cos(safe)) / (safe * safe))
    K = hat(w)
    eye = np.broadcast_to(np.eye(3), K.shape)
    return eye + s[..., None, None] * K + c[..., None, None] * (K @ K)


class State:
    """Cameras and points at one linearisation point (caller order)."""

    def __init__(self, R, t, calib, X):
        self.R = np.asarray(R, dtype=np.float64)          # [nc, 3, 3]
        self.t = np.asarray(t, dtype=np.float64)          # [nc, 3]
        self.calib = np.asarray(calib, dtype=np.float64)  # [nc, 3]  (f, k1, k2)
        self.X = np.asarray(X, dtype=np.float64)          # [np, 3]

    @classmethod
    def from_bal(cls, cams9, points):
        cams9 = np.asarray(cams9, dtype=np.float64)
        return cls(so3_exp(cams9[:, 0:3]), cams9[:, 3:6].copy(), cams9[:, 6:9].copy(),
                   np.asarray(points, dtype=np.float64).copy())

    def copy(self) -> "State":
        return State(self.R.copy(), self.t.copy(), self.calib.copy(), self.X.copy())

    @property
    def n_cams(self) -> int:
        return self.R.shape[0]

    @property
    def n_points(self) -> int:
        return self.X.shape[0]

    @property
    def n_params(self) -> int:
        return 9 * self.n_cams + 3 * self.n_points

    def retract(self, delta: np.ndarray) -> "State":
        """theta (+) delta: R Exp(dw), t + dt, calib + dc, X + dX (Section V)."""
        nc = self.n_cams
        dc = delta[: 9 * nc].reshape(nc, 9)
        dX = delta[9 * nc:].reshape(self.n_points, 3)
        return State(self.R @ so3_exp(dc[:, 0:3]), self.t + dc[:, 3:6], self.calib + dc[:, 6:9], self.X + dX)


def _sign_no_zero(x):
    return np.where(x >= 0.0, 1.0, -1.0)


def project(state: State, obs_cam, obs_pt, eps: float = EPS_F64):
    """Predicted pixels u [n_obs, 2] of the Snavely model (Section VI-A)."""
    R = state.R[obs_cam]
    P = np.einsum("oij,oj->oi", R, state.X[obs_pt]) + state.t[obs_cam]
    d = P[:, 2] + eps * _sign_no_zero(P[:, 2])
    p = -P[:, 0:2] / d[:, None]
    n2 = np.sum(p * p, axis=1)
    f, k1, k2 = (state.calib[obs_cam, i] for i in range(3))
    radial = 1.0 + k1 * n2 + k2 * n2 * n2
    return (f * radial)[:, None] * p


def residuals(state: State, obs_cam, obs_pt, obs_px, eps: float = EPS_F64):
    """r = predicted - measured, [n_obs, 2]."""
    return project(state, obs_cam, obs_pt, eps) - np.asarray(obs_px, dtype=np.float64)


def cost(state: State, obs_cam, obs_pt, obs_px) -> float:
    """F = 1/2 sum |r|^2 (the paper reports MSE = 2F / n_obs)."""
    r = residuals(state, obs_cam, obs_pt, obs_px)
    return 0.5 * float(np.sum(r * r))


def linearize(state: State, obs_cam, obs_pt, obs_px, eps: float = EPS_F64):
    """Residuals and tangent Jacobian blocks.

    Returns r [n,2], Jc [n,2,9] (columns dw, dt, df, dk1, dk2), Jp [n,2,3].
    Chain rule through P = R X + t, p = -P_xy/d, u = f radial(p) p.
    """
    obs_cam = np.asarray(obs_cam)
    obs_pt = np.asarray(obs_pt)
    R = state.R[obs_cam]
    X = state.X[obs_pt]
    P = np.einsum("oij,oj->oi", R, X) + state.t[obs_cam]
    d = P[:, 2] + eps * _sign_no_zero(P[:, 2])
    p = -P[:, 0:2] / d[:, None]
    n2 = np.sum(p * p, axis=1)
    f, k1, k2 = (state.calib[obs_cam, i] for i in range(3))
    radial = 1.0 + k1 * n2 + k2 * n2 * n2
    u = (f * radial)[:, None] * p
    r = u - np.asarray(obs_px, dtype=np.float64)

    n = obs_cam.shape[0]
    # du/dp = f (radial I + p * d(radial)/dp^T),  d(radial)/dp = 2 (k1 + 2 k2 n2) p
    dr_dn2 = k1 + 2.0 * k2 * n2
    du_dp = f[:, None, None] * (radial[:, None, None] * np.eye(2)[None]
                                + 2.0 * dr_dn2[:, None, None] * np.einsum("oi,oj->oij", p, p))
    # dp/dP = -(1/d) [I2 | p]
    dp_dP = np.zeros((n, 2, 3))
    dp_dP[:, 0, 0] = 1.0
    dp_dP[:, 1, 1] = 1.0
    dp_dP[:, :, 2] = p
    dp_dP *= (-1.0 / d)[:, None, None]
    du_dP = du_dp @ dp_dP                                  # [n, 2, 3]
    # dP/dw = -R [X]x  (right perturbation),  dP/dt = I,  dP/dX = R
    dP_dw = -R @ hat(X)
    Jc = np.empty((n, 2, 9))
    Jc[:, :, 0:3] = du_dP @ dP_dw
    Jc[:, :, 3:6] = du_dP
    Jc[:, :, 6] = radial[:, None] * p
    Jc[:, :, 7] = (f * n2)[:, None] * p
    Jc[:, :, 8] = (f * n2 * n2)[:, None] * p
    Jp = du_dP @ R
    return r, Jc, Jp


def gauge_generators(state: State) -> np.ndarray:
    """The 7 similarity-gauge directions in tangent coordinates, [7, N].

    World rotation about e_k: dX = e_k x X, dw = -e_k; world translation e_k:
    dX = e_k, dt = -R e_k; world scale: dX = X, dt = t.  Every residual is
    invariant to first order along each of them, so J n = 0.
    """
    nc, npnt = state.n_cams, state.n_points
    out = np.zeros((7, 9 * nc + 3 * npnt))
    cam = out[:, : 9 * nc].reshape(7, nc, 9)
    pt = out[:, 9 * nc:].reshape(7, npnt, 3)
    for k in range(3):
        e = np.zeros(3)
        e[k] = 1.0
        pt[k] = np.cross(e[None, :], state.X)
        cam[k, :, k] = -1.0
        pt[3 + k] = e[None, :]
        cam[3 + k, :, 3:6] = -state.R[:, :, k]
    pt[6] = state.X
    cam[6, :, 3:6] = state.t
    return out
