"""Pose between-factors on pairs of cameras (oracle).

TEST INFRASTRUCTURE ONLY.

The paper's solvers are generated per collection of factor types, an
odometry factor beside the reprojection factor being its example
(Section V, the solver description), and its memory accessors include
pairwise reads and adds for such chain factors (Section IV-A).  The paper
fixes no formula for the odometry residual; the reading taken here:

  camera pose   T_c = (R_c, t_c), world -> camera: x_c = R_c x + t_c
  relative pose T_ij = T_j T_i^-1 = (R_j R_i^T, t_j - R_j R_i^T t_i)
  measurement   Z = (Z_R, Z_t), given as angle-axis (3) and translation (3)
  residual      r = [ s_rot   Log(Z_R^T R_j R_i^T) ;
                      s_trans (t_j - R_j R_i^T t_i - Z_t) ]      (6 values)
  cost          1/2 |r|^2 per factor, added to the reprojection cost

with per-factor weights s_rot, s_trans > 0 (square roots of isotropic
information).  Derivatives in the camera tangent [dw, dt, df, dk1, dk2] with
R <- R Exp(dw), t <- t + dt (so R_i^T <- Exp(-dw) R_i^T); with
phi = Log(Z_R^T R_j R_i^T), u = R_i^T t_i and Jr^-1 the inverse right
Jacobian of SO(3):

  dr_rot/dw_i   = -s_rot Jr^-1(phi) R_i        dr_rot/dw_j   = s_rot Jr^-1(phi) R_i
  dr_trans/dw_i = -s_trans R_j [u]x            dr_trans/dw_j = s_trans R_j [u]x
  dr_trans/dt_i = -s_trans R_j R_i^T           dr_trans/dt_j = s_trans I
  (rotation rows do not depend on t; no factor depends on f, k1, k2).

Pins (tests/test_oracle_between.py): Log(Exp(phi)) = phi across small,
moderate and near-pi angles; Jr^-1 against central differences of
Log(Exp(phi) Exp(h e_k)); the residual vanishes when Z is the true relative
pose; the blocks against central differences of the residual through
State.retract; J n = 0 for the six rigid-motion gauge directions while the
scale direction is not in the null space.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp

from . import camera


def so3_log(R: np.ndarray) -> np.ndarray:
    """Log of rotation matrices [..., 3, 3] -> angle-axis [..., 3], angle in [0, pi].

    With v = (R - R^T)^vee / 2 = sin(theta) n and cos theta from the trace,
    theta = atan2(|v|, cos theta); phi = v theta / |v| (theta / sin theta by
    its series 1 + theta^2/6 below theta = 1e-4).  Above theta = 2, where v
    shrinks towards pi and its direction loses digits, the axis comes from the
    largest column of n n^T = (sym(R) - cos theta I) / (1 - cos theta),
    signed by v."""
    R = np.asarray(R, dtype=np.float64)
    out = np.empty(R.shape[:-1])
    flat_R = R.reshape(-1, 3, 3)
    flat = out.reshape(-1, 3)
    for k, M in enumerate(flat_R):
        c = np.clip((np.trace(M) - 1.0) / 2.0, -1.0, 1.0)
        v = 0.5 * np.array([M[2, 1] - M[1, 2], M[0, 2] - M[2, 0], M[1, 0] - M[0, 1]])  # sin(theta) n
        s = float(np.linalg.norm(v))
        theta = np.arctan2(s, c)
        if theta < 1e-4:
            flat[k] = v * (1.0 + theta * theta / 6.0)
        elif theta <= 2.0:
            flat[k] = v * (theta / s)
        else:
            S = (0.5 * (M + M.T) - c * np.eye(3)) / (1.0 - c)
            j = int(np.argmax(np.diag(S)))
            n = S[:, j] / np.sqrt(S[j, j])
            if n @ v < 0.0:
                n = -n
            flat[k] = theta * n
    return out


def so3_jr_inv(phi: np.ndarray) -> np.ndarray:
    """Inverse right Jacobian of SO(3): [..., 3] -> [..., 3, 3].

    Jr^-1(phi) = I + 1/2 [phi]x + (1/theta^2 - (1 + cos theta) / (2 theta sin theta)) [phi]x^2,
    the coefficient by its series 1/12 + theta^2/720 below theta = 1e-4."""
    phi = np.asarray(phi, dtype=np.float64)
    th2 = np.sum(phi * phi, axis=-1)
    th = np.sqrt(th2)
    small = th < 1e-4
    safe = np.where(small, 1.0, th)
    coef = np.where(small, 1.0 / 12.0 + th2 / 720.0,
                    1.0 / (safe * safe) - (1.0 + np.cos(safe)) / (2.0 * safe * np.sin(safe)))
    K = camera.hat(phi)
    eye = np.broadcast_to(np.eye(3), K.shape)
    return eye + 0.5 * K + coef[..., None, None] * (K @ K)


def residuals(state: camera.State, fi, fj, Z, w) -> np.ndarray:
    """r [n, 6] of the factors (fi[k], fj[k], Z[k], w[k])."""
    fi, fj = np.asarray(fi), np.asarray(fj)
    Z, w = np.asarray(Z, np.float64).reshape(-1, 6), np.asarray(w, np.float64).reshape(-1, 2)
    Ri, Rj, ti, tj = state.R[fi], state.R[fj], state.t[fi], state.t[fj]
    Rij = Rj @ np.swapaxes(Ri, -1, -2)
    ZR = camera.so3_exp(Z[:, 0:3])
    r_rot = so3_log(np.swapaxes(ZR, -1, -2) @ Rij)
    r_trans = tj - np.einsum("kab,kb->ka", Rij, ti) - Z[:, 3:6]
    return np.concatenate([w[:, 0:1] * r_rot, w[:, 1:2] * r_trans], axis=1)


def cost(state: camera.State, fi, fj, Z, w) -> float:
    r = residuals(state, fi, fj, Z, w)
    return 0.5 * float(np.sum(r * r))


def linearize(state: camera.State, fi, fj, Z, w):
    """r [n, 6] and the blocks Ji, Jj [n, 6, 9] (camera tangent columns)."""
    fi, fj = np.asarray(fi), np.asarray(fj)
    Z, w = np.asarray(Z, np.float64).reshape(-1, 6), np.asarray(w, np.float64).reshape(-1, 2)
    n = fi.shape[0]
    r = residuals(state, fi, fj, Z, w)
    phi = r[:, 0:3] / w[:, 0:1]
    Ri, Rj, ti = state.R[fi], state.R[fj], state.t[fi]
    Jr_inv = so3_jr_inv(phi)
    u = np.einsum("kba,kb->ka", Ri, ti)                      # R_i^T t_i
    Ji = np.zeros((n, 6, 9))
    Jj = np.zeros((n, 6, 9))
    A = Jr_inv @ Ri
    Ji[:, 0:3, 0:3] = -A
    Jj[:, 0:3, 0:3] = A
    B = Rj @ camera.hat(u)
    Ji[:, 3:6, 0:3] = -B
    Jj[:, 3:6, 0:3] = B
    Ji[:, 3:6, 3:6] = -(Rj @ np.swapaxes(Ri, -1, -2))
    Jj[:, 3:6, 3:6] = np.eye(3)
    Ji[:, 0:3] *= w[:, 0, None, None]
    Jj[:, 0:3] *= w[:, 0, None, None]
    Ji[:, 3:6] *= w[:, 1, None, None]
    Jj[:, 3:6] *= w[:, 1, None, None]
    return r, Ji, Jj


def jacobian_csr(Ji, Jj, fi, fj, n_cams, n_points) -> sp.csr_matrix:
    """Rows of the between factors (6 per factor) over the full tangent."""
    n = Ji.shape[0]
    rows = np.broadcast_to(np.arange(6 * n).reshape(n, 6, 1), (n, 6, 18))
    ci = (9 * np.asarray(fi, dtype=np.int64))[:, None] + np.arange(9)[None, :]
    cj = (9 * np.asarray(fj, dtype=np.int64))[:, None] + np.arange(9)[None, :]
    cols = np.broadcast_to(np.concatenate([ci, cj], axis=1)[:, None, :], (n, 6, 18))
    vals = np.concatenate([Ji, Jj], axis=2)
    N = 9 * n_cams + 3 * n_points
    return sp.csr_matrix((vals.ravel(), (rows.ravel(), cols.ravel())), shape=(6 * n, N))


def measurements(state_true: camera.State, fi, fj, rot_noise, trans_noise, rot_sigma: float,
                 trans_sigma: float):
    """Synthetic measurements from true poses: Z_R = (R_j R_i^T) Exp(rot_sigma n_rot),
    Z_t = t_j - R_j R_i^T t_i + trans_sigma n_trans (n_* the caller's draws),
    weights 1/sigma.  Returns Z [n, 6] (angle-axis, translation) and w [n, 2]."""
    fi, fj = np.asarray(fi), np.asarray(fj)
    Ri, Rj, ti, tj = state_true.R[fi], state_true.R[fj], state_true.t[fi], state_true.t[fj]
    Rij = Rj @ np.swapaxes(Ri, -1, -2)
    ZR = Rij @ camera.so3_exp(rot_sigma * np.asarray(rot_noise))
    Zt = tj - np.einsum("kab,kb->ka", Rij, ti) + trans_sigma * np.asarray(trans_noise)
    Z = np.concatenate([so3_log(ZR), Zt], axis=1)
    w = np.tile([1.0 / rot_sigma, 1.0 / trans_sigma], (fi.shape[0], 1))
    return Z, w


def rigid_gauge_generators(state: camera.State) -> np.ndarray:
    """The six rigid-motion rows of camera.gauge_generators (world rotation and
    translation); the seventh (scale) changes relative translations."""
    return camera.gauge_generators(state)[:6]
