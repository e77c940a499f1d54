"""Implicit adjoint of the LM optimum with respect to the observed pixels
(oracle).

At the optimum theta*, J^T r = 0 with r = u(theta) - px.  Differentiating
with the Gauss-Newton Hessian and the solver's damping gives
d theta*/d px = (J^T J + lambda D)^-1 J^T, hence for a loss L(theta*)
with tangent gradient g_theta:
    v = (J^T J + lambda D)^-1 g_theta,   dL/dpx_o = J_o v   (2 values / obs),
because dr/dpx = -I.

Pins (tests/test_oracle_adjoint.py): dense solve vs Schur solve, the
gauge-projection identity (removing the D-weighted gauge part of g leaves
J A^-1 g unchanged), central finite differences of the one-step linearised
map, symmetric JVP/VJP dot test.
"""
from __future__ import annotations

import numpy as np

import scipy.sparse as sp

from . import between as between_mod
from . import camera, linear, robust


def implicit_grad_obs(state: camera.State, obs_cam, obs_pt, obs_px, g_theta: np.ndarray,
                      lam: float, method: str = "schur", loss: str = "trivial",
                      loss_scale: float = 1.0, between=None) -> np.ndarray:
    """dL/dpx [n_obs, 2] for the tangent gradient g_theta at state.

    With a robust loss the IRLS weights are held fixed (the Gauss-Newton
    reading of the optimality condition sum_o w_o J_o^T r_o = 0): the system
    uses the sqrt(w)-scaled blocks J~ and dL/dpx_o = w_o J_o v =
    sqrt(w_o) J~_o v.  Pose between-factors (fi, fj, Z, w) join the system
    matrix; they hold no pixels, so dL/dpx keeps one row pair per
    observation."""
    if loss == "trivial":
        _, Jc, Jp = camera.linearize(state, obs_cam, obs_pt, obs_px)
        sw = np.ones(np.asarray(obs_cam).shape[0])
    else:
        _, _, Jc, Jp, w = robust.linearize(state, obs_cam, obs_pt, obs_px, loss, loss_scale)
        sw = np.sqrt(w)
    J = linear.jacobian_csr(Jc, Jp, obs_cam, obs_pt, state.n_cams, state.n_points)
    Jsys = J
    if between is not None:
        _, Ji, Jj = between_mod.linearize(state, *between)
        Jsys = sp.vstack([J, between_mod.jacobian_csr(Ji, Jj, between[0], between[1], state.n_cams,
                                                      state.n_points)]).tocsr()
    D = linear.damping_diagonal(Jsys)
    if method == "dense":
        v = linear.solve_dense(Jsys, D, lam, g_theta)
    else:
        v = linear.solve_schur(Jsys, D, lam, g_theta, state.n_cams, state.n_points)
    return (J @ v).reshape(-1, 2) * sw[:, None]


def point_norm_loss_grad(state: camera.State) -> np.ndarray:
    """Tangent gradient of L = sum |X_j|^2: zero on cameras, 2 X on points."""
    g = np.zeros(state.n_params)
    g[9 * state.n_cams:] = 2.0 * state.X.ravel()
    return g


def gauge_project(g: np.ndarray, N: np.ndarray, D: np.ndarray) -> np.ndarray:
    """g - D N (N^T D N)^-1 N^T g  (N: gauge vectors as rows, [7, N])."""
    DN = D[None, :] * N
    coef = np.linalg.solve(DN @ N.T, N @ g)
    return g - DN.T @ coef
