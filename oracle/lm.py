"""Levenberg-Marquardt on the Snavely problem (oracle).

Section V: LM with the quality-based (gain-ratio) damping update of Madsen
et al., linearisation and retraction in the tangent space, normal equations
(J^T J + lambda D) delta = -g solved without reduction on the GPU.  The
oracle solves the same damped system exactly (dense or Schur Cholesky) or
with the same PCG steps as the GPU (inner="pcg").

One iteration = one inner solve plus one trial, accepted or not:
  pred = 1/2 (b^T delta + delta^T r_inner + lambda delta^T D delta), b = -g
  rho  = (F - F(theta (+) delta)) / pred
  rho > 0 and pred > 0: accept, relinearise, lambda *= max(1/3, 1-(2 rho-1)^3),
                        nu = 2
  otherwise:            lambda *= nu, nu *= 2
  lambda clamped to [lambda_min, lambda_max].
Stops early when ||g||_inf <= grad_tol * max(1, ||g_0||_inf), F <= min_cost,
or (if pred_tol > 0) the step's predicted decrease pred <= pred_tol * F: below
the resolution of F the gain ratio is rounding noise.

Defaults: lambda_0 = 1e-2, the inverse of the initial trust-region radius
100 used in Section VI.

With a robust loss (robust.py) the cost is 1/2 sum rho(|r|^2) and each
linearisation uses the IRLS-scaled residuals and blocks; the gain ratio
compares the robust cost decrease with that weighted model's prediction.

With pose between-factors (between.py; the robust loss applies to the
reprojection factors only) their six residual rows join the system: the
cost adds 1/2 sum |r_b|^2 and J, g and D are those of the stacked rows.

Pins (tests/test_oracle_lm.py): zero-noise problems converge to F ~ 0,
accepted costs decrease monotonically, the noisy optimum matches the
chi-square expectation, an independent solver (scipy least_squares on an
additive angle-axis parametrisation with its own residual) reaches the same
final cost.  The gain ratio's denominator equals the decrease of the linear
model 1/2 |r + J delta|^2 with J taken by central differences of the
residual (for the solver's own steps and for arbitrary steps with their inner
residual); steps that the linear model predicts to within a percent (a
zero-noise start near the truth) divide lambda by exactly 3; runs of rejected
trials multiply it by 2, 4, 8, ..., and after an accepted trial the next
rejection multiplies it by 2 again.
"""
from __future__ import annotations

import dataclasses

import numpy as np
import scipy.sparse as sp

from . import between as between_mod
from . import camera, linear, pcg as pcg_mod, robust


@dataclasses.dataclass
class LMOptions:
    lambda0: float = 1e-2
    max_iters: int = 20
    inner: str = "schur"            # "dense" | "schur" | "pcg"
    pcg_tol: float = 1e-6
    pcg_max_iters: int = 500
    lambda_min: float = 1e-12
    lambda_max: float = 1e16
    grad_tol: float = 1e-12
    min_cost: float = 1e-30
    nu_max: float = 2.0 ** 60
    pred_tol: float = 0.0           # stop when pred <= pred_tol * F (0: never)
    loss: str = "trivial"           # "trivial" | "huber" | "cauchy" (robust.py)
    loss_scale: float = 1.0
    between: tuple | None = None    # (fi, fj, Z [n, 6], w [n, 2]) pose between-factors (between.py)


@dataclasses.dataclass
class LMIteration:
    cost: float          # F after the iteration (current state)
    trial_cost: float
    lam: float           # lambda used in this iteration's solve
    rho: float
    pred: float
    accepted: bool
    inner_iters: int
    nu: float = 2.0      # nu after the iteration's damping update
    step: np.ndarray | None = None  # the trial step delta (tangent vector)


@dataclasses.dataclass
class LMResult:
    state: camera.State
    initial_cost: float
    final_cost: float
    history: list
    final_lambda: float
    stop_reason: str


def _linearize(state, obs_cam, obs_pt, obs_px, loss="trivial", scale=1.0, between=None):
    if loss == "trivial":
        r, Jc, Jp = camera.linearize(state, obs_cam, obs_pt, obs_px)
        F = 0.5 * float(np.sum(r * r))
    else:
        F, r, Jc, Jp, _ = robust.linearize(state, obs_cam, obs_pt, obs_px, loss, scale)
    J = linear.jacobian_csr(Jc, Jp, obs_cam, obs_pt, state.n_cams, state.n_points)
    r = np.asarray(r).ravel()
    if between is not None:
        rb, Ji, Jj = between_mod.linearize(state, *between)
        F += 0.5 * float(np.sum(rb * rb))
        J = sp.vstack([J, between_mod.jacobian_csr(Ji, Jj, between[0], between[1], state.n_cams,
                                                   state.n_points)]).tocsr()
        r = np.concatenate([r, rb.ravel()])
    g = linear.gradient(J, r)
    D = linear.damping_diagonal(J)
    return F, J, g, D


def total_cost(state, obs_cam, obs_pt, obs_px, opts: "LMOptions") -> float:
    """The objective: reprojection cost (robust if set) plus the between-factor cost."""
    F = robust.cost(state, obs_cam, obs_pt, obs_px, opts.loss, opts.loss_scale)
    if opts.between is not None:
        F += between_mod.cost(state, *opts.between)
    return F


def predicted_decrease(b, delta, r_in, lam, D) -> float:
    """Decrease of the linear model L(d) = 1/2 |r + J d|^2 from d = 0 to
    d = delta, written with the inner solve's quantities (reading 5): with
    b = -J^T r and the inner residual r_in = b - (J^T J + lam D) delta,
      L(0) - L(delta) = -g^T delta - 1/2 |J delta|^2
                      = 1/2 (b^T delta + delta^T r_in + lam delta^T D delta).
    For an exact step r_in = 0."""
    return 0.5 * float(b @ delta + delta @ r_in + lam * delta @ (D * delta))


def damping_update(lam: float, nu: float, rho: float, opts: "LMOptions"):
    """Section V's quality-based update after Madsen and Nielsen.
    Returns (accepted, lambda, nu) for the gain ratio rho of a trial:
    rho > 0 accepts, lambda *= max(1/3, 1 - (2 rho - 1)^3) and nu = 2;
    otherwise lambda *= nu and nu doubles (capped at nu_max).  lambda is then
    clamped to [lambda_min, lambda_max]."""
    if rho > 0.0:
        lam *= max(1.0 / 3.0, 1.0 - (2.0 * rho - 1.0) ** 3)
        nu = 2.0
        accepted = True
    else:
        lam *= nu
        nu = min(2.0 * nu, opts.nu_max)
        accepted = False
    return accepted, min(max(lam, opts.lambda_min), opts.lambda_max), nu


def solve_step(J, D, lam, b, n_cams, n_points, opts: LMOptions):
    """Returns (delta, inner residual b - A delta, inner iterations)."""
    if opts.inner == "dense":
        x = linear.solve_dense(J, D, lam, b)
        return x, np.zeros_like(b), 0
    if opts.inner == "schur":
        x = linear.solve_schur(J, D, lam, b, n_cams, n_points)
        return x, np.zeros_like(b), 0
    if opts.inner == "pcg":
        Mc, Mp = linear.block_jacobi_inverse(J, D, lam, n_cams, n_points)
        x, r, k, _ = pcg_mod.pcg(J, D, lam, b, Mc, Mp, opts.pcg_tol, opts.pcg_max_iters)
        return x, r, k
    raise ValueError(opts.inner)


def solve(state: camera.State, obs_cam, obs_pt, obs_px, opts: LMOptions | None = None) -> LMResult:
    opts = opts or LMOptions()
    state = state.copy()
    lin = lambda st: _linearize(st, obs_cam, obs_pt, obs_px, opts.loss, opts.loss_scale, opts.between)
    F, J, g, D = lin(state)
    F0 = F
    g0 = float(np.max(np.abs(g))) if g.size else 0.0
    lam, nu = opts.lambda0, 2.0
    history = []
    reason = "max_iters"
    for _ in range(opts.max_iters):
        if float(np.max(np.abs(g))) <= opts.grad_tol * max(1.0, g0):
            reason = "gradient"
            break
        if F <= opts.min_cost:
            reason = "cost"
            break
        b = -g
        delta, r_in, k = solve_step(J, D, lam, b, state.n_cams, state.n_points, opts)
        pred = predicted_decrease(b, delta, r_in, lam, D)
        if opts.pred_tol > 0.0 and pred <= opts.pred_tol * F:
            reason = "pred"
            break
        trial = state.retract(delta)
        Ft = total_cost(trial, obs_cam, obs_pt, obs_px, opts)
        rho = (F - Ft) / pred if (pred > 0.0 and np.isfinite(Ft)) else -np.inf
        lam_used = lam
        accepted, lam, nu = damping_update(lam, nu, rho, opts)
        if accepted:
            state = trial
            F, J, g, D = lin(state)
        history.append(LMIteration(F, Ft, lam_used, rho, pred, accepted, k, nu, delta))
    return LMResult(state, F0, F, history, lam, reason)
