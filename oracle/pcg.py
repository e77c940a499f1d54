"""Block-Jacobi preconditioned conjugate gradients on the normal equations
(PCGNR, glossary and Section V of the paper), the oracle form.

Matrix-free: A p = J^T (J p) + lambda D p.  x0 = 0, stop when
||b - A x||_2 <= tol ||b||_2 (recurrence residual), on p^T A p <= 0, or after
max_iter products.  Returns the recurrence residual r = b - A x as well,
which the LM gain ratio uses.

Pins (tests/test_oracle_linear.py): finite termination within N steps on a
small SPD system (agrees with the direct solve), the lambda -> infinity case
where the preconditioned operator is the identity (one iteration), the
stopping bound checked with an independent dense product.
"""
from __future__ import annotations

import numpy as np

from . import linear


def pcg(J, D, lam, b, Mc_inv, Mp_inv, tol: float, max_iter: int):
    """Returns (x, r, iterations, reason) with reason in
    {"converged", "breakdown", "max_iter", "zero_rhs"}."""
    x = np.zeros_like(b)
    r = b.copy()
    bnorm = float(np.linalg.norm(b))
    if bnorm == 0.0:
        return x, r, 0, "zero_rhs"
    z = linear.apply_block_jacobi(Mc_inv, Mp_inv, r)
    p = z.copy()
    rho = float(r @ z)
    for k in range(1, max_iter + 1):
        w = linear.matvec(J, D, lam, p)
        pAp = float(p @ w)
        if not pAp > 0.0:
            return x, r, k, "breakdown"
        alpha = rho / pAp
        x += alpha * p
        r -= alpha * w
        if float(np.linalg.norm(r)) <= tol * bnorm:
            return x, r, k, "converged"
        z = linear.apply_block_jacobi(Mc_inv, Mp_inv, r)
        rho_new = float(r @ z)
        beta = rho_new / rho
        rho = rho_new
        p = z + beta * p
    return x, r, max_iter, "max_iter"
