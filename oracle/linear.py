"""Normal equations of the bundle-adjustment problem (oracle).

Sparse Jacobian J (2 n_obs x N, N = 9 n_cams + 3 n_points; tangent order
[cameras | points], caller indices), the damping diagonal, the damped
normal-equation product (J^T J + lambda D) p, the block-Jacobi
preconditioner with one block per node (Section V: one block per pose or
landmark), and the exact step by dense Cholesky or by the Schur complement
on the cameras.

Readings where the paper leaves it open: D = diag(J^T J) clamped to [1e-6, 1e32]; the
preconditioner blocks are the diagonal blocks of J^T J + lambda D.

Pins (tests/test_oracle_linear.py): matvec vs a dense J^T J product built
column by column from the Jacobian blocks; Schur step vs dense Cholesky vs
numpy.linalg.solve; block-Jacobi inverse vs numpy.linalg.inv of the dense
diagonal blocks; J^T J symmetric positive semi-definite with the 7 gauge
vectors in its null space.
"""
from __future__ import annotations

import numpy as np
import scipy.linalg
import scipy.sparse as sp

DIAG_MIN = 1e-6
DIAG_MAX = 1e32


def jacobian_csr(Jc, Jp, obs_cam, obs_pt, n_cams, n_points) -> sp.csr_matrix:
    """Assemble the sparse Jacobian from per-observation blocks."""
    n = Jc.shape[0]
    rows = np.repeat(np.arange(2 * n).reshape(n, 2), 12, axis=1).reshape(n, 2, 12)
    cols_c = (9 * np.asarray(obs_cam, dtype=np.int64))[:, None] + np.arange(9)[None, :]
    cols_p = (9 * n_cams + 3 * np.asarray(obs_pt, dtype=np.int64))[:, None] + np.arange(3)[None, :]
    cols = np.concatenate([cols_c, cols_p], axis=1)               # [n, 12]
    cols = np.broadcast_to(cols[:, None, :], (n, 2, 12))
    vals = np.concatenate([Jc, Jp], axis=2)                        # [n, 2, 12]
    N = 9 * n_cams + 3 * n_points
    return sp.csr_matrix((vals.ravel(), (rows.ravel(), cols.ravel())), shape=(2 * n, N))


def damping_diagonal(J: sp.spmatrix) -> np.ndarray:
    """D = clamp(diag(J^T J), 1e-6, 1e32): column squared norms of J."""
    d = np.asarray(J.multiply(J).sum(axis=0)).ravel()
    return np.clip(d, DIAG_MIN, DIAG_MAX)


def gradient(J: sp.spmatrix, r: np.ndarray) -> np.ndarray:
    """g = J^T r."""
    return J.T @ np.asarray(r).ravel()


def matvec(J: sp.spmatrix, D: np.ndarray, lam: float, p: np.ndarray) -> np.ndarray:
    """w = J^T (J p) + lambda D p  (J^T J is never formed)."""
    return J.T @ (J @ p) + lam * D * p


def normal_matrix_dense(J: sp.spmatrix, D: np.ndarray, lam: float) -> np.ndarray:
    """Dense A = J^T J + lambda D (small problems only)."""
    Jd = J.toarray()
    return Jd.T @ Jd + lam * np.diag(D)


def block_diagonal(J: sp.spmatrix, D: np.ndarray, lam: float, n_cams: int, n_points: int):
    """Diagonal blocks of J^T J + lambda D: cameras [nc, 9, 9], points [np, 3, 3]."""
    JtJ = (J.T @ J).tocsr()
    Hc = np.empty((n_cams, 9, 9))
    Hp = np.empty((n_points, 3, 3))
    for c in range(n_cams):
        s = slice(9 * c, 9 * c + 9)
        Hc[c] = JtJ[s, s].toarray() + lam * np.diag(D[s])
    base = 9 * n_cams
    if n_points:
        # points: gather the 3x3 blocks in one vectorised pass over the CSR rows
        JtJ_pp = JtJ[base:, base:].tocoo()
        keep = (JtJ_pp.row // 3) == (JtJ_pp.col // 3)
        Hp[:] = 0.0
        np.add.at(Hp, (JtJ_pp.row[keep] // 3, JtJ_pp.row[keep] % 3, JtJ_pp.col[keep] % 3),
                  JtJ_pp.data[keep])
        Dp = D[base:].reshape(n_points, 3)
        Hp += lam * np.einsum("ni,ij->nij", Dp, np.eye(3))
    return Hc, Hp


def block_jacobi_inverse(J, D, lam, n_cams, n_points):
    """Inverses of the diagonal blocks (the preconditioner M^-1)."""
    Hc, Hp = block_diagonal(J, D, lam, n_cams, n_points)
    return np.linalg.inv(Hc), np.linalg.inv(Hp)


def apply_block_jacobi(Mc_inv, Mp_inv, r: np.ndarray) -> np.ndarray:
    """z = M^-1 r with one block per camera and per point."""
    nc = Mc_inv.shape[0]
    zc = np.einsum("nij,nj->ni", Mc_inv, r[: 9 * nc].reshape(nc, 9))
    zp = np.einsum("nij,nj->ni", Mp_inv, r[9 * nc:].reshape(-1, 3))
    return np.concatenate([zc.ravel(), zp.ravel()])


def solve_dense(J, D, lam, b) -> np.ndarray:
    """Exact step: Cholesky of the dense J^T J + lambda D."""
    A = normal_matrix_dense(J, D, lam)
    return scipy.linalg.cho_solve(scipy.linalg.cho_factor(A), b)


def solve_schur(J, D, lam, b, n_cams: int, n_points: int) -> np.ndarray:
    """Exact step by eliminating the points (Schur complement on cameras).

    A = [[U, W], [W^T, V]] with V block-diagonal 3x3;
    S = U - W V^-1 W^T;  S dc = bc - W V^-1 bp;  dp = V^-1 (bp - W^T dc).
    """
    nc9 = 9 * n_cams
    JtJ = (J.T @ J).tocsr()
    U = JtJ[:nc9, :nc9].toarray() + lam * np.diag(D[:nc9])
    W = JtJ[:nc9, nc9:].tocsr()
    _, Hp = block_diagonal(J[:, nc9:], D[nc9:], lam, 0, n_points)
    Vinv = np.linalg.inv(Hp)
    Vinv_sp = sp.block_diag(list(Vinv), format="csr") if n_points else sp.csr_matrix((0, 0))
    bc, bp = b[:nc9], b[nc9:]
    WVinv = (W @ Vinv_sp).tocsr()
    S = U - (WVinv @ W.T).toarray()
    dc = scipy.linalg.cho_solve(scipy.linalg.cho_factor(S), bc - WVinv @ bp)
    dp = Vinv_sp @ (bp - W.T @ dc)
    return np.concatenate([dc, dp])
