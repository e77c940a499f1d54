"""Pins for the oracle's normal equations, block-Jacobi preconditioner and
PCG (Section V: normal equations solved directly, one preconditioner block
per node; glossary PCGNR)."""
import numpy as np
import pytest

from oracle import camera, linear, pcg

from helpers import small_scene, observed_pixels


def _problem(n_cams=4, n_points=30, seed=5, k=3):
    sc = small_scene(n_cams=n_cams, n_points=n_points, seed=seed, k=k)
    px = observed_pixels(sc)
    st = camera.State.from_bal(sc.cams_init, sc.points_init)
    r, Jc, Jp = camera.linearize(st, sc.obs_cam, sc.obs_pt, px)
    J = linear.jacobian_csr(Jc, Jp, sc.obs_cam, sc.obs_pt, sc.n_cams, sc.n_points)
    return sc, st, px, r, J


def test_jacobian_products_match_residual_directional_derivatives():
    # J p from central differences of the residual along the retraction,
    # J^T q from the adjoint identity q.(J p) = (J^T q).p
    sc, st, px, r, J = _problem()
    rng = np.random.default_rng(0)
    for _ in range(3):
        p = rng.normal(size=J.shape[1])
        h = 1e-6
        Jp_fd = (camera.residuals(st.retract(h * p), sc.obs_cam, sc.obs_pt, px)
                 - camera.residuals(st.retract(-h * p), sc.obs_cam, sc.obs_pt, px)).ravel() / (2 * h)
        Jp = J @ p
        assert np.linalg.norm(Jp - Jp_fd) <= 1e-6 * np.linalg.norm(Jp)
        q = rng.normal(size=J.shape[0])
        assert abs(q @ Jp_fd - (J.T @ q) @ p) <= 1e-6 * np.linalg.norm(q) * np.linalg.norm(Jp)


def test_matvec_is_symmetric_psd_and_matches_quadratic_form():
    sc, st, px, r, J = _problem()
    D = linear.damping_diagonal(J)
    rng = np.random.default_rng(1)
    lam = 0.37
    a, b = rng.normal(size=J.shape[1]), rng.normal(size=J.shape[1])
    Aa, Ab = linear.matvec(J, D, lam, a), linear.matvec(J, D, lam, b)
    assert abs(a @ Ab - b @ Aa) <= 1e-12 * np.linalg.norm(Aa) * np.linalg.norm(b)
    # p^T A p = |J p|^2 + lambda p^T D p with J p by finite differences
    h = 1e-6
    Ja_fd = (camera.residuals(st.retract(h * a), sc.obs_cam, sc.obs_pt, px)
             - camera.residuals(st.retract(-h * a), sc.obs_cam, sc.obs_pt, px)).ravel() / (2 * h)
    quad = Ja_fd @ Ja_fd + lam * a @ (D * a)
    assert abs(a @ Aa - quad) <= 1e-6 * quad


def test_damping_diagonal_is_clamped_column_norm():
    sc, st, px, r, J = _problem()
    D = linear.damping_diagonal(J)
    Jd = J.toarray()
    np.testing.assert_allclose(D, np.clip(np.sum(Jd * Jd, axis=0), 1e-6, 1e32), rtol=1e-14)
    # a column with no observations is clamped to the floor
    Jz = J.tolil()
    Jz[:, 0] = 0.0
    assert linear.damping_diagonal(Jz.tocsr())[0] == 1e-6


def test_block_jacobi_blocks_match_dense_normal_matrix():
    sc, st, px, r, J = _problem()
    D = linear.damping_diagonal(J)
    lam = 0.05
    A = linear.normal_matrix_dense(J, D, lam)
    Hc, Hp = linear.block_diagonal(J, D, lam, sc.n_cams, sc.n_points)
    for c in range(sc.n_cams):
        np.testing.assert_allclose(Hc[c], A[9 * c:9 * c + 9, 9 * c:9 * c + 9], rtol=1e-13, atol=1e-9)
    base = 9 * sc.n_cams
    for p in range(sc.n_points):
        s = slice(base + 3 * p, base + 3 * p + 3)
        np.testing.assert_allclose(Hp[p], A[s, s], rtol=1e-13, atol=1e-9)
    Mc, Mp = linear.block_jacobi_inverse(J, D, lam, sc.n_cams, sc.n_points)
    v = np.random.default_rng(2).normal(size=A.shape[0])
    z = linear.apply_block_jacobi(Mc, Mp, v)
    for c in range(sc.n_cams):
        s = slice(9 * c, 9 * c + 9)
        np.testing.assert_allclose(A[s, s] @ z[s], v[s], rtol=1e-9, atol=1e-9)


@pytest.mark.parametrize("lam", [1e-6, 1e-2, 1e2])
def test_exact_steps_agree(lam):
    sc, st, px, r, J = _problem(n_cams=3, n_points=12, k=2)
    D = linear.damping_diagonal(J)
    b = -linear.gradient(J, r.ravel())
    A = linear.normal_matrix_dense(J, D, lam)
    x_np = np.linalg.solve(A, b)
    x_dense = linear.solve_dense(J, D, lam, b)
    x_schur = linear.solve_schur(J, D, lam, b, sc.n_cams, sc.n_points)
    for x in (x_dense, x_schur):
        assert np.linalg.norm(A @ x - b) <= 1e-8 * np.linalg.norm(b)
        assert np.linalg.norm(x - x_np) <= 1e-6 * np.linalg.norm(x_np)


def test_pcg_terminates_on_small_system_and_matches_direct_solve():
    sc, st, px, r, J = _problem(n_cams=2, n_points=10, k=2)
    D = linear.damping_diagonal(J)
    lam = 1e-1
    b = -linear.gradient(J, r.ravel())
    Mc, Mp = linear.block_jacobi_inverse(J, D, lam, sc.n_cams, sc.n_points)
    x, rr, k, why = pcg.pcg(J, D, lam, b, Mc, Mp, tol=1e-12, max_iter=500)
    N = b.size
    assert why == "converged" and k <= N
    A = linear.normal_matrix_dense(J, D, lam)
    np.testing.assert_allclose(x, np.linalg.solve(A, b), rtol=1e-8, atol=1e-10 * np.abs(x).max())
    # the recurrence residual equals the true residual up to rounding
    assert np.linalg.norm(rr - (b - A @ x)) <= 1e-10 * np.linalg.norm(b)


def test_pcg_large_damping_is_one_iteration():
    # lambda -> infinity: A -> lambda D and M^-1 A -> I, so one step solves it
    sc, st, px, r, J = _problem()
    D = linear.damping_diagonal(J)
    lam = 1e12
    b = -linear.gradient(J, r.ravel())
    Mc, Mp = linear.block_jacobi_inverse(J, D, lam, sc.n_cams, sc.n_points)
    x, rr, k, why = pcg.pcg(J, D, lam, b, Mc, Mp, tol=1e-6, max_iter=50)
    assert why == "converged" and k == 1
    np.testing.assert_allclose(x, b / (lam * D), rtol=1e-6)


def test_pcg_zero_rhs():
    sc, st, px, r, J = _problem()
    D = linear.damping_diagonal(J)
    Mc, Mp = linear.block_jacobi_inverse(J, D, 1.0, sc.n_cams, sc.n_points)
    x, rr, k, why = pcg.pcg(J, D, 1.0, np.zeros(J.shape[1]), Mc, Mp, 1e-6, 10)
    assert why == "zero_rhs" and k == 0 and not x.any()


def test_pcg_stopping_bound_holds():
    sc, st, px, r, J = _problem(n_cams=6, n_points=80, k=3)
    D = linear.damping_diagonal(J)
    lam = 1e-3
    b = -linear.gradient(J, r.ravel())
    Mc, Mp = linear.block_jacobi_inverse(J, D, lam, sc.n_cams, sc.n_points)
    x, rr, k, why = pcg.pcg(J, D, lam, b, Mc, Mp, tol=1e-6, max_iter=500)
    A = linear.normal_matrix_dense(J, D, lam)
    assert why == "converged"
    assert np.linalg.norm(b - A @ x) <= 1.01e-6 * np.linalg.norm(b)
