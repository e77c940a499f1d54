"""Pins for the oracle's implicit adjoint of the LM optimum w.r.t. the
observed pixels (implicit function theorem on J^T r = 0 with the damped
Gauss-Newton matrix of Section V)."""
import numpy as np
import pytest

from oracle import adjoint, camera, linear, lm

from helpers import small_scene, observed_pixels


def _converged(noise_scale=1.0, n_cams=4, n_points=40, seed=21, k=3):
    sc = small_scene(n_cams=n_cams, n_points=n_points, seed=seed, k=k)
    px = observed_pixels(sc, noise_scale)
    st = camera.State.from_bal(sc.cams_init, sc.points_init)
    res = lm.solve(st, sc.obs_cam, sc.obs_pt, px, lm.LMOptions(max_iters=40, inner="dense"))
    return sc, px, res


def test_dense_and_schur_implicit_gradients_agree():
    sc, px, res = _converged()
    g = adjoint.point_norm_loss_grad(res.state)
    a = adjoint.implicit_grad_obs(res.state, sc.obs_cam, sc.obs_pt, px, g, 1e-4, "dense")
    b = adjoint.implicit_grad_obs(res.state, sc.obs_cam, sc.obs_pt, px, g, 1e-4, "schur")
    assert np.linalg.norm(a - b) <= 1e-8 * np.linalg.norm(a)


def test_gauge_projection_leaves_gradient_unchanged():
    sc, px, res = _converged()
    st = res.state
    g = adjoint.point_norm_loss_grad(st)
    _, Jc, Jp = camera.linearize(st, sc.obs_cam, sc.obs_pt, px)
    J = linear.jacobian_csr(Jc, Jp, sc.obs_cam, sc.obs_pt, sc.n_cams, sc.n_points)
    D = linear.damping_diagonal(J)
    N = camera.gauge_generators(st)
    gr = adjoint.gauge_project(g, N, D)
    assert np.linalg.norm(N @ gr) <= 1e-8 * np.linalg.norm(N @ g)
    lam = 1e-4
    a = adjoint.implicit_grad_obs(st, sc.obs_cam, sc.obs_pt, px, g, lam, "dense")
    b = adjoint.implicit_grad_obs(st, sc.obs_cam, sc.obs_pt, px, gr, lam, "dense")
    assert np.linalg.norm(a - b) <= 1e-6 * np.linalg.norm(a)


def test_one_step_linearised_map_finite_differences():
    # freeze J, D, lambda at the optimum; delta(px) = A^-1 J^T (px - u(theta*))
    # is linear in px, so central differences of L(theta* (+) delta) agree
    # with the adjoint up to the 2 delta_0 term, which vanishes at convergence
    sc, px, res = _converged()
    st = res.state
    lam = 1e-4
    _, Jc, Jp = camera.linearize(st, sc.obs_cam, sc.obs_pt, px)
    J = linear.jacobian_csr(Jc, Jp, sc.obs_cam, sc.obs_pt, sc.n_cams, sc.n_points)
    D = linear.damping_diagonal(J)
    A = linear.normal_matrix_dense(J, D, lam)
    u = camera.project(st, sc.obs_cam, sc.obs_pt)

    def loss(pxv):
        delta = np.linalg.solve(A, J.T @ (pxv - u).ravel())
        Xn = st.X + delta[9 * sc.n_cams:].reshape(-1, 3)
        return float(np.sum(Xn * Xn))

    g = adjoint.point_norm_loss_grad(st)
    grad = adjoint.implicit_grad_obs(st, sc.obs_cam, sc.obs_pt, px, g, lam, "dense")
    h = 1e-3
    rng = np.random.default_rng(0)
    for o in rng.choice(sc.n_obs, 6, replace=False):
        for c in range(2):
            e = np.zeros_like(px)
            e[o, c] = h
            fd = (loss(px + e) - loss(px - e)) / (2 * h)
            assert abs(fd - grad[o, c]) <= 1e-6 * max(1.0, np.abs(grad).max())


def test_vjp_jvp_dot_identity():
    sc, px, res = _converged()
    st = res.state
    lam = 1e-3
    _, Jc, Jp = camera.linearize(st, sc.obs_cam, sc.obs_pt, px)
    J = linear.jacobian_csr(Jc, Jp, sc.obs_cam, sc.obs_pt, sc.n_cams, sc.n_points)
    D = linear.damping_diagonal(J)
    A = linear.normal_matrix_dense(J, D, lam)
    rng = np.random.default_rng(3)
    g = rng.normal(size=A.shape[0])
    du = rng.normal(size=(sc.n_obs, 2))
    vjp = adjoint.implicit_grad_obs(st, sc.obs_cam, sc.obs_pt, px, g, lam, "dense")
    jvp = np.linalg.solve(A, J.T @ du.ravel())          # d theta for a pixel change du
    assert abs(np.sum(vjp * du) - g @ jvp) <= 1e-9 * abs(g @ jvp)


@pytest.mark.slow
def test_full_resolve_finite_differences_zero_noise():
    # noise-free problem: the Gauss-Newton matrix is the exact Hessian at the
    # optimum, so re-solving at px +- h matches the adjoint as lambda_adj -> 0
    sc, px, res = _converged(noise_scale=0.0, n_cams=4, n_points=30, seed=5, k=3)
    st = res.state
    g = adjoint.point_norm_loss_grad(st)
    grad = adjoint.implicit_grad_obs(st, sc.obs_cam, sc.obs_pt, px, g, 1e-9, "dense")
    h = 1e-4
    opts = lm.LMOptions(max_iters=30, inner="dense", lambda0=1e-8, grad_tol=0.0)
    rng = np.random.default_rng(1)
    for o in rng.choice(sc.n_obs, 4, replace=False):
        c = int(rng.integers(0, 2))
        vals = []
        for s in (+1, -1):
            e = np.zeros_like(px)
            e[o, c] = s * h
            r2 = lm.solve(st, sc.obs_cam, sc.obs_pt, px + e, opts)
            vals.append(float(np.sum(r2.state.X ** 2)))
        fd = (vals[0] - vals[1]) / (2 * h)
        assert abs(fd - grad[o, c]) <= 1e-4 * max(1.0, np.abs(grad).max()), (o, c, fd, grad[o, c])
