"""The implicit adjoint in the float32-mixed form (float32 blocks, products
and PCG vectors; float64 dots, alpha/beta and block-Jacobi inverses), the
backward of the large workload's configuration, against the float64 oracle's
dense implicit gradient at the same parameters.

Tolerance.  At the optimum of `tiny` the block-Jacobi preconditioned matrix
M^-1 (J^T J + lambda D) at lambda_adj = 1e-4 has its seven gauge eigenvalues
near lambda_adj and the rest in [0.087, 2.0] (float64 eigenvalues of the
dense matrix), a condition number of 23 off the gauge.  J v does not see the
gauge part of v (J N = 0), so with the gauge projection (which removes that
part from the right-hand side) the error of dL/dpx is that of a
well-conditioned solve: the float32 blocks carry a relative error of a few
u = 2^-24 from their evaluation (about ten roundings along the chain), which
the solve amplifies by at most the condition number, 23 * 10 u = 1.4e-5, plus
the PCG stopping residual (tolerance 1e-6, also amplified by at most 23):
bar 5e-5.  Without the projection v also holds the gauge component, about
sigma / lambda_adj = 0.087 / 1e-4 = 870 times the size of the rest (sigma: the
smallest eigenvalue off the gauge), and float32 blocks do not annihilate it
exactly: J v picks up a rounding residue of about 10 u |J| |v_N|, relative
10 u * 870 = 5.2e-4 of J v: bar 5e-4."""
import numpy as np
import pytest

from oracle import adjoint, camera
from synth import scene_config

from gpu_helpers import handle_for, observed_pixels, rel

pytestmark = pytest.mark.gpu

FP32_MIXED = 1


def _solved_mixed(name, rj):
    from paper_2605_30583_amd import SolveOptions
    sc = scene_config(name)
    px = observed_pixels(sc)
    ba = handle_for(sc, px, FP32_MIXED, rj=rj)
    ba.solve(SolveOptions(max_lm_iters=20, pcg_tol=1e-6))
    return sc, px, ba


@pytest.mark.parametrize("gauge", [False, True], ids=["plain", "gauge_projected"])
@pytest.mark.parametrize("rj", [False, True], ids=["stored", "recompute"])
@pytest.mark.parametrize("name", ["tiny", "medium"])
def test_fp32_mixed_adjoint_matches_oracle(name, rj, gauge):
    sc, px, ba = _solved_mixed(name, rj)
    cams, pts = ba.get_params()
    state = camera.State.from_bal(cams.cpu().numpy(), pts.cpu().numpy())
    lam = 1e-4
    ref = adjoint.implicit_grad_obs(state, sc.obs_cam, sc.obs_pt, px, adjoint.point_norm_loss_grad(state), lam,
                                    "schur")
    out = ba.backward(None, 2.0 * pts, lambda_adj=lam, pcg_tol=1e-6, max_pcg_iters=2000,
                      gauge_project=gauge).cpu().numpy()
    err = rel(out, ref)
    print(f"{name} rj={rj} gauge={gauge}: float32-mixed adjoint relative error {err:.3e}, "
          f"PCG {ba.last_backward_iters} iterations, residual {ba.last_backward_rel_resid:.2e}")
    assert ba.last_backward_rel_resid <= 1e-6
    assert err <= (5e-5 if gauge else 5e-4)
