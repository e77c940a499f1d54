"""caspar_ba_create_static: the handle built on the library's static device
workspace (no device allocation) gives the results of caspar_ba_create on
the same inputs, on two calls in a row (the second problem smaller) and on a
third with a robust loss (its IRLS weights live in the workspace too), and
refuses a second static handle on the same GPU and problems beyond the
array's size."""
import ctypes as C
import json
import os

import numpy as np
import pytest

from synth import make_scene, scene_config

from gpu_helpers import handle_for, observed_pixels, rel, t32i, t64

pytestmark = pytest.mark.gpu

GOLDEN = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "lm_reference.json")))["runs"]


def _static_handle(sc, px, precision, rj):
    from paper_2605_30583_amd import BundleAdjuster
    return BundleAdjuster(t64(sc.cams_init), t64(sc.points_init), t32i(sc.obs_cam), t32i(sc.obs_pt), t64(px),
                          precision, recompute_jacobian=rj, static_workspace=True)


def _compare(sc, precision, rj, golden=None, loss=None):
    from paper_2605_30583_amd import SolveOptions
    px = observed_pixels(sc)
    a = _static_handle(sc, px, precision, rj)
    b = handle_for(sc, px, precision, rj=rj)
    try:
        if loss is not None:
            a.set_loss(*loss)
            b.set_loss(*loss)
        la, lb = a.linearize(), b.linearize()
        assert abs(la["cost"] - lb["cost"]) <= 1e-12 * lb["cost"]
        for k in ("resid", "jac_cam", "jac_pt", "grad", "diag"):
            assert rel(la[k].cpu(), lb[k].cpu()) <= 1e-12, k
        p = t64(np.random.default_rng(5).normal(size=a.n_params))
        wa, papa = a.matvec(1e-2, p)
        wb, papb = b.matvec(1e-2, p)
        assert rel(wa.cpu(), wb.cpu()) <= 1e-12
        assert abs(papa - papb) <= 1e-12 * abs(papb)
        # converged runs (20 iterations, PCG to 1e-10): the final cost is the
        # optimum's, which rounding-order differences do not move
        opts = SolveOptions(max_lm_iters=20, pcg_tol=1e-10, max_pcg_iters=5000)
        sa, sb = a.solve(opts), b.solve(opts)
        assert abs(sa["final_cost"] - sb["final_cost"]) <= 1e-9 * sb["final_cost"]
        if golden is not None:
            assert abs(sa["final_cost"] - golden["final_cost"]) <= 1e-9 * golden["final_cost"]
        from paper_2605_30583_amd import project
        ca, pa = a.get_params()
        cb, pb = b.get_params()
        ua = project(ca, pa, t32i(sc.obs_cam), t32i(sc.obs_pt)).cpu().numpy()
        ub = project(cb, pb, t32i(sc.obs_cam), t32i(sc.obs_pt)).cpu().numpy()
        assert rel(ua, ub) <= 1e-9
        return a
    finally:
        b.close()


def test_static_workspace_matches_create_on_two_calls():
    from paper_2605_30583_amd import _native
    lib = _native.load()
    a = _compare(scene_config("tiny"), 0, False, GOLDEN["tiny"])
    small = make_scene(8, 300, 17, k_values=(3, 4), k_probs=(0.5, 0.5))
    try:
        # the array is held: a second static handle on this GPU is refused
        with pytest.raises(_native.CasparError, match="held by another handle"):
            _static_handle(small, observed_pixels(small), 0, True)
    finally:
        a.close()
    # second call, smaller problem, other Jacobian mode, after the first released the array
    b = _compare(small, 0, True)
    b.close()
    # third call: a robust loss, whose weights (per observation and in the
    # product's step order) are in the array as well
    c = _compare(small, 0, True, loss=("huber", 1.0))
    c.close()
    # beyond the array's size: refused before any input is read
    h = C.c_void_p()
    st = lib.caspar_ba_create_static(C.byref(h), 1000, 10_000_000, 60_000_000, None, None, None, None, None, 0,
                                     None)
    assert st == -3 and not h.value          # CASPAR_ENOMEM
    assert b"static workspace holds" in lib.caspar_last_error()
