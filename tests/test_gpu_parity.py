"""Parity of the HIP path (through the C ABI) with the float64 oracle on the
same seeded inputs: projection, linearisation, the fused normal-equation
product, the block-Jacobi preconditioner and PCG (Section V steps)."""
import numpy as np
import pytest

from oracle import camera, linear, pcg as opcg
from synth import scene_config

from gpu_helpers import handle_for, observed_pixels, oracle_lin, ragged_scene, rel, t32i, t64

pytestmark = pytest.mark.gpu

SCENES = {
    "tiny": lambda: scene_config("tiny"),
    "ragged": ragged_scene,
    "tiny_shuffled": lambda: scene_config("tiny").shuffled(3),
}


@pytest.fixture(scope="module", params=[(s, rj) for rj in (False, True) for s in SCENES],
                ids=lambda p: f"{p[0]}-{'recompute' if p[1] else 'stored'}")
def case(request):
    name, rj = request.param
    sc = SCENES[name]()
    px = observed_pixels(sc)
    ba = handle_for(sc, px, rj=rj)
    ref = oracle_lin(sc, px)
    yield name, sc, px, ba, ref
    ba.close()


def test_project_matches_oracle():
    from paper_2605_30583_amd import project
    sc = ragged_scene()
    rng = np.random.default_rng(0)
    cams = sc.cams_init.copy()
    cams[:, 7:9] = rng.normal(0, 0.05, size=(sc.n_cams, 2))
    u = project(t64(cams), t64(sc.points_init), t32i(sc.obs_cam), t32i(sc.obs_pt)).cpu().numpy()
    ref = camera.project(camera.State.from_bal(cams, sc.points_init), sc.obs_cam, sc.obs_pt)
    assert rel(u, ref) <= 1e-14


def test_params_roundtrip(case):
    name, sc, px, ba, ref = case
    cams, pts = ba.get_params()
    cams, pts = cams.cpu().numpy(), pts.cpu().numpy()
    np.testing.assert_allclose(pts, sc.points_init, rtol=0, atol=0)
    R = camera.so3_exp(cams[:, :3])
    np.testing.assert_allclose(R, ref.state.R, atol=1e-14)
    np.testing.assert_allclose(cams[:, 3:], sc.cams_init[:, 3:], rtol=0, atol=0)


def test_linearize_matches_oracle(case):
    name, sc, px, ba, ref = case
    out = ba.linearize()
    assert abs(out["cost"] - ref.cost) <= 1e-12 * ref.cost
    assert rel(out["resid"].cpu(), ref.r) <= 1e-11
    assert rel(out["jac_cam"].cpu(), ref.Jc) <= 1e-12
    assert rel(out["jac_pt"].cpu(), ref.Jp) <= 1e-12
    assert rel(out["grad"].cpu(), ref.g) <= 1e-12
    assert rel(out["diag"].cpu(), ref.D) <= 1e-12
    assert abs(ba.cost_fp64() - ref.cost) <= 1e-12 * ref.cost


@pytest.mark.parametrize("lam", [1e-6, 1e-2, 1e2])
def test_matvec_matches_oracle(case, lam):
    name, sc, px, ba, ref = case
    rng = np.random.default_rng(42)
    p = rng.normal(size=9 * sc.n_cams + 3 * sc.n_points)
    w, pap = ba.matvec(lam, t64(p))
    w_ref = linear.matvec(ref.J, ref.D, lam, p)
    assert rel(w.cpu(), w_ref) <= 1e-12
    assert abs(pap - p @ w_ref) <= 1e-12 * abs(p @ w_ref)


@pytest.mark.parametrize("lam", [1e-4, 1.0])
def test_block_jacobi_matches_oracle(case, lam):
    name, sc, px, ba, ref = case
    r = np.random.default_rng(7).normal(size=9 * sc.n_cams + 3 * sc.n_points)
    z = ba.block_jacobi_apply(lam, t64(r)).cpu().numpy()
    Mc, Mp = linear.block_jacobi_inverse(ref.J, ref.D, lam, sc.n_cams, sc.n_points)
    assert rel(z, linear.apply_block_jacobi(Mc, Mp, r)) <= 1e-12


@pytest.mark.parametrize("lam,tol", [(1e-2, 1e-6), (1e-4, 1e-10)])
def test_pcg_matches_oracle(case, lam, tol):
    name, sc, px, ba, ref = case
    b = -ref.g
    x, iters, relres = ba.pcg(lam, t64(b), tol, 500)
    x = x.cpu().numpy()
    Mc, Mp = linear.block_jacobi_inverse(ref.J, ref.D, lam, sc.n_cams, sc.n_points)
    xo, ro, ko, why = opcg.pcg(ref.J, ref.D, lam, b, Mc, Mp, tol, 500)
    assert why == "converged"
    # the stopping rule, checked with the oracle's product
    true_res = np.linalg.norm(b - linear.matvec(ref.J, ref.D, lam, x)) / np.linalg.norm(b)
    assert true_res <= 1.05 * tol + 1e-13
    assert abs(iters - ko) <= 1
    assert rel(x, xo) <= max(10 * tol, 1e-9)


def test_shuffled_observations_give_identical_products():
    sc = scene_config("tiny")
    px = observed_pixels(sc)
    sh = sc.shuffled(11)
    pxs = observed_pixels(sh)
    a, b = handle_for(sc, px), handle_for(sh, pxs)
    p = np.random.default_rng(5).normal(size=9 * sc.n_cams + 3 * sc.n_points)
    wa, pa = a.matvec(1e-3, t64(p))
    wb, pb = b.matvec(1e-3, t64(p))
    assert rel(wb.cpu(), wa.cpu()) <= 1e-13
    assert abs(a.linearize()["cost"] - b.linearize()["cost"]) <= 1e-13 * a.linearize()["cost"]


def test_layout_of_ragged_scene():
    sc = ragged_scene()
    ba = handle_for(sc, observed_pixels(sc))
    info = ba.layout_info()
    assert info["hot_cams"] == sc.n_cams and info["cold_obs"] == 0
    assert info["n_tiles"] >= 2


def test_create_rejects_bad_inputs():
    from paper_2605_30583_amd._native import CasparError
    sc = scene_config("tiny")
    px = observed_pixels(sc)
    bad = sc.obs_cam.copy()
    bad[5] = sc.n_cams
    with pytest.raises(CasparError, match="EINVAL"):
        from paper_2605_30583_amd import BundleAdjuster
        BundleAdjuster(t64(sc.cams_init), t64(sc.points_init), t32i(bad), t32i(sc.obs_pt), t64(px))
    pxn = px.copy()
    pxn[7, 1] = np.nan
    with pytest.raises(CasparError, match="EINVAL"):
        handle_for(sc, pxn)


@pytest.mark.parametrize("rj", [False, True])
@pytest.mark.parametrize("zipf", [None, 0.9])
def test_cold_camera_rows_and_full_lds(zipf, rj):
    # more cameras than the LDS holds: the least observed ones go through rows
    from synth import make_scene
    sc = make_scene(2300, 6000, 17, k_values=(2, 3, 4), k_probs=(0.3, 0.4, 0.3), zipf_s=zipf)
    px = observed_pixels(sc)
    ba = handle_for(sc, px, rj=rj)
    info = ba.layout_info()
    assert info["hot_cams"] == 2048 and info["cold_obs"] > 0      # float64: 2048 cameras in LDS
    ref = oracle_lin(sc, px)
    out = ba.linearize()
    assert rel(out["grad"].cpu(), ref.g) <= 1e-12
    assert rel(out["diag"].cpu(), ref.D) <= 1e-12
    p = np.random.default_rng(9).normal(size=9 * sc.n_cams + 3 * sc.n_points)
    for lam in (1e-6, 1.0):
        w, pap = ba.matvec(lam, t64(p))
        w_ref = linear.matvec(ref.J, ref.D, lam, p)
        assert rel(w.cpu(), w_ref) <= 1e-12
        assert abs(pap - p @ w_ref) <= 1e-12 * abs(p @ w_ref)


@pytest.mark.parametrize("rj", [False, True])
def test_mixed_precision_cold_rows_and_products(rj):
    # float32-mixed with cameras outside the LDS set; Zipf-skewed visibility
    # with points grouped by their least observed camera, so several
    # observations of one cold camera share a tile and a row
    from synth import make_scene
    sc = make_scene(5000, 20000, 19, k_values=(3, 4), k_probs=(0.5, 0.5), zipf_s=0.8)
    px = observed_pixels(sc)
    ba = handle_for(sc, px, precision=1, rj=rj)
    info = ba.layout_info()
    assert info["hot_cams"] == 2048 and info["cold_obs"] > 0
    ref = oracle_lin(sc, px)
    lin = ba.linearize()
    assert abs(lin["cost"] - ref.cost) <= 1e-6 * ref.cost
    assert rel(lin["jac_cam"].cpu(), ref.Jc) <= 1e-5
    p = np.random.default_rng(9).normal(size=9 * sc.n_cams + 3 * sc.n_points)
    w, pap = ba.matvec(1e-2, t64(p))
    w_ref = linear.matvec(ref.J, ref.D, 1e-2, p)
    assert rel(w.cpu(), w_ref) <= 2e-5
    assert abs(pap - p @ w_ref) <= 2e-5 * abs(p @ w_ref)


@pytest.mark.parametrize("precision", [0, 1], ids=["fp64", "fp32_mixed"])
@pytest.mark.parametrize("rj", [False, True], ids=["stored", "recompute"])
def test_product_repeats_to_rounding(rj, precision):
    """The hot-camera and window sums are LDS atomic adds in the order the
    waves reach them, so repeated products may differ in the camera entries
    at the rounding level: float64 sums of at most a few thousand terms (bar
    1e-13), and in the float32-mixed form the rounding of each workgroup's
    float64 sum to float32 can move by one unit in the last place (bar 1e-6).
    The point entries are summed in registers or by fixed-order scans and
    split rows, so they repeat bit for bit."""
    from synth import make_scene
    sc = make_scene(2300, 6000, 17, k_values=(2, 3, 4), k_probs=(0.3, 0.4, 0.3), zipf_s=0.9)
    px = observed_pixels(sc)
    ba = handle_for(sc, px, precision=precision, rj=rj)
    assert ba.layout_info()["cold_obs"] > 0
    ba.linearize(outputs=False)
    p = t64(np.random.default_rng(13).normal(size=9 * sc.n_cams + 3 * sc.n_points))
    ws = [ba.matvec(1e-2, p)[0].cpu().numpy() for _ in range(5)]
    nc9 = 9 * sc.n_cams
    bar = 1e-13 if precision == 0 else 1e-6
    for w in ws[1:]:
        assert np.array_equal(w[nc9:], ws[0][nc9:])
        assert rel(w[:nc9], ws[0][:nc9]) <= bar
    ba.close()
