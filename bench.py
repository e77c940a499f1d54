#!/usr/bin/env python3
"""Throughput of the bundle-adjustment hot path on one MI355X.

One step = one Levenberg-Marquardt iteration of the whole hot path on the
synthetic BAL-shaped workload: linearisation (residuals, Jacobian blocks,
cost, gradient, block sums), block-Jacobi preconditioner, the PCG solve
with the fused normal-equation products, retraction and trial cost, and the
accept/reject update.  W untimed iterations run first (from the initial
values), then the parameters are reset and exactly K iterations are timed
(early stopping off), with inputs resident in HBM.

The headline recomputes the Jacobian blocks inside every normal-equation
product (--jacobian recompute); the run with stored blocks follows it, then
the same solve with a Huber loss (robust re-weighting, scale 3 px).

Printed: one JSON line with LM iterations/s (value), the roofline of the
fused product (its average duration measured with HIP events on the
library's stream during the timed solve: priced on flops when the blocks are
recomputed, on HBM bytes when they are stored), the float64 plain solve
beside the float32-mixed one with the cost error between them, the other
Jacobian handling, the implicit-adjoint backward time, and the float64 CPU
oracle timed on a bounded sample.

    python bench.py [--gpus 1] [--steps 10] [--warmup 2]
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
HBM_PEAK_GBS = 8000.0
# Float32 / float64 vector FMA issue without packed math (the library is
# compiled without packed float32): 256 CUs x 4 SIMDs x 16 lanes x 2 flop x 2.4 GHz.
ALU_PEAK_TFLOPS = 256 * 4 * 16 * 2 * 2.4e9 / 1e12
# Algorithmic flops of the fused product per observation (FMA = 2).
# Stored blocks: q = J p (48), J_c^T q and J_p^T q (36), |q|^2 and the
# camera and point sums (16): 100.  Recomputed blocks, applied in factored
# form without forming them: R from the camera's unit quaternion (24); P,
# the projection, distortion and the 2x3 chain factor B (51); q = B (R (p_X +
# p_w x X) + p_t) + calibration term (50); B^T q, R^T B^T q, X x R^T B^T q,
# the calibration transposes and q.q (43); the sums as with stored blocks
# (16): 184.
FLOPS_PER_OBS = {"recompute": 184.0, "stored": 100.0}
PROFILES = os.path.join(ROOT, "profiles")


def parse():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10, help="timed LM iterations")
    ap.add_argument("--warmup", type=int, default=2, help="untimed LM iterations")
    ap.add_argument("--workload", default="large_zipf",
                    choices=["tiny", "medium", "bal1700", "large_zipf"])
    ap.add_argument("--precision", default="fp32_mixed", choices=["fp32_mixed", "fp64"])
    ap.add_argument("--pcg-tol", type=float, default=1e-3, help="PCG relative tolerance (paper: 1e-3)")
    ap.add_argument("--jacobian", default="recompute", choices=["stored", "recompute"],
                    help="store the Jacobian blocks at linearisation or evaluate them in every product")
    ap.add_argument("--no-alt-jacobian", action="store_true",
                    help="skip the run with the other Jacobian handling beside the headline one")
    ap.add_argument("--no-fp64", action="store_true", help="skip the float64 plain solve beside the mixed one")
    ap.add_argument("--no-adjoint", action="store_true")
    ap.add_argument("--no-robust", action="store_true", help="skip the Huber-loss solve beside the headline")
    ap.add_argument("--robust-scale", type=float, default=3.0, help="Huber scale in pixels")
    ap.add_argument("--no-between", action="store_true",
                    help="skip the solve with pose between-factors (camera chain plus loop closures)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-sample-points", type=int, default=150_000)
    ap.add_argument("--time-every", type=int, default=4,
                    help="HIP events around every k-th launch of the fused product (each pair idles the GPU a "
                         "few microseconds)")
    ap.add_argument("--copy-calibration-mib", type=int, default=0,
                    help="run one plain device copy of this many MiB first (counter calibration)")
    return ap.parse_args()


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def kernel_source_hash() -> str:
    h = hashlib.sha256()
    for f in ("matvec.hip", "model.hpp", "common.hpp"):
        h.update(open(os.path.join(ROOT, "paper_2605_30583_amd", "csrc", f), "rb").read())
    return h.hexdigest()[:16]


def counter_traffic(workload: str, precision: str, jacobian: str):
    """HBM bytes per fused-product launch from the committed rocprofv3
    counter summary, if it was taken on the current kernel source."""
    path = os.path.join(PROFILES, f"matvec_{workload}_{precision}_{jacobian}_counters.json")
    if not os.path.exists(path):
        return None
    rec = json.load(open(path))
    if rec.get("kernel_source_hash") != kernel_source_hash():
        return None
    return rec.get("hbm_bytes_per_launch")


def measure_copy(torch, dev, mib: int = 1024, reps: int = 10):
    """Rate of a plain device-to-device copy (read + write bytes), the
    practical HBM ceiling the bandwidth-bound kernels are compared with."""
    n = (mib << 20) // 4
    src = torch.ones(n, dtype=torch.float32, device=dev)
    dst = torch.empty_like(src)
    dst.copy_(src)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        dst.copy_(src)
    e1.record()
    torch.cuda.synchronize()
    gbs = 2.0 * 4 * n * reps / (e0.elapsed_time(e1) * 1e-3) / 1e9
    del src, dst
    torch.cuda.empty_cache()
    return {"what": f"device-to-device copy of a {mib} MiB float32 tensor, {reps} repetitions, "
                    "read plus written bytes over HIP event time", "gbs": gbs, "frac_of_peak": gbs / HBM_PEAK_GBS}


def cpu_baseline(sc, n_points: int, pcg_tol: float):
    """The oracle (float64, NumPy/SciPy, unchanged) on a bounded sample: the
    first n_points points with all their observations, one LM iteration with
    the same PCG inner solve; scaled to the full workload by observations."""
    from oracle import camera, lm
    m = sc.obs_pt < n_points
    oc, op = sc.obs_cam[m], sc.obs_pt[m]
    st_true = camera.State.from_bal(sc.cams_true, sc.points_true[:n_points])
    px = camera.project(st_true, oc, op) + sc.noise[m]
    st = camera.State.from_bal(sc.cams_init, sc.points_init[:n_points])
    try:
        from threadpoolctl import threadpool_info
        blas = max([i.get("num_threads", 1) for i in threadpool_info()] or [1])
    except Exception:
        blas = 1
    t = time.perf_counter()
    lm.solve(st, oc, op, px, lm.LMOptions(max_iters=1, inner="pcg", pcg_tol=pcg_tol))
    dt = time.perf_counter() - t
    frac = float(m.sum()) / sc.n_obs
    # the oracle's sparse product (J^T (J p) + lambda D p) on the same sample,
    # priced on the bytes the method must move (float64 B_mv)
    from oracle import linear
    _, Jc, Jp = camera.linearize(st, oc, op, px)
    J = linear.jacobian_csr(Jc, Jp, oc, op, sc.n_cams, n_points)
    D = linear.damping_diagonal(J)
    p = np.random.default_rng(0).normal(size=J.shape[1])
    times = []
    for _ in range(3):
        t = time.perf_counter()
        linear.matvec(J, D, 1e-2, p)
        times.append(time.perf_counter() - t)
    b_mv = float(m.sum()) * (24 * 8 + 8) + 3 * 8 * J.shape[1]
    return {
        "value": frac / dt,
        "unit": "LM iterations/s",
        "cores": int(blas),
        "kind": "oracle",
        "sample": (f"1 LM iteration (PCG inner, tol {pcg_tol:g}) on the first {n_points} points and their "
                   f"{int(m.sum())} observations ({100 * frac:.2f}% of the workload) in {dt:.1f} s; rate scaled "
                   f"by the observation fraction; sparse products run on one thread, BLAS on {blas}"),
        "matvec_gbs": b_mv / float(np.median(times)) / 1e9,
        "matvec_sample": "the oracle's sparse product on the same sample, float64 B_mv bytes over the median of 3 runs",
    }


def between_inputs(sc, rot_sigma=2e-3, trans_sigma=1e-2):
    """Pose between-factors for the workload: pairs and noise draws from synth,
    measured relative poses T_j T_i^-1 of the true cameras perturbed on the
    right by Exp(rot_sigma n) and in translation by trans_sigma n (SciPy's
    rotation-vector maps for the angle-axis conversions)."""
    from scipy.spatial.transform import Rotation
    from synth import between_draws
    d = between_draws(sc.n_cams, 21, sc.n_cams // 8)
    R = Rotation.from_rotvec(sc.cams_true[:, 0:3]).as_matrix()
    t = sc.cams_true[:, 3:6]
    Rij = R[d.fj] @ np.swapaxes(R[d.fi], 1, 2)
    ZR = Rij @ Rotation.from_rotvec(rot_sigma * d.rot_noise).as_matrix()
    Zt = t[d.fj] - np.einsum("kab,kb->ka", Rij, t[d.fi]) + trans_sigma * d.trans_noise
    Z = np.concatenate([Rotation.from_matrix(ZR).as_rotvec(), Zt], axis=1)
    w = np.tile([1.0 / rot_sigma, 1.0 / trans_sigma], (d.fi.shape[0], 1))
    return d.fi, d.fj, Z, w


def main():
    a = parse()
    if a.gpus != 1:
        print(f"bench.py measures one GPU; --gpus {a.gpus} is not supported (the library runs on a single GPU)",
              file=sys.stderr)
        sys.exit(2)
    import torch
    from paper_2605_30583_amd import FP32_MIXED, FP64, BundleAdjuster, SolveOptions, project
    from synth import scene_config

    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    if a.copy_calibration_mib > 0:
        n = a.copy_calibration_mib << 20
        src = torch.ones(n // 4, dtype=torch.float32, device=dev)
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        log(f"calibration copy: {n} bytes read, {n} bytes written")
        del src, dst
    copy = measure_copy(torch, dev)
    log(f"device copy: {copy['gbs']:.0f} GB/s")
    t = time.time()
    sc = scene_config(a.workload)
    log(f"scene {a.workload}: {sc.n_cams} cameras, {sc.n_points} points, {sc.n_obs} observations "
        f"({time.time() - t:.1f}s)")

    def t64(x):
        return torch.from_numpy(np.ascontiguousarray(x, dtype=np.float64)).to(dev)

    def t32(x):
        return torch.from_numpy(np.ascontiguousarray(x, dtype=np.int32)).to(dev)

    oc, op = t32(sc.obs_cam), t32(sc.obs_pt)
    px = project(t64(sc.cams_true), t64(sc.points_true), oc, op) + t64(sc.noise)
    cams0, pts0 = t64(sc.cams_init), t64(sc.points_init)
    prec = FP32_MIXED if a.precision == "fp32_mixed" else FP64

    create_s = {}

    def timed_solve(precision, label, jacobian=a.jacobian, loss=None, between=None):
        t = time.perf_counter()
        ba = BundleAdjuster(cams0, pts0, oc, op, px, precision, recompute_jacobian=(jacobian == "recompute"))
        torch.cuda.synchronize()
        create_s[label] = time.perf_counter() - t
        if loss is not None:
            ba.set_loss(*loss)
        if between is not None:
            ba.set_between(*between)
        torch.cuda.synchronize()
        log(f"{label}: create {create_s[label]:.2f}s, layout {ba.layout_info()}")
        if a.warmup > 0:
            ba.solve(SolveOptions(max_lm_iters=a.warmup, pcg_tol=a.pcg_tol))
            ba.set_params(cams0, pts0)
        opts = SolveOptions(max_lm_iters=a.steps, pcg_tol=a.pcg_tol, grad_tol=0.0, min_cost=0.0)
        ba.set_timing(True, every=a.time_every)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        st = ba.solve(opts, history=True)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        tim = ba.get_timing()
        ba.set_timing(False)
        log(f"{label}: {st['lm_iters']} LM iterations in {dt:.3f}s, PCG {st['pcg_iters_total']}, "
            f"F {st['initial_cost']:.6e} -> {st['final_cost']:.6e}")
        return ba, st, dt, tim

    def time_to_accuracy(handle, st, target, label):
        """First timed iteration k whose parameters have a float64 cost within
        1e-9 of target (the float64 run's final cost).  Costs come from
        re-runs of k iterations from the same start, re-evaluated in float64
        (accepted costs never increase, so k is found by bisection); the time
        to reach k is the timed run's host clock at the end of iteration k."""
        hist = st["history"]
        thr = target * (1.0 + 1e-9)

        def f64_at(k):
            handle.set_params(cams0, pts0)
            handle.solve(SolveOptions(max_lm_iters=k, pcg_tol=a.pcg_tol, grad_tol=0.0, min_cost=0.0))
            return handle.cost_fp64()

        lo, hi = 1, len(hist)
        if hi == 0 or f64_at(hi) > thr:
            return {"reached": False, "within": 1e-9, "of": "float64 run's final cost"}
        while lo < hi:
            mid = (lo + hi) // 2
            if f64_at(mid) <= thr:
                hi = mid
            else:
                lo = mid + 1
        sec = hist[lo - 1]["seconds"]
        log(f"{label}: cost within 1e-9 of the float64 final at iteration {lo}, {sec:.3f}s")
        return {"reached": True, "iteration": lo, "seconds": sec, "lm_iters_per_s": lo / sec, "within": 1e-9,
                "of": "float64 run's final cost",
                "how": "float64 cost of re-runs of k iterations from the same start (bisection over k); seconds "
                       "from the timed run's per-iteration host clock"}

    ba, st, dt, tim = timed_solve(prec, a.precision)
    iters = st["lm_iters"]
    value = iters / dt
    mv_avg_ms = tim["matvec_ms"] / max(1, tim["matvec_launches"])
    gbs = tim["matvec_bytes"] / (mv_avg_ms * 1e-3) / 1e9 if tim["matvec_launches"] else None
    tflops = FLOPS_PER_OBS[a.jacobian] * sc.n_obs / (mv_avg_ms * 1e-3) / 1e12 if tim["matvec_launches"] else None
    f_primary = ba.cost_fp64()

    extra = {}
    f_ref = None
    if prec == FP32_MIXED and not a.no_fp64:
        ba64, st64, dt64, tim64 = timed_solve(FP64, "fp64")
        f64 = ba64.cost_fp64()
        f_ref = f64
        mv64 = tim64["matvec_ms"] / max(1, tim64["matvec_launches"])
        extra["fp64"] = {
            "lm_iters_per_s": st64["lm_iters"] / dt64,
            "final_cost": f64,
            "pcg_iters_total": st64["pcg_iters_total"],
            "matvec_avg_ms": mv64,
            "matvec_gbs": tim64["matvec_bytes"] / (mv64 * 1e-3) / 1e9 if tim64["matvec_launches"] else None,
        }
        extra["fp32_mixed_cost_rel_error_vs_fp64"] = (f_primary - f64) / f64
        extra["fp64"]["time_to_accuracy"] = time_to_accuracy(ba64, st64, f_ref, "fp64")
        del ba64
        torch.cuda.empty_cache()

    if not a.no_alt_jacobian:
        alt = "recompute" if a.jacobian == "stored" else "stored"
        ba_alt, st_alt, dt_alt, tim_alt = timed_solve(prec, f"{a.precision}/{alt}", jacobian=alt)
        mv_alt = tim_alt["matvec_ms"] / max(1, tim_alt["matvec_launches"])
        gbs_alt = tim_alt["matvec_bytes"] / (mv_alt * 1e-3) / 1e9
        extra[f"{alt}_jacobian"] = {
            "lm_iters_per_s": st_alt["lm_iters"] / dt_alt,
            "ms_per_step": 1e3 * dt_alt / max(1, st_alt["lm_iters"]),
            "final_cost_fp64_eval": ba_alt.cost_fp64(),
            "pcg_iters_total": st_alt["pcg_iters_total"],
            "matvec_avg_ms": mv_alt,
            "matvec_algorithmic_bytes": tim_alt["matvec_bytes"],
            "matvec_gbs": gbs_alt,
            "matvec_hbm_frac": gbs_alt / HBM_PEAK_GBS,
            "matvec_frac_of_copy": gbs_alt / copy["gbs"],
            "matvec_tflops": FLOPS_PER_OBS[alt] * sc.n_obs / (mv_alt * 1e-3) / 1e12,
        }
        if f_ref is not None:
            extra[f"{alt}_jacobian"]["time_to_accuracy"] = time_to_accuracy(ba_alt, st_alt, f_ref,
                                                                             f"{a.precision}/{alt}")
        del ba_alt
        torch.cuda.empty_cache()

    if not a.no_robust:
        ba_r, st_r, dt_r, tim_r = timed_solve(prec, f"{a.precision}/huber", loss=("huber", a.robust_scale))
        mv_r = tim_r["matvec_ms"] / max(1, tim_r["matvec_launches"])
        extra["huber_loss"] = {
            "scale_px": a.robust_scale,
            "lm_iters_per_s": st_r["lm_iters"] / dt_r,
            "ms_per_step": 1e3 * dt_r / max(1, st_r["lm_iters"]),
            "pcg_iters_total": st_r["pcg_iters_total"],
            "matvec_avg_ms": mv_r,
            "final_robust_cost_fp64_eval": ba_r.cost_fp64(),
        }
        del ba_r
        torch.cuda.empty_cache()

    if not a.no_between:
        bf = between_inputs(sc)
        ba_b, st_b, dt_b, tim_b = timed_solve(prec, f"{a.precision}/between", between=bf)
        extra["between_factors"] = {
            "factors": int(bf[0].shape[0]),
            "recipe": "chain (c, c+1) over the cameras plus n_cams/8 random loop closures; measured relative "
                      "poses from the true cameras with 2e-3 rad / 1e-2 noise, weights 1/sigma",
            "lm_iters_per_s": st_b["lm_iters"] / dt_b,
            "ms_per_step": 1e3 * dt_b / max(1, st_b["lm_iters"]),
            "pcg_iters_total": st_b["pcg_iters_total"],
            "matvec_avg_ms": tim_b["matvec_ms"] / max(1, tim_b["matvec_launches"]),
            "final_cost_fp64_eval": ba_b.cost_fp64(),
        }
        del ba_b
        torch.cuda.empty_cache()

    if not a.no_adjoint:
        # backward at the headline solve's optimum (its own precision), then
        # the same backward in float64 at the same parameters as its reference
        cams_s, pts = ba.get_params()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        g = ba.backward(None, 2.0 * pts, lambda_adj=1e-4, pcg_tol=1e-6, max_pcg_iters=500)
        torch.cuda.synchronize()
        extra["adjoint"] = {"ms": 1e3 * (time.perf_counter() - t0), "pcg_iters": ba.last_backward_iters,
                            "pcg_rel_resid": ba.last_backward_rel_resid, "lambda_adj": 1e-4, "pcg_tol": 1e-6,
                            "loss": "sum of squared optimal point coordinates", "grad_norm": float(g.norm())}
        if prec == FP32_MIXED and not a.no_fp64:
            ba_ref = BundleAdjuster(cams_s, pts, oc, op, px, FP64, recompute_jacobian=True)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            g64 = ba_ref.backward(None, 2.0 * pts, lambda_adj=1e-4, pcg_tol=1e-10, max_pcg_iters=5000)
            torch.cuda.synchronize()
            extra["adjoint"]["fp64_reference"] = {
                "ms": 1e3 * (time.perf_counter() - t0), "pcg_iters": ba_ref.last_backward_iters,
                "pcg_tol": 1e-10, "pcg_rel_resid": ba_ref.last_backward_rel_resid}
            extra["adjoint"]["rel_error_vs_fp64"] = float((g - g64).norm() / g64.norm())
            log(f"adjoint: float32-mixed vs float64 relative error {extra['adjoint']['rel_error_vs_fp64']:.3e}")
            del ba_ref, g64
            torch.cuda.empty_cache()

    if f_ref is not None:
        # after the adjoint, which needs the headline handle at its optimum
        tta = time_to_accuracy(ba, st, f_ref, a.precision)
    else:
        tta = None

    if a.jacobian == "stored":
        # the blocks stream from HBM: priced on the bytes the product must move
        roofline = {"bound": "hbm", "achieved": gbs, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                    "frac": gbs / HBM_PEAK_GBS if gbs else None}
    else:
        # the blocks are evaluated in every product: priced on its flops
        roofline = {"bound": "alu", "achieved": tflops, "peak": ALU_PEAK_TFLOPS, "unit": "TFLOP/s",
                    "frac": tflops / ALU_PEAK_TFLOPS if tflops else None}
    roofline.update({
        "traffic": counter_traffic(a.workload, a.precision, a.jacobian),
        "kernel": "k_matvec_lanes" if a.jacobian == "recompute" else "k_matvec",
        "avg_ms": mv_avg_ms,
        "launches": tim["matvec_launches"],
        "timed_every": a.time_every,
        "algorithmic_bytes_per_launch": tim["matvec_bytes"],
        "algorithmic_flops_per_launch": FLOPS_PER_OBS[a.jacobian] * sc.n_obs,
        "hbm_gbs": gbs,
    })
    line = {
        "metric": "LM iterations/sec + PCG matvec HBM GB/s, FP32-mixed vs FP64 at stated cost error",
        "value": value,
        "unit": "LM iterations/s",
        "n_gpus": 1,
        "steps": iters,
        "warmup": a.warmup,
        "ms_per_step": 1e3 * dt / max(1, iters),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32" if prec == FP32_MIXED else "f64",
        "data": "synthetic",
        "config": {
            "workload": a.workload,
            "n_cams": sc.n_cams, "n_points": sc.n_points, "n_obs": sc.n_obs,
            "precision": a.precision, "jacobian": a.jacobian, "pcg_tol": a.pcg_tol,
            "pcg_iters_per_lm_iter": st["pcg_iters_total"] / max(1, iters),
            "accepted": st["accepted"],
            "final_cost_fp64_eval": f_primary,
            "parallelism": "single GPU",
        },
        "create_seconds": create_s[a.precision],
        "time_to_accuracy": tta,
        "roofline": roofline,
    }
    line["hbm_copy"] = copy
    line.update(extra)
    if not a.no_cpu_baseline:
        log("cpu baseline: oracle on a bounded sample")
        line["cpu_baseline"] = cpu_baseline(sc, a.cpu_sample_points, a.pcg_tol)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
