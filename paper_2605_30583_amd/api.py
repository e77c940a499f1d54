"""torch-facing wrapper of the C ABI: argument marshalling only.

Tensors must live on the GPU, be contiguous and have the dtypes of the C
signatures (float64 parameters and pixels, int32 indices).  Every call runs
on torch's current stream of the handle's device.
"""
from __future__ import annotations

import ctypes as C
import dataclasses

import torch

from . import _native
from ._native import FP64, FP32_MIXED, RECOMPUTE_JACOBIAN, check

library_path = _native.LIB_PATH


def _ptr(t):
    return C.c_void_p(0 if t is None else t.data_ptr())


def _stream():
    return C.c_void_p(torch.cuda.current_stream().cuda_stream)


def _dev(t: torch.Tensor, dtype, shape=None, name="tensor") -> torch.Tensor:
    if not (t.is_cuda and t.dtype == dtype and t.is_contiguous()):
        raise ValueError(f"{name} must be a contiguous {dtype} CUDA tensor")
    if shape is not None and tuple(t.shape) != tuple(shape):
        raise ValueError(f"{name} must have shape {tuple(shape)}, got {tuple(t.shape)}")
    return t


@dataclasses.dataclass
class SolveOptions:
    lambda0: float = 1e-2
    pcg_tol: float = 1e-3
    max_lm_iters: int = 20
    max_pcg_iters: int = 500
    lambda_min: float = 1e-12
    lambda_max: float = 1e16
    grad_tol: float = 1e-12
    min_cost: float = 1e-30
    pcg_check_every: int = 4
    pred_tol: float = 0.0

    def to_c(self) -> _native.SolveOpts:
        o = _native.SolveOpts()
        for f in dataclasses.fields(self):
            setattr(o, f.name, getattr(self, f.name))
        o.flags = 0
        return o


def project(cams: torch.Tensor, points: torch.Tensor, obs_cam: torch.Tensor, obs_pt: torch.Tensor) -> torch.Tensor:
    """Predicted pixels [n_obs, 2] of the Snavely model (float64)."""
    lib = _native.load()
    nc, npnt, no = cams.shape[0], points.shape[0], obs_cam.shape[0]
    _dev(cams, torch.float64, (nc, 9), "cams")
    _dev(points, torch.float64, (npnt, 3), "points")
    _dev(obs_cam, torch.int32, (no,), "obs_cam")
    _dev(obs_pt, torch.int32, (no,), "obs_pt")
    out = torch.empty((no, 2), dtype=torch.float64, device=cams.device)
    check(lib.caspar_project(nc, npnt, no, _ptr(cams), _ptr(points), _ptr(obs_cam), _ptr(obs_pt), _ptr(out),
                             _stream()))
    return out


class BundleAdjuster:
    """One problem on one GPU (a caspar_ba handle plus its workspace)."""

    def __init__(self, cams, points, obs_cam, obs_pt, obs_px, precision: int = FP64,
                 recompute_jacobian: bool = False, static_workspace: bool = False):
        """static_workspace: build the handle on the library's static device
        array (caspar_ba_create_static) instead of a workspace allocated here;
        one such handle per GPU at a time, problems up to 256 MiB of workspace."""
        lib = _native.load()
        self._lib = lib
        self.n_cams, self.n_points, self.n_obs = int(cams.shape[0]), int(points.shape[0]), int(obs_cam.shape[0])
        self.device = cams.device
        self.precision = precision
        self.recompute_jacobian = bool(recompute_jacobian)
        mode = precision | (RECOMPUTE_JACOBIAN if recompute_jacobian else 0)
        _dev(cams, torch.float64, (self.n_cams, 9), "cams")
        _dev(points, torch.float64, (self.n_points, 3), "points")
        _dev(obs_cam, torch.int32, (self.n_obs,), "obs_cam")
        _dev(obs_pt, torch.int32, (self.n_obs,), "obs_pt")
        _dev(obs_px, torch.float64, (self.n_obs, 2), "obs_px")
        h = C.c_void_p()
        if static_workspace:
            self.workspace = None
            check(lib.caspar_ba_create_static(C.byref(h), self.n_cams, self.n_points, self.n_obs, _ptr(cams),
                                              _ptr(points), _ptr(obs_cam), _ptr(obs_pt), _ptr(obs_px), mode,
                                              _stream()))
            self._h = h
            return
        nbytes = lib.caspar_ba_workspace_bytes(self.n_cams, self.n_points, self.n_obs, mode)
        if nbytes == 0:
            raise ValueError("unsupported problem size or precision")
        self.workspace = torch.empty(nbytes + 256, dtype=torch.uint8, device=self.device)
        base = self.workspace.data_ptr()
        off = (-base) % 256
        self._ws_ptr = C.c_void_p(base + off)
        self._ws_bytes = nbytes
        check(lib.caspar_ba_create(C.byref(h), self.n_cams, self.n_points, self.n_obs, _ptr(cams), _ptr(points),
                                   _ptr(obs_cam), _ptr(obs_pt), _ptr(obs_px), mode, self._ws_ptr,
                                   self._ws_bytes, _stream()))
        self._h = h

    @property
    def n_params(self) -> int:
        return 9 * self.n_cams + 3 * self.n_points

    def close(self):
        if getattr(self, "_h", None):
            self._lib.caspar_ba_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _vec(self):
        return torch.empty(self.n_params, dtype=torch.float64, device=self.device)

    def set_between(self, cam_i, cam_j, meas, weights):
        """Pose between-factors (caspar_ba_set_between): camera pairs [n] (int32),
        measured relative poses [n, 6] (angle-axis, translation of T_j T_i^-1)
        and square-root weights [n, 2] (rotation, translation), host arrays or
        tensors.  An empty set removes them.  The device workspace they need
        is allocated here and kept with the adjuster."""
        import numpy as np

        def host(v, dt):
            v = v.detach().cpu().numpy() if isinstance(v, torch.Tensor) else v
            return np.ascontiguousarray(v, dtype=dt)

        ci, cj = host(cam_i, np.int32).ravel(), host(cam_j, np.int32).ravel()
        n = ci.shape[0]
        z, w = host(meas, np.float64).reshape(n, 6), host(weights, np.float64).reshape(n, 2)
        if cj.shape[0] != n:
            raise ValueError("cam_i and cam_j must have the same length")
        if n == 0:
            check(self._lib.caspar_ba_set_between(self._h, 0, None, None, None, None, None, 0))
            self._between_ws = None
            return
        nbytes = self._lib.caspar_ba_between_workspace_bytes(n, self.n_cams)
        ws = torch.empty(nbytes + 256, dtype=torch.uint8, device=self.device)
        ptr = ws.data_ptr() + (-ws.data_ptr()) % 256
        check(self._lib.caspar_ba_set_between(self._h, n, _host(ci), _host(cj), _host(z), _host(w), C.c_void_p(ptr),
                                              nbytes))
        self._between_ws = ws

    def solve(self, opts: SolveOptions | None = None, history: bool = False):
        opts = opts or SolveOptions()
        st = _native.SolveStats()
        hist = (_native.IterRecord * max(1, opts.max_lm_iters))() if history else None
        check(self._lib.caspar_ba_solve(self._h, C.byref(opts.to_c()), C.byref(st), hist))
        stats = {f: getattr(st, f) for f, _ in _native.SolveStats._fields_}
        if history:
            stats["history"] = [{f: getattr(hist[i], f) for f, _ in _native.IterRecord._fields_}
                                for i in range(st.lm_iters)]
        return stats

    def get_params(self):
        cams = torch.empty((self.n_cams, 9), dtype=torch.float64, device=self.device)
        pts = torch.empty((self.n_points, 3), dtype=torch.float64, device=self.device)
        check(self._lib.caspar_ba_get_params(self._h, _ptr(cams), _ptr(pts)))
        return cams, pts

    def set_params(self, cams=None, points=None):
        if cams is not None:
            _dev(cams, torch.float64, (self.n_cams, 9), "cams")
        if points is not None:
            _dev(points, torch.float64, (self.n_points, 3), "points")
        check(self._lib.caspar_ba_set_params(self._h, _ptr(cams), _ptr(points)))

    LOSSES = {"trivial": _native.LOSS_TRIVIAL, "huber": _native.LOSS_HUBER, "cauchy": _native.LOSS_CAUCHY}

    def set_loss(self, kind: str = "trivial", scale: float = 1.0):
        """Robust loss of the squared residual norm (caspar_ba_set_loss):
        "trivial", "huber" or "cauchy" with scale in pixels."""
        if kind not in self.LOSSES:
            raise ValueError(f"unknown loss {kind!r}; expected one of {sorted(self.LOSSES)}")
        check(self._lib.caspar_ba_set_loss(self._h, self.LOSSES[kind], float(scale)))

    def set_observations(self, obs_px):
        _dev(obs_px, torch.float64, (self.n_obs, 2), "obs_px")
        check(self._lib.caspar_ba_set_observations(self._h, _ptr(obs_px)))

    def linearize(self, outputs=True):
        cost = C.c_double()
        if not outputs:
            check(self._lib.caspar_ba_linearize(self._h, C.byref(cost), None, None, None, None, None))
            return {"cost": cost.value}
        dev, no = self.device, self.n_obs
        r = torch.empty((no, 2), dtype=torch.float64, device=dev)
        jc = torch.empty((no, 2, 9), dtype=torch.float64, device=dev)
        jp = torch.empty((no, 2, 3), dtype=torch.float64, device=dev)
        g, d = self._vec(), self._vec()
        check(self._lib.caspar_ba_linearize(self._h, C.byref(cost), _ptr(r), _ptr(jc), _ptr(jp), _ptr(g), _ptr(d)))
        return {"cost": cost.value, "resid": r, "jac_cam": jc, "jac_pt": jp, "grad": g, "diag": d}

    def matvec(self, lam: float, p: torch.Tensor):
        _dev(p, torch.float64, (self.n_params,), "p")
        w = self._vec()
        pap = C.c_double()
        check(self._lib.caspar_ba_matvec(self._h, float(lam), _ptr(p), _ptr(w), C.byref(pap)))
        return w, pap.value

    def block_jacobi_apply(self, lam: float, r: torch.Tensor):
        _dev(r, torch.float64, (self.n_params,), "r")
        z = self._vec()
        check(self._lib.caspar_ba_block_jacobi_apply(self._h, float(lam), _ptr(r), _ptr(z)))
        return z

    def pcg(self, lam: float, b: torch.Tensor, tol: float, max_iters: int):
        _dev(b, torch.float64, (self.n_params,), "b")
        x = self._vec()
        it = C.c_int32()
        rel = C.c_double()
        check(self._lib.caspar_ba_pcg(self._h, float(lam), _ptr(b), float(tol), int(max_iters), _ptr(x),
                                      C.byref(it), C.byref(rel)))
        return x, it.value, rel.value

    def cost_fp64(self) -> float:
        c = C.c_double()
        check(self._lib.caspar_ba_cost_fp64(self._h, C.byref(c)))
        return c.value

    def backward(self, grad_cams=None, grad_points=None, lambda_adj=1e-4, pcg_tol=1e-10, max_pcg_iters=2000,
                 gauge_project=False):
        """dL/dpx (caspar_ba_backward).  The adjoint PCG's iteration count and
        relative residual are kept in last_backward_iters and
        last_backward_rel_resid; a solve that stopped at max_pcg_iters above
        pcg_tol raises a RuntimeWarning."""
        if grad_cams is not None:
            _dev(grad_cams, torch.float64, (self.n_cams, 9), "grad_cams")
        if grad_points is not None:
            _dev(grad_points, torch.float64, (self.n_points, 3), "grad_points")
        out = torch.empty((self.n_obs, 2), dtype=torch.float64, device=self.device)
        it = C.c_int32()
        rr = C.c_double()
        flags = _native.ADJ_GAUGE_PROJECT if gauge_project else 0
        check(self._lib.caspar_ba_backward(self._h, _ptr(grad_cams), _ptr(grad_points), float(lambda_adj),
                                           float(pcg_tol), int(max_pcg_iters), flags, _ptr(out), C.byref(it),
                                           C.byref(rr)))
        self.last_backward_iters = it.value
        self.last_backward_rel_resid = rr.value
        if rr.value > pcg_tol:
            import warnings
            warnings.warn(f"adjoint PCG stopped after {it.value} iterations at relative residual {rr.value:.3e} "
                          f"> pcg_tol {pcg_tol:.3e}; the gradient is inexact", RuntimeWarning, stacklevel=2)
        return out

    def set_timing(self, enable: bool, every: int = 1):
        """Event timing of the fused product (caspar_ba_set_timing): every
        `every`-th launch while enabled."""
        if enable and int(every) == 0:
            raise ValueError("every must be at least 1 when timing is enabled")
        check(self._lib.caspar_ba_set_timing(self._h, int(every) if enable else 0))

    def get_timing(self):
        t = _native.Timing()
        check(self._lib.caspar_ba_get_timing(self._h, C.byref(t)))
        return {"matvec_launches": t.matvec_launches, "matvec_ms": t.matvec_ms, "matvec_bytes": t.matvec_bytes}

    def layout_info(self):
        k, cold, tiles, groups = C.c_int32(), C.c_int64(), C.c_int64(), C.c_int32()
        check(self._lib.caspar_ba_layout_info(self._h, C.byref(k), C.byref(cold), C.byref(tiles), C.byref(groups)))
        return {"hot_cams": k.value, "cold_obs": cold.value, "n_tiles": tiles.value, "matvec_groups": groups.value}


def read_bal(path) -> dict:
    """A BAL problem file as host numpy arrays in the boundary's layout:
    cams [n_cams, 9] (angle-axis, t, f, k1, k2), points [n_points, 3],
    obs_cam / obs_pt [n_obs] (int32), px [n_obs, 2] (float64)."""
    import numpy as np
    lib = _native.load()
    bp = _path_bytes(path)
    nc, npnt, no = C.c_int32(), C.c_int32(), C.c_int64()
    check(lib.caspar_bal_read_header(bp, C.byref(nc), C.byref(npnt), C.byref(no)))
    out = {"cams": np.empty((nc.value, 9), np.float64), "points": np.empty((npnt.value, 3), np.float64),
           "obs_cam": np.empty(no.value, np.int32), "obs_pt": np.empty(no.value, np.int32),
           "px": np.empty((no.value, 2), np.float64)}
    check(lib.caspar_bal_read(bp, nc.value, npnt.value, no.value, *(_host_ptr(out[k]) for k in
                                                                      ("obs_cam", "obs_pt", "px", "cams", "points"))))
    return out


def write_bal(path, cams, points, obs_cam, obs_pt, px) -> None:
    """Write a problem (host arrays or tensors, boundary layout) as a BAL file."""
    import numpy as np
    lib = _native.load()
    a = {"cams": (cams, np.float64, 9), "points": (points, np.float64, 3), "obs_cam": (obs_cam, np.int32, None),
         "obs_pt": (obs_pt, np.int32, None), "px": (px, np.float64, 2)}
    h = {}
    for k, (v, dt, width) in a.items():
        v = v.detach().cpu().numpy() if isinstance(v, torch.Tensor) else v
        v = np.ascontiguousarray(v, dtype=dt)
        if width is not None and (v.ndim != 2 or v.shape[1] != width):
            raise ValueError(f"{k} must have shape [n, {width}]")
        h[k] = v
    no = h["obs_cam"].shape[0]
    if h["obs_pt"].shape != (no,) or h["px"].shape[0] != no:
        raise ValueError("obs_cam, obs_pt and px must describe the same observations")
    check(lib.caspar_bal_write(_path_bytes(path), h["cams"].shape[0], h["points"].shape[0], no,
                               *(_host_ptr(h[k]) for k in ("obs_cam", "obs_pt", "px", "cams", "points"))))


def _path_bytes(path) -> bytes:
    import os
    return os.fsencode(path)


def _host_ptr(a):
    return C.c_void_p(a.ctypes.data if a.size else 0)


_host = _host_ptr


class BAFunction(torch.autograd.Function):
    """(obs_px, cams0, points0) -> optimal (cams*, points*) with the implicit
    adjoint as backward: d L / d obs_px = J v, (J^T J + lambda_adj D) v = g.

    The optimum does not depend on the initial values to first order, so
    their gradients are None.
    """

    @staticmethod
    def forward(ctx, obs_px, cams0, points0, obs_cam, obs_pt, opts=None, precision=FP64, lambda_adj=1e-4,
                adj_tol=1e-10, adj_max_iters=2000, recompute_jacobian=False):
        ba = BundleAdjuster(cams0.detach().contiguous(), points0.detach().contiguous(), obs_cam, obs_pt,
                            obs_px.detach().contiguous(), precision, recompute_jacobian)
        stats = ba.solve(opts)
        cams, pts = ba.get_params()
        ctx.ba = ba
        ctx.stats = stats
        ctx.adj = (lambda_adj, adj_tol, adj_max_iters)
        return cams, pts

    @staticmethod
    def backward(ctx, grad_cams, grad_points):
        lam, tol, iters = ctx.adj
        gc = None if grad_cams is None else grad_cams.contiguous().to(torch.float64)
        gp = None if grad_points is None else grad_points.contiguous().to(torch.float64)
        # the handle stays open (freed with ctx), so a second backward of a
        # retained graph works
        g_obs = ctx.ba.backward(gc, gp, lam, tol, iters)
        return g_obs, None, None, None, None, None, None, None, None, None, None
