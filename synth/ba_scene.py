"""Seeded, synthetic, BAL-shaped bundle-adjustment scenes.

The paper evaluates on the BAL datasets (Section VI); those files are not
available here, so scenes of the same structure are synthesised:

* cameras on a circle of radius 10 in the z=0 plane, each looking at the
  origin (camera frame: BAL convention, points in front have negative depth),
  focal length 500, radial coefficients k1, k2 ~ N(0, 1e-3^2);
* points uniform in the cube [-2, 2]^3;
* every point observed by k distinct cameras, drawn uniformly or with a
  Zipf(s) weight over a random rank permutation of the cameras;
* pixel noise N(0, sigma^2) per coordinate (drawn here, added by the caller
  to the predicted pixels);
* initial values perturbed additively in the BAL parametrisation:
  angle-axis + N(0, 0.01^2), translation + N(0, 0.05^2), points
  + N(0, 0.05^2); f, k1, k2 exact.

* optionally a fraction of observations with gross outliers: their noise is
  replaced by N(0, outlier_px^2) (drawn last);
* optionally a hard start: the initial value of point 0 is moved a given
  fraction of the way from its true position toward the centre of the first
  camera that observes it (no draw), so that the first linear models
  mispredict the cost and trials get rejected.

Draw order is fixed: k1/k2, points, visibility, noise, perturbations,
outliers.

Only random draws and the scene layout live here.  The observed pixels
(prediction + noise) are formed by the consumer with its own projection,
so this module contains no part of the solver's arithmetic.
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np


@dataclasses.dataclass
class Scene:
    """A synthetic problem in BAL layout (caller order everywhere)."""

    cams_true: np.ndarray    # f64 [n_cams, 9]: angle-axis(3), t(3), f, k1, k2
    points_true: np.ndarray  # f64 [n_points, 3]
    obs_cam: np.ndarray      # int32 [n_obs]
    obs_pt: np.ndarray       # int32 [n_obs]
    noise: np.ndarray        # f64 [n_obs, 2], pixel noise to add to predictions
    cams_init: np.ndarray    # f64 [n_cams, 9]
    points_init: np.ndarray  # f64 [n_points, 3]

    @property
    def n_cams(self) -> int:
        return int(self.cams_true.shape[0])

    @property
    def n_points(self) -> int:
        return int(self.points_true.shape[0])

    @property
    def n_obs(self) -> int:
        return int(self.obs_cam.shape[0])

    def shuffled(self, seed: int) -> "Scene":
        """Same problem with the observation order permuted."""
        perm = np.random.default_rng(seed).permutation(self.n_obs)
        return dataclasses.replace(self, obs_cam=self.obs_cam[perm].copy(),
                                   obs_pt=self.obs_pt[perm].copy(),
                                   noise=self.noise[perm].copy())


def _matrix_to_angle_axis(R: np.ndarray) -> np.ndarray:
    """Angle-axis vector of each rotation matrix (via a unit quaternion).

    Scene set-up only: turns the look-at frames below into the BAL camera
    parametrisation.  Uses the largest-diagonal branch so that rotations by
    angles near pi stay accurate.
    """
    R = np.asarray(R, dtype=np.float64)
    out = np.empty((R.shape[0], 3))
    for i, m in enumerate(R):
        tr = m[0, 0] + m[1, 1] + m[2, 2]
        cand = [tr, m[0, 0], m[1, 1], m[2, 2]]
        k = int(np.argmax(cand))
        if k == 0:
            w = 0.5 * math.sqrt(1.0 + tr)
            s = 0.25 / w
            q = np.array([w, (m[2, 1] - m[1, 2]) * s, (m[0, 2] - m[2, 0]) * s, (m[1, 0] - m[0, 1]) * s])
        else:
            a = k - 1
            b, c = (a + 1) % 3, (a + 2) % 3
            v = np.zeros(3)
            v[a] = 0.5 * math.sqrt(max(0.0, 1.0 + m[a, a] - m[b, b] - m[c, c]))
            s = 0.25 / v[a]
            v[b] = (m[b, a] + m[a, b]) * s
            v[c] = (m[c, a] + m[a, c]) * s
            w = (m[c, b] - m[b, c]) * s
            q = np.array([w, v[0], v[1], v[2]])
        if q[0] < 0:
            q = -q
        vn = math.sqrt(q[1] ** 2 + q[2] ** 2 + q[3] ** 2)
        if vn < 1e-300:
            out[i] = 0.0
        else:
            ang = 2.0 * math.atan2(vn, q[0])
            out[i] = q[1:] * (ang / vn)
    return out


def _look_at_frames(n_cams: int, radius: float):
    """Rotation (rows x, y, z), translation and centre of cameras on a circle.

    Camera i sits at c_i = radius (cos phi_i, sin phi_i, 0), phi_i = 2 pi i / n.
    Its z axis points away from the origin, so the origin has depth -radius.
    """
    phi = 2.0 * np.pi * np.arange(n_cams) / n_cams
    c = radius * np.stack([np.cos(phi), np.sin(phi), np.zeros_like(phi)], axis=1)
    z = c / np.linalg.norm(c, axis=1, keepdims=True)
    up = np.array([0.0, 0.0, 1.0])
    x = np.cross(up[None, :], z)
    x /= np.linalg.norm(x, axis=1, keepdims=True)
    y = np.cross(z, x)
    R = np.stack([x, y, z], axis=1)          # rows are the camera axes
    t = -np.einsum("nij,nj->ni", R, c)
    return R, t, c


def _draw_visibility(rng, n_points, n_cams, k_values, k_probs, cam_weights):
    """k distinct cameras per point: 12-candidate rows, first k distinct kept,
    short rows redrawn."""
    ncand = 12
    k = rng.choice(np.asarray(k_values), size=n_points, p=np.asarray(k_probs, dtype=np.float64))
    if int(k.max()) > n_cams:
        raise ValueError("a point cannot see more distinct cameras than exist")
    chosen = np.full((n_points, int(k.max())), -1, dtype=np.int64)
    todo = np.arange(n_points)
    while todo.size:
        if cam_weights is None:
            cand = rng.integers(0, n_cams, size=(todo.size, ncand))
        else:
            cand = rng.choice(n_cams, size=(todo.size, ncand), p=cam_weights)
        first = np.ones(cand.shape, dtype=bool)
        for j in range(1, ncand):
            first[:, j] = np.all(cand[:, j:j + 1] != cand[:, :j], axis=1)
        rank = np.cumsum(first, axis=1)           # 1-based rank among distinct
        ok = rank[:, -1] >= k[todo]
        rows = todo[ok]
        cr, fr, rr = cand[ok], first[ok], rank[ok]
        kk = k[rows]
        for j in range(int(k.max())):
            sel = fr & (rr == j + 1)
            has = sel.any(axis=1) & (j < kk)
            col = np.argmax(sel, axis=1)
            chosen[rows[has], j] = cr[has, col[has]]
        todo = todo[~ok]
    obs_pt = np.repeat(np.arange(n_points), k)
    mask = np.arange(chosen.shape[1])[None, :] < k[:, None]
    obs_cam = chosen[mask]
    return obs_cam.astype(np.int32), obs_pt.astype(np.int32)


def make_scene(n_cams: int, n_points: int, seed: int, *, k_values=(4,), k_probs=(1.0,),
               zipf_s: float | None = None, radius: float = 10.0, focal: float = 500.0,
               kdist_std: float = 1e-3, point_half_width: float = 2.0,
               noise_px: float = 1.0, rot_std: float = 0.01, trans_std: float = 0.05,
               point_std: float = 0.05, outlier_frac: float = 0.0, outlier_px: float = 40.0,
               pull_first_point: float = 0.0) -> Scene:
    """Draw one synthetic scene (see module docstring for the recipe)."""
    rng = np.random.default_rng(seed)
    R, t, centres = _look_at_frames(n_cams, radius)
    kd = rng.normal(0.0, kdist_std, size=(n_cams, 2))
    cams = np.empty((n_cams, 9))
    cams[:, 0:3] = _matrix_to_angle_axis(R)
    cams[:, 3:6] = t
    cams[:, 6] = focal
    cams[:, 7:9] = kd
    pts = rng.uniform(-point_half_width, point_half_width, size=(n_points, 3))
    weights = None
    if zipf_s is not None:
        rank = rng.permutation(n_cams) + 1
        w = rank.astype(np.float64) ** (-zipf_s)
        weights = w / w.sum()
    obs_cam, obs_pt = _draw_visibility(rng, n_points, n_cams, k_values, k_probs, weights)
    noise = rng.normal(0.0, noise_px, size=(obs_cam.shape[0], 2))
    cams0 = cams.copy()
    cams0[:, 0:3] += rng.normal(0.0, rot_std, size=(n_cams, 3))
    cams0[:, 3:6] += rng.normal(0.0, trans_std, size=(n_cams, 3))
    pts0 = pts + rng.normal(0.0, point_std, size=(n_points, 3))
    if outlier_frac > 0.0:
        # gross outliers, drawn after everything else so the rest of the scene
        # is the same as without them: these observations get N(0, outlier_px)
        # pixel errors instead of the ordinary noise
        sel = rng.random(obs_cam.shape[0]) < outlier_frac
        noise[sel] = rng.normal(0.0, outlier_px, size=(int(sel.sum()), 2))
    if pull_first_point != 0.0:
        c = centres[obs_cam[0]]              # obs_pt is point-major: obs 0 sees point 0
        pts0[0] = pts[0] + pull_first_point * (c - pts[0])
    return Scene(cams, pts, obs_cam, obs_pt, noise, cams0, pts0)


# The five workloads: tiny, medium, BAL-shaped 1.7k cameras, medium with the
# adjoint (same scene as medium), and the large Zipf-skewed BAL shape; plus
# the tiny scene with planted outliers for the robust losses.
SCENE_CONFIGS = {
    "tiny":   dict(n_cams=16, n_points=1_000, seed=1, k_values=(4,), k_probs=(1.0,)),
    "medium": dict(n_cams=250, n_points=50_000, seed=2, k_values=(6,), k_probs=(1.0,)),
    "bal1700": dict(n_cams=1_700, n_points=160_000, seed=3, k_values=(5, 6), k_probs=(0.4, 0.6)),
    "medium_adjoint": dict(n_cams=250, n_points=50_000, seed=2, k_values=(6,), k_probs=(1.0,)),
    "large_zipf": dict(n_cams=13_700, n_points=4_400_000, seed=5, k_values=(6, 7),
                       k_probs=(0.41, 0.59), zipf_s=1.1),
    # robust losses: the tiny scene with 5% gross outliers (40 px)
    "tiny_outliers": dict(n_cams=16, n_points=1_000, seed=1, k_values=(4,), k_probs=(1.0,),
                          outlier_frac=0.05, outlier_px=40.0),
    # damping-rule trajectories: six cameras, 60 points, point 0 starting 90%
    # of the way toward a camera that sees it (rejected trials early on)
    "hard_start_a": dict(n_cams=6, n_points=60, seed=5, k_values=(3,), k_probs=(1.0,), pull_first_point=0.9),
    "hard_start_b": dict(n_cams=6, n_points=60, seed=3, k_values=(3,), k_probs=(1.0,), pull_first_point=0.9),
}


def scene_config(name: str, **overrides) -> Scene:
    """Build one of the named workloads; keyword overrides replace recipe values."""
    cfg = dict(SCENE_CONFIGS[name])
    cfg.update(overrides)
    return make_scene(**cfg)


@dataclasses.dataclass
class BetweenDraws:
    """Camera pairs for pose between-factors and their standard-normal noise
    draws; forming the measurements from the true poses is left to the
    caller (it is the factor's own arithmetic)."""
    fi: np.ndarray           # [n] int32 first camera of each pair
    fj: np.ndarray           # [n] int32 second camera
    rot_noise: np.ndarray    # [n, 3] N(0, 1)
    trans_noise: np.ndarray  # [n, 3] N(0, 1)


def between_draws(n_cams: int, seed: int, n_loops: int = 0) -> BetweenDraws:
    """A chain (c, c + 1) over the cameras in caller order, then n_loops
    random pairs of distinct cameras (loop closures), then the noise draws,
    in that order from default_rng(seed)."""
    rng = np.random.default_rng(seed)
    fi = list(range(n_cams - 1))
    fj = list(range(1, n_cams))
    for _ in range(n_loops):
        a, b = rng.choice(n_cams, size=2, replace=False)
        fi.append(int(a))
        fj.append(int(b))
    n = len(fi)
    return BetweenDraws(np.asarray(fi, np.int32), np.asarray(fj, np.int32), rng.normal(size=(n, 3)),
                        rng.normal(size=(n, 3)))
