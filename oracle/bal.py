"""BAL problem files in plain Python (oracle).

TEST INFRASTRUCTURE ONLY: the reference that the library's native BAL reader
and writer are checked against.

The paper evaluates on the Bundle Adjustment in the Large datasets
(Section VI).  Their text format is a stream of whitespace-separated tokens:
the counts n_cams n_points n_obs; n_obs records "camera point x y"; 9 values
per camera (angle-axis rotation, translation, f, k1, k2); 3 values per point.

read() splits the text on whitespace and converts each token with int() or
float() (correctly rounded); write() prints every real with repr(), the
shortest string that reads back to the same float64.

Pins (tests/test_bal_io.py): a hand-written file whose values are written
out literally in the test; write-then-read returns the arrays bit for bit.
"""
from __future__ import annotations

import math

import numpy as np


class BALFormatError(ValueError):
    pass


def read(path) -> dict:
    with open(path, "rb") as f:
        tok = f.read().decode("ascii").split()
    if len(tok) < 3:
        raise BALFormatError("file ends inside the header")
    try:
        nc, npnt, no = (int(t) for t in tok[:3])
    except ValueError as e:
        raise BALFormatError("header is not three integers") from e
    if min(nc, npnt, no) < 0:
        raise BALFormatError("negative count")
    want = 3 + 4 * no + 9 * nc + 3 * npnt
    if len(tok) != want:
        raise BALFormatError(f"{len(tok) - 3} values after the header, {want - 3} expected")
    obs_cam = np.empty(no, np.int32)
    obs_pt = np.empty(no, np.int32)
    px = np.empty((no, 2), np.float64)
    k = 3
    for i in range(no):
        c, p = int(tok[k]), int(tok[k + 1])
        if not (0 <= c < nc and 0 <= p < npnt):
            raise BALFormatError(f"observation {i}: index out of range")
        obs_cam[i], obs_pt[i] = c, p
        px[i] = float(tok[k + 2]), float(tok[k + 3])
        k += 4
    vals = np.array([float(t) for t in tok[k:]], dtype=np.float64)
    if not np.all(np.isfinite(vals)) or not np.all(np.isfinite(px)):
        raise BALFormatError("non-finite value")
    return {"cams": vals[:9 * nc].reshape(nc, 9).copy(), "points": vals[9 * nc:].reshape(npnt, 3).copy(),
            "obs_cam": obs_cam, "obs_pt": obs_pt, "px": px}


def write(path, cams, points, obs_cam, obs_pt, px) -> None:
    cams = np.asarray(cams, np.float64).reshape(-1, 9)
    points = np.asarray(points, np.float64).reshape(-1, 3)
    obs_cam = np.asarray(obs_cam).ravel()
    obs_pt = np.asarray(obs_pt).ravel()
    px = np.asarray(px, np.float64).reshape(-1, 2)
    lines = [f"{cams.shape[0]} {points.shape[0]} {obs_cam.shape[0]}"]
    for c, p, (x, y) in zip(obs_cam.tolist(), obs_pt.tolist(), px.tolist()):
        lines.append(f"{c} {p} {x!r} {y!r}")
    for v in cams.ravel().tolist() + points.ravel().tolist():
        if not math.isfinite(v):
            raise BALFormatError("non-finite value")
        lines.append(repr(v))
    with open(path, "w") as f:
        f.write("\n".join(lines) + "\n")
