"""BAL problem files: the native reader and writer (caspar_bal_read_header,
caspar_bal_read, caspar_bal_write) against the plain-Python reference
(oracle/bal.py), host only.

The oracle is pinned by a hand-written file (tests/golden/bal_hand_written.txt)
whose values are spelled out below.  The native reader must return the same
arrays bit for bit on that file, on files the oracle writes (one small enough
for one thread, one large enough to be split across threads), on files with
unusual but legal whitespace and number forms, and must refuse malformed
files with CASPAR_EINVAL (CASPAR_EIO for a missing file)."""
import os

import numpy as np
import pytest

from oracle import bal as obal
from synth import scene_config

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "bal_hand_written.txt")

EXPECTED = {
    "obs_cam": np.array([0, 1, 0, 1], np.int32),
    "obs_pt": np.array([0, 0, 2, 1], np.int32),
    "px": np.array([[-123.25, 45.5], [-31.25, 200.0], [1.5, -2.25], [700.0, -0.125]]),
    "cams": np.array([[0.01, -0.02, 0.03, 0.5, -0.25, 10.0, 480.0, 1e-7, -2.5e-13],
                      [0.0, 0.0, 0.0, 1.0, 2.0, 3.0, 500.0, 0.0, 0.0]]),
    "points": np.array([[-0.5, 0.25, -10.0], [1e-3, 200.0, -3.5], [0.0, 0.0, 0.0]]),
}
KEYS = ("cams", "points", "obs_cam", "obs_pt", "px")


def _native():
    from paper_2605_30583_amd import read_bal, write_bal
    from paper_2605_30583_amd._native import CasparError
    return read_bal, write_bal, CasparError


def _same(a, b):
    for k in KEYS:
        assert a[k].dtype == b[k].dtype and a[k].shape == b[k].shape, k
        assert np.array_equal(a[k], b[k]), k


def test_oracle_reads_the_hand_written_file():
    _same(obal.read(GOLDEN), EXPECTED)


def test_native_reader_matches_the_hand_written_file():
    read_bal, _, _ = _native()
    _same(read_bal(GOLDEN), EXPECTED)


def _scene_arrays(name, **kw):
    sc = scene_config(name, **kw)
    rng = np.random.default_rng(11)
    px = rng.normal(scale=200.0, size=(sc.n_obs, 2))
    return {"cams": sc.cams_init, "points": sc.points_init, "obs_cam": sc.obs_cam.astype(np.int32),
            "obs_pt": sc.obs_pt.astype(np.int32), "px": px}


@pytest.mark.parametrize("name,kw", [("tiny", {}), ("medium", {"n_points": 60_000})], ids=["one-thread", "threaded"])
def test_round_trips_are_exact(tmp_path, name, kw):
    read_bal, write_bal, _ = _native()
    a = _scene_arrays(name, **kw)
    a["cams"] = np.asarray(a["cams"], np.float64)
    a["points"] = np.asarray(a["points"], np.float64)
    f1 = tmp_path / "oracle.bal"
    obal.write(f1, a["cams"], a["points"], a["obs_cam"], a["obs_pt"], a["px"])
    if name != "tiny":
        assert os.path.getsize(f1) > 4 << 20          # several threads' worth of bytes
    _same(read_bal(f1), a)
    f2 = tmp_path / "native.bal"
    write_bal(f2, a["cams"], a["points"], a["obs_cam"], a["obs_pt"], a["px"])
    _same(obal.read(f2), a)
    _same(read_bal(f2), a)


def test_whitespace_and_number_forms(tmp_path):
    read_bal, _, _ = _native()
    text = open(GOLDEN).read()
    variants = [
        text.replace("\n", "\r\n"),
        text.replace("\n", " \t \n\n"),
        " ".join(text.split()),                                   # one line
        "\n".join(text.split()) + "\n\n\n",                       # one token per line, trailing blank lines
    ]
    for i, v in enumerate(variants):
        p = tmp_path / f"v{i}.bal"
        p.write_text(v)
        _same(read_bal(p), EXPECTED)
        _same(obal.read(p), EXPECTED)


def _expect_error(tmp_path, text, status_name, fragment):
    read_bal, _, CasparError = _native()
    p = tmp_path / "bad.bal"
    p.write_text(text)
    with pytest.raises(CasparError) as e:
        read_bal(p)
    assert status_name in str(e.value) and fragment in str(e.value), str(e.value)


def test_malformed_files_are_refused(tmp_path):
    good = open(GOLDEN).read()
    tok = good.split()
    _expect_error(tmp_path, " ".join(tok[:-1]), "CASPAR_EINVAL", "ends early")
    _expect_error(tmp_path, good + " 1.0\n", "CASPAR_EINVAL", "trailing data")
    _expect_error(tmp_path, "2 3\n", "CASPAR_EINVAL", "header")
    _expect_error(tmp_path, "-2 3 4\n", "CASPAR_EINVAL", "header")
    bad = list(tok)
    bad[3] = "2"                                             # camera index of observation 0 == n_cams
    _expect_error(tmp_path, " ".join(bad), "CASPAR_EINVAL", "observation 0: camera index 2 out of range")
    bad = list(tok)
    bad[8] = "3"                                             # point index of observation 1 == n_points
    _expect_error(tmp_path, " ".join(bad), "CASPAR_EINVAL", "observation 1: point index 3 out of range")
    bad = list(tok)
    bad[9] = "1.5e"                                          # pixel x of observation 1
    _expect_error(tmp_path, " ".join(bad), "CASPAR_EINVAL", "observation 1: pixel")
    bad = list(tok)
    bad[3 + 16 + 4] = "nan"                                  # camera 0, translation x
    _expect_error(tmp_path, " ".join(bad), "CASPAR_EINVAL", "camera 0")
    bad = list(tok)
    bad[-1] = "inf"                                          # last point coordinate
    _expect_error(tmp_path, " ".join(bad), "CASPAR_EINVAL", "point 2")
    bad = list(tok)
    bad[3] = "0.5"                                           # a camera index that is not an integer
    _expect_error(tmp_path, " ".join(bad), "CASPAR_EINVAL", "not an integer")


def test_missing_file_and_size_mismatch(tmp_path):
    import ctypes as C
    from paper_2605_30583_amd import _native as nat
    read_bal, _, CasparError = _native()
    with pytest.raises(CasparError) as e:
        read_bal(tmp_path / "absent.bal")
    assert "CASPAR_EIO" in str(e.value)
    lib = nat.load()
    a = {k: np.empty_like(v) for k, v in EXPECTED.items()}
    ptrs = [C.c_void_p(a[k].ctypes.data) for k in ("obs_cam", "obs_pt", "px", "cams", "points")]
    assert lib.caspar_bal_read(os.fsencode(GOLDEN), 2, 3, 5, *ptrs) == -1          # n_obs differs from the header
    assert lib.caspar_bal_read(os.fsencode(GOLDEN), 2, 3, 4, None, *ptrs[1:]) == -1   # null output array
    assert lib.caspar_bal_read(os.fsencode(GOLDEN), 2, 3, 4, *ptrs) == 0


def test_writer_refuses_bad_problems(tmp_path):
    _, write_bal, CasparError = _native()
    e = {k: v.copy() for k, v in EXPECTED.items()}
    e["obs_pt"][2] = 3
    with pytest.raises(CasparError, match="index out of range"):
        write_bal(tmp_path / "x.bal", e["cams"], e["points"], e["obs_cam"], e["obs_pt"], e["px"])
    e = {k: v.copy() for k, v in EXPECTED.items()}
    e["points"][1, 2] = np.nan
    with pytest.raises(CasparError, match="non-finite"):
        write_bal(tmp_path / "x.bal", e["cams"], e["points"], e["obs_cam"], e["obs_pt"], e["px"])
