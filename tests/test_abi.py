"""The C ABI boundary without a GPU: the library loads, exports every
function include/caspar_ba.h declares, and the ctypes mirrors of the public
structs have the C layout."""
import ctypes
import os
import re
import subprocess
import tempfile

import pytest

from paper_2605_30583_amd import _native

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "caspar_ba.h")


def _declared():
    text = open(HEADER).read()
    return sorted(set(re.findall(r"CASPAR_API[^;(]*?\b(caspar_\w+)\s*\(", text)))


def test_library_exports_every_declared_function():
    lib = _native.load()
    names = _declared()
    assert len(names) >= 15
    for n in names:
        assert hasattr(lib, n), n
    assert sorted(n for n, _, _ in _native.SIGNATURES) == names


def test_only_the_c_abi_is_exported():
    out = subprocess.run(["nm", "-D", "--defined-only", _native.LIB_PATH], capture_output=True, text=True,
                         check=True).stdout
    exported = sorted(l.split()[-1] for l in out.splitlines() if " T " in l)
    assert exported == _declared()


def test_struct_layouts_match_the_header():
    src = r'''
#include <stdio.h>
#include <stddef.h>
#include "caspar_ba.h"
int main(void) {
  printf("%zu %zu %zu %zu %zu %zu\n", sizeof(caspar_solve_opts), sizeof(caspar_solve_stats),
         sizeof(caspar_iter_record), offsetof(caspar_solve_opts, pcg_check_every),
         offsetof(caspar_solve_stats, seconds), offsetof(caspar_iter_record, pcg_iters));
  return 0;
}
'''
    with tempfile.TemporaryDirectory() as d:
        c = os.path.join(d, "s.c")
        exe = os.path.join(d, "s")
        open(c, "w").write(src)
        subprocess.run(["gcc", "-I", os.path.dirname(HEADER), c, "-o", exe], check=True)
        vals = [int(v) for v in subprocess.run([exe], capture_output=True, text=True, check=True).stdout.split()]
    assert vals == [ctypes.sizeof(_native.SolveOpts), ctypes.sizeof(_native.SolveStats),
                    ctypes.sizeof(_native.IterRecord), _native.SolveOpts.pcg_check_every.offset,
                    _native.SolveStats.seconds.offset, _native.IterRecord.pcg_iters.offset]


def test_default_options_and_size_validation():
    lib = _native.load()
    o = _native.SolveOpts()
    lib.caspar_default_solve_opts(ctypes.byref(o))
    assert o.lambda0 == 1e-2 and o.pcg_tol == 1e-3 and o.max_pcg_iters == 500
    # invalid sizes / precision are rejected before any device work
    assert lib.caspar_ba_workspace_bytes(-1, 10, 10, 0) == 0
    assert lib.caspar_ba_workspace_bytes(10, 10, 10, 7) == 0
    assert lib.caspar_ba_workspace_bytes(0, 10, 10, 0) == 0      # observations need cameras
    assert lib.caspar_ba_workspace_bytes(10, 10, 1 << 31, 0) == 0


def test_create_rejects_null_output_handle():
    lib = _native.load()
    st = lib.caspar_ba_create(None, 1, 1, 0, None, None, None, None, None, 0, None, 0, None)
    assert st == -1
    assert b"out is NULL" in lib.caspar_last_error()
