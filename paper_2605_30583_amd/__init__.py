"""MI355X (gfx950) bundle-adjustment hot path: Levenberg-Marquardt with a
matrix-free block-Jacobi PCG on the damped normal equations, hand-written
HIP behind a C ABI (include/caspar_ba.h).

The Python layer only marshals torch tensors (device memory, streams) into
the C calls; every step of the solve runs in the HIP library.  Importing the
package is cheap; the library is loaded on first use and its absence raises.
"""
from .api import (BundleAdjuster, SolveOptions, BAFunction, project, read_bal, write_bal,  # noqa: F401
                  FP64, FP32_MIXED, RECOMPUTE_JACOBIAN, library_path)
