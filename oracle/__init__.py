"""FP64 CPU oracle for the bundle-adjustment hot path.

TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the CPU
baseline leg of the benchmark may import or run anything in this package.
The GPU library never calls it and shares no code with it.

Everything is plain NumPy / SciPy in float64 and follows the paper:
Snavely reprojection factor (Section VI-A), Levenberg-Marquardt with the
gain-ratio damping update after Madsen et al. and tangent-space retraction
(Section V), normal equations solved without a Schur-based reduction on the
GPU side; here the exact step is taken by dense or Schur-complement Cholesky
(Section V), block-Jacobi preconditioned CG on the normal equations
(Section V, glossary PCGNR).

Parity status per function is listed in each module header.
"""
