"""Plain, slow FP64 CPU oracle of the filtered-property Lippmann-Schwinger solve.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import this
package: only the tests, the smoke check and the CPU-baseline leg of the
benchmark use it.  It shares no code with the HIP library; the two meet
only through the seeded inputs of the ``workloads`` package.

Reference: L. Gelebart, F. Ouaki, "Filtering material properties to improve
FFT-based methods for numerical homogenization" (arXiv:1412.3228).

Modules
-------
filter    sub-voxel phase fractions and interface normals (Section 2)
rules     Voigt, Reuss and 2-layer homogenisation rules (Section 2, eqs. 3-5)
solver    Lippmann-Schwinger fixed point, Green operator, equilibrium error,
          effective tensor (Section 2, eqs. 1-2)
gradient  derivative of the effective tensor by the Hill (energy) identity,
          cross-checked by the adjoint route through the fixed point
thermal, nphase, aniso, extrapolate
          conduction form, N-phase rules, anisotropic phases, Figure 4 series

Parity status: every function is pinned by the tests under ``tests/``.  One
convention has no pin because the paper does not fix it: the choice of
inclusion for the interface normal when the surfaces of several inclusions
are within the filter's reach of one voxel (see filter.normal_sphere); with
one surface in reach the choice and the normal are pinned.
"""
