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
gradient  derivative of the effective tensor by the Hill (energy) identity

Parity status: every function is pinned by the tests under ``tests/`` except
the choice of inclusion for the interface normal when several inclusions
are near a voxel ("parity unpinned": a convention, see filter.normal_sphere).
"""
