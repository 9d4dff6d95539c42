// Launch interface of the post-processing kernels: the truncated Fourier
// series of a grid field on a finer grid (Figure 4), a Mandel entry of the
// filtered stiffness per voxel (the field that figure extrapolates) and the
// local stress field of a solve (the maps of Figure 2).
#pragma once

#include <hip/hip_runtime.h>

namespace hm {

// One separable pass of the series: out[o][j'][i] = sum_j K[j'][j] in[o][j][i]
// (i contiguous, extent I; j contracted, extent n; j' extent mj; o extent O).
// K is stored transposed: K[j][j'] (n x mj).  When I == 1 the pass runs
// along contiguous lines.
struct AxisPass {
  const void* in;
  void* out;
  const void* K;
  long long I, O;
  int n, mj;
};

hipError_t launch_series_pass(const AxisPass& p, bool fp64, hipStream_t s);

// Mandel entry (I, J) of c~ at every voxel (rule of eqs. 3-5, pure phases
// where f is 0 or 1); flags[0] gets 1 for a fractional voxel under the
// no-filter rule, 2 for an interface sphere index out of range.
struct StiffnessArgs {
  const void* frac;
  const int* incl;
  const double* sph;  // [nsph][4]
  int nsph;
  int n[3];
  int dim;
  double pl[2], pm[2];
  int rule;
  int I, J;
  void* out;
  int* flags;
};

hipError_t launch_stiffness_component(const StiffnessArgs& a, bool fp64, hipStream_t s);

// Local stress sigma = c~ : eps at every voxel for n_load strain fields
// [load][6][N] (tensor components), written to sig with the same layout;
// the material arguments as above (I, J unused).
struct StressArgs {
  StiffnessArgs m;
  const void* eps;
  void* sig;
  int n_load;
};

hipError_t launch_stress_field(const StressArgs& a, bool fp64, hipStream_t s);

// Local flux q = k~ g of a conduction solve: the same arguments with the
// phase conductivities in m.pl, gradient fields [load][3][N] in eps and the
// fluxes written to sig with that layout.
hipError_t launch_flux_field(const StressArgs& a, bool fp64, hipStream_t s);

}  // namespace hm
