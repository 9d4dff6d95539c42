// Launch arguments of the effective-tensor gradient kernel.
#pragma once

#include <hip/hip_runtime.h>

namespace hm {

struct HillArgs {
  const void* eps;   // T[n_load][6][N] solution fields of the unit Mandel strains
  const void* frac;  // T[N]
  const int* incl;   // int32[N] or null
  const double* sph; // [nsph][4] voxel units
  int nsph;
  int n[3];
  int dim;
  int n_load;
  int rule;
  double pl[2], pm[2];  // phase Lame parameters
  double G[36];         // dL/dC (n_load x n_load, row-major)
  double* part;         // [blocks][4] per-block sums of the Lame derivatives
  void* dfrac;          // T[N] or null
};

hipError_t launch_hill(const HillArgs& a, bool fp64, int blocks, hipStream_t s);

}  // namespace hm
