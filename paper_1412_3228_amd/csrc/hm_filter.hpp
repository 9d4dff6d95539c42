// Launch arguments of the filter kernel (shared by the kernel and the C ABI).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace hm {

struct LatSphere {
  long long c[3];  // centre, lattice units u = voxel / (2 S)
  double t;        // radius, lattice units
  double R2;       // t * t
};

struct FilterArgs {
  const LatSphere* sph;
  int nsph;
  int n[3];
  int dim;
  long long S;     // sub-samples per voxel and axis (even)
  long long P[3];  // periods 2 n S
  double rho;      // filter radius, lattice units (2 r S)
  double rho2;     // rho * rho
  int m;           // floor(rho): bound of the odd offsets
  int M;           // stencil size (1 when there is no filter)
  int point;       // 1: no filter, indicator at the voxel centre
  uint32_t* count;
  void* frac;
  int32_t* incl;
  // multi-phase filter: inclusion phase (1..nlab) of every sphere, device;
  // null for the two-phase filter
  const int* lab;
  int nlab;
};

hipError_t launch_filter(const FilterArgs& a, bool fp64, hipStream_t s);

}  // namespace hm
