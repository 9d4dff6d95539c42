// Filter of material properties: sub-voxel phase fractions.
//
// Section 2: the filtered behaviour at a grid point uses the phase volume
// fractions inside a uniform filter centred on it, which may be estimated by
// averaging the phase indicators over a refined grid; the numerical setup
// gives the filter radius in pixel units and the interface normal as the
// direction from the inclusion centre to the grid point.
//
// Integer lattice: u = (voxel size) / (2 S).  Voxel a has its centre at
// (2a + 1) S; refined points sit at odd coordinates (spacing 2u); the filter
// keeps offsets o (odd per axis) with |o|^2 <= (2 r S)^2.  A refined point is
// inside the inclusion set when, for some sphere, its periodic minimum-image
// squared distance to the rounded centre is <= R^2, so every count is an
// exact integer.  One thread per voxel: spheres that cannot reach the filter
// ball are skipped and a sphere that contains the whole ball gives the full
// count without enumeration (both decisions are conservative by one lattice
// unit).  Remaining voxels count, row by row of the stencil (fixed odd oy,
// oz), the odd ox inside both the filter ball and some candidate sphere: each
// is an integer interval (integer square roots), so a row costs a few
// operations instead of one test per point.  That needs the minimum image of
// every stencil point to be the voxel's own image shifted by the offset
// (the ball does not straddle half a period from the sphere); otherwise, or
// with more candidates than the list holds, the points are tested one by one.
// A multi-phase filter counts each inclusion phase on its own (the spheres
// of other phases are skipped), which partitions the union when spheres of
// different phases do not overlap.
#include <math.h>
#include <stdint.h>

#include "hm_common.hpp"
#include "hm_filter.hpp"

namespace hm {

__device__ __forceinline__ long long min_image(long long d, long long P) {
  const long long h = P / 2;
  while (d >= h) d -= P;
  while (d < -h) d += P;
  return d;
}

constexpr int kMaxCand = 8;

// floor(sqrt(q)) for 0 <= q < 2^53, exact.
__device__ __forceinline__ long long isqrt(long long q) {
  long long r = (long long)sqrt((double)q);
  while (r * r > q) --r;
  while ((r + 1) * (r + 1) <= q) ++r;
  return r;
}

// Number of odd integers in [lo, hi].
__device__ __forceinline__ long long odd_count(long long lo, long long hi) {
  if (hi < lo) return 0;
  auto fdiv2 = [](long long v) { return v >= 0 ? v / 2 : -((1 - v) / 2); };
  return fdiv2(hi - 1) - fdiv2(lo) + 1;
}

// Refined points of the filter around the voxel centre X (lattice units)
// that lie inside the spheres of label `want` (every sphere when want is 0;
// labels are the inclusion phases of a multi-phase filter).
__device__ uint32_t filter_count(const FilterArgs& a, const long long X[3], int axes, int want) {
  auto take = [&](int k) { return want == 0 || a.lab[k] == want; };
  uint32_t cnt = 0;
  if (a.point) {
    for (int k = 0; k < a.nsph; ++k) {
      if (!take(k)) continue;
      long long d2 = 0;
      for (int ax = 0; ax < axes; ++ax) {
        const long long d = min_image(X[ax] - a.sph[k].c[ax], a.P[ax]);
        d2 += d * d;
      }
      if ((double)d2 <= a.sph[k].R2) {
        cnt = 1;
        break;
      }
    }
    return cnt;
  }
  int cand[kMaxCand];
  int nc = 0;
  bool overflow = false, full = false;
  for (int k = 0; k < a.nsph && !full; ++k) {
    if (!take(k)) continue;
    long long d2 = 0;
    for (int ax = 0; ax < axes; ++ax) {
      const long long d = min_image(X[ax] - a.sph[k].c[ax], a.P[ax]);
      d2 += d * d;
    }
    const double D = sqrt((double)d2);
    if (D + a.rho <= a.sph[k].t - 1.0) {
      full = true;
    } else if (D - a.rho <= a.sph[k].t + 1.0) {
      if (nc < kMaxCand)
        cand[nc++] = k;
      else
        overflow = true;
    }
  }
  // per-candidate minimum-image offset of the voxel centre; the row method
  // needs every stencil point's image to follow from it (no wrap)
  long long d0[kMaxCand][3] = {};
  long long rint[kMaxCand] = {};
  bool rows_ok = !overflow;
  if (!full && rows_ok) {
    for (int q = 0; q < nc; ++q) {
      const int k = cand[q];
      for (int ax = 0; ax < 3; ++ax) {
        const long long h = a.P[ax] / 2;
        const long long d = ax < axes ? min_image(X[ax] - a.sph[k].c[ax], a.P[ax]) : 0;
        d0[q][ax] = d;
        if (ax < axes && (d - a.m < -h || d + a.m >= h)) rows_ok = false;
      }
      rint[q] = (long long)floor(a.sph[k].R2);
    }
  }
  if (full) {
    cnt = (uint32_t)a.M;
  } else if (nc > 0 && rows_ok) {
    const long long rho_i = (long long)floor(a.rho2);
    const int zlo = axes == 3 ? -a.m : 0;
    const int zhi = axes == 3 ? a.m : 0;
    long long total = 0;
    for (int oz = zlo; oz <= zhi; ++oz) {
      if (axes == 3 && (oz & 1) == 0) continue;
      for (int oy = -a.m; oy <= a.m; ++oy) {
        if ((oy & 1) == 0) continue;
        const long long rest = rho_i - (long long)oy * oy - (long long)oz * oz;
        if (rest < 1) continue;
        const long long al = isqrt(rest);  // |ox| <= al inside the filter ball
        long long lo[kMaxCand], hi[kMaxCand];
        int ni = 0;
        for (int q = 0; q < nc; ++q) {
          const long long dy = d0[q][1] + oy, dz = d0[q][2] + oz;
          const long long Q = rint[q] - dy * dy - dz * dz;
          if (Q < 0) continue;
          const long long b = isqrt(Q);  // |d0x + ox| <= b inside sphere q
          const long long l = max(-al, -b - d0[q][0]), u = min(al, b - d0[q][0]);
          if (l > u) continue;
          // insert sorted by lower end
          int j = ni++;
          while (j > 0 && lo[j - 1] > l) {
            lo[j] = lo[j - 1];
            hi[j] = hi[j - 1];
            --j;
          }
          lo[j] = l;
          hi[j] = u;
        }
        // odd integers in the union of the sorted intervals
        long long cl = 0, ch = -1;
        bool open = false;
        for (int j = 0; j < ni; ++j) {
          if (open && lo[j] <= ch + 1) {
            ch = max(ch, hi[j]);
          } else {
            if (open) total += odd_count(cl, ch);
            cl = lo[j];
            ch = hi[j];
            open = true;
          }
        }
        if (open) total += odd_count(cl, ch);
      }
    }
    cnt = (uint32_t)total;
  } else if (nc > 0) {
    const int zlo = axes == 3 ? -a.m : 0;
    const int zhi = axes == 3 ? a.m : 0;
    for (int oz = zlo; oz <= zhi; ++oz) {
      if (axes == 3 && (oz & 1) == 0) continue;
      for (int oy = -a.m; oy <= a.m; ++oy) {
        if ((oy & 1) == 0) continue;
        for (int ox = -a.m; ox <= a.m; ++ox) {
          if ((ox & 1) == 0) continue;
          const long long o2 = (long long)ox * ox + (long long)oy * oy + (long long)oz * oz;
          if ((double)o2 > a.rho2) continue;
          const long long p[3] = {X[0] + ox, X[1] + oy, X[2] + oz};
          bool in = false;
          const int nk = overflow ? a.nsph : nc;
          for (int q = 0; q < nk && !in; ++q) {
            const int k = overflow ? q : cand[q];
            if (!take(k)) continue;
            long long d2 = 0;
            for (int ax = 0; ax < axes; ++ax) {
              const long long d = min_image(p[ax] - a.sph[k].c[ax], a.P[ax]);
              d2 += d * d;
            }
            in = (double)d2 <= a.sph[k].R2;
          }
          cnt += in ? 1u : 0u;
        }
      }
    }
  }
  return cnt;
}

// One thread per voxel.  NPH: counts and fractions per inclusion phase
// (labels 1..nlab, written to [label - 1][voxel]); otherwise one count for
// the union of all spheres and the normal-sphere id.
template <typename T, bool NPH>
__global__ __launch_bounds__(256) void k_filter(FilterArgs a) {
  const long long N = (long long)a.n[0] * a.n[1] * a.n[2];
  const long long v = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (v >= N) return;
  const int x = (int)(v % a.n[0]);
  const int y = (int)((v / a.n[0]) % a.n[1]);
  const int z = (int)(v / ((long long)a.n[0] * a.n[1]));
  const int axes = a.dim == 2 ? 2 : 3;
  const long long X[3] = {(2LL * x + 1) * a.S, (2LL * y + 1) * a.S, (2LL * z + 1) * a.S};
  if constexpr (NPH) {
    for (int p = 1; p <= a.nlab; ++p) {
      const uint32_t c = filter_count(a, X, axes, p);
      a.count[(size_t)(p - 1) * N + v] = c;
      static_cast<T*>(a.frac)[(size_t)(p - 1) * N + v] = (T)c / (T)a.M;
    }
    return;
  }
  const uint32_t cnt = filter_count(a, X, axes, 0);
  a.count[v] = cnt;
  static_cast<T*>(a.frac)[v] = (T)cnt / (T)a.M;
  if (a.incl) {
    int best = -1;
    if (cnt > 0 && cnt < (uint32_t)a.M) {
      double bd = INFINITY;
      for (int k = 0; k < a.nsph; ++k) {
        long long d2 = 0;
        for (int ax = 0; ax < axes; ++ax) {
          const long long d = min_image(X[ax] - a.sph[k].c[ax], a.P[ax]);
          d2 += d * d;
        }
        const double dist = fabs(sqrt((double)d2) - a.sph[k].t);
        if (dist < bd) {
          bd = dist;
          best = k;
        }
      }
    }
    a.incl[v] = best;
  }
}

hipError_t launch_filter(const FilterArgs& a, bool fp64, hipStream_t s) {
  const long long N = (long long)a.n[0] * a.n[1] * a.n[2];
  const dim3 grid((unsigned)((N + 255) / 256));
  if (fp64 && a.lab)
    hipLaunchKernelGGL((k_filter<double, true>), grid, dim3(256), 0, s, a);
  else if (fp64)
    hipLaunchKernelGGL((k_filter<double, false>), grid, dim3(256), 0, s, a);
  else if (a.lab)
    hipLaunchKernelGGL((k_filter<float, true>), grid, dim3(256), 0, s, a);
  else
    hipLaunchKernelGGL((k_filter<float, false>), grid, dim3(256), 0, s, a);
  return hipGetLastError();
}

}  // namespace hm
