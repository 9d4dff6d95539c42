// Post-processing kernels.
//
// Truncated Fourier series (Figure 4): on an odd grid the series with the
// FFT coefficients of a field, evaluated at a point y, is a sum of the grid
// values weighted by the Dirichlet kernel, separable over the axes:
//   F(y) = sum_x c(x) prod_d D_(n_d)(y_d - x_d),
//   D_n(t) = (1/n) sum_{a in J} exp(2 pi i a t) = sin(pi n t) / (n sin(pi t)).
// On a finer grid of m_d points per axis this is three dense contractions
// with (m_d x n_d) matrices, one axis at a time: no transform length
// restrictions on n or m.  The host fills the matrices; each pass here is
// a blocked matrix product on the vector ALUs (FP64 matrix cores run at
// the vector rate on this chip, and FP32 ones need no more than the
// contraction's 2 flops per loaded operand).
//
// Stiffness component: the filtered stiffness of Section 2 (eqs. 3-5) at
// each voxel applied to a unit Mandel strain, one Mandel entry kept.
// Stress field: the same stiffness applied to a solve's strain fields; flux
// field: a conduction solve's filtered conductivity applied to its gradients.
#include <math.h>

#include "hm_common.hpp"
#include "hm_extrapolate.hpp"
#include "hm_material.hpp"

namespace hm {

constexpr int kPassThreads = 256;
constexpr int kLinePass = 8;    // lines per block of the contiguous pass
constexpr int kStridedOut = 16; // outputs per thread of the strided pass
constexpr int kStridedCols = 2; // columns per thread of the strided pass

// Contiguous lines (I == 1): a block stages kLinePass input lines in LDS and
// its threads run along the outputs j'; the matrix is read transposed
// (Kt[j][j'], so consecutive threads read consecutive entries) and each
// entry serves all staged lines.
template <typename T>
__global__ __launch_bounds__(kPassThreads) void k_series_lines(const T* in, T* out, const T* Kt, long long O,
                                                               int n, int mj) {
  extern __shared__ unsigned char smem[];
  T* rows = reinterpret_cast<T*>(smem);  // [kLinePass][n]
  const long long o0 = (long long)blockIdx.y * kLinePass;
  const int jp = blockIdx.x * kPassThreads + threadIdx.x;
  for (int e = threadIdx.x; e < kLinePass * n; e += kPassThreads) {
    const int l = e / n, j = e - (e / n) * n;
    rows[e] = o0 + l < O ? in[(o0 + l) * n + j] : T(0);
  }
  __syncthreads();
  if (jp >= mj) return;
  T acc[kLinePass];
#pragma unroll
  for (int l = 0; l < kLinePass; ++l) acc[l] = T(0);
  for (int j = 0; j < n; ++j) {
    const T k = Kt[(size_t)j * mj + jp];
#pragma unroll
    for (int l = 0; l < kLinePass; ++l) acc[l] += rows[l * n + j] * k;
  }
#pragma unroll
  for (int l = 0; l < kLinePass; ++l)
    if (o0 + l < O) out[(o0 + l) * mj + jp] = acc[l];
}

// Strided axis (I > 1): threads run along i (coalesced), each computes
// kStridedOut consecutive outputs j' for kStridedCols columns i (256 apart,
// so every load stays coalesced).  The matrix entries are the same for every
// thread of the block, so they are read through the scalar cache (read-only,
// no aliasing) and each one feeds kStridedCols multiply-adds; each loaded
// input value feeds kStridedOut.  (Tile measured on the 125^3 -> 375^3
// series: 16 x 2 beat 32 x 1, 16 x 1, 8 x 4, 16 x 4 and 12 x 3.)
template <typename T>
__global__ __launch_bounds__(kPassThreads) void k_series_strided(const T* __restrict__ in, T* __restrict__ out,
                                                                 const T* __restrict__ K, long long I, int n,
                                                                 int mj) {
  const long long ib = (long long)blockIdx.x * kPassThreads * kStridedCols + threadIdx.x;
  const int j0 = blockIdx.y * kStridedOut;
  const long long o = blockIdx.z;
  bool ok[kStridedCols];
#pragma unroll
  for (int c = 0; c < kStridedCols; ++c) ok[c] = ib + (long long)kPassThreads * c < I;
  T acc[kStridedOut][kStridedCols];
#pragma unroll
  for (int t = 0; t < kStridedOut; ++t)
#pragma unroll
    for (int c = 0; c < kStridedCols; ++c) acc[t][c] = T(0);
  const T* src = in + (size_t)o * n * I + ib;
  // rows past mj repeat the last row (their results are not stored)
  const T* kr = K + (size_t)j0 * n;
  const int tmax = mj - 1 - j0;
#pragma unroll 2
  for (int j = 0; j < n; ++j) {
    T v[kStridedCols];
#pragma unroll
    for (int c = 0; c < kStridedCols; ++c) v[c] = ok[c] ? src[(size_t)j * I + kPassThreads * c] : T(0);
#pragma unroll
    for (int t = 0; t < kStridedOut; ++t) {
      const T k = kr[(size_t)(t < tmax ? t : tmax) * n + j];
#pragma unroll
      for (int c = 0; c < kStridedCols; ++c) acc[t][c] += k * v[c];
    }
  }
  T* dst = out + (size_t)o * mj * I + ib;
#pragma unroll
  for (int t = 0; t < kStridedOut; ++t)
#pragma unroll
    for (int c = 0; c < kStridedCols; ++c)
      if (j0 + t < mj && ok[c]) dst[(size_t)(j0 + t) * I + kPassThreads * c] = acc[t][c];
}

template <typename T> hipError_t series_pass(const AxisPass& p, hipStream_t s) {
  const T* in = static_cast<const T*>(p.in);
  T* out = static_cast<T*>(p.out);
  const T* K = static_cast<const T*>(p.K);
  if (p.I == 1) {
    const dim3 grid((unsigned)((p.mj + kPassThreads - 1) / kPassThreads), (unsigned)((p.O + kLinePass - 1) / kLinePass));
    hipLaunchKernelGGL((k_series_lines<T>), grid, dim3(kPassThreads), (size_t)kLinePass * p.n * sizeof(T), s, in, out,
                       K, p.O, p.n, p.mj);
  } else {
    const long long cols = (long long)kPassThreads * kStridedCols;
    const dim3 grid((unsigned)((p.I + cols - 1) / cols), (unsigned)((p.mj + kStridedOut - 1) / kStridedOut),
                    (unsigned)p.O);
    hipLaunchKernelGGL((k_series_strided<T>), grid, dim3(kPassThreads), 0, s, in, out, K, p.I, p.n, p.mj);
  }
  return hipGetLastError();
}

hipError_t launch_series_pass(const AxisPass& p, bool fp64, hipStream_t s) {
  return fp64 ? series_pass<double>(p, s) : series_pass<float>(p, s);
}

// Filtered stiffness c~ of voxel v in the transversely isotropic form of
// hm_material.hpp, in double: the phase tensor where f is 0 or 1, else the
// rule at f (flags as StiffnessArgs describes).
template <typename T> __device__ Coef<double> voxel_coef(const StiffnessArgs& a, long long v) {
  const double f = (double)static_cast<const T*>(a.frac)[v];
  Coef<double> c;
  c.n[0] = c.n[1] = c.n[2] = 0.0;
  c.a3 = c.a4 = c.a5 = 0.0;
  c.aniso = false;
  if (f == 0.0 || f == 1.0) {
    const int p = f == 0.0 ? 0 : 1;
    c.a1 = a.pl[p];
    c.a2 = 2.0 * a.pm[p];
  } else {
    int rule = a.rule;
    if (rule == RULE_NONE) {
      atomicOr(a.flags, 1);
      rule = RULE_VOIGT;
    }
    rule_coefficients<double>(rule, f, a.pl, a.pm, c);
    if (c.aniso) {
      const int k = a.incl ? a.incl[v] : -1;
      if (k >= a.nsph) atomicOr(a.flags, 2);
      if (k >= 0 && k < a.nsph) {
        const int x = (int)(v % a.n[0]), y = (int)((v / a.n[0]) % a.n[1]), z = (int)(v / ((long long)a.n[0] * a.n[1]));
        interface_normal<double>(a.sph, k, x, y, z, a.n[0], a.n[1], a.n[2], a.dim, c.n);
      } else {
        c.n[0] = 1.0;
      }
    }
  }
  return c;
}

template <typename T>
__global__ __launch_bounds__(256) void k_stiffness_component(StiffnessArgs a) {
  const long long N = (long long)a.n[0] * a.n[1] * a.n[2];
  const long long v = (long long)blockIdx.x * 256 + threadIdx.x;
  if (v >= N) return;
  const Coef<double> c = voxel_coef<T>(a, v);
  // unit Mandel strain J as tensor components, Mandel entry I of the stress
  const double r2 = 1.4142135623730950488;
  double e[6] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0}, s6[6];
  e[a.J] = a.J < 3 ? 1.0 : 1.0 / r2;
  apply_form<double>(c, e, s6);
  static_cast<T*>(a.out)[v] = (T)(a.I < 3 ? s6[a.I] : r2 * s6[a.I]);
}

template <typename T>
__global__ __launch_bounds__(256) void k_stress_field(StressArgs a) {
  const long long N = (long long)a.m.n[0] * a.m.n[1] * a.m.n[2];
  const long long v = (long long)blockIdx.x * 256 + threadIdx.x;
  if (v >= N) return;
  const Coef<double> c = voxel_coef<T>(a.m, v);
  const T* eps = static_cast<const T*>(a.eps);
  T* sig = static_cast<T*>(a.sig);
  for (int l = 0; l < a.n_load; ++l) {
    double e[6], s6[6];
#pragma unroll
    for (int k = 0; k < 6; ++k) e[k] = (double)eps[((size_t)l * 6 + k) * N + v];
    apply_form<double>(c, e, s6);
#pragma unroll
    for (int k = 0; k < 6; ++k) sig[((size_t)l * 6 + k) * N + v] = (T)s6[k];
  }
}

hipError_t launch_stress_field(const StressArgs& a, bool fp64, hipStream_t s) {
  const long long N = (long long)a.m.n[0] * a.m.n[1] * a.m.n[2];
  const dim3 grid((unsigned)((N + 255) / 256));
  if (fp64)
    hipLaunchKernelGGL((k_stress_field<double>), grid, dim3(256), 0, s, a);
  else
    hipLaunchKernelGGL((k_stress_field<float>), grid, dim3(256), 0, s, a);
  return hipGetLastError();
}

// Local flux: the conductivity of voxel v is k_p where f is 0 or 1, else
// the rule at f (Voigt <k>, Reuss <1/k>^-1, 2-layer <k> along the interface
// and <1/k>^-1 across it), held as k~ = a I + b n (x) n and applied to each
// gradient field.
template <typename T>
__global__ __launch_bounds__(256) void k_flux_field(StressArgs a) {
  const StiffnessArgs& m = a.m;
  const long long N = (long long)m.n[0] * m.n[1] * m.n[2];
  const long long v = (long long)blockIdx.x * 256 + threadIdx.x;
  if (v >= N) return;
  const double f = (double)static_cast<const T*>(m.frac)[v];
  double ka = f == 0.0 ? m.pl[0] : m.pl[1], kb = 0.0;
  double n[3] = {0.0, 0.0, 0.0};
  if (f != 0.0 && f != 1.0) {
    int rule = m.rule;
    if (rule == RULE_NONE) {
      atomicOr(m.flags, 1);
      rule = RULE_VOIGT;
    }
    const double arith = (1.0 - f) * m.pl[0] + f * m.pl[1];
    const double harm = 1.0 / ((1.0 - f) / m.pl[0] + f / m.pl[1]);
    ka = rule == RULE_REUSS ? harm : arith;
    if (rule == RULE_LAMINATE) {
      kb = harm - arith;
      const int k = m.incl ? m.incl[v] : -1;
      if (k >= m.nsph) atomicOr(m.flags, 2);
      if (k >= 0 && k < m.nsph) {
        const int x = (int)(v % m.n[0]), y = (int)((v / m.n[0]) % m.n[1]), z = (int)(v / ((long long)m.n[0] * m.n[1]));
        interface_normal<double>(m.sph, k, x, y, z, m.n[0], m.n[1], m.n[2], m.dim, n);
      } else {
        n[0] = 1.0;
      }
    }
  }
  const T* g = static_cast<const T*>(a.eps);
  T* q = static_cast<T*>(a.sig);
  for (int l = 0; l < a.n_load; ++l) {
    double gv[3];
#pragma unroll
    for (int c = 0; c < 3; ++c) gv[c] = (double)g[((size_t)l * 3 + c) * N + v];
    const double ng = n[0] * gv[0] + n[1] * gv[1] + n[2] * gv[2];
#pragma unroll
    for (int c = 0; c < 3; ++c) q[((size_t)l * 3 + c) * N + v] = (T)(ka * gv[c] + kb * ng * n[c]);
  }
}

hipError_t launch_flux_field(const StressArgs& a, bool fp64, hipStream_t s) {
  const long long N = (long long)a.m.n[0] * a.m.n[1] * a.m.n[2];
  const dim3 grid((unsigned)((N + 255) / 256));
  if (fp64)
    hipLaunchKernelGGL((k_flux_field<double>), grid, dim3(256), 0, s, a);
  else
    hipLaunchKernelGGL((k_flux_field<float>), grid, dim3(256), 0, s, a);
  return hipGetLastError();
}

hipError_t launch_stiffness_component(const StiffnessArgs& a, bool fp64, hipStream_t s) {
  const long long N = (long long)a.n[0] * a.n[1] * a.n[2];
  const dim3 grid((unsigned)((N + 255) / 256));
  if (fp64)
    hipLaunchKernelGGL((k_stiffness_component<double>), grid, dim3(256), 0, s, a);
  else
    hipLaunchKernelGGL((k_stiffness_component<float>), grid, dim3(256), 0, s, a);
  return hipGetLastError();
}

}  // namespace hm
