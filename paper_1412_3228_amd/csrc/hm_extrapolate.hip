// Post-processing kernels.
//
// Truncated Fourier series (Figure 4): on an odd grid the series with the
// FFT coefficients of a field, evaluated at a point y, is a sum of the grid
// values weighted by the Dirichlet kernel, separable over the axes:
//   F(y) = sum_x c(x) prod_d D_(n_d)(y_d - x_d),
//   D_n(t) = (1/n) sum_{a in J} exp(2 pi i a t) = sin(pi n t) / (n sin(pi t)).
// On a finer grid of m_d points per axis this is three dense contractions
// with (m_d x n_d) matrices, one axis at a time: no transform length
// restrictions on n or m.  The host fills the matrices; the pass along
// contiguous lines is a blocked product on the vector ALUs (lines staged in
// LDS), the strided passes run on the matrix cores.
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

// Matrix-core form of the contractions: one 16 x 16 x 4 MFMA takes a 16 x 4
// tile A (lane l holds row l % 16, column l / 16) and a 4 x 16 tile B (lane
// l holds row l / 16, column l % 16) and accumulates a 16 x 16 tile of C,
// four values per lane: rows l / 16 + 4 m (FP64) or 4 (l / 16) + m (FP32)
// of column l % 16.  A wave owns RT x CT such tiles, a block of four waves
// twice that in each direction (measured on the 125^3 -> 375^3 series:
// FP64 2 x 4, FP32 4 x 4).
template <typename T> struct Mfma;
template <> struct Mfma<double> {
  static constexpr int RT = 2, CT = 4;
  typedef double v4 __attribute__((ext_vector_type(4)));
  static __device__ __forceinline__ v4 mac(double a, double b, v4 c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
  }
  static __device__ __forceinline__ int row(int lane, int m) { return lane / 16 + 4 * m; }
};
template <> struct Mfma<float> {
  static constexpr int RT = 4, CT = 4;
  typedef float v4 __attribute__((ext_vector_type(4)));
  static __device__ __forceinline__ v4 mac(float a, float b, v4 c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
  }
  static __device__ __forceinline__ int row(int lane, int m) { return 4 * (lane / 16) + m; }
};


// Contiguous lines (I == 1): C = In Kt with In[o][j] the (O x n) lines and
// Kt the transposed matrix (n x mj): A tiles are 16 lines x 4 samples (a
// wave's reads of one line over successive steps share cache lines), B
// tiles 4 samples x 16 outputs j' (16 lanes read 16 consecutive entries),
// and each row of C is stored 16 consecutive j' at a time.
template <typename T>
__global__ __launch_bounds__(256) void k_series_lines(const T* __restrict__ in, T* __restrict__ out,
                                                      const T* __restrict__ Kt, long long O, int n, int mj) {
  using M = Mfma<T>;
  using v4 = typename M::v4;
  constexpr int RT = M::RT, CT = M::CT;
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const long long r0 = (long long)blockIdx.y * (2 * 16 * RT) + (wv >> 1) * 16 * RT;
  const int c0 = blockIdx.x * (2 * 16 * CT) + (wv & 1) * 16 * CT;
  const int lr = lane % 16, lk = lane / 16;
  // this lane's lines (clamped inside the field; their results past O are
  // not stored) and outputs (zero past mj)
  long long arow[RT];
#pragma unroll
  for (int a = 0; a < RT; ++a) arow[a] = r0 + 16 * a + lr < O ? r0 + 16 * a + lr : O - 1;
  bool cok[CT];
#pragma unroll
  for (int b = 0; b < CT; ++b) cok[b] = c0 + 16 * b + lr < mj;
  v4 acc[RT][CT];
#pragma unroll
  for (int a = 0; a < RT; ++a)
#pragma unroll
    for (int b = 0; b < CT; ++b) acc[a][b] = v4{T(0), T(0), T(0), T(0)};
#pragma unroll 2
  for (int k0 = 0; k0 < n; k0 += 4) {
    const int k = k0 + lk;
    const bool kok = k < n;
    T av[RT], bv[CT];
#pragma unroll
    for (int a = 0; a < RT; ++a) av[a] = kok ? in[(size_t)arow[a] * n + k] : T(0);
#pragma unroll
    for (int b = 0; b < CT; ++b) bv[b] = (kok && cok[b]) ? Kt[(size_t)k * mj + c0 + 16 * b + lr] : T(0);
#pragma unroll
    for (int a = 0; a < RT; ++a)
#pragma unroll
      for (int b = 0; b < CT; ++b) acc[a][b] = M::mac(av[a], bv[b], acc[a][b]);
  }
#pragma unroll
  for (int a = 0; a < RT; ++a)
#pragma unroll
    for (int m = 0; m < 4; ++m) {
      const long long row = r0 + 16 * a + M::row(lane, m);
      if (row >= O) continue;
#pragma unroll
      for (int b = 0; b < CT; ++b)
        if (cok[b]) out[(size_t)row * mj + c0 + 16 * b + lr] = acc[a][b][m];
    }
}

// Strided axis (I > 1): for each o, C = K In of the (mj x n) matrix and
// the (n x I) slab In[j][i] = in[o][j][i]: A tiles are 16 rows j' x 4 of K
// (stored transposed, so 16 lanes read 16 consecutive rows), B tiles 4 x 16
// consecutive i of the slab, one block per row block and column block
// (blocks that walk the row blocks of their columns, or read K row-major,
// were slower).  The contraction runs in steps of 4 with zeros past n; rows
// or columns past the edges are not stored.
template <typename T>
__global__ __launch_bounds__(256) void k_series_strided(const T* __restrict__ in, T* __restrict__ out,
                                                        const T* __restrict__ Kt, long long I, int n, int mj) {
  using M = Mfma<T>;
  using v4 = typename M::v4;
  constexpr int RT = M::RT, CT = M::CT;
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int r0 = blockIdx.y * (2 * 16 * RT) + (wv >> 1) * 16 * RT;
  const long long c0 = (long long)blockIdx.x * (2 * 16 * CT) + (wv & 1) * 16 * CT;
  const long long o = blockIdx.z;
  const T* src = in + (size_t)o * n * I;
  T* dst = out + (size_t)o * mj * I;
  const int lr = lane % 16, lk = lane / 16;
  // this lane's K rows (clamped inside the matrix; their products past mj
  // are not stored) and In columns (zero past I)
  int arow[RT];
#pragma unroll
  for (int a = 0; a < RT; ++a) arow[a] = min(r0 + 16 * a + lr, mj - 1);
  bool cok[CT];
#pragma unroll
  for (int b = 0; b < CT; ++b) cok[b] = c0 + 16 * b + lr < I;
  v4 acc[RT][CT];
#pragma unroll
  for (int a = 0; a < RT; ++a)
#pragma unroll
    for (int b = 0; b < CT; ++b) acc[a][b] = v4{T(0), T(0), T(0), T(0)};
#pragma unroll 2
  for (int k0 = 0; k0 < n; k0 += 4) {
    const int k = k0 + lk;
    const bool kok = k < n;
    T av[RT], bv[CT];
#pragma unroll
    for (int a = 0; a < RT; ++a) av[a] = kok ? Kt[(size_t)k * mj + arow[a]] : T(0);
#pragma unroll
    for (int b = 0; b < CT; ++b) bv[b] = (kok && cok[b]) ? src[(size_t)k * I + c0 + 16 * b + lr] : T(0);
#pragma unroll
    for (int a = 0; a < RT; ++a)
#pragma unroll
      for (int b = 0; b < CT; ++b) acc[a][b] = M::mac(av[a], bv[b], acc[a][b]);
  }
#pragma unroll
  for (int a = 0; a < RT; ++a)
#pragma unroll
    for (int m = 0; m < 4; ++m) {
      const int row = r0 + 16 * a + M::row(lane, m);
      if (row >= mj) continue;
#pragma unroll
      for (int b = 0; b < CT; ++b)
        if (cok[b]) dst[(size_t)row * I + c0 + 16 * b + lr] = acc[a][b][m];
    }
}

template <typename T> hipError_t series_pass(const AxisPass& p, hipStream_t s) {
  const T* in = static_cast<const T*>(p.in);
  T* out = static_cast<T*>(p.out);
  const T* K = static_cast<const T*>(p.K);
  constexpr int BR = 2 * 16 * Mfma<T>::RT, BC = 2 * 16 * Mfma<T>::CT;
  if (p.I == 1) {
    const dim3 grid((unsigned)((p.mj + BC - 1) / BC), (unsigned)((p.O + BR - 1) / BR));
    hipLaunchKernelGGL((k_series_lines<T>), grid, dim3(256), 0, s, in, out, K, p.O, p.n, p.mj);
  } else {
    const dim3 grid((unsigned)((p.I + BC - 1) / BC), (unsigned)((p.mj + BR - 1) / BR), (unsigned)p.O);
    hipLaunchKernelGGL((k_series_strided<T>), grid, dim3(256), 0, s, in, out, K, p.I, p.n, p.mj);
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
