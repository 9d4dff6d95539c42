// Gradient of a loss of the effective tensor with respect to the phase Lame
// parameters and the per-voxel fraction field.
//
// The discrete Lippmann-Schwinger operator is self-adjoint, so the adjoint
// state of the J-th unit-strain solve is that solve's own field, and at the
// discrete solution dC_KL/dtheta = (1/N) sum_x eps^K : dc~/dtheta : eps^L
// (Hill energy identity).  dc~/dtheta is obtained by forward-mode dual
// numbers through the coefficients of the homogenisation rules of Section 2
// (eqs. 3-5); pure voxels take the phase tensor's own Lame derivatives, the
// fraction derivative always follows the rule's formula.  Accumulation is in
// double whatever the field precision.
#include "hm_adjoint.hpp"
#include "hm_common.hpp"
#include "hm_material.hpp"

namespace hm {

// Value and K partial derivatives.
template <int K> struct Dual {
  double v;
  double d[K];
  __device__ Dual() : v(0.0) {
#pragma unroll
    for (int i = 0; i < K; ++i) d[i] = 0.0;
  }
  __device__ Dual(double x) : v(x) {
#pragma unroll
    for (int i = 0; i < K; ++i) d[i] = 0.0;
  }
};
template <int K> __device__ __forceinline__ Dual<K> operator+(const Dual<K>& a, const Dual<K>& b) {
  Dual<K> r(a.v + b.v);
#pragma unroll
  for (int i = 0; i < K; ++i) r.d[i] = a.d[i] + b.d[i];
  return r;
}
template <int K> __device__ __forceinline__ Dual<K> operator-(const Dual<K>& a, const Dual<K>& b) {
  Dual<K> r(a.v - b.v);
#pragma unroll
  for (int i = 0; i < K; ++i) r.d[i] = a.d[i] - b.d[i];
  return r;
}
template <int K> __device__ __forceinline__ Dual<K> operator*(const Dual<K>& a, const Dual<K>& b) {
  Dual<K> r(a.v * b.v);
#pragma unroll
  for (int i = 0; i < K; ++i) r.d[i] = a.d[i] * b.v + a.v * b.d[i];
  return r;
}
template <int K> __device__ __forceinline__ Dual<K> operator/(const Dual<K>& a, const Dual<K>& b) {
  const double inv = 1.0 / b.v;
  Dual<K> r(a.v * inv);
#pragma unroll
  for (int i = 0; i < K; ++i) r.d[i] = (a.d[i] - r.v * b.d[i]) * inv;
  return r;
}
template <int K> __device__ __forceinline__ Dual<K>& operator-=(Dual<K>& a, const Dual<K>& b) {
  a = a - b;
  return a;
}

using D5 = Dual<5>;  // derivatives: f, lambda_0, mu_0, lambda_1, mu_1

__device__ __forceinline__ Coef<double> slice(const Coef<D5>& c, int i) {
  Coef<double> o;
  o.a1 = c.a1.d[i];
  o.a2 = c.a2.d[i];
  o.a3 = c.a3.d[i];
  o.a4 = c.a4.d[i];
  o.a5 = c.a5.d[i];
  o.aniso = c.aniso;
  o.n[0] = c.n[0].v;
  o.n[1] = c.n[1].v;
  o.n[2] = c.n[2].v;
  return o;
}

// sum_L g^L : A(eps^L), tensor components with doubled shears.
__device__ __forceinline__ double pair_contract(const Coef<double>& A, const double (*eps)[6], const double (*g)[6],
                                                int nl) {
  double s = 0.0;
  for (int L = 0; L < nl; ++L) {
    double t[6];
    apply_form<double>(A, eps[L], t);
    s += g[L][0] * t[0] + g[L][1] * t[1] + g[L][2] * t[2] + 2.0 * (g[L][3] * t[3] + g[L][4] * t[4] + g[L][5] * t[5]);
  }
  return s;
}

template <typename T>
__global__ __launch_bounds__(256) void k_hill(HillArgs a) {
  __shared__ double red[4][4];
  const long long N = (long long)a.n[0] * a.n[1] * a.n[2];
  const long long v = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  double acc[4] = {0.0, 0.0, 0.0, 0.0};
  if (v < N) {
    const int nl = a.n_load;
    double eps[6][6], g[6][6];
    const T* E = static_cast<const T*>(a.eps);
    for (int L = 0; L < nl; ++L)
      for (int c = 0; c < 6; ++c) eps[L][c] = (double)E[((size_t)L * 6 + c) * N + v];
    for (int L = 0; L < nl; ++L)
      for (int c = 0; c < 6; ++c) {
        double s = 0.0;
        for (int K = 0; K < nl; ++K) s += a.G[K * nl + L] * eps[K][c];
        g[L][c] = s;
      }
    const double f = (double)static_cast<const T*>(a.frac)[v];
    const int x = (int)(v % a.n[0]);
    const int y = (int)((v / a.n[0]) % a.n[1]);
    const int z = (int)(v / ((long long)a.n[0] * a.n[1]));
    Coef<D5> cd;
    const int rule = a.rule == RULE_NONE ? RULE_VOIGT : a.rule;
    D5 fd(f), pl[2], pm[2];
    fd.d[0] = 1.0;
    pl[0] = D5(a.pl[0]);
    pl[0].d[1] = 1.0;
    pm[0] = D5(a.pm[0]);
    pm[0].d[2] = 1.0;
    pl[1] = D5(a.pl[1]);
    pl[1].d[3] = 1.0;
    pm[1] = D5(a.pm[1]);
    pm[1].d[4] = 1.0;
    rule_coefficients<D5>(rule, fd, pl, pm, cd);
    if (cd.aniso) {
      double nn[3] = {1.0, 0.0, 0.0};
      const int k = a.incl ? a.incl[v] : -1;
      if (k >= 0 && k < a.nsph) interface_normal<double>(a.sph, k, x, y, z, a.n[0], a.n[1], a.n[2], a.dim, nn);
      for (int i = 0; i < 3; ++i) cd.n[i] = D5(nn[i]);
    }
    double df = 0.0;
    if (a.rule != RULE_NONE) df = pair_contract(slice(cd, 0), eps, g, nl);
    if (f == 0.0 || f == 1.0) {
      const int p = f == 1.0 ? 1 : 0;
      Coef<double> A;
      A.aniso = false;
      A.a3 = A.a4 = A.a5 = 0.0;
      A.a1 = 1.0;
      A.a2 = 0.0;
      acc[2 * p] = pair_contract(A, eps, g, nl);
      A.a1 = 0.0;
      A.a2 = 2.0;
      acc[2 * p + 1] = pair_contract(A, eps, g, nl);
    } else {
      for (int q = 0; q < 4; ++q) acc[q] = pair_contract(slice(cd, q + 1), eps, g, nl);
    }
    if (a.dfrac) static_cast<T*>(a.dfrac)[v] = (T)(df / (double)N);
  }
  // deterministic block sums
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    double s = acc[q];
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) s += __shfl_down(s, off, 64);
    if (lane == 0) red[q][w] = s;
  }
  __syncthreads();
  if (threadIdx.x < 4) {
    const int q = threadIdx.x;
    a.part[(size_t)blockIdx.x * 4 + q] = red[q][0] + red[q][1] + red[q][2] + red[q][3];
  }
}

hipError_t launch_hill(const HillArgs& a, bool fp64, int blocks, hipStream_t s) {
  if (fp64)
    hipLaunchKernelGGL((k_hill<double>), dim3(blocks), dim3(256), 0, s, a);
  else
    hipLaunchKernelGGL((k_hill<float>), dim3(blocks), dim3(256), 0, s, a);
  return hipGetLastError();
}

}  // namespace hm
