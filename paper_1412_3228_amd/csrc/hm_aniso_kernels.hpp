// Anisotropic phases: the rules of Section 2 for two general phase tensors
// (Voigt eq. 3, Reuss eq. 4, 2-layer eq. 5), tabulated once per solve as
// general rows of c~ - c0, and the x-sweep instances that read them.  The
// y- and z-sweeps and the end of the iteration are the elastic ones (the
// reference medium stays isotropic).
//
// Mandel form throughout (order 11, 22, 33, 23, 13, 12, sqrt(2) on shear
// rows and columns): an orthonormal basis of symmetric tensors, so
// rotations act as orthogonal 6x6 matrices and the in-plane / out-of-plane
// split of eq. 5 is a split of the basis.  2-layer rule in the frame
// (t1, t2, n) of the interface normal, with P = {11, 22, 12} and
// O = {33, 23, 13}: both layers share the in-plane strain and the
// out-of-plane stress, so with each layer's blocks A_PP, A_PO, A_OO,
//   S = <A_OO^-1>,  T = <A_OO^-1 A_OP>,
//   C_OO = S^-1,  C_OP = S^-1 T,  C_PO = C_OP',
//   C_PP = <A_PP - A_PO A_OO^-1 A_OP> + T' S^-1 T
// (fraction-weighted means <.>), then rotated back.
#pragma once

#include "hm_solve_kernels.hpp"

namespace hm {

constexpr int kMandelI[6] = {0, 1, 2, 1, 0, 0};
constexpr int kMandelJ[6] = {0, 1, 2, 2, 2, 1};

// In-place inverse of an n x n symmetric positive definite matrix (row
// major) by Gauss-Jordan elimination; no pivoting is needed for SPD input.
template <int n> __device__ __forceinline__ void spd_inverse(double* a) {
  for (int k = 0; k < n; ++k) {
    const double p = 1.0 / a[k * n + k];
    a[k * n + k] = 1.0;
    for (int j = 0; j < n; ++j) a[k * n + j] *= p;
    for (int i = 0; i < n; ++i) {
      if (i == k) continue;
      const double f = a[i * n + k];
      a[i * n + k] = 0.0;
      for (int j = 0; j < n; ++j) a[i * n + j] -= f * a[k * n + j];
    }
  }
}

// Mandel rotation Q (6x6) for the frame whose basis vectors are the
// columns of R: e' = Q e for the components of a symmetric tensor.
__device__ __forceinline__ void mandel_rotation(const double R[3][3], double* Q) {
  const double r2 = 1.41421356237309504880;
  for (int A = 0; A < 6; ++A) {
    const int i = kMandelI[A], j = kMandelJ[A];
    const double wA = A < 3 ? 1.0 : r2;
    for (int B = 0; B < 6; ++B) {
      const int a = kMandelI[B], b = kMandelJ[B];
      Q[A * 6 + B] = B < 3 ? wA * R[a][i] * R[a][j] : wA * (R[a][i] * R[b][j] + R[b][i] * R[a][j]) / r2;
    }
  }
}

// out = Q M Q' (transpose = false) or Q' M Q (transpose = true).
__device__ __forceinline__ void mandel_congruence(const double* Q, const double* M, double* out, bool transpose) {
  double t[36];
  for (int A = 0; A < 6; ++A)
    for (int B = 0; B < 6; ++B) {
      double s = 0.0;
      for (int C = 0; C < 6; ++C) s += (transpose ? Q[C * 6 + A] : Q[A * 6 + C]) * M[C * 6 + B];
      t[A * 6 + B] = s;
    }
  for (int A = 0; A < 6; ++A)
    for (int B = 0; B < 6; ++B) {
      double s = 0.0;
      for (int C = 0; C < 6; ++C) s += t[A * 6 + C] * (transpose ? Q[C * 6 + B] : Q[B * 6 + C]);
      out[A * 6 + B] = s;
    }
}

// The 2-layer tensor of phases M0 (fraction 1 - f) and M1 (fraction f)
// with interface normal n, by the block formula above.
__device__ void laminate_general(double f, const double n[3], const double* M0, const double* M1, double* C) {
  // frame (t1, t2, n)
  double e[3] = {1.0, 0.0, 0.0};
  if (fabs(n[0]) >= 0.9) {
    e[0] = 0.0;
    e[1] = 1.0;
  }
  const double en = e[0] * n[0] + e[1] * n[1] + e[2] * n[2];
  double t1[3] = {e[0] - en * n[0], e[1] - en * n[1], e[2] - en * n[2]};
  const double tl = sqrt(t1[0] * t1[0] + t1[1] * t1[1] + t1[2] * t1[2]);
  for (int i = 0; i < 3; ++i) t1[i] /= tl;
  const double t2[3] = {n[1] * t1[2] - n[2] * t1[1], n[2] * t1[0] - n[0] * t1[2], n[0] * t1[1] - n[1] * t1[0]};
  double R[3][3];
  for (int i = 0; i < 3; ++i) {
    R[i][0] = t1[i];
    R[i][1] = t2[i];
    R[i][2] = n[i];
  }
  double Q[36];
  mandel_rotation(R, Q);
  constexpr int Pi[3] = {0, 1, 5}, Oi[3] = {2, 3, 4};
  double S[9] = {}, T[9] = {}, W[9] = {};
  for (int p = 0; p < 2; ++p) {
    const double w = p == 0 ? 1.0 - f : f;
    double A[36];
    mandel_congruence(Q, p == 0 ? M0 : M1, A, false);
    double iOO[9];
    for (int i = 0; i < 3; ++i)
      for (int j = 0; j < 3; ++j) iOO[i * 3 + j] = A[Oi[i] * 6 + Oi[j]];
    spd_inverse<3>(iOO);
    double iA[9];  // A_OO^-1 A_OP
    for (int i = 0; i < 3; ++i)
      for (int j = 0; j < 3; ++j) {
        double s = 0.0;
        for (int k = 0; k < 3; ++k) s += iOO[i * 3 + k] * A[Oi[k] * 6 + Pi[j]];
        iA[i * 3 + j] = s;
      }
    for (int i = 0; i < 3; ++i)
      for (int j = 0; j < 3; ++j) {
        double s = 0.0;
        for (int k = 0; k < 3; ++k) s += A[Pi[i] * 6 + Oi[k]] * iA[k * 3 + j];
        S[i * 3 + j] += w * iOO[i * 3 + j];
        T[i * 3 + j] += w * iA[i * 3 + j];
        W[i * 3 + j] += w * (A[Pi[i] * 6 + Pi[j]] - s);
      }
  }
  spd_inverse<3>(S);  // S^-1
  double ST[9];       // S^-1 T
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) {
      double s = 0.0;
      for (int k = 0; k < 3; ++k) s += S[i * 3 + k] * T[k * 3 + j];
      ST[i * 3 + j] = s;
    }
  double Cp[36];
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) {
      double s = 0.0;
      for (int k = 0; k < 3; ++k) s += T[k * 3 + i] * ST[k * 3 + j];
      Cp[Oi[i] * 6 + Oi[j]] = S[i * 3 + j];
      Cp[Oi[i] * 6 + Pi[j]] = ST[i * 3 + j];
      Cp[Pi[j] * 6 + Oi[i]] = ST[i * 3 + j];
      Cp[Pi[i] * 6 + Pi[j]] = W[i * 3 + j] + s;
    }
  mandel_congruence(Q, Cp, C, true);
}

// General rows of every fractional voxel (one thread per voxel, rows from
// 2 on through one atomic counter per wavefront, as k_material); rows 0 and
// 1 (the pure phases) are written by the host.  RULE_NONE with a fractional
// voxel raises the flag and uses Voigt.
template <typename T>
__global__ __launch_bounds__(256) void k_material_aniso(const SolveParams* prm, int prob, int nx, int ny, int nz,
                                                        int dim, int* mid, T* coef, int cap, int* count) {
  const ProblemParams& P = prm->probs[prob];
  const int N = nx * ny * nz;
  const int v = blockIdx.x * 256 + threadIdx.x;
  const int lane = threadIdx.x & 63;
  T fT = T(0);
  if (v < N) fT = static_cast<const T*>(P.frac)[v];
  const bool fr = v < N && fT != T(0) && fT != T(1);
  const unsigned long long m = __ballot(fr);
  int base = 0;
  if (m) {
    const int leader = __ffsll((long long)m) - 1;
    if (lane == leader) base = atomicAdd(&count[0], __popcll(m));
    base = __shfl(base, leader, 64);
  }
  if (v >= N) return;
  if (!fr) {
    mid[v] = fT == T(0) ? -1 : -2;
    return;
  }
  const int row = base + __popcll(m & ((1ull << lane) - 1ull));
  mid[v] = row;
  if (row >= cap) return;
  const double f = (double)fT;
  int rule = P.rule;
  if (rule == RULE_NONE) {
    atomicOr(&count[1], FLAG_NONE_FRACTIONAL);
    rule = RULE_VOIGT;
  }
  double C[36];
  if (rule == RULE_REUSS) {
    double S0[36], S1[36];
    for (int i = 0; i < 36; ++i) {
      S0[i] = P.cm[0][i];
      S1[i] = P.cm[1][i];
    }
    spd_inverse<6>(S0);
    spd_inverse<6>(S1);
    for (int i = 0; i < 36; ++i) C[i] = (1.0 - f) * S0[i] + f * S1[i];
    spd_inverse<6>(C);
  } else if (rule == RULE_LAMINATE) {
    double n[3] = {1.0, 0.0, 0.0};
    const int k = P.incl ? P.incl[v] : -1;
    if (k >= P.nsph) atomicOr(&count[1], FLAG_BAD_INCL);
    if (k >= 0 && k < P.nsph) {
      const int x = v % nx, y = (v / nx) % ny, z = v / (nx * ny);
      interface_normal<double>(P.sph, k, x, y, z, nx, ny, nz, dim, n);
    }
    laminate_general(f, n, P.cm[0], P.cm[1], C);
  } else {
    for (int i = 0; i < 36; ++i) C[i] = (1.0 - f) * P.cm[0][i] + f * P.cm[1][i];
  }
  // c~ - c0 (c0 = lambda0 on the normal block + 2 mu0 I), upper triangle
  T* r = coef + (size_t)row * kGenRow;
  int o = 0;
  for (int I = 0; I < 6; ++I)
    for (int J = I; J < 6; ++J) {
      double d = 0.5 * (C[I * 6 + J] + C[J * 6 + I]);
      if (I < 3 && J < 3) d -= P.rl;
      if (I == J) d -= 2.0 * P.rm;
      r[o++] = (T)d;
    }
  for (; o < kGenRow; ++o) r[o] = T(0);
}

// ------------------------------------------------------------ registry --
template <typename T, int NX, int MODE>
hipError_t launch_gx(const SolveArgs& a, hipStream_t s) {
  using TL = XTile<T, NX, 0>;
  hipLaunchKernelGGL((k_xsweep<T, NX, TL::L, TL::NT, MODE, TL::RMAX, true>), dim3(a.g2, a.n_load), dim3(TL::NT), 0,
                     s, a);
  return hipGetLastError();
}

struct AnisoKernels {
  int n;
  XKern x;
};

template <typename T, int N> AnisoKernels make_aniso_kernels() {
  using TL = XTile<T, N, 0>;
  AnisoKernels k;
  k.n = N;
  k.x = XKern{&launch_gx<T, N, MODE_FIRST>, &launch_gx<T, N, MODE_ITER>, &launch_gx<T, N, MODE_EXPORT>, TL::L,
              instance_name<8, T, N, TL::L, TL::NT, MODE_ITER, TL::RMAX, 1>("xsweep")};
  return k;
}

const AnisoKernels* aniso_kernels(bool fp64, int n);

}  // namespace hm
