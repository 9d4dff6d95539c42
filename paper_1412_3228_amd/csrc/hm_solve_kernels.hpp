// Kernels of one fixed-point iteration of the Lippmann-Schwinger solve
// (Section 2, eqs. 1-a, 1-b, 2) on an odd grid.
//
// Storage between iterations: the x-spectrum of the strain, i.e. for every
// (load, component, z, y) the half line kx = 0..(nx-1)/2 of the DFT along x
// (the other half follows by Hermitian symmetry of real data).  One
// iteration is four sweeps over that array:
//   xsweep  inverse x-DFT -> strain at the grid points -> polarization
//           tau = (c~ - c0) : eps -> forward x-DFT; per-block sums of tau
//   ysweep  forward y-DFT of every (component, z, kx) line
//   zsweep  forward z-DFT, eps^ = -Gamma0^ : tau^ (eps^(0) = E), the
//           equilibrium-error partial sums, inverse z-DFT
//   ysweep  inverse y-DFT; seven of its blocks per load case reduce the
//           partial sums and the last takes the error, the mean stress and
//           the stop decision
// The six real strain components are transformed as three complex lines
// (11 + i 22, 33 + i 23, 13 + i 12), which is exact for real data of any
// (odd) length.  The 1/N of the inverse transform is applied in zsweep.
//
// Equilibrium error: for xi != 0 and i >= 1, xi . sigma^_i =
// xi . (tau^_i - tau^_(i-1)) because xi . (c0 : Gamma0^ : t) = xi . t, and
// xi . sigma^_0 = xi . tau^_0 for the uniform first iterate.  zsweep keeps
// a_i = tau^_i . n (n = xi / |xi|) from the previous iteration and
// accumulates sum_xi w |xi|^2 |a_i - a_(i-1)|^2 over the half spectrum
// (w = 1 at kx = 0, 2 elsewhere).
#pragma once

#include <algorithm>
#include <cstdio>

#include "hm_common.hpp"
#include "hm_fft.hpp"
#include "hm_material.hpp"

namespace hm {

enum : int { MODE_FIRST = 0, MODE_ITER = 1, MODE_EXPORT = 2 };

// Block size of the CG scalar kernels (one block per load case).
constexpr int kCgScalarThreads = 1024;

// Deterministic block sum (fixed shuffle tree, then waves in order); the
// result is valid in thread 0.
template <int NT>
__device__ __forceinline__ double block_sum(double v, double* red) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  if (lane == 0) red[w] = v;
  __syncthreads();
  double s = 0.0;
  if (threadIdx.x == 0) {
#pragma unroll
    for (int i = 0; i < NT / 64; ++i) s += red[i];
  }
  __syncthreads();
  return s;
}

// Filtered stiffness of every fractional voxel, computed once per solve
// (one thread per voxel of problem `prob`): rows of coef are handed out per
// wavefront through one atomic counter (count[0]); the row order does not
// affect any result.  count[1] collects the data flags.  Rows at or beyond
// `cap` are not written; the caller re-runs with a larger table.
// COND: conduction rows (a - k0, b, 0, 0, 0, n) of k~ = a I + b n (x) n,
// from the phase conductivities in pl: Voigt a = <k>, b = 0; Reuss
// a = <1/k>^-1, b = 0; 2-layer a = <k>, b = <1/k>^-1 - <k> (layers in
// parallel along the interface, in series across it).
template <typename T, bool COND = false>
__global__ __launch_bounds__(256) void k_material(const SolveParams* prm, int prob, int nx, int ny, int nz, int dim,
                                                  int* mid, T* coef, int cap, int* count) {
  const ProblemParams& P = prm->probs[prob];
  const int N = nx * ny * nz;
  const int v = blockIdx.x * 256 + threadIdx.x;
  const int lane = threadIdx.x & 63;
  T f = T(0);
  if (v < N) f = static_cast<const T*>(P.frac)[v];
  const bool fr = v < N && f != T(0) && f != T(1);
  const unsigned long long m = __ballot(fr);
  int base = 0;
  if (m) {
    const int leader = __ffsll((long long)m) - 1;
    if (lane == leader) base = atomicAdd(&count[0], __popcll(m));
    base = __shfl(base, leader, 64);
  }
  if (v >= N) return;
  if (!fr) {
    mid[v] = f == T(0) ? -1 : -2;
    return;
  }
  const int row = base + __popcll(m & ((1ull << lane) - 1ull));
  mid[v] = row;
  const T pl[2] = {T(P.pl[0]), T(P.pl[1])};
  const T pm[2] = {T(P.pm[0]), T(P.pm[1])};
  int rule = P.rule;
  if (rule == RULE_NONE) {
    atomicOr(&count[1], FLAG_NONE_FRACTIONAL);
    rule = RULE_VOIGT;
  }
  Coef<T> c;
  c.n[0] = c.n[1] = c.n[2] = T(0);
  if constexpr (COND) {
    const T g = T(1) - f;
    const T arith = g * pl[0] + f * pl[1];
    const T harm = T(1) / (g / pl[0] + f / pl[1]);
    c.a1 = rule == RULE_REUSS ? harm : arith;
    c.a2 = rule == RULE_LAMINATE ? harm - arith : T(0);
    c.a3 = c.a4 = c.a5 = T(0);
    c.aniso = rule == RULE_LAMINATE;
  } else {
    rule_coefficients<T>(rule, f, pl, pm, c);
  }
  if (c.aniso) {
    const int k = P.incl ? P.incl[v] : -1;
    if (k >= P.nsph) atomicOr(&count[1], FLAG_BAD_INCL);
    if (k >= 0 && k < P.nsph) {
      const int x = v % nx, y = (v / nx) % ny, z = v / (nx * ny);
      interface_normal<T>(P.sph, k, x, y, z, nx, ny, nz, dim, c.n);
    } else {
      c.n[0] = T(1);
      c.n[1] = T(0);
      c.n[2] = T(0);
    }
  }
  if (row < cap) {
    T* r = coef + (size_t)row * 8;
    r[0] = c.a1 - T(P.rl);
    r[1] = COND ? c.a2 : c.a2 - T(2.0 * P.rm);
    r[2] = c.a3;
    r[3] = c.a4;
    r[4] = c.a5;
    r[5] = c.n[0];
    r[6] = c.n[1];
    r[7] = c.n[2];
  }
}

// Multi-phase form of k_material (eqs. 3-4 with Nphase phases): fractions
// f_1..f_(P-1) of the voxel, f_0 = 1 - (f_1 + ... + f_(P-1)); all zero is
// pure matrix (-1), f_1 = 1 pure phase 1 (-2), f_p = 1 for p >= 2 the
// reserved row p - 2; fractional voxels take a new row with the Voigt
// (sum f_i lambda_i, sum f_i mu_i) or Reuss (K = 1 / sum f_i / K_i,
// mu = 1 / sum f_i / mu_i) isotropic tensor.  count[0] starts at the number
// of reserved rows.
template <typename T>
__global__ __launch_bounds__(256) void k_material_nphase(const SolveParams* prm, int prob, int nx, int ny, int nz,
                                                         int* mid, T* coef, int cap, int* count) {
  const ProblemParams& P = prm->probs[prob];
  const int N = nx * ny * nz;
  const int v = blockIdx.x * 256 + threadIdx.x;
  const int lane = threadIdx.x & 63;
  const T* fr = static_cast<const T*>(P.frac);
  const int np = P.nphase;
  constexpr int kFractional = 1 << 30;
  T sum = T(0);
  int pure = kFractional;  // or -1 / -2: pure matrix / phase 1, r >= 0: reserved row
  if (v < N) {
    bool any = false;
    for (int p = 1; p < np; ++p) {
      const T f = fr[(size_t)(p - 1) * N + v];
      sum += f;
      any = any || f != T(0);
      if (f == T(1) && pure == kFractional) pure = p == 1 ? -2 : p - 2;
    }
    if (!any) pure = -1;
  }
  const bool frac_voxel = v < N && pure == kFractional;
  const unsigned long long m = __ballot(frac_voxel);
  int base = 0;
  if (m) {
    const int leader = __ffsll((long long)m) - 1;
    if (lane == leader) base = atomicAdd(&count[0], __popcll(m));
    base = __shfl(base, leader, 64);
  }
  if (v >= N) return;
  if (!frac_voxel) {
    mid[v] = pure;
    return;
  }
  const int row = base + __popcll(m & ((1ull << lane) - 1ull));
  mid[v] = row;
  int rule = P.rule;
  if (rule != RULE_VOIGT && rule != RULE_REUSS) {
    atomicOr(&count[1], FLAG_NONE_FRACTIONAL);
    rule = RULE_VOIGT;
  }
  const T f0 = T(1) - sum;
  T a1, a2;
  if (rule == RULE_REUSS) {
    T sk = f0 / (T(P.ph_l[0]) + T(2.0 / 3.0) * T(P.ph_m[0]));
    T sm = f0 / T(P.ph_m[0]);
    for (int p = 1; p < np; ++p) {
      const T f = fr[(size_t)(p - 1) * N + v];
      sk += f / (T(P.ph_l[p]) + T(2.0 / 3.0) * T(P.ph_m[p]));
      sm += f / T(P.ph_m[p]);
    }
    const T K = T(1) / sk, mu = T(1) / sm;
    a1 = K - T(2.0 / 3.0) * mu;
    a2 = T(2) * mu;
  } else {
    T l = f0 * T(P.ph_l[0]), u = f0 * T(P.ph_m[0]);
    for (int p = 1; p < np; ++p) {
      const T f = fr[(size_t)(p - 1) * N + v];
      l += f * T(P.ph_l[p]);
      u += f * T(P.ph_m[p]);
    }
    a1 = l;
    a2 = T(2) * u;
  }
  if (row < cap) {
    T* r = coef + (size_t)row * 8;
    r[0] = a1 - T(P.rl);
    r[1] = a2 - T(2.0 * P.rm);
#pragma unroll
    for (int i = 2; i < 8; ++i) r[i] = T(0);
  }
}

// Material constants of one problem in the working precision, copied into
// registers once per block (the voxel loop stores to global memory, so
// values read through the parameter pointer would otherwise be re-read for
// every voxel).
template <typename T> struct VoxelMaterial {
  T pure[4];  // (a1 - lambda0, a2 - 2 mu0) of the matrix, then the inclusion
  const T* coef;
  const int* mid;
  bool aniso;  // the rule's table rows use the normal
};

template <typename T> __device__ __forceinline__ VoxelMaterial<T> load_material(const ProblemParams& P) {
  VoxelMaterial<T> m;
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    if constexpr (sizeof(T) == 4)
      m.pure[i] = P.pure_f[i];
    else
      m.pure[i] = P.pure_d[i];
  }
  m.coef = static_cast<const T*>(P.coef);
  m.mid = P.mid;
  m.aniso = P.rule == RULE_LAMINATE;
  return m;
}

// Load through a pointer known to address device global memory (pointers
// read from the parameter blob are generic to the compiler, which would
// otherwise issue flat loads that also wait on the LDS counter).
template <typename V> __device__ __forceinline__ V load_global(const V* p) {
  return *(const __attribute__((address_space(1))) V*)(p);
}

// Eight table entries as two (FP32) or four (FP64) 16-byte loads; rows are
// 32 or 64 bytes, so every load is aligned.
typedef float v4f __attribute__((ext_vector_type(4)));
typedef double v2d __attribute__((ext_vector_type(2)));
template <typename T> __device__ __forceinline__ void load_row8(const T* r, T v[8]) {
  if constexpr (sizeof(T) == 4) {
    const v4f u0 = load_global(reinterpret_cast<const v4f*>(r));
    const v4f u1 = load_global(reinterpret_cast<const v4f*>(r) + 1);
    v[0] = u0.x; v[1] = u0.y; v[2] = u0.z; v[3] = u0.w;
    v[4] = u1.x; v[5] = u1.y; v[6] = u1.z; v[7] = u1.w;
  } else {
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const v2d u = load_global(reinterpret_cast<const v2d*>(r) + i);
      v[2 * i] = u.x;
      v[2 * i + 1] = u.y;
    }
  }
}

// The traction history is read and written once per iteration, by the
// z-sweep only: its accesses are marked non-temporal, so that the caches
// keep the spectrum, which every sweep reads and writes.
typedef float v2f __attribute__((ext_vector_type(2)));
template <typename T> __device__ __forceinline__ cx<T> load_stream(const cx<T>* p) {
  if constexpr (sizeof(T) == 4) {
    const v2f u = __builtin_nontemporal_load(reinterpret_cast<const v2f*>(p));
    return cx<T>{u.x, u.y};
  } else {
    const v2d u = __builtin_nontemporal_load(reinterpret_cast<const v2d*>(p));
    return cx<T>{u.x, u.y};
  }
}
template <typename T> __device__ __forceinline__ void store_stream(cx<T>* p, cx<T> v) {
  if constexpr (sizeof(T) == 4)
    __builtin_nontemporal_store(v2f{v.x, v.y}, reinterpret_cast<v2f*>(p));
  else
    __builtin_nontemporal_store(v2d{v.x, v.y}, reinterpret_cast<v2d*>(p));
}

// Stiffness row (a1 - lambda0, a2 - 2 mu0, a3, a4, a5, n) of the voxel with
// material id mv: a pure phase, or a row of the table (one global gather).
template <typename T> __device__ __forceinline__ void material_row(const VoxelMaterial<T>& M, int mv, T r[8]) {
  r[0] = mv == -1 ? M.pure[0] : M.pure[2];
  r[1] = mv == -1 ? M.pure[1] : M.pure[3];
#pragma unroll
  for (int i = 2; i < 8; ++i) r[i] = T(0);
  if (mv >= 0) load_row8<T>(M.coef + (size_t)mv * 8, r);
}

// Polarization tau = (c~ - c0) : e from a stiffness row.
template <typename T> __device__ __forceinline__ void row_tau(bool aniso, const T r[8], const T e[6], T tau[6]) {
  const Coef<T> c = {r[0], r[1], r[2], r[3], r[4], {r[5], r[6], r[7]}, aniso};
  apply_form<T>(c, e, tau);
}

// Polarization from a general (anisotropic) table row: the upper triangle,
// row by row, of the Mandel matrix D = c~ - c0 (21 reals, then 3 of
// padding); pure matrix (-1) and pure inclusion (-2) voxels use rows 0 and
// 1.  tau = D e in Mandel form, e and tau as tensor components.
constexpr int kGenRow = 24;
template <typename T> __device__ __forceinline__ void gen_tau(const T* coef, int mv, const T e[6], T tau[6]) {
  const int row = mv == -1 ? 0 : (mv == -2 ? 1 : mv);
  const T* r = coef + (size_t)row * kGenRow;
  T d[kGenRow];
  if constexpr (sizeof(T) == 4) {
#pragma unroll
    for (int i = 0; i < kGenRow / 4; ++i) {
      const v4f u = load_global(reinterpret_cast<const v4f*>(r) + i);
      d[4 * i] = u.x;
      d[4 * i + 1] = u.y;
      d[4 * i + 2] = u.z;
      d[4 * i + 3] = u.w;
    }
  } else {
#pragma unroll
    for (int i = 0; i < kGenRow / 2; ++i) {
      const v2d u = load_global(reinterpret_cast<const v2d*>(r) + i);
      d[2 * i] = u.x;
      d[2 * i + 1] = u.y;
    }
  }
  const T r2 = T(1.41421356237309504880), ir2 = T(0.70710678118654752440);
  const T em[6] = {e[0], e[1], e[2], r2 * e[3], r2 * e[4], r2 * e[5]};
  T sv[6] = {T(0), T(0), T(0), T(0), T(0), T(0)};
#pragma unroll
  for (int I = 0; I < 6; ++I)
#pragma unroll
    for (int J = 0; J < 6; ++J) {
      const int a = I < J ? I : J, b = I < J ? J : I;
      sv[I] += d[a * 6 - a * (a - 1) / 2 + (b - a)] * em[J];
    }
#pragma unroll
  for (int c = 0; c < 6; ++c) tau[c] = c < 3 ? sv[c] : ir2 * sv[c];
}

// ---------------------------------------------------------------- xsweep --
// A block owns L consecutive (y, z) lines.  All of its global reads (the
// six half-lines of each line and the material of its voxels) are issued
// into registers before any LDS work, so each block keeps its whole input
// in flight at once.  Element loops give each wavefront whole rows (a
// component pair of one line, or one line of voxels) with the lanes along
// kx or x, so row indices are wave-uniform and need no per-lane division.
// GEN: general (anisotropic) material rows, gathered per voxel in the
// polarization pass instead of before it.
// Single-precision blocks of 4 or more lines are held to 5 waves per SIMD
// (96 registers): the radix-27 form then fits without spills.
template <typename T, int L> constexpr int xsweep_min_waves() { return sizeof(T) == 4 && L >= 4 ? 5 : 1; }

template <typename T, int NX, int L, int NT, int MODE, int RMAX = max_radix<T>(), bool GEN = false>
__global__ __launch_bounds__(NT, (xsweep_min_waves<T, L>())) void k_xsweep(SolveArgs a) {
  constexpr int LL = 3 * L;
  constexpr int LD = LL | 1;  // odd row stride: element rows spread over the banks
  constexpr int H = (NX + 1) / 2;
  constexpr int NW = NT / 64;                   // waves
  constexpr int KH = (H + 63) / 64;             // 64-lane chunks of a half line
  constexpr int KX = (NX + 63) / 64;            // 64-lane chunks of a line
  constexpr int RP = (LL + NW - 1) / NW;        // (pair, line) rows per wave
  constexpr int RV = (L + NW - 1) / NW;         // voxel lines per wave
  __shared__ cx<T> buf[NX * LD];
  __shared__ cx<T> s_tw[NX];
  __shared__ double red[6][NW];
  const int tid = threadIdx.x;
  const int wv = tid >> 6, lane = tid & 63;
  const int load = blockIdx.y;
  SolverState* st = a.state + load;
  if (MODE != MODE_EXPORT && st->done) return;
  const LoadParams& LP = a.prm->loads[load];
  const ProblemParams& P = a.prm->probs[LP.prob];
  const VoxelMaterial<T> MAT = load_material<T>(P);
  const int nlines = a.ny * a.nz;
  const int line0 = blockIdx.x * L;
  const int Hp = a.Hp;
  const size_t cs = (size_t)nlines * Hp;
  cx<T>* spec = static_cast<cx<T>*>(a.spec) + (size_t)load * 6 * cs;
  const cx<T>* src = static_cast<const cx<T>*>(a.spec_in) + (size_t)load * 6 * cs;

  // row r = p * L + l: component pair p of line l (wave-uniform)
  cx<T> pa[RP][KH], pb[RP][KH];
  if (MODE != MODE_FIRST) {
#pragma unroll
    for (int i = 0; i < RP; ++i) {
      const int r = wv + NW * i;
      const int p = r / L, l = r - (r / L) * L;
      const int line = line0 + l;
      const bool rok = r < LL && line < nlines;
      const cx<T>* ra = src + (size_t)(2 * p) * cs + (size_t)line * Hp;
      const cx<T>* rb = ra + cs;
#pragma unroll
      for (int m = 0; m < KH; ++m) {
        const int k = lane + 64 * m;
        const bool ok = rok && k < H;
        pa[i][m] = ok ? ra[k] : cx<T>{T(0), T(0)};
        pb[i][m] = ok ? rb[k] : cx<T>{T(0), T(0)};
      }
    }
  }
  int mv[RV][KX];
  if (MODE != MODE_EXPORT) {
#pragma unroll
    for (int i = 0; i < RV; ++i) {
      const int l = wv + NW * i;
      const int line = line0 + l;
      const bool rok = l < L && line < nlines;
#pragma unroll
      for (int m = 0; m < KX; ++m) {
        const int x = lane + 64 * m;
        mv[i][m] = (rok && x < NX) ? load_global(MAT.mid + (size_t)line * NX + x) : -1;
      }
    }
  }
  load_twiddles<T, NX, NT>(s_tw, static_cast<const cx<T>*>(a.twx), tid);

  if (MODE != MODE_FIRST) {
#pragma unroll
    for (int i = 0; i < RP; ++i) {
      const int r = wv + NW * i;
      if (r >= LL) continue;
      const int p = r / L, l = r - (r / L) * L;
      const int col = p * L + l;
#pragma unroll
      for (int m = 0; m < KH; ++m) {
        const int k = lane + 64 * m;
        if (k < H) {
          const cx<T> A = pa[i][m], B = pb[i][m];
          buf[k * LD + col] = cx<T>{A.x - B.y, A.y + B.x};
          if (k > 0) buf[(NX - k) * LD + col] = cx<T>{A.x + B.y, B.x - A.y};
        }
      }
    }
    __syncthreads();
    fft_lines<T, NX, LL, NT, +1, LD, RMAX>(buf, s_tw, tid);
  }

  if (MODE == MODE_EXPORT) {
    const size_t N = (size_t)nlines * NX;
    T* out = static_cast<T*>(a.eps_out) + (size_t)load * 6 * N;
    for (int l = wv; l < L; l += NW) {
      const int line = line0 + l;
      if (line >= nlines) continue;
      for (int x = lane; x < NX; x += 64) {
#pragma unroll
        for (int p = 0; p < 3; ++p) {
          // a CG iterate is stored as its zero-mean fluctuation
          const cx<T> Z = buf[x * LD + p * L + l];
          out[(size_t)(2 * p) * N + (size_t)line * NX + x] = Z.x + (a.cg ? T(LP.E[2 * p]) : T(0));
          out[(size_t)(2 * p + 1) * N + (size_t)line * NX + x] = Z.y + (a.cg ? T(LP.E[2 * p + 1]) : T(0));
        }
      }
    }
    return;
  }

  // all table gathers of the thread's voxels first, then the polarizations
  T rows[RV][KX][8];
  if constexpr (!GEN) {
#pragma unroll
    for (int i = 0; i < RV; ++i)
#pragma unroll
      for (int m = 0; m < KX; ++m) material_row<T>(MAT, mv[i][m], rows[i][m]);
  }
  double acc[6] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};  // FP64 thread partials, then FP64 block sums
#pragma unroll
  for (int i = 0; i < RV; ++i) {
    const int l = wv + NW * i;
    if (l >= L) continue;
    const int line = line0 + l;
#pragma unroll
    for (int m = 0; m < KX; ++m) {
      const int x = lane + 64 * m;
      if (x >= NX) continue;
      T e[6];
      if (MODE == MODE_FIRST) {
#pragma unroll
        for (int c = 0; c < 6; ++c) e[c] = T(LP.E[c]);
      } else {
#pragma unroll
        for (int p = 0; p < 3; ++p) {
          const cx<T> Z = buf[x * LD + p * L + l];
          e[2 * p] = Z.x;
          e[2 * p + 1] = Z.y;
        }
      }
      T tau[6] = {T(0), T(0), T(0), T(0), T(0), T(0)};
      if (line < nlines) {
        if constexpr (GEN)
          gen_tau<T>(MAT.coef, mv[i][m], e, tau);
        else
          row_tau<T>(MAT.aniso && mv[i][m] >= 0, rows[i][m], e, tau);
#pragma unroll
        for (int c = 0; c < 6; ++c) acc[c] += (double)tau[c];
      }
#pragma unroll
      for (int p = 0; p < 3; ++p) buf[x * LD + p * L + l] = cx<T>{tau[2 * p], tau[2 * p + 1]};
    }
  }
  __syncthreads();
  fft_lines<T, NX, LL, NT, -1, LD, RMAX>(buf, s_tw, tid);

#pragma unroll
  for (int i = 0; i < RP; ++i) {
    const int r = wv + NW * i;
    if (r >= LL) continue;
    const int p = r / L, l = r - (r / L) * L;
    const int line = line0 + l;
    if (line >= nlines) continue;
    const int col = p * L + l;
    cx<T>* ra = spec + (size_t)(2 * p) * cs + (size_t)line * Hp;
    cx<T>* rb = ra + cs;
#pragma unroll
    for (int m = 0; m < KH; ++m) {
      const int k = lane + 64 * m;
      if (k < H) {
        const cx<T> Z = buf[k * LD + col];
        const cx<T> Zc = c_conj(buf[((NX - k) % NX) * LD + col]);
        ra[k] = cx<T>{T(0.5) * (Z.x + Zc.x), T(0.5) * (Z.y + Zc.y)};
        rb[k] = cx<T>{T(0.5) * (Z.y - Zc.y), T(-0.5) * (Z.x - Zc.x)};
      }
    }
  }
  // deterministic block sums of the six tau components
#pragma unroll
  for (int c = 0; c < 6; ++c) {
    double v = acc[c];
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
    if (lane == 0) red[c][wv] = v;
  }
  __syncthreads();
  if (tid < 6) {
    double s = 0.0;
#pragma unroll
    for (int i = 0; i < NW; ++i) s += red[tid][i];
    a.taupart[((size_t)load * a.g2 + blockIdx.x) * 6 + tid] = s;
  }
}

template <int NT>
__device__ __forceinline__ void fin_reduce_publish(const SolveArgs& a, int load, int k);

// ---------------------------------------------------------------- ysweep --
// A block owns W adjacent kx columns of one (load, component, z) plane;
// NC components per load (6 strain, or 3 gradient components).  The inverse
// sweep of the fixed point also ends the iteration: its first 7 n_load
// blocks in launch order each reduce one of the seven sums of a load case
// before their own transform, and the last of a load case's seven takes
// its stop decision.
template <typename T, int NY, int W, int NT, int SIGN, int NC = 6>
__global__ __launch_bounds__(NT) void k_ysweep(SolveArgs a) {
  constexpr int SL = NY * W;
  constexpr int Q = (SL + NT - 1) / NT;
  __shared__ cx<T> buf[SL];
  __shared__ cx<T> s_tw[NY];
  const int tid = threadIdx.x;
  const int z = blockIdx.y;
  // load cases in reverse block order: the x- and z-sweeps walk them
  // forward, so each sweep starts on the load cases the previous one wrote
  // last, which the last-level cache still holds when the state is not much
  // larger than it
  const int load = a.n_load - 1 - blockIdx.z / NC, comp = blockIdx.z - NC * (blockIdx.z / NC);
  int done;
  if constexpr (SIGN < 0) {
    done = a.state[load].done;
    // the inverse sweep reads the stop flag as it is now, while its own
    // blocks take this iteration's stop decision
    if (blockIdx.x == 0 && blockIdx.y == 0 && comp == 0 && tid == 0) a.done_snap[load] = done;
  } else if (a.cg) {
    done = a.state[load].done;
  } else {
    done = a.done_snap[load];
    // a grid of fewer than 7 n_load blocks (small 2D cells) takes turns
    const int nall = gridDim.x * gridDim.y * gridDim.z;
    for (int j = blockIdx.x + gridDim.x * (blockIdx.y + gridDim.y * blockIdx.z); j < 7 * a.n_load; j += nall) {
      fin_reduce_publish<NT>(a, j / 7, j - 7 * (j / 7));
      __syncthreads();  // the reduction's shared words are reused by the next turn
    }
  }
  if (done) return;
  const int H = a.H, Hp = a.Hp;
  const int kx0 = blockIdx.x * W;
  cx<T>* base = static_cast<cx<T>*>(a.spec) + ((size_t)(load * NC + comp) * a.nz + z) * (size_t)NY * Hp + kx0;
  cx<T> r[Q];
#pragma unroll
  for (int q = 0; q < Q; ++q) {
    const int s = tid + q * NT;
    r[q] = cx<T>{T(0), T(0)};
    if (s < SL) {
      const int j = s / W, w = s - j * W;
      if (kx0 + w < H) r[q] = base[(size_t)j * Hp + w];
    }
  }
  load_twiddles<T, NY, NT>(s_tw, static_cast<const cx<T>*>(a.twy), tid);
#pragma unroll
  for (int q = 0; q < Q; ++q) {
    const int s = tid + q * NT;
    if (s < SL) buf[s] = r[q];
  }
  __syncthreads();
  fft_lines<T, NY, W, NT, SIGN>(buf, s_tw, tid);
#pragma unroll
  for (int q = 0; q < Q; ++q) {
    const int s = tid + q * NT;
    if (s < SL) {
      const int j = s / W, w = s - j * W;
      if (kx0 + w < H) base[(size_t)j * Hp + w] = buf[s];
    }
  }
}

// ---------------------------------------------------------------- zsweep --
// A block owns W adjacent kx columns of one (load, ky) slab, i.e. W z-lines
// of every component; thread slot s = kz * W + w is one frequency.
// Gamma0^ : tau^ depends on tau^ only through a = tau^ . n, so the six
// components are transformed one at a time (the next one's global read in
// flight meanwhile) and folded into a; the inverse phase rebuilds each
// strain component from a before its inverse transform.

// Per-frequency registers of the z-sweep: unit normal and a = tau^ . n.
template <typename T> struct Slot {
  T n0, n1, n2;
  cx<T> a0, a1, a2;
};

// Tensor indices (i, j) of component c in the order 11, 22, 33, 23, 13, 12.
__device__ __forceinline__ int comp_i(int c) { return c < 3 ? c : (c == 3 ? 1 : 0); }
__device__ __forceinline__ int comp_j(int c) { return c < 3 ? c : (c == 5 ? 1 : 2); }

template <typename T> __device__ __forceinline__ T pick(int k, T v0, T v1, T v2) {
  return k == 0 ? v0 : (k == 1 ? v1 : v2);
}

// a_k += tau_c (d_ki n_j + d_kj n_i) for i != j, a_i += tau_c n_i for i == j.
// With c known at compile time (the unrolled loops) only the nonzero
// products are formed; in a rolled loop (c varies) the weights select them.
template <typename C, typename T> __device__ __forceinline__ void cfma(C& a, C v, T w) {
  a.x += v.x * w;
  a.y += v.y * w;
}
template <typename T>
__device__ __forceinline__ void fold_component_rolled(int c, cx<T> v, Slot<T>& z) {
  const int i = comp_i(c), j = comp_j(c);
  const T ni = pick(i, z.n0, z.n1, z.n2), nj = pick(j, z.n0, z.n1, z.n2);
  const T w0 = (i == 0 ? nj : T(0)) + (j == 0 && i != j ? ni : T(0));
  const T w1 = (i == 1 ? nj : T(0)) + (j == 1 && i != j ? ni : T(0));
  const T w2 = (i == 2 ? nj : T(0)) + (j == 2 && i != j ? ni : T(0));
  cfma(z.a0, v, w0);
  cfma(z.a1, v, w1);
  cfma(z.a2, v, w2);
}
template <typename T>
__device__ __forceinline__ void fold_component(int c, cx<T> v, Slot<T>& z) {
  switch (c) {
    case 0: cfma(z.a0, v, z.n0); break;
    case 1: cfma(z.a1, v, z.n1); break;
    case 2: cfma(z.a2, v, z.n2); break;
    case 3: cfma(z.a1, v, z.n2); cfma(z.a2, v, z.n1); break;
    case 4: cfma(z.a0, v, z.n2); cfma(z.a2, v, z.n0); break;
    default: cfma(z.a0, v, z.n1); cfma(z.a1, v, z.n0); break;
  }
}

// The z-sweep parks several frequency slots per thread in registers, so its
// butterflies stay at radix 9 or below.
// Entry (i, j) of m * [(n (x) a + a (x) n) / (2 mu0) - cc (n.a) n (x) n].
template <typename T>
__device__ __forceinline__ cx<T> gamma_entry(T ni, T nj, cx<T> ai, cx<T> aj, cx<T> na, T inv2mu, T cc, T m) {
  const T g = cc * ni * nj;
  return cx<T>{m * ((ni * aj.x + nj * ai.x) * inv2mu - g * na.x), m * ((ni * aj.y + nj * ai.y) * inv2mu - g * na.y)};
}

// Component c of m * [(n (x) a + a (x) n) / (2 mu0) - cc (n.a) n (x) n].
template <typename T>
__device__ __forceinline__ cx<T> strain_component(int c, const Slot<T>& z, cx<T> na, T inv2mu, T cc, T m) {
  const int i = comp_i(c), j = comp_j(c);
  const T ni = pick(i, z.n0, z.n1, z.n2), nj = pick(j, z.n0, z.n1, z.n2);
  const T aix = pick(i, z.a0.x, z.a1.x, z.a2.x), aiy = pick(i, z.a0.y, z.a1.y, z.a2.y);
  const T ajx = pick(j, z.a0.x, z.a1.x, z.a2.x), ajy = pick(j, z.a0.y, z.a1.y, z.a2.y);
  const T g = cc * ni * nj;
  return cx<T>{m * ((ni * ajx + nj * aix) * inv2mu - g * na.x), m * ((ni * ajy + nj * aiy) * inv2mu - g * na.y)};
}

// D is the prefetch depth: while one component group is transformed, the
// global reads of the next D - 1 groups are in flight (a ring of register
// buffers, so the forward loop is unrolled).  With single-component groups
// the ring slots that run past the sixth component fetch the traction
// history, which is then in flight during the last transforms.
template <typename T, int NZ, int W, int NT, int CG, int D, int PAD>
__global__ __launch_bounds__(NT, 4) void k_zsweep(SolveArgs a) {
  static_assert(6 % CG == 0, "component groups must divide 6");
  static_assert(D >= 1 && D <= 3, "prefetch depth 1..3");
  constexpr int NG = 6 / CG;      // component groups
  constexpr int SL = W * NZ;
  constexpr int Q = (SL + NT - 1) / NT;
  constexpr int LW = CG * W;      // lines per transform: CG components x W columns
  constexpr int LD = PAD ? (LW | 1) : LW;  // row stride: odd, or exactly the tile row
  constexpr int HR = CG == 1 ? (D < 3 ? D : 3) : 0;  // history components fetched through the ring
  __shared__ cx<T> buf[NZ * LD];
  __shared__ cx<T> s_tw[NZ];
  __shared__ double red[NT / 64];
  const int tid = threadIdx.x;
  const int tile = blockIdx.x, ky = blockIdx.y, load = blockIdx.z;
  if (a.state[load].done) return;
  const LoadParams& LP = a.prm->loads[load];
  const ProblemParams& P = a.prm->probs[LP.prob];
  const int H = a.H, Hp = a.Hp, ny = a.ny;
  const int kx0 = tile * W;
  const size_t zs = (size_t)ny * Hp;
  const size_t plane = (size_t)NZ * zs;
  cx<T>* sp = static_cast<cx<T>*>(a.spec) + (size_t)load * 6 * plane + (size_t)ky * Hp + kx0;
  cx<T>* hp = static_cast<cx<T>*>(a.hist) + (size_t)load * 3 * plane + (size_t)ky * Hp + kx0;
  const int ay = ky <= (ny - 1) / 2 ? ky : ky - ny;
  const double twopi = 6.283185307179586476925286766559;

  bool ok[Q];
  unsigned off[Q];
  unsigned lds[Q];  // LDS index of the slot's first component
  Slot<T> z[Q];
#pragma unroll
  for (int q = 0; q < Q; ++q) {
    const int s = tid + q * NT;
    const int kz = s / W, w = s - (s / W) * W;
    const int kx = kx0 + w;
    ok[q] = s < SL && kx < H;
    off[q] = (unsigned)(kz * zs + w);
    lds[q] = (unsigned)(kz * LD + w);
    const int az = kz <= (NZ - 1) / 2 ? kz : kz - NZ;
    if constexpr (sizeof(T) == 4) {
      // n = k / |k| from the integer wave vector (the 2 pi cancels); one
      // hardware reciprocal square root, well inside single precision
      const int k2 = kx * kx + ay * ay + az * az;
      const float rinv = k2 > 0 ? rsqrtf((float)k2) : 0.0f;
      z[q].n0 = (float)kx * rinv;
      z[q].n1 = (float)ay * rinv;
      z[q].n2 = (float)az * rinv;
    } else {
      const double x0 = twopi * kx, x1 = twopi * ay, x2 = twopi * az;
      const double q2 = x0 * x0 + x1 * x1 + x2 * x2;
      const double rinv = q2 > 0.0 ? 1.0 / sqrt(q2) : 0.0;
      z[q].n0 = T(x0 * rinv);
      z[q].n1 = T(x1 * rinv);
      z[q].n2 = T(x2 * rinv);
    }
    z[q].a0 = z[q].a1 = z[q].a2 = cx<T>{T(0), T(0)};
  }
  // ring[r] holds group r, r + D, ...; then (CG == 1) history components
  cx<T> ring[D][CG][Q];
  const bool hist_live = !a.first && !a.cg;
#pragma unroll
  for (int r = 0; r < D; ++r)
#pragma unroll
    for (int g = 0; g < CG; ++g)
#pragma unroll
      for (int q = 0; q < Q; ++q)
        ring[r][g][q] = (r < NG && ok[q]) ? sp[(size_t)(r * CG + g) * plane + off[q]] : cx<T>{T(0), T(0)};
  load_twiddles<T, NZ, NT>(s_tw, static_cast<const cx<T>*>(a.twz), tid);

  // depth 1: a rolled loop over the groups; deeper rings: fully unrolled,
  // so that ring slots are fixed registers
  constexpr int UN = D == 1 ? 1 : NG;
#pragma unroll 1
  for (int gb = 0; gb < NG; gb += UN) {
#pragma unroll
   for (int u = 0; u < UN; ++u) {
    const int gi = gb + u;
    const int r = gi % D;
#pragma unroll
    for (int g = 0; g < CG; ++g)
#pragma unroll
      for (int q = 0; q < Q; ++q)
        if (tid + q * NT < SL) buf[lds[q] + g * W] = ring[r][g][q];
    const int nx = gi + D;
    if (nx < NG) {
#pragma unroll
      for (int g = 0; g < CG; ++g)
#pragma unroll
        for (int q = 0; q < Q; ++q)
          ring[r][g][q] = ok[q] ? sp[(size_t)(nx * CG + g) * plane + off[q]] : cx<T>{T(0), T(0)};
    } else if (CG == 1 && nx - NG < HR) {
#pragma unroll
      for (int q = 0; q < Q; ++q)
        ring[r][0][q] = (ok[q] && hist_live) ? load_stream<T>(hp + (size_t)(nx - NG) * plane + off[q])
                                             : cx<T>{T(0), T(0)};
    }
    __syncthreads();
    fft_lines<T, NZ, LW, NT, -1, LD, 9>(buf, s_tw, tid);
#pragma unroll
    for (int g = 0; g < CG; ++g)
#pragma unroll
      for (int q = 0; q < Q; ++q)
        if (tid + q * NT < SL) {
          if constexpr (UN > 1)
            fold_component<T>(gi * CG + g, buf[lds[q] + g * W], z[q]);
          else
            fold_component_rolled<T>(gi * CG + g, buf[lds[q] + g * W], z[q]);
        }
    __syncthreads();
   }
  }

  // equilibrium error partial and traction history (not in CG mode)
  double S = 0.0;
#pragma unroll
  for (int q = 0; q < Q; ++q) {
    if (!ok[q] || a.cg) continue;
    const int s = tid + q * NT;
    const int kz = s / W, w = s - kz * W;
    const int az = kz <= (NZ - 1) / 2 ? kz : kz - NZ;
    const int kx = kx0 + w;
    cx<T>* h0 = hp + off[q];
    if (kx == 0 && ay == 0 && az == 0) {
      h0[0] = h0[plane] = h0[2 * plane] = cx<T>{T(0), T(0)};
      continue;
    }
    cx<T> pv[3];
#pragma unroll
    for (int h = 0; h < 3; ++h) {
      if (h < HR)
        pv[h] = ring[(NG + h) % D][0][q];  // fetched in the forward loop
      else
        pv[h] = hist_live ? load_stream<T>(h0 + (size_t)h * plane) : cx<T>{T(0), T(0)};
    }
    store_stream<T>(h0, z[q].a0);
    store_stream<T>(h0 + plane, z[q].a1);
    store_stream<T>(h0 + 2 * plane, z[q].a2);
    const double x0 = twopi * kx, x1 = twopi * ay, x2 = twopi * az;
    double dd;
    if constexpr (sizeof(T) == 4) {
      // differences of the single-precision values taken, squared and
      // summed in FP64
      const double d0x = (double)z[q].a0.x - (double)pv[0].x, d0y = (double)z[q].a0.y - (double)pv[0].y;
      const double d1x = (double)z[q].a1.x - (double)pv[1].x, d1y = (double)z[q].a1.y - (double)pv[1].y;
      const double d2x = (double)z[q].a2.x - (double)pv[2].x, d2y = (double)z[q].a2.y - (double)pv[2].y;
      dd = d0x * d0x + d0y * d0y + d1x * d1x + d1y * d1y + d2x * d2x + d2y * d2y;
    } else {
      const double d0x = z[q].a0.x - pv[0].x, d0y = z[q].a0.y - pv[0].y;
      const double d1x = z[q].a1.x - pv[1].x, d1y = z[q].a1.y - pv[1].y;
      const double d2x = z[q].a2.x - pv[2].x, d2y = z[q].a2.y - pv[2].y;
      dd = d0x * d0x + d0y * d0y + d1x * d1x + d1y * d1y + d2x * d2x + d2y * d2y;
    }
    S += (kx == 0 ? 1.0 : 2.0) * (x0 * x0 + x1 * x1 + x2 * x2) * dd;
  }

  // eps^_kh = -[(n_k a_h + n_h a_k) / (2 mu0) - cc (n.a) n_k n_h] / N, eps^(0) = E
  const double rl = P.rl, rm = P.rm;
  const T inv2mu = T(1.0 / (2.0 * rm));
  const T cc = T((rl + rm) / (rm * (rl + 2.0 * rm)));
  const T m = T(-1.0 / ((double)a.nx * (double)ny * (double)NZ));
  cx<T> na[Q];
#pragma unroll
  for (int q = 0; q < Q; ++q)
    na[q] = cx<T>{z[q].a0.x * z[q].n0 + z[q].a1.x * z[q].n1 + z[q].a2.x * z[q].n2,
                  z[q].a0.y * z[q].n0 + z[q].a1.y * z[q].n1 + z[q].a2.y * z[q].n2};
  // inverse transforms: rolled with depth 1, unrolled with deeper rings (the
  // component index is then a constant in the Gamma0^ contraction)
#pragma unroll 1
  for (int cb = 0; cb < 6; cb += CG * UN) {
#pragma unroll
   for (int u = 0; u < UN; ++u) {
    const int c0 = cb + u * CG;
#pragma unroll
    for (int g = 0; g < CG; ++g) {
      const T Ec = a.cg ? T(0) : T(LP.E[c0 + g]);
#pragma unroll
      for (int q = 0; q < Q; ++q) {
        if (tid + q * NT < SL) {
          const bool zero = z[q].n0 == T(0) && z[q].n1 == T(0) && z[q].n2 == T(0);
          buf[lds[q] + g * W] = zero ? cx<T>{Ec, T(0)} : strain_component<T>(c0 + g, z[q], na[q], inv2mu, cc, m);
        }
      }
    }
    __syncthreads();
    fft_lines<T, NZ, LW, NT, +1, LD, 9>(buf, s_tw, tid);
#pragma unroll
    for (int g = 0; g < CG; ++g)
#pragma unroll
      for (int q = 0; q < Q; ++q)
        if (tid + q * NT < SL && ok[q]) sp[(size_t)(c0 + g) * plane + off[q]] = buf[lds[q] + g * W];
    __syncthreads();
   }
  }
  const double tot = block_sum<NT>(S, red);
  if (tid == 0) a.errpart[(size_t)load * ((size_t)ny * a.ntx4) + (size_t)ky * a.ntx4 + tile] = tot;
}

// ------------------------------------------------------ wavefront sweeps --
// Variants in which each wavefront owns whole FFT lines, so the radix passes
// need no block barrier (see wave_sync).

// x-sweep: each of the NW waves of a block owns LW consecutive (y, z) lines
// (3 LW complex lines); one block barrier publishes the twiddles, one more
// combines the per-wave tau sums.
template <typename T, int NX, int LW, int NW, int MODE>
__global__ __launch_bounds__(64 * NW) void k_xsweep_wave(SolveArgs a) {
  constexpr int NT = 64 * NW;
  constexpr int LL = 3 * LW;
  constexpr int LD = LL | 1;
  constexpr int H = (NX + 1) / 2;
  constexpr int NLD = 3 * LW * H;  // (pair, line, kx) items of one wave
  constexpr int QL = (NLD + 63) / 64;
  constexpr int NV = LW * NX;  // voxels of one wave
  constexpr int QV = (NV + 63) / 64;
  __shared__ cx<T> bufs[NW][NX * LD];
  __shared__ cx<T> s_tw[NX];
  __shared__ double red[6][NW];
  const int tid = threadIdx.x, wv = tid >> 6, lane = tid & 63;
  const int load = blockIdx.y;
  SolverState* st = a.state + load;
  if (MODE != MODE_EXPORT && st->done) return;
  const LoadParams& LP = a.prm->loads[load];
  const ProblemParams& P = a.prm->probs[LP.prob];
  const VoxelMaterial<T> MAT = load_material<T>(P);
  const int nlines = a.ny * a.nz;
  const int line0 = (blockIdx.x * NW + wv) * LW;
  const int Hp = a.Hp;
  const size_t cs = (size_t)nlines * Hp;
  cx<T>* spec = static_cast<cx<T>*>(a.spec) + (size_t)load * 6 * cs;
  const cx<T>* src = static_cast<const cx<T>*>(a.spec_in) + (size_t)load * 6 * cs;
  cx<T>* buf = bufs[wv];

  cx<T> pa[QL], pb[QL];
  if (MODE != MODE_FIRST) {
#pragma unroll
    for (int q = 0; q < QL; ++q) {
      const int idx = lane + 64 * q;
      pa[q] = cx<T>{T(0), T(0)};
      pb[q] = cx<T>{T(0), T(0)};
      if (idx < NLD) {
        const int p = idx / (LW * H);
        const int rem = idx - p * (LW * H);
        const int l = rem / H;
        const int k = rem - l * H;
        const int line = line0 + l;
        if (line < nlines) {
          pa[q] = src[(size_t)(2 * p) * cs + (size_t)line * Hp + k];
          pb[q] = src[(size_t)(2 * p + 1) * cs + (size_t)line * Hp + k];
        }
      }
    }
  }
  int mv[QV];
  if (MODE != MODE_EXPORT) {
#pragma unroll
    for (int q = 0; q < QV; ++q) {
      const int idx = lane + 64 * q;
      const int l = idx / NX, x = idx - l * NX, line = line0 + l;
      mv[q] = (idx < NV && line < nlines) ? load_global(MAT.mid + (size_t)line * NX + x) : -1;
    }
  }
  load_twiddles<T, NX, NT>(s_tw, static_cast<const cx<T>*>(a.twx), tid);
  __syncthreads();

  if (MODE != MODE_FIRST) {
#pragma unroll
    for (int q = 0; q < QL; ++q) {
      const int idx = lane + 64 * q;
      if (idx < NLD) {
        const int p = idx / (LW * H);
        const int rem = idx - p * (LW * H);
        const int l = rem / H;
        const int k = rem - l * H;
        const cx<T> A = pa[q], B = pb[q];
        buf[k * LD + p * LW + l] = cx<T>{A.x - B.y, A.y + B.x};
        if (k > 0) buf[(NX - k) * LD + p * LW + l] = cx<T>{A.x + B.y, B.x - A.y};
      }
    }
    wave_sync();
    fft_lines_wave<T, NX, LL, +1, LD>(buf, s_tw, lane);
  }

  if (MODE == MODE_EXPORT) {
    const size_t N = (size_t)nlines * NX;
    T* out = static_cast<T*>(a.eps_out) + (size_t)load * 6 * N;
    for (int idx = lane; idx < NV; idx += 64) {
      const int l = idx / NX, x = idx - l * NX, line = line0 + l;
      if (line < nlines) {
#pragma unroll
        for (int p = 0; p < 3; ++p) {
          const cx<T> Z = buf[x * LD + p * LW + l];
          out[(size_t)(2 * p) * N + (size_t)line * NX + x] = Z.x + (a.cg ? T(LP.E[2 * p]) : T(0));
          out[(size_t)(2 * p + 1) * N + (size_t)line * NX + x] = Z.y + (a.cg ? T(LP.E[2 * p + 1]) : T(0));
        }
      }
    }
    return;
  }

  T rows[QV][8];
#pragma unroll
  for (int q = 0; q < QV; ++q) material_row<T>(MAT, mv[q], rows[q]);
  double acc[6] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
#pragma unroll
  for (int q = 0; q < QV; ++q) {
    const int idx = lane + 64 * q;
    if (idx >= NV) continue;
    const int l = idx / NX, x = idx - l * NX, line = line0 + l;
    T e[6];
    if (MODE == MODE_FIRST) {
#pragma unroll
      for (int c = 0; c < 6; ++c) e[c] = T(LP.E[c]);
    } else {
#pragma unroll
      for (int p = 0; p < 3; ++p) {
        const cx<T> Z = buf[x * LD + p * LW + l];
        e[2 * p] = Z.x;
        e[2 * p + 1] = Z.y;
      }
    }
    T tau[6] = {T(0), T(0), T(0), T(0), T(0), T(0)};
    if (line < nlines) {
      row_tau<T>(MAT.aniso && mv[q] >= 0, rows[q], e, tau);
#pragma unroll
      for (int c = 0; c < 6; ++c) acc[c] += (double)tau[c];
    }
#pragma unroll
    for (int p = 0; p < 3; ++p) buf[x * LD + p * LW + l] = cx<T>{tau[2 * p], tau[2 * p + 1]};
  }
  wave_sync();
  fft_lines_wave<T, NX, LL, -1, LD>(buf, s_tw, lane);

  for (int idx = lane; idx < NLD; idx += 64) {
    const int p = idx / (LW * H);
    const int rem = idx - p * (LW * H);
    const int l = rem / H;
    const int k = rem - l * H;
    const int line = line0 + l;
    if (line < nlines) {
      const cx<T> Z = buf[k * LD + p * LW + l];
      const cx<T> Zc = c_conj(buf[((NX - k) % NX) * LD + p * LW + l]);
      const cx<T> A = {T(0.5) * (Z.x + Zc.x), T(0.5) * (Z.y + Zc.y)};
      const cx<T> B = {T(0.5) * (Z.y - Zc.y), T(-0.5) * (Z.x - Zc.x)};
      spec[(size_t)(2 * p) * cs + (size_t)line * Hp + k] = A;
      spec[(size_t)(2 * p + 1) * cs + (size_t)line * Hp + k] = B;
    }
  }
#pragma unroll
  for (int c = 0; c < 6; ++c) {
    double v = acc[c];
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
    if (lane == 0) red[c][wv] = v;
  }
  __syncthreads();
  if (tid < 6) {
    double s = 0.0;
#pragma unroll
    for (int i = 0; i < NW; ++i) s += red[tid][i];
    a.taupart[((size_t)load * a.g2 + blockIdx.x) * 6 + tid] = s;
  }
}

// z-sweep: six waves per tile of W kx columns, wave c owning strain
// component c.  Each wave reads its component's tile and transforms it in
// its own LDS region; after one block barrier every thread applies the Green
// operator to its frequency slots across the six regions; after a second
// barrier each wave inverse-transforms and stores its component.  Tiles are
// taken in XCD-paired order (see xcd_pair_order) on a one-dimensional grid.
__device__ __forceinline__ int xcd_pair_order(int L) {
  const int g = L >> 4, r = L & 15;
  return 2 * (g * 8 + (r & 7)) + (r >> 3);
}

template <typename T, int NZ, int W>
__global__ __launch_bounds__(384) void k_zsweep_wave(SolveArgs a) {
  constexpr int NT = 384;
  constexpr int SL = W * NZ;
  constexpr int LD = W | 1;
  constexpr int RS = NZ * LD;
  constexpr int QC = (SL + 63) / 64;
  constexpr int QS = (SL + NT - 1) / NT;
  __shared__ cx<T> rg[6 * RS];
  __shared__ cx<T> s_tw[NZ];
  __shared__ double red[NT / 64];
  const int tid = threadIdx.x, c = tid >> 6, lane = tid & 63;
  const int ntiles = a.ntx4 * a.ny * a.n_load;
  const int t = xcd_pair_order(blockIdx.x);
  if (t >= ntiles) return;
  const int tile = t % a.ntx4;
  const int rest = t / a.ntx4;
  const int ny = a.ny;
  const int ky = rest % ny, load = rest / ny;
  if (a.state[load].done) return;
  const LoadParams& LP = a.prm->loads[load];
  const ProblemParams& P = a.prm->probs[LP.prob];
  const int H = a.H, Hp = a.Hp;
  const int kx0 = tile * W;
  const size_t zs = (size_t)ny * Hp;
  const size_t plane = (size_t)NZ * zs;
  cx<T>* sp = static_cast<cx<T>*>(a.spec) + (size_t)load * 6 * plane + (size_t)ky * Hp + kx0;
  cx<T>* hp = static_cast<cx<T>*>(a.hist) + (size_t)load * 3 * plane + (size_t)ky * Hp + kx0;
  const int ay = ky <= (ny - 1) / 2 ? ky : ky - ny;
  const double twopi = 6.283185307179586476925286766559;
  cx<T>* mine = rg + c * RS;

  cx<T> v[QC];
#pragma unroll
  for (int q = 0; q < QC; ++q) {
    const int e = lane + 64 * q;
    const int kz = e / W, w = e - (e / W) * W;
    v[q] = (e < SL && kx0 + w < H) ? sp[(size_t)c * plane + (size_t)kz * zs + w] : cx<T>{T(0), T(0)};
  }
  cx<T> h[QS][3];
#pragma unroll
  for (int q = 0; q < QS; ++q) {
    const int s = tid + NT * q;
    const int kz = s / W, w = s - (s / W) * W;
    const bool ok = s < SL && kx0 + w < H && !a.first && !a.cg;
#pragma unroll
    for (int d = 0; d < 3; ++d)
      h[q][d] = ok ? load_stream<T>(hp + (size_t)d * plane + (size_t)kz * zs + w) : cx<T>{T(0), T(0)};
  }
  load_twiddles<T, NZ, NT>(s_tw, static_cast<const cx<T>*>(a.twz), tid);
#pragma unroll
  for (int q = 0; q < QC; ++q) {
    const int e = lane + 64 * q;
    if (e < SL) mine[(e / W) * LD + (e % W)] = v[q];
  }
  __syncthreads();
  fft_lines_wave<T, NZ, W, -1, LD>(mine, s_tw, lane);
  __syncthreads();

  const double rl = P.rl, rm = P.rm;
  const T inv2mu = T(1.0 / (2.0 * rm));
  const T cc = T((rl + rm) / (rm * (rl + 2.0 * rm)));
  const T m = T(-1.0 / ((double)a.nx * (double)ny * (double)NZ));
  double S = 0.0;
#pragma unroll
  for (int q = 0; q < QS; ++q) {
    const int s = tid + NT * q;
    if (s >= SL) continue;
    const int kz = s / W, w = s - kz * W;
    const int kx = kx0 + w;
    if (kx >= H) continue;
    const int az = kz <= (NZ - 1) / 2 ? kz : kz - NZ;
    const int o = kz * LD + w;
    const size_t go = (size_t)kz * zs + w;
    if (kx == 0 && ay == 0 && az == 0) {
#pragma unroll
      for (int d = 0; d < 6; ++d) rg[d * RS + o] = cx<T>{a.cg ? T(0) : T(LP.E[d]), T(0)};
      if (!a.cg)
#pragma unroll
        for (int d = 0; d < 3; ++d) hp[(size_t)d * plane + go] = cx<T>{T(0), T(0)};
      continue;
    }
    const double x0 = twopi * kx, x1 = twopi * ay, x2 = twopi * az;
    const double q2 = x0 * x0 + x1 * x1 + x2 * x2;
    const double rinv = 1.0 / sqrt(q2);
    const T n0 = T(x0 * rinv), n1 = T(x1 * rinv), n2 = T(x2 * rinv);
    const cx<T> t11 = rg[o], t22 = rg[RS + o], t33 = rg[2 * RS + o];
    const cx<T> t23 = rg[3 * RS + o], t13 = rg[4 * RS + o], t12 = rg[5 * RS + o];
    const cx<T> a0 = {t11.x * n0 + t12.x * n1 + t13.x * n2, t11.y * n0 + t12.y * n1 + t13.y * n2};
    const cx<T> a1 = {t12.x * n0 + t22.x * n1 + t23.x * n2, t12.y * n0 + t22.y * n1 + t23.y * n2};
    const cx<T> a2 = {t13.x * n0 + t23.x * n1 + t33.x * n2, t13.y * n0 + t23.y * n1 + t33.y * n2};
    const cx<T> na = {a0.x * n0 + a1.x * n1 + a2.x * n2, a0.y * n0 + a1.y * n1 + a2.y * n2};
    const double d0x = (double)a0.x - (double)h[q][0].x, d0y = (double)a0.y - (double)h[q][0].y;
    const double d1x = (double)a1.x - (double)h[q][1].x, d1y = (double)a1.y - (double)h[q][1].y;
    const double d2x = (double)a2.x - (double)h[q][2].x, d2y = (double)a2.y - (double)h[q][2].y;
    if (!a.cg) {
      S += (kx == 0 ? 1.0 : 2.0) * q2 * (d0x * d0x + d0y * d0y + d1x * d1x + d1y * d1y + d2x * d2x + d2y * d2y);
      store_stream<T>(hp + go, a0);
      store_stream<T>(hp + plane + go, a1);
      store_stream<T>(hp + 2 * plane + go, a2);
    }
    rg[o] = gamma_entry<T>(n0, n0, a0, a0, na, inv2mu, cc, m);
    rg[RS + o] = gamma_entry<T>(n1, n1, a1, a1, na, inv2mu, cc, m);
    rg[2 * RS + o] = gamma_entry<T>(n2, n2, a2, a2, na, inv2mu, cc, m);
    rg[3 * RS + o] = gamma_entry<T>(n1, n2, a1, a2, na, inv2mu, cc, m);
    rg[4 * RS + o] = gamma_entry<T>(n0, n2, a0, a2, na, inv2mu, cc, m);
    rg[5 * RS + o] = gamma_entry<T>(n0, n1, a0, a1, na, inv2mu, cc, m);
  }
  __syncthreads();
  fft_lines_wave<T, NZ, W, +1, LD>(mine, s_tw, lane);
#pragma unroll
  for (int q = 0; q < QC; ++q) {
    const int e = lane + 64 * q;
    const int kz = e / W, w = e - (e / W) * W;
    if (e < SL && kx0 + w < H) sp[(size_t)c * plane + (size_t)kz * zs + w] = mine[kz * LD + w];
  }
  const double tot = block_sum<NT>(S, red);
  if (tid == 0) a.errpart[(size_t)load * ((size_t)ny * a.ntx4) + (size_t)ky * a.ntx4 + tile] = tot;
}

// ------------------------------------------------------ end of iteration --
__device__ __forceinline__ void neumaier_add(double& s, double& c, double x) {
  const double t = s + x;
  if (fabs(s) >= fabs(x))
    c += (s - t) + x;
  else
    c += (x - t) + s;
  s = t;
}

// Neumaier combination of two compensated partial sums (s, c) += (s2, c2).
__device__ __forceinline__ void neumaier_merge(double& s, double& c, double s2, double c2) {
  neumaier_add(s, c, s2);
  c += c2;
}

// Deterministic compensated block reduction of one of a load case's seven
// sums (k < 6: tau component k over the x-sweep partials; k = 6: the error
// sum over the z-sweep partials), valid in thread 0: a thread-strided
// compensated sum in index order with four loads in flight, then a fixed
// shuffle tree per wavefront and the wavefronts in order (the result does
// not depend on timing).  Every thread of the block calls it.
template <int NT>
__device__ __forceinline__ double finalize_reduce(const SolveArgs& a, int load, int k) {
  constexpr int NW = NT / 64;
  __shared__ double ws[NW], wc[NW];
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const size_t ne = (size_t)a.ny * a.ntx4;
  const double* src = k < 6 ? a.taupart + (size_t)load * a.g2 * 6 + k : a.errpart + (size_t)load * ne;
  const size_t n = k < 6 ? (size_t)a.g2 : ne, st = k < 6 ? 6 : 1;
  double s = 0.0, c = 0.0;
  size_t i = tid;
#pragma unroll 1
  for (; i + 3 * NT < n; i += 4 * NT) {
    const double x0 = src[i * st], x1 = src[(i + NT) * st], x2 = src[(i + 2 * NT) * st],
                 x3 = src[(i + 3 * NT) * st];
    neumaier_add(s, c, x0);
    neumaier_add(s, c, x1);
    neumaier_add(s, c, x2);
    neumaier_add(s, c, x3);
  }
#pragma unroll 1
  for (; i < n; i += NT) neumaier_add(s, c, src[i * st]);
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) {
    const double so = __shfl_down(s, off, 64), co = __shfl_down(c, off, 64);
    if (lane < off) neumaier_merge(s, c, so, co);
  }
  if (lane == 0) {
    ws[wv] = s;
    wc[wv] = c;
  }
  __syncthreads();
  if (tid != 0) return 0.0;
  double sk = ws[0], ck = wc[0];
#pragma unroll 1
  for (int w = 1; w < NW; ++w) neumaier_merge(sk, ck, ws[w], wc[w]);
  return sk + ck;
}

// The end of an iteration for one load case, from its published sums, by
// one whole wavefront (lane c < 6 owns component c, so that few registers
// are live: this runs inside the inverse y-sweep): the mean stress (or
// flux), the error, the history and the stop decision.
__device__ __forceinline__ void finalize_decide(const SolveArgs& a, int load, int lane) {
  SolverState* st = a.state + load;
  const SolveParams& S0 = *a.prm;
  const LoadParams& LP = S0.loads[load];
  const ProblemParams& P = S0.probs[LP.prob];
  const double* r = a.fin_red + (size_t)load * 8;
  const int c = lane < 6 ? lane : 0;
  const double t = __hip_atomic_load(r + c, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  const double S = __hip_atomic_load(r + 6, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  const double N = (double)a.nx * (double)a.ny * (double)a.nz;
  const double* E = LP.E;
  double sc;
  if (a.cond) {
    // mean flux <q> = k0 G + <tau>; shear slots stay zero
    sc = c < 3 ? t / N + P.rl * E[c] : 0.0;
  } else {
    sc = t / N + (c < 3 ? P.rl * (E[0] + E[1] + E[2]) : 0.0) + 2.0 * P.rm * E[c];
  }
  double sig[6];
#pragma unroll
  for (int k = 0; k < 6; ++k) sig[k] = __shfl(sc, k, 64);
  if (lane < 6) {
    const int i = st->iter;
    if (i < a.hist_cap) a.sighist[((size_t)load * a.hist_cap + i) * 6 + lane] = sc;
    st->sig[lane] = sc;
  }
  if (lane != 0) return;
  const double fro = sqrt(sig[0] * sig[0] + sig[1] * sig[1] + sig[2] * sig[2] +
                          2.0 * (sig[3] * sig[3] + sig[4] * sig[4] + sig[5] * sig[5]));
  const double den = N * fro;
  const double res = sqrt(S);
  const double e = den > 0.0 ? res / den : (S == 0.0 ? 0.0 : INFINITY);
  const int i = st->iter;
  if (i < a.hist_cap) a.errhist[(size_t)load * a.hist_cap + i] = e;
  if (i == 0) {
    st->err0 = e;
    st->res0 = res;
  }
  // divergence is judged on the residual: the mean stress in the
  // denominator of e can pass near zero while the iteration converges
  const double r0 = i == 0 ? res : st->res0;
  int status = ST_RUNNING;
  if (e < S0.tol) {
    status = ST_CONVERGED;
  } else if (!isfinite(e) || (r0 > 0.0 && res > kDivergenceFactor * r0)) {
    status = ST_DIVERGED;
  } else {
    if (i == 0 || e < kStallDecrease * st->ref) {
      st->ref = e;
      st->iref = i;
    }
    if (S0.stall_window > 0 && i - st->iref >= S0.stall_window)
      status = ST_STALLED;
    else if (i >= S0.max_iter)
      status = ST_NOT_CONVERGED;
  }
  st->err = e;
  st->iters = i;
  if (status != ST_RUNNING) {
    st->status = status;
    st->done = 1;
  }
  st->iter = i + 1;
}

// The end of an iteration runs inside the inverse y-sweep, which starts
// after the x- and z-sweeps have written every partial it reduces.  Seven
// blocks reduce one sum each of a live load case L, publish it and arrive
// on fin_count[L]; the seventh arrival takes the stop decision and puts the
// counter back to 0 for the next launch.  The sweep's own blocks read L's
// stop flag from the snapshot the forward y-sweep took, so the decision
// may land while they run.
template <int NT>
__device__ __forceinline__ void fin_reduce_publish(const SolveArgs& a, int load, int k) {
  if (a.done_snap[load]) return;
  const double v = finalize_reduce<NT>(a, load, k);
  if (threadIdx.x >= 64) return;
  const int lane = threadIdx.x;
  int old = 0;
  if (lane == 0) {
    __hip_atomic_store(a.fin_red + (size_t)load * 8 + k, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    __threadfence();
    old = atomicAdd(a.fin_count + load, 1);
  }
  old = __shfl(old, 0, 64);
  if (old != 6) return;
  __threadfence();
  finalize_decide(a, load, lane);
  if (lane == 0) __hip_atomic_store(a.fin_count + load, 0, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

template <int NT>
__global__ __launch_bounds__(NT) void k_reset_state(SolverState* st, int n_load) {
  const int l = blockIdx.x * blockDim.x + threadIdx.x;
  if (l >= n_load) return;
  SolverState z;
  z.iter = 0;
  z.done = 0;
  z.status = ST_RUNNING;
  z.iters = 0;
  z.iref = 0;
  z.pad0 = z.pad1 = 0;
  z.err = z.err0 = z.res0 = z.ref = 0.0;
  for (int c = 0; c < 6; ++c) z.sig[c] = 0.0;
  st[l] = z;
}

// ---------------------------------------------------- conjugate gradients --
// CG on the Galerkin form of the same operator (the Krylov alternative of
// Section 5), with the reference medium c0 = identity: the four sweeps then
// turn a direction p into w = -G((c~ - I) : p) (G the projection onto
// compatible zero-mean fields), so q = G(c~ : p) = p - w.  Vectors x, r, p
// and w live in the x-half-spectrum layout of the iterate (x-DFTs divided
// by nx); a sum over voxels of u : v is, by Parseval along x, nx times the
// sum over stored entries of w_c h_kx Re(u conj v) (w_c = 2 for shear
// components, h_kx = 2 for kx > 0).  Every vector kernel writes one FP64
// partial per block.

enum : int { CG_INIT = 0, CG_DOT = 1, CG_UPDATE = 2, CG_DIR = 3 };
enum : int { CGS_INIT = 0, CGS_ALPHA = 1, CGS_BETA = 2 };
constexpr int kCgThreads = 256;

template <typename T, int OP>
__global__ __launch_bounds__(kCgThreads) void k_cg_vec(SolveArgs a) {
  __shared__ double red[kCgThreads / 64];
  const int load = blockIdx.y;
  if (a.state[load].done) return;
  const unsigned plane = (unsigned)a.nz * (unsigned)a.ny * (unsigned)a.Hp;
  const unsigned total = 6u * plane;
  const size_t off = (size_t)load * total;
  cx<T>* W = static_cast<cx<T>*>(a.spec) + off;
  cx<T>* X = static_cast<cx<T>*>(a.cgx) + off;
  cx<T>* R = static_cast<cx<T>*>(a.cgr) + off;
  cx<T>* P = static_cast<cx<T>*>(a.cgp) + off;
  const T al = OP == CG_UPDATE ? T(a.cgs[load].alpha) : T(0);
  const T be = OP == CG_DIR ? T(a.cgs[load].beta) : T(0);
  double acc = 0.0;
  for (unsigned e = blockIdx.x * kCgThreads + threadIdx.x; e < total; e += gridDim.x * kCgThreads) {
    const unsigned kx = e % (unsigned)a.Hp;
    if (kx >= (unsigned)a.H) continue;
    const double wgt = (e / plane < 3u ? 1.0 : 2.0) * (kx == 0 ? 1.0 : 2.0);
    if (OP == CG_INIT) {
      const cx<T> w = W[e];
      X[e] = cx<T>{T(0), T(0)};
      R[e] = w;
      P[e] = w;
      acc += wgt * ((double)w.x * w.x + (double)w.y * w.y);
    } else if (OP == CG_DOT) {
      const cx<T> pv = P[e], w = W[e];
      const cx<T> q = {pv.x - w.x, pv.y - w.y};
      acc += wgt * ((double)pv.x * q.x + (double)pv.y * q.y);
    } else if (OP == CG_UPDATE) {
      const cx<T> pv = P[e], w = W[e], xv = X[e], rv = R[e];
      const cx<T> q = {pv.x - w.x, pv.y - w.y};
      const cx<T> rn = {rv.x - al * q.x, rv.y - al * q.y};
      X[e] = cx<T>{xv.x + al * pv.x, xv.y + al * pv.y};
      R[e] = rn;
      acc += wgt * ((double)rn.x * rn.x + (double)rn.y * rn.y);
    } else {
      const cx<T> rv = R[e], pv = P[e];
      P[e] = cx<T>{rv.x + be * pv.x, rv.y + be * pv.y};
    }
  }
  if (OP == CG_DIR) return;
  const double tot = block_sum<kCgThreads>(acc, red);
  if (threadIdx.x == 0) a.cgpart[(size_t)load * a.cg_blocks + blockIdx.x] = tot;
}

// One block per load case: reduces the partials of the preceding vector
// kernel (and, for INIT and ALPHA, the tau sums of the preceding x-sweep),
// then takes the CG step (alpha), the direction update (beta), the error
// e_k = sqrt(<r : r>) / |<sigma_k>| and the stop decision.
template <int NT, int STEP>
__global__ __launch_bounds__(NT) void k_cg_scalar(SolveArgs a) {
  constexpr int NW = NT / 64;
  constexpr int K = 7;
  __shared__ double ws[NW][K], wc[NW][K];
  const int load = blockIdx.x;
  SolverState* st = a.state + load;
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const double* pp = a.cgpart + (size_t)load * a.cg_blocks;
  const double* tp = a.taupart + (size_t)load * a.g2 * 6;
  const bool taus = STEP != CGS_BETA;
  double s[K], c[K];
#pragma unroll
  for (int k = 0; k < K; ++k) s[k] = c[k] = 0.0;
  if (st->done) return;
  for (int i = tid; i < a.cg_blocks; i += NT) neumaier_add(s[6], c[6], pp[i]);
  if (taus)
    for (int i = tid; i < a.g2; i += NT)
#pragma unroll
      for (int k = 0; k < 6; ++k) neumaier_add(s[k], c[k], tp[(size_t)i * 6 + k]);
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) {
#pragma unroll
    for (int k = 0; k < K; ++k) {
      const double so = __shfl_down(s[k], off, 64), co = __shfl_down(c[k], off, 64);
      if (lane < off) neumaier_merge(s[k], c[k], so, co);
    }
  }
  if (lane == 0)
#pragma unroll
    for (int k = 0; k < K; ++k) {
      ws[wv][k] = s[k];
      wc[wv][k] = c[k];
    }
  __syncthreads();
  if (tid != 0) return;
  double tot[K];
#pragma unroll
  for (int k = 0; k < K; ++k) {
    double sk = ws[0][k], ck = wc[0][k];
    for (int w = 1; w < NW; ++w) neumaier_merge(sk, ck, ws[w][k], wc[w][k]);
    tot[k] = sk + ck;
  }
  const SolveParams& S0 = *a.prm;
  const LoadParams& LP = S0.loads[load];
  CgState& cg = a.cgs[load];
  const double N = (double)a.nx * (double)a.ny * (double)a.nz;
  if (STEP == CGS_ALPHA) {
    // <c~ : p> = <tau> + <p>, and p has zero mean
    cg.alpha = cg.rr / tot[6];
#pragma unroll
    for (int k = 0; k < 6; ++k) cg.sx[k] += cg.alpha * (tot[k] / N);
    return;
  }
  const double rr = tot[6];
  if (STEP == CGS_INIT) {
#pragma unroll
    for (int k = 0; k < 6; ++k) {
      cg.sE[k] = tot[k] / N + LP.E[k];  // <c~ : E> = <tau_E> + I : E
      cg.sx[k] = 0.0;
    }
    cg.beta = 0.0;
  } else {
    cg.beta = rr / cg.rr;
  }
  cg.rr = rr;
  double sig[6];
#pragma unroll
  for (int k = 0; k < 6; ++k) sig[k] = cg.sE[k] + cg.sx[k];
  const double fro = sqrt(sig[0] * sig[0] + sig[1] * sig[1] + sig[2] * sig[2] +
                          2.0 * (sig[3] * sig[3] + sig[4] * sig[4] + sig[5] * sig[5]));
  const double rms = sqrt(fmax(rr, 0.0) * (double)a.nx / N);
  const double e = fro > 0.0 ? rms / fro : (rr == 0.0 ? 0.0 : INFINITY);
  const int i = STEP == CGS_INIT ? 0 : st->iter;
  if (i < a.hist_cap) {
    a.errhist[(size_t)load * a.hist_cap + i] = e;
#pragma unroll
    for (int k = 0; k < 6; ++k) a.sighist[((size_t)load * a.hist_cap + i) * 6 + k] = sig[k];
  }
  if (i == 0) {
    st->err0 = e;
    st->res0 = rms;
  }
  int status = ST_RUNNING;
  if (e < S0.tol)
    status = ST_CONVERGED;
  else if (!isfinite(e))
    status = ST_DIVERGED;
  else if (i >= S0.max_iter)
    status = ST_NOT_CONVERGED;
  st->err = e;
  st->iters = i;
#pragma unroll
  for (int k = 0; k < 6; ++k) st->sig[k] = sig[k];
  if (status != ST_RUNNING) {
    st->status = status;
    st->done = 1;
  }
  st->iter = i + 1;
}

// ------------------------------------------------------------ registry --
using solve_launch_fn = hipError_t (*)(const SolveArgs&, hipStream_t);

// Candidate schedules of one axis length, timed by the plan's autotuner.
struct XKern {
  solve_launch_fn first, iter, exp;
  int lines;         // (y, z) lines per block
  const char* name;  // iteration-mode instance, name<template arguments>
};
struct YKern {
  solve_launch_fn fwd, inv;
  int width;  // kx columns per block
  const char* fwd_name;
  const char* inv_name;
};
struct ZKern {
  solve_launch_fn run;
  int width;    // kx columns per block
  int threads;  // block size
  int groups;   // components per LDS transform (-1: one wavefront per component)
  const char* name;
};

template <typename T> constexpr const char* type_name() { return sizeof(T) == 8 ? "double" : "float"; }

// Instance names in the form profilers print them (spaces dropped), built
// once per instantiation.
template <int TAG, typename T, int... A> const char* instance_name(const char* base) {
  static char buf[64];
  static const int once = [&] {
    int o = snprintf(buf, sizeof buf, "%s<%s", base, type_name<T>());
    for (int v : {A...}) o += snprintf(buf + o, sizeof buf - (size_t)o, ",%d", v);
    snprintf(buf + o, sizeof buf - (size_t)o, ">");
    return 0;
  }();
  (void)once;
  return buf;
}
constexpr int kMaxVariants = 10;
struct AxisKernels {
  int n;
  int nxv, nyv, nzv;
  XKern x[kMaxVariants];
  YKern y[kMaxVariants];
  ZKern z[kMaxVariants];
};

constexpr int clamp_int(int v, int lo, int hi) { return v < lo ? lo : (v > hi ? hi : v); }
constexpr int round64(int v) { return (v + 63) / 64 * 64; }

// xsweep variant v: lines per block from {8, 4, 2}, limited to 56 KB of LDS;
// v = 3 is v = 0 with butterflies of radix 9 or below (fewer registers than
// the single-precision default of up to 27).
template <typename T, int N, int V> struct XTile {
  static constexpr int want = (V == 0 || V == 3) ? 8 : (V == 1 ? 4 : 2);
  static constexpr int RMAX = V == 3 ? 9 : max_radix<T>();
  static constexpr int cap = (56 * 1024) / (3 * N * (int)sizeof(cx<T>));
  static constexpr int L = clamp_int(want < cap ? want : cap, 1, 8);
  static constexpr int NT = 256;
};
// ysweep variant v: width 128 B (v = 0), 256 B (v = 1, 3) or 512 B (v = 2)
// of kx per row; 256 threads, or 512 for v = 2 and 3.
template <typename T, int N, int V> struct YTile {
  static constexpr int W = (V == 0 ? 128 : (V == 2 ? 512 : 256)) / (int)sizeof(cx<T>);
  static constexpr int NT = V >= 2 ? 512 : 256;
};
// zsweep variant v: width 128 B (v = 0) or 256 B (v = 1, 64 B when that
// would need more than 1024 threads); threads so that each holds at most QT
// frequency slots (2 in FP64, 4 in FP32; half that when radix-7 butterflies
// are in play) under a 128-register cap.
// Variant 2 transforms CG = 3 (or 2) components per LDS pass at width
// 128 B when that fits in 56 KB of LDS; it holds one frequency slot per
// thread (so needs W N <= 1024).
// Prefetch depth D: 1, except variants 3 and 6 (single precision only),
// which are variant 0 with depth 2 and 3 (a fourth was measured no faster).
// LDS rows are padded to an odd stride, except in variants 4, 5 and 7
// (variants 0, 3 and 6 with rows of exactly W values).
template <typename T, int N, int V> struct ZTile {
  static constexpr int W0 = 128 / (int)sizeof(cx<T>);
  static constexpr int W1 = 256 / (int)sizeof(cx<T>);
  static constexpr int QT =
      V == 2 ? 1 : (sizeof(T) == 8 ? 2 : 4) / ((N % 7 == 0 || N % 11 == 0 || N % 13 == 0) ? 2 : 1);
  static constexpr int W = V == 1 ? ((W1 * N + QT - 1) / QT <= 1024 ? W1 : W0 / 2) : W0;
  static constexpr int lds3 = N * ((3 * W) | 1) * (int)sizeof(cx<T>);
  static constexpr int lds2 = N * ((2 * W) | 1) * (int)sizeof(cx<T>);
  static constexpr int CG =
      (V == 2 && W * N <= 1024) ? (lds3 <= 56 * 1024 ? 3 : (lds2 <= 56 * 1024 ? 2 : 1)) : 1;
  static constexpr int NT = clamp_int(round64((W * N + QT - 1) / QT), 64, 1024);
  static constexpr int D = (V == 3 || V == 5) ? 2 : (V >= 6 ? 3 : 1);
  static constexpr int PAD = (V == 4 || V == 5 || V == 7) ? 0 : 1;
};

template <typename T, int NX, int MODE, int V>
hipError_t launch_x(const SolveArgs& a, hipStream_t s) {
  using TL = XTile<T, NX, V>;
  hipLaunchKernelGGL((k_xsweep<T, NX, TL::L, TL::NT, MODE, TL::RMAX>), dim3(a.g2, a.n_load), dim3(TL::NT), 0, s,
                     a);
  return hipGetLastError();
}
template <typename T, int NY, int SIGN, int V>
hipError_t launch_y(const SolveArgs& a, hipStream_t s) {
  using TL = YTile<T, NY, V>;
  hipLaunchKernelGGL((k_ysweep<T, NY, TL::W, TL::NT, SIGN>), dim3(a.ntx3, a.nz, 6 * a.n_load), dim3(TL::NT), 0,
                     s, a);
  return hipGetLastError();
}
template <typename T, int NX, int MODE, int LW, int NW>
hipError_t launch_x_wave(const SolveArgs& a, hipStream_t s) {
  hipLaunchKernelGGL((k_xsweep_wave<T, NX, LW, NW, MODE>), dim3(a.g2, a.n_load), dim3(64 * NW), 0, s, a);
  return hipGetLastError();
}

template <typename T, int NZ, int W>
hipError_t launch_z_wave(const SolveArgs& a, hipStream_t s) {
  const int tiles = a.ntx4 * a.ny * a.n_load;
  hipLaunchKernelGGL((k_zsweep_wave<T, NZ, W>), dim3((tiles + 15) / 16 * 16), dim3(384), 0, s, a);
  return hipGetLastError();
}

template <typename T, int NZ, int V>
hipError_t launch_z(const SolveArgs& a, hipStream_t s) {
  using TL = ZTile<T, NZ, V>;
  hipLaunchKernelGGL((k_zsweep<T, NZ, TL::W, TL::NT, TL::CG, TL::D, TL::PAD>), dim3(a.ntx4, a.ny, a.n_load),
                     dim3(TL::NT), 0, s, a);
  return hipGetLastError();
}

template <typename T, int N, int V> XKern make_x() {
  using TL = XTile<T, N, V>;
  return XKern{&launch_x<T, N, MODE_FIRST, V>, &launch_x<T, N, MODE_ITER, V>, &launch_x<T, N, MODE_EXPORT, V>, TL::L,
               instance_name<0, T, N, TL::L, TL::NT, MODE_ITER, TL::RMAX>("xsweep")};
}
template <typename T, int N, int V> YKern make_y() {
  using TL = YTile<T, N, V>;
  return YKern{&launch_y<T, N, -1, V>, &launch_y<T, N, +1, V>, TL::W,
               instance_name<1, T, N, TL::W, TL::NT, -1>("ysweep"), instance_name<1, T, N, TL::W, TL::NT, 1>("ysweep")};
}
template <typename T, int N, int V> ZKern make_z() {
  using TL = ZTile<T, N, V>;
  return ZKern{&launch_z<T, N, V>, TL::W, TL::NT, TL::CG, instance_name<2, T, N, TL::W, TL::NT, TL::CG, TL::D, TL::PAD>("zsweep")};
}

template <typename T, int N>
AxisKernels make_axis_kernels() {
  AxisKernels k;
  k.n = N;
  k.x[0] = make_x<T, N, 0>();
  k.nxv = 1;
  if (XTile<T, N, 1>::L != k.x[0].lines) k.x[k.nxv++] = make_x<T, N, 1>();
  if (XTile<T, N, 2>::L != k.x[k.nxv - 1].lines) k.x[k.nxv++] = make_x<T, N, 2>();
  if constexpr (FftPlan<N, XTile<T, N, 3>::RMAX>::passes() != FftPlan<N, XTile<T, N, 0>::RMAX>::passes())
    k.x[k.nxv++] = make_x<T, N, 3>();
  k.y[0] = make_y<T, N, 0>();
  k.y[1] = make_y<T, N, 1>();
  k.y[2] = make_y<T, N, 2>();
  k.y[3] = make_y<T, N, 3>();
  k.nyv = 4;
  k.z[0] = make_z<T, N, 0>();
  k.z[1] = make_z<T, N, 1>();
  k.nzv = 2;
  if constexpr (ZTile<T, N, 2>::CG > 1) k.z[k.nzv++] = make_z<T, N, 2>();
  // deeper prefetch: always in single precision; in double precision only up
  // to 128 points, beyond which the extra slots spill
  constexpr bool deep = sizeof(T) == 4 || N <= 128;
  if constexpr (deep) k.z[k.nzv++] = make_z<T, N, 3>();
  k.z[k.nzv++] = make_z<T, N, 4>();
  if constexpr (deep) k.z[k.nzv++] = make_z<T, N, 5>();
  if constexpr (deep) k.z[k.nzv++] = make_z<T, N, 6>();
  if constexpr (deep) k.z[k.nzv++] = make_z<T, N, 7>();
  // wavefront x-sweeps: (2 lines per wave, 2 waves) and (1 line per wave, 4 waves)
  if constexpr (2 * N * ((6 | 1)) * (int)sizeof(cx<T>) <= 56 * 1024) {
    k.x[k.nxv++] = XKern{&launch_x_wave<T, N, MODE_FIRST, 2, 2>, &launch_x_wave<T, N, MODE_ITER, 2, 2>,
                         &launch_x_wave<T, N, MODE_EXPORT, 2, 2>, 4,
                         instance_name<3, T, N, 2, 2, MODE_ITER>("xsweep_wave")};
  }
  if constexpr (4 * N * 3 * (int)sizeof(cx<T>) <= 56 * 1024) {
    k.x[k.nxv++] = XKern{&launch_x_wave<T, N, MODE_FIRST, 1, 4>, &launch_x_wave<T, N, MODE_ITER, 1, 4>,
                         &launch_x_wave<T, N, MODE_EXPORT, 1, 4>, 4,
                         instance_name<3, T, N, 1, 4, MODE_ITER>("xsweep_wave")};
  }
  // wavefront z-sweep on 64-byte tiles when its six regions fit in 64 KB
  {
    constexpr int W = 64 / (int)sizeof(cx<T>);
    if constexpr (6 * N * (W | 1) * (int)sizeof(cx<T>) <= 64 * 1024)
      k.z[k.nzv++] = ZKern{&launch_z_wave<T, N, W>, W, 384, -1, instance_name<4, T, N, W>("zsweep_wave")};
  }
  return k;
}

// One schedule per sweep (the first variant of each): the lengths with a
// factor 11 or 13, which the resolution study of Section 3 needs but the
// benchmark workloads do not.
template <typename T, int N>
AxisKernels make_axis_kernels_basic() {
  AxisKernels k;
  k.n = N;
  k.x[0] = make_x<T, N, 0>();
  k.y[0] = make_y<T, N, 0>();
  k.z[0] = make_z<T, N, 0>();
  k.nxv = k.nyv = k.nzv = 1;
  return k;
}

// Lookup across the size groups compiled in separate translation units.
const AxisKernels* axis_kernels(bool fp64, int n);

}  // namespace hm
