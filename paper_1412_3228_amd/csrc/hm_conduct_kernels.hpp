// Kernels of the conduction counterpart of the fixed-point iteration: the
// same Lippmann-Schwinger scheme (Section 2, eqs. 1-a, 1-b, 2) for a scalar
// property (thermal or electrical conductivity: the abstract expects the
// filters to give similar gains outside elasticity).
//
// The unknown is the gradient field g (three real components per voxel)
// with mean G; the flux is q = k~ g, the polarization tau = (k~ - k0) g for
// a scalar reference k0, and the Green operator of the reference medium
// acts as Gamma0^ tau^ = n (n . tau^) / k0 with n = xi / |xi|, so
// g^(xi) = -n (n . tau^) / k0 for xi != 0 and g^(0) = G.  The filtered
// conductivity of a fractional voxel follows the rules of Section 2 (eq. 3
// Voigt, eq. 4 Reuss, eq. 5 two-layer: the mean along the layers and the
// harmonic mean across them), held in the material table as
// k~ - k0 = (a - k0) I + b n (x) n.
//
// Storage and sweeps are those of the elastic solver with three components
// per load: x-half-spectra cx<T>[load][3][nz][ny][Hp]; xsweep (inverse
// x-DFT, tau, forward x-DFT), ysweep (shared kernel, NC = 3), zsweep
// (z-DFTs and Gamma0^), ysweep inverse with the end of the iteration
// (shared, conduction branch).  The xsweep packs components 0 and 1 of a line into one complex
// line and component 2 of two neighbouring lines into another.
//
// Equilibrium error: for xi != 0, xi . q^_i = |xi| (a_i - a_(i-1)) with
// a_i = n . tau^_i, because k0 xi . g^_i = -|xi| a_(i-1); the z-sweep keeps
// a (one complex value per frequency) from the previous iteration and
// accumulates sum w |xi|^2 |a_i - a_(i-1)|^2 over the half spectrum.
#pragma once

#include "hm_solve_kernels.hpp"

namespace hm {

// Complex row r of an x-sweep block of L lines: rows r < L pack components
// 0 and 1 of line r, rows L + j pack component 2 of lines 2j and 2j + 1.
struct CRow {
  int ca, la, cb, lb;
};
template <int L> __device__ __forceinline__ CRow crow(int r) {
  if (r < L) return CRow{0, r, 1, r};
  const int j = r - L;
  return CRow{2, 2 * j, 2, 2 * j + 1};
}

// Polarization tau = (k~ - k0) g from a table row (a - k0, b, ., ., ., n).
template <typename T> __device__ __forceinline__ void cond_tau(const T r[8], const T g[3], T tau[3]) {
  const T ng = r[5] * g[0] + r[6] * g[1] + r[7] * g[2];
  const T bn = r[1] * ng;
  tau[0] = r[0] * g[0] + bn * r[5];
  tau[1] = r[0] * g[1] + bn * r[6];
  tau[2] = r[0] * g[2] + bn * r[7];
}

// ---------------------------------------------------------------- xsweep --
// A block owns L consecutive (y, z) lines (L even); the global reads of its
// half-lines and material ids are issued into registers before any LDS
// work, as in the elastic x-sweep.
template <typename T, int NX, int L, int NT, int MODE>
__global__ __launch_bounds__(NT) void k_cxsweep(SolveArgs a) {
  static_assert(L % 2 == 0, "lines pair up for the third component");
  constexpr int LL = 3 * L / 2;
  constexpr int LD = LL | 1;
  constexpr int H = (NX + 1) / 2;
  constexpr int NW = NT / 64;
  constexpr int KH = (H + 63) / 64;
  constexpr int KX = (NX + 63) / 64;
  constexpr int RP = (LL + NW - 1) / NW;
  constexpr int RV = (L + NW - 1) / NW;
  __shared__ cx<T> buf[NX * LD];
  __shared__ cx<T> s_tw[NX];
  __shared__ double red[3][NW];
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
  cx<T>* spec = static_cast<cx<T>*>(a.spec) + (size_t)load * 3 * cs;
  const cx<T>* src = static_cast<const cx<T>*>(a.spec_in) + (size_t)load * 3 * cs;

  cx<T> pa[RP][KH], pb[RP][KH];
  if (MODE != MODE_FIRST) {
#pragma unroll
    for (int i = 0; i < RP; ++i) {
      const int r = wv + NW * i;
      const CRow R = crow<L>(r < LL ? r : 0);
      const bool oka = r < LL && line0 + R.la < nlines;
      const bool okb = r < LL && line0 + R.lb < nlines;
      const cx<T>* ra = src + (size_t)R.ca * cs + (size_t)(line0 + R.la) * Hp;
      const cx<T>* rb = src + (size_t)R.cb * cs + (size_t)(line0 + R.lb) * Hp;
#pragma unroll
      for (int m = 0; m < KH; ++m) {
        const int k = lane + 64 * m;
        pa[i][m] = (oka && k < H) ? ra[k] : cx<T>{T(0), T(0)};
        pb[i][m] = (okb && k < H) ? rb[k] : cx<T>{T(0), T(0)};
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
#pragma unroll
      for (int m = 0; m < KH; ++m) {
        const int k = lane + 64 * m;
        if (k < H) {
          const cx<T> A = pa[i][m], B = pb[i][m];
          buf[k * LD + r] = cx<T>{A.x - B.y, A.y + B.x};
          if (k > 0) buf[(NX - k) * LD + r] = cx<T>{A.x + B.y, B.x - A.y};
        }
      }
    }
    __syncthreads();
    fft_lines<T, NX, LL, NT, +1, LD>(buf, s_tw, tid);
  }

  // component c of line l at x, and its real slot in the LDS tile
  T* bufr = reinterpret_cast<T*>(buf);
  auto slot = [&](int x, int l, int c) -> int {
    return c < 2 ? 2 * (x * LD + l) + c : 2 * (x * LD + L + (l >> 1)) + (l & 1);
  };

  if (MODE == MODE_EXPORT) {
    const size_t N = (size_t)nlines * NX;
    T* out = static_cast<T*>(a.eps_out) + (size_t)load * 3 * N;
    for (int l = wv; l < L; l += NW) {
      const int line = line0 + l;
      if (line >= nlines) continue;
      for (int x = lane; x < NX; x += 64)
#pragma unroll
        for (int c = 0; c < 3; ++c) out[(size_t)c * N + (size_t)line * NX + x] = bufr[slot(x, l, c)];
    }
    return;
  }

  T rows[RV][KX][8];
#pragma unroll
  for (int i = 0; i < RV; ++i)
#pragma unroll
    for (int m = 0; m < KX; ++m) material_row<T>(MAT, mv[i][m], rows[i][m]);
  // each thread reads and then overwrites the same three real slots of its
  // voxel (component 2 shares a complex slot with the neighbouring line,
  // but in the other half), so the voxel pass needs no barrier of its own
  double acc[3] = {0.0, 0.0, 0.0};  // FP64 thread partials
#pragma unroll
  for (int i = 0; i < RV; ++i) {
    const int l = wv + NW * i;
    if (l >= L) continue;
    const int line = line0 + l;
#pragma unroll
    for (int m = 0; m < KX; ++m) {
      const int x = lane + 64 * m;
      if (x >= NX) continue;
      T g[3];
#pragma unroll
      for (int c = 0; c < 3; ++c) g[c] = MODE == MODE_FIRST ? T(LP.E[c]) : bufr[slot(x, l, c)];
      T tau[3] = {T(0), T(0), T(0)};
      if (line < nlines) {
        cond_tau<T>(rows[i][m], g, tau);
#pragma unroll
        for (int c = 0; c < 3; ++c) acc[c] += (double)tau[c];
      }
#pragma unroll
      for (int c = 0; c < 3; ++c) bufr[slot(x, l, c)] = tau[c];
    }
  }
  __syncthreads();
  fft_lines<T, NX, LL, NT, -1, LD>(buf, s_tw, tid);

#pragma unroll
  for (int i = 0; i < RP; ++i) {
    const int r = wv + NW * i;
    if (r >= LL) continue;
    const CRow R = crow<L>(r);
    const bool oka = line0 + R.la < nlines, okb = line0 + R.lb < nlines;
    cx<T>* ra = spec + (size_t)R.ca * cs + (size_t)(line0 + R.la) * Hp;
    cx<T>* rb = spec + (size_t)R.cb * cs + (size_t)(line0 + R.lb) * Hp;
#pragma unroll
    for (int m = 0; m < KH; ++m) {
      const int k = lane + 64 * m;
      if (k < H) {
        const cx<T> Z = buf[k * LD + r];
        const cx<T> Zc = c_conj(buf[((NX - k) % NX) * LD + r]);
        if (oka) ra[k] = cx<T>{T(0.5) * (Z.x + Zc.x), T(0.5) * (Z.y + Zc.y)};
        if (okb) rb[k] = cx<T>{T(0.5) * (Z.y - Zc.y), T(-0.5) * (Z.x - Zc.x)};
      }
    }
  }
  // deterministic block sums of the three tau components (slots 3..5 zero)
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    double v = acc[c];
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
    if (lane == 0) red[c][wv] = v;
  }
  __syncthreads();
  if (tid < 6) {
    double s = 0.0;
    if (tid < 3)
#pragma unroll
      for (int i = 0; i < NW; ++i) s += red[tid][i];
    a.taupart[((size_t)load * a.g2 + blockIdx.x) * 6 + tid] = s;
  }
}

// ---------------------------------------------------------------- zsweep --
// A block owns W adjacent kx columns of one (load, ky) slab; thread slot
// s = kz * W + w is one frequency.  The three components are transformed
// one at a time (unrolled, so that the normal component is a register) (the next one's global read in flight meanwhile, and after
// the last one the previous a) and folded into a = n . tau^; the inverse
// phase rebuilds each gradient component as -n_c a / (k0 N).
template <typename T, int NZ, int W, int NT>
__global__ __launch_bounds__(NT) void k_czsweep(SolveArgs a) {
  constexpr int SL = W * NZ;
  constexpr int Q = (SL + NT - 1) / NT;
  constexpr int LD = W | 1;
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
  cx<T>* sp = static_cast<cx<T>*>(a.spec) + (size_t)load * 3 * plane + (size_t)ky * Hp + kx0;
  cx<T>* hp = static_cast<cx<T>*>(a.hist) + (size_t)load * plane + (size_t)ky * Hp + kx0;
  const int ay = ky <= (ny - 1) / 2 ? ky : ky - ny;
  const double twopi = 6.283185307179586476925286766559;
  const bool hist_live = !a.first;

  bool ok[Q];
  unsigned off[Q], lds[Q];
  T n0[Q], n1[Q], n2[Q];
  cx<T> av[Q], cur[Q];
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
      const int k2 = kx * kx + ay * ay + az * az;
      const float rinv = k2 > 0 ? rsqrtf((float)k2) : 0.0f;
      n0[q] = (float)kx * rinv;
      n1[q] = (float)ay * rinv;
      n2[q] = (float)az * rinv;
    } else {
      const double x0 = twopi * kx, x1 = twopi * ay, x2 = twopi * az;
      const double q2 = x0 * x0 + x1 * x1 + x2 * x2;
      const double rinv = q2 > 0.0 ? 1.0 / sqrt(q2) : 0.0;
      n0[q] = T(x0 * rinv);
      n1[q] = T(x1 * rinv);
      n2[q] = T(x2 * rinv);
    }
    av[q] = cx<T>{T(0), T(0)};
    cur[q] = ok[q] ? sp[off[q]] : cx<T>{T(0), T(0)};
  }
  load_twiddles<T, NZ, NT>(s_tw, static_cast<const cx<T>*>(a.twz), tid);

#pragma unroll
  for (int c = 0; c < 3; ++c) {
#pragma unroll
    for (int q = 0; q < Q; ++q)
      if (tid + q * NT < SL) buf[lds[q]] = cur[q];
#pragma unroll
    for (int q = 0; q < Q; ++q) {
      if (c < 2)
        cur[q] = ok[q] ? sp[(size_t)(c + 1) * plane + off[q]] : cx<T>{T(0), T(0)};
      else
        cur[q] = (ok[q] && hist_live) ? hp[off[q]] : cx<T>{T(0), T(0)};
    }
    __syncthreads();
    fft_lines<T, NZ, W, NT, -1, LD, 9>(buf, s_tw, tid);
#pragma unroll
    for (int q = 0; q < Q; ++q) {
      if (tid + q * NT < SL) {
        const T nc = c == 0 ? n0[q] : (c == 1 ? n1[q] : n2[q]);
        const cx<T> v = buf[lds[q]];
        av[q].x += v.x * nc;
        av[q].y += v.y * nc;
      }
    }
    __syncthreads();
  }

  // equilibrium error partial; a kept for the next iteration
  double S = 0.0;
#pragma unroll
  for (int q = 0; q < Q; ++q) {
    if (!ok[q]) continue;
    const int s = tid + q * NT;
    const int kz = s / W, w = s - kz * W;
    const int az = kz <= (NZ - 1) / 2 ? kz : kz - NZ;
    const int kx = kx0 + w;
    if (kx == 0 && ay == 0 && az == 0) {
      hp[off[q]] = cx<T>{T(0), T(0)};
      continue;
    }
    hp[off[q]] = av[q];
    const double x0 = twopi * kx, x1 = twopi * ay, x2 = twopi * az;
    double dd;
    if constexpr (sizeof(T) == 4) {
      const double dx = (double)av[q].x - (double)cur[q].x, dy = (double)av[q].y - (double)cur[q].y;
      dd = dx * dx + dy * dy;
    } else {
      const double dx = av[q].x - cur[q].x, dy = av[q].y - cur[q].y;
      dd = dx * dx + dy * dy;
    }
    S += (kx == 0 ? 1.0 : 2.0) * (x0 * x0 + x1 * x1 + x2 * x2) * dd;
  }

  // g^_c = -n_c a / (k0 N) for xi != 0, g^(0) = G
  const T m = T(-1.0 / (P.rl * (double)a.nx * (double)ny * (double)NZ));
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    const T Gc = T(LP.E[c]);
#pragma unroll
    for (int q = 0; q < Q; ++q) {
      if (tid + q * NT < SL) {
        const bool zero = n0[q] == T(0) && n1[q] == T(0) && n2[q] == T(0);
        const T nc = m * (c == 0 ? n0[q] : (c == 1 ? n1[q] : n2[q]));
        buf[lds[q]] = zero ? cx<T>{Gc, T(0)} : cx<T>{nc * av[q].x, nc * av[q].y};
      }
    }
    __syncthreads();
    fft_lines<T, NZ, W, NT, +1, LD, 9>(buf, s_tw, tid);
#pragma unroll
    for (int q = 0; q < Q; ++q)
      if (tid + q * NT < SL && ok[q]) sp[(size_t)c * plane + off[q]] = buf[lds[q]];
    __syncthreads();
  }
  const double tot = block_sum<NT>(S, red);
  if (tid == 0) a.errpart[(size_t)load * ((size_t)ny * a.ntx4) + (size_t)ky * a.ntx4 + tile] = tot;
}

// ------------------------------------------------------------ registry --
// x: 8 lines per block while the tile fits in 56 KB of LDS, else fewer
template <typename T, int N> struct CXTile {
  static constexpr int fits(int L) { return N * (((3 * L) / 2) | 1) * (int)sizeof(cx<T>) <= 56 * 1024; }
  static constexpr int L = (sizeof(T) == 4 && fits(16)) ? 16 : (fits(8) ? 8 : (fits(4) ? 4 : 2));
  static constexpr int NT = 256;
};
// y: the elastic 256-byte tile (YTile variant 1); z: 128-byte tiles with at
// most 2 (FP64) or 4 (FP32) frequency slots per thread (half that with
// radix-7 butterflies)
template <typename T, int N> struct CZTile {
  static constexpr int W = 128 / (int)sizeof(cx<T>);
  static constexpr int QT = (sizeof(T) == 8 ? 2 : 4) / (N % 7 == 0 ? 2 : 1);
  static constexpr int NT = clamp_int(round64((W * N + QT - 1) / QT), 64, 1024);
};

template <typename T, int NX, int MODE>
hipError_t launch_cx(const SolveArgs& a, hipStream_t s) {
  using TL = CXTile<T, NX>;
  hipLaunchKernelGGL((k_cxsweep<T, NX, TL::L, TL::NT, MODE>), dim3(a.g2, a.n_load), dim3(TL::NT), 0, s, a);
  return hipGetLastError();
}
template <typename T, int NY, int SIGN>
hipError_t launch_cy(const SolveArgs& a, hipStream_t s) {
  using TL = YTile<T, NY, 1>;
  hipLaunchKernelGGL((k_ysweep<T, NY, TL::W, TL::NT, SIGN, 3>), dim3(a.ntx3, a.nz, 3 * a.n_load), dim3(TL::NT), 0,
                     s, a);
  return hipGetLastError();
}
template <typename T, int NZ>
hipError_t launch_cz(const SolveArgs& a, hipStream_t s) {
  using TL = CZTile<T, NZ>;
  hipLaunchKernelGGL((k_czsweep<T, NZ, TL::W, TL::NT>), dim3(a.ntx4, a.ny, a.n_load), dim3(TL::NT), 0, s, a);
  return hipGetLastError();
}

// The conduction kernels of one axis length (one schedule each).
struct CondKernels {
  int n;
  XKern x;
  YKern y;
  ZKern z;
};

template <typename T, int N> CondKernels make_cond_kernels() {
  using XT = CXTile<T, N>;
  using YT = YTile<T, N, 1>;
  using ZT = CZTile<T, N>;
  CondKernels k;
  k.n = N;
  k.x = XKern{&launch_cx<T, N, MODE_FIRST>, &launch_cx<T, N, MODE_ITER>, &launch_cx<T, N, MODE_EXPORT>, XT::L,
              instance_name<5, T, N, XT::L, XT::NT, MODE_ITER>("cxsweep")};
  k.y = YKern{&launch_cy<T, N, -1>, &launch_cy<T, N, +1>, YT::W,
              instance_name<6, T, N, YT::W, YT::NT, -1, 3>("ysweep"),
              instance_name<6, T, N, YT::W, YT::NT, 1, 3>("ysweep")};
  k.z = ZKern{&launch_cz<T, N>, ZT::W, ZT::NT, 1, instance_name<7, T, N, ZT::W, ZT::NT>("czsweep")};
  return k;
}

const CondKernels* cond_kernels(bool fp64, int n);

}  // namespace hm
