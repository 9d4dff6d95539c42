// Workgroup-cooperative mixed-radix (3, 5, 7) Stockham FFT on lines staged
// in LDS.  The discrete Fourier transforms of Section 2 run on odd grids, so
// every line length is a product of odd radices; no power-of-two tricks.
//
// Layout: a workgroup transforms L lines of length N held in LDS as
// buf[j * LD + l] (element j of line l, row stride LD >= L; an odd LD spreads
// strided accesses over all banks), so that consecutive threads touch
// consecutive addresses.  Each radix-R pass reads R inputs per butterfly into
// registers, synchronises, then writes the autosorted outputs back in place
// (read-all / barrier / write-all, so one buffer suffices).  Twiddles come
// from an LDS table tw[k] = exp(-2 pi i k / N).
//
// Pass p with radix R and stride Ns (product of the earlier radices):
// butterfly j takes x[j + r N/R], multiplies input r by
// exp(s 2 pi i (j mod Ns) r / (Ns R)), applies the size-R DFT and stores
// output r at (j div Ns) Ns R + (j mod Ns) + r Ns.  After the last pass the
// line holds X[k] = sum_j x[j] exp(s 2 pi i j k / N) in natural order.
#pragma once

#include "hm_common.hpp"

namespace hm {

// cos / sin (2 pi j / R), j = 0..R-1.
template <int R> struct Roots;
template <> struct Roots<3> {
  static constexpr double c[3] = {1.0, -0.5, -0.5};
  static constexpr double s[3] = {0.0, 0.8660254037844386467637, -0.8660254037844386467637};
};
template <> struct Roots<5> {
  static constexpr double c[5] = {1.0, 0.3090169943749474241023, -0.8090169943749474241023,
                                  -0.8090169943749474241023, 0.3090169943749474241023};
  static constexpr double s[5] = {0.0, 0.9510565162951535721164, 0.5877852522924731291687,
                                  -0.5877852522924731291687, -0.9510565162951535721164};
};
template <> struct Roots<7> {
  static constexpr double c[7] = {1.0, 0.623489801858733530525, -0.2225209339563144042889,
                                  -0.9009688679024191262361, -0.9009688679024191262361,
                                  -0.2225209339563144042889, 0.623489801858733530525};
  static constexpr double s[7] = {0.0, 0.7818314824680298087084, 0.9749279121818236070181,
                                  0.4338837391175581204758, -0.4338837391175581204758,
                                  -0.9749279121818236070181, -0.7818314824680298087084};
};

// In-register DFT of odd size R with exponent sign SIGN (-1 forward, +1 inverse):
// y_k = sum_m x_m w^(k m), w = exp(SIGN 2 pi i / R).  Pairs m, R - m share
// the cosine; the sine part changes sign between y_k and y_(R-k).
template <typename T, int R, int SIGN>
__device__ __forceinline__ void dft_small(cx<T>* x) {
  constexpr int H = (R - 1) / 2;
  cx<T> s[H + 1], d[H + 1];
#pragma unroll
  for (int m = 1; m <= H; ++m) {
    s[m] = c_add(x[m], x[R - m]);
    d[m] = c_sub(x[m], x[R - m]);
  }
  cx<T> y0 = x[0];
#pragma unroll
  for (int m = 1; m <= H; ++m) y0 = c_add(y0, s[m]);
  cx<T> y[R];
  y[0] = y0;
#pragma unroll
  for (int k = 1; k <= H; ++k) {
    cx<T> A = x[0];
    cx<T> B = {T(0), T(0)};
#pragma unroll
    for (int m = 1; m <= H; ++m) {
      const T cc = T(Roots<R>::c[(k * m) % R]);
      const T ss = T(Roots<R>::s[(k * m) % R]);
      A.x += cc * s[m].x;
      A.y += cc * s[m].y;
      B.x += ss * d[m].x;
      B.y += ss * d[m].y;
    }
    // i * B = (-B.y, B.x); y_k = A + SIGN i B, y_(R-k) = A - SIGN i B
    if (SIGN < 0) {
      y[k] = cx<T>{A.x + B.y, A.y - B.x};
      y[R - k] = cx<T>{A.x - B.y, A.y + B.x};
    } else {
      y[k] = cx<T>{A.x - B.y, A.y + B.x};
      y[R - k] = cx<T>{A.x + B.y, A.y - B.x};
    }
  }
#pragma unroll
  for (int k = 0; k < R; ++k) x[k] = y[k];
}

// Compile-time radix schedule of a length: 7s, then 5s, then 3s.
template <int N> struct FftPlan {
  static constexpr int passes() {
    int n = N, c = 0;
    while (n % 7 == 0) { n /= 7; ++c; }
    while (n % 5 == 0) { n /= 5; ++c; }
    while (n % 3 == 0) { n /= 3; ++c; }
    return n == 1 ? c : -1;
  }
  static constexpr int radix(int p) {
    int n = N, c = 0;
    while (n % 7 == 0) { if (c == p) return 7; n /= 7; ++c; }
    while (n % 5 == 0) { if (c == p) return 5; n /= 5; ++c; }
    while (n % 3 == 0) { if (c == p) return 3; n /= 3; ++c; }
    return 1;
  }
  static constexpr int stride(int p) {
    int s = 1;
    for (int q = 0; q < p; ++q) s *= radix(q);
    return s;
  }
  static_assert(passes() >= 0, "line length must be a product of 3, 5 and 7");
};

// Ordering of LDS accesses between the lanes of one wavefront: LDS executes
// a wave's instructions in order, so a code-motion barrier for the compiler
// is all that is needed (no s_barrier, no wait).
__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// WAVE = false: all NT threads of the block cooperate (block barriers).
// WAVE = true: one wavefront (NT = 64, tid = lane) owns the lines.
template <bool WAVE> __device__ __forceinline__ void pass_sync() {
  if constexpr (WAVE)
    wave_sync();
  else
    __syncthreads();
}

template <typename T, int N, int L, int NT, int R, int NS, int SIGN, int LD, bool WAVE = false>
__device__ __forceinline__ void fft_pass(cx<T>* buf, const cx<T>* tw, int tid) {
  constexpr int NB = N / R;
  constexpr int TOT = L * NB;
  constexpr int PER = (TOT + NT - 1) / NT;
  constexpr bool EXACT = (PER * NT == TOT);
  cx<T> v[PER][R];
#pragma unroll
  for (int q = 0; q < PER; ++q) {
    const int b = tid + q * NT;
    if (EXACT || b < TOT) {
      const int l = b % L, j = b / L;
#pragma unroll
      for (int r = 0; r < R; ++r) v[q][r] = buf[(j + r * NB) * LD + l];
    }
  }
  pass_sync<WAVE>();
#pragma unroll
  for (int q = 0; q < PER; ++q) {
    const int b = tid + q * NT;
    if (EXACT || b < TOT) {
      const int l = b % L, j = b / L;
      const int jm = j % NS;
      if (NS > 1) {
        constexpr int STEP = N / (NS * R);
#pragma unroll
        for (int r = 1; r < R; ++r) {
          cx<T> w = tw[jm * r * STEP];
          if (SIGN > 0) w.y = -w.y;
          v[q][r] = c_mul(v[q][r], w);
        }
      }
      dft_small<T, R, SIGN>(v[q]);
      const int base = (j / NS) * NS * R + jm;
#pragma unroll
      for (int r = 0; r < R; ++r) buf[(base + r * NS) * LD + l] = v[q][r];
    }
  }
  pass_sync<WAVE>();
}

// Transforms the L lines in buf.  The caller synchronises before the call
// (data staged); the buffer is complete and synchronised on return.
template <typename T, int N, int L, int NT, int SIGN, int LD = L, int P = 0>
__device__ __forceinline__ void fft_lines(cx<T>* buf, const cx<T>* tw, int tid) {
  if constexpr (P < FftPlan<N>::passes()) {
    fft_pass<T, N, L, NT, FftPlan<N>::radix(P), FftPlan<N>::stride(P), SIGN, LD>(buf, tw, tid);
    fft_lines<T, N, L, NT, SIGN, LD, P + 1>(buf, tw, tid);
  }
}

// Wavefront form: the 64 lanes of one wave transform the L lines in buf;
// the caller orders its own LDS writes before the call with wave_sync().
template <typename T, int N, int L, int SIGN, int LD = L, int P = 0>
__device__ __forceinline__ void fft_lines_wave(cx<T>* buf, const cx<T>* tw, int lane) {
  if constexpr (P < FftPlan<N>::passes()) {
    fft_pass<T, N, L, 64, FftPlan<N>::radix(P), FftPlan<N>::stride(P), SIGN, LD, true>(buf, tw, lane);
    fft_lines_wave<T, N, L, SIGN, LD, P + 1>(buf, tw, lane);
  }
}

// Copies the twiddle table of length N from global memory to LDS.
template <typename T, int N, int NT>
__device__ __forceinline__ void load_twiddles(cx<T>* s_tw, const cx<T>* g_tw, int tid) {
  for (int k = tid; k < N; k += NT) s_tw[k] = g_tw[k];
}

}  // namespace hm
