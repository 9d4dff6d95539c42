// Workgroup-cooperative mixed-radix Stockham FFT on lines staged in LDS;
// radices are the primes 3, 5, 7, 11, 13 and products of 3, 5 and 7
// (composite ones computed in registers).  The discrete Fourier transforms
// of Section 2 run on odd grids, so every line length is a product of odd
// radices; no power-of-two tricks.
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
#include "hm_roots.hpp"

namespace hm {

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

constexpr int smallest_factor(int r) {
  return r % 3 == 0 ? 3 : (r % 5 == 0 ? 5 : (r % 7 == 0 ? 7 : (r % 11 == 0 ? 11 : (r % 13 == 0 ? 13 : r))));
}

// In-register DFT of any radix R whose prime factors are 3, 5, 7, computed
// as A x B with A the smallest factor: with n = B n1 + n2 and k = k1 + A k2,
// X[k1 + A k2] = sum_n2 w_B^(n2 k2) w_R^(n2 k1) sum_n1 x[B n1 + n2] w_A^(n1 k1).
// The inner DFTs leave Y[n2][k1] at position B k1 + n2, the constant twiddles
// w_R^(n2 k1) follow, the outer DFTs leave X[k1 + A k2] at position
// B k1 + k2, and a final register permutation restores natural order.
template <typename T, int R, int SIGN>
__device__ __forceinline__ void dft_radix(cx<T>* x) {
  if constexpr (R == 3 || R == 5 || R == 7 || R == 11 || R == 13) {
    dft_small<T, R, SIGN>(x);
  } else {
    constexpr int A = smallest_factor(R);
    constexpr int B = R / A;
#pragma unroll
    for (int n2 = 0; n2 < B; ++n2) {
      cx<T> t[A];
#pragma unroll
      for (int n1 = 0; n1 < A; ++n1) t[n1] = x[B * n1 + n2];
      dft_small<T, A, SIGN>(t);
#pragma unroll
      for (int k1 = 0; k1 < A; ++k1) x[B * k1 + n2] = t[k1];
    }
#pragma unroll
    for (int k1 = 1; k1 < A; ++k1) {
#pragma unroll
      for (int n2 = 1; n2 < B; ++n2) {
        const int j = (n2 * k1) % R;
        const cx<T> w = {T(Roots<R>::c[j]), T(SIGN) * T(Roots<R>::s[j])};
        x[B * k1 + n2] = c_mul(x[B * k1 + n2], w);
      }
    }
#pragma unroll
    for (int k1 = 0; k1 < A; ++k1) dft_radix<T, B, SIGN>(x + B * k1);
    cx<T> y[R];
#pragma unroll
    for (int k = 0; k < R; ++k) y[k] = x[B * (k % A) + k / A];
#pragma unroll
    for (int k = 0; k < R; ++k) x[k] = y[k];
  }
}

// Largest radix of a precision's schedules: the butterflies live in
// registers, so doubles get smaller ones.
template <typename T> constexpr int max_radix() { return sizeof(T) == 8 ? 9 : 27; }

// Compile-time radix schedule of a length: its prime factors (13s, 11s,
// 7s, 5s, then 3s) merged greedily into radices no larger than RMAX,
// largest first (the first pass needs no twiddles).  An 11 or 13 is always a
// radix of its own (11 x 3 exceeds every RMAX).
template <int N, int RMAX> struct FftPlan {
  static constexpr int nprime() {
    int n = N, c = 0;
    while (n % 13 == 0) { n /= 13; ++c; }
    while (n % 11 == 0) { n /= 11; ++c; }
    while (n % 7 == 0) { n /= 7; ++c; }
    while (n % 5 == 0) { n /= 5; ++c; }
    while (n % 3 == 0) { n /= 3; ++c; }
    return n == 1 ? c : -1;
  }
  static constexpr int prime(int i) {
    int n = N, c = 0;
    while (n % 13 == 0) { if (c == i) return 13; n /= 13; ++c; }
    while (n % 11 == 0) { if (c == i) return 11; n /= 11; ++c; }
    while (n % 7 == 0) { if (c == i) return 7; n /= 7; ++c; }
    while (n % 5 == 0) { if (c == i) return 5; n /= 5; ++c; }
    while (n % 3 == 0) { if (c == i) return 3; n /= 3; ++c; }
    return 1;
  }
  // merged radices in factor order
  static constexpr int merged(int p, bool count_only) {
    int cnt = 0, cur = 1;
    for (int i = 0; i < nprime(); ++i) {
      const int f = prime(i);
      if (cur * f > RMAX && cur > 1) {
        if (!count_only && cnt == p) return cur;
        ++cnt;
        cur = 1;
      }
      cur *= f;
    }
    if (cur > 1) {
      if (!count_only && cnt == p) return cur;
      ++cnt;
    }
    return count_only ? cnt : 1;
  }
  static constexpr int passes() { return nprime() < 0 ? -1 : merged(0, true); }
  // pass p uses the merged radices sorted by decreasing size
  static constexpr int radix(int p) {
    int r[16] = {};
    const int n = passes();
    for (int i = 0; i < n; ++i) r[i] = merged(i, false);
    for (int i = 0; i < n; ++i)
      for (int j = i + 1; j < n; ++j)
        if (r[j] > r[i]) {
          const int t = r[i];
          r[i] = r[j];
          r[j] = t;
        }
    return r[p];
  }
  static constexpr int stride(int p) {
    int s = 1;
    for (int q = 0; q < p; ++q) s *= radix(q);
    return s;
  }
  static_assert(nprime() >= 0, "line length must be a product of 3, 5, 7, 11 and 13");
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
      dft_radix<T, R, SIGN>(v[q]);
      const int base = (j / NS) * NS * R + jm;
#pragma unroll
      for (int r = 0; r < R; ++r) buf[(base + r * NS) * LD + l] = v[q][r];
    }
  }
  pass_sync<WAVE>();
}

// Transforms the L lines in buf.  The caller synchronises before the call
// (data staged); the buffer is complete and synchronised on return.
template <typename T, int N, int L, int NT, int SIGN, int LD = L, int RMAX = max_radix<T>(), int P = 0>
__device__ __forceinline__ void fft_lines(cx<T>* buf, const cx<T>* tw, int tid) {
  using PL = FftPlan<N, RMAX>;
  if constexpr (P < PL::passes()) {
    fft_pass<T, N, L, NT, PL::radix(P), PL::stride(P), SIGN, LD>(buf, tw, tid);
    fft_lines<T, N, L, NT, SIGN, LD, RMAX, P + 1>(buf, tw, tid);
  }
}

// Wavefront form: the 64 lanes of one wave transform the L lines in buf;
// the caller orders its own LDS writes before the call with wave_sync().
template <typename T, int N, int L, int SIGN, int LD = L, int P = 0>
__device__ __forceinline__ void fft_lines_wave(cx<T>* buf, const cx<T>* tw, int lane) {
  using PL = FftPlan<N, max_radix<T>()>;
  if constexpr (P < PL::passes()) {
    fft_pass<T, N, L, 64, PL::radix(P), PL::stride(P), SIGN, LD, true>(buf, tw, lane);
    fft_lines_wave<T, N, L, SIGN, LD, P + 1>(buf, tw, lane);
  }
}

// Copies the twiddle table of length N from global memory to LDS.
template <typename T, int N, int NT>
__device__ __forceinline__ void load_twiddles(cx<T>* s_tw, const cx<T>* g_tw, int tid) {
  for (int k = tid; k < N; k += NT) s_tw[k] = g_tw[k];
}

}  // namespace hm
