// Shared types of the HIP library: complex vectors, solver state and the
// argument blocks passed to the kernels.  Included by device and host code.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace hm {

template <typename T> struct Vec2;
template <> struct Vec2<double> { using type = double2; };
template <> struct Vec2<float> { using type = float2; };
template <typename T> using cx = typename Vec2<T>::type;

template <typename C> __device__ __forceinline__ C c_add(C a, C b) { return C{a.x + b.x, a.y + b.y}; }
template <typename C> __device__ __forceinline__ C c_sub(C a, C b) { return C{a.x - b.x, a.y - b.y}; }
template <typename C> __device__ __forceinline__ C c_conj(C a) { return C{a.x, -a.y}; }
template <typename C> __device__ __forceinline__ C c_mul(C a, C b) {
  return C{a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x};
}
template <typename C, typename T> __device__ __forceinline__ C c_scale(C a, T s) { return C{a.x * s, a.y * s}; }

// Stop codes written at the end of an iteration (mirror the public HM_* codes).
enum : int { ST_RUNNING = -1, ST_CONVERGED = 0, ST_NOT_CONVERGED = 1, ST_STALLED = 2, ST_DIVERGED = 3 };
// Data flags raised while the material table is built.
enum : int { FLAG_NONE_FRACTIONAL = 1, FLAG_BAD_INCL = 2 };

constexpr double kDivergenceFactor = 1.0e3;
constexpr double kStallDecrease = 0.99;

// One per load case, in device memory.
struct SolverState {
  int iter;    // index of the next iterate to evaluate
  int done;    // nonzero once the load case has stopped
  int status;  // ST_*
  int iters;   // reported iterate index
  int iref;    // iteration of the last 1% improvement
  int pad0, pad1;
  double err;   // error of the last evaluated (or reported) iterate
  double err0;  // error of iterate 0
  double res0;  // equilibrium residual sqrt(sum |xi . sigma^|^2) of iterate 0
  double ref;   // error at iref
  double sig[6];  // <sigma> of the last evaluated (or reported) iterate
};

// Material of one problem (cell) of a solve.  A conduction solve keeps the
// phase conductivities in pl (pm unused) and the reference conductivity k0
// in rl (rm = 0); its table rows are (a - k0, b, 0, 0, 0, n0, n1, n2) for
// the filtered tensor k~ = a I + b n (x) n.
struct ProblemParams {
  double pl[2], pm[2];  // phase Lame parameters (0: matrix, 1: inclusion)
  double rl, rm;        // reference medium
  int rule;
  int nsph;
  const void* frac;   // T[N]
  const int* incl;    // int32[N] or null
  const double* sph;  // [nsph][4]: centre x, y, z, radius (voxel units)
  // Material table built once per solve from frac / incl: mid[v] = -1 for
  // a pure matrix voxel, -2 for a pure inclusion voxel, else the row of
  // coef (T[rows][8]: a1 - lambda0, a2 - 2 mu0, a3, a4, a5, n0, n1, n2) that
  // holds the voxel's filtered stiffness.
  const int* mid;
  const void* coef;
  // c~ - c0 of the two pure phases as (a1 - lambda0, a2 - 2 mu0) pairs
  // (conduction: (k - k0, 0)),
  // matrix then inclusion, rounded the way the working precision computes
  // them: in single precision from single-precision inputs, or in double
  float pure_f[4];
  double pure_d[4];
  // multi-phase cells (nphase >= 2 through the multi-phase entry points, 0
  // otherwise): Lame parameters of every phase (0: matrix), fractions of
  // phases 1..nphase-1 in frac as [phase - 1][N]; table rows 0..nphase-3
  // hold the pure phases 2..nphase-1
  int nphase;
  int gen;  // 1: anisotropic phases, general table rows (see below)
  double ph_l[8], ph_m[8];
  // anisotropic phases (gen = 1): Mandel matrices of the two phases,
  // row-major; the table holds rows of 24 reals (upper triangle of
  // c~ - c0, then padding), rows 0 and 1 the pure phases
  double cm[2][36];
};

// One load case: its macroscopic strain (tensor components) and problem;
// a conduction load keeps its mean gradient G in E[0..2] (E[3..5] = 0).
struct LoadParams {
  double E[6];
  int prob;
  int pad;
};

// Per-solve values read by the kernels through a device pointer, so that a
// captured graph stays valid from one solve to the next.  The load and
// problem arrays follow the header in the same device allocation.
struct SolveParams {
  double tol;
  int max_iter;
  int stall_window;
  int n_load;
  int n_prob;
  const LoadParams* loads;      // [n_load]
  const ProblemParams* probs;   // [n_prob]
};

// Plan-stable launch arguments.
// Conjugate-gradient scalars of one load case (FP64).
struct CgState {
  double rr;     // (r . r) of the current residual, Parseval-weighted sum
  double alpha;  // step of the current iteration
  double beta;   // direction update of the current iteration
  double pad;
  double sE[6];  // <c~ : E>
  double sx[6];  // <c~ : x> of the current iterate's fluctuation
};

struct SolveArgs {
  // elastic solves hold six components per load, conduction solves three
  // (the gradient), and one traction-history component instead of three
  void* spec;       // cx<T>[n_load][6][nz][ny][Hp]  x-spectrum / full spectrum
  const void* spec_in;  // x-sweep input (spec itself, or the CG direction)
  void* hist;       // cx<T>[n_load][3][nz][ny][Hp]  previous projected traction
  double* taupart;  // [n_load][g2][6]  per-block sums of tau
  double* errpart;  // [n_load][ny * ntx4]  per-block equilibrium sums
  SolverState* state;   // [n_load]
  double* errhist;      // [n_load][hist_cap]  error of every evaluated iterate
  double* sighist;      // [n_load][hist_cap][6]  <sigma> of every evaluated iterate
  const SolveParams* prm;
  void* eps_out;        // export target T[n_load][6][N]
  const void* twx;      // twiddles exp(-2 pi i k / n), per axis, cx<T>[n]
  const void* twy;
  const void* twz;
  int nx, ny, nz, H, dim, n_load;
  int Hp;  // row stride of spectrum and history (H rounded up to 128-byte rows)
  int g2, ntx3, ntx4;
  int hist_cap;
  int first;  // 1 on iterate 0 (uniform strain, empty traction history)
  // conjugate gradients (cg = 1): the sweeps apply -G to (c~ - I) : p with a
  // zero mean, no traction history; vectors x, r, p share spec's layout
  int cg;
  int cg_blocks;     // blocks per load of the CG vector kernels
  void* cgx;
  void* cgr;
  void* cgp;
  CgState* cgs;      // [n_load]
  double* cgpart;    // [n_load][cg_blocks]
  int cond;          // 1: conduction (3 gradient components), 0: elasticity
  // end of iteration inside the inverse y-sweep (fixed point only):
  // reducer arrivals per load case (0 between launches), the published sums
  // (six tau sums and the error sum, 8 doubles per load case) and the stop
  // flags as the forward y-sweep found them
  int* fin_count;
  double* fin_red;
  int* done_snap;
};

}  // namespace hm
