/*
 * hm.h - C ABI of the MI355X (gfx950) filtered-property Lippmann-Schwinger
 * solver.
 *
 * Method: L. Gelebart, F. Ouaki, "Filtering material properties to improve
 * FFT-based methods for numerical homogenization" (arXiv:1412.3228).
 * Section 2 defines the problem (a periodic cell of stiffness field c under
 * a macroscopic strain E), the Lippmann-Schwinger equations (eqs. 1-a, 1-b),
 * the Green operator in Fourier space (eq. 2), the odd truncated frequency
 * set J, the filtered stiffness c~(x_a) = HR(c, omega(x_a)) with phase
 * fractions from a refined grid, the Voigt, Reuss and 2-layer rules
 * (eqs. 3, 4, 5) and the numerical setup (filter radius in pixel units,
 * interface normal from the inclusion centre, stress-equilibrium criterion).
 *
 * Conventions shared by every call
 * --------------------------------
 * Grid      dim = 2 (plane strain) or 3.  n[0], n[1], n[2] are the voxel
 *           counts along x, y, z; every n[d] must be odd and a product of
 *           3, 5 and 7 no larger than 243 (n[2] == 1 when dim == 2).
 *           Voxel (i, j, k) has its centre at (i + 0.5, j + 0.5, k + 0.5)
 *           in voxel units; the cell is periodic.
 * Fields    Real per-voxel fields are stored [z][y][x] (x fastest).
 *           Strain fields are [load][component][z][y][x] with the tensor
 *           components in the order 11, 22, 33, 23, 13, 12 (no sqrt(2)).
 *           In 2D the six components are still stored (33, 23, 13 are 0).
 * Tensors   Effective tensors are Mandel matrices (order 11, 22, 33, 23,
 *           13, 12 with sqrt(2) on shear rows and columns), column-major
 *           = row-major because they are symmetric up to solver tolerance;
 *           in 2D the 3x3 in-plane block (11, 22, 12).
 * Phases    phases[0] is the matrix, phases[1] the inclusion; the fraction
 *           field holds the inclusion volume fraction f in each filter.
 * Precision HM_FP64: every field and transform in double.  HM_MIXED:
 *           fields, transforms and the polarization in float; the
 *           equilibrium-error norm, the mean stress and the effective
 *           tensor are accumulated in double.  Fraction fields are double
 *           for HM_FP64 and float for HM_MIXED.
 * Memory    Pointers named d_* are device pointers on the current HIP
 *           device, owned by the caller; other pointers are host memory,
 *           read or written synchronously before the call returns.  The
 *           library owns its per-grid plans and workspace (released by
 *           hm_release_plans).  Device work is ordered on `stream`
 *           (a hipStream_t, NULL for the default stream); calls that
 *           return host results synchronise that stream.
 * Errors    Calls return HM_OK (0) on success, a positive warning when the
 *           solve stopped without meeting the tolerance (outputs are still
 *           written), or a negative error with nothing written;
 *           hm_last_error() returns the calling thread's last message.
 *           Calls on one stream must not overlap in time from several host
 *           threads (the workspace of a plan is shared).
 */
#ifndef HM_H
#define HM_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Return codes. */
#define HM_OK 0
#define HM_NOT_CONVERGED 1 /* max_iter reached before e < tol          */
#define HM_STALLED 2       /* error stopped decreasing (stall window)  */
#define HM_DIVERGED 3      /* error not finite, or equilibrium residual
                              above 1e3 times that of iterate 0        */
#define HM_E_ARG (-1)      /* invalid argument                          */
#define HM_E_SIZE (-2)     /* unsupported grid size                     */
#define HM_E_NOMEM (-3)    /* device allocation failed                  */
#define HM_E_DEVICE (-4)   /* HIP runtime error                         */
#define HM_E_DATA (-5)     /* device input inconsistent with the rule   */

/* Enumerations are int-sized.  In C++ their underlying type is fixed to
 * int, so that any int a caller passes is a value of the type and the
 * library's range checks (which reject unknown values with HM_E_ARG) are
 * well defined. */
#ifdef __cplusplus
#define HM_ENUM enum : int
#else
#define HM_ENUM enum
#endif

/* Homogenisation rule of the filter (Section 2, eqs. 3-5). */
typedef HM_ENUM {
  HM_RULE_NONE = 0,     /* no filter: c~ = phase tensor at the grid point  */
  HM_RULE_VOIGT = 1,    /* eq. 3: fraction-weighted mean of stiffnesses    */
  HM_RULE_REUSS = 2,    /* eq. 4: inverse of the mean of compliances       */
  HM_RULE_LAMINATE = 3  /* eq. 5: two-phase laminate ("2-layer") rule      */
} hm_rule;

typedef HM_ENUM { HM_FP64 = 0, HM_MIXED = 1 } hm_prec;

typedef struct {
  int dim;  /* 2 or 3 */
  int n[3]; /* voxels along x, y, z */
} hm_grid;

/* Isotropic elastic phase: Lame parameters. */
typedef struct {
  double lambda, mu;
} hm_iso;

/* Spherical (3D) or circular (2D, c[2] ignored) inclusion, voxel units,
 * centre in [0, n[d]) per axis, radius > 0. */
typedef struct {
  double c[3];
  double r;
} hm_sphere;

typedef HM_ENUM { HM_FIXED_POINT = 0, HM_CONJUGATE_GRADIENT = 1 } hm_method;

typedef struct {
  hm_prec prec;     /* HM_FP64 or HM_MIXED                                   */
  double tol;       /* stop when the equilibrium error e_i < tol (0: never)   */
  int max_iter;     /* last iterate index evaluated (>= 0)                   */
  double c0_alpha;  /* reference medium = alpha * mean of min/max Lame (> 0) */
  int check_every;  /* host polls the stop flags every k iterations (>= 1)   */
  int stall_window; /* > 0: stop when e has not dropped 1% for this many its */
  int use_graph;    /* nonzero: replay the iteration through a HIP graph      */
  int profile;      /* nonzero: time every kernel launch with HIP events on
                       `stream` (forces direct launches); see hm_last_timing */
  int autotune;     /* nonzero: on a plan's first solve, time every compiled
                       tile schedule of the sweeps and keep the fastest     */
  int schedule;     /* with autotune == 0: -1 for the first compiled schedule,
                       else xv | yv << 4 | zv << 8 selecting the variants
                       counted by hm_schedule_count (for tests)             */
  int method;       /* HM_FIXED_POINT (the basic scheme of Section 2) or
                       HM_CONJUGATE_GRADIENT (Krylov alternative named in
                       Section 5: CG on the same operator with c0 = identity;
                       c0_alpha, stall_window and profile do not apply; the
                       error is sqrt(<r:r>)/|<sigma>| of the residual r =
                       -G(c~:eps), G the projection on compatible fields; the
                       returned strain is the reported iterate itself).  Not
                       available in hm_effective_tensor_batch.               */
} hm_solve_opts;

/* Average device duration per launch of each kernel of the iteration, over
 * the sampled iterations (1, 5, 9, ...: events around the kernels of those
 * only, an event record costing a few microseconds of device time) that a
 * profiled solve evaluated (the longest load case); iterations = 0 and all
 * durations 0 when the solve stopped at iterate 0. */
typedef struct {
  int iterations; /* sampled iterations averaged                           */
  int n_load;     /* load cases of the solve                               */
  double ms[5];   /* xsweep, forward ysweep, zsweep, inverse ysweep
                     (milliseconds per launch); ms[4] is 0: the inverse
                     ysweep ends the iteration itself                      */
  int x_lines;    /* schedule in use: grid lines per xsweep block,         */
  int y_width;    /*   kx columns per ysweep block,                        */
  int z_width;    /*   kx columns per zsweep block                         */
  int z_threads;  /*   zsweep block size                                   */
  int z_groups;   /*   and components per zsweep LDS transform             */
  char kernel[5][64]; /* instances of the five kernels (iteration mode), as
                         name<template arguments>, e.g. zsweep<float,125,
                         16,512,1,2> for k_zsweep                          */
  double active_loads; /* load cases still iterating, averaged over the
                          sampled iterations (what a launch processed)     */
} hm_timing;

/* Per-load-case outcome. */
typedef struct {
  int iters;      /* index i of the reported iterate                      */
  int status;     /* HM_OK, HM_NOT_CONVERGED, HM_STALLED or HM_DIVERGED   */
  double err;     /* equilibrium error e_i of the reported iterate        */
  double err0;    /* e_0                                                  */
  double seconds; /* wall time of the whole call                          */
} hm_report;

/*
 * hm_filter - per-voxel phase fractions of a sphere/disk microstructure.
 *
 * Section 2: c~(x_a) = HR(c, omega(x_a)) with omega a uniform filter
 * centred on the grid point, the fractions being averages of the phase
 * indicators on a refined grid; the numerical setup gives the filter
 * radius in pixel units.  Refined grid: `subsamples` = S (even, 2..32)
 * points per voxel and axis, on the global lattice of spacing 1/S voxel
 * whose points are the centres of the S^dim sub-cells of every voxel.  A
 * refined point belongs to the inclusion set when its periodic minimum-image
 * distance to some sphere centre is <= that sphere's radius (centres are
 * rounded to the nearest multiple of 1/(2S) voxel).  The filter keeps the
 * refined points within `radius_vox` voxels of the voxel centre (closed
 * ball); M is their number.  rule == HM_RULE_NONE ignores the radius and
 * takes the single indicator value at the voxel centre (M = 1).
 *
 * Outputs (device, N = n[0]*n[1]*n[2] entries each, [z][y][x]):
 *   d_count  uint32 number of filter points inside the inclusion set;
 *   d_frac   count / M as one IEEE division, double (HM_FP64) or float
 *            (HM_MIXED);
 *   d_incl   nullable; for voxels with 0 < count < M the index of the
 *            sphere whose surface is nearest to the voxel centre (lowest
 *            index on ties), -1 elsewhere.
 * Counts are exact integers; the call returns once the kernel is queued.
 */
int hm_filter(const hm_grid* grid, const hm_sphere* spheres, int n_spheres,
              double radius_vox, int subsamples, hm_rule rule, hm_prec prec,
              uint32_t* d_count, void* d_frac, int32_t* d_incl, void* stream);

/*
 * hm_filter_noalloc - hm_filter for callers that cannot allocate device or
 * pinned memory (tight serving loops, harnesses that forbid allocation):
 * the same arguments, outputs and errors as hm_filter (two-phase filter),
 * with the per-call sphere table staged in a fixed device array of the
 * library instead of an allocated one.  At most
 * HM_FILTER_NOALLOC_MAX_SPHERES spheres (HM_E_SIZE beyond).  The array is
 * one per GPU, shared by every call on that GPU: calls that overlap on one
 * GPU (from different streams or host threads without ordering) race on it.
 * Returns after the filter kernel has finished on `stream`.
 */
#define HM_FILTER_NOALLOC_MAX_SPHERES 3072
int hm_filter_noalloc(const hm_grid* grid, const hm_sphere* spheres, int n_spheres,
                      double radius_vox, int subsamples, hm_rule rule, hm_prec prec,
                      uint32_t* d_count, void* d_frac, int32_t* d_incl, void* stream);

/*
 * hm_solve - basic fixed-point Lippmann-Schwinger solve with the filtered
 * stiffness, for n_load macroscopic strains at once.
 *
 * Section 2, eqs. 1-a, 1-b and 2: tau = (c~ - c0) : eps,
 * eps^(xi) = -Gamma0^(xi) : tau^(xi) for xi != 0, eps^(0) = E, on the odd
 * frequency set J with xi = 2 pi a.  c~ per voxel: the phase tensor where
 * f is exactly 0 or 1, else `rule` applied to f (HM_RULE_LAMINATE uses the
 * normal from the centre of sphere d_incl[v] to the voxel centre; e_1 when
 * d_incl[v] < 0).  The cell has length 1 along every axis (so a voxel is
 * 1/n[d] long on axis d) while spheres, the filter and the normal are in
 * voxel units: on a grid with unequal n[d] a sphere is an ellipsoid in the
 * cell's metric and the laminate normal is taken in voxel units.  c0 is isotropic with Lame parameters c0_alpha times the
 * mean of the phases' smallest and largest values (Figure 3 caption).
 * Iterate i evaluates sigma_i = c~ : eps_i and its stress-equilibrium error
 * e_i = sqrt(sum_xi |xi . sigma^_i(xi)|^2) / |sigma^_i(0)| (Section 2 setup;
 * unnormalised DFT, Frobenius norms) and stops as hm_report describes.
 *
 * Inputs:  d_frac (N, precision of opts->prec), d_incl (N int32, required
 *          for HM_RULE_LAMINATE, else nullable), spheres (host, used for the
 *          laminate normals), E (host, 6 * n_load doubles, tensor
 *          components 11, 22, 33, 23, 13, 12 of each load case).
 * Outputs: sig_mean (host, 6 * n_load doubles, <sigma_i> of the reported
 *          iterate), rep (host, n_load entries, nullable), d_eps (nullable,
 *          device, 6 * N * n_load reals of the solve precision: the strain
 *          field produced by the update from the reported iterate).
 * Returns the largest status over load cases, or a negative error.
 * HM_E_DATA: a fractional voxel with HM_RULE_NONE, or d_incl out of range.
 * n_load is at most 4096.
 */
int hm_solve(const hm_grid* grid, const hm_iso phases[2], hm_rule rule,
             const void* d_frac, const int32_t* d_incl,
             const hm_sphere* spheres, int n_spheres,
             const double* E, int n_load, const hm_solve_opts* opts,
             void* d_eps, double* sig_mean, hm_report* rep, void* stream);

/*
 * hm_effective_tensor - effective stiffness from the mean stresses of the
 * unit Mandel strains (6 in 3D, 11/22/12 in 2D), all solved in one batched
 * launch (the paper's macroscopic output is the average stress, Section 3).
 * Column J of C_mandel is Mandel(<sigma>) under the J-th unit Mandel strain.
 * Inputs as hm_solve.  Outputs: C_mandel (host, 36 or 9 doubles, row-major),
 * rep (host, 6 or 3 entries, nullable), d_eps (nullable, device strain
 * fields of the 6 or 3 solves, as hm_solve).
 */
int hm_effective_tensor(const hm_grid* grid, const hm_iso phases[2], hm_rule rule,
                        const void* d_frac, const int32_t* d_incl,
                        const hm_sphere* spheres, int n_spheres,
                        const hm_solve_opts* opts, double* C_mandel,
                        void* d_eps, hm_report* rep, void* stream);

/*
 * hm_conduct_solve - the same filtered fixed-point scheme for a scalar
 * conductivity (thermal or electrical), for n_load mean gradients at once.
 *
 * Section 2's scheme applied to conduction, the other physical context in
 * which the abstract expects the filters to help: the unknown is the gradient
 * field g with mean G, the flux q = k~ g, tau = (k~ - k0) g, and
 * g^(xi) = -n (n . tau^(xi)) / k0 for xi != 0 (n = xi / |xi|), g^(0) = G,
 * the conduction form of eqs. 1-a, 1-b and 2.  k~ per voxel: k[p] I where
 * f is exactly 0 or 1, else the rule at f: HM_RULE_VOIGT <k> I (eq. 3),
 * HM_RULE_REUSS <1/k>^-1 I (eq. 4), HM_RULE_LAMINATE <k> (I - n n) +
 * <1/k>^-1 n n (eq. 5: layers along the interface in parallel, across it in
 * series; n from the centre of sphere d_incl[v] to the voxel centre, e_1
 * when d_incl[v] < 0).  k0 = c0_alpha times the mean of the smallest and
 * largest conductivity.  Error of iterate i:
 * e_i = sqrt(sum_xi |xi . q^_i(xi)|^2) / |q^_i(0)| (flux equilibrium, same
 * stop rules as hm_solve).
 *
 * Inputs:  k (host, 2 doubles > 0: matrix, inclusion), d_frac, d_incl,
 *          spheres as hm_solve, G (host, 3 * n_load doubles: the x, y, z
 *          components of each mean gradient; in 2D the z component is
 *          carried unchanged).  opts as hm_solve, except that only
 *          HM_FIXED_POINT is accepted, autotune is ignored and schedule
 *          must be -1 or 0 (one compiled schedule).
 * Outputs: flux_mean (host, 3 * n_load doubles, <q_i> of the reported
 *          iterate), rep (host, n_load entries, nullable), d_grad
 *          (nullable, device, 3 * N * n_load reals of the solve precision,
 *          [load][component][z][y][x]: the gradient field produced by the
 *          update from the reported iterate).
 * Returns the largest status over load cases, or a negative error
 * (HM_E_DATA as hm_solve).  n_load is at most 4096.
 */
int hm_conduct_solve(const hm_grid* grid, const double k[2], hm_rule rule,
                     const void* d_frac, const int32_t* d_incl,
                     const hm_sphere* spheres, int n_spheres,
                     const double* G, int n_load, const hm_solve_opts* opts,
                     void* d_grad, double* flux_mean, hm_report* rep, void* stream);

/*
 * hm_effective_conductivity - effective conductivity tensor from the mean
 * fluxes under the unit gradients e_1..e_dim, solved in one batched launch.
 * Column J of K is <q> under G = e_J.  Inputs as hm_conduct_solve.
 * Outputs: K (host, 9 doubles in 3D, 4 in 2D, row-major), rep (host, 3 or 2
 * entries, nullable), d_grad (nullable, device gradient fields of the 3 or
 * 2 solves, as hm_conduct_solve).
 */
int hm_effective_conductivity(const hm_grid* grid, const double k[2], hm_rule rule,
                              const void* d_frac, const int32_t* d_incl,
                              const hm_sphere* spheres, int n_spheres,
                              const hm_solve_opts* opts, double* K,
                              void* d_grad, hm_report* rep, void* stream);

/* One cell of a batch: grid, phases, rule and its device fraction / normal
 * fields and host sphere table, with the meanings of hm_solve. */
typedef struct {
  hm_grid grid;
  hm_iso phases[2];
  hm_rule rule;
  const void* d_frac;
  const int32_t* d_incl;
  const hm_sphere* spheres;
  int n_spheres;
} hm_problem;

/*
 * hm_effective_tensor_batch - effective tensors of many cells at once.
 *
 * The cells may have different grid sizes.  Cells that share a grid are
 * solved together: every launch of the iteration covers all load cases of
 * all of them (each load case with its own cell's material and reference
 * medium and its own stop decision), and the grid groups are iterated side
 * by side (one captured graph per block of check_every iterations when
 * opts->use_graph is set).  Outputs, in the order of `problems`:
 * C_mandel (host, 36 doubles per 3D cell and 9 per 2D cell, row-major) and
 * rep (host, 6 or 3 entries per cell, nullable).  Returns the largest
 * status, or a negative error (profiling is not available for batches).
 */
int hm_effective_tensor_batch(const hm_problem* problems, int n_problems, const hm_solve_opts* opts,
                              double* C_mandel, hm_report* rep, void* stream);

/*
 * hm_solve_adjoint - gradient of a loss L(C_eff) with respect to the phase
 * Lame parameters and the per-voxel fraction field.
 *
 * The discrete problem is self-adjoint (Gamma0 and c~ are symmetric), so
 * the adjoint fields of the unit-strain solves are those solves' own
 * fields and dC_KL/dtheta = (1/N) sum_x eps^K : dc~/dtheta : eps^L (Hill
 * energy identity at the discrete solution).  dc~/dtheta differentiates the
 * rule of eqs. 3-5 at each voxel's fraction and normal; pure voxels use the
 * phase tensor for the Lame derivatives; c0 is held fixed.
 *
 * Inputs:  dLdC (host, 36 or 9 doubles, row-major, = dL/dC_mandel),
 *          d_eps (device, the n_load = 6 or 3 fields written by
 *          hm_effective_tensor with the same inputs, solve precision),
 *          d_frac, d_incl, spheres as hm_solve.
 * Outputs: dLdphase (host, 4 doubles: dL/dlambda_0, dL/dmu_0, dL/dlambda_1,
 *          dL/dmu_1, accumulated in double), d_dLdfrac (nullable, device,
 *          N reals of the solve precision, zero for HM_RULE_NONE).
 */
int hm_solve_adjoint(const hm_grid* grid, const hm_iso phases[2], hm_rule rule,
                     const void* d_frac, const int32_t* d_incl,
                     const hm_sphere* spheres, int n_spheres, hm_prec prec,
                     const double* dLdC, const void* d_eps, int n_load,
                     double* dLdphase, void* d_dLdfrac, void* stream);

/*
 * Cells of more than two phases (Section 2: the Voigt rule of eq. 3 and the
 * Reuss rule of eq. 4 are written for Nphase phases).  Phase 0 is the
 * matrix; every inclusion carries a phase label in 1..n_phases-1
 * (n_phases in 2..8).
 *
 * hm_filter_phases - per-phase fractions: for each label p the refined
 * points of the filter inside the spheres of label p, counted exactly as
 * hm_filter counts the inclusion set (same lattice, stencil and rule ==
 * HM_RULE_NONE meaning).  Spheres of different labels must not overlap
 * (HM_E_ARG otherwise: a refined point would belong to two phases).
 * Inputs:  labels (host, n_spheres int32 in 1..n_phases-1), others as
 *          hm_filter.
 * Outputs: d_count (device, uint32 [n_phases-1][N]), d_frac (device,
 *          [n_phases-1][N] reals of the precision, count / M).
 */
int hm_filter_phases(const hm_grid* grid, const hm_sphere* spheres, const int32_t* labels,
                     int n_spheres, int n_phases, double radius_vox, int subsamples,
                     hm_rule rule, hm_prec prec, uint32_t* d_count, void* d_frac,
                     void* stream);

/*
 * hm_solve_phases / hm_effective_tensor_phases - hm_solve and
 * hm_effective_tensor for a multi-phase cell.  c~ per voxel: phase 0 where
 * all fractions are 0, phase p where f_p is exactly 1, else HM_RULE_VOIGT
 * (sum_i f_i c_i, eq. 3) or HM_RULE_REUSS ((sum_i f_i c_i^-1)^-1, eq. 4)
 * with f_0 = 1 - (f_1 + ... + f_(P-1)) summed in phase order; the 2-layer
 * rule (eq. 5, two phases) is refused.  c0 = c0_alpha times the mean of the
 * smallest and largest Lame parameters over all phases.
 * Inputs:  phases (host, n_phases isotropic phases, [0] the matrix),
 *          d_frac (device, [n_phases-1][N] as written by hm_filter_phases),
 *          E, n_load, opts as hm_solve (hm_solve_phases).
 * Outputs as hm_solve / hm_effective_tensor.  HM_E_DATA: a fractional voxel
 * with HM_RULE_NONE.  With n_phases == 2 the results equal hm_solve's on
 * the same fractions up to rounding.
 */
int hm_solve_phases(const hm_grid* grid, const hm_iso* phases, int n_phases, hm_rule rule,
                    const void* d_frac, const double* E, int n_load,
                    const hm_solve_opts* opts, void* d_eps, double* sig_mean,
                    hm_report* rep, void* stream);
int hm_effective_tensor_phases(const hm_grid* grid, const hm_iso* phases, int n_phases,
                               hm_rule rule, const void* d_frac, const hm_solve_opts* opts,
                               double* C_mandel, void* d_eps, hm_report* rep, void* stream);

/*
 * hm_solve_aniso / hm_effective_tensor_aniso - hm_solve and
 * hm_effective_tensor for two anisotropic phases (Section 2's rules are
 * written for general phase tensors).  c~ per voxel: the phase tensor where
 * f is 0 or 1, else Voigt (eq. 3), Reuss (eq. 4, compliances averaged) or
 * the 2-layer rule (eq. 5: continuous in-plane strain and out-of-plane
 * stress across an interface of normal n, with the fraction-weighted means
 * of the other parts), evaluated in double once per solve and stored as the
 * 21 upper-triangle entries of the Mandel matrix of c~ - c0.  Reference
 * medium: c0 = 2 mu0 I (lambda0 = 0) with 2 mu0 = c0_alpha times the mean
 * of the smallest and largest eigenvalue of the two phase Mandel matrices,
 * which keeps c - c0 within (-c0, c0).
 * Inputs:  C_phases (host, 2 x 36 doubles: the Mandel 6x6 matrices of the
 *          matrix then the inclusion phase, row-major, symmetric positive
 *          definite; order 11, 22, 33, 23, 13, 12 with sqrt(2) on shear
 *          rows and columns), other inputs and outputs as hm_solve /
 *          hm_effective_tensor (autotune times the y- and z-sweep
 *          schedules, the x-sweep being the one general-row form; with
 *          autotune == 0, schedule must be -1 or 0).
 * The tables of these solves hold 24 reals per fractional voxel and two
 * rows for the pure phases.
 */
int hm_solve_aniso(const hm_grid* grid, const double* C_phases, hm_rule rule,
                   const void* d_frac, const int32_t* d_incl,
                   const hm_sphere* spheres, int n_spheres,
                   const double* E, int n_load, const hm_solve_opts* opts,
                   void* d_eps, double* sig_mean, hm_report* rep, void* stream);
int hm_effective_tensor_aniso(const hm_grid* grid, const double* C_phases, hm_rule rule,
                              const void* d_frac, const int32_t* d_incl,
                              const hm_sphere* spheres, int n_spheres,
                              const hm_solve_opts* opts, double* C_mandel,
                              void* d_eps, hm_report* rep, void* stream);

/*
 * hm_fourier_series - the truncated Fourier series of a grid field,
 * evaluated on a finer grid (the extrapolated material properties of
 * Figure 4, Section 6).
 *
 * With the grid points at the voxel centres (a + 1/2) / n[d] of the unit
 * cell and the odd frequency set J of Section 2, the series
 * F(y) = sum_{a in J} c^(a) exp(2 pi i a . y), with c^ the normalised DFT
 * coefficients of the field, is real and equals the field at the grid
 * points; it is evaluated at the voxel centres (b + 1/2) / m[d] of an
 * m[0] x m[1] x m[2] grid (any m; odd multiples of n contain the grid
 * points).  Computed as three axis contractions with Dirichlet-kernel
 * matrices D_n(t) = sin(pi n t) / (n sin(pi t)), which is the same sum.
 *
 * Inputs:  grid (n[d] odd, 1..243, any odd value; n[2] = 1 in 2D),
 *          m (host, 3 ints in 1..4096, m[2] = 1 in 2D, at most 2^32
 *          points), d_field (device, n[0]*n[1]*n[2] reals [z][y][x],
 *          double for HM_FP64, float for HM_MIXED).
 * Output:  d_out (device, m[0]*m[1]*m[2] reals of the same type,
 *          [z][y][x]).  The call returns once the work is queued on
 *          `stream`; the Dirichlet matrices and two temporaries of each
 *          (n, m, precision) are kept until hm_release_plans, so calls with
 *          the same sizes on one stream must not overlap.
 */
int hm_fourier_series(const hm_grid* grid, const int m[3], hm_prec prec,
                      const void* d_field, void* d_out, void* stream);

/*
 * hm_stiffness_component - Mandel entry (I, J) of the filtered stiffness
 * c~(x_a) at every voxel (Section 2, eqs. 3-5 as in hm_solve: the phase
 * tensor where f is 0 or 1, else the rule at f with the interface normal
 * of d_incl), evaluated in double and stored in the precision of `prec`:
 * the per-voxel property field that Figure 4 extrapolates.
 * Inputs as hm_solve; I, J in 0..5 (Mandel order 11, 22, 33, 23, 13, 12).
 * Output: d_out (device, N reals [z][y][x]).  HM_E_DATA as hm_solve.
 */
int hm_stiffness_component(const hm_grid* grid, const hm_iso phases[2], hm_rule rule,
                           const void* d_frac, const int32_t* d_incl,
                           const hm_sphere* spheres, int n_spheres, hm_prec prec,
                           int I, int J, void* d_out, void* stream);

/*
 * hm_stress_field - local stress sigma = c~ : eps at every voxel (the
 * stress maps of Figure 2, Section 4), for strain fields such as the d_eps
 * written by hm_solve.  c~ as hm_solve builds it (evaluated in double).
 * Inputs:  material as hm_solve, d_eps (device, n_load x 6 x N reals of the
 *          precision, [load][component][z][y][x], tensor components 11, 22,
 *          33, 23, 13, 12).
 * Output:  d_sig (device, same layout and type).  Returns after the kernel;
 *          HM_E_DATA as hm_solve.
 */
int hm_stress_field(const hm_grid* grid, const hm_iso phases[2], hm_rule rule,
                    const void* d_frac, const int32_t* d_incl,
                    const hm_sphere* spheres, int n_spheres, hm_prec prec,
                    const void* d_eps, int n_load, void* d_sig, void* stream);

/*
 * hm_flux_field - local flux q = k~ g at every voxel for gradient fields
 * such as the d_grad written by hm_conduct_solve; k~ as hm_conduct_solve
 * builds it (evaluated in double).  Inputs as hm_conduct_solve, d_grad
 * (device, n_load x 3 x N reals of the precision, [load][component][z][y][x]).
 * Output: d_flux (device, same layout and type).  Returns after the kernel;
 * HM_E_DATA as hm_solve.
 */
int hm_flux_field(const hm_grid* grid, const double k[2], hm_rule rule,
                  const void* d_frac, const int32_t* d_incl,
                  const hm_sphere* spheres, int n_spheres, hm_prec prec,
                  const void* d_grad, int n_load, void* d_flux, void* stream);

/* Timing of the calling thread's last solve run with opts->profile set.
 * Returns HM_E_ARG when there is none. */
int hm_last_timing(hm_timing* out);

/*
 * hm_last_history - the iterates of the calling thread's last solve of one
 * grid (hm_solve, hm_effective_tensor and their conduction, multi-phase and
 * anisotropic forms; not hm_effective_tensor_batch): the equilibrium error
 * e_i of every evaluated iterate (Section 2 setup) and its mean stress
 * <sigma_i> (Section 3's average, tensor components 11, 22, 33, 23, 13, 12;
 * the mean flux in slots 0-2 for conduction), so that an effective-tensor
 * trajectory can be followed iterate by iterate.
 * n_load: the load count of that solve (HM_E_ARG otherwise).
 * cap:    iterates per load case the host arrays hold.
 * err:    host, n_load x cap doubles: err[l * cap + i] = e_i of load case l.
 * sig:    host, n_load x cap x 6 doubles, or NULL.
 * Iterates beyond a load case's reported one (hm_report.iters), or beyond
 * max_iter + 1, are set to NaN.  Synchronous device-to-host copies.  Fails
 * with HM_E_ARG when there is no such solve or its plans were released.
 */
int hm_last_history(int n_load, int cap, double* err, double* sig);

/* Number of compiled tile-schedule variants of the x, y and z sweeps for a
 * grid and precision (all > 0 on success). */
int hm_schedule_count(const hm_grid* grid, hm_prec prec, int* nx, int* ny, int* nz);

/* Message of the calling thread's last failed call ("" if none). */
const char* hm_last_error(void);

/* Frees every cached plan, workspace and graph (device memory). */
void hm_release_plans(void);

/* 1 if the library can launch on the current device, else 0. */
int hm_device_ok(void);

#ifdef __cplusplus
}
#endif

#endif /* HM_H */
