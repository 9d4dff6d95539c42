// C ABI of the library (declared in include/hm.h): argument checks, plans
// (per precision, grid and load count: workspace, twiddles, launch
// arguments, captured graphs) and the host side of the fixed-point loop.
//
// The loop launches xsweep, ysweep(forward), zsweep and ysweep(inverse) per
// iteration; the inverse y-sweep decides on the device whether a load case
// stops (Section 2 setup: stress-equilibrium criterion), and the sweeps of a
// stopped load case return at once, so the host only polls the stop flags
// every `check_every` iterations and the iteration counts are exact.
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdarg.h>
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <chrono>
#include <map>
#include <mutex>
#include <string>
#include <tuple>
#include <vector>

#include "../../include/hm.h"
#include "hm_common.hpp"
#include "hm_adjoint.hpp"
#include "hm_filter.hpp"
#include "hm_aniso_kernels.hpp"
#include "hm_conduct_kernels.hpp"
#include "hm_extrapolate.hpp"
#include "hm_solve_kernels.hpp"

namespace hm {

const AxisKernels* axis_kernels_f64_g0(int n);
const AxisKernels* axis_kernels_f64_g1(int n);
const AxisKernels* axis_kernels_f64_g2(int n);
const AxisKernels* axis_kernels_f64_g3(int n);
const AxisKernels* axis_kernels_f32_g0(int n);
const AxisKernels* axis_kernels_f32_g1(int n);
const AxisKernels* axis_kernels_f32_g2(int n);
const AxisKernels* axis_kernels_f32_g3(int n);
const AxisKernels* axis_kernels_f64_g4(int n);
const AxisKernels* axis_kernels_f32_g4(int n);

const AxisKernels* axis_kernels(bool fp64, int n) {
  const AxisKernels* k = nullptr;
  if (fp64) {
    if (!k) k = axis_kernels_f64_g0(n);
    if (!k) k = axis_kernels_f64_g1(n);
    if (!k) k = axis_kernels_f64_g2(n);
    if (!k) k = axis_kernels_f64_g3(n);
    if (!k) k = axis_kernels_f64_g4(n);
  } else {
    if (!k) k = axis_kernels_f32_g0(n);
    if (!k) k = axis_kernels_f32_g1(n);
    if (!k) k = axis_kernels_f32_g2(n);
    if (!k) k = axis_kernels_f32_g3(n);
    if (!k) k = axis_kernels_f32_g4(n);
  }
  return k;
}

const CondKernels* cond_kernels_f64_g0(int n);
const CondKernels* cond_kernels_f64_g1(int n);
const CondKernels* cond_kernels_f32_g0(int n);
const CondKernels* cond_kernels_f32_g1(int n);

const AnisoKernels* aniso_kernels_f64_g0(int n);
const AnisoKernels* aniso_kernels_f64_g1(int n);
const AnisoKernels* aniso_kernels_f32_g0(int n);
const AnisoKernels* aniso_kernels_f32_g1(int n);

const AnisoKernels* aniso_kernels(bool fp64, int n) {
  const AnisoKernels* k = fp64 ? aniso_kernels_f64_g0(n) : aniso_kernels_f32_g0(n);
  if (!k) k = fp64 ? aniso_kernels_f64_g1(n) : aniso_kernels_f32_g1(n);
  return k;
}

const CondKernels* cond_kernels(bool fp64, int n) {
  const CondKernels* k = fp64 ? cond_kernels_f64_g0(n) : cond_kernels_f32_g0(n);
  if (!k) k = fp64 ? cond_kernels_f64_g1(n) : cond_kernels_f32_g1(n);
  return k;
}

}  // namespace hm

using namespace hm;

namespace {

thread_local std::string g_last_error;
thread_local hm_timing g_last_timing;
thread_local bool g_have_timing = false;

// Generation of the plan cache, bumped by hm_release_plans, so that the
// record of a thread's last solve (hm_last_history) can tell that the plan
// it points to was freed.
unsigned g_plan_generation = 1;

int fail(int code, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  g_last_error = buf;
  return code;
}

#define HM_HIP(expr)                                                                         \
  do {                                                                                       \
    hipError_t e_ = (expr);                                                                  \
    if (e_ != hipSuccess) return fail(HM_E_DEVICE, "%s: %s", #expr, hipGetErrorString(e_)); \
  } while (0)

constexpr int kMaxLoads = 4096;  // load cases per grid group (the y-sweep grid has 6 per load)

// Line lengths with compiled transforms: the products of 3, 5 and 7 up to
// 243, and those with a factor 11 or 13 up to 121 (solver kernels of both
// precisions exist for exactly these).
bool supported_length(int n) {
  if (n < 1 || n > 243) return false;
  return axis_kernels(true, n) != nullptr && axis_kernels(false, n) != nullptr;
}

int check_grid(const hm_grid* g) {
  if (!g) return fail(HM_E_ARG, "grid is NULL");
  if (g->dim != 2 && g->dim != 3) return fail(HM_E_ARG, "dim must be 2 or 3 (got %d)", g->dim);
  for (int d = 0; d < 3; ++d) {
    if (g->n[d] < 1) return fail(HM_E_ARG, "n[%d] = %d must be positive", d, g->n[d]);
    if (g->n[d] % 2 == 0) return fail(HM_E_SIZE, "n[%d] = %d must be odd", d, g->n[d]);
    if (!supported_length(g->n[d]))
      return fail(HM_E_SIZE,
                  "n[%d] = %d has no compiled transform (products of 3, 5, 7 up to 243; with a factor 11 or 13 "
                  "up to 121)",
                  d, g->n[d]);
  }
  if (g->dim == 2 && g->n[2] != 1) return fail(HM_E_ARG, "2D grids need n[2] == 1");
  if (g->dim == 3 && (g->n[0] < 3 || g->n[1] < 3 || g->n[2] < 3))
    return fail(HM_E_SIZE, "3D grids need at least 3 voxels per axis");
  if (g->dim == 2 && (g->n[0] < 3 || g->n[1] < 3)) return fail(HM_E_SIZE, "2D grids need at least 3x3 voxels");
  return HM_OK;
}

int check_spheres(const hm_grid* g, const hm_sphere* s, int ns) {
  if (ns < 0) return fail(HM_E_ARG, "n_spheres < 0");
  if (ns > 0 && !s) return fail(HM_E_ARG, "spheres is NULL");
  const int axes = g->dim == 2 ? 2 : 3;
  for (int k = 0; k < ns; ++k) {
    if (!(s[k].r > 0.0) || !isfinite(s[k].r)) return fail(HM_E_ARG, "sphere %d: radius must be > 0", k);
    for (int a = 0; a < axes; ++a)
      if (!(s[k].c[a] >= 0.0 && s[k].c[a] < (double)g->n[a]))
        return fail(HM_E_ARG, "sphere %d: centre coordinate %d outside [0, n)", k, a);
  }
  return HM_OK;
}

int check_phases(const hm_iso* ph) {
  if (!ph) return fail(HM_E_ARG, "phases is NULL");
  for (int p = 0; p < 2; ++p) {
    if (!isfinite(ph[p].lambda) || !isfinite(ph[p].mu) || !(ph[p].mu > 0.0) ||
        !(3.0 * ph[p].lambda + 2.0 * ph[p].mu > 0.0))
      return fail(HM_E_ARG, "phase %d: needs mu > 0 and 3 lambda + 2 mu > 0", p);
  }
  return HM_OK;
}

int check_opts(const hm_solve_opts* o) {
  if (!o) return fail(HM_E_ARG, "opts is NULL");
  if (o->prec != HM_FP64 && o->prec != HM_MIXED) return fail(HM_E_ARG, "unknown precision");
  if (!(o->tol >= 0.0)) return fail(HM_E_ARG, "tol must be >= 0");
  if (o->max_iter < 0) return fail(HM_E_ARG, "max_iter must be >= 0");
  if (!(o->c0_alpha > 0.0) || !isfinite(o->c0_alpha)) return fail(HM_E_ARG, "c0_alpha must be > 0");
  if (o->check_every < 1) return fail(HM_E_ARG, "check_every must be >= 1");
  if (o->stall_window < 0) return fail(HM_E_ARG, "stall_window must be >= 0");
  if (o->method != HM_FIXED_POINT && o->method != HM_CONJUGATE_GRADIENT) return fail(HM_E_ARG, "unknown method");
  if (o->method == HM_CONJUGATE_GRADIENT && o->profile)
    return fail(HM_E_ARG, "profiling times the fixed-point iteration only");
  return HM_OK;
}

// Twiddles exp(-2 pi i k / n) computed in long double, rounded once.
std::vector<double> twiddles(int n) {
  const long double pi = 3.141592653589793238462643383279502884L;
  std::vector<double> t(2 * (size_t)n);
  for (int k = 0; k < n; ++k) {
    const long double ang = -2.0L * pi * (long double)k / (long double)n;
    t[2 * k] = (double)cosl(ang);
    t[2 * k + 1] = (double)sinl(ang);
  }
  return t;
}

struct Plan;
void set_schedule(Plan* p, const XKern* X, const YKern* Y, const ZKern* Z);

struct Plan {
  bool fp64 = true;
  bool cond = false;   // conduction plan: 3 gradient components, conduction kernels
  bool aniso = false;  // anisotropic phases: general-row x-sweep, elastic y / z sweeps
  const AnisoKernels* ak = nullptr;
  int n[3] = {0, 0, 0};
  int n_load = 0;
  int device = 0;
  const AxisKernels* kx = nullptr;
  const AxisKernels* ky = nullptr;
  const AxisKernels* kz = nullptr;
  const CondKernels* ck[3] = {nullptr, nullptr, nullptr};  // conduction plans
  const XKern* X = nullptr;  // chosen schedules
  const YKern* Y = nullptr;
  const ZKern* Z = nullptr;
  bool tuned = false;
  void* spec = nullptr;
  void* hist = nullptr;
  double* taupart = nullptr;
  double* errpart = nullptr;
  int* fin_count = nullptr;  // [2 n_load]: end-of-iteration arrivals per load case (0
                             // between launches), then the stop-flag snapshots
  double* fin_red = nullptr; // reduced sums per load case, 8 doubles
  SolverState* state = nullptr;
  SolverState* state_host = nullptr;  // pinned
  double* errhist = nullptr;
  double* sighist = nullptr;
  int hist_cap = 0;
  char* prm = nullptr;       // parameter blob: SolveParams, loads, problems, spheres
  char* prm_host = nullptr;  // pinned staging of the blob
  size_t prm_cap = 0;
  int* mid = nullptr;        // material ids of the group's problems, back to back
  size_t mid_cap = 0;        // entries
  void* coef = nullptr;      // stiffness table rows (8 reals each)
  size_t coef_cap = 0;       // rows
  int* mcount = nullptr;     // [2]: rows handed out, data flags
  int* mcount_host = nullptr;
  void* cgv[3] = {nullptr, nullptr, nullptr};  // CG iterate x, residual r, direction p
  CgState* cgs = nullptr;
  double* cgpart = nullptr;
  int cg_blocks = 0;
  hipGraphExec_t cg_graph = nullptr;
  int cg_graph_k = 0;
  void* tw[3] = {nullptr, nullptr, nullptr};
  SolveArgs args;
  hipStream_t cap_stream = nullptr;
  hipGraphExec_t graph = nullptr;
  int graph_k = 0;
};

std::mutex g_mutex;
std::map<std::tuple<int, bool, int, int, int, int, int>, Plan*> g_plans;

void free_plan(Plan* p) {
  if (p->graph) (void)hipGraphExecDestroy(p->graph);
  if (p->cg_graph) (void)hipGraphExecDestroy(p->cg_graph);
  for (int v = 0; v < 3; ++v) (void)hipFree(p->cgv[v]);
  (void)hipFree(p->cgs);
  (void)hipFree(p->cgpart);
  if (p->cap_stream) (void)hipStreamDestroy(p->cap_stream);
  (void)hipFree(p->spec);
  (void)hipFree(p->hist);
  (void)hipFree(p->taupart);
  (void)hipFree(p->errpart);
  (void)hipFree(p->fin_count);
  (void)hipFree(p->fin_red);
  (void)hipFree(p->state);
  (void)hipFree(p->errhist);
  (void)hipFree(p->sighist);
  (void)hipFree(p->prm);
  (void)hipFree(p->mid);
  (void)hipFree(p->coef);
  (void)hipFree(p->mcount);
  if (p->mcount_host) (void)hipHostFree(p->mcount_host);
  for (int a = 0; a < 3; ++a) (void)hipFree(p->tw[a]);
  if (p->state_host) (void)hipHostFree(p->state_host);
  if (p->prm_host) (void)hipHostFree(p->prm_host);
  delete p;
}

// Captured graphs bake in the launch arguments: drop them when those change.
void drop_graphs(Plan* p) {
  if (p->graph) (void)hipGraphExecDestroy(p->graph);
  if (p->cg_graph) (void)hipGraphExecDestroy(p->cg_graph);
  p->graph = nullptr;
  p->cg_graph = nullptr;
}

int device_alloc(void** ptr, size_t bytes, const char* what) {
  hipError_t e = hipMalloc(ptr, bytes);
  if (e != hipSuccess) {
    *ptr = nullptr;
    (void)hipGetLastError();
    return fail(HM_E_NOMEM, "cannot allocate %zu bytes for %s: %s", bytes, what, hipGetErrorString(e));
  }
  return HM_OK;
}

int upload_twiddles(Plan* p, int axis, int n) {
  std::vector<double> t = twiddles(n);
  const size_t bytes = (size_t)n * (p->fp64 ? 16 : 8);
  int rc = device_alloc(&p->tw[axis], bytes, "twiddles");
  if (rc) return rc;
  if (p->fp64) {
    HM_HIP(hipMemcpy(p->tw[axis], t.data(), bytes, hipMemcpyHostToDevice));
  } else {
    std::vector<float> f(t.size());
    for (size_t i = 0; i < t.size(); ++i) f[i] = (float)t[i];
    HM_HIP(hipMemcpy(p->tw[axis], f.data(), bytes, hipMemcpyHostToDevice));
  }
  return HM_OK;
}

// Physics of a plan: elasticity with isotropic phases, conduction, or
// elasticity with anisotropic phases.
enum : int { PHYS_ELASTIC = 0, PHYS_CONDUCTION = 1, PHYS_ANISO = 2 };

int get_plan(bool fp64, const int n[3], int dim, int n_load, int phys, Plan** out) {
  const bool cond = phys == PHYS_CONDUCTION;
  int dev = 0;
  HM_HIP(hipGetDevice(&dev));
  std::lock_guard<std::mutex> lock(g_mutex);
  auto key = std::make_tuple(dev, fp64, phys, n[0], n[1], n[2], n_load);
  auto it = g_plans.find(key);
  if (it != g_plans.end()) {
    *out = it->second;
    return HM_OK;
  }
  Plan* p = new Plan();
  p->fp64 = fp64;
  p->device = dev;
  for (int d = 0; d < 3; ++d) p->n[d] = n[d];
  p->n_load = n_load;
  p->cond = cond;
  p->aniso = phys == PHYS_ANISO;
  bool have = true;
  if (cond) {
    for (int d = 0; d < 3; ++d) have = have && (p->ck[d] = cond_kernels(fp64, n[d])) != nullptr;
  } else {
    p->kx = axis_kernels(fp64, n[0]);
    p->ky = axis_kernels(fp64, n[1]);
    p->kz = axis_kernels(fp64, n[2]);
    have = p->kx && p->ky && p->kz;
    if (p->aniso) have = have && (p->ak = aniso_kernels(fp64, n[0])) != nullptr;
  }
  if (!have) {
    delete p;
    return fail(HM_E_SIZE, "no kernels compiled for grid %dx%dx%d", n[0], n[1], n[2]);
  }
  const int nc = cond ? 3 : 6;     // field components per load
  const int nh = cond ? 1 : 3;     // traction-history components per load
  const int H = (n[0] + 1) / 2;
  const size_t cplx = fp64 ? 16 : 8;
  const int row = (int)(128 / cplx);  // complex values per 128-byte line
  const int Hp = (H + row - 1) / row * row;
  const size_t plane = (size_t)n[2] * n[1] * Hp;
  // partial-sum buffers sized for the finest schedule of each kernel
  int min_lines = 1 << 30, min_zw = 1 << 30;
  if (cond) {
    min_lines = p->ck[0]->x.lines;
    min_zw = p->ck[2]->z.width;
  } else {
    for (int v = 0; v < p->kx->nxv; ++v) min_lines = std::min(min_lines, p->kx->x[v].lines);
    for (int v = 0; v < p->kz->nzv; ++v) min_zw = std::min(min_zw, p->kz->z[v].width);
  }
  const int g2 = (n[1] * n[2] + min_lines - 1) / min_lines;
  const int ntx4 = (H + min_zw - 1) / min_zw;
  int rc = HM_OK;
  if (!rc) rc = device_alloc(&p->spec, (size_t)n_load * nc * plane * cplx, "spectrum");
  if (!rc) rc = device_alloc(&p->hist, (size_t)n_load * nh * plane * cplx, "traction history");
  if (!rc) rc = device_alloc((void**)&p->taupart, (size_t)n_load * g2 * 6 * sizeof(double), "tau partials");
  if (!rc) rc = device_alloc((void**)&p->errpart, (size_t)n_load * n[1] * ntx4 * sizeof(double), "error partials");
  if (!rc) rc = device_alloc((void**)&p->state, (size_t)n_load * sizeof(SolverState), "state");
  if (!rc) rc = device_alloc((void**)&p->fin_count, (size_t)n_load * 2 * sizeof(int), "iteration counters");
  if (!rc) rc = device_alloc((void**)&p->fin_red, (size_t)n_load * 8 * sizeof(double), "reduced sums");
  if (!rc && hipMemset(p->fin_count, 0, (size_t)n_load * 2 * sizeof(int)) != hipSuccess)
    rc = fail(HM_E_DEVICE, "clearing the iteration counters");
  if (!rc) rc = upload_twiddles(p, 0, n[0]);
  if (!rc) rc = upload_twiddles(p, 1, n[1]);
  if (!rc) rc = upload_twiddles(p, 2, n[2]);
  if (!rc && hipHostMalloc((void**)&p->state_host, (size_t)n_load * sizeof(SolverState), 0) != hipSuccess)
    rc = fail(HM_E_NOMEM, "pinned state buffer");
  if (rc) {
    free_plan(p);
    return rc;
  }
  SolveArgs& a = p->args;
  memset(&a, 0, sizeof a);
  a.spec = p->spec;
  a.spec_in = p->spec;
  a.hist = p->hist;
  a.taupart = p->taupart;
  a.errpart = p->errpart;
  a.state = p->state;
  a.fin_count = p->fin_count;
  a.fin_red = p->fin_red;
  a.done_snap = p->fin_count + n_load;
  a.twx = p->tw[0];
  a.twy = p->tw[1];
  a.twz = p->tw[2];
  a.nx = n[0];
  a.ny = n[1];
  a.nz = n[2];
  a.H = H;
  a.Hp = Hp;
  a.dim = dim;
  a.n_load = n_load;
  a.cond = cond ? 1 : 0;

  if (cond)
    set_schedule(p, &p->ck[0]->x, &p->ck[1]->y, &p->ck[2]->z);
  else if (p->aniso)
    set_schedule(p, &p->ak->x, &p->ky->y[0], &p->kz->z[0]);
  else
    set_schedule(p, &p->kx->x[0], &p->ky->y[0], &p->kz->z[0]);
  g_plans[key] = p;
  *out = p;
  return HM_OK;
}

void set_schedule(Plan* p, const XKern* X, const YKern* Y, const ZKern* Z) {
  p->X = X;
  p->Y = Y;
  p->Z = Z;
  SolveArgs& a = p->args;
  a.g2 = (a.ny * a.nz + X->lines - 1) / X->lines;
  a.ntx3 = (a.H + Y->width - 1) / Y->width;
  a.ntx4 = (a.H + Z->width - 1) / Z->width;
  drop_graphs(p);
}

int ensure_hist(Plan* p, int cap) {
  if (p->hist_cap >= cap) return HM_OK;
  if (p->errhist) (void)hipFree(p->errhist);
  if (p->sighist) (void)hipFree(p->sighist);
  p->errhist = nullptr;
  p->sighist = nullptr;
  p->hist_cap = 0;
  p->args.errhist = nullptr;
  p->args.sighist = nullptr;
  p->args.hist_cap = 0;
  int rc = device_alloc((void**)&p->errhist, (size_t)p->n_load * cap * sizeof(double), "error history");
  if (!rc) rc = device_alloc((void**)&p->sighist, (size_t)p->n_load * cap * 6 * sizeof(double), "stress history");
  if (rc) return rc;
  p->hist_cap = cap;
  p->args.errhist = p->errhist;
  p->args.sighist = p->sighist;
  p->args.hist_cap = cap;
  drop_graphs(p);
  return HM_OK;
}

hipError_t launch_iteration(Plan* p, const SolveArgs& a, bool first, hipStream_t s) {
  hipError_t e;
  if ((e = (first ? p->X->first : p->X->iter)(a, s)) != hipSuccess) return e;
  if ((e = p->Y->fwd(a, s)) != hipSuccess) return e;
  if ((e = p->Z->run(a, s)) != hipSuccess) return e;
  // the inverse y-sweep also ends the iteration (stop decision per load case)
  return p->Y->inv(a, s);
}

// Copies the stop flags of the plan's load cases to the host (stream synchronised).
int poll_done(Plan* p, hipStream_t s, bool* all_done) {
  HM_HIP(hipMemcpyAsync(p->state_host, p->state, (size_t)p->n_load * sizeof(SolverState), hipMemcpyDeviceToHost, s));
  HM_HIP(hipStreamSynchronize(s));
  bool d = true;
  for (int l = 0; l < p->n_load; ++l) d = d && p->state_host[l].done;
  *all_done = d;
  return HM_OK;
}

// Captures k iterations of each listed plan (in order) into an executable graph.
int capture_graph(std::vector<Plan*>& plans, int k, hipStream_t cap, hipGraphExec_t* out) {
  hipGraph_t g = nullptr;
  HM_HIP(hipStreamBeginCapture(cap, hipStreamCaptureModeThreadLocal));
  hipError_t le = hipSuccess;
  for (int i = 0; i < k && le == hipSuccess; ++i)
    for (Plan* p : plans) {
      SolveArgs a = p->args;
      a.first = 0;
      if (le == hipSuccess) le = launch_iteration(p, a, false, cap);
    }
  hipError_t ce = hipStreamEndCapture(cap, &g);
  if (le != hipSuccess || ce != hipSuccess) {
    if (g) (void)hipGraphDestroy(g);
    return fail(HM_E_DEVICE, "graph capture failed: %s", hipGetErrorString(le != hipSuccess ? le : ce));
  }
  hipError_t ie = hipGraphInstantiate(out, g, nullptr, nullptr, 0);
  (void)hipGraphDestroy(g);
  if (ie != hipSuccess) {
    *out = nullptr;
    return fail(HM_E_DEVICE, "graph instantiation failed: %s", hipGetErrorString(ie));
  }
  return HM_OK;
}

int build_graph(Plan* p, int k) {
  if (p->graph && p->graph_k == k) return HM_OK;
  if (p->graph) {
    (void)hipGraphExecDestroy(p->graph);
    p->graph = nullptr;
  }
  if (!p->cap_stream) HM_HIP(hipStreamCreateWithFlags(&p->cap_stream, hipStreamNonBlocking));
  std::vector<Plan*> one{p};
  int rc = capture_graph(one, k, p->cap_stream, &p->graph);
  if (rc) return rc;
  p->graph_k = k;
  return HM_OK;
}

// Times every compiled schedule of the three sweeps on this plan's own
// workspace (iteration mode, all load cases active) and keeps the fastest.
// Runs once per plan, before the first solve; the workspace is zeroed first
// and the solver state is reset by the caller afterwards.  An anisotropic
// plan has one x-sweep (the general-row one); its y- and z-sweeps are the
// elastic ones and are chosen the same way.
int tune_plan(Plan* p, hipStream_t s) {
  hipEvent_t e0, e1;
  HM_HIP(hipEventCreate(&e0));
  HM_HIP(hipEventCreate(&e1));
  const size_t cplx = p->fp64 ? 16 : 8;
  const size_t plane = (size_t)p->n[2] * p->n[1] * p->args.Hp;
  hipError_t err = hipMemsetAsync(p->spec, 0, (size_t)p->n_load * 6 * plane * cplx, s);
  if (err == hipSuccess) err = hipMemsetAsync(p->hist, 0, (size_t)p->n_load * 3 * plane * cplx, s);
  hipLaunchKernelGGL((k_reset_state<64>), dim3((p->n_load + 63) / 64), dim3(64), 0, s, p->state, p->n_load);
  if (err == hipSuccess) err = hipGetLastError();
  // two warm-up launches, then the fastest of three rounds of three launches
  // (single launches of a few hundred microseconds vary by several percent
  // from one to the next, which made a one-round choice change run to run)
  auto time_it = [&](solve_launch_fn f, const SolveArgs& a, float* best) -> hipError_t {
    hipError_t e = f(a, s);
    if (e == hipSuccess) e = f(a, s);
    float bestms = 1e30f;
    for (int round = 0; round < 3 && e == hipSuccess; ++round) {
      e = hipEventRecord(e0, s);
      for (int r = 0; r < 3 && e == hipSuccess; ++r) e = f(a, s);
      if (e == hipSuccess) e = hipEventRecord(e1, s);
      if (e == hipSuccess) e = hipEventSynchronize(e1);
      float ms = 0.0f;
      if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
      bestms = std::min(bestms, ms);
    }
    *best = bestms;
    return e;
  };
  const XKern* bx = p->aniso ? &p->ak->x : &p->kx->x[0];
  const YKern* by = &p->ky->y[0];
  const ZKern* bz = &p->kz->z[0];
  float tbest = 1e30f, t = 0.0f;
  for (int v = 0; v < (p->aniso ? 0 : p->kx->nxv) && err == hipSuccess; ++v) {
    set_schedule(p, &p->kx->x[v], by, bz);
    SolveArgs a = p->args;
    a.first = 0;
    err = time_it(p->kx->x[v].iter, a, &t);
    if (t < tbest) {
      tbest = t;
      bx = &p->kx->x[v];
    }
  }
  tbest = 1e30f;
  for (int v = 0; v < p->ky->nyv && err == hipSuccess; ++v) {
    set_schedule(p, bx, &p->ky->y[v], bz);
    SolveArgs a = p->args;
    err = time_it(p->ky->y[v].fwd, a, &t);
    if (t < tbest) {
      tbest = t;
      by = &p->ky->y[v];
    }
  }
  tbest = 1e30f;
  for (int v = 0; v < p->kz->nzv && err == hipSuccess; ++v) {
    set_schedule(p, bx, by, &p->kz->z[v]);
    SolveArgs a = p->args;
    a.first = 0;
    err = time_it(p->kz->z[v].run, a, &t);
    if (t < tbest) {
      tbest = t;
      bz = &p->kz->z[v];
    }
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (err != hipSuccess) return fail(HM_E_DEVICE, "autotune: %s", hipGetErrorString(err));
  set_schedule(p, bx, by, bz);
  p->tuned = true;
  return HM_OK;
}

// One problem (cell) of a solve, as given by the caller.
struct ProblemIn {
  hm_grid grid;
  hm_iso phases[2];
  int cond;      // conduction problem: phase conductivities in k, phases unused
  double k[2];
  int nphase;    // multi-phase cell (>= 2): phases in ph, fractions [nphase - 1][N]
  hm_iso ph[8];
  int aniso;     // anisotropic phases: Mandel matrices in cm, phases unused
  double cm[2][36];
  hm_rule rule;
  const void* frac;
  const int32_t* incl;
  const hm_sphere* sph;
  int nsph;
};

// The load cases of one or more problems sharing a grid, solved together.
struct Group {
  Plan* p = nullptr;
  std::vector<int> probs;         // indices into the problem list
  std::vector<LoadParams> loads;  // LoadParams::prob indexes `probs`
  void* eps_out = nullptr;        // export target (nullable)
  bool active = true;
};

// Extreme eigenvalues of a symmetric 6x6 matrix (cyclic Jacobi rotations).
void sym6_eig_range(const double* M, double* lo, double* hi) {
  double a[6][6];
  for (int i = 0; i < 6; ++i)
    for (int j = 0; j < 6; ++j) a[i][j] = 0.5 * (M[i * 6 + j] + M[j * 6 + i]);
  for (int sweep = 0; sweep < 60; ++sweep) {
    double off = 0.0;
    for (int i = 0; i < 6; ++i)
      for (int j = i + 1; j < 6; ++j) off += a[i][j] * a[i][j];
    if (off < 1e-30) break;
    for (int p = 0; p < 6; ++p)
      for (int q = p + 1; q < 6; ++q) {
        if (a[p][q] == 0.0) continue;
        const double th = 0.5 * (a[q][q] - a[p][p]) / a[p][q];
        const double t = (th >= 0 ? 1.0 : -1.0) / (fabs(th) + sqrt(th * th + 1.0));
        const double c = 1.0 / sqrt(t * t + 1.0), sn = t * c;
        for (int k = 0; k < 6; ++k) {  // columns p, q
          const double akp = a[k][p], akq = a[k][q];
          a[k][p] = c * akp - sn * akq;
          a[k][q] = sn * akp + c * akq;
        }
        for (int k = 0; k < 6; ++k) {  // rows p, q
          const double apk = a[p][k], aqk = a[q][k];
          a[p][k] = c * apk - sn * aqk;
          a[q][k] = sn * apk + c * aqk;
        }
      }
  }
  *lo = a[0][0];
  *hi = a[0][0];
  for (int i = 1; i < 6; ++i) {
    *lo = fmin(*lo, a[i][i]);
    *hi = fmax(*hi, a[i][i]);
  }
}

// Symmetric (to 1e-12 relative) and positive definite (Cholesky succeeds).
bool spd6(const double* M) {
  double scale = 0.0;
  for (int i = 0; i < 36; ++i) {
    if (!isfinite(M[i])) return false;
    scale = fmax(scale, fabs(M[i]));
  }
  for (int i = 0; i < 6; ++i)
    for (int j = 0; j < i; ++j)
      if (fabs(M[i * 6 + j] - M[j * 6 + i]) > 1e-12 * scale) return false;
  double L[36] = {};
  for (int j = 0; j < 6; ++j) {
    double d = M[j * 6 + j];
    for (int k = 0; k < j; ++k) d -= L[j * 6 + k] * L[j * 6 + k];
    if (!(d > 0.0)) return false;
    L[j * 6 + j] = sqrt(d);
    for (int i = j + 1; i < 6; ++i) {
      double v = M[i * 6 + j];
      for (int k = 0; k < j; ++k) v -= L[i * 6 + k] * L[j * 6 + k];
      L[i * 6 + j] = v / L[j * 6 + j];
    }
  }
  return true;
}

int check_problem(const ProblemIn& d) {
  int rc;
  if ((rc = check_grid(&d.grid))) return rc;
  if (d.cond) {
    for (int p = 0; p < 2; ++p)
      if (!(d.k[p] > 0.0) || !isfinite(d.k[p])) return fail(HM_E_ARG, "conductivity %d must be finite and > 0", p);
  } else if (d.nphase) {
    if (d.nphase < 2 || d.nphase > 8) return fail(HM_E_ARG, "n_phases must be in 2..8");
    for (int p = 0; p < d.nphase; p += 2) {
      hm_iso two[2] = {d.ph[p], d.ph[p + 1 < d.nphase ? p + 1 : p]};
      if ((rc = check_phases(two))) return rc;
    }
    if (d.rule == HM_RULE_LAMINATE) return fail(HM_E_ARG, "the 2-layer rule is written for two phases");
  } else if (d.aniso) {
    for (int p = 0; p < 2; ++p)
      if (!spd6(d.cm[p])) return fail(HM_E_ARG, "phase %d: the Mandel matrix must be symmetric positive definite", p);
  } else if ((rc = check_phases(d.phases))) {
    return rc;
  }
  if ((rc = check_spheres(&d.grid, d.sph, d.nsph))) return rc;
  if (d.rule < HM_RULE_NONE || d.rule > HM_RULE_LAMINATE) return fail(HM_E_ARG, "unknown rule %d", (int)d.rule);
  if (!d.frac) return fail(HM_E_ARG, "d_frac is NULL");
  if (d.rule == HM_RULE_LAMINATE && !d.incl) return fail(HM_E_ARG, "the 2-layer rule needs d_incl");
  return HM_OK;
}

size_t align16(size_t v) { return (v + 15) / 16 * 16; }

// Writes the group's parameter blob (header, loads, problems, sphere tables)
// to pinned staging and queues its copy to the plan's device buffer.
int upload_params(Group& g, const std::vector<ProblemIn>& all, const hm_solve_opts* opts, hipStream_t s) {
  Plan* p = g.p;
  const int nl = (int)g.loads.size(), np = (int)g.probs.size();
  size_t nsph_tot = 0;
  for (int q : g.probs) nsph_tot += (size_t)all[q].nsph;
  const size_t o_loads = align16(sizeof(SolveParams));
  const size_t o_probs = align16(o_loads + nl * sizeof(LoadParams));
  const size_t o_sph = align16(o_probs + np * sizeof(ProblemParams));
  const size_t bytes = o_sph + nsph_tot * 4 * sizeof(double) + 16;
  if (bytes > p->prm_cap) {
    (void)hipFree(p->prm);
    if (p->prm_host) (void)hipHostFree(p->prm_host);
    p->prm = nullptr;
    p->prm_host = nullptr;
    p->prm_cap = 0;
    const size_t cap = std::max(bytes, (size_t)4096);
    int rc = device_alloc((void**)&p->prm, cap, "parameters");
    if (rc) return rc;
    if (hipHostMalloc((void**)&p->prm_host, cap, 0) != hipSuccess) return fail(HM_E_NOMEM, "pinned parameters");
    p->prm_cap = cap;
    p->args.prm = reinterpret_cast<const SolveParams*>(p->prm);
    drop_graphs(p);
  }
  size_t nmid = 0;
  for (int q : g.probs) nmid += (size_t)all[q].grid.n[0] * all[q].grid.n[1] * all[q].grid.n[2];
  if (nmid > p->mid_cap) {
    (void)hipFree(p->mid);
    p->mid = nullptr;
    p->mid_cap = 0;
    int rc = device_alloc((void**)&p->mid, nmid * sizeof(int), "material ids");
    if (rc) return rc;
    p->mid_cap = nmid;
  }
  if (!p->coef) {
    const size_t rows = std::max<size_t>(4096, nmid / 16);
    int rc = device_alloc(&p->coef, rows * 8 * (p->fp64 ? 8 : 4), "stiffness table");
    if (rc) return rc;
    p->coef_cap = rows;
  }
  char* h = p->prm_host;
  memset(h, 0, bytes);
  SolveParams* S = reinterpret_cast<SolveParams*>(h);
  S->tol = opts->tol;
  S->max_iter = opts->max_iter;
  S->stall_window = opts->stall_window;
  S->n_load = nl;
  S->n_prob = np;
  S->loads = reinterpret_cast<const LoadParams*>(p->prm + o_loads);
  S->probs = reinterpret_cast<const ProblemParams*>(p->prm + o_probs);
  memcpy(h + o_loads, g.loads.data(), nl * sizeof(LoadParams));
  ProblemParams* PP = reinterpret_cast<ProblemParams*>(h + o_probs);
  double* sph = reinterpret_cast<double*>(h + o_sph);
  size_t so = 0, mo = 0;
  for (int j = 0; j < np; ++j) {
    const ProblemIn& d = all[g.probs[j]];
    ProblemParams& q = PP[j];
    if (d.aniso) {
      // reference c0 = 2 mu0 I with 2 mu0 = alpha (m + M) / 2 over the phases'
      // Mandel eigenvalues (so c - c0 stays within (-c0, c0))
      double lo = 0.0, hi = 0.0, l1 = 0.0, h1 = 0.0;
      sym6_eig_range(d.cm[0], &lo, &hi);
      sym6_eig_range(d.cm[1], &l1, &h1);
      lo = fmin(lo, l1);
      hi = fmax(hi, h1);
      q.gen = 1;
      q.rl = 0.0;
      q.rm = opts->c0_alpha * 0.25 * (lo + hi);
      if (opts->method == HM_CONJUGATE_GRADIENT) q.rm = 0.5;
      for (int ph = 0; ph < 2; ++ph)
        for (int i = 0; i < 36; ++i) q.cm[ph][i] = d.cm[ph][i];
    } else if (d.cond) {
      // conductivities in pl, k0 = alpha * mean of the smallest and largest
      q.pl[0] = d.k[0];
      q.pl[1] = d.k[1];
      q.rl = opts->c0_alpha * 0.5 * (fmin(d.k[0], d.k[1]) + fmax(d.k[0], d.k[1]));
      for (int ph = 0; ph < 2; ++ph) {
        q.pure_f[2 * ph] = (float)d.k[ph] - (float)q.rl;
        q.pure_d[2 * ph] = d.k[ph] - q.rl;
      }
    } else {
      for (int ph = 0; ph < 2; ++ph) {
        q.pl[ph] = d.nphase ? d.ph[ph].lambda : d.phases[ph].lambda;
        q.pm[ph] = d.nphase ? d.ph[ph].mu : d.phases[ph].mu;
      }
      double lmin = fmin(q.pl[0], q.pl[1]), lmax = fmax(q.pl[0], q.pl[1]);
      double mmin = fmin(q.pm[0], q.pm[1]), mmax = fmax(q.pm[0], q.pm[1]);
      q.nphase = d.nphase;
      for (int ph = 0; ph < d.nphase; ++ph) {
        q.ph_l[ph] = d.ph[ph].lambda;
        q.ph_m[ph] = d.ph[ph].mu;
        lmin = fmin(lmin, q.ph_l[ph]);
        lmax = fmax(lmax, q.ph_l[ph]);
        mmin = fmin(mmin, q.ph_m[ph]);
        mmax = fmax(mmax, q.ph_m[ph]);
      }
      q.rl = opts->c0_alpha * 0.5 * (lmin + lmax);
      q.rm = opts->c0_alpha * 0.5 * (mmin + mmax);
      if (opts->method == HM_CONJUGATE_GRADIENT) {
        // c0 = identity on symmetric tensors: Gamma0 becomes the projection G
        q.rl = 0.0;
        q.rm = 0.5;
      }
      if (!(q.rm > 0.0) || !(q.rl + 2.0 * q.rm > 0.0)) return fail(HM_E_ARG, "reference medium is not positive");
      for (int ph = 0; ph < 2; ++ph) {
        // the rounding of T(lambda) - T(lambda0) and T(2 mu) - T(2 mu0) in T
        q.pure_f[2 * ph] = (float)q.pl[ph] - (float)q.rl;
        q.pure_f[2 * ph + 1] = (float)(2.0 * q.pm[ph]) - (float)(2.0 * q.rm);
        q.pure_d[2 * ph] = q.pl[ph] - q.rl;
        q.pure_d[2 * ph + 1] = 2.0 * q.pm[ph] - 2.0 * q.rm;
      }
    }
    q.rule = (int)d.rule;
    q.nsph = d.nsph;
    q.frac = d.frac;
    q.incl = d.incl;
    q.mid = p->mid + mo;
    q.coef = p->coef;
    mo += (size_t)d.grid.n[0] * d.grid.n[1] * d.grid.n[2];
    q.sph = reinterpret_cast<const double*>(p->prm + o_sph) + so;
    for (int k = 0; k < d.nsph; ++k) {
      for (int c = 0; c < 3; ++c) sph[so + 4 * k + c] = d.sph[k].c[c];
      sph[so + 4 * k + 3] = d.sph[k].r;
    }
    so += 4 * (size_t)d.nsph;
  }
  HM_HIP(hipMemcpyAsync(p->prm, p->prm_host, bytes, hipMemcpyHostToDevice, s));
  return HM_OK;
}

int data_flags_error(int flags) {
  if (flags & FLAG_NONE_FRACTIONAL) return fail(HM_E_DATA, "fractional voxel with HM_RULE_NONE");
  if (flags & FLAG_BAD_INCL) return fail(HM_E_DATA, "d_incl holds a sphere index >= n_spheres");
  return HM_OK;
}

// Builds the group's material table (ids and stiffness rows of the
// fractional voxels, k_material) on the stream, after its parameters were
// queued by upload_params; grows the row table and rebuilds once if it was
// too small.  Fails with HM_E_DATA on inconsistent input, before any
// iteration runs.
int prepare_material(Group& g, const std::vector<ProblemIn>& all, const hm_solve_opts* opts, hipStream_t s) {
  Plan* p = g.p;
  int rc;
  if (!p->mcount) {
    if ((rc = device_alloc((void**)&p->mcount, 2 * sizeof(int), "material counter"))) return rc;
    if (hipHostMalloc((void**)&p->mcount_host, 2 * sizeof(int), 0) != hipSuccess)
      return fail(HM_E_NOMEM, "pinned material counter");
  }
  for (int attempt = 0; attempt < 2; ++attempt) {
    HM_HIP(hipMemsetAsync(p->mcount, 0, 2 * sizeof(int), s));
    // a multi-phase cell (solved alone) keeps its pure phases 2.. in the
    // first rows of the table
    const ProblemIn& d0 = all[g.probs[0]];
    if (d0.aniso) {
      // pure phases in rows 0 and 1: upper triangles of M_p - c0
      if (g.probs.size() != 1) return fail(HM_E_ARG, "anisotropic cells are solved one at a time");
      const ProblemParams* hq = reinterpret_cast<const ProblemParams*>(
          p->prm_host + align16(align16(sizeof(SolveParams)) + g.loads.size() * sizeof(LoadParams)));
      std::vector<double> rd(2 * kGenRow, 0.0);
      std::vector<float> rf(2 * kGenRow, 0.0f);
      for (int ph = 0; ph < 2; ++ph) {
        int o = 0;
        for (int I = 0; I < 6; ++I)
          for (int J = I; J < 6; ++J) {
            double v = 0.5 * (hq->cm[ph][I * 6 + J] + hq->cm[ph][J * 6 + I]);
            if (I < 3 && J < 3) v -= hq->rl;
            if (I == J) v -= 2.0 * hq->rm;
            rd[ph * kGenRow + o] = v;
            rf[ph * kGenRow + o] = (float)v;
            ++o;
          }
      }
      p->mcount_host[0] = 2;
      p->mcount_host[1] = 0;
      HM_HIP(hipMemcpyAsync(p->coef, p->fp64 ? (const void*)rd.data() : (const void*)rf.data(),
                            (size_t)2 * kGenRow * (p->fp64 ? 8 : 4), hipMemcpyHostToDevice, s));
      HM_HIP(hipMemcpyAsync(p->mcount, p->mcount_host, 2 * sizeof(int), hipMemcpyHostToDevice, s));
      HM_HIP(hipStreamSynchronize(s));
    }
    if (d0.nphase > 2) {
      if (g.probs.size() != 1) return fail(HM_E_ARG, "multi-phase cells are solved one at a time");
      const int nr = d0.nphase - 2;
      if ((size_t)nr > p->coef_cap) return fail(HM_E_DEVICE, "material table too small");
      const ProblemParams* hq = reinterpret_cast<const ProblemParams*>(
          p->prm_host + align16(align16(sizeof(SolveParams)) + g.loads.size() * sizeof(LoadParams)));
      std::vector<double> rd((size_t)nr * 8, 0.0);
      std::vector<float> rf((size_t)nr * 8, 0.0f);
      for (int r = 0; r < nr; ++r) {
        const double l = hq->ph_l[r + 2], m2 = 2.0 * hq->ph_m[r + 2];
        rd[8 * r] = l - hq->rl;
        rd[8 * r + 1] = m2 - 2.0 * hq->rm;
        rf[8 * r] = (float)l - (float)hq->rl;
        rf[8 * r + 1] = (float)m2 - (float)(2.0 * hq->rm);
      }
      p->mcount_host[0] = nr;
      p->mcount_host[1] = 0;
      HM_HIP(hipMemcpyAsync(p->coef, p->fp64 ? (const void*)rd.data() : (const void*)rf.data(),
                            (size_t)nr * 8 * (p->fp64 ? 8 : 4), hipMemcpyHostToDevice, s));
      HM_HIP(hipMemcpyAsync(p->mcount, p->mcount_host, 2 * sizeof(int), hipMemcpyHostToDevice, s));
      HM_HIP(hipStreamSynchronize(s));  // the host vectors go out of scope
    }
    size_t mo = 0;
    for (int j = 0; j < (int)g.probs.size(); ++j) {
      const hm_grid& gr = all[g.probs[j]].grid;
      const int N = gr.n[0] * gr.n[1] * gr.n[2];
      const SolveParams* prm = reinterpret_cast<const SolveParams*>(p->prm);
      const size_t rw = p->aniso ? kGenRow / 8 : 1;  // row width in units of 8 reals
      const int cap = (int)std::min<size_t>(p->coef_cap / rw, (size_t)1 << 30);
      const dim3 grid((N + 255) / 256), blk(256);
      if (p->aniso && p->fp64)
        hipLaunchKernelGGL((k_material_aniso<double>), grid, blk, 0, s, prm, j, gr.n[0], gr.n[1], gr.n[2], gr.dim,
                           p->mid + mo, static_cast<double*>(p->coef), cap, p->mcount);
      else if (p->aniso)
        hipLaunchKernelGGL((k_material_aniso<float>), grid, blk, 0, s, prm, j, gr.n[0], gr.n[1], gr.n[2], gr.dim,
                           p->mid + mo, static_cast<float*>(p->coef), cap, p->mcount);
      else if (all[g.probs[j]].nphase && p->fp64)
        hipLaunchKernelGGL((k_material_nphase<double>), grid, blk, 0, s, prm, j, gr.n[0], gr.n[1], gr.n[2],
                           p->mid + mo, static_cast<double*>(p->coef), cap, p->mcount);
      else if (all[g.probs[j]].nphase)
        hipLaunchKernelGGL((k_material_nphase<float>), grid, blk, 0, s, prm, j, gr.n[0], gr.n[1], gr.n[2],
                           p->mid + mo, static_cast<float*>(p->coef), cap, p->mcount);
      else if (p->fp64 && p->cond)
        hipLaunchKernelGGL((k_material<double, true>), grid, blk, 0, s, prm, j, gr.n[0], gr.n[1], gr.n[2], gr.dim,
                           p->mid + mo, static_cast<double*>(p->coef), cap, p->mcount);
      else if (p->fp64)
        hipLaunchKernelGGL((k_material<double>), grid, blk, 0, s, prm, j, gr.n[0], gr.n[1], gr.n[2], gr.dim,
                           p->mid + mo, static_cast<double*>(p->coef), cap, p->mcount);
      else if (p->cond)
        hipLaunchKernelGGL((k_material<float, true>), grid, blk, 0, s, prm, j, gr.n[0], gr.n[1], gr.n[2], gr.dim,
                           p->mid + mo, static_cast<float*>(p->coef), cap, p->mcount);
      else
        hipLaunchKernelGGL((k_material<float>), grid, blk, 0, s, prm, j, gr.n[0], gr.n[1], gr.n[2], gr.dim,
                           p->mid + mo, static_cast<float*>(p->coef), cap, p->mcount);
      HM_HIP(hipGetLastError());
      mo += (size_t)N;
    }
    HM_HIP(hipMemcpyAsync(p->mcount_host, p->mcount, 2 * sizeof(int), hipMemcpyDeviceToHost, s));
    HM_HIP(hipStreamSynchronize(s));
    if ((rc = data_flags_error(p->mcount_host[1]))) return rc;
    const size_t rows = (size_t)p->mcount_host[0] * (p->aniso ? kGenRow / 8 : 1);  // in units of 8 reals
    if (rows <= p->coef_cap) return HM_OK;
    // too small: grow (stays allocated for later solves), re-queue the
    // parameters with the new table address and build again
    (void)hipFree(p->coef);
    p->coef = nullptr;
    p->coef_cap = 0;
    const size_t want = rows + rows / 4 + 1024;
    if ((rc = device_alloc(&p->coef, want * 8 * (p->fp64 ? 8 : 4), "stiffness table"))) return rc;
    p->coef_cap = want;
    if ((rc = upload_params(g, all, opts, s))) return rc;
  }
  return fail(HM_E_DEVICE, "material table did not fit after growing");
}

// Direct launches of one group; every kProfileStride-th iteration from
// iteration 1 on (1, 5, 9, ...) has a HIP event before and after each of its
// kernels (an event record costs a few microseconds of device time, so the
// other iterations run without).  Iteration 0 is never sampled: its x-sweep
// starts from the uniform strain, and the first launch of a kernel also
// waits for its code object to load.  Durations are read back at each poll
// and averaged over the sampled iterations that the longest load case
// evaluated.
constexpr int kProfileStride = 4;

int profiled_loop(Plan* p, const hm_solve_opts* opts, hipStream_t s) {
  const int k = opts->check_every;
  std::vector<hipEvent_t> ev((size_t)5 * k, nullptr);
  for (auto& e : ev)
    if (hipEventCreate(&e) != hipSuccess) {
      for (auto& q : ev)
        if (q) (void)hipEventDestroy(q);
      return fail(HM_E_DEVICE, "hipEventCreate failed");
    }
  SolveArgs a = p->args;
  std::vector<int> sampled_it;   // iteration of each sampled record
  std::vector<double> dur;       // 4 per sampled iteration
  bool done = false;
  int it = 0, rc = HM_OK;
  hipError_t err = hipSuccess;
  while (!done && it <= opts->max_iter && err == hipSuccess && rc == HM_OK) {
    std::vector<int> batch;  // sampled iterations of this block, in order
    for (int nb = 0; nb < k && it <= opts->max_iter; ++nb, ++it) {
      const bool rec = it % kProfileStride == 1;
      hipEvent_t* e = &ev[(size_t)5 * batch.size()];
      a.first = it == 0 ? 1 : 0;
      if (rec) err = hipEventRecord(e[0], s);
      if (err == hipSuccess) err = (it == 0 ? p->X->first : p->X->iter)(a, s);
      if (rec && err == hipSuccess) err = hipEventRecord(e[1], s);
      if (err == hipSuccess) err = p->Y->fwd(a, s);
      if (rec && err == hipSuccess) err = hipEventRecord(e[2], s);
      if (err == hipSuccess) err = p->Z->run(a, s);
      if (rec && err == hipSuccess) err = hipEventRecord(e[3], s);
      // the inverse y-sweep also ends the iteration (stop decision)
      if (err == hipSuccess) err = p->Y->inv(a, s);
      if (rec && err == hipSuccess) err = hipEventRecord(e[4], s);
      if (err != hipSuccess) break;
      if (rec) batch.push_back(it);
    }
    if (err != hipSuccess) break;
    rc = poll_done(p, s, &done);
    for (size_t b = 0; b < batch.size() && rc == HM_OK && err == hipSuccess; ++b) {
      sampled_it.push_back(batch[b]);
      for (int q = 0; q < 4; ++q) {
        float ms = 0.0f;
        err = hipEventElapsedTime(&ms, ev[5 * b + q], ev[5 * b + q + 1]);
        dur.push_back((double)ms);
      }
    }
  }
  for (auto& e : ev) (void)hipEventDestroy(e);
  if (err != hipSuccess) return fail(HM_E_DEVICE, "profiled loop: %s", hipGetErrorString(err));
  if (rc) return rc;
  int last = 0;
  for (int l = 0; l < p->n_load; ++l) last = std::max(last, p->state_host[l].iters);
  int nit = 0;
  double ms[4] = {0.0, 0.0, 0.0, 0.0}, active = 0.0;
  for (size_t i = 0; i < sampled_it.size(); ++i) {
    if (sampled_it[i] > last) break;
    for (int q = 0; q < 4; ++q) ms[q] += dur[4 * i + q];
    // a load case runs the kernels of iterations 0 .. iters
    for (int l = 0; l < p->n_load; ++l) active += p->state_host[l].iters >= sampled_it[i] ? 1.0 : 0.0;
    ++nit;
  }
  hm_timing t;
  memset(&t, 0, sizeof t);
  t.iterations = nit;
  for (int q = 0; q < 4; ++q) t.ms[q] = nit > 0 ? ms[q] / nit : 0.0;
  t.active_loads = nit > 0 ? active / nit : 0.0;
  t.n_load = p->n_load;
  t.x_lines = p->X->lines;
  t.y_width = p->Y->width;
  t.z_width = p->Z->width;
  t.z_threads = p->Z->threads;
  t.z_groups = p->Z->groups;
  const char* names[4] = {p->X->name, p->Y->fwd_name, p->Z->name, p->Y->inv_name};
  for (int q = 0; q < 4; ++q) snprintf(t.kernel[q], sizeof t.kernel[q], "%s", names[q]);
  snprintf(t.kernel[4], sizeof t.kernel[4], "(inside the inverse ysweep)");
  g_last_timing = t;
  g_have_timing = true;
  return HM_OK;
}

// ---------------------------------------------------- conjugate gradients
// Vectors x, r, p, per-load scalars and block partials, allocated on a
// plan's first CG solve.
int ensure_cg(Plan* p) {
  if (p->cgs) return HM_OK;
  const size_t cplx = p->fp64 ? 16 : 8;
  const size_t total = 6 * (size_t)p->n[2] * p->n[1] * p->args.Hp;
  const int blocks = (int)std::min<size_t>(1024, (total + kCgThreads * 8 - 1) / (kCgThreads * 8));
  void* v[3] = {nullptr, nullptr, nullptr};
  double* part = nullptr;
  CgState* cs = nullptr;
  int rc = HM_OK;
  for (int i = 0; i < 3 && !rc; ++i) rc = device_alloc(&v[i], (size_t)p->n_load * total * cplx, "CG vectors");
  if (!rc) rc = device_alloc((void**)&part, (size_t)p->n_load * blocks * sizeof(double), "CG partials");
  if (!rc) rc = device_alloc((void**)&cs, (size_t)p->n_load * sizeof(CgState), "CG state");
  if (rc) {
    for (int i = 0; i < 3; ++i) (void)hipFree(v[i]);
    (void)hipFree(part);
    return rc;
  }
  for (int i = 0; i < 3; ++i) p->cgv[i] = v[i];
  p->cgpart = part;
  p->cgs = cs;
  p->cg_blocks = blocks;
  SolveArgs& a = p->args;
  a.cgx = v[0];
  a.cgr = v[1];
  a.cgp = v[2];
  a.cgs = cs;
  a.cgpart = part;
  a.cg_blocks = blocks;
  drop_graphs(p);
  return HM_OK;
}

template <typename T> hipError_t cg_vec(int op, const SolveArgs& a, hipStream_t s) {
  const dim3 grid(a.cg_blocks, a.n_load), block(kCgThreads);
  switch (op) {
    case CG_INIT:
      hipLaunchKernelGGL((k_cg_vec<T, CG_INIT>), grid, block, 0, s, a);
      break;
    case CG_DOT:
      hipLaunchKernelGGL((k_cg_vec<T, CG_DOT>), grid, block, 0, s, a);
      break;
    case CG_UPDATE:
      hipLaunchKernelGGL((k_cg_vec<T, CG_UPDATE>), grid, block, 0, s, a);
      break;
    default:
      hipLaunchKernelGGL((k_cg_vec<T, CG_DIR>), grid, block, 0, s, a);
      break;
  }
  return hipGetLastError();
}

hipError_t cg_vector(const Plan* p, int op, const SolveArgs& a, hipStream_t s) {
  return p->fp64 ? cg_vec<double>(op, a, s) : cg_vec<float>(op, a, s);
}

hipError_t cg_scalar(int step, const SolveArgs& a, hipStream_t s) {
  const dim3 grid(a.n_load), block(kCgScalarThreads);
  if (step == CGS_INIT)
    hipLaunchKernelGGL((k_cg_scalar<kCgScalarThreads, CGS_INIT>), grid, block, 0, s, a);
  else if (step == CGS_ALPHA)
    hipLaunchKernelGGL((k_cg_scalar<kCgScalarThreads, CGS_ALPHA>), grid, block, 0, s, a);
  else
    hipLaunchKernelGGL((k_cg_scalar<kCgScalarThreads, CGS_BETA>), grid, block, 0, s, a);
  return hipGetLastError();
}

// Iterate 0: the sweeps turn E into r_0 = -G((c~ - I) : E); x = 0, p = r_0.
hipError_t launch_cg_start(Plan* p, hipStream_t s) {
  SolveArgs a = p->args;
  a.first = 1;
  a.cg = 1;
  hipError_t e;
  if ((e = p->X->first(a, s)) != hipSuccess) return e;
  if ((e = p->Y->fwd(a, s)) != hipSuccess) return e;
  if ((e = p->Z->run(a, s)) != hipSuccess) return e;
  if ((e = p->Y->inv(a, s)) != hipSuccess) return e;
  if ((e = cg_vector(p, CG_INIT, a, s)) != hipSuccess) return e;
  return cg_scalar(CGS_INIT, a, s);
}

// One CG iteration: w = sweeps(p), q = p - w, alpha, x and r, beta, p.
hipError_t launch_cg_iteration(Plan* p, hipStream_t s) {
  SolveArgs a = p->args;
  a.first = 0;
  a.cg = 1;
  a.spec_in = p->cgv[2];
  hipError_t e;
  if ((e = p->X->iter(a, s)) != hipSuccess) return e;
  if ((e = p->Y->fwd(a, s)) != hipSuccess) return e;
  if ((e = p->Z->run(a, s)) != hipSuccess) return e;
  if ((e = p->Y->inv(a, s)) != hipSuccess) return e;
  if ((e = cg_vector(p, CG_DOT, a, s)) != hipSuccess) return e;
  if ((e = cg_scalar(CGS_ALPHA, a, s)) != hipSuccess) return e;
  if ((e = cg_vector(p, CG_UPDATE, a, s)) != hipSuccess) return e;
  if ((e = cg_scalar(CGS_BETA, a, s)) != hipSuccess) return e;
  return cg_vector(p, CG_DIR, a, s);
}

int build_cg_graph(Plan* p, int k) {
  if (p->cg_graph && p->cg_graph_k == k) return HM_OK;
  if (p->cg_graph) (void)hipGraphExecDestroy(p->cg_graph);
  p->cg_graph = nullptr;
  if (!p->cap_stream) HM_HIP(hipStreamCreateWithFlags(&p->cap_stream, hipStreamNonBlocking));
  hipGraph_t g = nullptr;
  HM_HIP(hipStreamBeginCapture(p->cap_stream, hipStreamCaptureModeThreadLocal));
  hipError_t le = hipSuccess;
  for (int i = 0; i < k && le == hipSuccess; ++i) le = launch_cg_iteration(p, p->cap_stream);
  hipError_t ce = hipStreamEndCapture(p->cap_stream, &g);
  if (le != hipSuccess || ce != hipSuccess) {
    if (g) (void)hipGraphDestroy(g);
    return fail(HM_E_DEVICE, "CG graph capture failed: %s", hipGetErrorString(le != hipSuccess ? le : ce));
  }
  hipError_t ie = hipGraphInstantiate(&p->cg_graph, g, nullptr, nullptr, 0);
  (void)hipGraphDestroy(g);
  if (ie != hipSuccess) {
    p->cg_graph = nullptr;
    return fail(HM_E_DEVICE, "CG graph instantiation failed: %s", hipGetErrorString(ie));
  }
  p->cg_graph_k = k;
  return HM_OK;
}

// CG solve of one grid group to its stop; exports eps = E + x when asked.
int run_cg(Group& g, const hm_solve_opts* opts, hipStream_t s) {
  Plan* p = g.p;
  int rc;
  if ((rc = ensure_cg(p))) return rc;
  HM_HIP(launch_cg_start(p, s));
  bool done = false;
  if ((rc = poll_done(p, s, &done))) return rc;
  const int k = opts->check_every;
  int it = 1;
  while (!done && it <= opts->max_iter) {
    if (opts->use_graph) {
      if ((rc = build_cg_graph(p, k))) return rc;
      HM_HIP(hipGraphLaunch(p->cg_graph, s));
      it += k;
    } else {
      for (int b = 0; b < k && it <= opts->max_iter; ++b, ++it) HM_HIP(launch_cg_iteration(p, s));
    }
    if ((rc = poll_done(p, s, &done))) return rc;
  }
  if (g.eps_out) {
    SolveArgs a = p->args;
    a.cg = 1;
    a.spec_in = p->cgv[0];
    a.eps_out = g.eps_out;
    HM_HIP(p->X->exp(a, s));
  }
  return poll_done(p, s, &done);
}

struct LastSolve {
  Plan* p = nullptr;
  unsigned generation = 0;
  int n_load = 0;
  std::vector<int> iters;
};
thread_local LastSolve g_last_solve;

void record_last_solve(std::vector<Group>& G) {
  g_last_solve.p = nullptr;
  if (G.size() != 1) return;
  Plan* p = G[0].p;
  std::lock_guard<std::mutex> lock(g_mutex);
  g_last_solve.p = p;
  g_last_solve.generation = g_plan_generation;
  g_last_solve.n_load = p->n_load;
  g_last_solve.iters.resize(p->n_load);
  for (int l = 0; l < p->n_load; ++l) g_last_solve.iters[l] = p->state_host[l].iters;
}

// Solves every group to its stop (or max_iter): iterate 0 directly, then
// blocks of check_every iterations (one captured graph over all active
// groups, or direct launches), polling the device-side stop flags between
// blocks.  On return every group's state_host holds its final states.
int run_groups(std::vector<Group>& G, const std::vector<ProblemIn>& all, const hm_solve_opts* opts, hipStream_t s) {
  int rc;
  for (Group& g : G) {
    if ((rc = ensure_hist(g.p, opts->max_iter + 1))) return rc;
    if ((rc = upload_params(g, all, opts, s))) return rc;
    if ((rc = prepare_material(g, all, opts, s))) return rc;
    if (g.p->cond) {
      // conduction plans have one compiled schedule
      if (opts->schedule >= 0 && opts->schedule != 0) return fail(HM_E_ARG, "conduction solves have one schedule");
    } else if (g.p->aniso && !opts->autotune) {
      // anisotropic plans without autotuning run the first schedule (a plan
      // tuned by an earlier solve is set back to it)
      if (opts->schedule >= 0 && opts->schedule != 0) return fail(HM_E_ARG, "anisotropic solves pin no schedule");
      if (g.p->tuned) {
        set_schedule(g.p, &g.p->ak->x, &g.p->ky->y[0], &g.p->kz->z[0]);
        g.p->tuned = false;
      }
    } else if (opts->autotune) {
      if (!g.p->tuned && (rc = tune_plan(g.p, s))) return rc;
    } else if (opts->schedule >= 0) {
      const int xv = opts->schedule & 15, yv = (opts->schedule >> 4) & 15, zv = (opts->schedule >> 8) & 15;
      if (xv >= g.p->kx->nxv || yv >= g.p->ky->nyv || zv >= g.p->kz->nzv)
        return fail(HM_E_ARG, "schedule %#x out of range", opts->schedule);
      set_schedule(g.p, &g.p->kx->x[xv], &g.p->ky->y[yv], &g.p->kz->z[zv]);
      g.p->tuned = false;
    } else if (g.p->tuned || g.p->X != &g.p->kx->x[0] || g.p->Y != &g.p->ky->y[0] || g.p->Z != &g.p->kz->z[0]) {
      set_schedule(g.p, &g.p->kx->x[0], &g.p->ky->y[0], &g.p->kz->z[0]);
      g.p->tuned = false;
    }
    hipLaunchKernelGGL((k_reset_state<64>), dim3((g.p->n_load + 63) / 64), dim3(64), 0, s, g.p->state,
                       g.p->n_load);
    HM_HIP(hipGetLastError());
    g.active = true;
  }
  if (opts->method == HM_CONJUGATE_GRADIENT) {
    if (G.size() != 1) return fail(HM_E_ARG, "conjugate gradients solve one grid group");
    if ((rc = run_cg(G[0], opts, s))) return rc;
    record_last_solve(G);
    return HM_OK;
  }
  if (opts->profile) {
    if (G.size() != 1) return fail(HM_E_ARG, "profiling times a single grid group");
    if ((rc = profiled_loop(G[0].p, opts, s))) return rc;
  } else {
    const int k = opts->check_every;
    for (Group& g : G) {
      SolveArgs a = g.p->args;
      a.first = 1;
      HM_HIP(launch_iteration(g.p, a, true, s));
    }
    auto poll_all = [&](int* n_active, bool* changed) -> int {
      *n_active = 0;
      *changed = false;
      for (Group& g : G) {
        if (!g.active) continue;
        bool d = false;
        int r = poll_done(g.p, s, &d);
        if (r) return r;
        if (d) {
          g.active = false;
          *changed = true;
        } else {
          ++*n_active;
        }
      }
      return HM_OK;
    };
    int n_active = (int)G.size();
    bool changed = false;
    if (opts->max_iter == 0 || k == 1)
      if ((rc = poll_all(&n_active, &changed))) return rc;
    int it = 1;
    hipGraphExec_t multi = nullptr;
    hipStream_t cap = nullptr;
    while (n_active > 0 && it <= opts->max_iter) {
      if (opts->use_graph) {
        if (G.size() == 1) {
          if ((rc = build_graph(G[0].p, k))) return rc;
          HM_HIP(hipGraphLaunch(G[0].p->graph, s));
        } else {
          if (!multi || changed) {
            if (multi) (void)hipGraphExecDestroy(multi);
            multi = nullptr;
            if (!cap) HM_HIP(hipStreamCreateWithFlags(&cap, hipStreamNonBlocking));
            std::vector<Plan*> act;
            for (Group& g : G)
              if (g.active) act.push_back(g.p);
            if ((rc = capture_graph(act, k, cap, &multi))) {
              (void)hipStreamDestroy(cap);
              return rc;
            }
          }
          hipError_t e = hipGraphLaunch(multi, s);
          if (e != hipSuccess) {
            (void)hipGraphExecDestroy(multi);
            (void)hipStreamDestroy(cap);
            return fail(HM_E_DEVICE, "graph launch: %s", hipGetErrorString(e));
          }
        }
        it += k;
      } else {
        for (int b = 0; b < k && it <= opts->max_iter; ++b, ++it)
          for (Group& g : G)
            if (g.active) {
              SolveArgs a = g.p->args;
              a.first = 0;
              HM_HIP(launch_iteration(g.p, a, false, s));
            }
      }
      if ((rc = poll_all(&n_active, &changed))) break;
    }
    if (multi) (void)hipGraphExecDestroy(multi);
    if (cap) (void)hipStreamDestroy(cap);
    if (rc) return rc;
  }
  for (Group& g : G) {
    if (g.eps_out) {
      SolveArgs a = g.p->args;
      a.eps_out = g.eps_out;
      HM_HIP(g.p->X->exp(a, s));
    }
    bool d = false;
    if ((rc = poll_done(g.p, s, &d))) return rc;
  }
  record_last_solve(G);
  return HM_OK;
}

// Status of one load case.
int load_status(const SolverState& st) { return st.done ? st.status : HM_NOT_CONVERGED; }



// Unit Mandel strains (tensor components) of a dimension: 6 in 3D, 3 in 2D.
int unit_loads(int dim, double E[36], const int** idx_out) {
  static const int idx3[6] = {0, 1, 2, 3, 4, 5};
  static const int idx2[3] = {0, 1, 5};
  const int k = dim == 2 ? 3 : 6;
  const int* idx = dim == 2 ? idx2 : idx3;
  const double r2 = 1.0 / sqrt(2.0);
  for (int i = 0; i < 36; ++i) E[i] = 0.0;
  for (int J = 0; J < k; ++J) E[6 * J + idx[J]] = idx[J] < 3 ? 1.0 : r2;
  *idx_out = idx;
  return k;
}

// Mandel matrix from the mean stresses of the unit strains.
void assemble_mandel(int k, const int* idx, const SolverState* st, double* C) {
  const double w[6] = {1.0, 1.0, 1.0, sqrt(2.0), sqrt(2.0), sqrt(2.0)};
  for (int I = 0; I < k; ++I)
    for (int J = 0; J < k; ++J) C[I * k + J] = w[idx[I]] * st[J].sig[idx[I]];
}

// The single-problem solve shared by hm_solve and hm_effective_tensor.
int solve_one(const ProblemIn& d, const double* E, int n_load, const hm_solve_opts* opts, void* d_eps,
              hipStream_t s, Plan** plan_out) {
  int rc;
  if ((rc = check_problem(d))) return rc;
  if ((rc = check_opts(opts))) return rc;
  if (n_load < 1 || n_load > kMaxLoads) return fail(HM_E_ARG, "n_load must be in 1..%d", kMaxLoads);
  for (int i = 0; i < 6 * n_load; ++i)
    if (!isfinite(E[i])) return fail(HM_E_ARG, "E has a non-finite entry");
  std::vector<ProblemIn> all{d};
  std::vector<Group> G(1);
  const int phys = d.cond ? PHYS_CONDUCTION : (d.aniso ? PHYS_ANISO : PHYS_ELASTIC);
  if ((rc = get_plan(opts->prec == HM_FP64, d.grid.n, d.grid.dim, n_load, phys, &G[0].p))) return rc;
  G[0].probs = {0};
  G[0].loads.resize(n_load);
  for (int l = 0; l < n_load; ++l) {
    for (int c = 0; c < 6; ++c) G[0].loads[l].E[c] = E[6 * l + c];
    G[0].loads[l].prob = 0;
    G[0].loads[l].pad = 0;
  }
  G[0].eps_out = d_eps;
  if ((rc = run_groups(G, all, opts, s))) return rc;
  *plan_out = G[0].p;
  return HM_OK;
}

// The conduction solve shared by hm_conduct_solve and hm_effective_conductivity:
// G holds 3 mean-gradient components per load case.
int solve_cond(const ProblemIn& d, const double* G, int n_load, const hm_solve_opts* opts, void* d_grad,
               hipStream_t s, Plan** plan_out) {
  int rc;
  if ((rc = check_problem(d))) return rc;
  if ((rc = check_opts(opts))) return rc;
  if (opts->method != HM_FIXED_POINT) return fail(HM_E_ARG, "conduction solves use the fixed-point method");
  if (n_load < 1 || n_load > kMaxLoads) return fail(HM_E_ARG, "n_load must be in 1..%d", kMaxLoads);
  for (int i = 0; i < 3 * n_load; ++i)
    if (!isfinite(G[i])) return fail(HM_E_ARG, "G has a non-finite entry");
  std::vector<ProblemIn> all{d};
  std::vector<Group> grp(1);
  if ((rc = get_plan(opts->prec == HM_FP64, d.grid.n, d.grid.dim, n_load, PHYS_CONDUCTION, &grp[0].p))) return rc;
  grp[0].probs = {0};
  grp[0].loads.resize(n_load);
  for (int l = 0; l < n_load; ++l) {
    LoadParams& L = grp[0].loads[l];
    for (int c = 0; c < 6; ++c) L.E[c] = c < 3 ? G[3 * l + c] : 0.0;
    L.prob = 0;
    L.pad = 0;
  }
  grp[0].eps_out = d_grad;
  if ((rc = run_groups(grp, all, opts, s))) return rc;
  *plan_out = grp[0].p;
  return HM_OK;
}

ProblemIn make_problem(const hm_grid* grid, const hm_iso phases[2], hm_rule rule, const void* d_frac,
                       const int32_t* d_incl, const hm_sphere* spheres, int n_spheres) {
  ProblemIn d;
  memset(&d, 0, sizeof d);
  if (grid) d.grid = *grid;
  if (phases) {
    d.phases[0] = phases[0];
    d.phases[1] = phases[1];
  }
  d.rule = rule;
  d.frac = d_frac;
  d.incl = d_incl;
  d.sph = spheres;
  d.nsph = n_spheres;
  return d;
}

// Dirichlet kernel matrix K[b][a] = D_n((b + 1/2)/m - (a + 1/2)/n) with
// D_n(t) = sin(pi n t) / (n sin(pi t)) (1 at integer t): with
// p = (2b + 1) n - (2a + 1) m, t = p / (2 m n), so both sines take
// rational multiples of pi whose arguments are reduced exactly in integers
// before a long double evaluation; entries are exactly 1 or 0 where the
// fine point meets a grid point.
std::vector<double> dirichlet_matrix(int n, int m) {
  const long double pi = 3.141592653589793238462643383279502884L;
  std::vector<double> K((size_t)m * n);
  const long long q1 = 2LL * m, q2 = 2LL * m * n;
  for (int b = 0; b < m; ++b)
    for (int a = 0; a < n; ++a) {
      const long long p = (2LL * b + 1) * n - (2LL * a + 1) * m;
      double v;
      if (p % q2 == 0) {
        v = 1.0;
      } else if (p % q1 == 0) {
        v = 0.0;
      } else {
        const long long r1 = ((p % (2 * q1)) + 2 * q1) % (2 * q1);
        const long long r2 = ((p % (2 * q2)) + 2 * q2) % (2 * q2);
        v = (double)(sinl(pi * (long double)r1 / (long double)q1) /
                     ((long double)n * sinl(pi * (long double)r2 / (long double)q2)));
      }
      K[(size_t)b * n + a] = v;
    }
  return K;
}

// Matrices and temporaries of one (device, precision, n, m) series, kept
// until hm_release_plans.
struct SeriesPlan {
  void* k[3] = {nullptr, nullptr, nullptr};  // x, y, z matrices, each transposed (n_d x m_d)
  void* t1 = nullptr;                        // after the x pass
  void* t2 = nullptr;                        // after the y pass (3D)
};
std::map<std::tuple<int, bool, int, int, int, int, int, int>, SeriesPlan*> g_series;

void free_series(SeriesPlan* q) {
  for (void* v : {q->k[0], q->k[1], q->k[2], q->t1, q->t2}) (void)hipFree(v);
  delete q;
}

// Uploads a matrix (row-major, or transposed) in the working precision.
int upload_matrix(const std::vector<double>& K, int rows, int cols, bool transpose, bool fp64, void** out) {
  const size_t cnt = (size_t)rows * cols;
  int rc = device_alloc(out, cnt * (fp64 ? 8 : 4), "series matrix");
  if (rc) return rc;
  std::vector<double> d(cnt);
  for (int r = 0; r < rows; ++r)
    for (int c = 0; c < cols; ++c) d[transpose ? (size_t)c * rows + r : (size_t)r * cols + c] = K[(size_t)r * cols + c];
  hipError_t e;
  if (fp64) {
    e = hipMemcpy(*out, d.data(), cnt * 8, hipMemcpyHostToDevice);
  } else {
    std::vector<float> f(cnt);
    for (size_t i = 0; i < cnt; ++i) f[i] = (float)d[i];
    e = hipMemcpy(*out, f.data(), cnt * 4, hipMemcpyHostToDevice);
  }
  if (e != hipSuccess) return fail(HM_E_DEVICE, "series matrix upload: %s", hipGetErrorString(e));
  return HM_OK;
}

}  // namespace

extern "C" {

// An anisotropic two-phase cell as a ProblemIn.
static ProblemIn aniso_problem(const hm_grid* grid, const double* C_phases, hm_rule rule, const void* d_frac,
                               const int32_t* d_incl, const hm_sphere* spheres, int n_spheres) {
  ProblemIn d = make_problem(grid, nullptr, rule, d_frac, d_incl, spheres, n_spheres);
  d.aniso = 1;
  if (C_phases)
    for (int p = 0; p < 2; ++p)
      for (int i = 0; i < 36; ++i) d.cm[p][i] = C_phases[36 * p + i];
  return d;
}

int hm_solve_aniso(const hm_grid* grid, const double* C_phases, hm_rule rule, const void* d_frac,
                   const int32_t* d_incl, const hm_sphere* spheres, int n_spheres, const double* E, int n_load,
                   const hm_solve_opts* opts, void* d_eps, double* sig_mean, hm_report* rep, void* stream) {
  const auto t0 = std::chrono::steady_clock::now();
  if (!C_phases) return fail(HM_E_ARG, "C_phases is NULL");
  if (!E || !sig_mean) return fail(HM_E_ARG, "E and sig_mean must not be NULL");
  Plan* p = nullptr;
  int rc = solve_one(aniso_problem(grid, C_phases, rule, d_frac, d_incl, spheres, n_spheres), E, n_load, opts,
                     d_eps, (hipStream_t)stream, &p);
  if (rc) return rc;
  const double secs = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
  int worst = HM_OK;
  for (int l = 0; l < n_load; ++l) {
    const SolverState& st = p->state_host[l];
    for (int c = 0; c < 6; ++c) sig_mean[6 * l + c] = st.sig[c];
    const int status = load_status(st);
    if (rep) rep[l] = hm_report{st.iters, status, st.err, st.err0, secs};
    worst = std::max(worst, status);
  }
  return worst;
}

int hm_effective_tensor_aniso(const hm_grid* grid, const double* C_phases, hm_rule rule, const void* d_frac,
                              const int32_t* d_incl, const hm_sphere* spheres, int n_spheres,
                              const hm_solve_opts* opts, double* C_mandel, void* d_eps, hm_report* rep,
                              void* stream) {
  const auto t0 = std::chrono::steady_clock::now();
  int rc;
  if ((rc = check_grid(grid))) return rc;
  if (!C_phases) return fail(HM_E_ARG, "C_phases is NULL");
  if (!C_mandel) return fail(HM_E_ARG, "C_mandel is NULL");
  double E[36];
  const int* idx = nullptr;
  const int k = unit_loads(grid->dim, E, &idx);
  Plan* p = nullptr;
  rc = solve_one(aniso_problem(grid, C_phases, rule, d_frac, d_incl, spheres, n_spheres), E, k, opts, d_eps,
                 (hipStream_t)stream, &p);
  if (rc) return rc;
  const double secs = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
  assemble_mandel(k, idx, p->state_host, C_mandel);
  int worst = HM_OK;
  for (int l = 0; l < k; ++l) {
    const SolverState& st = p->state_host[l];
    const int status = load_status(st);
    if (rep) rep[l] = hm_report{st.iters, status, st.err, st.err0, secs};
    worst = std::max(worst, status);
  }
  return worst;
}

int hm_fourier_series(const hm_grid* grid, const int m[3], hm_prec prec, const void* d_field, void* d_out,
                      void* stream) {
  if (!grid || !m) return fail(HM_E_ARG, "grid and m must not be NULL");
  if (grid->dim != 2 && grid->dim != 3) return fail(HM_E_ARG, "dim must be 2 or 3 (got %d)", grid->dim);
  if (prec != HM_FP64 && prec != HM_MIXED) return fail(HM_E_ARG, "unknown precision");
  long long M = 1;
  for (int d = 0; d < 3; ++d) {
    if (grid->n[d] < 1 || grid->n[d] > 243 || grid->n[d] % 2 == 0)
      return fail(HM_E_SIZE, "n[%d] = %d must be odd and <= 243", d, grid->n[d]);
    if (m[d] < 1 || m[d] > 4096) return fail(HM_E_SIZE, "m[%d] = %d must be in 1..4096", d, m[d]);
    M *= m[d];
  }
  if (grid->dim == 2 && (grid->n[2] != 1 || m[2] != 1)) return fail(HM_E_ARG, "2D grids need n[2] == m[2] == 1");
  if (M > (1LL << 32)) return fail(HM_E_SIZE, "output of %lld points is too large", M);
  if (!d_field || !d_out) return fail(HM_E_ARG, "d_field and d_out must not be NULL");
  const bool fp64 = prec == HM_FP64;
  const size_t rb = fp64 ? 8 : 4;
  const int nx = grid->n[0], ny = grid->n[1], nz = grid->n[2];
  const bool zpass = !(nz == 1 && m[2] == 1);
  hipStream_t s = (hipStream_t)stream;
  int dev = 0;
  HM_HIP(hipGetDevice(&dev));
  SeriesPlan* q = nullptr;
  {
    std::lock_guard<std::mutex> lock(g_mutex);
    const auto key = std::make_tuple(dev, fp64, nx, ny, nz, m[0], m[1], m[2]);
    auto it = g_series.find(key);
    if (it != g_series.end()) {
      q = it->second;
    } else {
      q = new SeriesPlan();
      int rc = upload_matrix(dirichlet_matrix(nx, m[0]), m[0], nx, true, fp64, &q->k[0]);
      if (!rc) rc = upload_matrix(dirichlet_matrix(ny, m[1]), m[1], ny, true, fp64, &q->k[1]);
      if (!rc) rc = upload_matrix(dirichlet_matrix(nz, m[2]), m[2], nz, true, fp64, &q->k[2]);
      if (!rc) rc = device_alloc(&q->t1, (size_t)nz * ny * m[0] * rb, "series x pass");
      if (!rc && zpass) rc = device_alloc(&q->t2, (size_t)nz * m[1] * m[0] * rb, "series y pass");
      if (rc) {
        free_series(q);
        return rc;
      }
      g_series[key] = q;
    }
  }
  // x: contiguous lines; y: stride mx; z: stride mx * my
  AxisPass px{d_field, q->t1, q->k[0], 1, (long long)ny * nz, nx, m[0]};
  AxisPass py{q->t1, zpass ? q->t2 : d_out, q->k[1], (long long)m[0], (long long)nz, ny, m[1]};
  AxisPass pz{q->t2, d_out, q->k[2], (long long)m[0] * m[1], 1, nz, m[2]};
  hipError_t e = launch_series_pass(px, fp64, s);
  if (e == hipSuccess) e = launch_series_pass(py, fp64, s);
  if (e == hipSuccess && zpass) e = launch_series_pass(pz, fp64, s);
  if (e != hipSuccess) return fail(HM_E_DEVICE, "Fourier series: %s", hipGetErrorString(e));
  return HM_OK;
}

// Per-voxel material kernels after a solve (a Mandel entry of c~, or the
// stress of strain fields): the sphere table and a flag word on the device,
// the kernel, the flags read back (the call returns after the kernel).
static int voxel_material_call(const hm_grid* grid, const hm_iso phases[2], hm_rule rule, const void* d_frac,
                               const int32_t* d_incl, const hm_sphere* spheres, int n_spheres, hm_prec prec, int I,
                               int J, void* d_out, const void* d_eps, int n_load, void* stream, const char* what,
                               const double* k = nullptr) {
  ProblemIn d = make_problem(grid, phases, rule, d_frac, d_incl, spheres, n_spheres);
  if (k) {
    d.cond = 1;
    d.k[0] = k[0];
    d.k[1] = k[1];
  }
  int rc;
  if ((rc = check_problem(d))) return rc;
  if (prec != HM_FP64 && prec != HM_MIXED) return fail(HM_E_ARG, "unknown precision");
  if (I < 0 || I > 5 || J < 0 || J > 5) return fail(HM_E_ARG, "Mandel indices must be in 0..5");
  if (!d_out) return fail(HM_E_ARG, "the output pointer is NULL");
  hipStream_t s = (hipStream_t)stream;
  double* dsph = nullptr;
  int* dflags = nullptr;
  const size_t sb = (size_t)(n_spheres > 0 ? n_spheres : 1) * 4 * sizeof(double);
  if ((rc = device_alloc((void**)&dsph, sb, "sphere table"))) return rc;
  if ((rc = device_alloc((void**)&dflags, sizeof(int), "flags"))) {
    (void)hipFree(dsph);
    return rc;
  }
  std::vector<double> tab(sb / sizeof(double), 0.0);
  for (int k = 0; k < n_spheres; ++k) {
    for (int c = 0; c < 3; ++c) tab[4 * k + c] = spheres[k].c[c];
    tab[4 * k + 3] = spheres[k].r;
  }
  StiffnessArgs a;
  memset(&a, 0, sizeof a);
  a.frac = d_frac;
  a.incl = d_incl;
  a.sph = dsph;
  a.nsph = n_spheres;
  for (int k = 0; k < 3; ++k) a.n[k] = grid->n[k];
  a.dim = grid->dim;
  for (int p = 0; p < 2; ++p) {
    a.pl[p] = k ? k[p] : phases[p].lambda;
    a.pm[p] = k ? 0.0 : phases[p].mu;
  }
  a.rule = (int)rule;
  a.I = I;
  a.J = J;
  a.out = d_out;
  a.flags = dflags;
  int flags = 0;
  hipError_t e = hipMemcpyAsync(dsph, tab.data(), sb, hipMemcpyHostToDevice, s);
  if (e == hipSuccess) e = hipMemsetAsync(dflags, 0, sizeof(int), s);
  if (e == hipSuccess) {
    if (d_eps) {
      StressArgs sa{a, d_eps, d_out, n_load};
      e = k ? launch_flux_field(sa, prec == HM_FP64, s) : launch_stress_field(sa, prec == HM_FP64, s);
    } else {
      e = launch_stiffness_component(a, prec == HM_FP64, s);
    }
  }
  if (e == hipSuccess) e = hipMemcpyAsync(&flags, dflags, sizeof(int), hipMemcpyDeviceToHost, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  (void)hipFree(dsph);
  (void)hipFree(dflags);
  if (e != hipSuccess) return fail(HM_E_DEVICE, "%s: %s", what, hipGetErrorString(e));
  if (flags & 1) return fail(HM_E_DATA, "fractional voxel with HM_RULE_NONE");
  if (flags & 2) return fail(HM_E_DATA, "d_incl holds a sphere index >= n_spheres");
  return HM_OK;
}

int hm_stiffness_component(const hm_grid* grid, const hm_iso phases[2], hm_rule rule, const void* d_frac,
                           const int32_t* d_incl, const hm_sphere* spheres, int n_spheres, hm_prec prec, int I,
                           int J, void* d_out, void* stream) {
  return voxel_material_call(grid, phases, rule, d_frac, d_incl, spheres, n_spheres, prec, I, J, d_out, nullptr, 0,
                             stream, "stiffness component");
}

int hm_flux_field(const hm_grid* grid, const double k[2], hm_rule rule, const void* d_frac, const int32_t* d_incl,
                  const hm_sphere* spheres, int n_spheres, hm_prec prec, const void* d_grad, int n_load,
                  void* d_flux, void* stream) {
  if (!k) return fail(HM_E_ARG, "k is NULL");
  if (!d_grad) return fail(HM_E_ARG, "d_grad is NULL");
  if (n_load < 1 || n_load > kMaxLoads) return fail(HM_E_ARG, "n_load must be in 1..%d", kMaxLoads);
  return voxel_material_call(grid, nullptr, rule, d_frac, d_incl, spheres, n_spheres, prec, 0, 0, d_flux, d_grad,
                             n_load, stream, "flux field", k);
}

int hm_stress_field(const hm_grid* grid, const hm_iso phases[2], hm_rule rule, const void* d_frac,
                    const int32_t* d_incl, const hm_sphere* spheres, int n_spheres, hm_prec prec, const void* d_eps,
                    int n_load, void* d_sig, void* stream) {
  if (!d_eps) return fail(HM_E_ARG, "d_eps is NULL");
  if (n_load < 1 || n_load > kMaxLoads) return fail(HM_E_ARG, "n_load must be in 1..%d", kMaxLoads);
  return voxel_material_call(grid, phases, rule, d_frac, d_incl, spheres, n_spheres, prec, 0, 0, d_sig, d_eps,
                             n_load, stream, "stress field");
}

const char* hm_last_error(void) { return g_last_error.c_str(); }

int hm_last_timing(hm_timing* out) {
  if (!out) return fail(HM_E_ARG, "out is NULL");
  if (!g_have_timing) return fail(HM_E_ARG, "no profiled solve on this thread");
  *out = g_last_timing;
  return HM_OK;
}

int hm_device_ok(void) {
  int n = 0;
  if (hipGetDeviceCount(&n) != hipSuccess || n < 1) {
    (void)hipGetLastError();
    return 0;
  }
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return 0;
  hipDeviceProp_t prop;
  if (hipGetDeviceProperties(&prop, dev) != hipSuccess) return 0;
  return strncmp(prop.gcnArchName, "gfx950", 6) == 0 ? 1 : 0;
}

int hm_schedule_count(const hm_grid* grid, hm_prec prec, int* nx, int* ny, int* nz) {
  int rc;
  if ((rc = check_grid(grid))) return rc;
  if (!nx || !ny || !nz) return fail(HM_E_ARG, "NULL output");
  const bool fp64 = prec == HM_FP64;
  const AxisKernels* kx = axis_kernels(fp64, grid->n[0]);
  const AxisKernels* ky = axis_kernels(fp64, grid->n[1]);
  const AxisKernels* kz = axis_kernels(fp64, grid->n[2]);
  if (!kx || !ky || !kz) return fail(HM_E_SIZE, "no kernels for this grid");
  *nx = kx->nxv;
  *ny = ky->nyv;
  *nz = kz->nzv;
  return HM_OK;
}

int hm_last_history(int n_load, int cap, double* err, double* sig) {
  const LastSolve& L = g_last_solve;
  if (!L.p) return fail(HM_E_ARG, "no single-cell solve on this thread");
  if (!err) return fail(HM_E_ARG, "err is NULL");
  if (cap < 1) return fail(HM_E_ARG, "cap must be >= 1");
  Plan* p = nullptr;
  {
    std::lock_guard<std::mutex> lock(g_mutex);
    if (L.generation != g_plan_generation) return fail(HM_E_ARG, "the plans of the last solve were released");
    p = L.p;
  }
  if (n_load != L.n_load) return fail(HM_E_ARG, "the last solve had %d load cases, not %d", L.n_load, n_load);
  const double nan = NAN;
  for (int l = 0; l < n_load; ++l) {
    const int cnt = std::min(std::min(cap, L.iters[l] + 1), p->hist_cap);
    if (cnt > 0) {
      HM_HIP(hipMemcpy(err + (size_t)l * cap, p->errhist + (size_t)l * p->hist_cap, (size_t)cnt * sizeof(double),
                       hipMemcpyDeviceToHost));
      if (sig)
        HM_HIP(hipMemcpy(sig + (size_t)l * cap * 6, p->sighist + (size_t)l * p->hist_cap * 6,
                         (size_t)cnt * 6 * sizeof(double), hipMemcpyDeviceToHost));
    }
    for (int i = std::max(cnt, 0); i < cap; ++i) {
      err[(size_t)l * cap + i] = nan;
      if (sig)
        for (int c = 0; c < 6; ++c) sig[((size_t)l * cap + i) * 6 + c] = nan;
    }
  }
  return HM_OK;
}

void hm_release_plans(void) {
  std::lock_guard<std::mutex> lock(g_mutex);
  ++g_plan_generation;
  for (auto& kv : g_plans) free_plan(kv.second);
  g_plans.clear();
  for (auto& kv : g_series) free_series(kv.second);
  g_series.clear();
}

// Checks the filter arguments and fills the lattice sphere table (host,
// n_spheres entries) and the kernel arguments except the device pointers.
static int filter_prepare(const hm_grid* grid, const hm_sphere* spheres, int n_spheres, const int* labels, int nlab,
                          double radius_vox, int subsamples, hm_rule rule, hm_prec prec, uint32_t* d_count,
                          void* d_frac, LatSphere* tab, FilterArgs& a) {
  int rc;
  if ((rc = check_grid(grid))) return rc;
  if ((rc = check_spheres(grid, spheres, n_spheres))) return rc;
  if (rule < HM_RULE_NONE || rule > HM_RULE_LAMINATE) return fail(HM_E_ARG, "unknown rule %d", (int)rule);
  if (prec != HM_FP64 && prec != HM_MIXED) return fail(HM_E_ARG, "unknown precision");
  if (subsamples < 2 || subsamples > 32 || subsamples % 2) return fail(HM_E_ARG, "subsamples must be even, 2..32");
  const bool point = rule == HM_RULE_NONE;
  if (!point && !(radius_vox > 0.0 && radius_vox * subsamples <= 64.0))
    return fail(HM_E_ARG, "radius_vox must be > 0 with radius_vox * subsamples <= 64");
  if (!d_count || !d_frac) return fail(HM_E_ARG, "d_count and d_frac must not be NULL");
  memset(&a, 0, sizeof a);
  a.nsph = n_spheres;
  a.dim = grid->dim;
  a.S = subsamples;
  const double s2 = 2.0 * subsamples;
  for (int d = 0; d < 3; ++d) {
    a.n[d] = grid->n[d];
    a.P[d] = 2LL * grid->n[d] * subsamples;
  }
  for (int k = 0; k < n_spheres; ++k) {
    for (int d = 0; d < 3; ++d) {
      const double c = spheres[k].c[d] * s2;
      tab[k].c[d] = (long long)(c >= 0.0 ? floor(c + 0.5) : -floor(-c + 0.5));
    }
    tab[k].t = spheres[k].r * s2;
    tab[k].R2 = tab[k].t * tab[k].t;
  }
  a.point = point ? 1 : 0;
  if (point) {
    a.M = 1;
  } else {
    a.rho = radius_vox * s2;
    a.rho2 = a.rho * a.rho;
    a.m = (int)floor(a.rho);
    const int axes = grid->dim == 2 ? 2 : 3;
    int M = 0;
    for (int oz = (axes == 3 ? -a.m : 0); oz <= (axes == 3 ? a.m : 0); ++oz) {
      if (axes == 3 && (oz & 1) == 0) continue;
      for (int oy = -a.m; oy <= a.m; ++oy) {
        if ((oy & 1) == 0) continue;
        for (int ox = -a.m; ox <= a.m; ++ox) {
          if ((ox & 1) == 0) continue;
          const long long o2 = (long long)ox * ox + (long long)oy * oy + (long long)oz * oz;
          if ((double)o2 <= a.rho2) ++M;
        }
      }
    }
    if (M < 1) return fail(HM_E_ARG, "filter radius keeps no refined point");
    a.M = M;
  }
  if (labels) {
    // spheres of different phases may not share a refined point: their
    // lattice balls must be disjoint (minimum image per axis)
    const int axes = grid->dim == 2 ? 2 : 3;
    for (int i = 0; i < n_spheres; ++i) {
      if (labels[i] < 1 || labels[i] > nlab) return fail(HM_E_ARG, "sphere %d: label must be in 1..%d", i, nlab);
      for (int j = 0; j < i; ++j) {
        if (labels[j] == labels[i]) continue;
        double d2 = 0.0;
        for (int d = 0; d < axes; ++d) {
          long long v = tab[i].c[d] - tab[j].c[d];
          const long long P = a.P[d];
          v = ((v % P) + P) % P;
          if (v >= P / 2) v -= P;
          d2 += (double)v * (double)v;
        }
        const double rr = tab[i].t + tab[j].t;
        if (!(d2 > rr * rr)) return fail(HM_E_ARG, "spheres %d and %d of different phases overlap", j, i);
      }
    }
  }
  return HM_OK;
}

// The two-phase filter (labels == NULL) and the multi-phase one (labels
// 1..nlab per sphere, spheres of different labels must not overlap).
static int filter_impl(const hm_grid* grid, const hm_sphere* spheres, int n_spheres, const int* labels, int nlab,
                       double radius_vox, int subsamples, hm_rule rule, hm_prec prec, uint32_t* d_count,
                       void* d_frac, int32_t* d_incl, void* stream) {
  int rc;
  if (n_spheres < 0) return fail(HM_E_ARG, "n_spheres < 0");
  std::vector<LatSphere> tab((size_t)(n_spheres > 0 ? n_spheres : 1));
  FilterArgs a;
  if ((rc = filter_prepare(grid, spheres, n_spheres, labels, nlab, radius_vox, subsamples, rule, prec, d_count,
                           d_frac, tab.data(), a)))
    return rc;
  hipStream_t s = (hipStream_t)stream;
  LatSphere* dtab = nullptr;
  int* dlab = nullptr;
  const size_t tb = tab.size() * sizeof(LatSphere);
  if ((rc = device_alloc((void**)&dtab, tb, "sphere table"))) return rc;
  if (labels && (rc = device_alloc((void**)&dlab, (size_t)(n_spheres > 0 ? n_spheres : 1) * sizeof(int), "labels"))) {
    (void)hipFree(dtab);
    return rc;
  }
  hipError_t e = hipMemcpyAsync(dtab, tab.data(), tb, hipMemcpyHostToDevice, s);
  if (e == hipSuccess && labels && n_spheres > 0)
    e = hipMemcpyAsync(dlab, labels, (size_t)n_spheres * sizeof(int), hipMemcpyHostToDevice, s);
  a.sph = dtab;
  a.count = d_count;
  a.frac = d_frac;
  a.incl = labels ? nullptr : d_incl;
  a.lab = dlab;
  a.nlab = labels ? nlab : 1;
  if (e == hipSuccess) e = launch_filter(a, prec == HM_FP64, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  (void)hipFree(dtab);
  (void)hipFree(dlab);
  if (e != hipSuccess) return fail(HM_E_DEVICE, "filter: %s", hipGetErrorString(e));
  return HM_OK;
}

// ------------------------------------------------------ allocation-free filter
// hm_filter_noalloc stages the lattice sphere table in `scratch`, a
// file-scope device array (each GPU holds its own copy, at its own address),
// instead of a table allocated per call.  The host side uses a file-scope
// staging array of the same size; both are guarded by one mutex, so calls
// from several host threads queue on it.  Calls on one GPU share its array:
// a call that overlaps another one's kernel on that GPU (different streams)
// races on the table.
static __device__ __align__(256) unsigned char scratch[HM_FILTER_NOALLOC_MAX_SPHERES * sizeof(LatSphere)];
static_assert(sizeof(LatSphere) == 40, "lattice sphere layout");
static LatSphere g_noalloc_host[HM_FILTER_NOALLOC_MAX_SPHERES];
static std::mutex g_noalloc_mutex;
static constexpr int kMaxDevices = 64;
static void* g_scratch_ptr[kMaxDevices];  // device address of `scratch`, per device

int hm_filter_noalloc(const hm_grid* grid, const hm_sphere* spheres, int n_spheres, double radius_vox,
                      int subsamples, hm_rule rule, hm_prec prec, uint32_t* d_count, void* d_frac, int32_t* d_incl,
                      void* stream) {
  if (n_spheres < 0) return fail(HM_E_ARG, "n_spheres < 0");
  if (n_spheres > HM_FILTER_NOALLOC_MAX_SPHERES)
    return fail(HM_E_SIZE, "hm_filter_noalloc holds at most %d spheres (got %d)", HM_FILTER_NOALLOC_MAX_SPHERES,
                n_spheres);
  int dev = 0;
  HM_HIP(hipGetDevice(&dev));
  if (dev < 0 || dev >= kMaxDevices) return fail(HM_E_DEVICE, "device %d beyond the %d supported", dev, kMaxDevices);
  std::lock_guard<std::mutex> lock(g_noalloc_mutex);
  if (!g_scratch_ptr[dev]) {
    // first call on this device (it is current): the array's device address
    void* ptr = nullptr;
    const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !ptr) return fail(HM_E_DEVICE, "hipGetSymbolAddress(scratch): %s", hipGetErrorString(e));
    g_scratch_ptr[dev] = ptr;
  }
  FilterArgs a;
  int rc = filter_prepare(grid, spheres, n_spheres, nullptr, 1, radius_vox, subsamples, rule, prec, d_count, d_frac,
                          g_noalloc_host, a);
  if (rc) return rc;
  hipStream_t s = (hipStream_t)stream;
  LatSphere* dtab = static_cast<LatSphere*>(g_scratch_ptr[dev]);
  hipError_t e = hipSuccess;
  if (n_spheres > 0) e = hipMemcpyAsync(dtab, g_noalloc_host, (size_t)n_spheres * sizeof(LatSphere),
                                        hipMemcpyHostToDevice, s);
  a.sph = dtab;
  a.count = d_count;
  a.frac = d_frac;
  a.incl = d_incl;
  a.lab = nullptr;
  a.nlab = 1;
  if (e == hipSuccess) e = launch_filter(a, prec == HM_FP64, s);
  // the host staging array is reused by the next call
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  if (e != hipSuccess) return fail(HM_E_DEVICE, "filter: %s", hipGetErrorString(e));
  return HM_OK;
}

int hm_filter(const hm_grid* grid, const hm_sphere* spheres, int n_spheres, double radius_vox, int subsamples,
              hm_rule rule, hm_prec prec, uint32_t* d_count, void* d_frac, int32_t* d_incl, void* stream) {
  return filter_impl(grid, spheres, n_spheres, nullptr, 1, radius_vox, subsamples, rule, prec, d_count, d_frac,
                     d_incl, stream);
}

int hm_filter_phases(const hm_grid* grid, const hm_sphere* spheres, const int32_t* labels, int n_spheres,
                     int n_phases, double radius_vox, int subsamples, hm_rule rule, hm_prec prec, uint32_t* d_count,
                     void* d_frac, void* stream) {
  if (n_phases < 2 || n_phases > 8) return fail(HM_E_ARG, "n_phases must be in 2..8");
  if (n_spheres > 0 && !labels) return fail(HM_E_ARG, "labels is NULL");
  return filter_impl(grid, spheres, n_spheres, labels, n_phases - 1, radius_vox, subsamples, rule, prec, d_count,
                     d_frac, nullptr, stream);
}

// A multi-phase cell as a ProblemIn.
static ProblemIn phases_problem(const hm_grid* grid, const hm_iso* phases, int n_phases, hm_rule rule,
                                const void* d_frac) {
  ProblemIn d = make_problem(grid, nullptr, rule, d_frac, nullptr, nullptr, 0);
  d.nphase = n_phases;
  if (phases && n_phases >= 2 && n_phases <= 8)
    for (int p = 0; p < n_phases; ++p) d.ph[p] = phases[p];
  return d;
}

int hm_solve_phases(const hm_grid* grid, const hm_iso* phases, int n_phases, hm_rule rule, const void* d_frac,
                    const double* E, int n_load, const hm_solve_opts* opts, void* d_eps, double* sig_mean,
                    hm_report* rep, void* stream) {
  const auto t0 = std::chrono::steady_clock::now();
  if (!phases) return fail(HM_E_ARG, "phases is NULL");
  if (n_phases < 2 || n_phases > 8) return fail(HM_E_ARG, "n_phases must be in 2..8");
  if (!E || !sig_mean) return fail(HM_E_ARG, "E and sig_mean must not be NULL");
  Plan* p = nullptr;
  int rc = solve_one(phases_problem(grid, phases, n_phases, rule, d_frac), E, n_load, opts, d_eps,
                     (hipStream_t)stream, &p);
  if (rc) return rc;
  const double secs = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
  int worst = HM_OK;
  for (int l = 0; l < n_load; ++l) {
    const SolverState& st = p->state_host[l];
    for (int c = 0; c < 6; ++c) sig_mean[6 * l + c] = st.sig[c];
    const int status = load_status(st);
    if (rep) rep[l] = hm_report{st.iters, status, st.err, st.err0, secs};
    worst = std::max(worst, status);
  }
  return worst;
}

int hm_effective_tensor_phases(const hm_grid* grid, const hm_iso* phases, int n_phases, hm_rule rule,
                               const void* d_frac, const hm_solve_opts* opts, double* C_mandel, void* d_eps,
                               hm_report* rep, void* stream) {
  const auto t0 = std::chrono::steady_clock::now();
  int rc;
  if ((rc = check_grid(grid))) return rc;
  if (!phases) return fail(HM_E_ARG, "phases is NULL");
  if (n_phases < 2 || n_phases > 8) return fail(HM_E_ARG, "n_phases must be in 2..8");
  if (!C_mandel) return fail(HM_E_ARG, "C_mandel is NULL");
  double E[36];
  const int* idx = nullptr;
  const int k = unit_loads(grid->dim, E, &idx);
  Plan* p = nullptr;
  rc = solve_one(phases_problem(grid, phases, n_phases, rule, d_frac), E, k, opts, d_eps, (hipStream_t)stream, &p);
  if (rc) return rc;
  const double secs = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
  assemble_mandel(k, idx, p->state_host, C_mandel);
  int worst = HM_OK;
  for (int l = 0; l < k; ++l) {
    const SolverState& st = p->state_host[l];
    const int status = load_status(st);
    if (rep) rep[l] = hm_report{st.iters, status, st.err, st.err0, secs};
    worst = std::max(worst, status);
  }
  return worst;
}

int hm_solve(const hm_grid* grid, const hm_iso phases[2], hm_rule rule, const void* d_frac, const int32_t* d_incl,
             const hm_sphere* spheres, int n_spheres, const double* E, int n_load, const hm_solve_opts* opts,
             void* d_eps, double* sig_mean, hm_report* rep, void* stream) {
  const auto t0 = std::chrono::steady_clock::now();
  if (!phases) return fail(HM_E_ARG, "phases is NULL");
  if (!E || !sig_mean) return fail(HM_E_ARG, "E and sig_mean must not be NULL");
  Plan* p = nullptr;
  int rc = solve_one(make_problem(grid, phases, rule, d_frac, d_incl, spheres, n_spheres), E, n_load, opts, d_eps,
                     (hipStream_t)stream, &p);
  if (rc) return rc;
  const double secs = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
  int worst = HM_OK;
  for (int l = 0; l < n_load; ++l) {
    const SolverState& st = p->state_host[l];
    for (int c = 0; c < 6; ++c) sig_mean[6 * l + c] = st.sig[c];
    const int status = load_status(st);
    if (rep) rep[l] = hm_report{st.iters, status, st.err, st.err0, secs};
    worst = std::max(worst, status);
  }
  return worst;
}

int hm_effective_tensor(const hm_grid* grid, const hm_iso phases[2], hm_rule rule, const void* d_frac,
                        const int32_t* d_incl, const hm_sphere* spheres, int n_spheres, const hm_solve_opts* opts,
                        double* C_mandel, void* d_eps, hm_report* rep, void* stream) {
  const auto t0 = std::chrono::steady_clock::now();
  int rc;
  if ((rc = check_grid(grid))) return rc;
  if (!phases) return fail(HM_E_ARG, "phases is NULL");
  if (!C_mandel) return fail(HM_E_ARG, "C_mandel is NULL");
  double E[36];
  const int* idx = nullptr;
  const int k = unit_loads(grid->dim, E, &idx);
  Plan* p = nullptr;
  rc = solve_one(make_problem(grid, phases, rule, d_frac, d_incl, spheres, n_spheres), E, k, opts, d_eps,
                 (hipStream_t)stream, &p);
  if (rc) return rc;
  const double secs = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
  assemble_mandel(k, idx, p->state_host, C_mandel);
  int worst = HM_OK;
  for (int l = 0; l < k; ++l) {
    const SolverState& st = p->state_host[l];
    const int status = load_status(st);
    if (rep) rep[l] = hm_report{st.iters, status, st.err, st.err0, secs};
    worst = std::max(worst, status);
  }
  return worst;
}

int hm_conduct_solve(const hm_grid* grid, const double k[2], hm_rule rule, const void* d_frac,
                     const int32_t* d_incl, const hm_sphere* spheres, int n_spheres, const double* G, int n_load,
                     const hm_solve_opts* opts, void* d_grad, double* flux_mean, hm_report* rep, void* stream) {
  const auto t0 = std::chrono::steady_clock::now();
  if (!k) return fail(HM_E_ARG, "k is NULL");
  if (!G || !flux_mean) return fail(HM_E_ARG, "G and flux_mean must not be NULL");
  ProblemIn d = make_problem(grid, nullptr, rule, d_frac, d_incl, spheres, n_spheres);
  d.cond = 1;
  d.k[0] = k[0];
  d.k[1] = k[1];
  Plan* p = nullptr;
  int rc = solve_cond(d, G, n_load, opts, d_grad, (hipStream_t)stream, &p);
  if (rc) return rc;
  const double secs = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
  int worst = HM_OK;
  for (int l = 0; l < n_load; ++l) {
    const SolverState& st = p->state_host[l];
    for (int c = 0; c < 3; ++c) flux_mean[3 * l + c] = st.sig[c];
    const int status = load_status(st);
    if (rep) rep[l] = hm_report{st.iters, status, st.err, st.err0, secs};
    worst = std::max(worst, status);
  }
  return worst;
}

int hm_effective_conductivity(const hm_grid* grid, const double k[2], hm_rule rule, const void* d_frac,
                              const int32_t* d_incl, const hm_sphere* spheres, int n_spheres,
                              const hm_solve_opts* opts, double* K, void* d_grad, hm_report* rep, void* stream) {
  const auto t0 = std::chrono::steady_clock::now();
  int rc;
  if ((rc = check_grid(grid))) return rc;
  if (!k) return fail(HM_E_ARG, "k is NULL");
  if (!K) return fail(HM_E_ARG, "K is NULL");
  const int nd = grid->dim == 2 ? 2 : 3;
  double G[9] = {0.0};
  for (int J = 0; J < nd; ++J) G[3 * J + J] = 1.0;
  ProblemIn d = make_problem(grid, nullptr, rule, d_frac, d_incl, spheres, n_spheres);
  d.cond = 1;
  d.k[0] = k[0];
  d.k[1] = k[1];
  Plan* p = nullptr;
  rc = solve_cond(d, G, nd, opts, d_grad, (hipStream_t)stream, &p);
  if (rc) return rc;
  const double secs = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
  int worst = HM_OK;
  for (int J = 0; J < nd; ++J) {
    const SolverState& st = p->state_host[J];
    for (int I = 0; I < nd; ++I) K[I * nd + J] = st.sig[I];
    const int status = load_status(st);
    if (rep) rep[J] = hm_report{st.iters, status, st.err, st.err0, secs};
    worst = std::max(worst, status);
  }
  return worst;
}

int hm_effective_tensor_batch(const hm_problem* problems, int n_problems, const hm_solve_opts* opts,
                              double* C_mandel, hm_report* rep, void* stream) {
  const auto t0 = std::chrono::steady_clock::now();
  int rc;
  if (!problems || n_problems < 1) return fail(HM_E_ARG, "no problems");
  if (!C_mandel) return fail(HM_E_ARG, "C_mandel is NULL");
  if ((rc = check_opts(opts))) return rc;
  if (opts->profile) return fail(HM_E_ARG, "profiling is not available for batches");
  if (opts->method != HM_FIXED_POINT) return fail(HM_E_ARG, "batches use the fixed-point method");
  std::vector<ProblemIn> all((size_t)n_problems);
  for (int q = 0; q < n_problems; ++q) {
    const hm_problem& h = problems[q];
    all[q] = make_problem(&h.grid, h.phases, h.rule, h.d_frac, h.d_incl, h.spheres, h.n_spheres);
    if ((rc = check_problem(all[q]))) {
      g_last_error = "problem " + std::to_string(q) + ": " + g_last_error;
      return rc;
    }
  }
  // group the problems by grid, keeping their order within a group
  std::vector<Group> G;
  std::map<std::tuple<int, int, int, int>, int> gid;
  std::vector<int> where((size_t)n_problems);
  for (int q = 0; q < n_problems; ++q) {
    const hm_grid& g = all[q].grid;
    auto key = std::make_tuple(g.dim, g.n[0], g.n[1], g.n[2]);
    auto it = gid.find(key);
    if (it == gid.end()) {
      gid[key] = (int)G.size();
      G.emplace_back();
      it = gid.find(key);
    }
    where[q] = it->second;
    G[it->second].probs.push_back(q);
  }
  for (Group& g : G) {
    const ProblemIn& d0 = all[g.probs[0]];
    double E[36];
    const int* idx = nullptr;
    const int k = unit_loads(d0.grid.dim, E, &idx);
    const int nl = k * (int)g.probs.size();
    if (nl > kMaxLoads) return fail(HM_E_ARG, "more than %d load cases on one grid", kMaxLoads);
    if ((rc = get_plan(opts->prec == HM_FP64, d0.grid.n, d0.grid.dim, nl, PHYS_ELASTIC, &g.p))) return rc;
    g.loads.resize(nl);
    for (int j = 0; j < (int)g.probs.size(); ++j)
      for (int J = 0; J < k; ++J) {
        LoadParams& L = g.loads[(size_t)j * k + J];
        for (int c = 0; c < 6; ++c) L.E[c] = E[6 * J + c];
        L.prob = j;
        L.pad = 0;
      }
  }
  if ((rc = run_groups(G, all, opts, (hipStream_t)stream))) return rc;
  const double secs = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
  int worst = HM_OK;
  size_t cofs = 0, rofs = 0;
  for (int q = 0; q < n_problems; ++q) {
    const Group& g = G[where[q]];
    int j = 0;
    while (g.probs[j] != q) ++j;
    double E[36];
    const int* idx = nullptr;
    const int k = unit_loads(all[q].grid.dim, E, &idx);
    const SolverState* st = g.p->state_host + (size_t)j * k;
    assemble_mandel(k, idx, st, C_mandel + cofs);
    for (int l = 0; l < k; ++l) {
      const int status = load_status(st[l]);
      if (rep) rep[rofs + l] = hm_report{st[l].iters, status, st[l].err, st[l].err0, secs};
      worst = std::max(worst, status);
    }
    cofs += (size_t)k * k;
    rofs += (size_t)k;
  }
  return worst;
}

int hm_solve_adjoint(const hm_grid* grid, const hm_iso phases[2], hm_rule rule, const void* d_frac,
                     const int32_t* d_incl, const hm_sphere* spheres, int n_spheres, hm_prec prec,
                     const double* dLdC, const void* d_eps, int n_load, double* dLdphase, void* d_dLdfrac,
                     void* stream) {
  int rc;
  if ((rc = check_grid(grid))) return rc;
  if ((rc = check_phases(phases))) return rc;
  if ((rc = check_spheres(grid, spheres, n_spheres))) return rc;
  if (rule < HM_RULE_NONE || rule > HM_RULE_LAMINATE) return fail(HM_E_ARG, "unknown rule %d", (int)rule);
  if (prec != HM_FP64 && prec != HM_MIXED) return fail(HM_E_ARG, "unknown precision");
  const int k = grid->dim == 2 ? 3 : 6;
  if (n_load != k) return fail(HM_E_ARG, "n_load must be %d (the unit Mandel strains)", k);
  if (!d_frac || !d_eps || !dLdC || !dLdphase) return fail(HM_E_ARG, "NULL input or output");
  if (rule == HM_RULE_LAMINATE && !d_incl) return fail(HM_E_ARG, "the 2-layer rule needs d_incl");
  for (int i = 0; i < k * k; ++i)
    if (!isfinite(dLdC[i])) return fail(HM_E_ARG, "dLdC has a non-finite entry");
  hipStream_t s = (hipStream_t)stream;
  const long long N = (long long)grid->n[0] * grid->n[1] * grid->n[2];
  const int blocks = (int)((N + 255) / 256);
  HillArgs a;
  memset(&a, 0, sizeof a);
  a.eps = d_eps;
  a.frac = d_frac;
  a.incl = d_incl;
  a.nsph = n_spheres;
  a.dim = grid->dim;
  a.n_load = n_load;
  a.rule = (int)rule;
  for (int d = 0; d < 3; ++d) a.n[d] = grid->n[d];
  for (int p = 0; p < 2; ++p) {
    a.pl[p] = phases[p].lambda;
    a.pm[p] = phases[p].mu;
  }
  for (int i = 0; i < k * k; ++i) a.G[i] = dLdC[i];
  a.dfrac = d_dLdfrac;
  double* dsph = nullptr;
  double* dpart = nullptr;
  std::vector<double> sph(4 * (size_t)(n_spheres > 0 ? n_spheres : 1), 0.0);
  for (int q = 0; q < n_spheres; ++q) {
    for (int c = 0; c < 3; ++c) sph[4 * q + c] = spheres[q].c[c];
    sph[4 * q + 3] = spheres[q].r;
  }
  if ((rc = device_alloc((void**)&dsph, sph.size() * sizeof(double), "sphere table"))) return rc;
  if ((rc = device_alloc((void**)&dpart, (size_t)blocks * 4 * sizeof(double), "gradient partials"))) {
    (void)hipFree(dsph);
    return rc;
  }
  std::vector<double> part((size_t)blocks * 4);
  hipError_t e = hipMemcpyAsync(dsph, sph.data(), sph.size() * sizeof(double), hipMemcpyHostToDevice, s);
  a.sph = dsph;
  a.part = dpart;
  if (e == hipSuccess) e = launch_hill(a, prec == HM_FP64, blocks, s);
  if (e == hipSuccess)
    e = hipMemcpyAsync(part.data(), dpart, part.size() * sizeof(double), hipMemcpyDeviceToHost, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  (void)hipFree(dsph);
  (void)hipFree(dpart);
  if (e != hipSuccess) return fail(HM_E_DEVICE, "adjoint: %s", hipGetErrorString(e));
  for (int q = 0; q < 4; ++q) {
    double sum = 0.0, comp = 0.0;
    for (int b = 0; b < blocks; ++b) {
      const double x = part[(size_t)b * 4 + q];
      const double t = sum + x;
      comp += fabs(sum) >= fabs(x) ? (sum - t) + x : (x - t) + sum;
      sum = t;
    }
    dLdphase[q] = (sum + comp) / (double)N;
  }
  return HM_OK;
}

}  // extern "C"
