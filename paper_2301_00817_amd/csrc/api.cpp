// C-ABI of lesjet (declared in include/lesjet.h): argument validation,
// context and device-memory ownership, and the RK5 driver that chains the
// ghost fill, residual and stage-update kernels on the caller's stream.
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <new>
#include <string>

#include <rocprofiler-sdk-roctx/roctx.h>
#include <vector>

#include "lesjet.h"
#include "launch.hpp"

using namespace lesjet;

// Device scratch of les_diagnostics_noalloc: the per-block partial sums of
// the conservation totals (5 per block, at most DIAG_MAX_PARTIALS blocks), in
// a static array that every GPU the library runs on holds until the process
// ends.  Host code never passes `scratch` itself (on the host it names a
// stand-in, not the device array): it takes each device's address once, with
// that device current, and keeps it in g_scratch_ptr.
constexpr size_t NOALLOC_SCRATCH_DOUBLES = 5 * (size_t)DIAG_MAX_PARTIALS;   // 80 KiB
static __device__ __align__(256) double scratch[NOALLOC_SCRATCH_DOUBLES];

constexpr int MAX_DEVICES = 64;
static std::mutex g_scratch_mu;
static double* g_scratch_ptr[MAX_DEVICES];

// The address of `scratch` on the current device `dev` (taken on the first
// call for that device).
static hipError_t scratch_address(int dev, double** out) {
  *out = nullptr;
  if (dev < 0 || dev >= MAX_DEVICES) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* ptr = nullptr;
    const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    g_scratch_ptr[dev] = (double*)ptr;
  }
  *out = g_scratch_ptr[dev];
  return hipSuccess;
}

struct les_ctx {
  les_params p;
  Grid g;
  CGrid cg;
  Phys<double> ph64;
  Phys<float> ph32;
  int device = 0;
  int num_cu = 256;
  int kc = 16;                 // k-chunk of the fused kernel
  double* coords = nullptr;    // padded coordinates (3 ghost layers), freed by les_metrics
  void* M = nullptr;           // metrics, 10 padded variables of the storage type
  double* inflow = nullptr;    // entrance target primitives (5, nth, nr)
  void* stage[3] = {nullptr, nullptr, nullptr};   // RK stage states (storage type; the
                                                 // third for FP32 with held boundary values)
  void* visc = nullptr;        // held mu + mu_sgs and conductivity (2 padded variables)
  double* dyn_scr = nullptr;   // dynamic SGS model: scratch (DYN_SCRATCH_VARS variables, FP64),
  double* dyn_part = nullptr;  // per-block sums
  double* dyn = nullptr;       // and coefficients (DYN_COEF_DOUBLES)
  void* R = nullptr;           // residual buffer (storage type)
  void* PT = nullptr;          // point-quantity scratch of the two-pass residual
  double* part = nullptr;      // per-block partial sums of the diagnostics
  double* part_static = nullptr;   // the same in this device's static scratch (no allocation)
  double* adj = nullptr;       // residual-adjoint scratch (VJP_SCRATCH_VARS variables, FP64)
  double* adj_stage = nullptr; // RK5-step adjoint: stage states 1..4 and one cotangent (25 vars)
  unsigned long long* maxbits = nullptr;
  double* dt = nullptr;
  int* flag = nullptr;
  bool metrics_done = false;
  bool inflow_set = false;
  size_t bytes = 0;
  std::string err;
  // kernel timing (les_profile)
  bool prof = false;
  std::vector<hipEvent_t> ev;   // start/stop pairs
  size_t ev_used = 0;           // pairs recorded since the last read
};

// Record the start event of a timed launch; returns the pair index or -1.
static long prof_begin(les_ctx* c, hipStream_t s) {
  if (!c->prof) return -1;
  if (2 * (c->ev_used + 1) > c->ev.size()) {
    hipEvent_t a, b;
    if (hipEventCreate(&a) != hipSuccess) return -1;
    if (hipEventCreate(&b) != hipSuccess) { (void)hipEventDestroy(a); return -1; }
    c->ev.push_back(a);
    c->ev.push_back(b);
  }
  const long k = (long)c->ev_used++;
  if (hipEventRecord(c->ev[2 * k], s) != hipSuccess) { --c->ev_used; return -1; }
  return k;
}

static void prof_end(les_ctx* c, long k, hipStream_t s) {
  if (k >= 0) (void)hipEventRecord(c->ev[2 * k + 1], s);
}

// Host-side range (ROCTx) around an API call or an RK stage, for
// rocprofv3 --marker-trace: it spans the enqueueing of the call's kernels
// on the host timeline (inert when no tool is attached).
struct Range {
  explicit Range(const char* name) { roctxRangePushA(name); }
  ~Range() { roctxRangePop(); }
  Range(const Range&) = delete;
  Range& operator=(const Range&) = delete;
};

static thread_local std::string t_err;

static int fail(les_ctx* c, int code, const std::string& msg) {
  if (c) c->err = msg;
  t_err = msg;
  return code;
}

static int hip_fail(les_ctx* c, hipError_t e, const char* where) {
  return fail(c, LES_EHIP, std::string(where) + ": " + hipGetErrorString(e));
}

#define HIP_TRY(c, expr)                                  \
  do {                                                    \
    hipError_t e_ = (expr);                               \
    if (e_ != hipSuccess) return hip_fail((c), e_, #expr); \
  } while (0)

static bool finite_pos(double x) { return std::isfinite(x) && x > 0.0; }

static int validate(const les_params* p, std::string& why) {
  if (!p) { why = "params is NULL"; return LES_EINVAL; }
  if (p->nx < 5 || p->nr < 5 || p->nth < 5) { why = "each of nx, nr, nth must be >= 5"; return LES_EINVAL; }
  const int* b = p->bc;
  for (int f = 0; f < 6; ++f)
    if (b[f] < LES_BC_PERIODIC || b[f] > LES_BC_AXIS_NODE) { why = "unknown boundary kind"; return LES_EINVAL; }
  for (int f = 0; f < 6; ++f)
    if (b[f] == LES_BC_AXIS_NODE && f != 2) { why = "axis_node is an eta- condition"; return LES_EINVAL; }
  for (int d = 0; d < 3; ++d)
    if ((b[2 * d] == LES_BC_PERIODIC) != (b[2 * d + 1] == LES_BC_PERIODIC)) {
      why = "a periodic direction must be periodic on both faces";
      return LES_EINVAL;
    }
  if (!(b[0] == LES_BC_PERIODIC || b[0] == LES_BC_INFLOW)) { why = "xi- must be periodic or inflow"; return LES_EINVAL; }
  if (!(b[1] == LES_BC_PERIODIC || b[1] == LES_BC_OUTFLOW)) { why = "xi+ must be periodic or outflow"; return LES_EINVAL; }
  if (!(b[2] == LES_BC_PERIODIC || b[2] == LES_BC_AXIS || b[2] == LES_BC_AXIS_NODE)) {
    why = "eta- must be periodic, axis or axis_node";
    return LES_EINVAL;
  }
  if (!(b[3] == LES_BC_PERIODIC || b[3] == LES_BC_FARFIELD)) { why = "eta+ must be periodic or far field"; return LES_EINVAL; }
  if (b[4] != LES_BC_PERIODIC || b[5] != LES_BC_PERIODIC) { why = "zeta must be periodic"; return LES_EINVAL; }
  if ((b[2] == LES_BC_AXIS || b[2] == LES_BC_AXIS_NODE) && (p->nth % 2) != 0) {
    why = "the axis conditions need an even nth";
    return LES_EINVAL;
  }
  if (!(std::isfinite(p->gamma) && p->gamma > 1.0)) { why = "gamma must be > 1"; return LES_EINVAL; }
  if (!finite_pos(p->Pr) || !finite_pos(p->Pr_sgs)) { why = "Prandtl numbers must be > 0"; return LES_EINVAL; }
  if (!(std::isfinite(p->visc_coef) && p->visc_coef >= 0.0)) { why = "visc_coef must be >= 0"; return LES_EINVAL; }
  if (!finite_pos(p->suth_S)) { why = "suth_S must be > 0"; return LES_EINVAL; }
  if (!(std::isfinite(p->Cs) && p->Cs >= 0.0)) { why = "Cs must be >= 0"; return LES_EINVAL; }
  if (!(std::isfinite(p->k2) && p->k2 >= 0.0 && std::isfinite(p->k4) && p->k4 >= 0.0)) { why = "k2, k4 must be >= 0"; return LES_EINVAL; }
  if (!finite_pos(p->cfl)) { why = "cfl must be > 0"; return LES_EINVAL; }
  for (int l = 0; l < 5; ++l)
    if (!std::isfinite(p->rk_alpha[l])) { why = "rk_alpha must be finite"; return LES_EINVAL; }
  for (int d = 0; d < 3; ++d)
    for (int c = 0; c < 3; ++c)
      if (!std::isfinite(p->period[d][c])) { why = "period must be finite"; return LES_EINVAL; }
  if (b[3] == LES_BC_FARFIELD) {
    for (int c = 0; c < 5; ++c)
      if (!std::isfinite(p->ref_prim[c])) { why = "ref_prim must be finite"; return LES_EINVAL; }
    if (!(p->ref_prim[0] > 0.0 && p->ref_prim[4] > 0.0)) { why = "ref_prim needs rho > 0 and p > 0"; return LES_EINVAL; }
  }
  if (b[1] == LES_BC_OUTFLOW && !finite_pos(p->p_exit)) { why = "p_exit must be > 0"; return LES_EINVAL; }
  if (p->sgs_model != LES_SGS_NONE && p->sgs_model != LES_SGS_SMAGORINSKY &&
      p->sgs_model != LES_SGS_VREMAN && p->sgs_model != LES_SGS_DYNAMIC) {
    why = "unknown sgs_model";
    return LES_EINVAL;
  }
  if (p->sgs_model != LES_SGS_NONE && p->visc_coef == 0.0 &&
      (p->Cs != 0.0 || p->sgs_model == LES_SGS_DYNAMIC)) {
    why = "an SGS model needs visc_coef > 0 (mu_sgs is in units of the jet viscosity)";
    return LES_EINVAL;
  }
  if (p->sgs_model == LES_SGS_DYNAMIC && b[2] == LES_BC_AXIS_NODE) {
    // the test filter would average the axis row, where J^-1 = 0 leaves the
    // strain undefined
    why = "the dynamic SGS model does not cover the axis_node centerline";
    return LES_EUNSUPPORTED;
  }
  if (p->precision != LES_FP64 && p->precision != LES_FP32_STORAGE) { why = "unknown precision"; return LES_EINVAL; }
  if (p->schedule != LES_SCHEDULE_STAGE && p->schedule != LES_SCHEDULE_STEP) {
    why = "unknown schedule";
    return LES_EINVAL;
  }
  return LES_OK;
}

static int make_layout(const les_params* p, Grid& g, CGrid& cg, std::string& why) {
  const long long pitch = ((long long)p->nx + 2 * NG + 15) / 16 * 16;
  const long long plane = pitch * (p->nr + 2 * NG);
  const long long vs = plane * (p->nth + 2 * NG);
  const long long cpitch = (long long)p->nx + 2 * NGC;
  const long long cplane = cpitch * (p->nr + 2 * NGC);
  const long long cvs = cplane * (p->nth + 2 * NGC);
  if (vs > 2147483647LL || cvs > 2147483647LL) {
    why = "one padded variable exceeds 2^31 - 1 elements";
    return LES_EUNSUPPORTED;
  }
  // With at least nine planes per variable (nth >= 5) a plane of FP64 data
  // then stays below 2^31 bytes: the byte range of the stage kernel's
  // per-plane buffer resources.
  g.nx = p->nx; g.nr = p->nr; g.nth = p->nth;
  g.pitch = (int)pitch; g.plane = (int)plane; g.vs = (int)vs;
  cg.nx = p->nx; cg.nr = p->nr; cg.nth = p->nth;
  cg.pitch = (int)cpitch; cg.plane = (int)cplane; cg.vs = (int)cvs;
  return LES_OK;
}

template <typename T>
static Phys<T> make_phys(const les_params* p) {
  Phys<T> ph;
  ph.gamma = (T)p->gamma;
  ph.gm1 = (T)(p->gamma - 1.0);
  ph.igm1 = (T)(1.0 / (p->gamma - 1.0));
  ph.Pr_inv = (T)(1.0 / p->Pr);
  ph.Prs_inv = (T)(1.0 / p->Pr_sgs);
  ph.Cv = (T)p->visc_coef;
  ph.suth = (T)p->suth_S;
  ph.suth1 = (T)(1.0 + p->suth_S);
  ph.viscous = p->visc_coef != 0.0;
  // the dynamic model takes no constant; its coefficients are set per launch
  ph.sgs = ph.viscous && (p->Cs != 0.0 || p->sgs_model == LES_SGS_DYNAMIC) ? p->sgs_model : 0;
  // Vreman's constant is c = 2.5 Cs^2
  const double c = p->sgs_model == LES_SGS_VREMAN ? 2.5 * p->Cs * p->Cs : p->Cs * p->Cs;
  ph.sgs_coef = ph.sgs && ph.sgs != LES_SGS_DYNAMIC ? (T)(c / p->visc_coef) : T(0);
  ph.iso_coef = T(0);
  ph.k2 = (T)p->k2;
  ph.k4 = (T)p->k4;
  ph.axis_node = p->bc[2] == LES_BC_AXIS_NODE;
  for (int d = 0; d < 3; ++d)
    for (int s = 0; s < 2; ++s) {
      const int b = p->bc[2 * d + s];
      ph.phys_face[d][s] = (b == LES_BC_INFLOW || b == LES_BC_OUTFLOW || b == LES_BC_FARFIELD);
    }
  return ph;
}

static size_t storage_size(const les_params* p) {
  return p->precision == LES_FP32_STORAGE ? sizeof(float) : sizeof(double);
}

static void free_all(les_ctx* c) {
  void* ptrs[] = {c->coords, c->M, c->inflow, c->stage[0], c->stage[1], c->stage[2], c->visc,
                  c->dyn_scr, c->dyn_part, c->dyn, c->R, c->PT, c->part, c->adj, c->adj_stage,
                  c->maxbits, c->dt, c->flag};
  for (void* q : ptrs)
    if (q) (void)hipFree(q);
  c->coords = nullptr; c->M = nullptr; c->inflow = nullptr;
  c->stage[0] = c->stage[1] = c->stage[2] = nullptr;
  c->visc = nullptr;
  c->dyn_scr = nullptr; c->dyn_part = nullptr; c->dyn = nullptr;
  c->R = nullptr; c->PT = nullptr; c->part = nullptr;
  c->adj = nullptr; c->adj_stage = nullptr;
  c->maxbits = nullptr; c->dt = nullptr; c->flag = nullptr;
}

static int dalloc(les_ctx* c, void** ptr, size_t bytes, const char* what) {
  if (*ptr) return LES_OK;
  hipError_t e = hipMalloc(ptr, bytes);
  if (e != hipSuccess) {
    *ptr = nullptr;
    (void)hipGetLastError();
    return fail(c, LES_ENOMEM, std::string("device allocation of ") + what + " (" +
                                   std::to_string(bytes) + " bytes) failed: " + hipGetErrorString(e));
  }
  c->bytes += bytes;
  // test hook: LESJET_POISON=1 fills new buffers with NaN bit patterns, so
  // a kernel that reads memory no pass has written shows up in the results
  if (const char* ps = std::getenv("LESJET_POISON")) {
    if (ps[0] == '1') {
      e = hipMemset(*ptr, 0xFF, bytes);
      if (e != hipSuccess) return hip_fail(c, e, "poisoning a new buffer");
    }
  }
  return LES_OK;
}

// The exported functions below take C linkage from their declarations in
// lesjet.h.

int les_validate(const les_params* p) {
  std::string why;
  const int r = validate(p, why);
  return r == LES_OK ? r : fail(nullptr, r, why);
}

int les_layout(const les_params* p, int64_t* pitch, int64_t dims[3], int64_t* var_stride) {
  std::string why;
  int r = validate(p, why);
  if (r != LES_OK) return fail(nullptr, r, why);
  Grid g;
  CGrid cg;
  r = make_layout(p, g, cg, why);
  if (r != LES_OK) return fail(nullptr, r, why);
  if (pitch) *pitch = g.pitch;
  if (dims) { dims[0] = p->nth + 2 * NG; dims[1] = p->nr + 2 * NG; dims[2] = g.pitch; }
  if (var_stride) *var_stride = g.vs;
  return LES_OK;
}

int les_device_bytes(const les_params* p, size_t* bytes) {
  std::string why;
  int r = validate(p, why);
  if (r != LES_OK) return fail(nullptr, r, why);
  if (!bytes) return fail(nullptr, LES_EINVAL, "bytes is NULL");
  Grid g;
  CGrid cg;
  r = make_layout(p, g, cg, why);
  if (r != LES_OK) return fail(nullptr, r, why);
  const size_t ts = storage_size(p);
  // metrics + two stage states (the two-pass reference form adds 21 scratch
  // variables when it is used); the per-step schedule adds the two held
  // viscosities and, in FP32, a third stage state
  size_t vars = 10 + 5 + 5;
  if (p->sgs_model == LES_SGS_DYNAMIC && p->visc_coef != 0.0)
    vars += (size_t)DYN_SCRATCH_VARS * sizeof(double) / ts;
  if (p->schedule == LES_SCHEDULE_STEP) {
    if (p->visc_coef != 0.0) vars += 2;
    if (p->precision == LES_FP32_STORAGE) vars += 5;
  }
  *bytes = (size_t)g.vs * ts * vars + (size_t)5 * p->nth * p->nr * sizeof(double);
  return LES_OK;
}

// Host table X[nx], R[nr], cos(theta)[nth], sin(theta)[nth] of a cylindrical
// product mesh; the maps may be host or device arrays.  The angle functions
// are those of the host C library, so a caller that forms its own
// coordinates with the same functions gets the same mesh bitwise.
static int product_table(const les_params* p, const double* X, const double* R, const double* TH,
                         std::vector<double>& tab, std::string& why) {
  const size_t nx = (size_t)p->nx, nr = (size_t)p->nr, nth = (size_t)p->nth;
  tab.assign(nx + nr + 2 * nth, 0.0);
  std::vector<double> th(nth);
  hipError_t e = hipMemcpy(tab.data(), X, nx * sizeof(double), hipMemcpyDefault);
  if (e == hipSuccess) e = hipMemcpy(tab.data() + nx, R, nr * sizeof(double), hipMemcpyDefault);
  if (e == hipSuccess) e = hipMemcpy(th.data(), TH, nth * sizeof(double), hipMemcpyDefault);
  if (e != hipSuccess) {
    (void)hipGetLastError();
    why = std::string("reading the 1-D maps: ") + hipGetErrorString(e);
    return LES_EHIP;
  }
  for (size_t k = 0; k < nx + nr; ++k)
    if (!std::isfinite(tab[k])) { why = "X and R must be finite"; return LES_EINVAL; }
  for (size_t k = 0; k < nth; ++k) {
    if (!std::isfinite(th[k])) { why = "TH must be finite"; return LES_EINVAL; }
    tab[nx + nr + k] = std::cos(th[k]);
    tab[nx + nr + nth + k] = std::sin(th[k]);
  }
  return LES_OK;
}

int les_init_grid(les_ctx** out, const les_params* p, const double* xyz, const double* X,
                  const double* R, const double* TH, void* stream) {
  const Range range("les_init_grid");
  if (!out) return fail(nullptr, LES_EINVAL, "out is NULL");
  *out = nullptr;
  std::string why;
  int r = validate(p, why);
  if (r != LES_OK) return fail(nullptr, r, why);
  const bool maps = X || R || TH;
  if (maps && !(X && R && TH)) return fail(nullptr, LES_EINVAL, "X, R and TH go together");
  if (!xyz == !maps) return fail(nullptr, LES_EINVAL, "give either xyz or the maps X, R, TH");
  std::vector<double> tab;
  if (maps) {
    r = product_table(p, X, R, TH, tab, why);
    if (r != LES_OK) return fail(nullptr, r, why);
  }
  les_ctx* c = new (std::nothrow) les_ctx();
  if (!c) return fail(nullptr, LES_ENOMEM, "host allocation failed");
  c->p = *p;
  r = make_layout(p, c->g, c->cg, why);
  if (r != LES_OK) { delete c; return fail(nullptr, r, why); }
  c->ph64 = make_phys<double>(p);
  c->ph32 = make_phys<float>(p);
  hipError_t e = hipGetDevice(&c->device);
  if (e != hipSuccess) { delete c; return hip_fail(nullptr, e, "hipGetDevice"); }
  // once per device, with the device current: the address of the static
  // scratch of the entry points that allocate nothing
  e = scratch_address(c->device, &c->part_static);
  if (e != hipSuccess) { delete c; return hip_fail(nullptr, e, "hipGetSymbolAddress(scratch)"); }
  e = hipDeviceGetAttribute(&c->num_cu, hipDeviceAttributeMultiprocessorCount, c->device);
  if (e != hipSuccess) { delete c; return hip_fail(nullptr, e, "hipDeviceGetAttribute"); }
  c->kc = p->precision == LES_FP32_STORAGE ? fused_chunk<float>(c->g, c->num_cu)
                                          : fused_chunk<double>(c->g, c->num_cu);
  if (const char* kc = std::getenv("LESJET_KCHUNK")) {   // tuning / test override
    const int v = std::atoi(kc);
    if (v >= 1) c->kc = v;
  }
  hipStream_t s = (hipStream_t)stream;
  r = dalloc(c, (void**)&c->coords, (size_t)3 * c->cg.vs * sizeof(double), "coordinates");
  if (r == LES_OK) r = dalloc(c, (void**)&c->maxbits, sizeof(unsigned long long), "reduction slot");
  if (r == LES_OK) r = dalloc(c, (void**)&c->dt, sizeof(double), "dt");
  if (r == LES_OK) r = dalloc(c, (void**)&c->flag, sizeof(int), "flag");
  if (r != LES_OK) { t_err = c->err; free_all(c); delete c; return r; }
  double* tab_d = nullptr;   // device copy of the product-mesh table (freed below)
  e = hipSuccess;
  if (maps) {
    e = hipMalloc((void**)&tab_d, tab.size() * sizeof(double));
    if (e == hipSuccess)
      e = hipMemcpyAsync(tab_d, tab.data(), tab.size() * sizeof(double), hipMemcpyHostToDevice, s);
  }
  if (e == hipSuccess) e = launch_coords(xyz, tab_d, c->coords, c->cg, p->bc, p->period, s);
  if (e == hipSuccess) e = launch_reset(c->maxbits, c->flag, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  if (tab_d) (void)hipFree(tab_d);
  if (e != hipSuccess) {
    (void)hipGetLastError();
    hip_fail(nullptr, e, "les_init_grid");
    free_all(c);
    delete c;
    return LES_EHIP;
  }
  *out = c;
  return LES_OK;
}

int les_metrics(les_ctx* c, double* metrics_out, void* stream) {
  const Range range("les_metrics");
  if (!c) return fail(nullptr, LES_EINVAL, "ctx is NULL");
  if (c->metrics_done) return fail(c, LES_ESTATE, "metrics already computed");
  if (!c->coords) return fail(c, LES_ESTATE, "no coordinates");
  hipStream_t s = (hipStream_t)stream;
  int r = dalloc(c, &c->M, (size_t)10 * c->g.vs * storage_size(&c->p), "metrics");
  if (r != LES_OK) return r;
  hipError_t e;
  if (c->p.precision == LES_FP32_STORAGE)
    e = launch_metrics<float>(c->coords, c->cg, (float*)c->M, c->g, metrics_out, s);
  else
    e = launch_metrics<double>(c->coords, c->cg, (double*)c->M, c->g, metrics_out, s);
  if (e != hipSuccess) return hip_fail(c, e, "metrics kernel");
  HIP_TRY(c, hipStreamSynchronize(s));
  HIP_TRY(c, hipFree(c->coords));
  c->bytes -= (size_t)3 * c->cg.vs * sizeof(double);
  c->coords = nullptr;
  c->metrics_done = true;
  return LES_OK;
}

int les_set_inflow(les_ctx* c, const double* prim_in, void* stream) {
  if (!c) return fail(nullptr, LES_EINVAL, "ctx is NULL");
  if (!prim_in) return fail(c, LES_EINVAL, "prim_in is NULL");
  const size_t bytes = (size_t)5 * c->p.nth * c->p.nr * sizeof(double);
  int r = dalloc(c, (void**)&c->inflow, bytes, "inflow data");
  if (r != LES_OK) return r;
  HIP_TRY(c, hipMemcpyAsync(c->inflow, prim_in, bytes, hipMemcpyDeviceToDevice, (hipStream_t)stream));
  c->inflow_set = true;
  return LES_OK;
}

static int ready(les_ctx* c) {
  if (!c) return fail(nullptr, LES_EINVAL, "ctx is NULL");
  if (!c->metrics_done) return fail(c, LES_ESTATE, "les_metrics has not been called");
  if (c->p.bc[0] == LES_BC_INFLOW && !c->inflow_set)
    return fail(c, LES_ESTATE, "les_set_inflow has not been called");
  return LES_OK;
}

template <typename T>
static hipError_t ghosts(les_ctx* c, T* Q, hipStream_t s);
template <typename T>
static const Phys<T>& phys(les_ctx* c);

template <>
hipError_t ghosts<double>(les_ctx* c, double* Q, hipStream_t s) {
  return launch_ghosts<double>(Q, c->g, (const double*)c->M, c->inflow, c->ph64, c->p.bc,
                               c->p.ref_prim, c->p.p_exit, nullptr, s);
}
template <>
hipError_t ghosts<float>(les_ctx* c, float* Q, hipStream_t s) {
  return launch_ghosts<float>(Q, c->g, (const float*)c->M, c->inflow, c->ph32, c->p.bc,
                              c->p.ref_prim, c->p.p_exit, nullptr, s);
}
// Ghosts with the physical-face values and centerline row of `held`.
template <typename T>
static hipError_t ghosts_held(les_ctx* c, T* Q, const T* held, hipStream_t s) {
  return launch_ghosts<T>(Q, c->g, (const T*)c->M, c->inflow, phys<T>(c), c->p.bc,
                          c->p.ref_prim, c->p.p_exit, held, s);
}

template <>
const Phys<double>& phys<double>(les_ctx* c) { return c->ph64; }
template <>
const Phys<float>& phys<float>(les_ctx* c) { return c->ph32; }

static bool dynamic_model(const les_ctx* c) { return c->ph64.sgs == LES_SGS_DYNAMIC; }

// Buffers of the dynamic model (allocated on first use).
static int dynamic_ready(les_ctx* c) {
  int r = dalloc(c, (void**)&c->dyn_scr, (size_t)DYN_SCRATCH_VARS * c->g.vs * sizeof(double),
                 "dynamic-model scratch");
  if (r == LES_OK)
    r = dalloc(c, (void**)&c->dyn_part, (size_t)7 * dyn_blocks(c->g) * sizeof(double),
               "dynamic-model sums");
  if (r == LES_OK) r = dalloc(c, (void**)&c->dyn, DYN_COEF_DOUBLES * sizeof(double), "dynamic coefficients");
  return r;
}

// Coefficients of the dynamic model for the ghost-filled state Q into c->dyn.
template <typename T>
static hipError_t dynamic_coefs(les_ctx* c, const T* Q, hipStream_t s) {
  return launch_dynamic<T>(Q, (const T*)c->M, c->g, c->p.gamma, c->p.visc_coef, c->p.Pr_sgs,
                           c->dyn_scr, c->dyn_part, c->dyn, s);
}

// R(Q) into R_out (ghosts of Q filled first), fused kernel.
template <typename T>
static int residual_into(les_ctx* c, T* Q, T* R_out, hipStream_t s) {
  if (dynamic_model(c)) {
    const int r = dynamic_ready(c);
    if (r != LES_OK) return r;
  }
  hipError_t e = ghosts<T>(c, Q, s);
  if (e == hipSuccess && dynamic_model(c)) e = dynamic_coefs<T>(c, Q, s);
  if (e == hipSuccess) {
    const long k = prof_begin(c, s);
    e = launch_fused<T>(Q, (const T*)c->M, c->g, phys<T>(c), c->kc, FUSED_EPI_R, R_out, nullptr,
                        nullptr, 0.0, nullptr, c->ph64, nullptr, FUSED_LAG_NONE, nullptr, c->dyn,
                        s);
    prof_end(c, k, s);
  }
  if (e != hipSuccess) return hip_fail(c, e, "residual kernel");
  return LES_OK;
}

// Same, with the two-pass reference kernels (the dynamic coefficients are
// read back to the host for them: this path synchronises).
template <typename T>
static int residual_ref_into(les_ctx* c, T* Q, T* R_out, hipStream_t s) {
  int r = dalloc(c, &c->PT, (size_t)21 * c->g.vs * sizeof(T), "point scratch");
  if (r == LES_OK && dynamic_model(c)) r = dynamic_ready(c);
  if (r != LES_OK) return r;
  hipError_t e = ghosts<T>(c, Q, s);
  Phys<T> ph = phys<T>(c);
  if (e == hipSuccess && dynamic_model(c)) {
    double d[3] = {0.0, 0.0, 0.0};
    e = dynamic_coefs<T>(c, Q, s);
    if (e == hipSuccess) e = hipMemcpyAsync(d, c->dyn, sizeof(d), hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    ph.sgs_coef = (T)d[0];
    ph.Prs_inv = (T)d[1];
    ph.iso_coef = (T)d[2];
  }
  if (e == hipSuccess)
    e = launch_residual_ref<T>(Q, (const T*)c->M, c->g, ph, (T*)c->PT, R_out, s);
  if (e != hipSuccess) return hip_fail(c, e, "reference residual kernels");
  return LES_OK;
}

int les_dynamic_coefficients(les_ctx* c, void* Q, double* coef, void* stream) {
  int r = ready(c);
  if (r != LES_OK) return r;
  if (!Q || !coef) return fail(c, LES_EINVAL, "Q or coef is NULL");
  if (!dynamic_model(c)) return fail(c, LES_EINVAL, "the context does not use the dynamic SGS model");
  r = dynamic_ready(c);
  if (r != LES_OK) return r;
  hipStream_t s = (hipStream_t)stream;
  hipError_t e;
  if (c->p.precision == LES_FP32_STORAGE) {
    e = ghosts<float>(c, (float*)Q, s);
    if (e == hipSuccess) e = dynamic_coefs<float>(c, (const float*)Q, s);
  } else {
    e = ghosts<double>(c, (double*)Q, s);
    if (e == hipSuccess) e = dynamic_coefs<double>(c, (const double*)Q, s);
  }
  double d[DYN_COEF_DOUBLES];
  if (e == hipSuccess) e = hipMemcpyAsync(d, c->dyn, sizeof(d), hipMemcpyDeviceToHost, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  if (e != hipSuccess) return hip_fail(c, e, "dynamic-model kernels");
  coef[0] = d[3];                         // C_I
  coef[1] = d[4];                         // C_ds
  coef[2] = d[5];                         // Pr_sgs as computed
  coef[3] = 1.5 * d[2];                   // C_I used
  coef[4] = d[0] * c->p.visc_coef;        // C_ds used
  coef[5] = 1.0 / d[1];                   // Pr_sgs used
  return LES_OK;
}

int les_fill_ghosts(les_ctx* c, void* Q, void* stream) {
  int r = ready(c);
  if (r != LES_OK) return r;
  if (!Q) return fail(c, LES_EINVAL, "Q is NULL");
  hipError_t e = c->p.precision == LES_FP32_STORAGE
                     ? ghosts<float>(c, (float*)Q, (hipStream_t)stream)
                     : ghosts<double>(c, (double*)Q, (hipStream_t)stream);
  if (e != hipSuccess) return hip_fail(c, e, "ghost kernels");
  return LES_OK;
}

int les_residual_reference(les_ctx* c, void* Q, void* R, void* stream) {
  int r = ready(c);
  if (r != LES_OK) return r;
  if (!Q || !R) return fail(c, LES_EINVAL, "Q or R is NULL");
  if (Q == R) return fail(c, LES_EINVAL, "Q and R must not alias");
  hipStream_t s = (hipStream_t)stream;
  if (c->p.precision == LES_FP32_STORAGE) return residual_ref_into<float>(c, (float*)Q, (float*)R, s);
  return residual_ref_into<double>(c, (double*)Q, (double*)R, s);
}

int les_residual(les_ctx* c, void* Q, void* R, void* stream) {
  const Range range("les_residual");
  int r = ready(c);
  if (r != LES_OK) return r;
  if (!Q || !R) return fail(c, LES_EINVAL, "Q or R is NULL");
  if (Q == R) return fail(c, LES_EINVAL, "Q and R must not alias");
  hipStream_t s = (hipStream_t)stream;
  if (c->p.precision == LES_FP32_STORAGE) return residual_into<float>(c, (float*)Q, (float*)R, s);
  return residual_into<double>(c, (double*)Q, (double*)R, s);
}

template <typename T>
static int rk5_steps(les_ctx* c, double* Qn, int nsteps, double dt_fixed, double* dt_out,
                     hipStream_t s) {
  const bool fp32 = sizeof(T) == sizeof(float);
  // LES_SCHEDULE_STEP: stage 1 fills the ghosts of Q^n (its state buffer is
  // kept through the step as `held`) and stores the viscosities; stages 2-5
  // copy the physical-face ghosts from it and read the held viscosities
  const bool held_sched = c->p.schedule == LES_SCHEDULE_STEP;
  const int lagv = held_sched && c->ph64.viscous;
  const int nbuf = fp32 && held_sched ? 3 : 2;   // FP64 keeps Q^n in Qn itself
  const size_t fb = (size_t)5 * c->g.vs * sizeof(T);
  int r = LES_OK;
  for (int b = 0; b < nbuf && r == LES_OK; ++b) r = dalloc(c, &c->stage[b], fb, "stage state");
  if (r == LES_OK && lagv) r = dalloc(c, &c->visc, (size_t)2 * c->g.vs * sizeof(T), "held viscosities");
  if (r == LES_OK && dynamic_model(c)) r = dynamic_ready(c);
  if (r != LES_OK) return r;
  const bool cfl = dt_fixed <= 0.0;
  T* B[3] = {(T*)c->stage[0], (T*)c->stage[1], (T*)c->stage[2]};
  const T* M = (const T*)c->M;
  hipError_t e = launch_reset(c->maxbits, c->flag, s);
  // FP32 storage: the stage-0 state is an FP32 copy of Q^n
  T* cur = (T*)Qn;
  if (fp32 && e == hipSuccess) {
    e = launch_to_float(Qn, (float*)B[1], (long long)5 * c->g.vs, s);
    cur = B[1];
  }
  for (int n = 0; n < nsteps && e == hipSuccess; ++n) {
    // dt of this step: the first step reduces over Q^n here, later steps
    // take the maximum accumulated by the previous step's last stage
    if (cfl && n == 0) {
      if (fp32) e = launch_lambda_max<double, float>(Qn, (const float*)c->M, c->g, c->ph64, c->maxbits, s);
      else e = launch_lambda_max<double, double>(Qn, (const double*)c->M, c->g, c->ph64, c->maxbits, s);
    }
    if (e == hipSuccess)
      e = launch_dt_finalize(c->maxbits, c->p.cfl, dt_fixed, c->dt, dt_out ? dt_out + n : nullptr,
                             c->flag, s);
    T* const held = cur;
    T* src = cur;
    for (int l = 0; l < 5 && e == hipSuccess; ++l) {
      static const char* const stage_name[5] = {"lesjet RK stage 1", "lesjet RK stage 2",
                                                "lesjet RK stage 3", "lesjet RK stage 4",
                                                "lesjet RK stage 5"};
      const Range rs(stage_name[l]);
      e = l > 0 && held_sched ? ghosts_held<T>(c, src, held, s) : ghosts<T>(c, src, s);
      // dynamic model: coefficients of this stage's state (held: of Q^n)
      if (e == hipSuccess && dynamic_model(c) && (l == 0 || !held_sched))
        e = dynamic_coefs<T>(c, src, s);
      if (e != hipSuccess) break;
      // destination: a buffer other than the source and, while later stages
      // still copy from it, other than the held state
      T* dst = nullptr;
      double* q64 = nullptr;
      int epi = FUSED_EPI_RK;
      if (l == 4) epi = (cfl && n + 1 < nsteps) || fp32 ? FUSED_EPI_RK_LAST : FUSED_EPI_RK;
      if (l == 4 && !fp32) {
        dst = (T*)Qn;
      } else {
        for (int b = 0; b < nbuf && !dst; ++b)
          if (B[b] != src && !(held_sched && l < 4 && B[b] == held)) dst = B[b];
        if (l == 4) q64 = Qn;          // Q^(n+1) in FP64 + its FP32 copy
      }
      const int lag = !lagv ? FUSED_LAG_NONE : (l == 0 ? FUSED_LAG_WRITE : FUSED_LAG_READ);
      const long k = prof_begin(c, s);
      e = launch_fused<T>(src, M, c->g, phys<T>(c), c->kc, epi, dst, Qn, q64, c->p.rk_alpha[l],
                          c->dt, c->ph64, c->maxbits, lag, (T*)c->visc, c->dyn, s);
      prof_end(c, k, s);
      src = dst;
    }
    cur = src;
  }
  // centerline through the nodes: the axis row is not advanced; on return it
  // holds the azimuthal mean of the returned state's row j = 1
  if (e == hipSuccess && c->p.bc[2] == LES_BC_AXIS_NODE) e = launch_centerline<double>(Qn, c->g, s);
  if (e != hipSuccess) return hip_fail(c, e, "rk5 kernels");
  int flag = 0;
  HIP_TRY(c, hipMemcpyAsync(&flag, c->flag, sizeof(int), hipMemcpyDeviceToHost, s));
  HIP_TRY(c, hipStreamSynchronize(s));
  if (flag) return fail(c, LES_ENONFINITE, "time-step reduction was not finite (state diverged)");
  return LES_OK;
}

int les_rk5_step(les_ctx* c, double* Qn, int32_t nsteps, double dt_fixed, double* dt_out,
                 void* stream) {
  const Range range("les_rk5_step");
  int r = ready(c);
  if (r != LES_OK) return r;
  if (!Qn) return fail(c, LES_EINVAL, "Qn is NULL");
  if (nsteps < 0) return fail(c, LES_EINVAL, "nsteps must be >= 0");
  if (!std::isfinite(dt_fixed)) return fail(c, LES_EINVAL, "dt_fixed must be finite");
  if (nsteps == 0) return LES_OK;
  hipStream_t s = (hipStream_t)stream;
  if (c->p.precision == LES_FP32_STORAGE) return rk5_steps<float>(c, Qn, nsteps, dt_fixed, dt_out, s);
  return rk5_steps<double>(c, Qn, nsteps, dt_fixed, dt_out, s);
}

int les_diagnostics(les_ctx* c, const double* Qn, double* totals, double* sum1, double* sum2,
                    void* stream) {
  const Range range("les_diagnostics");
  int r = ready(c);
  if (r != LES_OK) return r;
  if (!Qn) return fail(c, LES_EINVAL, "Qn is NULL");
  if (totals) {
    r = dalloc(c, (void**)&c->part, (size_t)5 * diag_partials(c->g) * sizeof(double), "partials");
    if (r != LES_OK) return r;
  }
  hipError_t e;
  if (c->p.precision == LES_FP32_STORAGE)
    e = launch_diagnostics<float>(Qn, (const float*)c->M, c->g, c->ph64, c->part, totals, sum1,
                                  sum2, (hipStream_t)stream);
  else
    e = launch_diagnostics<double>(Qn, (const double*)c->M, c->g, c->ph64, c->part, totals, sum1,
                                   sum2, (hipStream_t)stream);
  if (e != hipSuccess) return hip_fail(c, e, "diagnostics kernels");
  return LES_OK;
}

int les_diagnostics_noalloc(les_ctx* c, const double* Qn, double* totals, double* sum1,
                            double* sum2, void* stream) {
  int r = ready(c);
  if (r != LES_OK) return r;
  if (!Qn) return fail(c, LES_EINVAL, "Qn is NULL");
  if (!c->part_static) return fail(c, LES_ESTATE, "no static scratch on this device");
  const size_t need = (size_t)5 * diag_partials(c->g);
  if (need > NOALLOC_SCRATCH_DOUBLES)
    return fail(c, LES_EUNSUPPORTED,
                "the totals need " + std::to_string(need) + " partial sums, beyond the " +
                    std::to_string(NOALLOC_SCRATCH_DOUBLES) + " of the static scratch");
  // every partial slot the final reduction reads is written by the partial
  // pass of the same call first, so nothing needs clearing
  hipError_t e;
  if (c->p.precision == LES_FP32_STORAGE)
    e = launch_diagnostics<float>(Qn, (const float*)c->M, c->g, c->ph64, c->part_static, totals,
                                  sum1, sum2, (hipStream_t)stream);
  else
    e = launch_diagnostics<double>(Qn, (const double*)c->M, c->g, c->ph64, c->part_static, totals,
                                   sum1, sum2, (hipStream_t)stream);
  if (e != hipSuccess) return hip_fail(c, e, "diagnostics kernels");
  return LES_OK;
}

// Qb = (dR/dQ)^T Rb at Q (ghosts of Q filled here); inflow_bar accumulated.
static int residual_vjp_into(les_ctx* c, double* Q, const double* Rb, double* Qb,
                             double* inflow_bar, hipStream_t s) {
  int r = dalloc(c, (void**)&c->adj, (size_t)VJP_SCRATCH_VARS * c->g.vs * sizeof(double),
                 "adjoint scratch");
  if (r != LES_OK) return r;
  hipError_t e = ghosts<double>(c, Q, s);
  if (e == hipSuccess) {
    e = launch_residual_vjp(Q, (const double*)c->M, c->g, c->ph64, c->p.bc, c->p.ref_prim,
                            c->p.p_exit, c->inflow, Rb, c->adj, Qb,
                            c->p.bc[0] == LES_BC_INFLOW ? inflow_bar : nullptr, s);
  }
  if (e != hipSuccess) return hip_fail(c, e, "residual adjoint kernels");
  return LES_OK;
}

static int adjoint_ready(les_ctx* c) {
  int r = ready(c);
  if (r != LES_OK) return r;
  if (c->p.precision != LES_FP64)
    return fail(c, LES_EUNSUPPORTED, "the adjoint is available for the FP64 precision only");
  if (dynamic_model(c))
    return fail(c, LES_EUNSUPPORTED, "the adjoint does not cover the dynamic SGS model");
  return LES_OK;
}

static int step_adjoint_ready(les_ctx* c) {
  int r = adjoint_ready(c);
  if (r != LES_OK) return r;
  if (c->p.schedule != LES_SCHEDULE_STAGE)
    return fail(c, LES_EUNSUPPORTED, "the step adjoint covers LES_SCHEDULE_STAGE only");
  return LES_OK;
}

int les_residual_vjp(les_ctx* c, double* Q, const double* Rbar, double* Qbar, double* inflow_bar,
                     void* stream) {
  const Range range("les_residual_vjp");
  int r = adjoint_ready(c);
  if (r != LES_OK) return r;
  if (!Q || !Rbar || !Qbar) return fail(c, LES_EINVAL, "Q, Rbar or Qbar is NULL");
  if (Q == Qbar || Q == Rbar) return fail(c, LES_EINVAL, "Q must not alias Rbar or Qbar");
  return residual_vjp_into(c, Q, Rbar, Qbar, inflow_bar, (hipStream_t)stream);
}

int les_rk5_step_vjp(les_ctx* c, double* Qn, double dt, const double* Qbar_np1, double* Qbar_n,
                     double* inflow_bar, void* stream) {
  const Range range("les_rk5_step_vjp");
  int r = step_adjoint_ready(c);
  if (r != LES_OK) return r;
  if (!Qn || !Qbar_np1 || !Qbar_n) return fail(c, LES_EINVAL, "Qn, Qbar_np1 or Qbar_n is NULL");
  if (Qn == Qbar_np1 || Qn == Qbar_n) return fail(c, LES_EINVAL, "Qn must not alias a cotangent");
  if (!(std::isfinite(dt) && dt > 0.0)) return fail(c, LES_EINVAL, "dt must be finite and > 0");
  const long long v5 = 5LL * c->g.vs;
  r = dalloc(c, (void**)&c->adj_stage, (size_t)5 * v5 * sizeof(double), "adjoint stage states");
  if (r != LES_OK) return r;
  hipStream_t s = (hipStream_t)stream;
  // forward: the stage states Q^(0) = Q^n, Q^(1..4) with the fixed dt, by the
  // same kernels as les_rk5_step
  double* X[5] = {Qn, c->adj_stage, c->adj_stage + v5, c->adj_stage + 2 * v5,
                  c->adj_stage + 3 * v5};
  double* B = c->adj_stage + 4 * v5;
  const double* al = c->p.rk_alpha;
  hipError_t e = launch_reset(c->maxbits, c->flag, s);
  if (e == hipSuccess) e = launch_dt_finalize(c->maxbits, c->p.cfl, dt, c->dt, nullptr, c->flag, s);
  for (int l = 1; l <= 4 && e == hipSuccess; ++l) {
    e = ghosts<double>(c, X[l - 1], s);
    if (e == hipSuccess)
      e = launch_fused<double>(X[l - 1], (const double*)c->M, c->g, c->ph64, c->kc, FUSED_EPI_RK,
                               X[l], Qn, nullptr, al[l - 1], c->dt, c->ph64, c->maxbits,
                               FUSED_LAG_NONE, nullptr, nullptr, s);
  }
  if (e != hipSuccess) return hip_fail(c, e, "rk5 adjoint forward kernels");
  // reverse: b5 = Qbar^(n+1); b(l-1) = -alpha_l dt J(Q^(l-1))^T b(l);
  // Qbar^n = b5 + b4 + ... + b0
  e = launch_scale(Qbar_np1, -al[4] * dt, B, v5, s);
  if (e == hipSuccess) e = launch_interior_copy(Qbar_np1, Qbar_n, c->g, s);
  // centerline through the nodes: the returned axis row is the mean of the
  // returned row 1, so its cotangent goes to row 1 first
  if (e == hipSuccess && c->p.bc[2] == LES_BC_AXIS_NODE) e = launch_centerline_transpose(B, c->g, s);
  if (e == hipSuccess && c->p.bc[2] == LES_BC_AXIS_NODE)
    e = launch_centerline_transpose(Qbar_n, c->g, s);
  if (e != hipSuccess) return hip_fail(c, e, "rk5 adjoint kernels");
  for (int l = 5; l >= 1; --l) {
    if (l < 5) {
      e = launch_scale(B, -al[l - 1] * dt, B, v5, s);
      if (e != hipSuccess) return hip_fail(c, e, "rk5 adjoint kernels");
    }
    r = residual_vjp_into(c, X[l - 1], B, B, inflow_bar, s);
    if (r != LES_OK) return r;
    e = launch_accumulate(B, Qbar_n, v5, s);
    if (e != hipSuccess) return hip_fail(c, e, "rk5 adjoint kernels");
  }
  return LES_OK;
}

int les_profile(les_ctx* c, int32_t enable) {
  if (!c) return fail(nullptr, LES_EINVAL, "ctx is NULL");
  c->prof = enable != 0;
  return LES_OK;
}

int les_profile_read(les_ctx* c, int64_t* launches, double* total_ms) {
  if (!c) return fail(nullptr, LES_EINVAL, "ctx is NULL");
  double tot = 0.0;
  for (size_t k = 0; k < c->ev_used; ++k) {
    HIP_TRY(c, hipEventSynchronize(c->ev[2 * k + 1]));
    float ms = 0.f;
    HIP_TRY(c, hipEventElapsedTime(&ms, c->ev[2 * k], c->ev[2 * k + 1]));
    tot += ms;
  }
  if (launches) *launches = (int64_t)c->ev_used;
  if (total_ms) *total_ms = tot;
  c->ev_used = 0;
  return LES_OK;
}

int les_query(const les_ctx* c, int64_t dims_padded[4], int64_t* pitch, size_t* device_bytes) {
  if (!c) return fail(nullptr, LES_EINVAL, "ctx is NULL");
  if (dims_padded) {
    dims_padded[0] = 5;
    dims_padded[1] = c->p.nth + 2 * NG;
    dims_padded[2] = c->p.nr + 2 * NG;
    dims_padded[3] = c->g.pitch;
  }
  if (pitch) *pitch = c->g.pitch;
  if (device_bytes) *device_bytes = c->bytes;
  return LES_OK;
}

const char* les_last_error(const les_ctx* c) {
  return c ? c->err.c_str() : t_err.c_str();
}

void les_free(les_ctx* c) {
  if (!c) return;
  (void)hipDeviceSynchronize();
  for (hipEvent_t e : c->ev) (void)hipEventDestroy(e);
  free_all(c);
  delete c;
}
