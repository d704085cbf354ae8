// api.cpp -- the C ABI of libdgsem.so (declared in include/dgsem.h): host-side mesh and
// connectivity, the device memory plan inside the caller's buffer, argument checking and
// error reporting, the launch sequence of each call, the block-size autotuner of the
// mixed-order stage kernel, and HIP-graph replay of RK steps.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <memory>
#include <mutex>
#include <new>
#include <stdexcept>
#include <numeric>
#include <string>
#include <vector>

#include "dg_internal.h"
#include "halo.h"
#include "svv.h"
#include "dgsem.h"

namespace dg {
void gll_tables(int N, double* xi, double* w, double* D, double* Dh);
void gl_tables(int N, double* xi, double* w, double* D, double* lb);
void lobatto_to_gauss(int N, double* xl, double* Dl, double* I);
void mortar_tables(int N, int M, double* I, double* P);
}

// Message of the last failure on this thread.  g_err_fixed, when set, takes precedence: it is a
// static message used where building the string itself could fail (no host memory).
static thread_local std::string g_err;
static thread_local const char* g_err_fixed = nullptr;

static int fail_fixed(int code, const char* msg) noexcept {
  g_err_fixed = msg;
  return code;
}

static int fail(int code, const std::string& msg) noexcept {
  try {
    g_err = msg;
    g_err_fixed = nullptr;
  } catch (...) {
    g_err_fixed = "host memory ran out while the error message was formed";
  }
  return code;
}

static int hip_fail(hipError_t e, const char* what) {
  return fail(DG_EHIP, std::string(what) + ": " + hipGetErrorName(e) + " (" + hipGetErrorString(e) + ")");
}

// Every entry point is a function-try-block whose handler returns this, so that no exception
// crosses the C ABI: a failed host allocation becomes DG_ENOMEM, anything else DG_EINVAL.
// Called only from inside a catch handler (the bare throw rethrows the exception in flight).
static int abi_exception() noexcept {
  try {
    throw;
  } catch (const std::bad_alloc&) {
    return fail_fixed(DG_ENOMEM, "host memory allocation failed");
  } catch (const std::exception& e) {
    return fail(DG_EINVAL, std::string("internal error: ") + e.what());
  } catch (...) {
    return fail_fixed(DG_EINVAL, "internal error");
  }
}

#define DG_HIP(call, what)                      \
  do {                                          \
    hipError_t _e = (call);                     \
    if (_e != hipSuccess) return hip_fail(_e, what); \
  } while (0)

struct dg_mesh {
  int ex, ey, ez;
  double lo[3], hi[3];
  int deform;
  double amp;
  int N;                    // the order of a uniform mesh, the largest order of a mixed one
  bool mixed = false;
  bool gauss = false;       // Gauss-Legendre nodes
  bool halo = false;        // periodic neighbours through ghost elements and a halo exchange
  std::vector<int> orders;  // mixed meshes: orders[3 e + d]
};

namespace {
// faces on the box boundary (the ghost elements of a halo box): x, y and z faces of both sides
long long halo_faces(const dg_mesh& m) {
  return 2LL * ((long long)m.ey * m.ez + (long long)m.ex * m.ez + (long long)m.ex * m.ey);
}
}  // namespace

struct ProfRecord {
  int cls;
  hipEvent_t a, b;
};

struct dg_solver {
  dg_mesh mesh;
  dg_physics phys;
  dg::View v;
  hipStream_t stream = nullptr;
  bool bound = false;
  int device = 0;                    // HIP device of the bound buffer
  int cur = 0;
  long long E = 0, ntot = 0;
  std::vector<long long> off;        // first node of every element, and the total at [E]
  bool profiling = false;
  std::vector<ProfRecord> prof;      // records of the current profile region
  std::vector<hipEvent_t> ev_pool;   // events reused across regions
  size_t ev_used = 0;
  int mix_tiles = 0;                 // mixed-order stage: bit b = two nodes per lane in bucket b
  bool mix_concurrent = false;       // mixed-order stage: buckets on the side streams of `mix`
  dg::MixStreams mix{};
  // RK-step graphs: graph[p] advances one step starting from state buffer p with step graph_dt[p]
  bool use_graphs = true;
  hipStream_t cap_stream = nullptr;
  hipGraphExec_t graph[2] = {nullptr, nullptr};
  double graph_dt[2] = {0.0, 0.0};
  // kMultiSteps steps in one graph (fewer graph launches for small solves), same keys as graph[]
  hipGraphExec_t mgraph[2] = {nullptr, nullptr};
  double mgraph_dt[2] = {0.0, 0.0};
  double last_dt = 0.0;
  // adaptive-step graphs: agraph[p] advances one step from buffer p with the step size chosen on
  // the device for CFL number agraph_cfl[p]
  hipGraphExec_t agraph[2] = {nullptr, nullptr};
  double agraph_cfl[2] = {0.0, 0.0};
  dg::View* dev_view = nullptr;      // device copy of v (inside the caller's buffer)
  int scheme = DG_RK3_WILLIAMSON;    // time scheme of dg_rk_step
  bool svv_on = false;               // spectral vanishing viscosity in every stage
  dg::SvvArgs svv{};
  dg::HaloArgs halo{};               // halo boxes: the exchange's map and buffers (halo.K > 0)
};

namespace {

struct Plan {
  size_t tab, nbr, X, Ja, J, invJ, U0, U1, dU, R, Fvf, part, diag, adapt, elem, work, mtab, Fs, fdesc, Tr, Sf, Jt, Mt, svvtab,
      hmap, hsend, hrecv, hsendv, hrecvv,
      Fa, self, total;
  size_t tab_n, mtab_n;
};

long long nodes_of(const dg_mesh& m, long long e) {
  if (!m.mixed) return (long long)(m.N + 1) * (m.N + 1) * (m.N + 1);
  const int* o = &m.orders[3 * e];
  return (long long)(o[0] + 1) * (o[1] + 1) * (o[2] + 1);
}

Plan make_plan(const dg_solver* s) {
  const bool mixed = s->mesh.mixed;
  const size_t n = (size_t)s->mesh.N + 1, nf = n * n;
  const size_t E = (size_t)s->E, nt = (size_t)s->ntot;
  size_t off = 0;
  auto take = [&](size_t bytes) {
    const size_t o = off;
    off = (off + bytes + 255) & ~(size_t)255;
    return o;
  };
  Plan p;
  p.tab_n = 0;
  p.mtab_n = 0;
  if (mixed) {
    for (int N = 1; N <= dg::kMaxOrder; N++) p.tab_n += dg::tab_size(N + 1);
    for (int N = 1; N <= dg::kMaxOrder; N++)
      for (int M = N + 1; M <= dg::kMaxOrder; M++) p.mtab_n += 2 * (N + 1) * (M + 1);
  } else {
    p.tab_n = dg::tab_size((int)n) + (s->mesh.gauss ? dg::tab_gauss_geo_size((int)n) : 0);
  }
  p.tab = take(sizeof(double) * p.tab_n);
  p.nbr = take(sizeof(int) * 6 * E);
  p.X = take(sizeof(double) * 3 * nt);
  // halo boxes: K ghost elements after the E elements of the state, the face viscous fluxes, the
  // filtered SVV flux and J (of the ghosts only the faces are used)
  const size_t K = s->mesh.halo ? (size_t)halo_faces(s->mesh) : 0;
  p.Ja = take(sizeof(double) * 9 * nt);
  p.J = take(sizeof(double) * (nt + K * n * nf));
  p.invJ = take(sizeof(double) * nt);
  p.U0 = take(sizeof(double) * 5 * (nt + K * n * nf));
  p.U1 = take(sizeof(double) * 5 * (nt + K * n * nf));
  p.dU = take(sizeof(double) * 5 * nt);
  p.R = take(sizeof(double) * 5 * nt);
  p.Fvf = s->phys.Re > 0 ? take(sizeof(double) * (E + K) * 6 * 4 * nf) : 0;
  p.hmap = K ? take(sizeof(int4) * K) : 0;
  p.hsend = K ? take(sizeof(double) * K * 5 * nf) : 0;
  p.hrecv = K ? take(sizeof(double) * K * 5 * nf) : 0;
  p.hsendv = K && s->phys.Re > 0 ? take(sizeof(double) * K * 4 * nf) : 0;
  p.hrecvv = K && s->phys.Re > 0 ? take(sizeof(double) * K * 4 * nf) : 0;
  p.part = take(sizeof(double) * E * dg::kDiagSlots);
  p.diag = take(sizeof(double) * dg::kDiagSlots);
  p.adapt = take(sizeof(double) * 8);
  p.elem = mixed ? take(sizeof(int4) * E) : 0;
  p.work = mixed ? take(sizeof(int4) * E) : 0;
  p.mtab = mixed ? take(sizeof(double) * p.mtab_n) : 0;
  p.Fs = mixed ? take(sizeof(double) * dg::kMixFaceDoubles * E) : 0;
  p.fdesc = mixed ? take(sizeof(int4) * 3 * E) : 0;
  p.Tr = s->mesh.gauss ? take(sizeof(double) * E * 6 * 5 * nf) : 0;
  p.Sf = s->mesh.gauss ? take(sizeof(double) * E * 9 * nf) : 0;
  const bool jt = s->mesh.gauss && s->phys.Re > 0 && s->phys.visc_flux == DG_VISC_IP;
  p.Jt = jt ? take(sizeof(double) * E * 6 * nf) : 0;
  const bool mt = s->mesh.gauss && s->phys.Re > 0 && s->phys.visc_flux == DG_VISC_BR2;
  p.Mt = mt ? take(sizeof(double) * E * 18 * nf) : 0;
  const bool svv = s->phys.svv_mu > 0 || s->phys.les_cs > 0;
  p.svvtab = svv ? take(sizeof(double) * n * n) : 0;
  p.Fa = svv ? take(sizeof(double) * 12 * (nt + K * n * nf)) : 0;
  p.self = take(sizeof(dg::View));  // device copy of the View, read by batched launches
  p.total = off;
  return p;
}

bool finite_positive_state(const dg_solver* s, const double* U, std::string& why) {
  const double gamma = s->phys.gamma;
  for (long long e = 0; e < s->E; e++) {
    const long long nn = s->off[e + 1] - s->off[e];
    const double* u = U + s->off[e] * 5;
    for (long long q = 0; q < nn; q++) {
      const double r = u[q], m1 = u[nn + q], m2 = u[2 * nn + q], m3 = u[3 * nn + q], en = u[4 * nn + q];
      if (!std::isfinite(r) || !std::isfinite(m1) || !std::isfinite(m2) || !std::isfinite(m3) ||
          !std::isfinite(en)) {
        why = "non-finite value at element " + std::to_string(e) + ", node " + std::to_string(q);
        return false;
      }
      const double p = (gamma - 1.0) * (en - 0.5 * (m1 * m1 + m2 * m2 + m3 * m3) / r);
      if (!(r > 0.0) || !(p > 0.0)) {
        why = "non-positive density or pressure at element " + std::to_string(e) + ", node " +
              std::to_string(q);
        return false;
      }
    }
  }
  return true;
}

hipEvent_t take_event(dg_solver* s) {
  if (s->ev_used == s->ev_pool.size()) {
    hipEvent_t e;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    s->ev_pool.push_back(e);
  }
  return s->ev_pool[s->ev_used++];
}

// launch `fn` on the solver's stream, bracketed by events when profiling
template <class F>
hipError_t timed(dg_solver* s, int cls, F fn) {
  if (!s->profiling) return fn();
  ProfRecord r{cls, take_event(s), take_event(s)};
  if (!r.a || !r.b) return hipErrorOutOfMemory;
  hipError_t e = hipEventRecord(r.a, s->stream);
  if (e != hipSuccess) return e;
  e = fn();
  if (e != hipSuccess) return e;
  e = hipEventRecord(r.b, s->stream);
  if (e != hipSuccess) return e;
  s->prof.push_back(r);
  return hipSuccess;
}

hipError_t launch_stage_any(dg_solver* s, double dt, double a, double b, int mode) {
  if (s->v.mixed)
    return dg::launch_stage_mixed(s->v, s->cur, dt, a, b, mode, s->mix_tiles, s->stream,
                                  s->mix_concurrent ? &s->mix : nullptr);
  if (s->v.gauss) return dg::launch_stage_gauss(s->v, s->cur, dt, a, b, mode, s->stream);
  return dg::launch_stage(s->v, s->cur, dt, a, b, mode, s->stream);
}

// work a stage needs before its kernels: the global wave speed for Lax-Friedrichs (global)
hipError_t pre_stage(const dg_solver* s, int cur, hipStream_t st) {
  if (s->v.surf == DG_SURF_LF_GLOBAL) return dg::launch_lambda_max(s->v, cur, st);
  return hipSuccess;
}

// spectral vanishing viscosity on Navier-Stokes with the standard fluxes: the filtered flux of the
// stage's input is formed first and the stage kernel adds it to the viscous flux (no correction
// pass after it); otherwise the two SVV kernels correct the stage kernel's output
bool svv_folded(const dg_solver* s) {
  return s->svv_on && s->v.viscous && dg::flux_family(s->v.vol, s->v.surf) == 0;
}

hipError_t run_stage(dg_solver* s, double dt, double a, double b, int mode) {
  if (s->v.surf == DG_SURF_LF_GLOBAL) {
    hipError_t e = timed(s, DG_K_OTHER, [&] { return pre_stage(s, s->cur, s->stream); });
    if (e != hipSuccess) return e;
  }
  if (s->halo.K) {  // the ghosts' face state of this stage's input
    hipError_t e = timed(s, DG_K_OTHER, [&] { return dg::halo_exchange_state(s->v, s->cur, s->halo, s->stream); });
    if (e != hipSuccess) return e;
  }
  if (svv_folded(s)) {  // (takes its own gradient pass)
    hipError_t e;
    if (s->v.visc_flux == DG_VISC_BR1) {  // the gradient pass and the SVV flux in one launch
      e = timed(s, DG_K_GRADIENT, [&] { return dg::launch_grad_svv(s->v, s->cur, s->svv, s->stream); });
    } else {
      e = timed(s, DG_K_GRADIENT, [&] { return dg::launch_gradient(s->v, s->cur, s->stream); });
      if (e == hipSuccess)
        e = timed(s, DG_K_OTHER, [&] { return dg::launch_svv_flux(s->v, s->cur, s->svv, s->stream); });
    }
    if (e == hipSuccess && s->halo.K) {  // the ghosts' face viscous fluxes and filtered fluxes
      e = timed(s, DG_K_OTHER, [&] { return dg::halo_exchange_viscous(s->v, s->halo, s->stream); });
      if (e == hipSuccess)
        e = timed(s, DG_K_OTHER, [&] { return dg::halo_exchange_svv(s->v, s->svv.Fa, s->halo, s->stream); });
    }
    if (e != hipSuccess) return e;
    dg::View vf = s->v;
    vf.Fa = s->svv.Fa;
    return timed(s, DG_K_STAGE, [&] { return dg::launch_stage(vf, s->cur, dt, a, b, mode, s->stream); });
  }
  if (s->v.viscous && !s->v.gauss) {  // (Gauss-Legendre solvers take their gradients in their stage launch)
    hipError_t e = timed(s, DG_K_GRADIENT, [&] { return dg::launch_gradient(s->v, s->cur, s->stream); });
    if (e != hipSuccess) return e;
    if (s->halo.K) {  // and their face viscous fluxes
      e = timed(s, DG_K_OTHER, [&] { return dg::halo_exchange_viscous(s->v, s->halo, s->stream); });
      if (e != hipSuccess) return e;
    }
  }
  hipError_t e = timed(s, DG_K_STAGE, [&] { return launch_stage_any(s, dt, a, b, mode); });
  if (e != hipSuccess || !s->svv_on) return e;
  if (!s->halo.K)
    return timed(s, DG_K_OTHER, [&] { return dg::launch_svv(s->v, s->cur, s->svv, dt, b, mode, s->stream); });
  // halo box: the filtered flux, its exchange, then its divergence
  e = timed(s, DG_K_OTHER, [&] { return dg::launch_svv_flux(s->v, s->cur, s->svv, s->stream); });
  if (e == hipSuccess)
    e = timed(s, DG_K_OTHER, [&] { return dg::halo_exchange_svv(s->v, s->svv.Fa, s->halo, s->stream); });
  if (e != hipSuccess) return e;
  return timed(s, DG_K_OTHER, [&] { return dg::launch_svv_div(s->v, s->cur, s->svv, dt, b, mode, s->stream); });
}

hipError_t launch_diag_any(dg_solver* s) {
  return s->v.mixed ? dg::launch_diagnostics_mixed(s->v, s->cur, s->stream)
                    : dg::launch_diagnostics(s->v, s->cur, s->stream);
}

}  // namespace

// ------------------------------------------------------------------ diagnostics without allocation
// dg_diagnostics_noalloc keeps its per-element partial sums and the reduced slots in this array,
// not in the caller's buffer: a diagnostics call then needs no device memory beyond the bound
// solver's state and geometry and the caller's 112-byte output.  Each device holds its own copy
// for the life of the process; every call on a device shares it (calls that overlap on one device
// race).  In host code the name is only a stand-in: kernels get the address that
// hipGetSymbolAddress returns for the current device.
constexpr long long kNoAllocMaxElements = 32768;
static __device__ __align__(256) double scratch[(kNoAllocMaxElements + 1) * dg::kDiagSlots];

namespace {

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
double* g_scratch_ptr[kMaxDevices] = {};

// device address of `scratch` on the current device `dev` (looked up once per device)
hipError_t scratch_on(int dev, double** out) {
  if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    g_scratch_ptr[dev] = static_cast<double*>(p);
  }
  *out = g_scratch_ptr[dev];
  return hipSuccess;
}

// the reduced slots (see diag_kernel) as a dg_diag record in device memory
__global__ void diag_record_kernel(const double* h, dg_diag* out) {
  if (threadIdx.x != 0) return;
  for (int k = 0; k < 5; k++) out->mass[k] = h[k];
  out->entropy_paper = h[5];
  out->entropy = h[6];
  out->volume = h[13];
  out->ke = h[7] / h[13];
  out->enstrophy = h[8] / h[13];
  out->lambda_max = h[9];
  out->rho_min = h[10];
  out->p_min = h[11];
  out->nonfinite = (long long)h[12];
}

// restores the calling thread's current device on scope exit
struct DeviceGuard {
  int prev = -1;
  ~DeviceGuard() {
    if (prev >= 0) (void)hipSetDevice(prev);
  }
};

// Williamson's low-storage RK3
// Low-storage (2N) Runge-Kutta schemes: per stage k, dU <- A_k dU + dt R; U <- U + B_k dU.
struct RkScheme {
  int stages;
  double A[5], B[5];
};
// Williamson's RK3, and Carpenter and Kennedy's five-stage fourth-order scheme (their published
// rational coefficients, evaluated in double)
const RkScheme kRk[2] = {
    {3, {0.0, -5.0 / 9.0, -153.0 / 128.0, 0.0, 0.0}, {1.0 / 3.0, 15.0 / 16.0, 8.0 / 15.0, 0.0, 0.0}},
    {5,
     {0.0, -567301805773.0 / 1357537059087.0, -2404267990393.0 / 2016746695238.0,
      -3550918686646.0 / 2091501179385.0, -1275806237668.0 / 842570457699.0},
     {1432997174477.0 / 9575080441755.0, 5161836677717.0 / 13612068292357.0,
      1720146321549.0 / 2090206949498.0, 3134564353537.0 / 4481467310338.0,
      2277821191437.0 / 14882151754819.0}}};

// (waits for the solver's stream first, so that no replay of a graph is still in flight)
void drop_graphs(dg_solver* s) {
  if (!s->graph[0] && !s->graph[1] && !s->agraph[0] && !s->agraph[1] && !s->mgraph[0] && !s->mgraph[1]) return;
  (void)hipStreamSynchronize(s->stream);
  for (int k = 0; k < 2; k++) {
    if (s->graph[k]) (void)hipGraphExecDestroy(s->graph[k]);
    if (s->agraph[k]) (void)hipGraphExecDestroy(s->agraph[k]);
    if (s->mgraph[k]) (void)hipGraphExecDestroy(s->mgraph[k]);
    s->graph[k] = nullptr;
    s->agraph[k] = nullptr;
    s->mgraph[k] = nullptr;
  }
}

// copy the View to its device slot (synchronously: s->v is the source)
int upload_view(dg_solver* s) {
  DG_HIP(hipMemcpyAsync(s->dev_view, &s->v, sizeof(dg::View), hipMemcpyHostToDevice, s->stream),
         "upload view");
  DG_HIP(hipStreamSynchronize(s->stream), "upload view");
  return DG_OK;
}

// FP32-bulk reference state: volume means of density and pressure of the state just set
// (any constant is exact; the closer to the state, the smaller the deviations).
int update_reference(dg_solver* s) {
  drop_graphs(s);  // captured launches hold the reference state by value
  if (!s->v.fp32) return DG_OK;
  double h[dg::kDiagSlots];
  DG_HIP(launch_diag_any(s), "reference-state reduction");
  DG_HIP(hipMemcpyAsync(h, s->v.diag, sizeof(h), hipMemcpyDeviceToHost, s->stream), "reference state");
  DG_HIP(hipStreamSynchronize(s->stream), "reference state");
  if (!(h[13] > 0) || !(h[0] > 0) || !(h[14] > 0) || !std::isfinite(h[0]) || !std::isfinite(h[14]))
    return fail(DG_ENONFINITE, "state has no positive finite mean density and pressure");
  s->v.rho_r = h[0] / h[13];
  s->v.p_r = h[14] / h[13];
  return upload_view(s);
}

// one RK step from buffer s->cur with step size dt (ignored by the kernels while s->v.dtp is set)
hipError_t run_step(dg_solver* s, double dt) {
  const RkScheme& rk = kRk[s->scheme];
  hipError_t err = hipSuccess;
  for (int k = 0; k < rk.stages && err == hipSuccess; k++) {
    err = run_stage(s, dt, rk.A[k], rk.B[k], dg::kModeRK);
    s->cur ^= 1;
  }
  return err;
}

// the viscosity of the step-size cap: physical plus artificial (spectral vanishing viscosity)
double mu_eff(const dg_solver* s) {
  return (s->v.viscous ? s->v.mu : 0.0) + (s->svv_on ? s->svv.mu : 0.0);
}

// the step size of the coming step, chosen on the device from the state in buffer s->cur
hipError_t run_step_size(dg_solver* s, double cfl) {
  const dg::View& v = s->v;
  const double hmin = std::fmin(v.h[0], std::fmin(v.h[1], v.h[2]));
  return timed(s, DG_K_OTHER, [&] {
    return dg::launch_step_size(v, s->cur, cfl, hmin, v.N + 1.0, s->phys.gamma, s->phys.Pr, mu_eff(s), s->stream);
  });
}

// Record the launches `record` makes for one RK step that starts from state buffer s->cur on the
// library's capture stream (the solver's stream is swapped for it meanwhile), instantiate them
// into *slot (replacing a previous graph).
template <class F>
int capture_into(dg_solver* s, hipGraphExec_t* slot, F record) {
  const int parity = s->cur;
  if (*slot) {
    (void)hipStreamSynchronize(s->stream);  // no replay of the old graph still in flight
    (void)hipGraphExecDestroy(*slot);
    *slot = nullptr;
  }
  hipStream_t user = s->stream;
  s->stream = s->cap_stream;
  hipGraph_t g = nullptr;
  hipError_t err = hipStreamBeginCapture(s->cap_stream, hipStreamCaptureModeThreadLocal);
  if (err == hipSuccess) {
    err = record();
    const hipError_t e2 = hipStreamEndCapture(s->cap_stream, &g);
    if (err == hipSuccess) err = e2;
  }
  s->stream = user;
  s->cur = parity;
  if (err != hipSuccess) {
    if (g) (void)hipGraphDestroy(g);
    return hip_fail(err, "capture of an RK step");
  }
  hipGraphExec_t ex = nullptr;
  err = hipGraphInstantiate(&ex, g, nullptr, nullptr, 0);
  (void)hipGraphDestroy(g);
  if (err != hipSuccess) return hip_fail(err, "instantiation of the RK-step graph");
  *slot = ex;
  return DG_OK;
}

int capture_step(dg_solver* s, double dt) {
  const int parity = s->cur;
  const int rc = capture_into(s, &s->graph[parity], [&] { return run_step(s, dt); });
  if (rc == DG_OK) s->graph_dt[parity] = dt;
  return rc;
}

// kMultiSteps consecutive steps in one graph
constexpr int kMultiSteps = 8;
int capture_multi_step(dg_solver* s, double dt) {
  const int parity = s->cur;
  const int rc = capture_into(s, &s->mgraph[parity], [&] {
    hipError_t e = hipSuccess;
    for (int k = 0; k < kMultiSteps && e == hipSuccess; k++) e = run_step(s, dt);
    return e;
  });
  if (rc == DG_OK) s->mgraph_dt[parity] = dt;
  return rc;
}

// the launches of one adaptive step: step size, then the stages (s->v.dtp is set by the caller)
int capture_adaptive_step(dg_solver* s, double cfl) {
  const int parity = s->cur;
  const int rc = capture_into(s, &s->agraph[parity], [&] {
    hipError_t e = run_step_size(s, cfl);
    return e == hipSuccess ? run_step(s, 0.0) : e;
  });
  if (rc == DG_OK) s->agraph_cfl[parity] = cfl;
  return rc;
}

int check_bound(const dg_solver* s) {
  if (!s) return fail(DG_EINVAL, "NULL solver");
  if (!s->bound) return fail(DG_ESTATE, "solver is not bound to device memory (dg_solver_bind)");
  return DG_OK;
}

}  // namespace

extern "C" {

const char* dg_last_error(void) { return g_err_fixed ? g_err_fixed : g_err.c_str(); }

int dg_mesh_create_box(const dg_box_desc* d, dg_mesh** out) try {
  if (!d || !out) return fail(DG_EINVAL, "NULL argument");
  *out = nullptr;
  if (d->ex < 1 || d->ey < 1 || d->ez < 1) return fail(DG_EINVAL, "element counts must be >= 1");
  if ((long long)d->ex * d->ey * d->ez > (1LL << 30)) return fail(DG_EINVAL, "too many elements");
  for (int k = 0; k < 3; k++)
    if (!(d->hi[k] > d->lo[k])) return fail(DG_EINVAL, "box requires hi > lo in every direction");
  if (d->deform != DG_DEFORM_NONE && d->deform != DG_DEFORM_SINSIN)
    return fail(DG_EINVAL, "unknown deformation");
  if (d->nodes != DG_NODES_LOBATTO && d->nodes != DG_NODES_GAUSS) return fail(DG_EINVAL, "unknown node set");
  const long long E = (long long)d->ex * d->ey * d->ez;
  int N = d->n_uniform;
  bool mixed = false;
  int nmax = 0;
  long long nodes = 0;
  if (d->orders) {
    N = d->orders[0];
    for (long long i = 0; i < 3 * E; i++) {
      if (d->orders[i] < 1 || d->orders[i] > dg::kMaxOrder)
        return fail(DG_EINVAL, "orders must lie in [1, 7]");
      if (d->orders[i] != N) mixed = true;
      nmax = std::max(nmax, d->orders[i]);
    }
    for (long long e = 0; e < E; e++)
      nodes += (long long)(d->orders[3 * e] + 1) * (d->orders[3 * e + 1] + 1) * (d->orders[3 * e + 2] + 1);
    if (mixed && nmax > dg::kMixMaxOrder)
      return fail(DG_EUNSUPPORTED, "elements of mixed-order meshes take orders up to 6");
    if (mixed && nodes >= (1LL << 31))
      return fail(DG_EUNSUPPORTED, "mixed-order meshes take fewer than 2^31 nodes");
  }
  if (N < 1 || N > dg::kMaxOrder) return fail(DG_EINVAL, "order must lie in [1, 7]");
  std::unique_ptr<dg_mesh> m(new dg_mesh);
  m->ex = d->ex; m->ey = d->ey; m->ez = d->ez;
  for (int k = 0; k < 3; k++) { m->lo[k] = d->lo[k]; m->hi[k] = d->hi[k]; }
  m->deform = d->deform;
  m->amp = d->deform_amp;
  m->mixed = mixed;
  m->gauss = d->nodes == DG_NODES_GAUSS;
  if (m->gauss && mixed) return fail(DG_EUNSUPPORTED, "Gauss-Legendre nodes are built for uniform-order boxes");
  if (d->halo != 0 && d->halo != 1) return fail(DG_EINVAL, "halo must be 0 or 1");
  m->halo = d->halo == 1;
  if (m->halo && (mixed || m->gauss))
    return fail(DG_EUNSUPPORTED, "halo exchange: uniform-order Gauss-Lobatto boxes");
  if (m->halo && E + halo_faces(*m) >= (1LL << 31))
    return fail(DG_EUNSUPPORTED, "halo exchange: elements and ghost elements must number fewer than 2^31");
  m->N = mixed ? nmax : N;
  if (mixed) m->orders.assign(d->orders, d->orders + 3 * E);
  *out = m.release();
  return DG_OK;
} catch (...) {
  return abi_exception();
}

void dg_mesh_destroy(dg_mesh* m) try { delete m; } catch (...) {}

int dg_mesh_info(const dg_mesh* m, long long* n_elements, long long* n_nodes, int* n_max) try {
  if (!m) return fail(DG_EINVAL, "NULL mesh");
  const long long E = (long long)m->ex * m->ey * m->ez;
  long long nodes = 0;
  if (m->mixed)
    for (long long e = 0; e < E; e++) nodes += nodes_of(*m, e);
  else
    nodes = E * nodes_of(*m, 0);
  if (n_elements) *n_elements = E;
  if (n_nodes) *n_nodes = nodes;
  if (n_max) *n_max = m->N;
  return DG_OK;
} catch (...) {
  return abi_exception();
}

int dg_solver_create(const dg_mesh* m, const dg_physics* p, dg_solver** out) try {
  if (!m || !p || !out) return fail(DG_EINVAL, "NULL argument");
  *out = nullptr;
  if (!(p->gamma > 1.0)) return fail(DG_EINVAL, "gamma must exceed 1");
  if (p->Re > 0 && !(p->Pr > 0)) return fail(DG_EINVAL, "Pr must be positive");
  if (!(p->Ma > 0)) return fail(DG_EINVAL, "Ma must be positive");
  if (p->vol_flux < DG_VOL_EC || p->vol_flux > DG_VOL_MORINISHI) return fail(DG_EINVAL, "unknown volume flux");
  if (p->surf_flux < DG_SURF_ROE || p->surf_flux > DG_SURF_LF_GLOBAL)
    return fail(DG_EINVAL, "unknown surface flux");
  if (p->precision != DG_FP64 && p->precision != DG_FP32_BULK) return fail(DG_EINVAL, "unknown precision");
  if (p->visc_flux < DG_VISC_BR1 || p->visc_flux > DG_VISC_IP) return fail(DG_EINVAL, "unknown viscous flux");
  if (!(p->visc_eta >= 0) || !std::isfinite(p->visc_eta)) return fail(DG_EINVAL, "visc_eta must be >= 0");
  if (m->N < 1 || m->N > dg::kMaxOrder) return fail(DG_EUNSUPPORTED, "no kernel for this order");
  if (p->precision == DG_FP32_BULK && (p->vol_flux >= DG_VOL_IR || p->surf_flux >= DG_SURF_ES))
    return fail(DG_EUNSUPPORTED, "FP32-bulk covers the EC and central volume fluxes and the Roe, LLF, EC and "
                                 "central surface fluxes; the others are evaluated in FP64");
  if (m->mixed && p->Re > 0)
    return fail(DG_EUNSUPPORTED, "mixed-order meshes are evaluated for the Euler equations (Re <= 0)");
  if (m->gauss && (p->precision != DG_FP64 || p->vol_flux != DG_VOL_CENTRAL))
    return fail(DG_EUNSUPPORTED, "Gauss-Legendre nodes: FP64, volume flux DG_VOL_CENTRAL (the plain weak "
                                 "form)");
  if (!(p->svv_mu >= 0) || !std::isfinite(p->svv_mu)) return fail(DG_EINVAL, "svv_mu must be >= 0");
  if (!(p->les_cs >= 0) || !std::isfinite(p->les_cs)) return fail(DG_EINVAL, "les_cs must be >= 0");
  if (p->les_cs > 0 && p->les_model != DG_LES_SMAGORINSKY && p->les_model != DG_LES_WALE &&
      p->les_model != DG_LES_VREMAN)
    return fail(DG_EINVAL, "unknown LES model");
  if (p->svv_mu > 0 || p->les_cs > 0) {
    if (p->svv_kernel != DG_SVV_TADMOR && p->svv_kernel != DG_SVV_MADAY) return fail(DG_EINVAL, "unknown SVV kernel");
    if (p->svv_cutoff < -1 || p->svv_cutoff > m->N) return fail(DG_EINVAL, "SVV cutoff outside [-1, N]");
    if (!(p->Pr > 0)) return fail(DG_EINVAL, "Pr must be positive");
    if (std::isnan(p->svv_sensor)) return fail(DG_EINVAL, "SVV sensor threshold is NaN");
    if (m->mixed || m->gauss)
      return fail(DG_EUNSUPPORTED, "spectral vanishing viscosity: uniform-order Gauss-Lobatto meshes");
  }
  std::unique_ptr<dg_solver> s(new dg_solver);
  s->mesh = *m;
  s->phys = *p;
  s->E = (long long)m->ex * m->ey * m->ez;
  s->off.resize(s->E + 1);
  s->off[0] = 0;
  for (long long e = 0; e < s->E; e++) s->off[e + 1] = s->off[e] + nodes_of(*m, e);
  s->ntot = s->off[s->E];
  std::memset(&s->v, 0, sizeof(s->v));
  dg::View& v = s->v;
  v.E = (int)s->E;
  v.N = m->N;
  v.ex = m->ex; v.ey = m->ey; v.ez = m->ez;
  v.deform = m->deform;
  v.amp = m->amp;
  for (int k = 0; k < 3; k++) {
    v.lo[k] = m->lo[k];
    v.h[k] = (m->hi[k] - m->lo[k]) / (k == 0 ? m->ex : (k == 1 ? m->ey : m->ez));
  }
  v.gamma = p->gamma;
  v.Ma = p->Ma;
  v.viscous = p->Re > 0 ? 1 : 0;
  v.mu = v.viscous ? 1.0 / p->Re : 0.0;
  v.kappa = v.viscous ? v.mu * p->gamma / ((p->gamma - 1.0) * p->Pr) : 0.0;
  v.visc_flux = p->visc_flux;
  v.visc_eta = p->visc_eta > 0 ? p->visc_eta : (p->visc_flux == DG_VISC_BR2 ? 2.0 : 1.0);
  v.vol = p->vol_flux;
  v.surf = p->surf_flux;
  v.fp32 = p->precision == DG_FP32_BULK ? 1 : 0;
  v.rho_r = 1.0;
  v.p_r = 1.0 / (p->gamma * p->Ma * p->Ma);
  v.mixed = m->mixed ? 1 : 0;
  v.nmax = m->N;
  *out = s.release();
  return DG_OK;
} catch (...) {
  return abi_exception();
}

int dg_solver_required_bytes(const dg_solver* s, size_t* bytes) try {
  if (!s || !bytes) return fail(DG_EINVAL, "NULL argument");
  *bytes = make_plan(s).total;
  return DG_OK;
} catch (...) {
  return abi_exception();
}

int dg_solver_bind(dg_solver* s, void* dev_ptr, size_t bytes, void* hip_stream) try {
  if (!s || !dev_ptr) return fail(DG_EINVAL, "NULL argument");
  if (s->bound) return fail(DG_ESTATE, "solver already bound");
  const Plan p = make_plan(s);
  if (bytes < p.total)
    return fail(DG_ENOMEM, "device buffer of " + std::to_string(bytes) + " bytes is smaller than the " +
                               std::to_string(p.total) + " bytes required");
  if (((uintptr_t)dev_ptr & 255) != 0) return fail(DG_EINVAL, "device buffer must be 256-byte aligned");
  char* b = static_cast<char*>(dev_ptr);
  dg::View& v = s->v;
  const bool mixed = v.mixed != 0;
  v.tab = reinterpret_cast<const double*>(b + p.tab);
  v.nbr = reinterpret_cast<const int*>(b + p.nbr);
  v.X = reinterpret_cast<double*>(b + p.X);
  v.Ja = reinterpret_cast<double*>(b + p.Ja);
  v.J = reinterpret_cast<double*>(b + p.J);
  v.invJ = reinterpret_cast<double*>(b + p.invJ);
  v.U[0] = reinterpret_cast<double*>(b + p.U0);
  v.U[1] = reinterpret_cast<double*>(b + p.U1);
  v.dU = reinterpret_cast<double*>(b + p.dU);
  v.R = reinterpret_cast<double*>(b + p.R);
  v.Fvf = v.viscous ? reinterpret_cast<double*>(b + p.Fvf) : nullptr;
  if (s->mesh.halo) {
    s->halo.map = reinterpret_cast<const int4*>(b + p.hmap);
    s->halo.K = (int)halo_faces(s->mesh);
    s->halo.send = reinterpret_cast<double*>(b + p.hsend);
    s->halo.recv = reinterpret_cast<double*>(b + p.hrecv);
    s->halo.sendv = v.viscous ? reinterpret_cast<double*>(b + p.hsendv) : nullptr;
    s->halo.recvv = v.viscous ? reinterpret_cast<double*>(b + p.hrecvv) : nullptr;
  }
  v.part = reinterpret_cast<double*>(b + p.part);
  v.diag = reinterpret_cast<double*>(b + p.diag);
  v.adapt = reinterpret_cast<double*>(b + p.adapt);
  v.dtp = nullptr;
  v.elem = mixed ? reinterpret_cast<const int4*>(b + p.elem) : nullptr;
  v.work = mixed ? reinterpret_cast<const int4*>(b + p.work) : nullptr;
  v.mtab = mixed ? reinterpret_cast<const double*>(b + p.mtab) : nullptr;
  v.Fs = mixed ? reinterpret_cast<double*>(b + p.Fs) : nullptr;
  v.fdesc = mixed ? reinterpret_cast<const int4*>(b + p.fdesc) : nullptr;
  v.gauss = s->mesh.gauss ? 1 : 0;
  v.Tr = s->mesh.gauss ? reinterpret_cast<double*>(b + p.Tr) : nullptr;
  v.Sf = s->mesh.gauss ? reinterpret_cast<double*>(b + p.Sf) : nullptr;
  v.Jt = p.Jt ? reinterpret_cast<double*>(b + p.Jt) : nullptr;
  v.Mt = p.Mt ? reinterpret_cast<double*>(b + p.Mt) : nullptr;
  s->svv_on = s->phys.svv_mu > 0 || s->phys.les_cs > 0;
  if (s->svv_on) {
    s->svv.mu = s->phys.svv_mu;
    s->svv.kfac = s->phys.gamma / ((s->phys.gamma - 1.0) * s->phys.Pr);
    s->svv.kappa = s->phys.svv_mu * s->svv.kfac;
    s->svv.les_c = s->phys.les_cs;
    s->svv.les_model = s->phys.les_model;
    s->svv.sensor = s->phys.svv_sensor;
    s->svv.filt = reinterpret_cast<const double*>(b + p.svvtab);
    s->svv.Fa = reinterpret_cast<double*>(b + p.Fa);
  }
  s->dev_view = reinterpret_cast<dg::View*>(b + p.self);
  s->stream = static_cast<hipStream_t>(hip_stream);

  // Lobatto tables: of the one order, or of every order (at tab_off[N]) for a mixed mesh
  std::vector<double> tab(p.tab_n);
  auto fill = [&](int N, double* t) {
    const int n = N + 1;
    if (s->mesh.gauss) {
      dg::gl_tables(N, t + dg::tab_xi(n), t + dg::tab_w(n), t + dg::tab_D(n), t + dg::tab_Dh(n));
      double* g = t + dg::tab_size(n);
      dg::lobatto_to_gauss(N, g, g + n, g + n + n * n);
    }
    else
      dg::gll_tables(N, t + dg::tab_xi(n), t + dg::tab_w(n), t + dg::tab_D(n), t + dg::tab_Dh(n));
  };
  if (mixed) {
    size_t o = 0;
    for (int N = 1; N <= dg::kMaxOrder; N++) {
      v.tab_off[N] = (int)o;
      fill(N, tab.data() + o);
      o += dg::tab_size(N + 1);
    }
  } else {
    fill(v.N, tab.data());
  }
  std::vector<int> nbr(6 * s->E);
  const int ex = v.ex, ey = v.ey, ez = v.ez;
  for (long long e = 0; e < s->E; e++) {
    const int a = (int)(e % ex), bb = (int)((e / ex) % ey), c = (int)(e / ((long long)ex * ey));
    nbr[6 * e + 0] = ((a + ex - 1) % ex) + ex * (bb + ey * c);
    nbr[6 * e + 1] = ((a + 1) % ex) + ex * (bb + ey * c);
    nbr[6 * e + 2] = a + ex * (((bb + ey - 1) % ey) + ey * c);
    nbr[6 * e + 3] = a + ex * (((bb + 1) % ey) + ey * c);
    nbr[6 * e + 4] = a + ex * (bb + ey * ((c + ez - 1) % ez));
    nbr[6 * e + 5] = a + ex * (bb + ey * ((c + 1) % ez));
  }
  DG_HIP(hipMemcpyAsync(b + p.tab, tab.data(), sizeof(double) * tab.size(), hipMemcpyHostToDevice, s->stream),
         "upload tables");
  std::vector<double> svvtab;
  if (s->svv_on) {
    const int n = v.N + 1;
    svvtab.resize((size_t)n * n);
    dg::svv_filter_table(v.N, s->phys.svv_kernel, s->phys.svv_cutoff, tab.data() + dg::tab_xi(n),
                         tab.data() + dg::tab_w(n), svvtab.data());
    DG_HIP(hipMemcpyAsync(b + p.svvtab, svvtab.data(), sizeof(double) * svvtab.size(), hipMemcpyHostToDevice,
                          s->stream),
           "upload the SVV filter");
  }
  DG_HIP(hipMemcpyAsync(b + p.nbr, nbr.data(), sizeof(int) * nbr.size(), hipMemcpyHostToDevice, s->stream),
         "upload connectivity");
  if (mixed) {
    // mortar matrices I_{N->M} ((M+1) x (N+1)) then P_{M->N} ((N+1) x (M+1)) at mort_off[N][M]
    std::vector<double> mtab(p.mtab_n);
    size_t o = 0;
    for (int N = 1; N <= dg::kMaxOrder; N++)
      for (int M = N + 1; M <= dg::kMaxOrder; M++) {
        v.mort_off[N][M] = (int)o;
        dg::mortar_tables(N, M, mtab.data() + o, mtab.data() + o + (N + 1) * (M + 1));
        o += 2 * (N + 1) * (M + 1);
      }
    // element table (node counts, first node) and the launch order: largest elements first
    std::vector<int4> elem(s->E);
    for (long long e = 0; e < s->E; e++) {
      const int* n = &s->mesh.orders[3 * e];
      elem[e] = make_int4(n[0] + 1, n[1] + 1, n[2] + 1, (int)s->off[e]);
    }
    // face table of the face pass: one entry per face 3 e + d (the face on e's +d side)
    static_assert(dg::kMixMaxOrder + 1 < 8, "a node count takes 3 bits");
    std::vector<int4> fdesc(3 * s->E);
    for (long long e = 0; e < s->E; e++)
      for (int d = 0; d < 3; d++) {
        const int r = nbr[6 * e + 2 * d + 1];
        const int4 L = elem[e], R = elem[r];
        const int counts = L.x | L.y << 3 | L.z << 6 | R.x << 9 | R.y << 12 | R.z << 15;
        fdesc[3 * e + d] = make_int4(r, counts, L.w, R.w);
      }
    std::vector<int> work(s->E);
    std::iota(work.begin(), work.end(), 0);
    std::stable_sort(work.begin(), work.end(), [&](int x, int y) {
      return s->off[x + 1] - s->off[x] > s->off[y + 1] - s->off[y];
    });
    // buckets of the launch: 64 b < nodes <= 64 (b + 1), contiguous in the sorted list
    for (int bk = 0; bk < dg::kMixBuckets; bk++) {
      v.mix_beg[bk] = 0;
      v.mix_cnt[bk] = 0;
    }
    for (long long i = 0; i < s->E; i++) {
      const long long nn = s->off[work[i] + 1] - s->off[work[i]];
      const int bk = (int)((nn - 1) / 64);
      if (v.mix_cnt[bk] == 0) v.mix_beg[bk] = (int)i;
      v.mix_cnt[bk]++;
    }
    // A launch of few workgroups is mostly its tail: from the largest elements down, a bucket
    // joins the launch above it (whose workgroups are sized for larger elements) while that
    // launch holds fewer than kMinLaunch elements.  The ranges stay contiguous in the list.
    constexpr int kMinLaunch = 2048;
    int top = -1;
    for (int bk = dg::kMixBuckets - 1; bk >= 0; bk--) {
      if (v.mix_cnt[bk] == 0) continue;
      if (top >= 0 && v.mix_cnt[top] < kMinLaunch) {
        v.mix_cnt[top] += v.mix_cnt[bk];
        v.mix_cnt[bk] = 0;
      } else {
        top = bk;
      }
    }
    DG_HIP(hipMemcpyAsync(b + p.mtab, mtab.data(), sizeof(double) * mtab.size(), hipMemcpyHostToDevice,
                          s->stream), "upload mortar matrices");
    DG_HIP(hipMemcpyAsync(b + p.elem, elem.data(), sizeof(int4) * elem.size(), hipMemcpyHostToDevice,
                          s->stream), "upload element table");
    DG_HIP(hipMemcpyAsync(b + p.fdesc, fdesc.data(), sizeof(int4) * fdesc.size(), hipMemcpyHostToDevice,
                          s->stream), "upload face table");
    // the work list's entries carry the element's table entry (one load in the stage kernel)
    std::vector<int4> witem(s->E);
    for (long long i = 0; i < s->E; i++) {
      const int4 q = elem[work[i]];
      witem[i] = make_int4(work[i], q.x | q.y << 3 | q.z << 6, q.w, q.x * q.y * q.z);
    }
    DG_HIP(hipMemcpyAsync(b + p.work, witem.data(), sizeof(int4) * witem.size(), hipMemcpyHostToDevice,
                          s->stream), "upload work list");
    DG_HIP(dg::launch_geometry_mixed(v, s->stream), "geometry kernel");
    // the host vectors must outlive the copies
    DG_HIP(hipStreamSynchronize(s->stream), "upload");
  } else {
    DG_HIP(dg::launch_geometry(v, s->stream), "geometry kernel");
    if (v.Jt || v.Mt) DG_HIP(dg::launch_jtrace_gauss(v, s->stream), "face factor kernel");
  }
  std::vector<int> hnbr;
  std::vector<int4> hmap;
  if (s->mesh.halo) {
    // The geometry above took the -d faces' metric from their owners through the direct periodic
    // neighbours (in a split run, a one-time exchange at set-up).  From here on each face on the
    // box boundary reads ghost element E + k, filled by the exchange before every stage from the
    // block's periodic image of its neighbour (the same face number on both).
    hnbr = nbr;
    const long long E = s->E;
    for (long long e = 0; e < E; e++) {
      const int a = (int)(e % ex), bb = (int)((e / ex) % ey), c = (int)(e / ((long long)ex * ey));
      const int idx[3] = {a, bb, c}, cnt[3] = {ex, ey, ez};
      for (int f = 0; f < 6; f++) {
        const int d = f >> 1, side = f & 1;
        if (idx[d] != (side ? cnt[d] - 1 : 0)) continue;  // not on the box boundary
        const long long g = E + (long long)hmap.size();
        hmap.push_back(make_int4(nbr[6 * e + f], f ^ 1, (int)g, f ^ 1));
        hnbr[6 * e + f] = (int)g;
      }
    }
    if ((long long)hmap.size() != s->halo.K) return fail(DG_EINVAL, "internal error: halo face count");
    for (const int4& m : hmap)
      if (m.x < 0 || m.x >= E || m.z < E || m.z >= E + s->halo.K || m.y < 0 || m.y > 5)
        return fail(DG_EINVAL, "internal error: halo map out of range");
    DG_HIP(hipStreamSynchronize(s->stream), "geometry");
    DG_HIP(hipMemcpyAsync(b + p.nbr, hnbr.data(), sizeof(int) * hnbr.size(), hipMemcpyHostToDevice, s->stream),
           "upload halo connectivity");
    DG_HIP(hipMemcpyAsync(b + p.hmap, hmap.data(), sizeof(int4) * hmap.size(), hipMemcpyHostToDevice, s->stream),
           "upload halo map");
    // the ghosts' Jacobian on their faces (read by the interior penalty), once
    DG_HIP(dg::halo_exchange_jacobian(v, s->halo, s->stream), "halo exchange of J");
  }
  DG_HIP(hipMemsetAsync(v.dU, 0, sizeof(double) * 5 * s->ntot, s->stream), "clear RK register");
  DG_HIP(hipStreamSynchronize(s->stream), "geometry");
  int rc = upload_view(s);
  if (rc) return rc;
  DG_HIP(hipStreamCreateWithFlags(&s->cap_stream, hipStreamNonBlocking), "capture stream");
  if (s->v.mixed) {
    for (int i = 0; i < dg::kMixSide; i++) {
      DG_HIP(hipStreamCreateWithFlags(&s->mix.side[i], hipStreamNonBlocking), "side stream");
      DG_HIP(hipEventCreateWithFlags(&s->mix.join[i], hipEventDisableTiming), "event");
    }
    DG_HIP(hipEventCreateWithFlags(&s->mix.fork, hipEventDisableTiming), "event");
    s->mix_concurrent = true;
  }
  hipPointerAttribute_t attr;
  if (hipPointerGetAttributes(&attr, dev_ptr) == hipSuccess && attr.device >= 0) {
    s->device = attr.device;
  } else {
    (void)hipGetLastError();
    DG_HIP(hipGetDevice(&s->device), "current device");
  }
  s->bound = true;
  s->cur = 0;
  return DG_OK;
} catch (...) {
  return abi_exception();
}

int dg_set_initial_condition(dg_solver* s, int ic, const double* params) try {
  int rc = check_bound(s);
  if (rc) return rc;
  if (ic < DG_IC_UNIFORM || ic > DG_IC_DENSITY_WAVE) return fail(DG_EINVAL, "unknown initial condition");
  if (ic != DG_IC_TGV && !params) return fail(DG_EINVAL, "this initial condition needs parameters");
  double P[9] = {0};
  const int np = ic == DG_IC_UNIFORM ? 5 : (ic == DG_IC_VORTEX ? 5 : (ic == DG_IC_DENSITY_WAVE ? 9 : 0));
  for (int k = 0; k < np; k++) {
    if (!std::isfinite(params[k])) return fail(DG_EINVAL, "non-finite initial-condition parameter");
    P[k] = params[k];
  }
  if (ic == DG_IC_UNIFORM && (!(P[0] > 0) || !(P[4] > 0)))
    return fail(DG_EINVAL, "uniform state needs rho > 0 and p > 0");
  DG_HIP(timed(s, DG_K_OTHER,
               [&] {
                 return s->v.mixed ? dg::launch_ic_mixed(s->v, s->cur, ic, P, s->stream)
                                   : dg::launch_ic(s->v, s->cur, ic, P, s->stream);
               }),
         "initial-condition kernel");
  return update_reference(s);
} catch (...) {
  return abi_exception();
}

int dg_set_state(dg_solver* s, const double* host_U, size_t n) try {
  int rc = check_bound(s);
  if (rc) return rc;
  if (!host_U) return fail(DG_EINVAL, "NULL state");
  if (n != (size_t)(5 * s->ntot)) return fail(DG_EINVAL, "state size must be 5 * number of nodes");
  std::string why;
  if (!finite_positive_state(s, host_U, why)) return fail(DG_ENONFINITE, why);
  DG_HIP(hipMemcpyAsync(s->v.U[s->cur], host_U, sizeof(double) * n, hipMemcpyHostToDevice, s->stream),
         "upload state");
  DG_HIP(hipMemsetAsync(s->v.dU, 0, sizeof(double) * n, s->stream), "clear RK register");
  DG_HIP(hipStreamSynchronize(s->stream), "upload state");
  return update_reference(s);
} catch (...) {
  return abi_exception();
}

int dg_get_state(const dg_solver* s, double* host_U, size_t n) try {
  int rc = check_bound(s);
  if (rc) return rc;
  if (!host_U) return fail(DG_EINVAL, "NULL output");
  if (n != (size_t)(5 * s->ntot)) return fail(DG_EINVAL, "state size must be 5 * number of nodes");
  DG_HIP(hipMemcpyAsync(host_U, s->v.U[s->cur], sizeof(double) * n, hipMemcpyDeviceToHost, s->stream),
         "download state");
  DG_HIP(hipStreamSynchronize(s->stream), "download state");
  return DG_OK;
} catch (...) {
  return abi_exception();
}

int dg_residual(dg_solver* s, double* host_R, size_t n) try {
  int rc = check_bound(s);
  if (rc) return rc;
  if (host_R && n != (size_t)(5 * s->ntot)) return fail(DG_EINVAL, "residual size must be 5 * number of nodes");
  DG_HIP(run_stage(s, 0.0, 0.0, 0.0, dg::kModeResidual), "residual kernels");
  if (host_R) {
    DG_HIP(hipMemcpyAsync(host_R, s->v.R, sizeof(double) * n, hipMemcpyDeviceToHost, s->stream),
           "download residual");
    DG_HIP(hipStreamSynchronize(s->stream), "residual");
  }
  return DG_OK;
} catch (...) {
  return abi_exception();
}

int dg_rk_step(dg_solver* s, double dt, int nsteps) try {
  int rc = check_bound(s);
  if (rc) return rc;
  if (nsteps < 0) return fail(DG_EINVAL, "nsteps must be >= 0");
  if (!std::isfinite(dt) || !(dt > 0)) return fail(DG_EINVAL, "dt must be positive and finite");
  // replay a captured step when the same dt recurs (several steps in this call, or the same dt
  // as the previous call); a step size seen once runs eagerly
  const bool replay = s->use_graphs && !s->profiling && nsteps > 0 && (nsteps > 1 || dt == s->last_dt);
  s->last_dt = dt;
  // every stage moves the state to the other buffer
  const int flips = kRk[s->scheme].stages & 1;
  for (int it = 0; it < nsteps;) {
    if (replay && nsteps - it >= kMultiSteps) {  // kMultiSteps steps per graph launch
      const int par = s->cur;
      if (!s->mgraph[par] || s->mgraph_dt[par] != dt) {
        rc = capture_multi_step(s, dt);
        if (rc) return rc;
      }
      DG_HIP(hipGraphLaunch(s->mgraph[par], s->stream), "RK multi-step graph launch");
      s->cur ^= (kMultiSteps * flips) & 1;
      it += kMultiSteps;
    } else if (replay) {
      const int par = s->cur;
      if (!s->graph[par] || s->graph_dt[par] != dt) {
        rc = capture_step(s, dt);
        if (rc) return rc;
      }
      DG_HIP(hipGraphLaunch(s->graph[par], s->stream), "RK-step graph launch");
      s->cur ^= flips;
      it++;
    } else {
      DG_HIP(run_step(s, dt), "RK stage kernels");
      it++;
    }
  }
  return DG_OK;
} catch (...) {
  return abi_exception();
}

int dg_rk_step_adaptive(dg_solver* s, double cfl, int nsteps, double* t_advanced) try {
  int rc = check_bound(s);
  if (rc) return rc;
  if (nsteps < 0) return fail(DG_EINVAL, "nsteps must be >= 0");
  if (!std::isfinite(cfl) || !(cfl > 0)) return fail(DG_EINVAL, "cfl must be positive and finite");
  DG_HIP(dg::launch_adapt_reset(s->v, s->stream), "adaptive-step reset");
  const bool replay = s->use_graphs && !s->profiling && nsteps > 1;
  s->v.dtp = s->v.adapt;  // the stage kernels read the step size the device chose
  hipError_t err = hipSuccess;
  const char* what = "adaptive RK step";
  for (int it = 0; it < nsteps && err == hipSuccess; it++) {
    if (replay) {
      const int par = s->cur;
      if (!s->agraph[par] || s->agraph_cfl[par] != cfl) {
        rc = capture_adaptive_step(s, cfl);
        if (rc) {
          s->v.dtp = nullptr;
          return rc;
        }
      }
      err = hipGraphLaunch(s->agraph[par], s->stream);
      what = "adaptive-step graph launch";
      s->cur ^= 1;  // an odd number of stages, each moving the state to the other buffer
    } else {
      err = run_step_size(s, cfl);
      if (err == hipSuccess) err = run_step(s, 0.0);
    }
  }
  s->v.dtp = nullptr;
  DG_HIP(err, what);
  double h[4];
  DG_HIP(hipMemcpyAsync(h, s->v.adapt, sizeof(h), hipMemcpyDeviceToHost, s->stream), "adaptive-step result");
  DG_HIP(hipStreamSynchronize(s->stream), "adaptive-step result");
  if (t_advanced) *t_advanced = h[1];
  if (h[2] > 0)
    return fail(DG_ENONFINITE, "the state held non-finite or non-physical values (rho or p <= 0) at the start of a "
                               "step; from there on the steps had size 0");
  return DG_OK;
} catch (...) {
  return abi_exception();
}

int dg_solver_set_scheme(dg_solver* s, int scheme) try {
  if (!s) return fail(DG_EINVAL, "NULL solver");
  if (scheme != DG_RK3_WILLIAMSON && scheme != DG_RK4_CARPENTER_KENNEDY) return fail(DG_EINVAL, "unknown time scheme");
  if (scheme != s->scheme) {
    drop_graphs(s);
    s->scheme = scheme;
  }
  return DG_OK;
} catch (...) {
  return abi_exception();
}

int dg_solver_use_graphs(dg_solver* s, int enable) try {
  if (!s) return fail(DG_EINVAL, "NULL solver");
  s->use_graphs = enable != 0;
  if (!s->use_graphs) drop_graphs(s);
  return DG_OK;
} catch (...) {
  return abi_exception();
}

int dg_solver_set_tiles(dg_solver* s, int tiles) try {
  if (!s) return fail(DG_EINVAL, "NULL solver");
  if (!s->v.mixed) {
    if (tiles != 0) return fail(DG_EINVAL, "uniform-order meshes have one launch shape (tiles = 0)");
    return DG_OK;
  }
  if (tiles < 0 || tiles >= (1 << dg::kMixBuckets)) return fail(DG_EINVAL, "tiles must be a 6-bit mask");
  s->mix_tiles = tiles;
  drop_graphs(s);
  return DG_OK;
} catch (...) {
  return abi_exception();
}

int dg_autotune(dg_solver* s, int* tiles, double* us) try {
  int rc = check_bound(s);
  if (rc) return rc;
  if (!s->v.mixed) {
    if (tiles) *tiles = 0;
    if (us) *us = 0.0;
    return DG_OK;
  }
  const int reps = 5;
  hipEvent_t a = nullptr, b = nullptr;
  DG_HIP(hipEventCreate(&a), "event");
  if (hipEventCreate(&b) != hipSuccess) {
    (void)hipEventDestroy(a);
    return fail(DG_EHIP, "event");
  }
  hipError_t err = hipSuccess;
  int best_tiles = 0;
  double total = 0.0;
  err = dg::launch_faces_mixed(s->v, s->cur, s->stream);  // the buckets read the face fluxes
  for (int bk = 0; bk < dg::kMixBuckets && err == hipSuccess; bk++) {
    if (s->v.mix_cnt[bk] == 0) continue;
    double best = 1e300;
    for (int npl = 1; npl <= 2 && err == hipSuccess; npl++) {
      err = dg::launch_stage_mixed_bucket(s->v, bk, npl, s->cur, 0.0, 0.0, 0.0, dg::kModeResidual, s->stream);
      if (err == hipSuccess) err = hipEventRecord(a, s->stream);
      for (int r = 0; r < reps && err == hipSuccess; r++)
        err = dg::launch_stage_mixed_bucket(s->v, bk, npl, s->cur, 0.0, 0.0, 0.0, dg::kModeResidual, s->stream);
      if (err == hipSuccess) err = hipEventRecord(b, s->stream);
      if (err == hipSuccess) err = hipEventSynchronize(b);
      float ms = 0.f;
      if (err == hipSuccess) err = hipEventElapsedTime(&ms, a, b);
      const double t_us = 1e3 * ms / reps;
      if (err == hipSuccess && t_us < best) {
        best = t_us;
        best_tiles = npl == 2 ? (best_tiles | (1 << bk)) : (best_tiles & ~(1 << bk));
      }
    }
    total += best;
  }
  (void)hipEventDestroy(a);
  (void)hipEventDestroy(b);
  if (err != hipSuccess) return hip_fail(err, "autotune");
  s->mix_tiles = best_tiles;
  drop_graphs(s);
  if (tiles) *tiles = best_tiles;
  if (us) *us = total;
  return DG_OK;
} catch (...) {
  return abi_exception();
}

int dg_diagnostics(dg_solver* s, dg_diag* out) try {
  int rc = check_bound(s);
  if (rc) return rc;
  if (!out) return fail(DG_EINVAL, "NULL output");
  DG_HIP(timed(s, DG_K_DIAGNOSTICS, [&] { return launch_diag_any(s); }), "diagnostics kernels");
  double h[dg::kDiagSlots];
  DG_HIP(hipMemcpyAsync(h, s->v.diag, sizeof(h), hipMemcpyDeviceToHost, s->stream), "download diagnostics");
  DG_HIP(hipStreamSynchronize(s->stream), "diagnostics");
  for (int k = 0; k < 5; k++) out->mass[k] = h[k];
  out->entropy_paper = h[5];
  out->entropy = h[6];
  out->volume = h[13];
  out->ke = h[7] / h[13];
  out->enstrophy = h[8] / h[13];
  out->lambda_max = h[9];
  out->rho_min = h[10];
  out->p_min = h[11];
  out->nonfinite = (long long)h[12];
  return DG_OK;
} catch (...) {
  return abi_exception();
}

int dg_diagnostics_noalloc(dg_solver* s, dg_diag* dev_out) try {
  int rc = check_bound(s);
  if (rc) return rc;
  if (!dev_out) return fail(DG_EINVAL, "NULL output");
  if (s->E > kNoAllocMaxElements)
    return fail(DG_EUNSUPPORTED, "dg_diagnostics_noalloc takes meshes of at most " +
                                     std::to_string(kNoAllocMaxElements) + " elements (its static scratch "
                                     "holds that many partial sums); use dg_diagnostics");
  DeviceGuard guard;
  int dev = 0;
  DG_HIP(hipGetDevice(&dev), "current device");
  if (dev != s->device) {
    guard.prev = dev;
    DG_HIP(hipSetDevice(s->device), "select the solver's device");
  }
  double* ptr = nullptr;
  DG_HIP(scratch_on(s->device, &ptr), "address of the static diagnostics scratch");
  dg::View v = s->v;  // the solver's view with the partial sums and the slots in the scratch
  v.part = ptr;
  v.diag = ptr + kNoAllocMaxElements * dg::kDiagSlots;
  DG_HIP(v.mixed ? dg::launch_diagnostics_mixed(v, s->cur, s->stream) : dg::launch_diagnostics(v, s->cur, s->stream),
         "diagnostics kernels");
  hipLaunchKernelGGL(diag_record_kernel, dim3(1), dim3(64), 0, s->stream, v.diag, dev_out);
  DG_HIP(hipGetLastError(), "diagnostics record kernel");
  return DG_OK;
} catch (...) {
  return abi_exception();
}

int dg_suggest_dt(dg_solver* s, double cfl, double* dt) try {
  if (!dt) return fail(DG_EINVAL, "NULL output");
  if (!(cfl > 0) || !std::isfinite(cfl)) return fail(DG_EINVAL, "cfl must be positive");
  dg_diag d;
  int rc = dg_diagnostics(s, &d);
  if (rc) return rc;
  if (d.nonfinite || !(d.lambda_max > 0)) return fail(DG_ENONFINITE, "state is not finite");
  const dg::View& v = s->v;
  const double hmin = std::fmin(v.h[0], std::fmin(v.h[1], v.h[2]));
  const double n1 = v.N + 1.0;
  double r = cfl * hmin / (n1 * n1 * d.lambda_max);
  const double mu = mu_eff(s);
  if (mu > 0.0) {
    const double rv = 0.25 * hmin * hmin / (n1 * n1 * n1 * n1 * s->phys.gamma * mu / (s->phys.Pr * d.rho_min));
    r = std::fmin(r, rv);
  }
  *dt = r;
  return DG_OK;
} catch (...) {
  return abi_exception();
}

int dg_get_geometry(dg_solver* s, double* host_X, double* host_Ja, double* host_J) try {
  int rc = check_bound(s);
  if (rc) return rc;
  const size_t nt = (size_t)s->ntot;
  if (host_X)
    DG_HIP(hipMemcpyAsync(host_X, s->v.X, sizeof(double) * 3 * nt, hipMemcpyDeviceToHost, s->stream), "X");
  if (host_Ja)
    DG_HIP(hipMemcpyAsync(host_Ja, s->v.Ja, sizeof(double) * 9 * nt, hipMemcpyDeviceToHost, s->stream), "Ja");
  if (host_J)
    DG_HIP(hipMemcpyAsync(host_J, s->v.J, sizeof(double) * nt, hipMemcpyDeviceToHost, s->stream), "J");
  DG_HIP(hipStreamSynchronize(s->stream), "geometry download");
  return DG_OK;
} catch (...) {
  return abi_exception();
}

int dg_device_pointers(dg_solver* s, void** dev_U, void** dev_R) try {
  int rc = check_bound(s);
  if (rc) return rc;
  if (dev_U) *dev_U = s->v.U[s->cur];
  if (dev_R) *dev_R = s->v.R;
  return DG_OK;
} catch (...) {
  return abi_exception();
}

int dg_synchronize(dg_solver* s) try {
  int rc = check_bound(s);
  if (rc) return rc;
  DG_HIP(hipStreamSynchronize(s->stream), "synchronize");
  return DG_OK;
} catch (...) {
  return abi_exception();
}

int dg_profile_begin(dg_solver* s) try {
  int rc = check_bound(s);
  if (rc) return rc;
  s->profiling = true;
  s->prof.clear();
  s->ev_used = 0;
  return DG_OK;
} catch (...) {
  return abi_exception();
}

int dg_profile_end(dg_solver* s, dg_profile* out) try {
  int rc = check_bound(s);
  if (rc) return rc;
  if (!out) return fail(DG_EINVAL, "NULL output");
  if (!s->profiling) return fail(DG_ESTATE, "no profile region is open");
  s->profiling = false;
  DG_HIP(hipStreamSynchronize(s->stream), "profile synchronize");
  for (int k = 0; k < DG_K_CLASSES; k++) {
    out->ms[k] = 0.0;
    out->launches[k] = 0;
  }
  for (const ProfRecord& r : s->prof) {
    float ms = 0.f;
    DG_HIP(hipEventElapsedTime(&ms, r.a, r.b), "event elapsed time");
    out->ms[r.cls] += ms;
    out->launches[r.cls] += 1;
  }
  s->prof.clear();
  s->ev_used = 0;
  return DG_OK;
} catch (...) {
  return abi_exception();
}

// ------------------------------------------------------------------ batches of solvers
struct dg_batch {
  struct Group {  // uniform-order members of one order, precision and surface-flux family, viscous or not
    int N;
    bool fp32, visc;
    int fx;   // flux family
    bool xv;  // BR2 or interior-penalty face viscous flux
    std::vector<int> idx;
  };
  struct Graph {
    std::vector<int> par;       // state buffer of every member at the step start
    std::vector<double> dts;
    int steps;                  // RK steps in the graph: 1 or kMultiSteps
    hipGraphExec_t exec;
  };
  std::vector<dg_solver*> m;
  std::vector<Group> groups;    // each with at most kMaxBatch members
  std::vector<int> solo;        // mixed-order and Gauss-Legendre members: launches of their own
  hipStream_t stream = nullptr;
  hipStream_t cap_stream = nullptr;
  std::vector<Graph> graphs;    // most recent last
  std::vector<double> last_dts;
  bool use_graphs = true;
  int scheme = DG_RK3_WILLIAMSON;  // the members' common time scheme
};

namespace {

constexpr size_t kBatchGraphs = 8;  // one- and multi-step graphs of both parities, twice

void batch_drop_graphs(dg_batch* b) {
  if (b->graphs.empty()) return;
  (void)hipStreamSynchronize(b->stream);
  for (auto& g : b->graphs) (void)hipGraphExecDestroy(g.exec);
  b->graphs.clear();
}

// one RK stage of every member on stream st; afterwards every member's state has moved to its
// other buffer
hipError_t batch_stage(dg_batch* b, const double* dts, int k, hipStream_t st) {
  for (dg_solver* s : b->m) {
    hipError_t e = pre_stage(s, s->cur, st);
    if (e != hipSuccess) return e;
  }
  for (const auto& g : b->groups) {
    dg::BatchArgs B;
    std::memset(&B, 0, sizeof(B));
    B.n = (int)g.idx.size();
    B.start[0] = 0;
    for (int j = 0; j < B.n; j++) {
      dg_solver* s = b->m[g.idx[j]];
      B.view[j] = s->dev_view;
      B.cur[j] = s->cur;
      B.dt[j] = dts[g.idx[j]];
      B.start[j + 1] = B.start[j] + (int)s->E;
    }
    hipError_t e;
    if (g.visc) {
      e = dg::launch_gradient_batch(B, g.N, g.fp32, g.xv, st);
      if (e != hipSuccess) return e;
    }
    e = dg::launch_stage_batch(B, g.N, g.fp32, g.visc, g.fx, kRk[b->scheme].A[k], kRk[b->scheme].B[k],
                               dg::kModeRK, st);
    if (e != hipSuccess) return e;
  }
  for (int i : b->solo) {
    dg_solver* s = b->m[i];
    const double A = kRk[b->scheme].A[k], Bk = kRk[b->scheme].B[k];
    hipError_t e;
    if (s->v.mixed) {
      e = dg::launch_stage_mixed(s->v, s->cur, dts[i], A, Bk, dg::kModeRK, s->mix_tiles, st,
                                 s->mix_concurrent ? &s->mix : nullptr);
    } else if (s->v.gauss) {
      e = dg::launch_stage_gauss(s->v, s->cur, dts[i], A, Bk, dg::kModeRK, st);
    } else {  // spectral vanishing viscosity: the solver's own stage sequence
      if (svv_folded(s)) {
        if (s->v.visc_flux == DG_VISC_BR1) {
          e = dg::launch_grad_svv(s->v, s->cur, s->svv, st);
        } else {
          e = dg::launch_gradient(s->v, s->cur, st);
          if (e == hipSuccess) e = dg::launch_svv_flux(s->v, s->cur, s->svv, st);
        }
        dg::View vf = s->v;
        vf.Fa = s->svv.Fa;
        if (e == hipSuccess) e = dg::launch_stage(vf, s->cur, dts[i], A, Bk, dg::kModeRK, st);
      } else {
        e = s->v.viscous ? dg::launch_gradient(s->v, s->cur, st) : hipSuccess;
        if (e == hipSuccess) e = dg::launch_stage(s->v, s->cur, dts[i], A, Bk, dg::kModeRK, st);
        if (e == hipSuccess) e = dg::launch_svv(s->v, s->cur, s->svv, dts[i], Bk, dg::kModeRK, st);
      }
    }
    if (e != hipSuccess) return e;
  }
  for (dg_solver* s : b->m) s->cur ^= 1;
  return hipSuccess;
}

int batch_capture(dg_batch* b, const double* dts, int steps) {
  const size_t n = b->m.size();
  dg_batch::Graph G;
  G.par.resize(n);
  for (size_t i = 0; i < n; i++) G.par[i] = b->m[i]->cur;
  G.dts.assign(dts, dts + n);
  G.steps = steps;
  hipGraph_t g = nullptr;
  hipError_t err = hipStreamBeginCapture(b->cap_stream, hipStreamCaptureModeThreadLocal);
  if (err == hipSuccess) {
    for (int st = 0; st < steps && err == hipSuccess; st++)
      for (int k = 0; k < kRk[b->scheme].stages && err == hipSuccess; k++)
        err = batch_stage(b, dts, k, b->cap_stream);
    const hipError_t e2 = hipStreamEndCapture(b->cap_stream, &g);
    if (err == hipSuccess) err = e2;
  }
  for (size_t i = 0; i < n; i++) b->m[i]->cur = G.par[i];  // capture launched nothing
  if (err != hipSuccess) {
    if (g) (void)hipGraphDestroy(g);
    return hip_fail(err, "capture of a batch RK step");
  }
  err = hipGraphInstantiate(&G.exec, g, nullptr, nullptr, 0);
  (void)hipGraphDestroy(g);
  if (err != hipSuccess) return hip_fail(err, "instantiation of the batch RK-step graph");
  if (b->graphs.size() == kBatchGraphs) {
    (void)hipStreamSynchronize(b->stream);
    (void)hipGraphExecDestroy(b->graphs.front().exec);
    b->graphs.erase(b->graphs.begin());
  }
  b->graphs.push_back(std::move(G));
  return DG_OK;
}

}  // namespace

int dg_batch_create(dg_solver* const* solvers, int n, void* hip_stream, dg_batch** out) try {
  if (!solvers || !out) return fail(DG_EINVAL, "NULL argument");
  *out = nullptr;
  if (n < 1) return fail(DG_EINVAL, "a batch needs at least one solver");
  for (int i = 0; i < n; i++) {
    int rc = check_bound(solvers[i]);
    if (rc) return rc;
    if (solvers[i]->mesh.halo) return fail(DG_EUNSUPPORTED, "solvers of halo boxes are not batched");
    for (int j = 0; j < i; j++)
      if (solvers[j] == solvers[i]) return fail(DG_EINVAL, "a solver appears twice in the batch");
  }
  for (int i = 1; i < n; i++)
    if (solvers[i]->scheme != solvers[0]->scheme)
      return fail(DG_EINVAL, "the solvers of a batch must use one time scheme");
  std::unique_ptr<dg_batch> b(new dg_batch);
  b->m.assign(solvers, solvers + n);
  b->scheme = solvers[0]->scheme;
  b->stream = static_cast<hipStream_t>(hip_stream);
  for (int i = 0; i < n; i++) {
    const dg_solver* s = solvers[i];
    if (s->v.mixed || s->v.gauss || s->svv_on) {  // launched one by one within the batch's stages
      b->solo.push_back(i);
      continue;
    }
    const bool fp32 = s->v.fp32 != 0, visc = s->v.viscous != 0;
    const int fx = dg::flux_family(s->v.vol, s->v.surf);
    const bool xv = s->v.viscous && s->v.visc_flux != 0;
    dg_batch::Group* g = nullptr;
    for (auto& x : b->groups)
      if (x.N == s->v.N && x.fp32 == fp32 && x.visc == visc && x.fx == fx && x.xv == xv && (int)x.idx.size() < dg::kMaxBatch)
        g = &x;
    if (!g) {
      b->groups.push_back({s->v.N, fp32, visc, fx, xv, {}});
      g = &b->groups.back();
    }
    g->idx.push_back(i);
  }
  long long blocks = 0;
  for (const auto& g : b->groups) {
    blocks = 0;
    for (int i : g.idx) blocks += b->m[i]->E;
    if (blocks >= (1LL << 31)) return fail(DG_EINVAL, "a batched launch would exceed 2^31 workgroups");
  }
  hipError_t e = hipStreamCreateWithFlags(&b->cap_stream, hipStreamNonBlocking);
  if (e != hipSuccess) return hip_fail(e, "capture stream");
  *out = b.release();
  return DG_OK;
} catch (...) {
  return abi_exception();
}

int dg_batch_rk_step(dg_batch* b, const double* dts, int nsteps) try {
  if (!b || !dts) return fail(DG_EINVAL, "NULL argument");
  if (nsteps < 0) return fail(DG_EINVAL, "nsteps must be >= 0");
  const size_t n = b->m.size();
  for (size_t i = 0; i < n; i++)
    if (!std::isfinite(dts[i]) || !(dts[i] > 0)) return fail(DG_EINVAL, "every dt must be positive and finite");
  const bool same = b->last_dts.size() == n && std::equal(dts, dts + n, b->last_dts.begin());
  const bool replay = b->use_graphs && nsteps > 0 && (nsteps > 1 || same);
  b->last_dts.assign(dts, dts + n);
  for (int it = 0; it < nsteps;) {
    if (!replay) {
      for (int k = 0; k < kRk[b->scheme].stages; k++)
        DG_HIP(batch_stage(b, dts, k, b->stream), "batch RK stage kernels");
      it++;
      continue;
    }
    // kMultiSteps steps per graph launch while that many remain, then single steps
    const int steps = nsteps - it >= kMultiSteps ? kMultiSteps : 1;
    const dg_batch::Graph* G = nullptr;
    for (const auto& g : b->graphs) {
      bool hit = g.steps == steps && std::equal(dts, dts + n, g.dts.begin());
      for (size_t i = 0; hit && i < n; i++) hit = g.par[i] == b->m[i]->cur;
      if (hit) G = &g;
    }
    if (!G) {
      int rc = batch_capture(b, dts, steps);
      if (rc) return rc;
      G = &b->graphs.back();
    }
    DG_HIP(hipGraphLaunch(G->exec, b->stream), "batch RK-step graph launch");
    const int flips = (steps * kRk[b->scheme].stages) & 1;  // each stage moves every state
    for (dg_solver* s : b->m) s->cur ^= flips;
    it += steps;
  }
  return DG_OK;
} catch (...) {
  return abi_exception();
}

int dg_batch_use_graphs(dg_batch* b, int enable) try {
  if (!b) return fail(DG_EINVAL, "NULL batch");
  b->use_graphs = enable != 0;
  if (!b->use_graphs) batch_drop_graphs(b);
  return DG_OK;
} catch (...) {
  return abi_exception();
}

int dg_batch_launches(const dg_batch* b, int* launches_per_stage) try {
  if (!b || !launches_per_stage) return fail(DG_EINVAL, "NULL argument");
  int k = 0;
  for (const auto& g : b->groups) k += g.visc ? 2 : 1;
  *launches_per_stage = k + (int)b->solo.size();
  return DG_OK;
} catch (...) {
  return abi_exception();
}

void dg_batch_destroy(dg_batch* b) try {
  if (!b) return;
  batch_drop_graphs(b);
  if (b->cap_stream) (void)hipStreamDestroy(b->cap_stream);
  delete b;
} catch (...) {
}

void dg_solver_destroy(dg_solver* s) try {
  if (!s) return;
  if (s->bound) (void)hipStreamSynchronize(s->stream);
  drop_graphs(s);
  if (s->cap_stream) (void)hipStreamDestroy(s->cap_stream);
  for (int i = 0; i < dg::kMixSide; i++) {
    if (s->mix.side[i]) (void)hipStreamSynchronize(s->mix.side[i]);
    if (s->mix.side[i]) (void)hipStreamDestroy(s->mix.side[i]);
    if (s->mix.join[i]) (void)hipEventDestroy(s->mix.join[i]);
  }
  if (s->mix.fork) (void)hipEventDestroy(s->mix.fork);
  for (hipEvent_t e : s->ev_pool) (void)hipEventDestroy(e);
  delete s;
} catch (...) {
}

}  // extern "C"
