// Host runtime of the C ABI declared in include/rhd.h: parameter validation,
// workspace carving, stage-kernel launches on the caller's stream and the
// device error word. No device memory is allocated here.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <climits>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/rhd.h"
#include "rhd_internal.hpp"

struct Layout_ptrs {
  double* states;
  double* lam;
};

struct rhd_handle {
  rhd_params p;
  rhd::DevParams dp;
  const double* rho;
  const double* kP;
  const double* kF;           // == kP when aliased
  hipStream_t stream;
  char* ws;
  size_t ws_bytes;
  int adj_len;
  // carved workspace
  unsigned long long* err;    // 2 words
  double* yhalf;              // nvar * N
  double* partial;            // reduction scratch
  int partial_blocks;
  Layout_ptrs adj;            // adjoint storage (segment states and adjoint scratch)
  // last error
  rhd_status last;
  long long last_cell;
  std::string last_msg;
};

namespace {

constexpr size_t kAlign = 256;
constexpr int kPartialBlocks = 1024;

size_t align_up(size_t x) { return (x + kAlign - 1) / kAlign * kAlign; }

int nvar_of(const rhd_params* p) { return 2 + 2 * p->ndim; }

long long ncells(const rhd_params* p) { return p->n[0] * p->n[1] * p->n[2]; }

bool finite_pos(double x) { return std::isfinite(x) && x > 0.0; }

// Returns an empty string when valid, else the reason.
std::string validate(const rhd_params* p) {
  if (!p) return "params is NULL";
  if (p->ndim < 1 || p->ndim > 3) return "ndim must be 1, 2 or 3";
  for (int d = 0; d < 3; ++d) {
    if (d < p->ndim) {
      if (p->n[d] < 1) return "n[d] must be >= 1 on active axes";
      if (p->n[d] > (1LL << 24)) return "n[d] too large";
      if (p->bc[d] != RHD_BC_PERIODIC && p->bc[d] != RHD_BC_REFLECT && p->bc[d] != RHD_BC_INFLOW)
        return "bc must be periodic, reflect or inflow";
      if (p->bc[d] != RHD_BC_PERIODIC && p->n[d] < 3) return "reflecting and inflow axes need n >= 3";
    } else if (p->n[d] != 1) {
      return "axes beyond ndim must have n = 1";
    }
  }
  if (ncells(p) > (1LL << 40)) return "grid too large";
  if (!finite_pos(p->dx)) return "dx must be > 0";
  if (!finite_pos(p->c)) return "c must be > 0";
  if (!finite_pos(p->chat) || p->chat > p->c) return "chat must satisfy 0 < chat <= c";
  if (!std::isfinite(p->gamma) || p->gamma <= 1.0) return "gamma must be > 1";
  if (!finite_pos(p->a_r)) return "a_r must be > 0";
  if (!finite_pos(p->kB_over_mu)) return "kB_over_mu must be > 0";
  if (p->closure != RHD_CLOSURE_M1 && p->closure != RHD_CLOSURE_EDDINGTON) return "unknown closure";
  if (p->v_order != 1 && p->v_order != 2) return "v_order must be 1 or 2";
  if (p->precision != RHD_FP64 && p->precision != RHD_MIXED) return "unknown precision";
  if (p->newton_maxit < 1 || p->newton_maxit > 100000) return "newton_maxit out of range";
  if (p->outer_maxit < 1 || p->outer_maxit > 100000) return "outer_maxit out of range";
  if (p->scheme != RHD_SCHEME_PDARS && p->scheme != RHD_SCHEME_RK2SSP) return "unknown scheme";
  if (!(p->newton_rtol > 0.0) || !std::isfinite(p->newton_rtol)) return "newton_rtol must be > 0";
  if (!(p->outer_rtol >= 0.0) || !std::isfinite(p->outer_rtol)) return "outer_rtol must be >= 0";
  if (!(p->hll_eps_cells >= 0.0) || !std::isfinite(p->hll_eps_cells))
    return "hll_eps_cells must be >= 0 and finite";
  if (!std::isfinite(p->kappa_T_power)) return "kappa_T_power must be finite";
  if (p->kappa_T_power != 0.0 && p->hll_eps_cells > 0.0)
    return "kappa_T_power != 0 needs hll_eps_cells = 0";
  if (!std::isfinite(p->inflow_E) || !std::isfinite(p->inflow_F)) return "inflow state must be finite";
  return "";
}

struct Layout {
  size_t err, yhalf, partial, adj, states, lam, total;
};

Layout layout(const rhd_params* p, int adj_len) {
  const size_t N = (size_t)ncells(p);
  const size_t nv = (size_t)nvar_of(p);
  Layout L{};
  size_t off = 0;
  L.err = off;
  off = align_up(off + 2 * sizeof(unsigned long long));
  L.yhalf = off;
  off = align_up(off + nv * N * sizeof(double));
  L.partial = off;
  off = align_up(off + (size_t)kPartialBlocks * 4 * sizeof(double));
  L.adj = off;
  if (adj_len > 0) {
    // y^1..y^k and y^{1/2}..y^{k-1/2} of a segment (y^0 is the caller's state0),
    // and two adjoint vectors (the third is the caller's lambda)
    L.states = off;
    off = align_up(off + (size_t)(2 * adj_len) * nv * N * sizeof(double));
    L.lam = off;
    off = align_up(off + 2 * nv * N * sizeof(double));
  }
  L.total = off;
  return L;
}

// The longest adjoint segment (steps) whose storage fits in ws_bytes after the
// forward part of the layout, capped at kMaxSegment; 0 if none fits.
constexpr int kMaxSegment = 1000000;
int adjoint_capacity(const rhd_params* p, size_t ws_bytes) {
  if (layout(p, 1).total > ws_bytes) return 0;
  // the layout grows by 2 states per step: bisect on the exact size
  int lo = 1, hi = kMaxSegment;
  while (lo < hi) {
    const int mid = lo + (hi - lo + 1) / 2;
    if (layout(p, mid).total <= ws_bytes) lo = mid;
    else hi = mid - 1;
  }
  return lo;
}

rhd::DevParams make_dev(const rhd_params* p, bool alias) {
  rhd::DevParams d{};
  d.ndim = p->ndim;
  d.closure = p->closure;
  d.v_order = p->v_order;
  for (int k = 0; k < 3; ++k) {
    d.bc[k] = p->bc[k];
    d.n[k] = (int)p->n[k];
  }
  d.newton_maxit = p->newton_maxit;
  d.outer_maxit = p->outer_maxit;
  d.N = ncells(p);
  d.dx = p->dx;
  d.inv_dx = 1.0 / p->dx;
  d.c = p->c;
  d.chat = p->chat;
  d.c_over_chat = p->c / p->chat;
  d.chat_over_c = p->chat / p->c;
  d.c_chat = p->c * p->chat;
  d.inv_c_chat = 1.0 / (p->c * p->chat);
  d.inv_c2 = 1.0 / (p->c * p->c);
  d.a_r = p->a_r;
  d.gamma = p->gamma;
  d.gm1 = p->gamma - 1.0;
  d.inv_gm1 = 1.0 / d.gm1;
  d.cv_mass = p->kB_over_mu / (p->gamma - 1.0);
  d.inv_cv_mass = 1.0 / d.cv_mass;
  d.newton_rtol = p->newton_rtol;
  d.outer_rtol = p->outer_rtol;
  d.kF_alias = alias ? 1 : 0;
  d.scheme = p->scheme;
  d.eps_dx = p->hll_eps_cells * p->dx;
  d.kT_pow = p->kappa_T_power;
  d.kT_isint = (p->kappa_T_power == std::nearbyint(p->kappa_T_power) && std::fabs(p->kappa_T_power) <= 16.0);
  d.kT_int = d.kT_isint ? (int)p->kappa_T_power : 0;
  d.inflow_E = p->inflow_E;
  d.inflow_F = p->inflow_F;
  return d;
}

rhd_status set_err(rhd_handle* h, rhd_status st, long long cell, const std::string& msg) {
  h->last = st;
  h->last_cell = cell;
  h->last_msg = msg;
  return st;
}

rhd_status hip_fail(rhd_handle* h, hipError_t e, const char* where) {
  return set_err(h, RHD_EHIP, -1, std::string(where) + ": " + hipGetErrorString(e));
}

// Read the device error word (one synchronisation of the handle's stream).
rhd_status finish(rhd_handle* h) {
  unsigned long long w[2] = {0, 0};
  hipError_t e = hipMemcpyAsync(w, h->err, sizeof(w), hipMemcpyDeviceToHost, h->stream);
  if (e != hipSuccess) return hip_fail(h, e, "hipMemcpyAsync(error word)");
  e = hipStreamSynchronize(h->stream);
  if (e != hipSuccess) return hip_fail(h, e, "hipStreamSynchronize");
  if (w[1] == 0) return set_err(h, RHD_OK, -1, "");
  const long long cell = (w[0] == ULLONG_MAX) ? -1 : (long long)w[0];
  if (w[1] & rhd::ERR_NEWTON)
    return set_err(h, RHD_ENEWTON, cell, "inner Newton did not converge (smallest failing cell reported)");
  return set_err(h, RHD_ENONPHYS, cell, "non-physical state: E <= 0 or internal energy <= 0");
}

bool misaligned(const void* ptr) { return (reinterpret_cast<uintptr_t>(ptr) % 8) != 0; }

// nsteps PD-ARS (or RK2-SSP) steps of state on the handle's stream: one
// single-workgroup launch for a 1-D line that fits one workgroup, else two
// fused stage kernels per step (y^{n+1/2} in the workspace).
hipError_t run_steps(const rhd::DevParams& dp, bool mixed, double* state, double* yhalf,
                     const double* rho, const double* kP, const double* kF, double dt, int nsteps,
                     unsigned long long* err, hipStream_t stream) {
  if (rhd::line_kernel_applies(dp))
    return rhd::launch_line_steps(dp, mixed, state, rho, kP, kF, dt, nsteps, err, stream);
  for (int n = 0; n < nsteps; ++n) {
    hipError_t e = rhd::launch_stage(dp, rhd::MODE_STAGE1, mixed, state, state, yhalf, rho, kP,
                                     kF, dt, err, stream);
    if (e != hipSuccess) return e;
    e = rhd::launch_stage(dp, rhd::MODE_STAGE2, mixed, yhalf, state, state, rho, kP, kF, dt, err,
                          stream);
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

hipError_t run_steps(rhd_handle* h, double* state, double dt, int nsteps) {
  return run_steps(h->dp, h->p.precision == RHD_MIXED, state, h->yhalf, h->rho, h->kP, h->kF, dt,
                   nsteps, h->err, h->stream);
}

// ---------------------------------------------------------------------------
// Scratch of the allocation-free step (rhd_step_noalloc): the error word at
// offset 0 and y^{n+1/2} from offset 256, in a file-scope device array that
// every GPU the library runs on holds until the process ends. Host code uses
// its device address from hipGetSymbolAddress (one lookup per device, with that
// device current), never the array's name.
// ---------------------------------------------------------------------------
constexpr size_t kNoallocScratchBytes = size_t(64) << 20;
constexpr size_t kNoallocYhalf = 256;
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};

}  // namespace

static __device__ __align__(256) unsigned char scratch[kNoallocScratchBytes];

namespace {

// Device address of `scratch` on the current device (looked up once per device).
hipError_t noalloc_scratch(void** out) {
  int dev = -1;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* ptr = nullptr;
    e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    if (!ptr) return hipErrorInvalidSymbol;
    g_scratch_ptr[dev] = ptr;
  }
  *out = g_scratch_ptr[dev];
  return hipSuccess;
}

}  // namespace

extern "C" {

size_t rhd_workspace_bytes(const rhd_params* p, int32_t adjoint_segment_len) {
  if (!validate(p).empty() || adjoint_segment_len < 0) return 0;
  return layout(p, adjoint_segment_len).total;
}

rhd_status rhd_create(const rhd_params* p, const double* rho, const double* kappa_P,
                      const double* kappa_F, void* workspace, size_t ws_bytes, void* hip_stream,
                      rhd_handle** out) {
  if (!out) return RHD_EINVAL;
  if (!validate(p).empty()) return RHD_EINVAL;
  if (!rho || !kappa_P || misaligned(rho) || misaligned(kappa_P) || misaligned(kappa_F))
    return RHD_EINVAL;
  const bool alias = (kappa_F == nullptr || kappa_F == kappa_P);
  if (!workspace || (reinterpret_cast<uintptr_t>(workspace) % kAlign) != 0 ||
      ws_bytes < layout(p, 0).total)
    return RHD_EWORKSPACE;
  const int adjoint_segment_len = adjoint_capacity(p, ws_bytes);
  const Layout L = layout(p, adjoint_segment_len);
  rhd_handle* h = new (std::nothrow) rhd_handle();
  if (!h) return RHD_EINVAL;
  h->p = *p;
  h->dp = make_dev(p, alias);
  h->rho = rho;
  h->kP = kappa_P;
  h->kF = alias ? kappa_P : kappa_F;
  h->stream = reinterpret_cast<hipStream_t>(hip_stream);
  h->ws = reinterpret_cast<char*>(workspace);
  h->ws_bytes = ws_bytes;
  h->adj_len = adjoint_segment_len;
  h->err = reinterpret_cast<unsigned long long*>(h->ws + L.err);
  h->yhalf = reinterpret_cast<double*>(h->ws + L.yhalf);
  h->partial = reinterpret_cast<double*>(h->ws + L.partial);
  h->partial_blocks = kPartialBlocks;
  if (adjoint_segment_len > 0) {
    h->adj.states = reinterpret_cast<double*>(h->ws + L.states);
    h->adj.lam = reinterpret_cast<double*>(h->ws + L.lam);
  } else {
    h->adj = Layout_ptrs{nullptr, nullptr};
  }
  h->last = RHD_OK;
  h->last_cell = -1;
  *out = h;
  return RHD_OK;
}

rhd_status rhd_step(rhd_handle* h, double* state, double dt, int32_t nsteps) {
  if (!h) return RHD_EINVAL;
  if (!state || misaligned(state) || !std::isfinite(dt) || !(dt > 0.0) || nsteps < 0)
    return set_err(h, RHD_EINVAL, -1, "invalid state pointer, dt or nsteps");
  hipError_t e = rhd::launch_reset_err(h->err, h->stream);
  if (e != hipSuccess) return hip_fail(h, e, "reset");
  e = run_steps(h, state, dt, nsteps);
  if (e != hipSuccess) return hip_fail(h, e, "step launch");
  return finish(h);
}

rhd_status rhd_step_noalloc(const rhd_params* p, const double* rho, const double* kappa_P,
                            const double* kappa_F, double* state, double dt, int32_t nsteps,
                            void* hip_stream, int64_t* fail_cell) {
  if (fail_cell) *fail_cell = -1;
  if (!validate(p).empty()) return RHD_EINVAL;
  if (!rho || !kappa_P || !state || misaligned(rho) || misaligned(kappa_P) ||
      misaligned(kappa_F) || misaligned(state) || !std::isfinite(dt) || !(dt > 0.0) || nsteps < 0)
    return RHD_EINVAL;
  // y^{n+1/2} of the two-kernel path must fit the static scratch
  const size_t need = kNoallocYhalf + (size_t)nvar_of(p) * (size_t)ncells(p) * sizeof(double);
  if (need > kNoallocScratchBytes) return RHD_EWORKSPACE;
  const bool alias = (kappa_F == nullptr || kappa_F == kappa_P);
  const rhd::DevParams dp = make_dev(p, alias);
  void* base = nullptr;
  if (noalloc_scratch(&base) != hipSuccess) return RHD_EHIP;
  auto* err = reinterpret_cast<unsigned long long*>(base);
  auto* yhalf = reinterpret_cast<double*>(reinterpret_cast<char*>(base) + kNoallocYhalf);
  hipStream_t stream = reinterpret_cast<hipStream_t>(hip_stream);
  // the error word starts each call from its reset value (a kernel, not a memset)
  if (rhd::launch_reset_err(err, stream) != hipSuccess) return RHD_EHIP;
  if (run_steps(dp, p->precision == RHD_MIXED, state, yhalf, rho, kappa_P,
                alias ? kappa_P : kappa_F, dt, nsteps, err, stream) != hipSuccess)
    return RHD_EHIP;
  unsigned long long w[2] = {0, 0};
  if (hipMemcpyAsync(w, err, sizeof(w), hipMemcpyDeviceToHost, stream) != hipSuccess)
    return RHD_EHIP;
  if (hipStreamSynchronize(stream) != hipSuccess) return RHD_EHIP;
  if (w[1] == 0) return RHD_OK;
  if (fail_cell) *fail_cell = (w[0] == ULLONG_MAX) ? -1 : (int64_t)w[0];
  return (w[1] & rhd::ERR_NEWTON) ? RHD_ENEWTON : RHD_ENONPHYS;
}

rhd_status rhd_step_timed(rhd_handle* h, double* state, double dt, int32_t nsteps,
                          double* stage_ms) {
  if (!h) return RHD_EINVAL;
  if (!state || !stage_ms || misaligned(state) || !std::isfinite(dt) || !(dt > 0.0) || nsteps < 0)
    return set_err(h, RHD_EINVAL, -1, "invalid state pointer, dt, nsteps or stage_ms");
  const bool mixed = (h->p.precision == RHD_MIXED);
  std::vector<hipEvent_t> ev((size_t)2 * nsteps + 1, nullptr);
  auto cleanup = [&]() {
    for (auto& x : ev)
      if (x) (void)hipEventDestroy(x);
  };
  hipError_t e = hipSuccess;
  for (auto& x : ev) {
    e = hipEventCreate(&x);
    if (e != hipSuccess) {
      cleanup();
      return hip_fail(h, e, "hipEventCreate");
    }
  }
  e = rhd::launch_reset_err(h->err, h->stream);
  if (e == hipSuccess) e = hipEventRecord(ev[0], h->stream);
  for (int n = 0; n < nsteps && e == hipSuccess; ++n) {
    e = rhd::launch_stage(h->dp, rhd::MODE_STAGE1, mixed, state, state, h->yhalf, h->rho, h->kP,
                          h->kF, dt, h->err, h->stream);
    if (e == hipSuccess) e = hipEventRecord(ev[2 * n + 1], h->stream);
    if (e == hipSuccess)
      e = rhd::launch_stage(h->dp, rhd::MODE_STAGE2, mixed, h->yhalf, state, state, h->rho, h->kP,
                            h->kF, dt, h->err, h->stream);
    if (e == hipSuccess) e = hipEventRecord(ev[2 * n + 2], h->stream);
  }
  if (e != hipSuccess) {
    cleanup();
    return hip_fail(h, e, "timed step launch");
  }
  rhd_status st = finish(h);
  stage_ms[0] = stage_ms[1] = 0.0;
  for (int n = 0; n < nsteps; ++n) {
    float a = 0.f, b = 0.f;
    if (hipEventElapsedTime(&a, ev[2 * n], ev[2 * n + 1]) == hipSuccess) stage_ms[0] += a;
    if (hipEventElapsedTime(&b, ev[2 * n + 1], ev[2 * n + 2]) == hipSuccess) stage_ms[1] += b;
  }
  cleanup();
  return st;
}

rhd_status rhd_stage1(rhd_handle* h, const double* y, double* yh, double dt) {
  if (!h) return RHD_EINVAL;
  if (!y || !yh || y == yh || misaligned(y) || misaligned(yh) || !std::isfinite(dt) || !(dt > 0.0))
    return set_err(h, RHD_EINVAL, -1, "invalid arguments");
  hipError_t e = rhd::launch_reset_err(h->err, h->stream);
  if (e != hipSuccess) return hip_fail(h, e, "reset");
  e = rhd::launch_stage(h->dp, rhd::MODE_STAGE1, h->p.precision == RHD_MIXED, y, y, yh, h->rho,
                        h->kP, h->kF, dt, h->err, h->stream);
  if (e != hipSuccess) return hip_fail(h, e, "stage 1 launch");
  return finish(h);
}

rhd_status rhd_transport(rhd_handle* h, const double* y, double* s) {
  if (!h) return RHD_EINVAL;
  if (!y || !s || y == s || misaligned(y) || misaligned(s))
    return set_err(h, RHD_EINVAL, -1, "invalid arguments");
  hipError_t e = rhd::launch_reset_err(h->err, h->stream);
  if (e != hipSuccess) return hip_fail(h, e, "reset");
  e = rhd::launch_stage(h->dp, rhd::MODE_TRANSPORT, h->p.precision == RHD_MIXED, y, y, s, h->rho,
                        h->kP, h->kF, 0.0, h->err, h->stream);
  if (e != hipSuccess) return hip_fail(h, e, "transport launch");
  return finish(h);
}

rhd_status rhd_source(rhd_handle* h, double* y, double tau) {
  if (!h) return RHD_EINVAL;
  if (!y || misaligned(y) || !std::isfinite(tau) || !(tau > 0.0))
    return set_err(h, RHD_EINVAL, -1, "invalid arguments");
  hipError_t e = rhd::launch_reset_err(h->err, h->stream);
  if (e != hipSuccess) return hip_fail(h, e, "reset");
  e = rhd::launch_source(h->dp, y, h->rho, h->kP, h->kF, tau, h->err, h->stream);
  if (e != hipSuccess) return hip_fail(h, e, "source launch");
  return finish(h);
}

rhd_status rhd_conserved_totals(rhd_handle* h, const double* state, double* out) {
  if (!h) return RHD_EINVAL;
  if (!state || !out || misaligned(state)) return set_err(h, RHD_EINVAL, -1, "invalid arguments");
  const int no = 1 + h->p.ndim;
  hipError_t e = rhd::launch_totals(h->dp, state, h->partial, h->partial_blocks, h->stream);
  if (e != hipSuccess) return hip_fail(h, e, "totals launch");
  std::vector<double> part((size_t)h->partial_blocks * no);
  e = hipMemcpyAsync(part.data(), h->partial, part.size() * sizeof(double), hipMemcpyDeviceToHost,
                     h->stream);
  if (e != hipSuccess) return hip_fail(h, e, "hipMemcpyAsync(totals)");
  e = hipStreamSynchronize(h->stream);
  if (e != hipSuccess) return hip_fail(h, e, "hipStreamSynchronize");
  for (int m = 0; m < no; ++m) out[m] = 0.0;
  for (int b = 0; b < h->partial_blocks; ++b)
    for (int m = 0; m < no; ++m) out[m] += part[(size_t)b * no + m];
  return set_err(h, RHD_OK, -1, "");
}

// Hydro arguments: state and rho valid and aligned, rho the bound density.
static rhd_status hydro_args(rhd_handle* h, const double* state, const double* rho, double dt) {
  if (!state || !rho || misaligned(state) || misaligned(rho) || !std::isfinite(dt) || !(dt > 0.0))
    return set_err(h, RHD_EINVAL, -1, "invalid state, rho or dt");
  if (rho != h->rho)
    return set_err(h, RHD_EINVAL, -1, "rho must be the density bound at rhd_create");
  return RHD_OK;
}

rhd_status rhd_hydro_step(rhd_handle* h, double* state, double* rho, double dt, int32_t nsteps) {
  if (!h) return RHD_EINVAL;
  if (nsteps < 0) return set_err(h, RHD_EINVAL, -1, "nsteps must be >= 0");
  rhd_status st = hydro_args(h, state, rho, dt);
  if (st != RHD_OK) return st;
  hipError_t e = rhd::launch_reset_err(h->err, h->stream);
  if (e != hipSuccess) return hip_fail(h, e, "reset");
  for (int n = 0; n < nsteps; ++n) {
    e = rhd::launch_hydro_step(h->dp, state, rho, h->yhalf, dt, h->err, h->stream);
    if (e != hipSuccess) return hip_fail(h, e, "hydro launch");
  }
  return finish(h);
}

rhd_status rhd_rhd_step(rhd_handle* h, double* state, double* rho, double dt, int32_t nsub,
                        int32_t nsteps) {
  if (!h) return RHD_EINVAL;
  if (nsteps < 0 || nsub < 1) return set_err(h, RHD_EINVAL, -1, "need nsteps >= 0 and nsub >= 1");
  rhd_status st = hydro_args(h, state, rho, dt);
  if (st != RHD_OK) return st;
  const double dtr = dt / nsub;
  hipError_t e = rhd::launch_reset_err(h->err, h->stream);
  if (e != hipSuccess) return hip_fail(h, e, "reset");
  for (int n = 0; n < nsteps; ++n) {
    e = rhd::launch_hydro_step(h->dp, state, rho, h->yhalf, dt, h->err, h->stream);
    if (e != hipSuccess) return hip_fail(h, e, "hydro launch");
    e = run_steps(h, state, dtr, nsub);
    if (e != hipSuccess) return hip_fail(h, e, "radiation step launch");
  }
  return finish(h);
}

rhd_status rhd_hydro_signal_speed(rhd_handle* h, const double* state, const double* rho,
                                  double* out) {
  if (!h) return RHD_EINVAL;
  if (!out || !state || !rho || misaligned(state) || misaligned(rho))
    return set_err(h, RHD_EINVAL, -1, "invalid state, rho or out");
  hipError_t e = rhd::launch_hydro_speed(h->dp, state, rho, h->partial, h->partial_blocks, h->stream);
  if (e != hipSuccess) return hip_fail(h, e, "signal speed launch");
  std::vector<double> part((size_t)h->partial_blocks);
  e = hipMemcpyAsync(part.data(), h->partial, part.size() * sizeof(double), hipMemcpyDeviceToHost,
                     h->stream);
  if (e != hipSuccess) return hip_fail(h, e, "hipMemcpyAsync(signal speed)");
  e = hipStreamSynchronize(h->stream);
  if (e != hipSuccess) return hip_fail(h, e, "hipStreamSynchronize");
  double m = 0.0;
  for (double x : part) m = std::max(m, x);
  *out = m;
  return set_err(h, RHD_OK, -1, "");
}

rhd_status rhd_step_adjoint(rhd_handle* h, const double* state0, double dt, int32_t nsteps,
                            double* lambda, double* g_kappa_P, double* g_kappa_F) {
  if (!h) return RHD_EINVAL;
  if (h->adj_len <= 0)
    return set_err(h, RHD_EINVAL, -1, "handle created without adjoint workspace (adjoint_segment_len = 0)");
  if (nsteps < 1 || nsteps > h->adj_len)
    return set_err(h, RHD_EINVAL, -1, "nsteps must be in 1..adjoint_segment_len");
  if (!state0 || !lambda || !g_kappa_P || misaligned(state0) || misaligned(lambda) ||
      misaligned(g_kappa_P) || misaligned(g_kappa_F) || !std::isfinite(dt) || !(dt > 0.0))
    return set_err(h, RHD_EINVAL, -1, "invalid state0, lambda, g_kappa_P, g_kappa_F or dt");
  {
    // the reversal runs in lambda and reads state0 until it ends: no overlaps
    const size_t nst = (size_t)nvar_of(&h->p) * (size_t)h->dp.N, nf = (size_t)h->dp.N;
    auto overlap = [](const double* a, size_t na, const double* b, size_t nb) {
      const uintptr_t ua = reinterpret_cast<uintptr_t>(a), ub = reinterpret_cast<uintptr_t>(b);
      return b && ua < ub + nb * sizeof(double) && ub < ua + na * sizeof(double);
    };
    if (overlap(state0, nst, lambda, nst) || overlap(state0, nst, g_kappa_P, nf) ||
        overlap(state0, nst, g_kappa_F, nf) || overlap(lambda, nst, g_kappa_P, nf) ||
        overlap(lambda, nst, g_kappa_F, nf))
      return set_err(h, RHD_EINVAL, -1, "state0, lambda and the gradient arrays must not overlap");
  }
  if (!h->dp.kF_alias && !g_kappa_F)
    return set_err(h, RHD_EINVAL, -1, "a separate kappa_F needs g_kappa_F");
  if (h->p.scheme != RHD_SCHEME_PDARS)
    return set_err(h, RHD_EINVAL, -1, "the adjoint is available for the PD-ARS scheme only");
  if (h->p.hll_eps_cells > 0.0)
    return set_err(h, RHD_EINVAL, -1, "the adjoint does not cover the HLL eps correction");
  if (h->p.kappa_T_power != 0.0)
    return set_err(h, RHD_EINVAL, -1, "the adjoint does not cover temperature-dependent opacities");
  for (int d = 0; d < h->p.ndim; ++d)
    if (h->p.bc[d] != RHD_BC_PERIODIC)
      return set_err(h, RHD_EINVAL, -1, "the adjoint supports periodic axes only");
  hipError_t e = rhd::launch_reset_err(h->err, h->stream);
  if (e != hipSuccess) return hip_fail(h, e, "reset");
  const size_t M = (size_t)nvar_of(&h->p) * (size_t)h->dp.N;
  rhd::AdjointArgs A;
  A.P = h->dp;
  A.mixed = (h->p.precision == RHD_MIXED);
  A.state0 = state0;
  A.dt = dt;
  A.nsteps = nsteps;
  A.lambda = lambda;
  A.gkP = g_kappa_P;
  A.gkF = g_kappa_F;
  A.rho = h->rho;
  A.kP = h->kP;
  A.kF = h->kF;
  A.states = h->adj.states;
  A.lam_b = h->adj.lam;
  A.lam_c = h->adj.lam + M;
  A.err = h->err;
  A.stream = h->stream;
  e = rhd::launch_adjoint(A);
  if (e != hipSuccess) return hip_fail(h, e, "adjoint launch");
  return finish(h);
}

rhd_status rhd_set_energy_opacity(rhd_handle* h, const double* kappa_E) {
  if (!h) return RHD_EINVAL;
  if (misaligned(kappa_E)) return set_err(h, RHD_EINVAL, -1, "misaligned kappa_E");
  h->dp.kE = (kappa_E == h->kP) ? nullptr : kappa_E;
  return set_err(h, RHD_OK, -1, "");
}

rhd_status rhd_set_radiation_source(rhd_handle* h, const double* j) {
  if (!h) return RHD_EINVAL;
  if (misaligned(j)) return set_err(h, RHD_EINVAL, -1, "misaligned radiation source");
  h->dp.jS = j;
  return set_err(h, RHD_OK, -1, "");
}

rhd_status rhd_last_error(const rhd_handle* h, int64_t* cell, char* msg, size_t len) {
  if (!h) return RHD_EINVAL;
  if (cell) *cell = h->last_cell;
  if (msg && len > 0) {
    std::snprintf(msg, len, "%s", h->last_msg.c_str());
  }
  return h->last;
}

void rhd_destroy(rhd_handle* h) { delete h; }

}  // extern "C"
