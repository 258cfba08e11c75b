// Forward kernels of the radiation step for gfx950, apart from the 2-D stage
// instantiations (rhd_stage2d.hip):
//  - the fused stage kernel k_stage (rhd_stage.hpp) for 1-D and 3-D grids;
//  - k_line1d: whole steps of a short 1-D line in one single-workgroup launch;
//  - the source-only and transport-only entry points' kernels, the error-word
//    reset and the conserved-totals reduction;
//  - launch_stage, which picks the instantiation for the grid.
#include <climits>
#include <cmath>

#include "rhd_stage.hpp"

namespace rhd {

// ---------------------------------------------------------------------------
// Whole steps of a 1-D line that fits one workgroup, in one launch.
//
// A short 1-D grid (the reflecting 256-cell pulse, the 60-cell Marshak wave) has
// too little work per stage to fill the chip, and two launches per step cost
// more than the work itself. Here one workgroup of NT >= n + 2 threads owns the
// whole line for all nsteps steps: thread i holds cell i's y^n and y^{n+1/2} in
// registers, the stencil values with their 3 ghost cells per side, the edge
// states and the face fluxes go through LDS, and barriers separate the phases.
// The arithmetic per stage is that of k_stage (same PPM edges, HLL flux,
// divergence, y(t) and local source), so results agree with the two-kernel path
// to rounding. State is read once at the start and written once at the end.
// ---------------------------------------------------------------------------
constexpr int LINE_MAX_THREADS = 512;
constexpr int LINE_MAX_CELLS = LINE_MAX_THREADS - 2;   // cells -1..n need edge states

template <typename TT, int VAR>
__global__ void __launch_bounds__(LINE_MAX_THREADS)
k_line1d(DevParams P, double* __restrict__ y, const double* __restrict__ rho,
         const double* __restrict__ kP, const double* __restrict__ kF, double dt, int nsteps,
         unsigned long long* err) {
  constexpr int SV = (VAR == VAR_PLAIN) ? SRC_LEAN : (VAR == VAR_TDEP ? SRC_TDEP : SRC_GEN);
  constexpr int NR = 2;                                 // E, F
  __shared__ double s_a[NR][LINE_MAX_CELLS + 6];        // stencil values, 3 ghosts per side;
                                                        // later the face fluxes (faces 0..n)
  __shared__ double s_l[NR][LINE_MAX_CELLS + 2], s_r[NR][LINE_MAX_CELLS + 2];  // cells -1..n
  const int n = P.n[0];
  const int i = threadIdx.x;
  const bool own = i < n;
  const long long N = P.N;
  const double c = P.c, ch = P.chat, chc = P.chat_over_c, cch = P.c_chat;
  const int clo = P.closure;
  // ghost source cell and sign of ghost position g = i - 3 (threads 0..5: i < 3
  // below the line, else n + i - 6 above it)
  int gsrc = 0;
  bool gflip = false, gfix = false;
  if (i < 6) {
    const int g = (i < 3) ? i - 3 : n + i - 3;
    gsrc = ghost(g, n, P.bc[0], gflip);
    gfix = (g < 0) && P.bc[0] == BC_INFLOW;
  }
  double yn[4] = {0.0, 0.0, 0.0, 0.0}, yh[4] = {0.0, 0.0, 0.0, 0.0};
  double c_rho = 1.0, c_kp = 0.0, c_kf = 0.0, c_ke = 0.0, c_j = 0.0;
  if (own) {
#pragma unroll
    for (int r = 0; r < 4; ++r) yn[r] = y[r * N + i];
    c_rho = rho[i];
    c_kp = kP[i];
    c_kf = P.kF_alias ? c_kp : kF[i];
    if constexpr (SV >= SRC_GEN) {
      c_ke = P.kE ? P.kE[i] : c_kp;
      if (P.jS) c_j = P.jS[i];
    }
  }
  // s = -div(flux) of the stencil state st (own cell's E, F), through LDS
  auto transport = [&](const double* st, double* s) {
    __syncthreads();   // previous readers of s_a / s_l / s_r are done
    if (own) {
      s_a[0][i + 3] = st[0];
      s_a[1][i + 3] = st[1];
    }
    __syncthreads();
    if (i < 6) {
      const int t = (i < 3) ? i : n + i;   // tile slot of the ghost position
#pragma unroll
      for (int r = 0; r < NR; ++r) {
        const double v = s_a[r][gsrc + 3];
        s_a[r][t] = gfix ? inflow_value(P, r, 0) : ((gflip && r == 1) ? -v : v);
      }
    }
    __syncthreads();
    if (i < n + 2) {   // edge states of cell i - 1
#pragma unroll
      for (int r = 0; r < NR; ++r) {
        const double* a = &s_a[r][i];
        double l, rr;
        ppm_edges5<TT>(a[0], a[1], a[2], a[3], a[4], l, rr);
        s_l[r][i] = l;
        s_r[r][i] = rr;
      }
    }
    __syncthreads();
    if (i <= n) {      // face i, between cells i - 1 and i
      double Um[NR], Up[NR], fl[NR];
#pragma unroll
      for (int r = 0; r < NR; ++r) {
        Um[r] = s_r[r][i];
        Up[r] = s_l[r][i + 1];
      }
      hll_flux<1, 0, TT>(clo, c, ch, chc, cch, Um, Up, fl, 1.0);
#pragma unroll
      for (int r = 0; r < NR; ++r) s_a[r][i] = fl[r];
    }
    __syncthreads();
    if (own) {
#pragma unroll
      for (int r = 0; r < NR; ++r) s[r] = -(s_a[r][i + 1] - s_a[r][i]) * P.inv_dx;
    }
  };
  auto source = [&](double* v, double tau) {
    const unsigned st = source_cell<1, SV>(P, v[0], &v[1], v[2], &v[3], c_rho, c_kp, c_kf, c_ke,
                                           c_j * tau, tau, rcp(tau * ch));
    if (st) report(err, i, st);
  };
  const double tau2 = (P.scheme == 0) ? 0.5 * dt : dt;
  for (int step = 0; step < nsteps; ++step) {
    double s[NR] = {0.0, 0.0};
    // stage 1: y(t) = y^n + dt s(y^n); y^{n+1/2} = Src(y(t), dt) (RK2-SSP: no source)
    transport(yn, s);
    if (own) {
      yh[0] = yn[0] + dt * s[0];
      yh[1] = yn[1] + dt * s[1];
      yh[2] = yn[2];
      yh[3] = yn[3];
      if (P.scheme == 0) source(yh, dt);
    }
    // stage 2: y(t) = (y^n + y^{n+1/2})/2 + dt/2 s(y^{n+1/2}); y^{n+1} = Src(y(t), tau2)
    transport(yh, s);
    if (own) {
      const double hdt = 0.5 * dt;
      yn[0] = 0.5 * (yn[0] + yh[0]) + hdt * s[0];
      yn[1] = 0.5 * (yn[1] + yh[1]) + hdt * s[1];
      yn[2] = 0.5 * (yn[2] + yh[2]);
      yn[3] = 0.5 * (yn[3] + yh[3]);
      source(yn, tau2);
    }
  }
  if (own) {
#pragma unroll
    for (int r = 0; r < 4; ++r) y[r * N + i] = yn[r];
  }
}

// Source only (no transport), one cell per thread.
template <int ND, int SV>
__global__ void __launch_bounds__(NTHREADS)
k_source(DevParams P, double* y, const double* __restrict__ rho, const double* __restrict__ kP,
         const double* __restrict__ kF, double tau, unsigned long long* err) {
  const long long q = (long long)blockIdx.x * NTHREADS + threadIdx.x;
  if (q >= P.N) return;
  const long long N = P.N;
  double E = y[q], Eg = y[(1 + ND) * N + q], F[ND], Pm[ND];
#pragma unroll
  for (int k = 0; k < ND; ++k) {
    F[k] = y[(1 + k) * N + q];
    Pm[k] = y[(2 + ND + k) * N + q];
  }
  const double kp = kP[q];
  const unsigned st = source_cell<ND, SV>(P, E, F, Eg, Pm, rho[q], kp, P.kF_alias ? kp : kF[q],
                                         P.kE ? P.kE[q] : kp, P.jS ? P.jS[q] * tau : 0.0, tau,
                                         rcp(tau * P.chat));
  if (st) report(err, q, st);
  y[q] = E;
  y[(1 + ND) * N + q] = Eg;
#pragma unroll
  for (int k = 0; k < ND; ++k) {
    y[(1 + k) * N + q] = F[k];
    y[(2 + ND + k) * N + q] = Pm[k];
  }
}

__global__ void k_reset_err(unsigned long long* err) {
  if (threadIdx.x == 0) {
    err[0] = ULLONG_MAX;
    err[1] = 0ull;
  }
}

// Per-block partial sums of the conserved totals (diagnostics).
template <int ND>
__global__ void __launch_bounds__(NTHREADS)
k_totals(DevParams P, const double* __restrict__ y, double* __restrict__ partial) {
  constexpr int NO = 1 + ND;
  __shared__ double red[NO][NTHREADS];
  double acc[NO];
#pragma unroll
  for (int m = 0; m < NO; ++m) acc[m] = 0.0;
  const long long N = P.N;
  for (long long q = (long long)blockIdx.x * NTHREADS + threadIdx.x; q < N;
       q += (long long)gridDim.x * NTHREADS) {
    acc[0] += y[(1 + ND) * N + q] + P.c_over_chat * y[q];
#pragma unroll
    for (int k = 0; k < ND; ++k) acc[1 + k] += y[(2 + ND + k) * N + q] + y[(1 + k) * N + q] * P.inv_c_chat;
  }
#pragma unroll
  for (int m = 0; m < NO; ++m) red[m][threadIdx.x] = acc[m];
  __syncthreads();
  for (int s = NTHREADS / 2; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s) {
#pragma unroll
      for (int m = 0; m < NO; ++m) red[m][threadIdx.x] += red[m][threadIdx.x + s];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
#pragma unroll
    for (int m = 0; m < NO; ++m) partial[blockIdx.x * NO + m] = red[m][0];
  }
}

// ---------------------------------------------------------------------------
// Launchers
// ---------------------------------------------------------------------------
hipError_t launch_stage(const DevParams& P, int mode, bool mixed, const double* ysten,
                        const double* yown, double* yout, const double* rho, const double* kP,
                        const double* kF, double dt, unsigned long long* err, hipStream_t s) {
  switch (P.ndim) {
    case 1: return launch_stage_nd<1>(P, mode, mixed, ysten, yown, yout, rho, kP, kF, dt, err, s);
    case 2: return launch_stage_2d(P, mode, mixed, ysten, yown, yout, rho, kP, kF, dt, err, s);
    case 3: return launch_stage_nd<3>(P, mode, mixed, ysten, yown, yout, rho, kP, kF, dt, err, s);
    default: return hipErrorInvalidValue;
  }
}

bool line_kernel_applies(const DevParams& P) {
  return P.ndim == 1 && P.n[0] <= LINE_MAX_CELLS && !(P.eps_dx > 0.0);
}

template <typename TT>
static hipError_t launch_line_tt(const DevParams& P, double* y, const double* rho,
                                 const double* kP, const double* kF, double dt, int nsteps,
                                 unsigned long long* err, hipStream_t s) {
  const int nt = ((P.n[0] + 2 + 63) / 64) * 64;
  switch (source_variant(P)) {
    case SRC_LEAN:
      hipLaunchKernelGGL((k_line1d<TT, VAR_PLAIN>), dim3(1), dim3(nt), 0, s, P, y, rho, kP, kF, dt,
                         nsteps, err);
      break;
    case SRC_GEN:
      hipLaunchKernelGGL((k_line1d<TT, VAR_GEN>), dim3(1), dim3(nt), 0, s, P, y, rho, kP, kF, dt,
                         nsteps, err);
      break;
    default:
      hipLaunchKernelGGL((k_line1d<TT, VAR_TDEP>), dim3(1), dim3(nt), 0, s, P, y, rho, kP, kF, dt,
                         nsteps, err);
      break;
  }
  return hipGetLastError();
}

hipError_t launch_line_steps(const DevParams& P, bool mixed, double* y, const double* rho,
                             const double* kP, const double* kF, double dt, int nsteps,
                             unsigned long long* err, hipStream_t s) {
  if (!line_kernel_applies(P)) return hipErrorInvalidValue;
  if (nsteps <= 0) return hipSuccess;
  return mixed ? launch_line_tt<float>(P, y, rho, kP, kF, dt, nsteps, err, s)
               : launch_line_tt<double>(P, y, rho, kP, kF, dt, nsteps, err, s);
}

hipError_t launch_source(const DevParams& P, double* y, const double* rho, const double* kP,
                         const double* kF, double tau, unsigned long long* err, hipStream_t s) {
  const unsigned blocks = (unsigned)((P.N + NTHREADS - 1) / NTHREADS);
  const int sv = source_variant(P);
  switch (P.ndim * 3 + sv) {
    case 3: hipLaunchKernelGGL((k_source<1, SRC_LEAN>), dim3(blocks), dim3(NTHREADS), 0, s, P, y, rho, kP, kF, tau, err); break;
    case 4: hipLaunchKernelGGL((k_source<1, SRC_GEN>), dim3(blocks), dim3(NTHREADS), 0, s, P, y, rho, kP, kF, tau, err); break;
    case 5: hipLaunchKernelGGL((k_source<1, SRC_TDEP>), dim3(blocks), dim3(NTHREADS), 0, s, P, y, rho, kP, kF, tau, err); break;
    case 6: hipLaunchKernelGGL((k_source<2, SRC_LEAN>), dim3(blocks), dim3(NTHREADS), 0, s, P, y, rho, kP, kF, tau, err); break;
    case 7: hipLaunchKernelGGL((k_source<2, SRC_GEN>), dim3(blocks), dim3(NTHREADS), 0, s, P, y, rho, kP, kF, tau, err); break;
    case 8: hipLaunchKernelGGL((k_source<2, SRC_TDEP>), dim3(blocks), dim3(NTHREADS), 0, s, P, y, rho, kP, kF, tau, err); break;
    case 9: hipLaunchKernelGGL((k_source<3, SRC_LEAN>), dim3(blocks), dim3(NTHREADS), 0, s, P, y, rho, kP, kF, tau, err); break;
    case 10: hipLaunchKernelGGL((k_source<3, SRC_GEN>), dim3(blocks), dim3(NTHREADS), 0, s, P, y, rho, kP, kF, tau, err); break;
    case 11: hipLaunchKernelGGL((k_source<3, SRC_TDEP>), dim3(blocks), dim3(NTHREADS), 0, s, P, y, rho, kP, kF, tau, err); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_reset_err(unsigned long long* err, hipStream_t s) {
  hipLaunchKernelGGL(k_reset_err, dim3(1), dim3(64), 0, s, err);
  return hipGetLastError();
}

hipError_t launch_totals(const DevParams& P, const double* y, double* partial, int nblocks,
                         hipStream_t s) {
  switch (P.ndim) {
    case 1: hipLaunchKernelGGL(k_totals<1>, dim3(nblocks), dim3(NTHREADS), 0, s, P, y, partial); break;
    case 2: hipLaunchKernelGGL(k_totals<2>, dim3(nblocks), dim3(NTHREADS), 0, s, P, y, partial); break;
    case 3: hipLaunchKernelGGL(k_totals<3>, dim3(nblocks), dim3(NTHREADS), 0, s, P, y, partial); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

}  // namespace rhd
