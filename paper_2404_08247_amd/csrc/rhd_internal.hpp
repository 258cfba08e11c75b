// Internal declarations shared by the host runtime (rhd_api.cpp) and the HIP
// kernels (rhd_forward.hip, rhd_adjoint.hip). Not part of the public ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <cstddef>
#include <cstdint>

namespace rhd {

// Kernel-side constants of one handle, passed by value to every launch.
struct DevParams {
  int ndim;
  int closure;        // 0 = M1, 1 = Eddington
  int v_order;        // 1 or 2
  int bc[3];          // 0 periodic, 1 reflect
  int n[3];           // nx, ny, nz
  int newton_maxit;
  int outer_maxit;
  long long N;        // cells
  double dx, inv_dx;
  double c, chat;
  double c_over_chat, chat_over_c, c_chat, inv_c_chat, inv_c2;
  double a_r;
  double gamma, gm1, inv_gm1;   // adiabatic index, gamma - 1, 1 / (gamma - 1)
  double cv_mass;     // kB_over_mu / (gamma - 1)
  double inv_cv_mass; // 1 / cv_mass
  double newton_rtol, outer_rtol;
  int kF_alias;       // 1: kappa_F == kappa_P
  int scheme;         // 0 PD-ARS, 1 RK2-SSP comparator
  double eps_dx;      // hll_eps_cells * dx (0: plain HLL)
  double kT_pow;      // opacity temperature exponent (0: constant opacities)
  int kT_isint, kT_int;   // kT_pow is the integer kT_int (|kT_int| <= 16)
  double inflow_E, inflow_F;   // ghost state of RHD_BC_INFLOW axes
  const double* kE;   // energy-mean opacity per unit mass (device), or null: kappa_P
  const double* jS;   // radiation injection rate per unit volume (device), or null: none
};

// Device error word layout (in the workspace): [0] smallest failing cell
// (initialised to INT64_MAX), [1] bit mask of failure kinds.
enum : unsigned { ERR_NEWTON = 1u, ERR_NONPHYS = 2u };

enum StageMode : int { MODE_STAGE1 = 0, MODE_STAGE2 = 1, MODE_TRANSPORT = 2 };
// boundary kinds of DevParams::bc (the values of the public header's RHD_BC_*)
enum BoundaryKind : int { BC_PERIODIC = 0, BC_REFLECT = 1, BC_INFLOW = 2 };

// Forward launchers (rhd_forward.hip). All return hipSuccess or the launch error.
hipError_t launch_stage(const DevParams& P, int mode, bool mixed, const double* ysten,
                        const double* yown, double* yout, const double* rho, const double* kP,
                        const double* kF, double dt, unsigned long long* err, hipStream_t s);
// launch_stage for a 2-D grid (rhd_stage2d.hip)
hipError_t launch_stage_2d(const DevParams& P, int mode, bool mixed, const double* ysten,
                           const double* yown, double* yout, const double* rho, const double* kP,
                           const double* kF, double dt, unsigned long long* err, hipStream_t s);
// 1-D grids of at most 510 cells without the eps correction: whole steps in one
// single-workgroup launch (rhd_forward.hip)
bool line_kernel_applies(const DevParams& P);
hipError_t launch_line_steps(const DevParams& P, bool mixed, double* y, const double* rho,
                             const double* kP, const double* kF, double dt, int nsteps,
                             unsigned long long* err, hipStream_t s);
hipError_t launch_source(const DevParams& P, double* y, const double* rho, const double* kP,
                         const double* kF, double tau, unsigned long long* err, hipStream_t s);
hipError_t launch_reset_err(unsigned long long* err, hipStream_t s);
// rhd_hydro.hip: one RK2-SSP hydro step of (rho, E_gas, rho v) in place; ws holds
// (2 + ndim) N doubles (the intermediate state)
hipError_t launch_hydro_step(const DevParams& P, double* y, double* rho, double* ws, double dt,
                             unsigned long long* err, hipStream_t s);
// per-block maxima of max_d |v_d| + c_s into partial[0..nblocks)
hipError_t launch_hydro_speed(const DevParams& P, const double* y, const double* rho,
                              double* partial, int nblocks, hipStream_t s);
hipError_t launch_totals(const DevParams& P, const double* y, double* partial, int nblocks,
                         hipStream_t s);

// Arguments of one adjoint segment (rhd_adjoint.hip).
struct AdjointArgs {
  DevParams P;
  bool mixed;
  const double* state0;   // segment start (caller)
  double dt;
  int nsteps;
  double* lambda;         // caller's adjoint vector (in: end, out: start)
  double* gkP;
  double* gkF;            // may be null
  const double* rho;
  const double* kP;
  const double* kF;
  double* states;         // 2 nsteps states: y^1..y^k, then y^{1/2}..y^{k-1/2}
  double* lam_b;          // two adjoint vectors of nvar N doubles
  double* lam_c;
  unsigned long long* err;
  hipStream_t stream;
};

hipError_t launch_adjoint(const AdjointArgs& A);

}  // namespace rhd
