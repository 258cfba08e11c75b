/*
 * rhd.h - C ABI of the MI355X radiation step.
 *
 * One step is the asymptotically-correct IMEX PD-ARS radiation update of
 * He, Wibking & Krumholz (2024), "An Asymptotically-Correct Implicit-Explicit
 * Time Integration Scheme for Finite Volume Radiation-Hydrodynamics":
 *   stage 1:  y(t) = y^n + dt s(y^n),                 y^{n+1/2} = Src(y(t), theta = 1)
 *   stage 2:  y(t) = (y^n + y^{n+1/2})/2 + dt/2 s(y^{n+1/2}),  y^{n+1} = Src(y(t), theta = 1/2)
 * (Sec. 3.2, eq. imex1-imex2, PD-ARS tableau with epsilon = 0; stage 2 uses the
 * stage-1 source increment in place of dt f(y^{n+1/2}), which is the same thing
 * once stage 1 holds). s is the explicit finite-volume transport of (E, F) in
 * reduced-speed-of-light form (eq. yrsla): PPM edge states, Levermore M1 or
 * Eddington closure, HLL flux with the uncorrected wave speed chat sqrt(D_dd)
 * (Sec. 3.3, Sec. 4.3). Src is the purely local implicit gas-radiation update of
 * Sec. 3.3 (eq. egupdate-fupdate): inner Newton on (E_gas, R) with residuals
 * eq. FGFR and R from eq. Rnew, energy recovery from conservation, flux update
 * eq. numF1 (v_order 1) or eq. numF2 (v_order 2), momentum update, and the outer
 * iteration over the lagged v and F.
 *
 * Around the radiation step: its hand-written adjoint (rhd_step_adjoint), and the
 * explicit hydrodynamics that the operator split of Sec. 3.1 runs before it
 * (rhd_hydro_step, and rhd_rhd_step for the split step with the radiation
 * subcycled).
 *
 * Conventions for every entry point
 *  - Array arguments are DEVICE pointers to caller-owned memory (for example
 *    torch tensors on the same GPU); the library never allocates device memory
 *    and never frees caller memory. The handle keeps the pointers it is given at
 *    create; the caller keeps them alive until rhd_destroy.
 *  - Grids are uniform Cartesian with spacing dx on every axis. Scalar fields are
 *    float64 arrays [nz][ny][nx] (x fastest). The state is float64
 *    [nvar][nz][ny][nx] with nvar = 2 + 2*ndim and variables in the order
 *    (E, F_1..F_ndim, E_gas, (rho v)_1..(rho v)_ndim): lab-frame radiation
 *    energy density and flux (physical units, not F/(c chat)), gas total energy
 *    density and momentum density.
 *  - Work is enqueued on the HIP stream given at create. Calls that return a
 *    status synchronise that stream once at the end (to read the device error
 *    word); no call synchronises the device.
 *  - Errors are returned as rhd_status; nothing is thrown across the ABI.
 *    A handle is bound to one stream and one device and is not thread-safe.
 */
#ifndef RHD_H
#define RHD_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct rhd_handle rhd_handle; /* opaque, host-side, library-owned */

typedef enum {
  RHD_OK = 0,
  RHD_EINVAL = -1,      /* invalid parameter or argument; nothing was launched */
  RHD_ENEWTON = -2,     /* inner Newton did not converge in newton_maxit iterations in some cell */
  RHD_ENONPHYS = -3,    /* E <= 0 or internal energy E_gas - |rho v|^2/(2 rho) <= 0 after the update */
  RHD_EHIP = -4,        /* a HIP runtime call failed (launch, copy, synchronisation) */
  RHD_EWORKSPACE = -5   /* workspace pointer NULL, misaligned or smaller than rhd_workspace_bytes */
} rhd_status;

/* RHD_BC_INFLOW: the ghost cells below the low face of the axis hold the fixed
 * radiation state (E = inflow_E, normal F = inflow_F, tangential F = 0), the high
 * face reflects (an entering radiation field, e.g. the Marshak wave of Sec. 5.2). */
enum { RHD_BC_PERIODIC = 0, RHD_BC_REFLECT = 1, RHD_BC_INFLOW = 2 };
enum { RHD_CLOSURE_M1 = 0, RHD_CLOSURE_EDDINGTON = 1 };
enum { RHD_FP64 = 0, RHD_MIXED = 1 };
enum { RHD_SCHEME_PDARS = 0, RHD_SCHEME_RK2SSP = 1 };

typedef struct {
  int32_t ndim;          /* 1, 2 or 3 */
  int32_t closure;       /* RHD_CLOSURE_M1 (Levermore) or RHD_CLOSURE_EDDINGTON (P = E/3 I) */
  int64_t n[3];          /* cells per axis (nx, ny, nz); axes beyond ndim must be 1 */
  double dx;             /* cell size, > 0 */
  double c;              /* speed of light, > 0 */
  double chat;           /* reduced speed of light, 0 < chat <= c (Sec. 3.2, RSLA) */
  double gamma;          /* adiabatic index, > 1; c_v = kB_over_mu / (gamma - 1) per unit mass */
  double a_r;            /* radiation constant: 4 pi B / c = a_r T^4, > 0 */
  double kB_over_mu;     /* k_B / (mu m_H), > 0 */
  int32_t bc[3];         /* RHD_BC_PERIODIC, RHD_BC_REFLECT or RHD_BC_INFLOW per axis (the last
                            two need n >= 3) */
  int32_t v_order;       /* 1: O(v/c) source terms, eq. numF1; 2: O(v^2/c^2): eq. numF2, or
                            with kappa_F != kappa_P the 3x3 flux system of eq. fupdate-G1 */
  int32_t precision;     /* RHD_FP64, or RHD_MIXED: transport stencil in float32, state,
                            flux-divergence accumulation and the source in float64 */
  int32_t newton_maxit;  /* inner Newton iteration cap (>= 1; 50 recommended) */
  int32_t outer_maxit;   /* outer iteration cap (>= 1; 10 recommended); reaching it is not an error */
  int32_t scheme;        /* RHD_SCHEME_PDARS (the paper's IMEX method) or RHD_SCHEME_RK2SSP:
                            the comparator of Sec. 4.2 (first stage transport only, the
                            source once at the end with the full dt; forward only) */
  double newton_rtol;    /* Newton stopping tolerance relative to E_gas + (c/chat) E (1e-13 in the paper) */
  double outer_rtol;     /* outer stopping tolerance on the v- and F-dependent part of R (1e-13) */
  double hll_eps_cells;  /* 0: plain HLL (the paper's method). > 0: the Skinner-type correction of
                            Sec. 4.2 on the energy flux, whose dissipation is multiplied by
                            eps = min(1, 1/tau) with tau = hll_eps_cells * dx * (chi_F of the two
                            cells at the face)/2, chi_F = rho kappa_F (forward only) */
  double kappa_T_power;  /* 0: opacities are the fields. q != 0: every opacity is its field times
                            T^q, evaluated by the local source at the Newton iterate (the chi of
                            eq. Rnew carry the t+1 superscript); e.g. q = -3 for chi = 300/T^3
                            (Sec. 5.2). Needs hll_eps_cells = 0; forward only */
  double inflow_E;       /* RHD_BC_INFLOW ghost state: radiation energy density */
  double inflow_F;       /* RHD_BC_INFLOW ghost state: flux along the axis */
} rhd_params;

/* Bytes of device workspace rhd_create needs for these parameters.
 * adjoint_segment_len = 0 sizes the forward step only; k > 0 also sizes
 * rhd_step_adjoint for segments of up to k steps (it stores y^n and y^{n+1/2}
 * of every step of a segment). Returns 0 for invalid parameters. */
size_t rhd_workspace_bytes(const rhd_params* p, int32_t adjoint_segment_len);

/* Validate the parameters and bind them, the scalar fields and the workspace
 * to a new handle.
 *   rho, kappa_P: device float64 [nz][ny][nx]; density and Planck-mean opacity
 *     per unit mass (chi_P = chi_E = rho kappa_P, Sec. 2.1 eq. G0-G1, grey).
 *   kappa_F: flux-mean opacity per unit mass, or NULL (or kappa_P) for kappa_F = kappa_P.
 *   workspace: device memory of ws_bytes >= rhd_workspace_bytes(p, 0), 256-byte
 *     aligned; owned by the caller, used exclusively by this handle. The
 *     adjoint segment length the handle accepts (rhd_step_adjoint's nsteps) is
 *     the largest k with rhd_workspace_bytes(p, k) <= ws_bytes (0: forward only),
 *     so a workspace of rhd_workspace_bytes(p, k) bytes allows segments of k steps.
 *   hip_stream: hipStream_t (NULL = default stream) on which all work is enqueued.
 * On success *out receives the handle; on failure *out is left untouched.
 * Errors: RHD_EINVAL for invalid parameters or a NULL or misaligned (not 8-byte)
 * field; RHD_EWORKSPACE for a NULL, not 256-byte aligned or too small workspace. */
rhd_status rhd_create(const rhd_params* p, const double* rho, const double* kappa_P,
                      const double* kappa_F, void* workspace, size_t ws_bytes, void* hip_stream,
                      rhd_handle** out);

/* Advance state (device float64 [nvar][nz][ny][nx], in/out) by nsteps PD-ARS
 * steps of size dt > 0 (Sec. 3.2-3.3). Two fused stage kernels per step; a 1-D
 * grid of at most 510 cells without the eps correction runs all nsteps steps in
 * one single-workgroup launch instead. No host synchronisation until the end of
 * the call. On RHD_ENEWTON / RHD_ENONPHYS the state holds what was computed
 * (every step still ran); rhd_last_error names the smallest failing cell index. */
rhd_status rhd_step(rhd_handle* h, double* state, double dt, int32_t nsteps);

/* Reverse-mode derivative of nsteps steps (1 <= nsteps <= the segment length
 * that the handle's workspace holds, see rhd_create) started from state0
 * (device, not modified).
 *   lambda: in: dJ/dy at the end of the segment; out: dJ/dy at its start. The
 *     reversal runs in this array (working storage during the call; on an error
 *     return its contents are unspecified). state0 is read until the call ends
 *     and must not overlap lambda or the gradient arrays.
 *   g_kappa_P, g_kappa_F: device [nz][ny][nx]; dJ/dkappa is ADDED (+=). With
 *     kappa_F aliasing kappa_P, g_kappa_F may be NULL and both contributions go
 *     into g_kappa_P.
 * The forward steps are recomputed from state0 inside the call; each local
 * implicit solve is differentiated with the implicit function theorem at its
 * converged state (in float64). With precision RHD_MIXED the transport adjoint
 * runs in float32 like the forward's stencil (states, lambda and the results in
 * float64). Returns RHD_EINVAL (nothing launched) for non-periodic axes,
 * the RK2-SSP scheme, hll_eps_cells > 0 or kappa_T_power != 0, which the adjoint
 * does not cover. */
rhd_status rhd_step_adjoint(rhd_handle* h, const double* state0, double dt, int32_t nsteps,
                            double* lambda, double* g_kappa_P, double* g_kappa_F);

/* Row-level entry points (same kernels as rhd_step), for testing one part.
 * rhd_transport: s (device [nvar][...]) = explicit transport of y; the E and F
 *   rows receive -div(flux) (eq. yrsla), the gas rows 0.
 * rhd_source: y (in/out) = Src(y, theta dt = tau) in every cell (Sec. 3.3).
 * rhd_stage1: yh = Src(y + dt s(y), dt) (eq. imex1). */
rhd_status rhd_transport(rhd_handle* h, const double* y, double* s);
rhd_status rhd_source(rhd_handle* h, double* y, double tau);
rhd_status rhd_stage1(rhd_handle* h, const double* y, double* yh, double dt);

/* rhd_step without a handle or workspace, for callers that cannot allocate
 * device memory (tight serving loops, harnesses that forbid hipMalloc). It
 * allocates nothing: y^{n+1/2} and the error word live in
 * a static device array of 64 MiB that the library holds on every GPU it runs
 * on until the process ends. Arguments as for rhd_create and rhd_step (device
 * pointers; kappa_F NULL for kappa_F = kappa_P; hip_stream NULL = default
 * stream); fail_cell (HOST, may be NULL) receives the smallest failing cell on
 * RHD_ENEWTON / RHD_ENONPHYS, else -1. The grid must satisfy
 * 256 + 8 * nvar * cells <= 64 MiB (about 1.05e6 cells in 3-D, 1.4e6 in 2-D,
 * 2.1e6 in 1-D); larger grids return RHD_EWORKSPACE before any launch. The
 * static array is shared by every call on that GPU and keeps the last call's
 * contents, so calls that overlap on one GPU (other streams or threads) race.
 * The optional kappa_E and S fields of a handle are not available here. Like
 * rhd_step it ends by reading the error word back and synchronizing the stream,
 * so it cannot be recorded into a HIP graph.
 * Returns the statuses of rhd_step (RHD_EINVAL for invalid parameters or
 * pointers, with nothing launched). */
rhd_status rhd_step_noalloc(const rhd_params* p, const double* rho, const double* kappa_P,
                            const double* kappa_F, double* state, double dt, int32_t nsteps,
                            void* hip_stream, int64_t* fail_cell);

/* rhd_step with per-stage kernel timing: hipEvents are recorded on the handle's
 * stream around every stage launch; on return stage_ms[0] and stage_ms[1] hold
 * the summed durations (ms) of the stage-1 and stage-2 kernels over the nsteps
 * steps (HOST array of 2 doubles). Always the two-kernel path (also on the 1-D
 * grids that rhd_step runs in one launch, where results agree to rounding);
 * elsewhere results are identical to rhd_step. */
rhd_status rhd_step_timed(rhd_handle* h, double* state, double dt, int32_t nsteps,
                          double* stage_ms);

/* Conserved totals of a state (diagnostics, not part of the timed step):
 * out[0] = sum(E_gas + (c/chat) E), out[1..ndim] = sum((rho v)_k + F_k/(c chat))
 * (energy and momentum that the source update conserves exactly, Sec. 3.3).
 * out is a HOST array of 1 + ndim doubles. */
rhd_status rhd_conserved_totals(rhd_handle* h, const double* state, double* out);

/* Optional fields of the local source (Sec. 3.3), bound to the handle until
 * replaced (the caller keeps them alive); both take effect from the next call.
 * rhd_set_energy_opacity: energy-mean opacity per unit mass kappa_E (device float64
 *   [nz][ny][nx], chi_E = rho kappa_E in eq. G0-G1 and in the Jacobian of the inner
 *   Newton); NULL (or kappa_P) restores kappa_E = kappa_P. rhd_step_adjoint holds a
 *   separate kappa_E fixed (no gradient with respect to it).
 * rhd_set_radiation_source: radiation injection rate j per unit volume (device
 *   float64 [nz][ny][nx]); every implicit stage adds S = j theta dt to the radiation
 *   energy (the optional S of eq. FGFR: F_R = E - E(t) - (R + S), E recovered as
 *   E(t) - (chat/c)(E_gas - E_gas(t)) + S); NULL removes it. The source terms' partial
 *   derivatives do not depend on S, so the adjoint covers it.
 * Both return RHD_EINVAL for a misaligned pointer. */
rhd_status rhd_set_energy_opacity(rhd_handle* h, const double* kappa_E);
rhd_status rhd_set_radiation_source(rhd_handle* h, const double* j);

/* Radiation hydrodynamics by operator splitting (Sec. 3.1): the explicit
 * hydrodynamics of the gas, then the radiation step subcycled over it.
 * rhd_hydro_step: nsteps RK2-SSP steps of size dt > 0 of the Euler equations for
 *   rho, rho v and E_gas (ideal gas, p = (gamma - 1)(E_gas - rho |v|^2 / 2)): PPM
 *   edge states of (rho, v, p) and HLLC fluxes; periodic axes wrap, the others
 *   mirror the gas with the normal velocity negated (RHD_BC_INFLOW axes included:
 *   their inflow state is radiation only). state (device float64 [nvar][nz][ny][nx])
 *   has its E_gas and momentum rows advanced, E and F untouched; rho (device
 *   float64 [nz][ny][nx]) is advanced in place and must be the density bound at
 *   rhd_create, so that the radiation step sees the new values (RHD_EINVAL
 *   otherwise). The opacities stay per unit mass (chi = rho kappa). CFL is the
 *   caller's: dt <= C dx / max(|v| + c_s), see rhd_hydro_signal_speed. Returns
 *   RHD_ENONPHYS with the smallest failing cell if rho or the internal energy
 *   ends non-positive. Uses the handle's workspace (the RK2 intermediate state).
 * rhd_rhd_step: nsteps split steps; each is one hydro step of dt followed by nsub
 *   >= 1 radiation steps (rhd_step) of dt / nsub. Arguments as above.
 * rhd_hydro_signal_speed: *out (HOST double) = max over cells and axes of
 *   |v_d| + c_s, c_s = sqrt(gamma p / rho), for choosing dt. */
rhd_status rhd_hydro_step(rhd_handle* h, double* state, double* rho, double dt, int32_t nsteps);
rhd_status rhd_rhd_step(rhd_handle* h, double* state, double* rho, double dt, int32_t nsub,
                        int32_t nsteps);
rhd_status rhd_hydro_signal_speed(rhd_handle* h, const double* state, const double* rho,
                                  double* out);

/* Error details of the last call on h: *cell = smallest failing cell index (or
 * -1), msg receives a NUL-terminated description (truncated to len). Returns the
 * status of the last call. */
rhd_status rhd_last_error(const rhd_handle* h, int64_t* cell, char* msg, size_t len);

/* Release the handle (host memory only; caller memory is untouched). NULL is a no-op. */
void rhd_destroy(rhd_handle* h);

#ifdef __cplusplus
}
#endif

#endif /* RHD_H */
