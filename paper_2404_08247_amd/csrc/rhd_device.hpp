// Device math of the radiation step: PPM edge states, closure, HLL flux and the
// local implicit source update. Everything here is a __device__ function; the
// kernels that use it live in rhd_forward.hip and rhd_adjoint.hip.
//
// T is the arithmetic type of the transport stencil (double, or float in the
// mixed-precision path); the source update is always double.
#pragma once

#include "rhd_internal.hpp"

namespace rhd {

// ---------------------------------------------------------------------------
// Reciprocal: hardware estimate refined by two Newton-Raphson steps
// (r <- r + r (1 - x r)), full double precision for the positive, normal
// arguments it is used on.
// ---------------------------------------------------------------------------
__device__ __forceinline__ double rcp(double x) {
  double r = __builtin_amdgcn_rcp(x);
  double e = fma(-x, r, 1.0);
  r = fma(r, e, r);
  e = fma(-x, r, 1.0);
  return fma(r, e, r);
}
__device__ __forceinline__ float rcp(float x) { return __builtin_amdgcn_rcpf(x); }
// One refinement step only (relative error about 2^-48): for quantities whose
// rounding does not reach the result, such as the step length of an iteration
// whose convergence test uses exact residuals.
__device__ __forceinline__ double rcp1(double x) {
  const double r = __builtin_amdgcn_rcp(x);
  return fma(r, fma(-x, r, 1.0), r);
}

// Square root of an argument in [1, 4] (the closure's sqrt(4 - 3 f^2)), by
// Goldschmidt's iteration on the hardware reciprocal-square-root estimate
// (about 24 correct bits): s -> x y, h -> y/2, one step r = 1/2 - s h,
// s += s r, h += h r (48 bits), then the Newton correction s += h (x - s^2).
// No range reduction or special cases, which the argument range makes
// unnecessary; within 0.5 ulp of the correctly rounded root on [1, 4].
__device__ __forceinline__ double sqrt_1_4(double x) {
  const double y = __builtin_amdgcn_rsq(x);
  double s = x * y, h = 0.5 * y;
  const double r = fma(-s, h, 0.5);
  s = fma(s, r, s);
  h = fma(h, r, h);
  return fma(fma(-s, s, x), h, s);
}
__device__ __forceinline__ float sqrt_1_4(float x) { return __builtin_amdgcn_sqrtf(x); }
// Square root of a normal positive argument to about 2^-46 relative: one
// Goldschmidt step on the hardware estimate (s = x y, h = y/2, s += s (1/2 - s h)).
// For the closure and the HLL speed of the transport, whose rounding stays far
// below the flux differences.
__device__ __forceinline__ double sqrt_g1(double x) {
  const double y = __builtin_amdgcn_rsq(x);
  const double s = x * y;
  return fma(s, fma(-s, 0.5 * y, 0.5), s);
}
// The same iteration for 0 or a normal positive argument (the HLL signal
// speed sqrt(D_dd), D_dd in [0, 1]); zero maps to zero.
__device__ __forceinline__ double sqrt_nonneg(double x) {
  return x > 0.0 ? sqrt_g1(x) : 0.0;
}
// float: clamped at zero. In float32 the closure's D_dd across a saturated beam
// (f = 1, F_d = 0) is 1/3 - f^2 h, which the 1-ulp hardware reciprocal can leave
// a few ulp below zero.
__device__ __forceinline__ float sqrt_nonneg(float x) { return __builtin_amdgcn_sqrtf(fmaxf(x, 0.f)); }

// ---------------------------------------------------------------------------
// PPM (Colella & Woodward 1984), method-of-lines form: limited slopes,
// fourth-order interface values, monotonicity constraint on each cell's
// parabola (the paper reconstructs E and F with PPM, Sec. 3.3).
//
// Delta form: every quantity is an offset from the cell's own average, formed
// in double and then handled in T, so the float path keeps the relative
// precision of the (small) differences instead of that of the values.
// ---------------------------------------------------------------------------
// MC-limited slope from dl = a0 - a(-1), dr = a(+1) - a0: sgn(dc) min(|dc|,
// 2|dl|, 2|dr|) with dc = (dl + dr)/2 if dl and dr have the same sign, else 0,
// written as (sgn dl + sgn dr) min(|dl + dr|/4, |dl|, |dr|) (the same value:
// only power-of-two scalings differ), which needs no compare and select
template <typename T>
__device__ __forceinline__ T mc_slope(T dl, T dr) {
  const T m = fmin(T(0.25) * fabs(dl + dr), fmin(fabs(dl), fabs(dr)));
  return (copysign(T(1), dl) + copysign(T(1), dr)) * m;
}

// Monotonised edge offsets (l, r) of a cell from its raw interface offsets.
// The CW84 constraint in offset form: if l and r do not have opposite signs
// (the cell is a local extremum) both become 0; otherwise the parabola
// overshoots exactly when one offset exceeds twice the other in magnitude
// (del a6 > del^2 <=> |l| > 2|r|, del a6 < -del^2 <=> |r| > 2|l|), and that
// offset is set to minus twice the other. Both cases at once:
//   l' = (sgn l - sgn r) min(|l|/2, |r|),  r' = (sgn r - sgn l) min(|r|/2, |l|),
// branch-free and without selects.
template <typename T>
__device__ __forceinline__ void ppm_monotone(T& l, T& r) {
  const T t = copysign(T(1), l) - copysign(T(1), r);   // +-2 if opposite signs, else 0
  const T nl = t * fmin(T(0.5) * fabs(l), fabs(r));
  const T nr = -t * fmin(T(0.5) * fabs(r), fabs(l));
  l = nl;
  r = nr;
}

// Ghost rule along one axis: returns the source cell of (possibly outside)
// coordinate g and whether the normal vector component (radiation flux or gas
// velocity) flips sign (bc 0 periodic, any other kind mirrors). Positions
// further than 3 cells outside the grid are clamped; no real cell's stencil
// reads them.
__device__ __forceinline__ int ghost(int g, int n, int bc, bool& flip) {
  flip = false;
  if (g >= 0 && g < n) return g;
  if (bc == 0) {
    if (g < 0 && g + n >= 0) return g + n;   // one period away
    if (g >= n && g - n < n) return g - n;
    int m = g % n;
    return m < 0 ? m + n : m;
  }
  flip = true;
  int m = (g < 0) ? -1 - g : 2 * n - 1 - g;
  return m < 0 ? 0 : (m >= n ? n - 1 : m);
}

__device__ __forceinline__ void report(unsigned long long* err, long long cell, unsigned bits) {
  atomicMin(err, (unsigned long long)cell);
  atomicOr(reinterpret_cast<unsigned int*>(err + 1), bits);
}

// edge states of the middle cell of a[0..4] (double values in, double out)
template <typename T>
__device__ __forceinline__ void ppm_edges5(double a0, double a1, double a2, double a3, double a4,
                                           double& l, double& r) {
  const T d01 = T(a1 - a0), d12 = T(a2 - a1), d23 = T(a3 - a2), d34 = T(a4 - a3);
  const T s1 = mc_slope(d01, d12);
  const T s2 = mc_slope(d12, d23);
  const T s3 = mc_slope(d23, d34);
  // interface offsets from a2: left = -d12/2 - (s2 - s1)/6, right = d23/2 - (s3 - s2)/6
  T lo = T(-0.5) * d12 - (s2 - s1) * T(1.0 / 6.0);
  T ro = T(0.5) * d23 - (s3 - s2) * T(1.0 / 6.0);
  ppm_monotone(lo, ro);
  l = a2 + double(lo);
  r = a2 + double(ro);
}

// ---------------------------------------------------------------------------
// Closure, cancellation-free form. With f^2 = min(|F|^2/(cE)^2, 1) and
// s = sqrt(4 - 3 f^2), the Levermore Eddington factor is
//   chi = (3 + 4 f^2)/(5 + 2 s) = 1/3 + 2 f^2/(2 + s),
// and D = (1-chi)/2 I + (3chi-1)/2 n n = I/3 + dD with
//   dD_jk = -f^2 h delta_jk + 3 h F_j F_k r,   h = 1/(2+s), r = 1/max(|F|^2, (cE)^2).
// Only dD (small in thick regions) goes through T. Ddd is D_DIR,DIR, the
// component under the square root of the HLL speed.
//
// float32: the same tensor written with u = (cE)^2 - |F|^2 (formed in double,
// so exact enough), b = sqrt((cE)^2 + 3u) = cE s and q = 1/(cE (cE + b) (2cE + b)):
//   K = 1/(w (2 + s)) = q (cE + b),  dD_jk = K (3 F_j F_k - |F|^2 delta_jk),
//   D_DIR,DIR = (s - 1)/3 + 3 K F_DIR^2 = u q (2cE + b) + 3 K F_DIR^2,
// a sum of two non-negative terms; at |F| >= cE (u <= 0, the beam limit f = 1)
// K = 1/(3|F|^2) and the first term is 0. Across a saturated beam (F_DIR = 0,
// f = 1) D_DIR,DIR is then exactly 0, where 1/3 + dD_DIR,DIR would leave a
// rounding residue of a few float ulp, whose square root is a speed error of
// order 1e-4 chat. One reciprocal and one square root per evaluation.
// ---------------------------------------------------------------------------
template <int ND, int DIR, typename T>
__device__ __forceinline__ void closure_dD(int closure, double c, double E, const double* F,
                                           T* dD, T& Ddd) {
  if (closure == 1) {
#pragma unroll
    for (int k = 0; k < ND; ++k) dD[k] = T(0);
    Ddd = T(1.0 / 3.0);
    return;
  }
  const double cEd = c * E;
  if constexpr (sizeof(T) < sizeof(double)) {
    // dD depends on F/(cE) only. In float, |F|^2 and (cE)^2 leave the float range
    // for values of physical size (cE ~ 1e19 and above), so F and cE are first
    // scaled by the power of two that brings cE into [1/2, 1): exact, and the
    // same result as unscaled wherever that stays in range.
    const double sc = ldexp(1.0, -__builtin_amdgcn_frexp_exp(cEd));
    double F2d = 0.0;
    T Ft[ND];
#pragma unroll
    for (int k = 0; k < ND; ++k) {
      const double fk = F[k] * sc;
      Ft[k] = T(fk);
      F2d += fk * fk;
    }
    const double ce = cEd * sc;
    const T u = T(ce * ce - F2d);
    const T cE = T(ce), F2 = T(F2d);
    const bool thin = !(u > T(0));
    const T b = sqrt_1_4(cE * cE + T(3) * fmax(u, T(0)));
    const T cpb = cE + b, tpb = cE + cpb;
    const T q = rcp(thin ? T(3) * F2 : cE * cpb * tpb);
    const T K = thin ? q : q * cpb;
    const T iso = thin ? T(0) : u * q * tpb;
    const T g = T(3) * K * Ft[DIR];
#pragma unroll
    for (int k = 0; k < ND; ++k) dD[k] = g * Ft[k] - ((k == DIR) ? F2 * K : T(0));
    Ddd = iso + g * Ft[DIR];
  } else {
    T F2 = T(0);
#pragma unroll
    for (int k = 0; k < ND; ++k) F2 += T(F[k]) * T(F[k]);
    const T cE = T(cEd);
    const T r = rcp1(fmax(F2, cE * cE));
    const T f2 = F2 * r;
    const T h = rcp1(T(2) + sqrt_g1(T(4) - T(3) * f2));
    const T g = T(3) * h * r * T(F[DIR]);
#pragma unroll
    for (int k = 0; k < ND; ++k) dD[k] = g * T(F[k]) - ((k == DIR) ? f2 * h : T(0));
    Ddd = T(1.0 / 3.0) + dD[DIR];
  }
}

// HLL flux along DIR between edge states Um = (E, F..) and Up (RSLA form):
// Phi_E = (chat/c) F_DIR, Phi_Fk = c chat E D_DIR,k, signal speed
// chat sqrt(max D_DIR,DIR) (the uncorrected speed, Sec. 4.3). The O(1) parts are
// formed in double, the closure deviation dD in T.
// eps_e multiplies the dissipation of the energy component (1: plain HLL; the
// optional Skinner-type correction of Sec. 4.2 passes face_eps()).
template <int ND, int DIR, typename T>
__device__ __forceinline__ void hll_flux(int closure, double c, double chat, double chat_over_c,
                                         double c_chat, const double* Um, const double* Up,
                                         double* fl, double eps_e = 1.0) {
  T dm[ND], dp[ND], Dm, Dp;
  closure_dD<ND, DIR, T>(closure, c, Um[0], Um + 1, dm, Dm);
  closure_dD<ND, DIR, T>(closure, c, Up[0], Up + 1, dp, Dp);
  const double hS = 0.5 * chat * double(sqrt_nonneg(fmax(Dm, Dp)));
  fl[0] = 0.5 * chat_over_c * (Um[1 + DIR] + Up[1 + DIR]) - eps_e * hS * (Up[0] - Um[0]);
  const T em = T(Um[0]), ep = T(Up[0]);
  const double half_cc = 0.5 * c_chat;
#pragma unroll
  for (int k = 0; k < ND; ++k) {
    double iso = (k == DIR) ? (Um[0] + Up[0]) * (1.0 / 3.0) : 0.0;
    fl[1 + k] = half_cc * (iso + double(em * dm[k] + ep * dp[k])) - hS * (Up[1 + k] - Um[1 + k]);
  }
}

// Skinner-type eps of a face between cells with flux-mean absorption chi_a, chi_b:
// tau = hll_eps_cells dx (chi_a + chi_b)/2 (eps_dx = hll_eps_cells dx),
// eps = min(1, 1/tau).
__device__ __forceinline__ double face_eps(double eps_dx, double chi_a, double chi_b) {
  const double tau = eps_dx * 0.5 * (chi_a + chi_b);
  return tau > 1.0 ? rcp(tau) : 1.0;
}

// ---------------------------------------------------------------------------
// Local implicit source update of one cell (Sec. 3.3), float64, in registers.
// In: the state after the explicit part, y(t); out: y(t+1). tau = theta dt.
// Returns 0, or ERR_NEWTON / ERR_NONPHYS bits.
//
// Inner stage: Newton-Raphson on x = (E_gas, R) for
//   F_G = E_gas - E_gas(t) + (c/chat) R,   F_R = E(E_gas, R) - E(t) - R,
// where R = -chat G0 tau (eq. Rnew) is solved for E with v, F and the closure
// tensor D frozen: E = (A(T) + C - R/(tau chat)) / B. Jacobian as printed in
// the paper (beta^2 terms dropped, d(kappa_P/kappa_E)/dT = 0). Stop when
// |F_G| and (c/chat)|F_R| are below newton_rtol (E_gas(t) + (c/chat) E(t)).
// Then E from energy conservation, F from eq. numF1/numF2, rho v from momentum
// conservation; repeat with the new v and F until the v- and F-dependent part
// of R changes by <= outer_rtol (relatively, or relative to R).
// ---------------------------------------------------------------------------
// (iso, g) of the closure tensor D = iso I + g F F^T (M1: iso = 1/3 - f^2 h,
// g = 3 h / max(|F|^2, (cE)^2); Eddington: iso = 1/3, g = 0), evaluated as
//   u = (cE)^2 - |F|^2, b = sqrt((cE)^2 + 3u) = cE s, q = 1/(cE (cE + b) (2cE + b)),
//   g = 3 q (cE + b), iso = (s - 1)/3 = u q (2cE + b),
// and at |F| >= cE (f = 1): g = 1/|F|^2, iso = 0. One square root and one
// reciprocal (refined once: the closure enters the flux update, whose rounding
// does not reach the converged result at the tolerance of the iteration).
__device__ __forceinline__ void closure_ig(int closure, double c, double E, double F2, double& iso,
                                           double& g) {
  iso = 1.0 / 3.0;
  g = 0.0;
  if (closure != 1) {
    const double cE = c * E;
    const double u = fma(cE, cE, -F2);
    const bool thin = !(u > 0.0);
    const double b = sqrt_1_4(fma(3.0, fmax(u, 0.0), cE * cE));
    const double cpb = cE + b, tpb = cE + cpb;
    const double q = rcp1(thin ? 3.0 * F2 : cE * cpb * tpb);
    g = 3.0 * (thin ? q : q * cpb);
    iso = thin ? 0.0 : u * q * tpb;
  }
}

// inv_tch = 1/(tau chat) is passed in (uniform over a launch). kE: energy-mean
// opacity (kP when it is not a separate field); Ssrc: the radiation source S of
// eq. FGFR over this sub-step (0 when absent).
//
// Three instantiations: SRC_LEAN, the common case, takes chi_E = chi_P, S = 0,
// constant opacities and (at order 2) chi_F = chi_E, and ignores kE and Ssrc;
// SRC_GEN handles a separate kappa_E, the source S and chi_F != chi_E at order 2;
// SRC_TDEP adds temperature-dependent opacities. The host picks the leanest one
// that applies (each extra costs registers in the whole stage kernel).
//
// Temperature-dependent opacities (SRC_TDEP, kT_pow = q != 0): every absorption coefficient is chi_X = rho kappa_X T^q (q = kT_pow),
// taken at the temperature of the current Newton iterate (the chi of eq. Rnew
// are at t+1) and at the converged T for the flux update and the outer test.
// All of A, B and C of E(E_gas, R) are linear in the chi, so only the R/(tau chat)
// term and dF_R/dR see the factor: with g = T^-q and the pass coefficients taken
// at the field values (chi_X = rho kappa_X),
//   E = (A + C - g R/(tau chat)) / B,  dF_R/dR = -g/(tau chat chi_E) - 1,
// while dF_R/dE_gas keeps the ratio chi_P/chi_E, which T^q leaves unchanged (the
// simplified Jacobian carries no d chi/dT).
enum SourceVariant : int { SRC_LEAN = 0, SRC_GEN = 1, SRC_TDEP = 2 };

// x^n for an integer n that is uniform over the launch (binary powering)
__device__ __forceinline__ double ipow(double x, int n) {
  unsigned m = n < 0 ? 0u - (unsigned)n : (unsigned)n;
  double r = 1.0, b = x;
  while (m) {
    if (m & 1u) r *= b;
    b *= b;
    m >>= 1;
  }
  return n < 0 ? rcp(r) : r;
}

// T^(s q) for s = +1 or -1: repeated products when q is a small integer, else pow
__device__ __forceinline__ double opacity_tpow(const DevParams& P, double T, int s) {
  return P.kT_isint ? ipow(T, s * P.kT_int) : pow(T, s * P.kT_pow);
}

template <int ND, int SV>
__device__ unsigned source_cell(const DevParams& P, double& E, double* F, double& Eg, double* Pm,
                                double rho, double kP, double kF, double kE_in, double S_in,
                                double tau, double inv_tch) {
  constexpr bool GEN = (SV >= SRC_GEN);
  constexpr bool tdep = (SV == SRC_TDEP);
  const double kE = GEN ? kE_in : kP;
  const double Ssrc = GEN ? S_in : 0.0;
  double chiP = rho * kP;
  double chiE = rho * kE;
  double chiF = rho * kF;
  // field values (the pass coefficients below); chiP/E/F follow T when tdep
  const double chiP0 = chiP, chiE0 = chiE, chiF0 = chiF;
  if (chiP == 0.0 && chiE == 0.0 && chiF == 0.0) {   // no coupling: E += S only
    if constexpr (GEN) E += Ssrc;
    return 0u;
  }
  const double ch = P.chat;
  const double k_cc = P.c_over_chat;
  const double Cv = rho * P.cv_mass;
  const double inv_rho = rcp(rho);
  const double inv_Cv = inv_rho * P.inv_cv_mass;
  const double inv_chiE = rcp(chiE);
  const double ar = P.a_r;
  const bool o2 = (P.v_order == 2);

  // inputs y(t) (kept for every outer pass): E, E_gas, F, rho v
  const double E0 = E, Eg0 = Eg;
  // lagged v and F of the current pass (start: y(t)); F and momentum carry the
  // latest iterate, the input F(t) and (rho v)(t) are kept in F0 / P0
  double F0[ND], P0[ND], v[ND], Fb[ND];
#pragma unroll
  for (int k = 0; k < ND; ++k) {
    F0[k] = F[k];
    P0[k] = Pm[k];
    v[k] = P0[k] * inv_rho;
    Fb[k] = F0[k];
  }
  double Eb = E0;
  double Egas = Eg0;
  double R = 0.0;
  // (x + 0 is not folded away, since it maps -0 to +0: the lean path skips the
  // S terms explicitly)
  const double tol = P.newton_rtol * (Eg0 + k_cc * (GEN ? E0 + Ssrc : E0));
  // simplified Jacobian (fixed for the call): dF_R/dR and the T^3 factor of
  // dF_R/dE_gas = (1/C_v) d/dT (chi_P/chi_E a T^4)
  const double J22c = -inv_tch * inv_chiE;
  const double J22 = J22c - 1.0;
  const double J21c = 4.0 * ar * inv_Cv * ((!GEN || kP == kE) ? 1.0 : chiP * inv_chiE);
  const double ctau = ch * tau;
  // order 1: 1/B = 1/chi_E and the flux denominator do not change between passes
  const double inv_den_o1 = o2 ? 0.0 : rcp(1.0 + ctau * chiF);
  // The lean source at order 2 has one opacity field (chi_F = chi_E = chi_P, the
  // same products rho kappa_P): every (chi_F - chi_E) term is exactly zero, and
  // skipping it leaves the results unchanged bit for bit.
  const bool dchi_zero = (SV == SRC_LEAN) && o2;
  double Enew = E0;
  unsigned status = 0u;

  for (int ko = 0; ko < P.outer_maxit; ++ko) {
    double v2 = 0.0, vF = 0.0, F2 = 0.0;
#pragma unroll
    for (int k = 0; k < ND; ++k) {
      v2 += v[k] * v[k];
      vF += v[k] * Fb[k];
      F2 += Fb[k] * Fb[k];
    }
    const double KE = 0.5 * rho * v2;
    const double b2 = v2 * P.inv_c2;
    // D frozen for this pass. The lean source needs it only in the flux update
    // after the inner solve (v.D.v enters only (chi_F - chi_E) terms, which are
    // zero or absent there), so its evaluation overlaps the energy recovery; the
    // general one needs v.D.v in B before the solve.
    double iso = 1.0 / 3.0, g = 0.0, vDv = 0.0;
    if constexpr (GEN) {
      closure_ig(P.closure, P.c, Eb, F2, iso, g);
      vDv = iso * v2 + g * vF * vF;
    }
    // R/(tau chat) = A(T) - B E + C  =>  E(E_gas, R) = (A(T) + C - R/(tau chat)) / B.
    // Order 2: B = chi_E a1 - (chi_F - chi_E)(beta^2 + v.D.v/c^2) with
    // a1 = 1 + beta^2/2, and the flux update divides by a2 = 1 + chat tau chi_F a1.
    // With chi_F = chi_E, B = chi_E a1 and one reciprocal of a1 a2 gives both.
    double inv_B, inv_den, a2 = 1.0;
    if (o2) {
      const double a1 = 1.0 + 0.5 * b2;
      a2 = 1.0 + ctau * chiF0 * a1;
      if (!GEN || chiF0 == chiE0) {
        const double q = rcp(a1 * a2);
        inv_B = q * a2 * inv_chiE;
        inv_den = q * a1;
      } else {
        inv_B = rcp(chiE0 * a1 - (chiF0 - chiE0) * (b2 + vDv * P.inv_c2));
        inv_den = rcp(a2);
      }
    } else {
      inv_B = inv_chiE;
      inv_den = inv_den_o1;
    }
    const double Cc = (2.0 * chiE0 - chiF0) * vF * P.inv_c2;
    const double Aco = chiP0 * ar * (o2 ? 1.0 + 0.5 * b2 : 1.0);

    // ---- inner Newton on (E_gas, R) ----
    // E(E_gas, R) = A' T^4 + C' - R t' with the pass constants A' = Aco/B,
    // C' = C/B, t' = 1/(tau chat B) and T = E_gas/C_v - KE/C_v; the temperature
    // of the converged iterate is kept for the energy recovery below.
    const double AcoB = Aco * inv_B, CcB = Cc * inv_B, itB = inv_tch * inv_B;
    const double KEc = KE * inv_Cv;
    const double E0R = GEN ? E0 + Ssrc : E0;
    bool conv = false;
    double T = 0.0, T2 = 0.0;
    for (int it = 0;; ++it) {
      T = fma(Egas, inv_Cv, -KEc);
      T2 = T * T;
      const double gT = tdep ? opacity_tpow(P, T, -1) : 1.0;   // chi(field) / chi(T)
      const double Er = fma(AcoB, T2 * T2, fma(-R * gT, itB, CcB));
      const double FG = fma(k_cc, R, Egas - Eg0);
      const double FR = Er - (E0R + R);
      if (fabs(FG) < tol && k_cc * fabs(FR) < tol) {
        conv = true;
        break;
      }
      if (it >= P.newton_maxit) break;
      const double J21 = J21c * T2 * T;
      const double J22t = tdep ? J22c * gT - 1.0 : J22;
      const double inv_det = rcp1(J22t - k_cc * J21);
      Egas += (k_cc * FR - J22t * FG) * inv_det;
      R += (J21 * FG - FR) * inv_det;
    }
    if (!conv) {
      status |= ERR_NEWTON;
      break;
    }

    // ---- energy from conservation; flux and momentum ----
    // Order 1: eq. numF1. Order 2: eq. fupdate with eq. G1 at t+1 is
    //   a F + b v (v.F) = rhs,  a = 1 + chat tau chi_F (1 + beta^2/2),
    //   b = 2 chat tau (chi_F - chi_E)/c^2,
    //   rhs = F(t) + chat tau [chi_P a T^4 v + chi_F E D v + (chi_F - chi_E) E v],
    // solved by Sherman-Morrison: F = (rhs - b v (v.rhs)/(a + b v^2))/a (eq. numF2
    // when chi_F = chi_E).
    if constexpr (!GEN) closure_ig(P.closure, P.c, Eb, F2, iso, g);
    Enew = E0 - P.chat_over_c * (Egas - Eg0);
    if constexpr (GEN) Enew += Ssrc;
    const double Tn = T;
    if constexpr (tdep) {   // absorption at the converged T for the flux and the outer test
      const double fT = opacity_tpow(P, Tn, 1);
      chiP = chiP0 * fT;
      chiE = chiE0 * fT;
      chiF = chiF0 * fT;
      if (o2) {
        a2 = 1.0 + ctau * chiF * (1.0 + 0.5 * b2);
        inv_den = rcp(a2);
      } else {
        inv_den = rcp(1.0 + ctau * chiF);
      }
    }
    const double Tn2 = T2;
    const double Bn = ar * Tn2 * Tn2;
    const double xv = dchi_zero ? chiP * Bn : chiP * Bn + (chiF - chiE) * Enew;
    const double gvF = g * vF;
    double rhs[ND];
    double vr = 0.0;
#pragma unroll
    for (int k = 0; k < ND; ++k) {
      const double Dvk = iso * v[k] + gvF * Fb[k];       // (D v)_k with the frozen D
      rhs[k] = F0[k] + ctau * (xv * v[k] + chiF * Enew * Dvk);
      vr += v[k] * rhs[k];
    }
    double corr = 0.0;   // b (v.rhs)/(a + b v^2)
    if (GEN && o2 && chiF != chiE) {
      const double bb = 2.0 * ctau * (chiF - chiE) * P.inv_c2;
      corr = bb * vr * rcp(a2 + bb * v2);
    }
    double v2n = 0.0, wF_new = 0.0, Fv_new = 0.0;
#pragma unroll
    for (int k = 0; k < ND; ++k) {
      const double Fn = (GEN ? rhs[k] - corr * v[k] : rhs[k]) * inv_den;
      const double vn = (P0[k] - (Fn - F0[k]) * P.inv_c_chat) * inv_rho;
      v2n += vn * vn;
      wF_new += vn * Fn;
      if (!dchi_zero) Fv_new += Fb[k] * vn;               // for v_new . D . v_new
      F[k] = Fn;                                          // F_new (output candidate)
      Pm[k] = vn;                                         // v_new (momentum formed below)
    }

    // ---- outer test on the v- and F-dependent part of R (eq. Rnew) ----
    double W_old = (2.0 * chiE - chiF) * vF * P.inv_c2;
    double W_new = (2.0 * chiE - chiF) * wF_new * P.inv_c2;
    if (o2) {
      const double b2n = v2n * P.inv_c2;
      const double Tq = (Egas - 0.5 * rho * v2n) * inv_Cv;
      const double Tq2 = Tq * Tq;
      W_old += (chiP * Bn - chiE * Enew) * 0.5 * b2;
      W_new += (chiP * ar * Tq2 * Tq2 - chiE * Enew) * 0.5 * b2n;
      if (!dchi_zero) {
        const double wDw_new = iso * v2n + g * Fv_new * Fv_new;
        W_old += (chiF - chiE) * (b2 * Enew + Enew * vDv * P.inv_c2);
        W_new += (chiF - chiE) * (b2n * Enew + Enew * wDw_new * P.inv_c2);
      }
    }
    W_old *= ctau;
    W_new *= ctau;
#pragma unroll
    for (int k = 0; k < ND; ++k) {
      v[k] = Pm[k];
      Fb[k] = F[k];
    }
    Eb = Enew;
    R = Enew - E0 - Ssrc;
    const double dW = fabs(W_new - W_old);
    if (dW <= P.outer_rtol * fabs(W_old) || dW <= P.outer_rtol * fabs(R)) break;
  }

  // outputs: F holds F_new, momentum from conservation
  double p2 = 0.0;
#pragma unroll
  for (int k = 0; k < ND; ++k) {
    Pm[k] = P0[k] - (Fb[k] - F0[k]) * P.inv_c_chat;
    p2 += Pm[k] * Pm[k];
  }
  if (status == 0u) {
    const double eint = Egas - 0.5 * p2 * inv_rho;
    if (!(eint > 0.0) || !(Enew > 0.0)) status |= ERR_NONPHYS;
  }
  E = Enew;
  Eg = Egas;
#pragma unroll
  for (int k = 0; k < ND; ++k) F[k] = Fb[k];
  return status;
}

}  // namespace rhd
