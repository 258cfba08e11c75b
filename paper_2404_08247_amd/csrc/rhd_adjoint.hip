// Adjoint (reverse-mode derivative) of the PD-ARS radiation step, gfx950.
//
// For one step (stage s(y) = transport, Src = local implicit source):
//   stage 1: t1 = y^n + dt s(y^n),                 h = Src(t1; dt)
//   stage 2: t2 = (y^n + h)/2 + dt/2 s(h),          y^{n+1} = Src(t2; dt/2)
// the reverse sweep given lambda = dJ/dy^{n+1} is
//   mu2 = Src adjoint at y^{n+1};  lh = mu2/2 + (dt/2) s'(h)^T mu2;  ln = mu2/2
//   mu1 = Src adjoint at h on lh;   ln += mu1 + dt s'(y^n)^T mu1.
//
// Src adjoint (implicit function theorem at the converged state z of the local
// system r(z) = z - z_in - tau f(z; kappa) = 0, f the mixed-frame four-force
// terms of eq. G0-G1 in RSLA form, eq. egupdate-fupdate): with A = I - tau df/dz,
//   lambda_in = A^{-T} lambda_out,   dJ/dkappa += tau (df/dkappa)^T lambda_in.
// df/dz and df/dkappa are exact: the chain rule written out by hand through the
// intermediates of f (source_jac). The fixed point of the paper's inner/outer iteration
// is the solution of r(z) = 0 with the closure tensor evaluated at z, so this is
// the derivative of what the forward step computes (to the outer tolerance).
//
// Transport adjoint s'(y)^T lambda (gather form, no atomics), one fused kernel
// per axis d, staged in LDS:
//   1. per face i+1/2: phi = dJ/dPhi = (lambda_{i+1} - lambda_i)/dx, and the
//      adjoints of its two edge states mu-/mu+ = (dPhi/dU-/+)^T phi (the closure
//      row and its partials, differentiated by hand, per side);
//   2. per cell i: PPM partials of its edge states w.r.t. the 5 stencil values
//      (constants of the limiter branch recorded when the edges were formed)
//      times mu- of face i+1/2 and mu+ of face i-1/2, giving its contribution
//      to each of the cells i-2..i+2;
//   3. per cell j: sum of the contributions addressed to j.
// On a mixed-precision handle the limiter, closure and stencil adjoints run in
// float32, as the forward's stencil does; states, lambda and results stay double.
// Periodic axes only (the library rejects reflecting axes for the adjoint).
#include "rhd_device.hpp"

namespace rhd {

constexpr int ATHREADS = 256;

// PPM edge states of the middle cell of a0..a4 (the forward's method, Sec. 3.3),
// with the branch taken by each step in a byte: bits 0-1, 2-3, 4-5 the cases of
// the three MC slopes (0 across an extremum, 1 centred, 2 left-limited, 3
// right-limited), bits 6-7 the monotonicity case (0 flattened, 1 l = -2 r,
// 2 r = -2 l, 3 unchanged). The edges are linear in a0..a4 within a branch, so
// the code alone fixes their derivatives. Ties go to the earlier case in that
// order, the same choice as the oracle's dual numbers. Branch-free: the lanes of
// a wave take different cases. T is the limiter's arithmetic type: double, or
// float on differences formed in double (the forward's delta form), which takes
// the branches the mixed-precision forward step took.
template <typename T>
__device__ __forceinline__ unsigned slope_case(T dl, T dr, T& s) {
  // sgn(dc) min(|dc|, 2|dl|, 2|dr|), dc = (dl + dr)/2, compared at half scale
  const T al = fabs(dl), ar = fabs(dr);
  const T ac = T(0.25) * fabs(dl + dr);
  const T mlr = fmin(al, ar);
  const unsigned c = (ac <= mlr) ? 1u : (al <= ar ? 2u : 3u);
  const bool same = dl * dr > T(0);   // then sgn(dc) = sgn(dl)
  s = same ? copysign(T(2) * fmin(ac, mlr), dl) : T(0);
  return same ? c : 0u;
}

template <typename T>
__device__ __forceinline__ unsigned ppm_edges_code(double a0, double a1, double a2, double a3,
                                                   double a4, double& l, double& r) {
  const T d01 = T(a1 - a0), d12 = T(a2 - a1), d23 = T(a3 - a2), d34 = T(a4 - a3);
  T s1, s2, s3;
  const unsigned c1 = slope_case<T>(d01, d12, s1);
  const unsigned c2 = slope_case<T>(d12, d23, s2);
  const unsigned c3 = slope_case<T>(d23, d34, s3);
  const T sixth = T(1.0 / 6.0);
  const T lo0 = T(-0.5) * d12 - sixth * (s2 - s1);
  const T ro0 = T(0.5) * d23 - sixth * (s3 - s2);
  // CW84 monotonicity: flatten at an extremum, else cap the overshooting side
  const bool flat = ro0 * lo0 >= T(0);
  const T del = ro0 - lo0;
  const T da = del * (T(-3) * (lo0 + ro0)), dd = del * del;
  const bool capl = da > dd, capr = da < -dd;   // never both
  const unsigned cm = flat ? 0u : (capl ? 1u : (capr ? 2u : 3u));
  const T lo = flat ? T(0) : (capl ? T(-2) * ro0 : lo0);
  const T ro = flat ? T(0) : (capr ? T(-2) * lo0 : ro0);
  l = a2 + double(lo);
  r = a2 + double(ro);
  return c1 | (c2 << 2) | (c3 << 4) | (cm << 6);
}

// ga[o] = gl dl/da_o + gr dr/da_o in the branch recorded by ppm_edges_code
template <typename T>
__device__ __forceinline__ void ppm_vjp_code(unsigned code, T gl, T gr, T* ga) {
  auto kl = [](unsigned c) { return c == 1 ? T(0.5) : (c == 2 ? T(2) : T(0)); };
  auto kr = [](unsigned c) { return c == 1 ? T(0.5) : (c == 3 ? T(2) : T(0)); };
  const unsigned c1 = code & 3u, c2 = (code >> 2) & 3u, c3 = (code >> 4) & 3u, cm = code >> 6;
  const T glo = (cm == 3) ? gl : (cm == 2 ? gl - T(2) * gr : T(0));
  const T gro = (cm == 3) ? gr : (cm == 1 ? gr - T(2) * gl : T(0));
  const T sixth = T(1.0 / 6.0);
  const T gs1 = sixth * glo;
  const T gs2 = sixth * (gro - glo);
  const T gs3 = -sixth * gro;
  const T g01 = kl(c1) * gs1;
  const T g12 = T(-0.5) * glo + kr(c1) * gs1 + kl(c2) * gs2;
  const T g23 = T(0.5) * gro + kr(c2) * gs2 + kl(c3) * gs3;
  const T g34 = kr(c3) * gs3;
  ga[0] = -g01;
  ga[1] = g01 - g12;
  ga[2] = g12 - g23 + gl + gr;
  ga[3] = g23 - g34;
  ga[4] = g34;
}

// Row DIR of the closure tensor at U = (E, F_1..F_ND) with the partials the HLL
// adjoint needs. The closure depends on F/(cE) only; it is evaluated on the scaled
// variables e = sc cE and x = sc F in the arithmetic type T; for float, sc is the
// power of two that brings cE into [1/2, 1) (exact, and in the float range for any
// units), for double sc = 1:
//   Dk[k] = D_DIR,k,   A[j] = sum_k W_k dD_DIR,k/dz_j,   dD[j] = dD_DIR,DIR/dz_j,
// z = (e, x_1..x_ND); d/dE = c sc d/de and d/dF_k = sc d/dx_k. Returns sc.
// M1 (the forward's formulas): w = max(|x|^2, e^2), r = 1/w, f2 = |x|^2 r,
// s = sqrt(4 - 3 f2), h = 1/(2 + s), g = 3 h r x_DIR and
// D_DIR,k = g x_k + [k = DIR](1/3 - f2 h). Differentiated by hand (exact, the chain
// rule on these formulas):
//   df2 = r (d|x|^2 - f2 dw),   dh = h' df2 with h' = 3 h^2/(2 s),
//   dg = 3 x_DIR (h' r df2 - h r^2 dw) + 3 h r e_DIR,
//   dD_DIR,k = x_k dg + g e_k - [k = DIR](h + f2 h') df2.
// Eddington: D = I/3, no partials.
template <int ND, int DIR, typename T>
__device__ __forceinline__ double closure_row_vjp(const DevParams& P, const double* U, const T* W,
                                                  T* Dk, T* A, T* dD) {
  const double cEd = P.c * U[0];
  // (double holds the squares of any physical values: no scaling there)
  const double sc = (sizeof(T) < sizeof(double)) ? ldexp(1.0, -__builtin_amdgcn_frexp_exp(cEd))
                                                 : 1.0;
  if (P.closure == 1) {
#pragma unroll
    for (int k = 0; k < ND; ++k) Dk[k] = (k == DIR) ? T(1.0 / 3.0) : T(0);
#pragma unroll
    for (int j = 0; j <= ND; ++j) A[j] = dD[j] = T(0);
    return sc;
  }
  const T e = T(cEd * sc);
  T x[ND];
  T X2 = T(0), PF = T(0);
#pragma unroll
  for (int k = 0; k < ND; ++k) {
    x[k] = T(U[1 + k] * sc);
    X2 += x[k] * x[k];
    PF += W[k] * x[k];
  }
  const bool thin = !(X2 < e * e);   // the branch max() takes
  const T r = rcp(thin ? X2 : e * e);
  const T f2 = X2 * r;
  const T sq = sqrt_1_4(T(4) - T(3) * f2);
  const T h = rcp(T(2) + sq);
  const T xD = x[DIR];
  const T g = T(3) * h * r * xD;
  const T hp = T(1.5) * h * h * rcp(sq);
  const T qp = h + f2 * hp;
  const T a = T(3) * xD * hp * r, b = T(-3) * xD * h * r * r;
  const T wq = W[DIR] * qp;
#pragma unroll
  for (int j = 0; j <= ND; ++j) {
    const T dX2 = (j == 0) ? T(0) : T(2) * x[j - 1];
    const T dw = thin ? dX2 : ((j == 0) ? T(2) * e : T(0));
    const T df2 = r * (dX2 - f2 * dw);
    T dg = a * df2 + b * dw;
    if (j == 1 + DIR) dg += T(3) * h * r;
    A[j] = PF * dg - wq * df2 + ((j >= 1) ? g * W[j - 1] : T(0));
    dD[j] = xD * dg - qp * df2 + ((j == 1 + DIR) ? g : T(0));
  }
#pragma unroll
  for (int k = 0; k < ND; ++k) Dk[k] = g * x[k] + ((k == DIR) ? T(1.0 / 3.0) - f2 * h : T(0));
  return sc;
}

// The mixed-frame four-force terms per cell, z = (E, F_1..F_ND, E_gas, p_1..p_ND):
// g = (-c G0, -G_1..-G_ND) from eq. G0-G1 (order 2; order 1 keeps the O(v/c)
// terms), P = D(E, F) E. The source terms are f = U g with the constant map
//   f_E = (chat/c) g_0, f_Egas = -g_0, f_F_k = c chat g_k, f_p_k = -g_k
// (eq. egupdate-fupdate in RSLA form). With v = p/rho, T = (E_gas - rho v^2/2)/(rho c_v),
// B = a_r T^4, b2 = v^2/c^2, Dv = D v = iso v + gc F (v.F) and vDv = v.D v, where the
// closure is D = iso I + gc F F^T (M1: gc = 3 h r, iso = 1/3 - f2 h as in the
// forward; Eddington: gc = 0, iso = 1/3):
//   order 2, hb = 1 + b2/2, L = E - 2 (v.F)/c^2:
//     g_0 = c (chiP B - chiE E) hb + (2 chiE - chiF)(v.F)/c + c (chiF - chiE)(b2 E + E vDv/c^2)
//     g_k = (-chiF F_k hb + chiP B v_k + chiF E Dv_k + (chiF - chiE) L v_k)/c
//   order 1: hb = 1, L = E and no (chiF - chiE) term in g_0.
// g is linear in the opacities, g = chiP aP + chiF aF + chiE aE, which gives its
// opacity derivatives. source_jac returns those coefficients and G = dg/dz (m x M,
// m = 1 + ND, M = 2 + 2 ND), differentiated by hand (the chain rule through the
// intermediates above, whose partials are sparse: v and b2 depend on p only, T on
// E_gas and p, the closure scalars on E and F).
template <int ND>
__device__ __forceinline__ void source_jac(const DevParams& P, const double* z, double rho,
                                           double chiP, double chiF, double chiE,
                                           double (*G)[2 + 2 * ND], double* aP, double* aF,
                                           double* aE) {
  constexpr int m = 1 + ND;
  const double c = P.c, ic = 1.0 / P.c, ic2 = P.inv_c2;
  const double dchi = chiF - chiE;
  const double ir = rcp(rho);
  const double E = z[0], Eg = z[1 + ND];
  const double* F = z + 1;
  double v[ND];
  double v2 = 0.0, vF = 0.0, F2 = 0.0;
#pragma unroll
  for (int k = 0; k < ND; ++k) {
    v[k] = z[2 + ND + k] * ir;
    v2 += v[k] * v[k];
    vF += v[k] * F[k];
    F2 += F[k] * F[k];
  }
  const double b2 = v2 * ic2;
  const double iT = rcp(rho * P.cv_mass);
  const double T = (Eg - 0.5 * rho * v2) * iT;
  const double T2 = T * T;
  const double B = P.a_r * (T2 * T2);
  const double dBE = 4.0 * P.a_r * T2 * T * iT;   // dB/dE_gas; dB/dp_j = -dBE v_j
  // closure scalars and their partials over (E, F_1..F_ND) (as in closure_row_vjp)
  double gc = 0.0, iso = 1.0 / 3.0, dgc[m], diso[m];
#pragma unroll
  for (int j = 0; j < m; ++j) dgc[j] = diso[j] = 0.0;
  if (P.closure != 1) {
    const double cE = c * E;
    const bool thin = !(F2 < cE * cE);
    const double r = rcp(thin ? F2 : cE * cE);
    const double f2 = F2 * r;
    const double sq = sqrt_1_4(4.0 - 3.0 * f2);
    const double h = rcp(2.0 + sq);
    gc = 3.0 * h * r;
    iso = (1.0 / 3.0) - f2 * h;
    const double hp = 1.5 * h * h * rcp(sq);
    const double qp = h + f2 * hp;
#pragma unroll
    for (int j = 0; j < m; ++j) {
      const double dF2 = (j == 0) ? 0.0 : 2.0 * F[j - 1];
      const double dw = thin ? dF2 : ((j == 0) ? 2.0 * c * cE : 0.0);
      const double df2 = r * (dF2 - f2 * dw);
      dgc[j] = 3.0 * (hp * r * df2 - h * r * r * dw);
      diso[j] = -qp * df2;
    }
  }
  double Dv[ND];
#pragma unroll
  for (int k = 0; k < ND; ++k) Dv[k] = iso * v[k] + gc * F[k] * vF;
  const double vDv = iso * v2 + gc * vF * vF;
  const bool o2 = (P.v_order == 2);
  const double hb = o2 ? 1.0 + 0.5 * b2 : 1.0;
  const double L = o2 ? E - 2.0 * vF * ic2 : E;
  const double Q = o2 ? b2 * E + E * vDv * ic2 : 0.0;   // order-2 bracket of g_0
  const double a1 = (2.0 * chiE - chiF) * ic;

  // column E
  {
    const double dvDv = diso[0] * v2 + dgc[0] * vF * vF;
    G[0][0] = -c * chiE * hb + (o2 ? c * dchi * (b2 + vDv * ic2 + E * dvDv * ic2) : 0.0);
#pragma unroll
    for (int k = 0; k < ND; ++k) {
      const double dDv = diso[0] * v[k] + dgc[0] * F[k] * vF;
      G[1 + k][0] = ic * (chiF * Dv[k] + chiF * E * dDv + dchi * v[k]);
    }
  }
  // columns F_j
#pragma unroll
  for (int j = 0; j < ND; ++j) {
    const double dvDv = diso[1 + j] * v2 + dgc[1 + j] * vF * vF + 2.0 * gc * vF * v[j];
    G[0][1 + j] = a1 * v[j] + (o2 ? c * dchi * E * dvDv * ic2 : 0.0);
#pragma unroll
    for (int k = 0; k < ND; ++k) {
      const double dDv = diso[1 + j] * v[k] + dgc[1 + j] * F[k] * vF + (k == j ? gc * vF : 0.0) +
                         gc * F[k] * v[j];
      G[1 + k][1 + j] = ic * ((k == j ? -chiF * hb : 0.0) + chiF * E * dDv +
                              (o2 ? -2.0 * dchi * v[j] * ic2 * v[k] : 0.0));
    }
  }
  // column E_gas
  G[0][1 + ND] = c * chiP * dBE * hb;
#pragma unroll
  for (int k = 0; k < ND; ++k) G[1 + k][1 + ND] = ic * chiP * dBE * v[k];
  // columns p_j
#pragma unroll
  for (int j = 0; j < ND; ++j) {
    const double dBp = -dBE * v[j];
    const double dvDv = 2.0 * (iso * v[j] + gc * vF * F[j]) * ir;
    if (o2) {
      const double db2 = 2.0 * v[j] * ir * ic2;
      G[0][2 + ND + j] = c * chiP * dBp * hb + 0.5 * c * (chiP * B - chiE * E) * db2 +
                         a1 * F[j] * ir + c * dchi * (db2 * E + E * dvDv * ic2);
    } else {
      G[0][2 + ND + j] = c * chiP * dBp + a1 * F[j] * ir;
    }
#pragma unroll
    for (int k = 0; k < ND; ++k) {
      const double dDv = ((k == j ? iso : 0.0) + gc * F[k] * F[j]) * ir;
      double t = chiP * (dBp * v[k] + (k == j ? B * ir : 0.0)) + chiF * E * dDv +
                 (k == j ? dchi * L * ir : 0.0);
      if (o2) t += -chiF * F[k] * v[j] * ir * ic2 - 2.0 * dchi * F[j] * ir * ic2 * v[k];
      G[1 + k][2 + ND + j] = ic * t;
    }
  }
  // opacity coefficients
  aP[0] = c * B * hb;
  aF[0] = -vF * ic + c * Q;
  aE[0] = -c * E * hb + 2.0 * vF * ic - c * Q;
#pragma unroll
  for (int k = 0; k < ND; ++k) {
    aP[1 + k] = B * v[k] * ic;
    aF[1 + k] = (-F[k] * hb + E * Dv[k] + L * v[k]) * ic;
    aE[1 + k] = -L * v[k] * ic;
  }
}

// Source adjoint, one cell per thread, at the converged state zs:
//   lambda = ls lsrc + [tin; 0]   (tin: the first 1 + ND rows, or null),
//   mu = A^{-T} lambda into mout,  gkP/gkF += tau (dg/dkappa)^T U^T mu,
//   and optionally o2 = mu + b2 lsrc.
// mout may be lsrc or tin (each cell is read in full before it is written).
template <int ND>
__global__ void __launch_bounds__(ATHREADS)
k_src_adj(DevParams P, const double* __restrict__ zs, const double* lsrc, double ls,
          const double* tin, double* mout, const double* __restrict__ rho,
          const double* __restrict__ kP, const double* __restrict__ kF, double tau, double* gkP,
          double* gkF, double* __restrict__ o2, double b2) {
  constexpr int M = 2 + 2 * ND;
  constexpr int NRr = 1 + ND;
  const long long q = (long long)blockIdx.x * ATHREADS + threadIdx.x;
  if (q >= P.N) return;
  const long long N = P.N;
  // every load is issued here, ahead of the arithmetic, so that the addend of o2
  // and the accumulated gradients do not wait behind the solve at the end
  double z[M], lv[M], sv[M];
#pragma unroll
  for (int j = 0; j < M; ++j) {
    z[j] = zs[j * N + q];
    sv[j] = lsrc[j * N + q];
    lv[j] = ls * sv[j] + ((tin && j < NRr) ? tin[j * N + q] : 0.0);
  }
  const double gP0 = gkP[q];
  const double gF0 = gkF ? gkF[q] : 0.0;
  auto outputs = [&](const double* mu) {
#pragma unroll
    for (int i = 0; i < M; ++i) {
      mout[i * N + q] = mu[i];
      if (o2) o2[i * N + q] = mu[i] + b2 * sv[i];
    }
  };
  const double rq = rho[q], kp = kP[q], kf = P.kF_alias ? kp : kF[q];
  // energy-mean opacity: a separate field (held fixed: no gradient), or kappa_P
  // (then its tangent is kappa_P's: eP = 1)
  const double ke = P.kE ? P.kE[q] : kp;
  const double eP = P.kE ? 0.0 : 1.0;
  if (rq * kp == 0.0 && rq * kf == 0.0 && rq * ke == 0.0) {   // Src is E += S there: mu = lam
    outputs(lv);
    return;
  }

  // The rows of df/dz are dependent: df/dz = U G with G = dg/dz (m x M, m = 1 + ND)
  // and U the constant M x m map above. Hence A^T = I - tau G^T U^T and, by the
  // push-through identity, mu = A^{-T} lam = lam + tau G^T x with
  //   K x = U^T lam,   K = I_m - tau (G U)^T,
  // an m x m system instead of the M x M one.
  constexpr int m = 1 + ND;
  const double chc = P.chat_over_c, cch = P.c_chat;
  // G = dg/dz and the opacity coefficients of g, in registers
  double Gm[m][M], aP[m], aF[m], aE[m];
  source_jac<ND>(P, z, rq, rq * kp, rq * kf, rq * ke, Gm, aP, aF, aE);
  auto G = [&](int i, int j) -> double { return Gm[i][j]; };
  // K[k][i] = delta_ki - tau (G U)[i][k]; (G U)[i][0] = (chat/c) G[i][E] - G[i][Egas],
  // (G U)[i][1+k] = c chat G[i][F_k] - G[i][p_k]; rhs w = U^T lam
  double K[m][m], w[m];
#pragma unroll
  for (int i = 0; i < m; ++i) {
    K[0][i] = ((i == 0) ? 1.0 : 0.0) - tau * (chc * G(i, 0) - G(i, 1 + ND));
#pragma unroll
    for (int k = 0; k < ND; ++k)
      K[1 + k][i] = ((i == 1 + k) ? 1.0 : 0.0) - tau * (cch * G(i, 1 + k) - G(i, 2 + ND + k));
  }
  w[0] = chc * lv[0] - lv[1 + ND];
#pragma unroll
  for (int k = 0; k < ND; ++k) w[1 + k] = cch * lv[1 + k] - lv[2 + ND + k];
  // equilibrate (rows, then columns: the unknowns carry different units), then
  // Gaussian elimination with partial pivoting, fully unrolled
  double cs[m];
#pragma unroll
  for (int r = 0; r < m; ++r) {
    double mx = 0.0;
#pragma unroll
    for (int j = 0; j < m; ++j) mx = fmax(mx, fabs(K[r][j]));
    const double inv = mx > 0.0 ? 1.0 / mx : 1.0;
#pragma unroll
    for (int j = 0; j < m; ++j) K[r][j] *= inv;
    w[r] *= inv;
  }
#pragma unroll
  for (int j = 0; j < m; ++j) {
    double mx = 0.0;
#pragma unroll
    for (int r = 0; r < m; ++r) mx = fmax(mx, fabs(K[r][j]));
    cs[j] = mx > 0.0 ? 1.0 / mx : 1.0;
#pragma unroll
    for (int r = 0; r < m; ++r) K[r][j] *= cs[j];
  }
#pragma unroll
  for (int k = 0; k < m; ++k) {
    int p = k;
    double best = fabs(K[k][k]);
#pragma unroll
    for (int i = k + 1; i < m; ++i) {
      const double a = fabs(K[i][k]);
      if (a > best) {
        best = a;
        p = i;
      }
    }
#pragma unroll
    for (int i = k + 1; i < m; ++i) {
      if (i == p) {
#pragma unroll
        for (int j = 0; j < m; ++j) {
          const double t = K[k][j];
          K[k][j] = K[i][j];
          K[i][j] = t;
        }
        const double t = w[k];
        w[k] = w[i];
        w[i] = t;
      }
    }
    const double inv = 1.0 / K[k][k];
#pragma unroll
    for (int i = k + 1; i < m; ++i) {
      const double f = K[i][k] * inv;
#pragma unroll
      for (int j = k + 1; j < m; ++j) K[i][j] -= f * K[k][j];
      w[i] -= f * w[k];
    }
  }
  double x[m];
#pragma unroll
  for (int i = m - 1; i >= 0; --i) {
    double acc = w[i];
#pragma unroll
    for (int j = i + 1; j < m; ++j) acc -= K[i][j] * x[j];
    x[i] = acc / K[i][i];
  }
#pragma unroll
  for (int i = 0; i < m; ++i) x[i] *= cs[i];   // undo the column scaling
  double mu[M];
#pragma unroll
  for (int j = 0; j < M; ++j) {
    double acc = 0.0;
#pragma unroll
    for (int i = 0; i < m; ++i) acc += G(i, j) * x[i];
    mu[j] = lv[j] + tau * acc;
  }

  // dJ/dkappa: tau (df/dkappa)^T mu = tau (dg/dkappa)^T (U^T mu)
  double um[m];
  um[0] = chc * mu[0] - mu[1 + ND];
#pragma unroll
  for (int k = 0; k < ND; ++k) um[1 + k] = cch * mu[1 + k] - mu[2 + ND + k];
  // the opacity derivatives of g = chiP aP + chiF aF + chiE aE, chi = rho kappa:
  // gk[0] along kappa_P (with kappa_F when it aliases kappa_P and has no gradient of
  // its own, and kappa_E = kappa_P unless a separate kappa_E is held fixed),
  // gk[1] along kappa_F
  const double kF0 = (P.kF_alias && !gkF) ? 1.0 : 0.0;
  double gk[2] = {0.0, 0.0};
#pragma unroll
  for (int i = 0; i < m; ++i) {
    gk[0] += rq * (aP[i] + kF0 * aF[i] + eP * aE[i]) * um[i];
    gk[1] += rq * aF[i] * um[i];
  }
  if (gkF) {
    gkP[q] = gP0 + tau * gk[0];
    gkF[q] = gF0 + tau * gk[1];
  } else {
    const double g = gP0 + tau * gk[0];
    gkP[q] = P.kF_alias ? g : g + tau * gk[1];
  }
  outputs(mu);
}

// phi^T dPhi/dU-+ of the HLL flux along DIR between edge states Um | Up:
//   Phi_0 = (chat/c)(F-_D + F+_D)/2 - hS (E+ - E-),
//   Phi_1+k = c chat (E- D-_Dk + E+ D+_Dk)/2 - hS (F+_k - F-_k),
//   hS = chat sqrt(max(D-_DD, D+_DD))/2,
// with the closure rows and their partials w.r.t. (E, F) of each side from
// closure_row_vjp in the arithmetic type T; states, phi and the results in double.
// gm = (dPhi/dU-)^T phi, gp = (dPhi/dU+)^T phi.
template <int ND, int DIR, typename T>
__device__ __forceinline__ void hll_vjp(const DevParams& P, const double* Um, const double* Up,
                                        const double* phi, double* gm, double* gp) {
  constexpr int NR = 1 + ND;
  T W[ND];   // weights of the flux components
#pragma unroll
  for (int k = 0; k < ND; ++k) W[k] = T(phi[1 + k]);
  T Dm[ND], Dp[ND], Am[NR], Ap[NR], dDm[NR], dDp[NR];
  const double scm = closure_row_vjp<ND, DIR, T>(P, Um, W, Dm, Am, dDm);
  const double scp = closure_row_vjp<ND, DIR, T>(P, Up, W, Dp, Ap, dDp);
  const bool mside = !(Dm[DIR] < Dp[DIR]);   // the side max() takes
  const T sqT = sqrt_nonneg(mside ? Dm[DIR] : Dp[DIR]);
  const double hS = 0.5 * P.chat * double(sqT);
  const double dhS = sqT > T(0) ? 0.25 * P.chat * double(rcp(sqT)) : 0.0;   // d hS / d D_DD
  double Sig = 0.0;   // sum_r phi_r (U+_r - U-_r)
#pragma unroll
  for (int r = 0; r < NR; ++r) Sig += phi[r] * (Up[r] - Um[r]);
  T WDm = T(0), WDp = T(0);
#pragma unroll
  for (int k = 0; k < ND; ++k) {
    WDm += W[k] * Dm[k];
    WDp += W[k] * Dp[k];
  }
  // E d/dE = e d/de and E d/dF_k = (sc E) d/dx_k on each side
  const T em = T(P.c * Um[0] * scm), ep = T(P.c * Up[0] * scp);
  const T Em = T(Um[0] * scm), Ep = T(Up[0] * scp);
  const double hcc = 0.5 * P.c_chat;
  const double sd = Sig * dhS;
#pragma unroll
  for (int r = 0; r < NR; ++r) {
    // sum_k phi_1+k d(E D_Dk)/dU_r on each side
    const T tm = (r == 0) ? em * Am[0] + WDm : Em * Am[r];
    const T tp = (r == 0) ? ep * Ap[0] + WDp : Ep * Ap[r];
    gm[r] = hcc * double(tm) + hS * phi[r];
    gp[r] = hcc * double(tp) - hS * phi[r];
    if (r == 1 + DIR) {
      gm[r] += 0.5 * P.chat_over_c * phi[0];
      gp[r] += 0.5 * P.chat_over_c * phi[0];
    }
    if (mside) {
      gm[r] -= sd * double(dDm[r]) * ((r == 0) ? P.c * scm : scm);
    } else {
      gp[r] -= sd * double(dDp[r]) * ((r == 0) ? P.c * scp : scp);
    }
  }
}

// Transport adjoint along DIR, out += scale s_DIR'(y)^T lam restricted to (E, F),
// one launch per axis. A workgroup owns TL cells along DIR on each of TP lines
// (lines are neighbours along x, or along y when DIR = 0) and stages in LDS:
//   y of cells [-5, TL+4] of each line (periodic wrap; lam is read directly),
//   face adjoints mu-/mu+ of the faces f+1/2, f in [-3, TL+1],
//   then per variable the PPM contributions C of cells [-2, TL+1] to their five
//   stencil cells, and gathers them into its own cells (no atomics).
//   face f+1/2: phi = scale (lam_{f+1} - lam_f)/dx, mu-+ = (dPhi/dU-+)^T phi;
//   cell c: C_o = d aR_c/d y_{c+o} mu-_{c+1/2} + d aL_c/d y_{c+o} mu+_{c-1/2};
//   cell j: out_j += sum_o C_o(j - o).
// Tile shapes: along x the lines are y neighbours and a long tile halves the share
// of recomputed halo faces; along y and z the lines are x neighbours, and 8 of
// them keep the staging loads in 64-byte runs.
template <int ND, int DIR> struct TvjpShape { static constexpr int TL = 32, TP = 8; };
template <> struct TvjpShape<1, 0> { static constexpr int TL = 256, TP = 1; };
template <> struct TvjpShape<2, 0> { static constexpr int TL = 64, TP = 4; };
template <> struct TvjpShape<3, 0> { static constexpr int TL = 64, TP = 4; };
constexpr int TV_NT = 320;

// TT: arithmetic type of the limiter, closure and the face and stencil adjoints
// (double; float for a mixed-precision handle, as in its forward step). States,
// lambda, phi and the outputs stay double.
template <int ND, int DIR, typename TT>
__global__ void __launch_bounds__(TV_NT)
k_tvjp(DevParams P, const double* __restrict__ y, const double* __restrict__ lam, double scale,
       double* __restrict__ out, int accumulate) {
  constexpr int NR = 1 + ND;
  constexpr int TL = TvjpShape<ND, DIR>::TL, TP = TvjpShape<ND, DIR>::TP;
  constexpr int NYv = TL + 10, NF = TL + 5, NC = TL + 4, NE = TL + 6;
  static_assert(NE * TP <= TV_NT && NC * TP <= TV_NT, "one item round per phase");
  // Work items of a phase: along x the cells of a line are consecutive in memory
  // and run fastest; along y and z the lines do, so the global loads and stores
  // of a wave cover runs of TP consecutive x cells. The LDS arrays follow the
  // same order (index [..][p][t] along x, [..][t][p] along y and z), so a wave's
  // LDS accesses are consecutive words.
  constexpr bool LF = (DIR != 0);
  // Two LDS regions, each holding what one phase reads and the next one writes:
  //   A: staged y (edge phase), then the face adjoints (contribution phase);
  //   B: edge states of the cells next to the faces, local y index e + 2 (face
  //      phase), then the PPM contributions (gather);
  // plus the branch codes. A barrier separates every reuse.
  // (sizes in doubles; the face adjoints and contributions are TT)
  constexpr int NYB = NR * TP * NYv, NFB = (int)((2 * NR * TP * NF * sizeof(TT) + 7) / 8);
  constexpr int NEB = 2 * NR * TP * NE, NCB = (int)((5 * TP * NC * sizeof(TT) + 7) / 8);
  __shared__ double s_a[NYB > NFB ? NYB : NFB];
  __shared__ double s_b[NEB > NCB ? NEB : NCB];
  __shared__ unsigned char s_code[NR * TP * NE];
  // index of (array k, line p, position t) in an array set of length L per line
  auto at = [](int k, int p, int t, int L) {
    return LF ? (k * L + t) * TP + p : (k * TP + p) * L + t;
  };
  constexpr int TS = LF ? TP : 1;   // LDS stride between neighbours along the line
  double* s_y = s_a;                           // [NR] x NYv, cells t0-5+t
  TT* s_fm = reinterpret_cast<TT*>(s_a);       // [2 NR] x NF: mu- (k < NR), mu+ (k >= NR)
  double* s_eL = s_b;                          // [NR] x NE
  double* s_eR = s_b + NR * TP * NE;
  TT* s_c = reinterpret_cast<TT*>(s_b);        // [5] x NC

  const int tid = threadIdx.x;
  const long long N = P.N;
  const int nx = P.n[0], ny = P.n[1];
  // axis length, perpendicular line axis, and the strides of the three roles
  const int na = P.n[DIR];
  const int pax = (DIR == 0) ? 1 : 0;                  // lines are consecutive along this axis
  const int np = (ND >= 2) ? P.n[pax] : 1;
  const long long sa = (DIR == 0) ? 1 : (DIR == 1 ? (long long)nx : (long long)nx * ny);
  const long long sp = (pax == 0) ? 1 : (long long)nx;
  // the remaining axis (3-D): z for DIR 0/1, y for DIR 2
  const long long so = (ND == 3) ? ((DIR == 2) ? (long long)nx : (long long)nx * ny) : 0;
  // Workgroups are dealt round-robin to the 8 XCDs (each with its own L2).
  // Renumber them so that each XCD gets a contiguous run of tiles, in the order
  // in which neighbours share cache lines: along x the tiles of a line (they
  // share halo cells), along y and z the line blocks (TP doubles are half a
  // 128-byte line).
  int bt = blockIdx.x, bp = blockIdx.y, bo = blockIdx.z;
  {
    const int gt = gridDim.x, gp = gridDim.y;
    const int nb = gt * gp * gridDim.z;
    if ((nb % 8) == 0) {
      const int lin = (blockIdx.z * gp + blockIdx.y) * gt + blockIdx.x;
      const int lid = (lin % 8) * (nb / 8) + lin / 8;
      if (LF) {
        bp = lid % gp;
        bt = (lid / gp) % gt;
      } else {
        bt = lid % gt;
        bp = (lid / gt) % gp;
      }
      bo = lid / (gt * gp);
    }
  }
  const int t0 = bt * TL;
  const int p0 = bp * TP;
  const long long obase = (long long)bo * so;
  auto cell = [&](int a, int p) {   // a wrapped into [0, na)
    return obase + (long long)a * sa + (long long)(p0 + p) * sp;
  };
  auto wrap = [&](int a) {
    while (a < 0) a += na;
    while (a >= na) a -= na;
    return a;
  };
  // line and position of work item i of a phase with L positions per line
  auto item = [](int i, int L, int& p, int& t) {
    p = LF ? i % TP : i / L;
    t = LF ? i / TP : i % L;
  };

  // ---- stage y ----
  for (int it = tid; it < TP * NYv; it += TV_NT) {
    int p, t;
    item(it, NYv, p, t);
    if (p0 + p < np) {
      const long long q = cell(wrap(t0 - 5 + t), p);
#pragma unroll
      for (int r = 0; r < NR; ++r) s_y[at(r, p, t, NYv)] = y[r * N + q];
    }
  }
  __syncthreads();

  // ---- PPM edge states and branch codes, once per cell (local y index e + 2) ----
  if (tid < TP * NE) {
    int p, e;
    item(tid, NE, p, e);
    if (p0 + p < np) {
#pragma unroll
      for (int r = 0; r < NR; ++r) {
        const double* a = &s_y[at(r, p, e, NYv)];
        double l, rr;
        s_code[at(r, p, e, NE)] =
            (unsigned char)ppm_edges_code<TT>(a[0], a[TS], a[2 * TS], a[3 * TS], a[4 * TS], l, rr);
        s_eL[at(r, p, e, NE)] = l;
        s_eR[at(r, p, e, NE)] = rr;
      }
    }
  }
  __syncthreads();

  // ---- face adjoints: face f (local), between cells f-3 and f-2 of the tile ----
  if (tid < TP * NF) {
    int p, f;
    item(tid, NF, p, f);
    if (p0 + p < np) {
      const long long qb = cell(wrap(t0 - 3 + f), p), qa = cell(wrap(t0 - 2 + f), p);
      double phi[NR], Um[NR], Up[NR];
#pragma unroll
      for (int r = 0; r < NR; ++r) {
        phi[r] = scale * (lam[r * N + qa] - lam[r * N + qb]) * P.inv_dx;
        Um[r] = s_eR[at(r, p, f, NE)];        // right edge of the cell below the face
        Up[r] = s_eL[at(r, p, f + 1, NE)];    // left edge of the cell above it
      }
      double gm[NR], gp[NR];
      hll_vjp<ND, DIR, TT>(P, Um, Up, phi, gm, gp);
#pragma unroll
      for (int r = 0; r < NR; ++r) {
        s_fm[at(r, p, f, NF)] = TT(gm[r]);
        s_fm[at(NR + r, p, f, NF)] = TT(gp[r]);
      }
    }
  }
  __syncthreads();

  // ---- per variable: PPM contributions, then the gather into registers; the
  // own cells' outputs are loaded first and stored once at the end, so the loop
  // waits on no global load ----
  int gpi, gti;   // gather item: line and cell of the tile
  item(tid, TL, gpi, gti);
  const bool gown = tid < TP * TL && p0 + gpi < np && t0 + gti < na;
  const long long gq = gown ? cell(t0 + gti, gpi) : 0;
  double acc[NR];
#pragma unroll
  for (int r = 0; r < NR; ++r) acc[r] = (gown && accumulate) ? out[r * N + gq] : 0.0;
#pragma unroll
  for (int r = 0; r < NR; ++r) {
    if (tid < TP * NC) {
      int p, c;   // cell t0 - 2 + c, local y index c + 3
      item(tid, NC, p, c);
      if (p0 + p < np) {
        const TT mum = s_fm[at(r, p, c + 1, NF)];    // its right face, w.r.t. aR
        const TT mup = s_fm[at(NR + r, p, c, NF)];   // its left face, w.r.t. aL
        TT ga[5];
        ppm_vjp_code<TT>(s_code[at(r, p, c + 1, NE)], mup, mum, ga);
#pragma unroll
        for (int o = 0; o < 5; ++o) s_c[at(o, p, c, NC)] = ga[o];
      }
    }
    __syncthreads();
    if (gown) {
      // cell j = t0 + t receives C_o of cell j - (o - 2), local index t + 4 - o
      TT sum = TT(0);
#pragma unroll
      for (int o = 0; o < 5; ++o) sum += s_c[at(o, gpi, gti + 4 - o, NC)];
      acc[r] += double(sum);
    }
    __syncthreads();
  }
  if (gown) {
#pragma unroll
    for (int r = 0; r < NR; ++r) out[r * N + gq] = acc[r];
  }
}

// ---------------------------------------------------------------------------
// Host side of one segment (called by rhd_step_adjoint).
// ---------------------------------------------------------------------------
static unsigned blocks_for(long long n) { return (unsigned)((n + ATHREADS - 1) / ATHREADS); }

template <int ND, int DIR, typename TT>
static void launch_tvjp(const DevParams& P, const double* y, const double* lam, double scale,
                        double* out, bool accumulate, hipStream_t s) {
  constexpr int TL = TvjpShape<ND, DIR>::TL, TP = TvjpShape<ND, DIR>::TP;
  const int na = P.n[DIR];
  const int np = (ND >= 2) ? P.n[DIR == 0 ? 1 : 0] : 1;
  const int no = (ND == 3) ? P.n[DIR == 2 ? 1 : 2] : 1;
  const dim3 grid((na + TL - 1) / TL, (np + TP - 1) / TP, no);
  hipLaunchKernelGGL((k_tvjp<ND, DIR, TT>), grid, dim3(TV_NT), 0, s, P, y, lam, scale, out,
                     accumulate ? 1 : 0);
}

// out (rows E, F) = scale s'(y)^T lam, added to what out holds when accumulate,
// else written over it: the x launch sets or adds, y and z add
template <int ND, typename TT>
static hipError_t transport_vjp_t(const DevParams& P, const double* y, const double* lam,
                                  double scale, double* out, bool accumulate, hipStream_t s) {
  launch_tvjp<ND, 0, TT>(P, y, lam, scale, out, accumulate, s);
  if constexpr (ND >= 2) launch_tvjp<ND, 1, TT>(P, y, lam, scale, out, true, s);
  if constexpr (ND >= 3) launch_tvjp<ND, 2, TT>(P, y, lam, scale, out, true, s);
  return hipGetLastError();
}

// float32 stencil for a mixed-precision handle, double otherwise
template <int ND>
static hipError_t transport_vjp(const DevParams& P, bool mixed, const double* y, const double* lam,
                                double scale, double* out, bool accumulate, hipStream_t s) {
  return mixed ? transport_vjp_t<ND, float>(P, y, lam, scale, out, accumulate, s)
               : transport_vjp_t<ND, double>(P, y, lam, scale, out, accumulate, s);
}

template <int ND>
static hipError_t adjoint_nd(const AdjointArgs& A) {
  const DevParams& P = A.P;
  const long long N = P.N;
  const int nv = 2 + 2 * ND;
  const long long M = (long long)nv * N;
  hipStream_t s = A.stream;
  hipError_t e;
  // y^0 is the caller's state0 (read only); y^1..y^k and y^{1/2}..y^{k-1/2} are
  // written into the workspace
  auto Yw = [&](int n) { return A.states + (long long)(n - 1) * M; };          // y^n, n >= 1
  auto Y = [&](int n) -> const double* { return n == 0 ? A.state0 : Yw(n); };
  auto H = [&](int n) { return A.states + (long long)(A.nsteps + n) * M; };    // y^{n+1/2}
  // forward recompute of the segment
  for (int n = 0; n < A.nsteps; ++n) {
    e = launch_stage(P, MODE_STAGE1, A.mixed, Y(n), Y(n), H(n), A.rho, A.kP, A.kF, A.dt, A.err, s);
    if (e != hipSuccess) return e;
    e = launch_stage(P, MODE_STAGE2, A.mixed, H(n), Y(n), Yw(n + 1), A.rho, A.kP, A.kF, A.dt,
                     A.err, s);
    if (e != hipSuccess) return e;
  }
  // the adjoint runs in place in the caller's lambda and two workspace vectors;
  // the swaps leave it in lambda after an even number of steps, else one copy
  double* Lc = A.lambda;
  double* La = A.lam_b;
  double* Ln = A.lam_c;
  const unsigned nbc = blocks_for(N);
  const double dt = A.dt;
  for (int n = A.nsteps - 1; n >= 0; --n) {
    // stage 2 source at y^{n+1}: mu2 into Lc (in place)
    hipLaunchKernelGGL((k_src_adj<ND>), dim3(nbc), dim3(ATHREADS), 0, s, P, Y(n + 1), Lc, 1.0,
                       nullptr, Lc, A.rho, A.kP, A.kF, 0.5 * dt, A.gkP, A.gkF, nullptr, 0.0);
    // its transport: La (rows E, F) = dt/2 s'(y^{n+1/2})^T mu2
    e = transport_vjp<ND>(P, A.mixed, H(n), Lc, 0.5 * dt, La, false, s);
    if (e != hipSuccess) return e;
    // stage 1 source at y^{n+1/2} with lambda = mu2/2 + La: mu1 into La, and
    // Ln = mu1 + mu2/2 (mu2 still in Lc)
    hipLaunchKernelGGL((k_src_adj<ND>), dim3(nbc), dim3(ATHREADS), 0, s, P, H(n), Lc, 0.5, La, La,
                       A.rho, A.kP, A.kF, dt, A.gkP, A.gkF, Ln, 0.5);
    e = transport_vjp<ND>(P, A.mixed, Y(n), La, dt, Ln, true, s);
    if (e != hipSuccess) return e;
    double* t = Lc;
    Lc = Ln;
    Ln = t;
  }
  if (Lc != A.lambda) {
    e = hipMemcpyAsync(A.lambda, Lc, M * sizeof(double), hipMemcpyDeviceToDevice, s);
    if (e != hipSuccess) return e;
  }
  return hipGetLastError();
}

hipError_t launch_adjoint(const AdjointArgs& A) {
  switch (A.P.ndim) {
    case 1: return adjoint_nd<1>(A);
    case 2: return adjoint_nd<2>(A);
    case 3: return adjoint_nd<3>(A);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace rhd
