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
// df/dz and df/dkappa are exact: f is evaluated in forward-mode dual numbers
// seeded along each unknown. The fixed point of the paper's inner/outer iteration
// is the solution of r(z) = 0 with the closure tensor evaluated at z, so this is
// the derivative of what the forward step computes (to the outer tolerance).
//
// Transport adjoint s'(y)^T lambda (gather form, no atomics), one fused kernel
// per axis d, staged in LDS:
//   1. per face i+1/2: phi = dJ/dPhi = (lambda_{i+1} - lambda_i)/dx, and the
//      adjoints of its two edge states mu-/mu+ = (dPhi/dU-/+)^T phi (the closure
//      and its partials from one multi-tangent dual evaluation per side);
//   2. per cell i: PPM partials of its edge states w.r.t. the 5 stencil values
//      (constants of the limiter branch recorded when the edges were formed)
//      times mu- of face i+1/2 and mu+ of face i-1/2, giving its contribution
//      to each of the cells i-2..i+2;
//   3. per cell j: sum of the contributions addressed to j.
// Periodic axes only (the library rejects reflecting axes for the adjoint).
#include "rhd_device.hpp"

namespace rhd {

constexpr int ATHREADS = 256;

// ---------------------------------------------------------------------------
// Scalar types: double, a one-tangent dual, and a five-tangent dual.
// Comparisons, min/max and sign decisions use the value only.
// ---------------------------------------------------------------------------
struct Dd {
  double v, d;
};
template <typename S> __device__ __forceinline__ S mk0(double x);
template <> __device__ __forceinline__ double mk0<double>(double x) { return x; }
template <> __device__ __forceinline__ Dd mk0<Dd>(double x) { return Dd{x, 0.0}; }
__device__ __forceinline__ Dd mk(double v, double d = 0.0) { return Dd{v, d}; }
__device__ __forceinline__ Dd operator+(Dd a, Dd b) { return mk(a.v + b.v, a.d + b.d); }
__device__ __forceinline__ Dd operator-(Dd a, Dd b) { return mk(a.v - b.v, a.d - b.d); }
__device__ __forceinline__ Dd operator-(Dd a) { return mk(-a.v, -a.d); }
__device__ __forceinline__ Dd operator*(Dd a, Dd b) { return mk(a.v * b.v, a.d * b.v + a.v * b.d); }
__device__ __forceinline__ Dd operator*(double a, Dd b) { return mk(a * b.v, a * b.d); }
__device__ __forceinline__ Dd operator*(Dd a, double b) { return mk(a.v * b, a.d * b); }
__device__ __forceinline__ Dd operator+(Dd a, double b) { return mk(a.v + b, a.d); }
__device__ __forceinline__ Dd operator+(double a, Dd b) { return mk(a + b.v, b.d); }
__device__ __forceinline__ Dd operator-(double a, Dd b) { return mk(a - b.v, -b.d); }
__device__ __forceinline__ Dd operator-(Dd a, double b) { return mk(a.v - b, a.d); }
// Quotients and square roots of the derivative types use the refined hardware
// reciprocal and square root (rhd_device.hpp): they feed derivatives only.
__device__ __forceinline__ Dd operator/(Dd a, Dd b) {
  const double ib = rcp(b.v);
  const double q = a.v * ib;
  return mk(q, (a.d - q * b.d) * ib);
}
__device__ __forceinline__ Dd operator/(double a, Dd b) {
  const double ib = rcp(b.v);
  const double q = a * ib;
  return mk(q, -q * b.d * ib);
}
__device__ __forceinline__ Dd dsqrt(Dd a) {
  const double s = sqrt_nonneg(a.v);
  return mk(s, s > 0.0 ? a.d * (0.5 * rcp(s)) : 0.0);
}
__device__ __forceinline__ double dsqrt(double a) { return sqrt_nonneg(a); }
// 1/x on double or a derivative type
__device__ __forceinline__ double dinv(double x) { return rcp(x); }
__device__ __forceinline__ Dd dinv(Dd x) { return 1.0 / x; }
__device__ __forceinline__ double vof(double a) { return a; }
__device__ __forceinline__ double vof(Dd a) { return a.v; }
template <typename S> __device__ __forceinline__ S smax(S a, S b) { return vof(a) < vof(b) ? b : a; }

// N-tangent dual (value and N partial derivatives).
template <int N>
struct DT {
  double v, d[N];
};
template <int N> __device__ __forceinline__ DT<N> dtc(double x) {   // constant
  DT<N> r;
  r.v = x;
#pragma unroll
  for (int i = 0; i < N; ++i) r.d[i] = 0.0;
  return r;
}
template <int N> __device__ __forceinline__ DT<N> operator+(const DT<N>& a, const DT<N>& b) {
  DT<N> r;
  r.v = a.v + b.v;
#pragma unroll
  for (int i = 0; i < N; ++i) r.d[i] = a.d[i] + b.d[i];
  return r;
}
template <int N> __device__ __forceinline__ DT<N> operator-(const DT<N>& a, const DT<N>& b) {
  DT<N> r;
  r.v = a.v - b.v;
#pragma unroll
  for (int i = 0; i < N; ++i) r.d[i] = a.d[i] - b.d[i];
  return r;
}
template <int N> __device__ __forceinline__ DT<N> operator-(const DT<N>& a) {
  DT<N> r;
  r.v = -a.v;
#pragma unroll
  for (int i = 0; i < N; ++i) r.d[i] = -a.d[i];
  return r;
}
template <int N> __device__ __forceinline__ DT<N> operator*(double a, const DT<N>& b) {
  DT<N> r;
  r.v = a * b.v;
#pragma unroll
  for (int i = 0; i < N; ++i) r.d[i] = a * b.d[i];
  return r;
}
template <int N> __device__ __forceinline__ DT<N> operator*(const DT<N>& a, double b) {
  return b * a;
}
template <int N> __device__ __forceinline__ DT<N> operator*(const DT<N>& a, const DT<N>& b) {
  DT<N> r;
  r.v = a.v * b.v;
#pragma unroll
  for (int i = 0; i < N; ++i) r.d[i] = a.d[i] * b.v + a.v * b.d[i];
  return r;
}
template <int N> __device__ __forceinline__ DT<N> operator+(const DT<N>& a, double b) {
  DT<N> r = a;
  r.v += b;
  return r;
}
template <int N> __device__ __forceinline__ DT<N> operator+(double a, const DT<N>& b) {
  return b + a;
}
template <int N> __device__ __forceinline__ DT<N> operator-(double a, const DT<N>& b) {
  return (-b) + a;
}
template <int N> __device__ __forceinline__ DT<N> operator/(double a, const DT<N>& b) {
  const double ib = rcp(b.v);
  const double q = a * ib;
  const double s = -q * ib;
  DT<N> r;
  r.v = q;
#pragma unroll
  for (int i = 0; i < N; ++i) r.d[i] = s * b.d[i];
  return r;
}
template <int N> __device__ __forceinline__ DT<N> operator/(const DT<N>& a, const DT<N>& b) {
  const double ib = rcp(b.v);
  const double q = a.v * ib;
  DT<N> r;
  r.v = q;
#pragma unroll
  for (int i = 0; i < N; ++i) r.d[i] = (a.d[i] - q * b.d[i]) * ib;
  return r;
}
template <int N> __device__ __forceinline__ DT<N> dinv(const DT<N>& x) { return 1.0 / x; }
template <int N> __device__ __forceinline__ DT<N> dsqrt(const DT<N>& a) {
  const double sq = sqrt_nonneg(a.v);
  const double f = sq > 0.0 ? 0.5 * rcp(sq) : 0.0;
  DT<N> r;
  r.v = sq;
#pragma unroll
  for (int i = 0; i < N; ++i) r.d[i] = f * a.d[i];
  return r;
}
template <int N> __device__ __forceinline__ double vof(const DT<N>& a) { return a.v; }
template <> __device__ __forceinline__ DT<3> mk0<DT<3>>(double x) { return dtc<3>(x); }
template <> __device__ __forceinline__ DT<4> mk0<DT<4>>(double x) { return dtc<4>(x); }
template <> __device__ __forceinline__ DT<2> mk0<DT<2>>(double x) { return dtc<2>(x); }

// PPM edge states of the middle cell of a0..a4 (the forward's method, Sec. 3.3),
// with the branch taken by each step in a byte: bits 0-1, 2-3, 4-5 the cases of
// the three MC slopes (0 across an extremum, 1 centred, 2 left-limited, 3
// right-limited), bits 6-7 the monotonicity case (0 flattened, 1 l = -2 r,
// 2 r = -2 l, 3 unchanged). The edges are linear in a0..a4 within a branch, so
// the code alone fixes their derivatives. Ties go to the earlier case in that
// order, the same choice as the oracle's dual numbers. Branch-free: the lanes of
// a wave take different cases.
__device__ __forceinline__ unsigned slope_case(double dl, double dr, double& s) {
  // sgn(dc) min(|dc|, 2|dl|, 2|dr|), dc = (dl + dr)/2, compared at half scale
  const double al = fabs(dl), ar = fabs(dr);
  const double ac = 0.25 * fabs(dl + dr);
  const double mlr = fmin(al, ar);
  const unsigned c = (ac <= mlr) ? 1u : (al <= ar ? 2u : 3u);
  const bool same = dl * dr > 0.0;   // then sgn(dc) = sgn(dl)
  s = same ? copysign(2.0 * fmin(ac, mlr), dl) : 0.0;
  return same ? c : 0u;
}

__device__ __forceinline__ unsigned ppm_edges_code(double a0, double a1, double a2, double a3,
                                                   double a4, double& l, double& r) {
  const double d01 = a1 - a0, d12 = a2 - a1, d23 = a3 - a2, d34 = a4 - a3;
  double s1, s2, s3;
  const unsigned c1 = slope_case(d01, d12, s1);
  const unsigned c2 = slope_case(d12, d23, s2);
  const unsigned c3 = slope_case(d23, d34, s3);
  const double lo0 = (-0.5) * d12 - (1.0 / 6.0) * (s2 - s1);
  const double ro0 = 0.5 * d23 - (1.0 / 6.0) * (s3 - s2);
  // CW84 monotonicity: flatten at an extremum, else cap the overshooting side
  const bool flat = ro0 * lo0 >= 0.0;
  const double del = ro0 - lo0;
  const double da = del * (-3.0 * (lo0 + ro0)), dd = del * del;
  const bool capl = da > dd, capr = da < -dd;   // never both
  const unsigned cm = flat ? 0u : (capl ? 1u : (capr ? 2u : 3u));
  const double lo = flat ? 0.0 : (capl ? (-2.0) * ro0 : lo0);
  const double ro = flat ? 0.0 : (capr ? (-2.0) * lo0 : ro0);
  l = a2 + lo;
  r = a2 + ro;
  return c1 | (c2 << 2) | (c3 << 4) | (cm << 6);
}

// ga[o] = gl dl/da_o + gr dr/da_o in the branch recorded by ppm_edges_code
__device__ __forceinline__ void ppm_vjp_code(unsigned code, double gl, double gr, double* ga) {
  auto kl = [](unsigned c) { return c == 1 ? 0.5 : (c == 2 ? 2.0 : 0.0); };
  auto kr = [](unsigned c) { return c == 1 ? 0.5 : (c == 3 ? 2.0 : 0.0); };
  const unsigned c1 = code & 3u, c2 = (code >> 2) & 3u, c3 = (code >> 4) & 3u, cm = code >> 6;
  const double glo = (cm == 3) ? gl : (cm == 2 ? gl - 2.0 * gr : 0.0);
  const double gro = (cm == 3) ? gr : (cm == 1 ? gr - 2.0 * gl : 0.0);
  const double gs1 = (1.0 / 6.0) * glo;
  const double gs2 = (1.0 / 6.0) * (gro - glo);
  const double gs3 = -(1.0 / 6.0) * gro;
  const double g01 = kl(c1) * gs1;
  const double g12 = -0.5 * glo + kr(c1) * gs1 + kl(c2) * gs2;
  const double g23 = 0.5 * gro + kr(c2) * gs2 + kl(c3) * gs3;
  const double g34 = kr(c3) * gs3;
  ga[0] = -g01;
  ga[1] = g01 - g12;
  ga[2] = g12 - g23 + gl + gr;
  ga[3] = g23 - g34;
  ga[4] = g34;
}

// Row DIR of the closure tensor at U = (E, F_1..F_ND) (the forward's formulas)
// with the partials the HLL adjoint needs, for weights W_k:
//   Dk[k] = D_DIR,k,   A[j] = sum_k W_k dD_DIR,k/dU_j,   dD[j] = dD_DIR,DIR/dU_j.
// M1: w = max(|F|^2, (cE)^2), r = 1/w, f2 = |F|^2 r, s = sqrt(4 - 3 f2),
// h = 1/(2 + s), g = 3 h r F_DIR and D_DIR,k = g F_k + [k = DIR](1/3 - f2 h).
// Differentiated by hand (exact, the chain rule on these formulas):
//   df2 = r (d|F|^2 - f2 dw),   dh = h' df2 with h' = 3 h^2/(2 s),
//   dg = 3 F_DIR (h' r df2 - h r^2 dw) + 3 h r e_DIR,
//   dD_DIR,k = F_k dg + g e_k - [k = DIR](h + f2 h') df2.
// Eddington: D = I/3, no partials.
template <int ND, int DIR>
__device__ __forceinline__ void closure_row_vjp(const DevParams& P, const double* U,
                                                const double* W, double* Dk, double* A,
                                                double* dD) {
  if (P.closure == 1) {
#pragma unroll
    for (int k = 0; k < ND; ++k) Dk[k] = (k == DIR) ? 1.0 / 3.0 : 0.0;
#pragma unroll
    for (int j = 0; j <= ND; ++j) A[j] = dD[j] = 0.0;
    return;
  }
  double F2 = 0.0, PF = 0.0;
#pragma unroll
  for (int k = 0; k < ND; ++k) {
    F2 += U[1 + k] * U[1 + k];
    PF += W[k] * U[1 + k];
  }
  const double cE = P.c * U[0];
  const bool thin = !(F2 < cE * cE);   // the branch max() takes
  const double r = rcp(thin ? F2 : cE * cE);
  const double f2 = F2 * r;
  const double sq = sqrt_1_4(4.0 - 3.0 * f2);
  const double h = rcp(2.0 + sq);
  const double FD = U[1 + DIR];
  const double g = 3.0 * h * r * FD;
  const double hp = 1.5 * h * h * rcp(sq);
  const double qp = h + f2 * hp;
  const double a = 3.0 * FD * hp * r, b = -3.0 * FD * h * r * r;
  const double wq = W[DIR] * qp;
#pragma unroll
  for (int j = 0; j <= ND; ++j) {
    const double dF2 = (j == 0) ? 0.0 : 2.0 * U[j];
    const double dw = thin ? dF2 : ((j == 0) ? 2.0 * P.c * cE : 0.0);
    const double df2 = r * (dF2 - f2 * dw);
    double dg = a * df2 + b * dw;
    if (j == 1 + DIR) dg += 3.0 * h * r;
    A[j] = PF * dg - wq * df2 + ((j >= 1) ? g * W[j - 1] : 0.0);
    dD[j] = FD * dg - qp * df2 + ((j == 1 + DIR) ? g : 0.0);
  }
#pragma unroll
  for (int k = 0; k < ND; ++k) Dk[k] = g * U[1 + k] + ((k == DIR) ? (1.0 / 3.0) - f2 * h : 0.0);
}

// The mixed-frame four-force terms per cell, z = (E, F_1..F_ND, E_gas, p_1..p_ND):
// g = (-c G0, -G_1..-G_ND) from eq. G0-G1 (order 2; order 1 keeps the O(v/c)
// terms), P = D(E, F) E. The source terms are f = U g with the constant map
//   f_E = (chat/c) g_0, f_Egas = -g_0, f_F_k = c chat g_k, f_p_k = -g_k
// (eq. egupdate-fupdate in RSLA form).
template <int ND, typename S>
__device__ void source_g(const DevParams& P, const S* z, S rho, S kP, S kF, S kE, S* gout) {
  const double c = P.c;
  const S chiP = rho * kP, chiE = rho * kE, chiF = rho * kF;
  const S E = z[0], Eg = z[1 + ND];
  S v[ND];
  S v2 = mk0<S>(0.0), vF = mk0<S>(0.0), F2 = mk0<S>(0.0);
#pragma unroll
  for (int k = 0; k < ND; ++k) {
    v[k] = z[2 + ND + k] / rho;
    v2 = v2 + v[k] * v[k];
    vF = vF + v[k] * z[1 + k];
    F2 = F2 + z[1 + k] * z[1 + k];
  }
  const S b2 = v2 * P.inv_c2;
  const S T = (Eg - 0.5 * rho * v2) / (rho * P.cv_mass);
  const S T2 = T * T;
  const S B = P.a_r * (T2 * T2);
  S g = mk0<S>(0.0), iso = mk0<S>(1.0 / 3.0);
  if (P.closure != 1) {
    const S cE = c * E;
    const S r = dinv(smax(F2, cE * cE));
    const S f2 = F2 * r;
    const S h = dinv(2.0 + dsqrt(4.0 - 3.0 * f2));
    g = 3.0 * h * r;
    iso = (1.0 / 3.0) - f2 * h;
  }
  S Dv[ND];
#pragma unroll
  for (int k = 0; k < ND; ++k) Dv[k] = iso * v[k] + g * z[1 + k] * vF;
  const S vDv = iso * v2 + g * vF * vF;
  S mcG0, mG[ND];
  if (P.v_order == 2) {
    const S hb = 1.0 + 0.5 * b2;
    mcG0 = c * (chiP * B - chiE * E) * hb + (2.0 * chiE - chiF) * vF * (1.0 / c) +
           c * (chiF - chiE) * (b2 * E + E * vDv * P.inv_c2);
#pragma unroll
    for (int k = 0; k < ND; ++k)
      mG[k] = (-1.0 / c) * chiF * z[1 + k] * hb + (1.0 / c) * chiP * B * v[k] +
              (1.0 / c) * chiF * E * Dv[k] +
              (1.0 / c) * (chiF - chiE) * (E - 2.0 * vF * P.inv_c2) * v[k];
  } else {
    mcG0 = c * (chiP * B - chiE * E) + (2.0 * chiE - chiF) * vF * (1.0 / c);
#pragma unroll
    for (int k = 0; k < ND; ++k)
      mG[k] = (-1.0 / c) * chiF * z[1 + k] + (1.0 / c) * chiP * B * v[k] +
              (1.0 / c) * chiF * E * Dv[k] + (1.0 / c) * (chiF - chiE) * E * v[k];
  }
  gout[0] = mcG0;
#pragma unroll
  for (int k = 0; k < ND; ++k) gout[1 + k] = mG[k];
}

// ---------------------------------------------------------------------------
// Kernels
// ---------------------------------------------------------------------------
// Src adjoint: mu = A^{-T} lam at the converged cell state z, written back to lam;
// g_kappa += tau (df/dkappa)^T mu; and the vector updates that follow it in the
// reverse step: o1 = a1 mu (if o1), o2 = a2 mu + b2 o2 (if o2).
template <int ND>
__global__ void __launch_bounds__(ATHREADS)
k_src_adj(DevParams P, const double* __restrict__ zs, double* __restrict__ lam,
          const double* __restrict__ rho, const double* __restrict__ kP,
          const double* __restrict__ kF, double tau, double* gkP, double* gkF,
          double* __restrict__ o1, double a1, double* __restrict__ o2, double a2, double b2) {
  constexpr int M = 2 + 2 * ND;
  const long long q = (long long)blockIdx.x * ATHREADS + threadIdx.x;
  if (q >= P.N) return;
  const long long N = P.N;
  double z[M], lv[M];
#pragma unroll
  for (int j = 0; j < M; ++j) {
    z[j] = zs[j * N + q];
    lv[j] = lam[j * N + q];
  }
  auto outputs = [&](const double* mu) {
#pragma unroll
    for (int i = 0; i < M; ++i) {
      if (o1) o1[i * N + q] = a1 * mu[i];
      if (o2) o2[i * N + q] = a2 * mu[i] + (b2 == 0.0 ? 0.0 : b2 * o2[i * N + q]);
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
  // G = dg/dz. In 1-D/2-D: columns j..j+m-1 from an m-tangent evaluation (M = 2 m),
  // held in registers. In 3-D that needs more registers than two waves per SIMD
  // allow, so there: column j from a dual evaluation seeded along z_j, in a rolled
  // loop (the values of g are the same in every pass and stay in registers, only the
  // tangent is evaluated per pass), G in LDS, one slot per thread.
  constexpr bool GLDS = (ND == 3);
  __shared__ double s_G[GLDS ? m * M : 1][ATHREADS];
  double Greg[GLDS ? 1 : m][GLDS ? 1 : M];
  if constexpr (GLDS) {
#pragma unroll 1
    for (int j = 0; j < M; ++j) {
      Dd zd[M], gd[m];
#pragma unroll
      for (int i = 0; i < M; ++i) zd[i] = mk(z[i], i == j ? 1.0 : 0.0);
      source_g<ND, Dd>(P, zd, mk(rq), mk(kp), mk(kf), mk(ke), gd);
#pragma unroll
      for (int i = 0; i < m; ++i) s_G[i * M + j][threadIdx.x] = gd[i].d;
    }
  } else {
#pragma unroll
    for (int j = 0; j < M; j += m) {
      DT<m> zd[M], gd[m];
#pragma unroll
      for (int i = 0; i < M; ++i) {
        zd[i] = dtc<m>(z[i]);
        if (i >= j && i < j + m) zd[i].d[i - j] = 1.0;
      }
      source_g<ND, DT<m>>(P, zd, dtc<m>(rq), dtc<m>(kp), dtc<m>(kf), dtc<m>(ke), gd);
#pragma unroll
      for (int i = 0; i < m; ++i)
#pragma unroll
        for (int t = 0; t < m; ++t) Greg[i][j + t] = gd[i].d[t];
    }
  }
  auto G = [&](int i, int j) -> double {
    if constexpr (GLDS) return s_G[i * M + j][threadIdx.x];
    else return Greg[i][j];
  };
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
  // the kappa derivatives: tangent 0 along kappa_P (with kappa_F when it aliases
  // kappa_P and has no gradient of its own, and kappa_E = kappa_P through eP),
  // tangent 1 along kappa_F; one 2-tangent evaluation, or in 3-D two dual ones in a
  // rolled loop (registers, as above)
  const double kF0 = (P.kF_alias && !gkF) ? 1.0 : 0.0;
  double gk[2] = {0.0, 0.0};
  if constexpr (GLDS) {
#pragma unroll 1
    for (int t = 0; t < 2; ++t) {
      Dd zd[M], gd[m];
#pragma unroll
      for (int i = 0; i < M; ++i) zd[i] = mk(z[i]);
      source_g<ND, Dd>(P, zd, mk(rq), mk(kp, t == 0 ? 1.0 : 0.0), mk(kf, t == 0 ? kF0 : 1.0),
                       mk(ke, t == 0 ? eP : 0.0), gd);
      double acc = 0.0;
#pragma unroll
      for (int i = 0; i < m; ++i) acc += gd[i].d * um[i];
      if (t == 0) gk[0] = acc;
      else gk[1] = acc;
    }
  } else {
    DT<2> zd[M], gd[m];
#pragma unroll
    for (int i = 0; i < M; ++i) zd[i] = dtc<2>(z[i]);
    DT<2> kpd = dtc<2>(kp), kfd = dtc<2>(kf), ked = dtc<2>(ke);
    kpd.d[0] = 1.0;
    kfd.d[0] = kF0;
    kfd.d[1] = 1.0;
    ked.d[0] = eP;
    source_g<ND, DT<2>>(P, zd, dtc<2>(rq), kpd, kfd, ked, gd);
#pragma unroll
    for (int i = 0; i < m; ++i) {
      gk[0] += gd[i].d[0] * um[i];
      gk[1] += gd[i].d[1] * um[i];
    }
  }
  gkP[q] += tau * gk[0];
  if (gkF) gkF[q] += tau * gk[1];
  else if (!P.kF_alias) gkP[q] += tau * gk[1];
#pragma unroll
  for (int i = 0; i < M; ++i) lam[i * N + q] = mu[i];
  outputs(mu);
}

// phi^T dPhi/dU-+ of the HLL flux along DIR between edge states Um | Up:
//   Phi_0 = (chat/c)(F-_D + F+_D)/2 - hS (E+ - E-),
//   Phi_1+k = c chat (E- D-_Dk + E+ D+_Dk)/2 - hS (F+_k - F-_k),
//   hS = chat sqrt(max(D-_DD, D+_DD))/2,
// with the closure rows and their partials w.r.t. (E, F) of each side from
// closure_row_vjp. gm = (dPhi/dU-)^T phi, gp = (dPhi/dU+)^T phi.
template <int ND, int DIR>
__device__ __forceinline__ void hll_vjp(const DevParams& P, const double* Um, const double* Up,
                                        const double* phi, double* gm, double* gp) {
  constexpr int NR = 1 + ND;
  const double* W = phi + 1;   // weights of the flux components
  double Dm[ND], Dp[ND], Am[NR], Ap[NR], dDm[NR], dDp[NR];
  closure_row_vjp<ND, DIR>(P, Um, W, Dm, Am, dDm);
  closure_row_vjp<ND, DIR>(P, Up, W, Dp, Ap, dDp);
  const bool mside = !(Dm[DIR] < Dp[DIR]);   // the side max() takes
  const double Dmax = mside ? Dm[DIR] : Dp[DIR];
  const double sq = sqrt_nonneg(Dmax);
  const double hS = 0.5 * P.chat * sq;
  const double dhS = sq > 0.0 ? 0.25 * P.chat * rcp(sq) : 0.0;   // d hS / d D_DD
  double Sig = 0.0;   // sum_r phi_r (U+_r - U-_r)
#pragma unroll
  for (int r = 0; r < NR; ++r) Sig += phi[r] * (Up[r] - Um[r]);
  double WDm = 0.0, WDp = 0.0;
#pragma unroll
  for (int k = 0; k < ND; ++k) {
    WDm += W[k] * Dm[k];
    WDp += W[k] * Dp[k];
  }
  const double hcc = 0.5 * P.c_chat;
  const double sd = Sig * dhS;
#pragma unroll
  for (int r = 0; r < NR; ++r) {
    // sum_k phi_1+k d(E D_Dk)/dU_r on each side
    const double tm = Um[0] * Am[r] + (r == 0 ? WDm : 0.0);
    const double tp = Up[0] * Ap[r] + (r == 0 ? WDp : 0.0);
    gm[r] = hcc * tm + hS * phi[r];
    gp[r] = hcc * tp - hS * phi[r];
    if (r == 1 + DIR) {
      gm[r] += 0.5 * P.chat_over_c * phi[0];
      gp[r] += 0.5 * P.chat_over_c * phi[0];
    }
    if (mside) {
      gm[r] -= sd * dDm[r];
    } else {
      gp[r] -= sd * dDp[r];
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

template <int ND, int DIR>
__global__ void __launch_bounds__(TV_NT)
k_tvjp(DevParams P, const double* __restrict__ y, const double* __restrict__ lam, double scale,
       double* __restrict__ out) {
  constexpr int NR = 1 + ND;
  constexpr int TL = TvjpShape<ND, DIR>::TL, TP = TvjpShape<ND, DIR>::TP;
  constexpr int NYv = TL + 10, NF = TL + 5, NC = TL + 4, NE = TL + 6;
  static_assert(NE * TP <= TV_NT && NC * TP <= TV_NT, "one item round per phase");
  // work items of a phase: along x the cells of a line are consecutive in memory
  // and run fastest; along y and z the lines do, so the global loads and stores
  // of a wave cover runs of TP consecutive x cells
  constexpr bool LF = (DIR != 0);
  // Two LDS regions, each holding what one phase reads and the next one writes:
  //   A: staged y (edge phase), then the face adjoints (contribution phase);
  //   B: edge states of the cells next to the faces, local y index e + 2 (face
  //      phase), then the PPM contributions (gather);
  // plus the branch codes. A barrier separates every reuse.
  constexpr int NYB = NR * TP * NYv, NFB = 2 * NR * TP * NF;
  constexpr int NEB = 2 * NR * TP * NE, NCB = 5 * TP * NC;
  __shared__ double s_a[NYB > NFB ? NYB : NFB];
  __shared__ double s_b[NEB > NCB ? NEB : NCB];
  __shared__ unsigned char s_code[NR][TP][NE];
  double(*s_y)[TP][NYv] = reinterpret_cast<double(*)[TP][NYv]>(s_a);
  double(*s_fm)[TP][NF] = reinterpret_cast<double(*)[TP][NF]>(s_a);
  double(*s_eL)[TP][NE] = reinterpret_cast<double(*)[TP][NE]>(s_b);
  double(*s_eR)[TP][NE] = reinterpret_cast<double(*)[TP][NE]>(s_b + NR * TP * NE);
  double(*s_c)[TP][NC] = reinterpret_cast<double(*)[TP][NC]>(s_b);

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
  const int t0 = blockIdx.x * TL;
  const int p0 = blockIdx.y * TP;
  const long long obase = (long long)blockIdx.z * so;
  auto cell = [&](int a, int p) {   // a wrapped into [0, na)
    return obase + (long long)a * sa + (long long)(p0 + p) * sp;
  };
  auto wrap = [&](int a) {
    while (a < 0) a += na;
    while (a >= na) a -= na;
    return a;
  };

  // ---- stage y and lam ----
  for (int it = tid; it < TP * NYv; it += TV_NT) {
    const int p = LF ? it % TP : it / NYv, t = LF ? it / TP : it % NYv;
    if (p0 + p < np) {
      const long long q = cell(wrap(t0 - 5 + t), p);
#pragma unroll
      for (int r = 0; r < NR; ++r) s_y[r][p][t] = y[r * N + q];
    }
  }
  __syncthreads();

  // ---- PPM edge states and branch codes, once per cell (local y index e + 2) ----
  if (tid < TP * NE) {
    const int p = LF ? tid % TP : tid / NE, e = LF ? tid / TP : tid % NE;
    if (p0 + p < np) {
#pragma unroll
      for (int r = 0; r < NR; ++r) {
        const double* a = &s_y[r][p][e];
        double l, rr;
        s_code[r][p][e] = (unsigned char)ppm_edges_code(a[0], a[1], a[2], a[3], a[4], l, rr);
        s_eL[r][p][e] = l;
        s_eR[r][p][e] = rr;
      }
    }
  }
  __syncthreads();

  // ---- face adjoints: face f (local), between cells f-3 and f-2 of the tile ----
  if (tid < TP * NF) {
    const int p = LF ? tid % TP : tid / NF, f = LF ? tid / TP : tid % NF;
    if (p0 + p < np) {
      const long long qb = cell(wrap(t0 - 3 + f), p), qa = cell(wrap(t0 - 2 + f), p);
      double phi[NR], Um[NR], Up[NR];
#pragma unroll
      for (int r = 0; r < NR; ++r) {
        phi[r] = scale * (lam[r * N + qa] - lam[r * N + qb]) * P.inv_dx;
        Um[r] = s_eR[r][p][f];                // right edge of the cell below the face
        Up[r] = s_eL[r][p][f + 1];            // left edge of the cell above it
      }
      double gm[NR], gp[NR];
      hll_vjp<ND, DIR>(P, Um, Up, phi, gm, gp);
#pragma unroll
      for (int r = 0; r < NR; ++r) {
        s_fm[r][p][f] = gm[r];
        s_fm[NR + r][p][f] = gp[r];
      }
    }
  }
  __syncthreads();

  // ---- per variable: PPM contributions, then the gather ----
  for (int r = 0; r < NR; ++r) {
    if (tid < TP * NC) {
      // cell t0 - 2 + c, local y index c + 3
      const int p = LF ? tid % TP : tid / NC, c = LF ? tid / TP : tid % NC;
      if (p0 + p < np) {
        const double mum = s_fm[r][p][c + 1];      // its right face, w.r.t. aR
        const double mup = s_fm[NR + r][p][c];     // its left face, w.r.t. aL
        double ga[5];
        ppm_vjp_code(s_code[r][p][c + 1], mup, mum, ga);
#pragma unroll
        for (int o = 0; o < 5; ++o) s_c[o][p][c] = ga[o];
      }
    }
    __syncthreads();
    if (tid < TP * TL) {
      const int p = LF ? tid % TP : tid / TL, t = LF ? tid / TP : tid % TL;
      if (p0 + p < np && t0 + t < na) {
        // cell j = t0 + t receives C_o of cell j - (o - 2), local index t + 4 - o
        double acc = 0.0;
#pragma unroll
        for (int o = 0; o < 5; ++o) acc += s_c[o][p][t + 4 - o];
        out[r * N + cell(t0 + t, p)] += acc;
      }
    }
    __syncthreads();
  }
}

// ---------------------------------------------------------------------------
// Host driver of one segment (called by rhd_step_adjoint).
// ---------------------------------------------------------------------------
static unsigned blocks_for(long long n) { return (unsigned)((n + ATHREADS - 1) / ATHREADS); }

template <int ND, int DIR>
static void launch_tvjp(const DevParams& P, const double* y, const double* lam, double scale,
                        double* out, hipStream_t s) {
  constexpr int TL = TvjpShape<ND, DIR>::TL, TP = TvjpShape<ND, DIR>::TP;
  const int na = P.n[DIR];
  const int np = (ND >= 2) ? P.n[DIR == 0 ? 1 : 0] : 1;
  const int no = (ND == 3) ? P.n[DIR == 2 ? 1 : 2] : 1;
  const dim3 grid((na + TL - 1) / TL, (np + TP - 1) / TP, no);
  hipLaunchKernelGGL((k_tvjp<ND, DIR>), grid, dim3(TV_NT), 0, s, P, y, lam, scale, out);
}

template <int ND>
static hipError_t transport_vjp(const DevParams& P, const double* y, const double* lam, double scale,
                                double* out, hipStream_t s) {
  launch_tvjp<ND, 0>(P, y, lam, scale, out, s);
  if constexpr (ND >= 2) launch_tvjp<ND, 1>(P, y, lam, scale, out, s);
  if constexpr (ND >= 3) launch_tvjp<ND, 2>(P, y, lam, scale, out, s);
  return hipGetLastError();
}

template <int ND>
static hipError_t adjoint_nd(const AdjointArgs& A) {
  const DevParams& P = A.P;
  const long long N = P.N;
  const int nv = 2 + 2 * ND;
  const long long M = (long long)nv * N;
  hipStream_t s = A.stream;
  hipError_t e;
  auto Y = [&](int n) { return A.states + (long long)n * M; };                 // y^n, n = 0..k
  auto H = [&](int n) { return A.states + (long long)(A.nsteps + 1 + n) * M; }; // y^{n+1/2}
  // forward recompute of the segment
  e = hipMemcpyAsync(Y(0), A.state0, M * sizeof(double), hipMemcpyDeviceToDevice, s);
  if (e != hipSuccess) return e;
  for (int n = 0; n < A.nsteps; ++n) {
    e = launch_stage(P, MODE_STAGE1, A.mixed, Y(n), Y(n), H(n), A.rho, A.kP, A.kF, A.dt, A.err, s);
    if (e != hipSuccess) return e;
    e = launch_stage(P, MODE_STAGE2, A.mixed, H(n), Y(n), Y(n + 1), A.rho, A.kP, A.kF, A.dt, A.err, s);
    if (e != hipSuccess) return e;
  }
  double* Lc = A.lam_a;
  double* La = A.lam_b;
  double* Ln = A.lam_c;
  e = hipMemcpyAsync(Lc, A.lambda, M * sizeof(double), hipMemcpyDeviceToDevice, s);
  if (e != hipSuccess) return e;
  const unsigned nbc = blocks_for(N);
  const double dt = A.dt;
  for (int n = A.nsteps - 1; n >= 0; --n) {
    // stage 2 source at y^{n+1}: mu2 in Lc, La = Ln = mu2/2
    hipLaunchKernelGGL((k_src_adj<ND>), dim3(nbc), dim3(ATHREADS), 0, s, P, Y(n + 1), Lc, A.rho,
                       A.kP, A.kF, 0.5 * dt, A.gkP, A.gkF, La, 0.5, Ln, 0.5, 0.0);
    e = transport_vjp<ND>(P, H(n), Lc, 0.5 * dt, La, s);
    if (e != hipSuccess) return e;
    // stage 1 source at y^{n+1/2}: mu1 in La, Ln += mu1
    hipLaunchKernelGGL((k_src_adj<ND>), dim3(nbc), dim3(ATHREADS), 0, s, P, H(n), La, A.rho, A.kP,
                       A.kF, dt, A.gkP, A.gkF, nullptr, 0.0, Ln, 1.0, 1.0);
    e = transport_vjp<ND>(P, Y(n), La, dt, Ln, s);
    if (e != hipSuccess) return e;
    double* t = Lc;
    Lc = Ln;
    Ln = t;
  }
  e = hipMemcpyAsync(A.lambda, Lc, M * sizeof(double), hipMemcpyDeviceToDevice, s);
  if (e != hipSuccess) return e;
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
