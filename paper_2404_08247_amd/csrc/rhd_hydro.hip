// Hydrodynamics kernels for gfx950: the explicit first half of the operator
// split of Sec. 3.1 (the Euler equations for rho, rho v, E_gas with the ideal-gas
// pressure p = (gamma - 1)(E_gas - rho |v|^2 / 2)), integrated with RK2-SSP as the
// paper does. The paper leaves the spatial scheme open; here it is a method of
// lines with PPM edge states of the primitive variables (rho, v, p), the same
// limited reconstruction as the radiation transport, and HLLC fluxes (Toro,
// Riemann Solvers and Numerical Methods for Fluid Dynamics, Sec. 10.4, with the
// wave-speed bounds S_L = min(u_L - a_L, u_R - a_R), S_R = max(u_L + a_L, u_R + a_R)).
//
// One thread per cell and RK stage: the thread reads the 7-cell stencil of its
// cell along each axis (neighbouring threads share these reads through L1/L2),
// forms the edge states of the three cells around its two faces and the two
// HLLC fluxes, and accumulates the flux divergence in registers. Each face flux
// is thus formed by the two cells that share it; the hydro step is not the hot
// path of the method (the radiation step, subcycled several times per hydro
// step, is), and this layout needs no flux arrays and no workspace beyond the
// RK2 intermediate state.
#include "rhd_device.hpp"

namespace rhd {

constexpr int HNT = 256;

// State pointers of the gas: rho, E_gas and the momentum rows (stride N).
struct GasPtrs {
  const double* r;
  const double* eg;
  const double* m;
};

// Primitive state W = (rho, v_0..v_{ND-1}, p) of cell q; flip negates v_axis.
template <int ND>
__device__ __forceinline__ void load_prim(const DevParams& P, const GasPtrs& U, long long q,
                                          int axis, bool flip, double* W) {
  const long long N = P.N;
  const double r = U.r[q];
  const double ir = rcp(r);
  double v2 = 0.0;
  W[0] = r;
#pragma unroll
  for (int k = 0; k < ND; ++k) {
    const double v = U.m[k * N + q] * ir;
    v2 += v * v;
    W[1 + k] = (flip && k == axis) ? -v : v;
  }
  W[1 + ND] = P.gm1 * (U.eg[q] - 0.5 * r * v2);
}

// HLLC flux along axis D between primitive states WL | WR; flux order
// (rho, rho v_0..v_{ND-1}, E_gas).
template <int ND, int D>
__device__ __forceinline__ void hllc_flux(double gamma, double inv_gm1, const double* WL,
                                          const double* WR, double* flux) {
  constexpr int NH = 2 + ND;
  const double rL = WL[0], rR = WR[0], uL = WL[1 + D], uR = WR[1 + D];
  const double pL = WL[1 + ND], pR = WR[1 + ND];
  const double aL = sqrt_nonneg(gamma * pL * rcp(rL));
  const double aR = sqrt_nonneg(gamma * pR * rcp(rR));
  const double SL = fmin(uL - aL, uR - aR);
  const double SR = fmax(uL + aL, uR + aR);
  // contact speed S*; mL < 0 < mR for any physical pair of states
  const double mL = rL * (SL - uL), mR = rR * (SR - uR);
  const double Ss = (pR - pL + mL * uL - mR * uR) * rcp(mL - mR);
  // the side whose state enters the flux: L for 0 <= S_L (supersonic) or
  // S_L < 0 <= S*; R for S* < 0 or S_R <= 0
  const bool sideL = !(SL < 0.0) || (SR > 0.0 && !(Ss < 0.0));
  const double* W = sideL ? WL : WR;
  const double r = sideL ? rL : rR, u = sideL ? uL : uR, p = sideL ? pL : pR;
  double v2 = 0.0;
#pragma unroll
  for (int k = 0; k < ND; ++k) v2 += W[1 + k] * W[1 + k];
  const double E = p * inv_gm1 + 0.5 * r * v2;
  double Fc[NH], Uc[NH];
  Uc[0] = r;
  Fc[0] = r * u;
#pragma unroll
  for (int k = 0; k < ND; ++k) {
    Uc[1 + k] = r * W[1 + k];
    Fc[1 + k] = Uc[1 + k] * u + (k == D ? p : 0.0);
  }
  Uc[1 + ND] = E;
  Fc[1 + ND] = (E + p) * u;
  if (!(SL < 0.0) || !(SR > 0.0)) {   // supersonic: the upwind state's flux
#pragma unroll
    for (int q = 0; q < NH; ++q) flux[q] = Fc[q];
    return;
  }
  // star state of side K: F*_K = F_K + S_K (U*_K - U_K)
  const double SK = sideL ? SL : SR;
  const double mK = sideL ? mL : mR;
  const double fac = mK * rcp(SK - Ss);
  double Us[NH];
  Us[0] = fac;
#pragma unroll
  for (int k = 0; k < ND; ++k) Us[1 + k] = fac * (k == D ? Ss : W[1 + k]);
  Us[1 + ND] = fac * (E * rcp(r) + (Ss - u) * (Ss + p * rcp(mK)));
#pragma unroll
  for (int q = 0; q < NH; ++q) flux[q] = Fc[q] + SK * (Us[q] - Uc[q]);
}

// -div of the gas fluxes along axis D at cell q (coordinate c along D, extent
// n, stride st), added to acc.
template <int ND, int D>
__device__ __forceinline__ void axis_divergence(const DevParams& P, const GasPtrs& U, long long q,
                                                int c, int n, long long st, double* acc) {
  constexpr int NH = 2 + ND;
  double W[7][NH];
#pragma unroll
  for (int m = 0; m < 7; ++m) {
    bool flip;
    const int s = ghost(c - 3 + m, n, P.bc[D], flip);
    load_prim<ND>(P, U, q + (long long)(s - c) * st, D, flip, W[m]);
  }
  // edge states of cells c-1, c, c+1 (index 0, 1, 2)
  double eL[3][NH], eR[3][NH];
#pragma unroll
  for (int j = 0; j < 3; ++j)
#pragma unroll
    for (int v = 0; v < NH; ++v)
      ppm_edges5<double>(W[j][v], W[j + 1][v], W[j + 2][v], W[j + 3][v], W[j + 4][v], eL[j][v],
                         eR[j][v]);
  double fm[NH], fp[NH];
  hllc_flux<ND, D>(P.gamma, P.inv_gm1, eR[0], eL[1], fm);
  hllc_flux<ND, D>(P.gamma, P.inv_gm1, eR[1], eL[2], fp);
#pragma unroll
  for (int v = 0; v < NH; ++v) acc[v] -= (fp[v] - fm[v]) * P.inv_dx;
}

// One RK2-SSP stage. STAGE 1: out = S + dt L(S). STAGE 2: out = (B + S + dt L(S))/2,
// B being the state at the start of the step (own cell only; out may alias B).
template <int ND, int STAGE>
__global__ void __launch_bounds__(HNT)
k_hydro(DevParams P, GasPtrs S, const double* Br, const double* Beg, const double* Bm, double* Or,
        double* Oeg, double* Om, double dt, unsigned long long* err) {
  constexpr int NH = 2 + ND;
  const long long q = (long long)blockIdx.x * HNT + threadIdx.x;
  const long long N = P.N;
  if (q >= N) return;
  const int nx = P.n[0], ny = P.n[1], nz = P.n[2];
  const int i = (int)(q % nx);
  const int j = (int)((q / nx) % ny);
  const int k = (int)(q / ((long long)nx * ny));
  double acc[NH];
#pragma unroll
  for (int v = 0; v < NH; ++v) acc[v] = 0.0;
  axis_divergence<ND, 0>(P, S, q, i, nx, 1, acc);
  if constexpr (ND >= 2) axis_divergence<ND, 1>(P, S, q, j, ny, nx, acc);
  if constexpr (ND >= 3) axis_divergence<ND, 2>(P, S, q, k, nz, (long long)nx * ny, acc);
  double r = S.r[q] + dt * acc[0];
  double eg = S.eg[q] + dt * acc[1 + ND];
  double m[ND];
#pragma unroll
  for (int d = 0; d < ND; ++d) m[d] = S.m[d * N + q] + dt * acc[1 + d];
  if constexpr (STAGE == 2) {
    r = 0.5 * (Br[q] + r);
    eg = 0.5 * (Beg[q] + eg);
#pragma unroll
    for (int d = 0; d < ND; ++d) m[d] = 0.5 * (Bm[d * N + q] + m[d]);
    double m2 = 0.0;
#pragma unroll
    for (int d = 0; d < ND; ++d) m2 += m[d] * m[d];
    if (!(r > 0.0) || !(eg - 0.5 * m2 * rcp(r) > 0.0)) report(err, q, ERR_NONPHYS);
  }
  Or[q] = r;
  Oeg[q] = eg;
#pragma unroll
  for (int d = 0; d < ND; ++d) Om[d * N + q] = m[d];
}

// Per-block maxima of max_d |v_d| + c_s (grid-stride loop).
template <int ND>
__global__ void __launch_bounds__(HNT)
k_hydro_speed(DevParams P, const double* __restrict__ rho, const double* __restrict__ y,
              double* __restrict__ partial) {
  __shared__ double red[HNT];
  const long long N = P.N;
  double smax = 0.0;
  for (long long q = (long long)blockIdx.x * HNT + threadIdx.x; q < N; q += (long long)gridDim.x * HNT) {
    const double r = rho[q];
    const double ir = rcp(r);
    double v2 = 0.0, vmax = 0.0;
#pragma unroll
    for (int d = 0; d < ND; ++d) {
      const double v = y[(2 + ND + d) * N + q] * ir;
      v2 += v * v;
      vmax = fmax(vmax, fabs(v));
    }
    const double p = P.gm1 * (y[(1 + ND) * N + q] - 0.5 * r * v2);
    smax = fmax(smax, vmax + sqrt_nonneg(fmax(P.gamma * p * ir, 0.0)));
  }
  red[threadIdx.x] = smax;
  __syncthreads();
  for (int s = HNT / 2; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s) red[threadIdx.x] = fmax(red[threadIdx.x], red[threadIdx.x + s]);
    __syncthreads();
  }
  if (threadIdx.x == 0) partial[blockIdx.x] = red[0];
}

template <int ND>
static hipError_t hydro_nd(const DevParams& P, double* y, double* rho, double* ws, double dt,
                           unsigned long long* err, hipStream_t s) {
  const long long N = P.N;
  const unsigned blocks = (unsigned)((N + HNT - 1) / HNT);
  GasPtrs U{rho, y + (1 + ND) * N, y + (2 + ND) * N};
  double* w_r = ws;
  double* w_eg = ws + N;
  double* w_m = ws + 2 * N;
  hipLaunchKernelGGL((k_hydro<ND, 1>), dim3(blocks), dim3(HNT), 0, s, P, U, nullptr, nullptr,
                     nullptr, w_r, w_eg, w_m, dt, err);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  GasPtrs W1{w_r, w_eg, w_m};
  hipLaunchKernelGGL((k_hydro<ND, 2>), dim3(blocks), dim3(HNT), 0, s, P, W1, rho, y + (1 + ND) * N,
                     y + (2 + ND) * N, rho, y + (1 + ND) * N, y + (2 + ND) * N, dt, err);
  return hipGetLastError();
}

hipError_t launch_hydro_step(const DevParams& P, double* y, double* rho, double* ws, double dt,
                             unsigned long long* err, hipStream_t s) {
  switch (P.ndim) {
    case 1: return hydro_nd<1>(P, y, rho, ws, dt, err, s);
    case 2: return hydro_nd<2>(P, y, rho, ws, dt, err, s);
    case 3: return hydro_nd<3>(P, y, rho, ws, dt, err, s);
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_hydro_speed(const DevParams& P, const double* y, const double* rho,
                              double* partial, int nblocks, hipStream_t s) {
  switch (P.ndim) {
    case 1: hipLaunchKernelGGL(k_hydro_speed<1>, dim3(nblocks), dim3(HNT), 0, s, P, rho, y, partial); break;
    case 2: hipLaunchKernelGGL(k_hydro_speed<2>, dim3(nblocks), dim3(HNT), 0, s, P, rho, y, partial); break;
    case 3: hipLaunchKernelGGL(k_hydro_speed<3>, dim3(nblocks), dim3(HNT), 0, s, P, rho, y, partial); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

}  // namespace rhd
