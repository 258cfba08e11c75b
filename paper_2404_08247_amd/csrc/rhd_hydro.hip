// Hydrodynamics kernels for gfx950: the explicit first half of the operator
// split of Sec. 3.1 (the Euler equations for rho, rho v, E_gas with the ideal-gas
// pressure p = (gamma - 1)(E_gas - rho |v|^2 / 2)), integrated with RK2-SSP as the
// paper does. The paper leaves the spatial scheme open; here it is a method of
// lines with PPM edge states of the primitive variables (rho, v, p), the same
// limited reconstruction as the radiation transport, and HLLC fluxes (Toro,
// Riemann Solvers and Numerical Methods for Fluid Dynamics, Sec. 10.4, with the
// wave-speed bounds S_L = min(u_L - a_L, u_R - a_R), S_R = max(u_L + a_L, u_R + a_R)).
//
// Tiling, as in the radiation stage kernels: a workgroup of 256 threads owns a
// TX x TY column of cells (32 x 8 in 2-D/3-D, 256 x 1 in 1-D) and marches along
// z. Per plane, the primitive variables of the tile and a 3-cell halo are staged
// in LDS; PPM edge states are formed once per cell and HLLC fluxes once per face
// (flattened loops over the tile, halo work spread over all waves), fluxes go
// back into LDS. Along z every thread keeps its column's PPM pipeline in
// registers (values, limited slope, raw interface, right edge, flux below), so
// each z face is formed once without LDS. The RK2 intermediate state is the only
// workspace.
#include "rhd_device.hpp"

namespace rhd {

constexpr int HNT = 256;

// State pointers of the gas: rho, E_gas and the momentum rows (stride N).
struct GasPtrs {
  const double* r;
  const double* eg;
  const double* m;
};

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

template <int ND> struct HTile;
template <> struct HTile<1> { static constexpr int TX = 256, TY = 1; };
template <> struct HTile<2> { static constexpr int TX = 32, TY = 8; };
template <> struct HTile<3> { static constexpr int TX = 32, TY = 8; };
constexpr int HH = 3;   // halo width (PPM stencil)

// Raw primitive state (rho, v_0..v_{ND-1}, p) of in-range cell q.
template <int ND>
__device__ __forceinline__ void load_prim_raw(const DevParams& P, const GasPtrs& U, long long q,
                                              double* W) {
  const long long N = P.N;
  const double r = U.r[q];
  const double ir = rcp(r);
  double v2 = 0.0;
  W[0] = r;
#pragma unroll
  for (int k = 0; k < ND; ++k) {
    const double v = U.m[k * N + q] * ir;
    v2 += v * v;
    W[1 + k] = v;
  }
  W[1 + ND] = P.gm1 * (U.eg[q] - 0.5 * r * v2);
}

// One RK2-SSP stage. STAGE 1: out = S + dt L(S). STAGE 2: out = (B + S + dt L(S))/2,
// B being the state at the start of the step (own cell only; out may alias B).
template <int ND, int STAGE>
__global__ void __launch_bounds__(HNT)
k_hydro(DevParams P, GasPtrs S, const double* Br, const double* Beg, const double* Bm, double* Or,
        double* Oeg, double* Om, double dt, int zchunk, unsigned long long* err) {
  constexpr int TX = HTile<ND>::TX;
  constexpr int TY = HTile<ND>::TY;
  constexpr int NH = 2 + ND;                 // rho, v_0..v_{ND-1}, p
  constexpr int TW = TX + 2 * HH;
  constexpr int TH = (ND >= 2) ? TY + 2 * HH : 1;
  constexpr int NTILE = TW * TH;
  constexpr int NEX = (TX + 2) * TY;
  constexpr int NEY = (ND >= 2) ? TX * (TY + 2) : 0;
  constexpr int NFX = (TX + 1) * TY;
  constexpr int NFY = (ND >= 2) ? TX * (TY + 1) : 0;
  constexpr int NFYs = NFY > 0 ? NFY : 1;
  // primitive tile; edge states per face (s_exR[f] / s_exL[f]: left / right of x
  // face f), overwritten by the face's flux; the last slot of each edge array takes
  // the one edge of a halo cell that no face needs
  __shared__ double s_w[NH][NTILE];
  __shared__ double s_exL[NH][NFX + 1], s_exR[NH][NFX + 1];
  __shared__ double s_eyL[NH][NFYs + 1], s_eyR[NH][NFYs + 1];

  const int tid = threadIdx.x;
  const int tx = tid % TX;
  const int ty = tid / TX;
  const int nx = P.n[0], ny = P.n[1], nz = P.n[2];
  // XCD-contiguous renumbering of the workgroups (as in the stage kernels)
  int bx = blockIdx.x, by = blockIdx.y, bz = blockIdx.z;
  {
    const int gxn = gridDim.x, gyn = gridDim.y;
    const int nb = gxn * gyn * gridDim.z;
    if ((nb % 8) == 0) {
      const int lin = (blockIdx.z * gyn + blockIdx.y) * gxn + blockIdx.x;
      const int log_id = (lin % 8) * (nb / 8) + lin / 8;
      bx = log_id % gxn;
      by = (log_id / gxn) % gyn;
      bz = log_id / (gxn * gyn);
    }
  }
  const int x0 = bx * TX;
  const int y0 = by * TY;
  const int z0 = bz * zchunk;
  const int z1 = min(z0 + zchunk, nz);
  const int gx = x0 + tx, gy = y0 + ty;
  const bool valid = (gx < nx) && (gy < ny);
  // in-range source column (ragged tiles: a ghost cell of the tile)
  bool own_fx = false, own_fy = false;
  const int cx = ghost(gx, nx, P.bc[0], own_fx);
  const int cy = (ND >= 2) ? ghost(gy, ny, P.bc[1], own_fy) : 0;
  const long long N = P.N;
  const long long plane = (long long)nx * ny;
  const long long colq = (long long)cy * nx + cx;
  const long long outq = (long long)gy * nx + gx;
  const double gamma = P.gamma, inv_gm1 = P.inv_gm1;

  // ---- z pipeline (ND == 3): values of planes k, k+1, k+2; limited slope of
  // k+1; raw left interface of k+1; right edge of k; z-flux at k-1/2 ----
  double zc[NH], zv1[NH], zv2[NH], zaR[NH], zfl[NH], zs[NH], zIo[NH];
  auto zload = [&](int g, double* W) {   // plane g of this column, z-mirror applied
    bool flip;
    const int gz = ghost(g, nz, P.bc[2], flip);
    load_prim_raw<ND>(P, S, (long long)gz * plane + colq, W);
    if (flip) W[3] = -W[3];
  };
  if constexpr (ND == 3) {
    double w[6][NH];
#pragma unroll
    for (int m = 0; m < 6; ++m) zload(z0 - 3 + m, w[m]);
    double Um[NH], Up[NH];
#pragma unroll
    for (int r = 0; r < NH; ++r) {
      const double d01 = w[1][r] - w[0][r], d12 = w[2][r] - w[1][r];
      const double d23 = w[3][r] - w[2][r], d34 = w[4][r] - w[3][r];
      const double d45 = w[5][r] - w[4][r];
      const double sA = mc_slope(d01, d12), sB = mc_slope(d12, d23);
      const double sC = mc_slope(d23, d34), sD = mc_slope(d34, d45);
      double lm = -0.5 * d12 - (sB - sA) * (1.0 / 6.0);
      double rm = 0.5 * d23 - (sC - sB) * (1.0 / 6.0);
      ppm_monotone(lm, rm);               // cell z0-1
      double l0 = -0.5 * d23 - (sC - sB) * (1.0 / 6.0);
      double r0 = 0.5 * d34 - (sD - sC) * (1.0 / 6.0);
      ppm_monotone(l0, r0);               // cell z0
      Um[r] = w[2][r] + rm;
      Up[r] = w[3][r] + l0;
      zaR[r] = w[3][r] + r0;
      zIo[r] = -0.5 * d34 - (sD - sC) * (1.0 / 6.0);
      zs[r] = sD;
      zc[r] = w[3][r];
      zv1[r] = w[4][r];
      zv2[r] = w[5][r];
    }
    hllc_flux<ND, 2 % ND>(gamma, inv_gm1, Um, Up, zfl);
  }

  // halo position of this thread (at most one) and its source cell in a plane
  constexpr int NHX = 2 * HH * TY;
  constexpr int NHY = (ND >= 2) ? 2 * HH * TX : 0;
  static_assert(NHX + NHY <= HNT, "one halo position per thread");
  long long hoff = -1;
  int htile = 0;
  bool hfx = false, hfy = false;
  if (tid < NHX + NHY) {
    int lx, ly;
    if (tid < NHX) {
      const int row = tid / (2 * HH), j = tid % (2 * HH);
      lx = (j < HH) ? j : TX + j;
      ly = row + (ND >= 2 ? HH : 0);
    } else {
      const int h2 = tid - NHX;
      const int col = h2 % TX, j = h2 / TX;
      lx = col + HH;
      ly = (j < HH) ? j : TY + j;
    }
    const int sx = ghost(x0 + lx - HH, nx, P.bc[0], hfx);
    const int sy = (ND >= 2) ? ghost(y0 + ly - HH, ny, P.bc[1], hfy) : 0;
    hoff = (long long)sy * nx + sx;
    htile = ly * TW + lx;
  }

  for (int k = z0; k < z1; ++k) {
    // ---- stage the plane's primitive tile ----
    double own[NH];
    if constexpr (ND == 3) {
#pragma unroll
      for (int r = 0; r < NH; ++r) own[r] = zc[r];
    } else {
      load_prim_raw<ND>(P, S, (long long)k * plane + colq, own);
    }
    {
      const int t = (ty + (ND >= 2 ? HH : 0)) * TW + tx + HH;
#pragma unroll
      for (int r = 0; r < NH; ++r)
        s_w[r][t] = ((own_fx && r == 1) || (own_fy && r == 2)) ? -own[r] : own[r];
    }
    if (hoff >= 0) {
      double hv[NH];
      load_prim_raw<ND>(P, S, (long long)k * plane + hoff, hv);
#pragma unroll
      for (int r = 0; r < NH; ++r)
        s_w[r][htile] = ((hfx && r == 1) || (hfy && r == 2)) ? -hv[r] : hv[r];
    }
    double w3[NH];   // plane k+3 of this column for the z pipeline
    if constexpr (ND == 3) zload(k + 3, w3);
    // own-cell conserved state of the stencil input (and of B in stage 2)
    double u_own[NH], b_own[NH];
    if (valid) {
      const long long q = (long long)k * plane + outq;
      u_own[0] = S.r[q];
#pragma unroll
      for (int d = 0; d < ND; ++d) u_own[1 + d] = S.m[d * N + q];
      u_own[1 + ND] = S.eg[q];
      if constexpr (STAGE == 2) {
        b_own[0] = Br[q];
#pragma unroll
        for (int d = 0; d < ND; ++d) b_own[1 + d] = Bm[d * N + q];
        b_own[1 + ND] = Beg[q];
      }
    }
    __syncthreads();

    // ---- z face k+1/2 from the register pipeline (half of the waves during the
    // edge phase, the other half after the flux phase) ----
    double divz[NH];
#pragma unroll
    for (int r = 0; r < NH; ++r) divz[r] = 0.0;
    auto zface = [&]() {
      if constexpr (ND == 3) {
        double aL1[NH], aR1[NH];
#pragma unroll
        for (int r = 0; r < NH; ++r) {
          const double d12 = zv2[r] - zv1[r];
          const double d23 = w3[r] - zv2[r];
          const double s2 = mc_slope(d12, d23);                   // cell k+2
          double lo = zIo[r];
          double ro = 0.5 * d12 - (s2 - zs[r]) * (1.0 / 6.0);     // cell k+1
          zIo[r] = -0.5 * d12 - (s2 - zs[r]) * (1.0 / 6.0);       // left of cell k+2
          ppm_monotone(lo, ro);
          aL1[r] = zv1[r] + lo;
          aR1[r] = zv1[r] + ro;
          zs[r] = s2;
          zc[r] = zv1[r];
          zv1[r] = zv2[r];
          zv2[r] = w3[r];
        }
        double f3[NH];
        hllc_flux<ND, 2 % ND>(gamma, inv_gm1, zaR, aL1, f3);
#pragma unroll
        for (int r = 0; r < NH; ++r) {
          divz[r] = f3[r] - zfl[r];
          zfl[r] = f3[r];
          zaR[r] = aR1[r];
        }
      }
    };

    // ---- PPM edge states, once per cell (y items first) ----
    for (int e = tid; e < NEX + NEY; e += HNT) {
      if (ND >= 2 && e < NEY) {
        const int col = e % TX, row = e / TX;                // cell y0 + row - 1
        const int base = row * TW + col + HH;
        const int fl = (row > 0) ? (row - 1) * TX + col : NFY;
        const int fr = (row <= TY) ? row * TX + col : NFY;
#pragma unroll
        for (int r = 0; r < NH; ++r) {
          const double* a = &s_w[r][base];
          double l, rr;
          ppm_edges5<double>(a[0], a[TW], a[2 * TW], a[3 * TW], a[4 * TW], l, rr);
          s_eyL[r][fl] = l;
          s_eyR[r][fr] = rr;
        }
      } else {
        const int ex = e - NEY;
        const int row = ex / (TX + 2), col = ex % (TX + 2);  // cell x0 + col - 1
        const int base = (row + (ND >= 2 ? HH : 0)) * TW + col;
        const int fl = (col > 0) ? row * (TX + 1) + col - 1 : NFX;
        const int fr = (col <= TX) ? row * (TX + 1) + col : NFX;
#pragma unroll
        for (int r = 0; r < NH; ++r) {
          const double* a = &s_w[r][base];
          double l, rr;
          ppm_edges5<double>(a[0], a[1], a[2], a[3], a[4], l, rr);
          s_exL[r][fl] = l;
          s_exR[r][fr] = rr;
        }
      }
    }
    if (ND == 3 && tid >= HNT / 2) zface();
    __syncthreads();

    // ---- HLLC fluxes, once per face (x faces padded to a multiple of 64) ----
    constexpr int NFXP = (ND >= 2) ? ((NFX + 63) / 64) * 64 : NFX;
    const int ftid = (tid + HNT / 2) % HNT;
    for (int f = ftid; f < NFXP + NFY; f += HNT) {
      double Um[NH], Up[NH], fl[NH];
      if (f < NFXP) {
        if (f < NFX) {
#pragma unroll
          for (int r = 0; r < NH; ++r) {
            Um[r] = s_exR[r][f];
            Up[r] = s_exL[r][f];
          }
          hllc_flux<ND, 0>(gamma, inv_gm1, Um, Up, fl);
#pragma unroll
          for (int r = 0; r < NH; ++r) s_exR[r][f] = fl[r];
        }
      } else if constexpr (ND >= 2) {
        const int f2 = f - NFXP;
#pragma unroll
        for (int r = 0; r < NH; ++r) {
          Um[r] = s_eyR[r][f2];
          Up[r] = s_eyL[r][f2];
        }
        hllc_flux<ND, (ND >= 2 ? 1 : 0)>(gamma, inv_gm1, Um, Up, fl);
#pragma unroll
        for (int r = 0; r < NH; ++r) s_eyR[r][f2] = fl[r];
      }
    }
    if (!(ND == 3 && tid >= HNT / 2)) zface();
    __syncthreads();

    // ---- divergence and update of the own cell ----
    if (valid) {
      double out[NH];
#pragma unroll
      for (int r = 0; r < NH; ++r) {
        double d = s_exR[r][ty * (TX + 1) + tx + 1] - s_exR[r][ty * (TX + 1) + tx];
        if constexpr (ND >= 2) d += s_eyR[r][(ty + 1) * TX + tx] - s_eyR[r][ty * TX + tx];
        d += divz[r];
        out[r] = u_own[r] - dt * d * P.inv_dx;
        if constexpr (STAGE == 2) out[r] = 0.5 * (b_own[r] + out[r]);
      }
      const long long q = (long long)k * plane + outq;
      if constexpr (STAGE == 2) {
        double m2 = 0.0;
#pragma unroll
        for (int d = 0; d < ND; ++d) m2 += out[1 + d] * out[1 + d];
        if (!(out[0] > 0.0) || !(out[1 + ND] - 0.5 * m2 * rcp(out[0]) > 0.0))
          report(err, q, ERR_NONPHYS);
      }
      Or[q] = out[0];
#pragma unroll
      for (int d = 0; d < ND; ++d) Om[d * N + q] = out[1 + d];
      Oeg[q] = out[1 + ND];
    }
    // no barrier here: the next plane's staging writes s_w, which nobody has read
    // since the barrier after the edge states; the edge/flux arrays it overwrites
    // next are written only after the staging barrier
  }
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
  constexpr int TX = HTile<ND>::TX, TY = HTile<ND>::TY;
  const long long N = P.N;
  const int nx = P.n[0], ny = P.n[1], nz = P.n[2];
  const int gxn = (nx + TX - 1) / TX, gyn = (ny + TY - 1) / TY;
  int zchunk = nz;
  if (ND == 3) {   // >= 1024 workgroups while chunks stay >= 8 planes
    const long long cols = (long long)gxn * gyn;
    zchunk = 16;
    while (zchunk > 8 && cols * ((nz + zchunk - 1) / zchunk) < 1024) zchunk /= 2;
    if (zchunk > nz) zchunk = nz;
  }
  const int gzn = (nz + zchunk - 1) / zchunk;
  GasPtrs U{rho, y + (1 + ND) * N, y + (2 + ND) * N};
  double* w_r = ws;
  double* w_eg = ws + N;
  double* w_m = ws + 2 * N;
  hipLaunchKernelGGL((k_hydro<ND, 1>), dim3(gxn, gyn, gzn), dim3(HNT), 0, s, P, U, nullptr,
                     nullptr, nullptr, w_r, w_eg, w_m, dt, zchunk, err);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  GasPtrs W1{w_r, w_eg, w_m};
  hipLaunchKernelGGL((k_hydro<ND, 2>), dim3(gxn, gyn, gzn), dim3(HNT), 0, s, P, W1, rho,
                     y + (1 + ND) * N, y + (2 + ND) * N, rho, y + (1 + ND) * N, y + (2 + ND) * N,
                     dt, zchunk, err);
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
