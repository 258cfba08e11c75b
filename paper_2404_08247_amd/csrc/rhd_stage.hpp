#pragma once
// The fused PD-ARS stage kernel k_stage and its launcher for one grid
// dimensionality. One kernel per stage (Sec. 3.2, eq. imex1 / imex2): the
// explicit transport s(y) of (E, F) and the local implicit source of every cell
// of a tile run in the same launch, so y(t) never goes to HBM. Included by
// rhd_forward.hip, which instantiates it for 1-D and 3-D grids, and by
// rhd_stage2d.hip, which instantiates it for 2-D grids: the two files are
// compiled with different instruction schedulers (build.py).
//
// Tiling. A workgroup of 256 threads owns a TX x TY column of cells (32 x 8 in
// 2-D/3-D, 256 x 1 in 1-D) and marches along z over a chunk of planes:
//  - x and y faces: the plane's (E, F) tile with a 3-cell halo is staged in LDS;
//    PPM edge states are computed once per cell and HLL fluxes once per face,
//    both as flattened loops over the tile so the halo work is spread over the
//    whole workgroup; fluxes are written back into the tile's LDS.
//  - z faces: each thread keeps its own column's PPM pipeline in registers
//    (values k+1..k+3, the limited slope and raw interface value ahead, the
//    monotonised right edge of cell k and the z-flux below), so every z-face is
//    computed once and z needs neither LDS nor a halo exchange.
// Halo cells come from the ghost rule (periodic wrap, or mirror with the normal
// flux component negated; below an inflow axis, the fixed inflow state), applied
// on load.

#include <climits>
#include <cmath>
#include <type_traits>

#include "rhd_device.hpp"
#include "rhd_internal.hpp"

namespace rhd {

constexpr int HALO = 3;
constexpr int NTHREADS = 256;
// Minimum waves per SIMD the stage kernels are compiled for (caps VGPRs at
// 512 / RHD_STAGE_WAVES; excess live values go to AGPRs).
#ifndef RHD_STAGE_WAVES
#define RHD_STAGE_WAVES 1
#endif
#ifndef RHD_TX
#define RHD_TX 32
#endif
#ifndef RHD_ZCHUNK_MAX
#define RHD_ZCHUNK_MAX 128
#endif
#ifndef RHD_STAGE_SLOTS
#define RHD_STAGE_SLOTS 512
#endif
#ifndef RHD_ZBAL
#define RHD_ZBAL 1
#endif
#ifndef RHD_XCD_REMAP
#define RHD_XCD_REMAP 1
#endif
template <int ND> struct TileShape;
template <> struct TileShape<1> { static constexpr int TX = 256, TY = 1; };
template <> struct TileShape<2> { static constexpr int TX = RHD_TX, TY = 256 / RHD_TX; };
template <> struct TileShape<3> { static constexpr int TX = RHD_TX, TY = 256 / RHD_TX; };

// Value of radiation variable r (E, F_1..F_ND) in a ghost cell below an inflow
// axis: the fixed inflow state, with its flux along the axis.
__device__ __forceinline__ double inflow_value(const DevParams& P, int r, int axis) {
  return r == 0 ? P.inflow_E : (r == 1 + axis ? P.inflow_F : 0.0);
}

// Kernel variants (separate instantiations, so the plain path carries none of
// their code): VAR_PLAIN, plain HLL with the lean local source; VAR_GEN, plain
// HLL with the general source (a separate kappa_E, the source S, chi_F != chi_E
// at order 2); VAR_TDEP, the general source with temperature-dependent
// opacities; VAR_EPS, the optional Skinner-type eps on the HLL energy flux, which
// stages chi_F = rho kappa_F of the tile in LDS, with the general source.
enum { VAR_PLAIN = 0, VAR_EPS = 1, VAR_GEN = 2, VAR_TDEP = 3 };

// The plain 2-D kernels fit 128 VGPRs without spills (under the default
// scheduler, which their file uses): four waves per SIMD, so with their 39 KB of
// LDS four workgroups share a CU and a 512^2 grid (1024 tiles) runs in one round
// instead of two. The other variants keep RHD_STAGE_WAVES.
template <int ND, int VAR>
constexpr int stage_waves() { return (ND == 2 && VAR == VAR_PLAIN) ? 4 : RHD_STAGE_WAVES; }

template <int ND, int MODE, typename TT, int VAR>
__global__ void __launch_bounds__(NTHREADS) __attribute__((amdgpu_waves_per_eu(stage_waves<ND, VAR>())))
k_stage(DevParams P, const double* __restrict__ ys, const double* yo, double* yw,
        const double* __restrict__ rho, const double* __restrict__ kP,
        const double* __restrict__ kF, double dt, int zchunk, unsigned long long* err) {
  constexpr bool EPS = (VAR == VAR_EPS);
  constexpr int SV = (VAR == VAR_PLAIN) ? SRC_LEAN : (VAR == VAR_TDEP ? SRC_TDEP : SRC_GEN);
  constexpr int TX = TileShape<ND>::TX;
  constexpr int TY = TileShape<ND>::TY;
  constexpr int NR = 1 + ND;                 // radiation variables E, F_1..F_ND
  constexpr int TW = TX + 2 * HALO;          // tile row length
  constexpr int TH = (ND >= 2) ? TY + 2 * HALO : 1;
  constexpr int NTILE = TW * TH;
  constexpr int NEX = (TX + 2) * TY;         // cells that need x edge states
  constexpr int NEY = (ND >= 2) ? TX * (TY + 2) : 0;
  constexpr int NFX = (TX + 1) * TY;         // x faces
  constexpr int NFY = (ND >= 2) ? TX * (TY + 1) : 0;
  constexpr int NFYs = NFY > 0 ? NFY : 1;

  // LDS holds values, edge states and fluxes in double; TT is the arithmetic
  // type of the limiter and closure (delta form, see rhd_device.hpp). Edge
  // states are stored per face: s_exR[f] / s_exL[f] are the states left / right
  // of x face f (the right edge of the cell before it, the left edge of the cell
  // after it), so a face item reads index f of both and then overwrites it with
  // the face's flux; the (E, F) tile is free again once the edge states exist.
  // The last slot of each edge array takes the one edge of a halo cell that no
  // face needs, so that every edge item stores unconditionally.
  __shared__ double s_area[NR][NTILE];       // (E, F) tile
  __shared__ double s_exL[NR][NFX + 1], s_exR[NR][NFX + 1];
  __shared__ double s_eyL[NR][NFYs + 1], s_eyR[NR][NFYs + 1];
  __shared__ double s_chi[EPS ? NTILE : 1];  // chi_F of the tile (EPS only)

  const int tid = threadIdx.x;
  const int tx = tid % TX;
  const int ty = tid / TX;
  const int nx = P.n[0], ny = P.n[1], nz = P.n[2];
  // Workgroups are dealt round-robin to the 8 XCDs (each with its own L2).
  // Renumber them so that each XCD gets a contiguous run of tiles (x fastest,
  // then y, then z) and the halo planes/rows that neighbouring tiles share are
  // read through the same L2.
  int bx = blockIdx.x, by = blockIdx.y, bz = blockIdx.z;
  {
    const int gxn = gridDim.x, gyn = gridDim.y;
    const int nb = gxn * gyn * gridDim.z;
    if (RHD_XCD_REMAP && (nb % 8) == 0) {
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
  // In-range source column of this thread. Threads of a ragged last tile sit
  // past the grid edge; their column then acts as a ghost cell of the tile and
  // takes the ghost rule (including the sign flip of the normal flux).
  bool own_fx = false, own_fy = false;
  const int cx = ghost(gx, nx, P.bc[0], own_fx);
  const int cy = (ND >= 2) ? ghost(gy, ny, P.bc[1], own_fy) : 0;
  const long long N = P.N;
  const long long plane = (long long)nx * ny;
  const long long colq = (long long)cy * nx + cx;   // in-range column of this thread
  const long long outq = (long long)gy * nx + gx;   // own column (valid threads)
  const double* __restrict__ kFv = P.kF_alias ? kP : kF;   // flux-mean opacity

  const double c = P.c, ch = P.chat, chc = P.chat_over_c, cch = P.c_chat;
  const int clo = P.closure;
  // theta dt of this stage's source (PD-ARS: dt in stage 1, dt/2 in stage 2;
  // the RK2-SSP comparator: dt) and 1/(theta dt chat), the same for every cell
  const double tau_src = (MODE == MODE_STAGE2 && P.scheme == 0) ? 0.5 * dt : dt;
  const double inv_tch = rcp(tau_src * ch);

  // ---- z pipeline state (ND == 3) ----
  // a_k, a_{k+1}, a_{k+2}; limited slope of cell k+1; raw left interface of
  // cell k+1 (offset from a_{k+1}); monotonised right edge of cell k; z-flux at
  // face k-1/2.
  double zc[NR], zv1[NR], zv2[NR], zaR[NR], zfl_prev[NR];
  TT zs[NR], zIo[NR];
  if constexpr (ND == 3) {
    double w[6][NR];
#pragma unroll
    for (int m = 0; m < 6; ++m) {
      bool flip;
      const int gz = ghost(z0 - 3 + m, nz, P.bc[2], flip);
      const bool fixz = (z0 - 3 + m < 0) && P.bc[2] == BC_INFLOW;
      const long long q = gz * plane + colq;
#pragma unroll
      for (int r = 0; r < NR; ++r) {
        const double val = ys[r * N + q];
        w[m][r] = fixz ? inflow_value(P, r, 2) : ((flip && r == 3) ? -val : val);
      }
    }
    double Um[NR], Up[NR];
#pragma unroll
    for (int r = 0; r < NR; ++r) {
      const TT d01 = TT(w[1][r] - w[0][r]), d12 = TT(w[2][r] - w[1][r]);
      const TT d23 = TT(w[3][r] - w[2][r]), d34 = TT(w[4][r] - w[3][r]);
      const TT d45 = TT(w[5][r] - w[4][r]);
      const TT sA = mc_slope(d01, d12);   // cell z0-2
      const TT sB = mc_slope(d12, d23);   // cell z0-1
      const TT sC = mc_slope(d23, d34);   // cell z0
      const TT sD = mc_slope(d34, d45);   // cell z0+1
      TT lm = TT(-0.5) * d12 - (sB - sA) * TT(1.0 / 6.0);
      TT rm = TT(0.5) * d23 - (sC - sB) * TT(1.0 / 6.0);
      ppm_monotone(lm, rm);               // cell z0-1
      TT l0 = TT(-0.5) * d23 - (sC - sB) * TT(1.0 / 6.0);
      TT r0 = TT(0.5) * d34 - (sD - sC) * TT(1.0 / 6.0);
      ppm_monotone(l0, r0);               // cell z0
      Um[r] = w[2][r] + double(rm);
      Up[r] = w[3][r] + double(l0);
      zaR[r] = w[3][r] + double(r0);
      zIo[r] = TT(-0.5) * d34 - (sD - sC) * TT(1.0 / 6.0);
      zs[r] = sD;
      zc[r] = w[3][r];
      zv1[r] = w[4][r];
      zv2[r] = w[5][r];
    }
    double eps0 = 1.0;
    if constexpr (EPS) {
      bool fl_;
      const long long qa = ghost(z0 - 1, nz, P.bc[2], fl_) * plane + colq;
      const long long qb = (long long)z0 * plane + colq;
      eps0 = face_eps(P.eps_dx, rho[qa] * kFv[qa], rho[qb] * kFv[qb]);
    }
    hll_flux<ND, 2 % ND, TT>(clo, c, ch, chc, cch, Um, Up, zfl_prev, eps0);
  }

  // halo position of this thread and its source cell within a plane
  constexpr int NHX = 2 * HALO * TY;
  constexpr int NHY = (ND >= 2) ? 2 * HALO * TX : 0;
  static_assert(NHX + NHY <= NTHREADS, "one halo position per thread");
  long long hoff = -1;
  int htile = 0;
  bool hfx = false, hfy = false;
  int hfix = -1;   // axis whose inflow state this halo position holds (-1: none)
  // some halo position of this workgroup lies below an inflow axis (uniform)
  const bool inflow_blk = (x0 < HALO && P.bc[0] == BC_INFLOW) ||
                          (ND >= 2 && y0 < HALO && P.bc[1] == BC_INFLOW);
  if (tid < NHX + NHY) {
    int lx, ly;
    if (tid < NHX) {
      const int row = tid / (2 * HALO), j = tid % (2 * HALO);
      lx = (j < HALO) ? j : TX + j;
      ly = row + (ND >= 2 ? HALO : 0);
    } else {
      const int h2 = tid - NHX;
      const int col = h2 % TX, j = h2 / TX;
      lx = col + HALO;
      ly = (j < HALO) ? j : TY + j;
    }
    const int sx = ghost(x0 + lx - HALO, nx, P.bc[0], hfx);
    const int sy = (ND >= 2) ? ghost(y0 + ly - HALO, ny, P.bc[1], hfy) : 0;
    // halo positions lie outside the tile along one axis only (no corners)
    if (x0 + lx - HALO < 0 && P.bc[0] == BC_INFLOW) hfix = 0;
    if (ND >= 2 && y0 + ly - HALO < 0 && P.bc[1] == BC_INFLOW) hfix = 1;
    hoff = (long long)sy * nx + sx;
    htile = ly * TW + lx;
  }

  // Global loads for plane k+1 are issued while plane k is processed: the
  // thread's halo position (hv) and, in 3-D, the z-pipeline value of plane k+4
  // (zn, zn_flip); they are consumed one iteration later.
  double hv[NR], zn[NR];
  bool zn_flip = false;
  auto load_halo = [&](int kk) {
    if (hoff >= 0) {
      const long long q = (long long)kk * plane + hoff;
#pragma unroll
      for (int r = 0; r < NR; ++r) hv[r] = ys[r * N + q];
    }
  };
  auto load_zplane = [&](int kk) {   // the plane 3 above plane kk
    const int gz = ghost(kk + 3, nz, P.bc[2], zn_flip);
    const long long q = gz * plane + colq;
#pragma unroll
    for (int r = 0; r < NR; ++r) zn[r] = ys[r * N + q];
  };
  load_halo(z0);
  if constexpr (ND == 3) load_zplane(z0);

  for (int k = z0; k < z1; ++k) {
    // Wave priority: the transport phases of a plane are chained by barriers, the
    // source phase that follows has none. Two workgroups share a CU; issuing the
    // barrier-chained phases first shortens each workgroup's critical path while
    // the other one's source work fills the VALU (6 % on the 128^3 step).
    __builtin_amdgcn_s_setprio(1);
    // ---- source-phase inputs of the own cell, issued before the transport so
    // their latency overlaps it: E_gas and rho v of the stencil state, and for
    // stage 2 the whole own-cell y^n; rho and kappa.
    constexpr int NPRE = (MODE == MODE_STAGE2) ? (1 + ND) + (2 + 2 * ND) : (1 + ND);
    double pre[NPRE];
    double pre_rho = 1.0, pre_kp = 0.0, pre_kf = 0.0, pre_ke = 0.0, pre_j = 0.0;
    if constexpr (MODE != MODE_TRANSPORT) {
      const long long qc = k * plane + colq;   // in range for every thread
#pragma unroll
      for (int m = 0; m <= ND; ++m) pre[m] = ys[(1 + ND + m) * N + qc];
      if constexpr (MODE == MODE_STAGE2) {
#pragma unroll
        for (int m = 0; m < 2 + 2 * ND; ++m) pre[1 + ND + m] = yo[m * N + qc];
      }
      pre_rho = rho[qc];
      pre_kp = kP[qc];
      pre_kf = P.kF_alias ? pre_kp : kF[qc];
      if constexpr (SV >= SRC_GEN) {
        pre_ke = P.kE ? P.kE[qc] : pre_kp;
        if (P.jS) pre_j = P.jS[qc];
      }
    }
    // ---------------- stage the plane's (E, F) tile in LDS ----------------
    double own[NR];
    if constexpr (ND == 3) {
#pragma unroll
      for (int r = 0; r < NR; ++r) own[r] = zc[r];
    } else {
      const long long q = k * plane + colq;
#pragma unroll
      for (int r = 0; r < NR; ++r) own[r] = ys[r * N + q];
    }
    {
      const int t = (ty + (ND >= 2 ? HALO : 0)) * TW + tx + HALO;
#pragma unroll
      for (int r = 0; r < NR; ++r)
        s_area[r][t] = ((own_fx && r == 1) || (own_fy && r == 2)) ? -own[r] : own[r];
    }
    // halo (3 columns left/right of every row, 3 rows above/below): each thread
    // copies at most one position, whose source offset was resolved once per
    // block (hoff < 0: no position); its values were loaded one plane ahead
    if (hoff >= 0) {
#pragma unroll
      for (int r = 0; r < NR; ++r)
        s_area[r][htile] = ((hfx && r == 1) || (hfy && r == 2)) ? -hv[r] : hv[r];
      // below an inflow axis the fixed state replaces the loaded value (same
      // thread, same address: program order)
      if (inflow_blk && hfix >= 0) {
#pragma unroll
        for (int r = 0; r < NR; ++r) s_area[r][htile] = inflow_value(P, r, hfix);
      }
    }
    double chi_k = 0.0, chi_k1 = 0.0;   // chi_F of the own cell at planes k and k+1 (EPS)
    if constexpr (EPS) {
      const long long qo = k * plane + colq;
      chi_k = rho[qo] * kFv[qo];
      s_chi[(ty + (ND >= 2 ? HALO : 0)) * TW + tx + HALO] = chi_k;
      if (hoff >= 0) {
        const long long qh = k * plane + hoff;
        s_chi[htile] = rho[qh] * kFv[qh];
      }
      if constexpr (ND == 3) {
        bool fl_;
        const long long q1 = ghost(k + 1, nz, P.bc[2], fl_) * plane + colq;
        chi_k1 = rho[q1] * kFv[q1];
      }
    }
    double w3n[NR];
    bool w3_flip = false;
    if constexpr (ND == 3) {
#pragma unroll
      for (int r = 0; r < NR; ++r) w3n[r] = zn[r];
      w3_flip = zn_flip;
    }
    if (k + 1 < z1) {
      load_halo(k + 1);
      if constexpr (ND == 3) load_zplane(k + 1);
    }
    __syncthreads();

    // ---------------- z face k+1/2 from the register pipeline ----------------
    // (no LDS: run by half of the waves during the edge phase, in which they
    // have one item round fewer, and by the other half after the flux phase)
    double divz[NR];
#pragma unroll
    for (int r = 0; r < NR; ++r) divz[r] = 0.0;
    auto zface = [&]() {
      if constexpr (ND == 3) {
        double aL1[NR], fz[NR];
#pragma unroll
        for (int r = 0; r < NR; ++r) {
          const double w3 = (w3_flip && r == 3) ? -w3n[r] : w3n[r];
          const TT d12 = TT(zv2[r] - zv1[r]);
          const TT d23 = TT(w3 - zv2[r]);
          const TT s2 = mc_slope(d12, d23);                       // cell k+2
          TT lo = zIo[r];
          TT ro = TT(0.5) * d12 - (s2 - zs[r]) * TT(1.0 / 6.0);   // cell k+1
          zIo[r] = TT(-0.5) * d12 - (s2 - zs[r]) * TT(1.0 / 6.0); // left of cell k+2
          ppm_monotone(lo, ro);
          aL1[r] = zv1[r] + double(lo);
          const double aR1 = zv1[r] + double(ro);
          zs[r] = s2;
          zc[r] = zv1[r];
          zv1[r] = zv2[r];
          zv2[r] = w3;
          fz[r] = aR1;   // kept until the flux below is formed
        }
        double fl3[NR];
        hll_flux<ND, 2 % ND, TT>(clo, c, ch, chc, cch, zaR, aL1, fl3,
                                 EPS ? face_eps(P.eps_dx, chi_k, chi_k1) : 1.0);
#pragma unroll
        for (int r = 0; r < NR; ++r) {
          divz[r] = fl3[r] - zfl_prev[r];
          zfl_prev[r] = fl3[r];
          zaR[r] = fz[r];
        }
      }
    };

    // ---------------- PPM edge states, once per cell ----------------
    // y items first: their count TX (TY + 2) is a multiple of 64 for the 2-D/3-D
    // tiles, so no wave mixes x and y items
    for (int e = tid; e < NEX + NEY; e += NTHREADS) {
      if (ND >= 2 && e < NEY) {
        const int col = e % TX, row = e / TX;                // cell y0 + row - 1
        const int base = row * TW + col + HALO;              // = centre - 2 rows
        // left edge -> face row-1 (below the cell), right edge -> face row
        const int fl = (row > 0) ? (row - 1) * TX + col : NFY;
        const int fr = (row <= TY) ? row * TX + col : NFY;
#pragma unroll
        for (int r = 0; r < NR; ++r) {
          const double* a = &s_area[r][base];
          double l, rr;
          ppm_edges5<TT>(a[0], a[TW], a[2 * TW], a[3 * TW], a[4 * TW], l, rr);
          s_eyL[r][fl] = l;
          s_eyR[r][fr] = rr;
        }
      } else {
        const int ex = e - NEY;
        const int row = ex / (TX + 2), col = ex % (TX + 2);  // cell x0 + col - 1
        const int base = (row + (ND >= 2 ? HALO : 0)) * TW + col;  // = centre - 2
        const int fl = (col > 0) ? row * (TX + 1) + col - 1 : NFX;
        const int fr = (col <= TX) ? row * (TX + 1) + col : NFX;
#pragma unroll
        for (int r = 0; r < NR; ++r) {
          const double* a = &s_area[r][base];
          double l, rr;
          ppm_edges5<TT>(a[0], a[1], a[2], a[3], a[4], l, rr);
          s_exL[r][fl] = l;
          s_exR[r][fr] = rr;
        }
      }
    }
    if (RHD_ZBAL && ND == 3 && tid >= NTHREADS / 2) zface();
    __syncthreads();

    // ---------------- HLL fluxes, once per face (into the tile's LDS) -------
    // x faces occupy items [0, NFXP) (padded to a multiple of 64 so no wave
    // mixes x and y faces), y faces follow
    constexpr int NFXP = (ND >= 2) ? ((NFX + 63) / 64) * 64 : NFX;
    // item order rotated by half a block, so that the last (partial) round of
    // face items falls to the waves that run the z face after the edge phase
    const int ftid = RHD_ZBAL ? (tid + NTHREADS / 2) % NTHREADS : tid;
    for (int f = ftid; f < NFXP + NFY; f += NTHREADS) {
      double Um[NR], Up[NR], fl[NR];
      if (f < NFXP) {
        if (f < NFX) {
#pragma unroll
          for (int r = 0; r < NR; ++r) {
            Um[r] = s_exR[r][f];
            Up[r] = s_exL[r][f];
          }
          double eps_f = 1.0;
          if constexpr (EPS) {
            const int row = f / (TX + 1), fx = f % (TX + 1);   // between cells fx-1 | fx
            const int b = (row + (ND >= 2 ? HALO : 0)) * TW + fx + HALO;
            eps_f = face_eps(P.eps_dx, s_chi[b - 1], s_chi[b]);
          }
          hll_flux<ND, 0, TT>(clo, c, ch, chc, cch, Um, Up, fl, eps_f);
#pragma unroll
          for (int r = 0; r < NR; ++r) s_exR[r][f] = fl[r];
        }
      } else if constexpr (ND >= 2) {
        const int f2 = f - NFXP;
#pragma unroll
        for (int r = 0; r < NR; ++r) {
          Um[r] = s_eyR[r][f2];
          Up[r] = s_eyL[r][f2];
        }
        double eps_f = 1.0;
        if constexpr (EPS) {
          const int col = f2 % TX, fy = f2 / TX;               // between rows fy-1 | fy
          const int b = (fy + HALO) * TW + col + HALO;
          eps_f = face_eps(P.eps_dx, s_chi[b - TW], s_chi[b]);
        }
        hll_flux<ND, (ND >= 2 ? 1 : 0), TT>(clo, c, ch, chc, cch, Um, Up, fl, eps_f);
#pragma unroll
        for (int r = 0; r < NR; ++r) s_eyR[r][f2] = fl[r];
      }
    }

    if (!(RHD_ZBAL && ND == 3 && tid >= NTHREADS / 2)) zface();
    __syncthreads();

    // ---------------- divergence of the own cell ----------------
    double s[NR];
#pragma unroll
    for (int r = 0; r < NR; ++r) {
      double d = s_exR[r][ty * (TX + 1) + tx + 1] - s_exR[r][ty * (TX + 1) + tx];
      if constexpr (ND >= 2) d += s_eyR[r][(ty + 1) * TX + tx] - s_eyR[r][ty * TX + tx];
      d += divz[r];
      s[r] = -d * P.inv_dx;
    }
    // no barrier here: the next plane is staged into s_area, which nobody has
    // read since the barrier after the edge states; the flux arrays it overwrites
    // next are written only after the staging barrier

    __builtin_amdgcn_s_setprio(0);
    if (!valid) continue;
    const long long q = k * plane + outq;
    if constexpr (MODE == MODE_TRANSPORT) {
#pragma unroll
      for (int r = 0; r < NR; ++r) yw[r * N + q] = s[r];
#pragma unroll
      for (int r = NR; r < 2 + 2 * ND; ++r) yw[r * N + q] = 0.0;
      continue;
    } else {
      // y(t): stage 1 = y^n + dt s(y^n); stage 2 = (y^n + y^{n+1/2})/2 + dt/2 s(y^{n+1/2})
      double E, F[ND], Eg, Pm[ND];
      if constexpr (MODE == MODE_STAGE1) {
        E = own[0] + dt * s[0];
#pragma unroll
        for (int k2 = 0; k2 < ND; ++k2) F[k2] = own[1 + k2] + dt * s[1 + k2];
        Eg = pre[0];
#pragma unroll
        for (int k2 = 0; k2 < ND; ++k2) Pm[k2] = pre[1 + k2];
      } else {
        const double hdt = 0.5 * dt;
        E = 0.5 * (pre[1 + ND] + own[0]) + hdt * s[0];
#pragma unroll
        for (int k2 = 0; k2 < ND; ++k2)
          F[k2] = 0.5 * (pre[2 + ND + k2] + own[1 + k2]) + hdt * s[1 + k2];
        Eg = 0.5 * (pre[2 + 2 * ND] + pre[0]);
#pragma unroll
        for (int k2 = 0; k2 < ND; ++k2) Pm[k2] = 0.5 * (pre[3 + 2 * ND + k2] + pre[1 + k2]);
      }
      // RK2-SSP comparator: transport only in stage 1, the source once at the end
      // of the step with the full dt
      const unsigned st = (MODE == MODE_STAGE1 && P.scheme == 1)
                              ? 0u
                              : source_cell<ND, SV>(P, E, F, Eg, Pm, pre_rho, pre_kp, pre_kf, pre_ke,
                                                    pre_j * tau_src, tau_src, inv_tch);
      if (st) report(err, q, st);
      yw[q] = E;
#pragma unroll
      for (int k2 = 0; k2 < ND; ++k2) yw[(1 + k2) * N + q] = F[k2];
      yw[(1 + ND) * N + q] = Eg;
#pragma unroll
      for (int k2 = 0; k2 < ND; ++k2) yw[(2 + ND + k2) * N + q] = Pm[k2];
    }
  }
}

// ---------------------------------------------------------------------------
// Launcher of k_stage for one dimensionality
// ---------------------------------------------------------------------------
// The leanest source instantiation whose assumptions hold.
inline int source_variant(const DevParams& P) {
  if (P.kT_pow != 0.0) return SRC_TDEP;
  if (P.kE != nullptr || P.jS != nullptr || (P.v_order == 2 && !P.kF_alias)) return SRC_GEN;
  return SRC_LEAN;
}

template <int ND, int MODE, typename TT, int VAR>
static hipError_t launch_nd(const DevParams& P, const double* ys, const double* yo, double* yw,
                            const double* rho, const double* kP, const double* kF, double dt,
                            unsigned long long* err, hipStream_t s) {
  constexpr int TX = TileShape<ND>::TX, TY = TileShape<ND>::TY;
  const int nx = P.n[0], ny = P.n[1], nz = P.n[2];
  const int gxn = (nx + TX - 1) / TX, gyn = (ny + TY - 1) / TY;
  int zchunk = nz;
  if (ND == 3) {
    // Planes per workgroup: long chunks amortise the z-pipeline start and the halo
    // planes, but the workgroups must still fill the chip. RHD_STAGE_SLOTS of them
    // run at once (two per CU: the kernel is VGPR-bound). Take the longest chunk of
    // RHD_ZCHUNK_MAX, half that, ... down to 8 planes whose workgroups fill at least
    // one such round with the last round at least 95 % full; else 8.
    const long long cols = (long long)gxn * gyn;
    zchunk = 8;
    for (int zc = RHD_ZCHUNK_MAX; zc >= 8; zc /= 2) {
      const double rounds = double(cols * ((nz + zc - 1) / zc)) / RHD_STAGE_SLOTS;
      if (rounds >= 1.0 && rounds >= 0.95 * std::ceil(rounds)) {
        zchunk = zc;
        break;
      }
    }
    if (zchunk > nz) zchunk = nz;
  }
  const int gzn = (nz + zchunk - 1) / zchunk;
  hipLaunchKernelGGL((k_stage<ND, MODE, TT, VAR>), dim3(gxn, gyn, gzn), dim3(NTHREADS), 0, s, P, ys,
                     yo, yw, rho, kP, kF, dt, zchunk, err);
  return hipGetLastError();
}

// k_stage of the given mode and precision on an ND-dimensional grid, with the
// leanest kernel variant that applies
template <int ND>
hipError_t launch_stage_nd(const DevParams& P, int mode, bool mixed, const double* ys,
                           const double* yo, double* yw, const double* rho, const double* kP,
                           const double* kF, double dt, unsigned long long* err, hipStream_t s) {
  // the transport-only mode runs no source, so it needs neither VAR_GEN nor
  // VAR_TDEP; the host rejects eps together with T-dependent opacities
  const int sv = (mode == MODE_TRANSPORT) ? SRC_LEAN : source_variant(P);
  const int var = P.eps_dx > 0.0 ? VAR_EPS
                                 : (sv == SRC_TDEP ? VAR_TDEP : (sv == SRC_GEN ? VAR_GEN : VAR_PLAIN));
  auto by_var = [&](auto mode_c, auto tt) -> hipError_t {
    constexpr int MODE = decltype(mode_c)::value;
    using TT = decltype(tt);
    switch (var) {
      case VAR_PLAIN: return launch_nd<ND, MODE, TT, VAR_PLAIN>(P, ys, yo, yw, rho, kP, kF, dt, err, s);
      case VAR_EPS: return launch_nd<ND, MODE, TT, VAR_EPS>(P, ys, yo, yw, rho, kP, kF, dt, err, s);
      case VAR_GEN:
        if constexpr (MODE == MODE_TRANSPORT) return hipErrorInvalidValue;
        else return launch_nd<ND, MODE, TT, VAR_GEN>(P, ys, yo, yw, rho, kP, kF, dt, err, s);
      case VAR_TDEP:
        if constexpr (MODE == MODE_TRANSPORT) return hipErrorInvalidValue;
        else return launch_nd<ND, MODE, TT, VAR_TDEP>(P, ys, yo, yw, rho, kP, kF, dt, err, s);
      default: return hipErrorInvalidValue;
    }
  };
  using S1 = std::integral_constant<int, MODE_STAGE1>;
  using S2 = std::integral_constant<int, MODE_STAGE2>;
  using ST = std::integral_constant<int, MODE_TRANSPORT>;
  if (mixed) {
    switch (mode) {
      case MODE_STAGE1: return by_var(S1{}, float{});
      case MODE_STAGE2: return by_var(S2{}, float{});
      default: return by_var(ST{}, float{});
    }
  }
  switch (mode) {
    case MODE_STAGE1: return by_var(S1{}, double{});
    case MODE_STAGE2: return by_var(S2{}, double{});
    default: return by_var(ST{}, double{});
  }
}

}  // namespace rhd
