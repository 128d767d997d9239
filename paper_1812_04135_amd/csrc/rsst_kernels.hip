// Fused RSST stage kernels for gfx950.
//
// One launch computes one SSP-RK2 stage (Sec. 4.1, items 2-8) for the whole
// grid in a single pass over HBM:
//   stage 1: U1 = Un + dt R(Un)
//   stage 2: Un <- (Un + (U1 + dt R(U1))) / 2, plus the CFL reduction of the
//            new state that gives the next dt (item 1).
// R(U) = MC-limited MUSCL reconstruction of the conservative variables, LLF
// flux with c_tot = |V| + a/xi, flux divergence, Delta P, the per-form
// correction (eq. pvs_dt, App. A) and gravity (App. B).
//
// Work decomposition (x = axis 0, contiguous in memory):
//   * lanes run along x: a workgroup holds whole rows of nx cells spread
//     over nwx = ceil(nx/64) waves, so x needs no halo: neighbours come from
//     the adjacent lane by DPP, from the adjacent wave through a few LDS
//     "seam" slots, and periodic or mirror walls are applied in-row;
//   * 3D: ts rows along y are stacked in the workgroup; y neighbours and
//     y-face states are exchanged through LDS, and the two rows just outside
//     the tile are read from global memory by the edge rows;
//   * the last axis (z in 3D, y in 2D) is marched: each thread keeps three
//     planes of its own column in registers, so every z face is computed
//     once and z needs no exchange at all;
//   * every face state (U +- sigma/2, its pressure, c_tot and normal
//     velocity) is computed once, by the cell that owns it; each face flux
//     is computed once, by the cell above it, and handed to the cell below.
//   * workgroup ids are remapped so that consecutive tiles (which share
//     halo rows) run on the same XCD and share its L2.
#include "rsst_device.h"
#include "rsst_internal.h"

#pragma clang fp contract(off)

namespace rsstk {

// ---------------------------------------------------------------- loads

// Read cell (i, j, k) in kernel axes (x, s, m) as FP64.  j and k may lie up
// to two cells outside the grid: periodic sides wrap, reflecting sides
// mirror (ghost -1-q takes cell q) and flip the normal momentum.  The FP32
// perturbation form adds the FP64 background.
template <int NDIM, typename ST>
__device__ __forceinline__ void load_cell(const StageArgs& A, const ST* __restrict__ p, int i,
                                          int j, int k, double (&u)[NDIM + 2]) {
  constexpr int NV = NDIM + 2;
  const Geometry& G = A.geo;
  bool neg_s = false, neg_m = false;
  if constexpr (NDIM == 3) {
    if (j < 0) {
      if (A.bc_lo[1]) { j = -1 - j; neg_s = true; } else { j += G.ns; }
    } else if (j >= G.ns) {
      if (A.bc_hi[1]) { j = 2 * G.ns - 1 - j; neg_s = true; } else { j -= G.ns; }
    }
  }
  if constexpr (NDIM >= 2) {
    constexpr int am = NDIM - 1;
    if (k < 0) {
      if (A.bc_lo[am]) { k = -1 - k; neg_m = true; } else { k += G.nm; }
    } else if (k >= G.nm) {
      if (A.bc_hi[am]) { k = 2 * G.nm - 1 - k; neg_m = true; } else { k -= G.nm; }
    }
  }
  const long long c = ((long long)k * G.ns + j) * G.nx + i;
#pragma unroll
  for (int v = 0; v < NV; ++v) u[v] = (double)p[v * A.ncell + c];
  if constexpr (sizeof(ST) == 4) {
    int b = 0;
    if (A.bg_axis == 0) b = i;
    else if (A.bg_axis == 1) b = (NDIM == 3) ? j : k;
    else if (A.bg_axis == 2) b = k;
#pragma unroll
    for (int v = 0; v < NV; ++v) u[v] += A.bg[v * A.nbg + b];
  }
  if constexpr (NDIM == 3) { if (neg_s) u[2] = -u[2]; }
  if constexpr (NDIM >= 2) { if (neg_m) u[NDIM] = -u[NDIM]; }
}

template <int NV>
__device__ __forceinline__ void put_face(double* p, int stride, const Face<NV>& s) {
#pragma unroll
  for (int v = 0; v < NV; ++v) p[v * stride] = s.u[v];
  p[NV * stride] = s.P;
  p[(NV + 1) * stride] = s.c;
  p[(NV + 2) * stride] = s.vn;
}

template <int NV>
__device__ __forceinline__ void get_face(const double* p, int stride, Face<NV>& s) {
#pragma unroll
  for (int v = 0; v < NV; ++v) s.u[v] = p[v * stride];
  s.P = p[NV * stride];
  s.c = p[(NV + 1) * stride];
  s.vn = p[(NV + 2) * stride];
}

template <int NV>
__device__ __forceinline__ Face<NV> face_from_left(const Face<NV>& s) {
  Face<NV> r;
#pragma unroll
  for (int v = 0; v < NV; ++v) r.u[v] = from_left(s.u[v]);
  r.P = from_left(s.P);
  r.c = from_left(s.c);
  r.vn = from_left(s.vn);
  return r;
}

// ---------------------------------------------------------------- stage

template <int NDIM, int STAGE, typename ST, int MAXT>
__global__ void __launch_bounds__(MAXT) stage_kernel(const StageArgs A) {
  constexpr int NV = NDIM + 2;
  constexpr int PL = NV + 3;          // face payload: U, P, c_tot, V_normal
  constexpr bool HS = (NDIM == 3);    // stacked y rows
  constexpr bool HM = (NDIM >= 2);    // marched last axis
  constexpr int DM = NDIM - 1;        // physical axis of the march
  const Geometry& G = A.geo;
  const int nwx = G.nwx, nxp = nwx * 64, TS = G.ts;

  extern __shared__ double lds[];
  double* Urow = lds;                                  // [NV][TS][nxp]
  double* Prow = Urow + (HS ? NV * TS * nxp : 0);      // [PL][TS][nxp]
  double* Frow = Prow + (HS ? PL * TS * nxp : 0);      // [NV][TS][nxp]
  double* seamU = Frow + (HS ? NV * TS * nxp : 0);     // [TS][nwx][2][NV]
  double* seamUl = seamU + TS * nwx * 2 * NV;          // [TS][NV]  cell nx-1
  double* seamP = seamUl + TS * NV;                    // [TS][nwx][PL] lane 63
  double* seamPl = seamP + TS * nwx * PL;              // [TS][PL]  cell nx-1
  double* seamF = seamPl + TS * PL;                    // [TS][nwx][NV] lane 0
  double* red = seamF + TS * nwx * NV;                 // [16]

  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const int wx = w % nwx, row = w / nwx;
  const int i_raw = wx * 64 + lane;

  // consecutive tiles on one XCD (dispatch is round-robin over 8 XCDs)
  int L = blockIdx.x;
  const int nblk = gridDim.x;
  if ((nblk & 7) == 0) L = (L & 7) * (nblk >> 3) + (L >> 3);
  const int tile_s = L % G.ntile_s, chunk = L / G.ntile_s;
  const int j0 = tile_s * TS;
  const int ts_eff = HS ? min(TS, G.ns - j0) : 1;
  const bool xin = i_raw < G.nx;
  const bool active = xin && row < ts_eff;
  const int i = xin ? i_raw : G.nx - 1;
  const int j = HS ? j0 + min(row, ts_eff - 1) : 0;
  const int k0 = chunk * G.km;
  const int k1 = min(k0 + G.km, G.nm);
  const bool last_x = (i_raw == G.nx - 1);
  const bool first_row = HS && row == 0;
  const bool last_row = HS && row == ts_eff - 1;
  const bool x_per_lo = A.bc_lo[0] == 0, x_per_hi = A.bc_hi[0] == 0;
  const int row_up = min(row + 1, TS - 1);  // idle rows past the tile read in range

  const Consts K{A.gamma, A.gm1, A.inv_gm1, A.inv_xi, A.f};
  const double g[3] = {A.g[0], A.g[1], A.g[2]};
  const double dt = (A.dt_fixed > 0.0) ? A.dt_fixed : A.scal[kDtCur];
  const ST* __restrict__ uin = (const ST*)A.uin;
  const ST* __restrict__ unp = (const ST*)A.un;
  ST* __restrict__ uout = (ST*)A.uout;

  double q0[NV], q1[NV], q2[NV], sm0[NV], Fm_lo[NV];
  double cmax = 0.0;
  unsigned bad = 0;

  if constexpr (HM) {
    double qa[NV], qb[NV], sa[NV];
    load_cell<NDIM, ST>(A, uin, i, j, k0 - 2, qa);
    load_cell<NDIM, ST>(A, uin, i, j, k0 - 1, qb);
    load_cell<NDIM, ST>(A, uin, i, j, k0, q0);
    load_cell<NDIM, ST>(A, uin, i, j, k0 + 1, q1);
    load_cell<NDIM, ST>(A, uin, i, j, k0 + 2, q2);
#pragma unroll
    for (int v = 0; v < NV; ++v) {
      sa[v] = mc_slope(qb[v] - qa[v], q0[v] - qb[v]);
      sm0[v] = mc_slope(q0[v] - qb[v], q1[v] - q0[v]);
    }
    Face<NV> fl, fr;
    make_face<NDIM, DM>(qb, sa, 1.0, K, fl);
    make_face<NDIM, DM>(q0, sm0, -1.0, K, fr);
    llf<NDIM, DM>(fl, fr, Fm_lo);
  } else {
    load_cell<NDIM, ST>(A, uin, i, 0, 0, q0);
  }

  for (int k = k0; k < k1; ++k) {
    // ---- prefetch: next plane of the march, edge-row halo, step-start state
    double qn[NV], un[NV], h1[NV], h2[NV];
    if constexpr (HM) load_cell<NDIM, ST>(A, uin, i, j, k + 3, qn);
    if constexpr (STAGE == 2) load_cell<NDIM, ST>(A, unp, i, j, k, un);
    if constexpr (HS) {
      if (first_row) {
        load_cell<NDIM, ST>(A, uin, i, j0 - 1, k, h1);
        load_cell<NDIM, ST>(A, uin, i, j0 - 2, k, h2);
      } else if (last_row) {
        load_cell<NDIM, ST>(A, uin, i, j0 + ts_eff, k, h1);
        load_cell<NDIM, ST>(A, uin, i, j0 + ts_eff + 1, k, h2);
      }
    }

    // ---- P1: publish this plane's cell state
    if constexpr (HS) {
#pragma unroll
      for (int v = 0; v < NV; ++v) Urow[(v * TS + row) * nxp + i_raw] = q0[v];
    }
    {
      double* s = seamU + ((row * nwx + wx) * 2) * NV;
      if (lane == 0) {
#pragma unroll
        for (int v = 0; v < NV; ++v) s[v] = q0[v];
      }
      if (lane == 63) {
#pragma unroll
        for (int v = 0; v < NV; ++v) s[NV + v] = q0[v];
      }
      if (last_x) {
#pragma unroll
        for (int v = 0; v < NV; ++v) seamUl[row * NV + v] = q0[v];
      }
    }
    __syncthreads();  // B1

    // ---- P2: slopes and face states along x and y
    Face<NV> fxm, pL, fym;
    double wall_hi;
    double Fy_own[NV];
    {
      double uL[NV], uR[NV], sx[NV];
#pragma unroll
      for (int v = 0; v < NV; ++v) { uL[v] = from_left(q0[v]); uR[v] = from_right(q0[v]); }
      if (lane == 0) {
        if (wx > 0) {
          const double* s = seamU + ((row * nwx + wx - 1) * 2 + 1) * NV;
#pragma unroll
          for (int v = 0; v < NV; ++v) uL[v] = s[v];
        } else if (x_per_lo) {
#pragma unroll
          for (int v = 0; v < NV; ++v) uL[v] = seamUl[row * NV + v];
        } else {
#pragma unroll
          for (int v = 0; v < NV; ++v) uL[v] = q0[v];
          uL[1] = -q0[1];
        }
      }
      if (last_x) {
        if (x_per_hi) {
          const double* s = seamU + ((row * nwx) * 2) * NV;
#pragma unroll
          for (int v = 0; v < NV; ++v) uR[v] = s[v];
        } else {
#pragma unroll
          for (int v = 0; v < NV; ++v) uR[v] = q0[v];
          uR[1] = -q0[1];
        }
      } else if (lane == 63 && xin) {
        const double* s = seamU + ((row * nwx + wx + 1) * 2) * NV;
#pragma unroll
        for (int v = 0; v < NV; ++v) uR[v] = s[v];
      }
#pragma unroll
      for (int v = 0; v < NV; ++v) sx[v] = mc_slope(q0[v] - uL[v], uR[v] - q0[v]);
      Face<NV> fxp;
      make_face<NDIM, 0>(q0, sx, -1.0, K, fxm);
      make_face<NDIM, 0>(q0, sx, 1.0, K, fxp);
      // closed free-slip wall above the last cell: the LLF flux of the state
      // and its mirror image carries only normal momentum m v + P + c m.
      wall_hi = fma(fxp.c, fxp.u[1], fma(fxp.u[1], fxp.vn, fxp.P));
      pL = face_from_left(fxp);
      if (lane == 63) put_face(seamP + (row * nwx + wx) * PL, 1, fxp);
      if (last_x) put_face(seamPl + row * PL, 1, fxp);
    }
    if constexpr (HS) {
      // A one-row tile (ragged end) is both first and last row: its lower
      // halo was prefetched, its upper halo is read here, and its upper flux
      // goes to the idle row's LDS slot.
      double uD[NV], uU[NV], hh1[NV], hh2[NV], sy[NV];
      if (last_row) {
        if (first_row) {
          load_cell<NDIM, ST>(A, uin, i, j0 + 1, k, hh1);
          load_cell<NDIM, ST>(A, uin, i, j0 + 2, k, hh2);
        } else {
#pragma unroll
          for (int v = 0; v < NV; ++v) { hh1[v] = h1[v]; hh2[v] = h2[v]; }
        }
      }
      if (first_row) {
#pragma unroll
        for (int v = 0; v < NV; ++v) uD[v] = h1[v];
      } else {
#pragma unroll
        for (int v = 0; v < NV; ++v) uD[v] = Urow[(v * TS + row - 1) * nxp + i_raw];
      }
      if (last_row) {
#pragma unroll
        for (int v = 0; v < NV; ++v) uU[v] = hh1[v];
      } else {
#pragma unroll
        for (int v = 0; v < NV; ++v) uU[v] = Urow[(v * TS + row_up) * nxp + i_raw];
      }
#pragma unroll
      for (int v = 0; v < NV; ++v) sy[v] = mc_slope(q0[v] - uD[v], uU[v] - q0[v]);
      Face<NV> fyp;
      make_face<NDIM, 1>(q0, sy, -1.0, K, fym);
      make_face<NDIM, 1>(q0, sy, 1.0, K, fyp);
      put_face(Prow + row * nxp + i_raw, TS * nxp, fyp);
      if (first_row) {
        // plus state of the row below the tile, and the flux between
        double sh[NV];
#pragma unroll
        for (int v = 0; v < NV; ++v) sh[v] = mc_slope(h1[v] - h2[v], q0[v] - h1[v]);
        Face<NV> fh;
        make_face<NDIM, 1>(h1, sh, 1.0, K, fh);
        llf<NDIM, 1>(fh, fym, Fy_own);
      }
      if (last_row) {
        // minus state of the row above the tile, and the flux between
        double sh[NV], Fh[NV];
#pragma unroll
        for (int v = 0; v < NV; ++v) sh[v] = mc_slope(hh1[v] - q0[v], hh2[v] - hh1[v]);
        Face<NV> fh;
        make_face<NDIM, 1>(hh1, sh, -1.0, K, fh);
        llf<NDIM, 1>(fyp, fh, Fh);
        if (first_row) {
#pragma unroll
          for (int v = 0; v < NV; ++v) Frow[(v * TS + row + 1) * nxp + i_raw] = Fh[v];
        } else {
#pragma unroll
          for (int v = 0; v < NV; ++v) Fy_own[v] = Fh[v];
        }
      }
    }
    __syncthreads();  // B2

    // ---- P3: fluxes through the lower faces
    double Fx_lo[NV], Fy_lo[NV];
    if (lane == 0) {
      if (wx > 0) get_face(seamP + (row * nwx + wx - 1) * PL, 1, pL);
      else if (x_per_lo) get_face(seamPl + row * PL, 1, pL);
      else pL = mirror<NDIM, 0>(fxm);
    }
    llf<NDIM, 0>(pL, fxm, Fx_lo);
    if (lane == 0) {
#pragma unroll
      for (int v = 0; v < NV; ++v) seamF[(row * nwx + wx) * NV + v] = Fx_lo[v];
    }
    if constexpr (HS) {
      if (first_row) {
#pragma unroll
        for (int v = 0; v < NV; ++v) Fy_lo[v] = Fy_own[v];
      } else {
        Face<NV> pD;
        get_face(Prow + (row - 1) * nxp + i_raw, TS * nxp, pD);
        llf<NDIM, 1>(pD, fym, Fy_lo);
      }
      if (row < ts_eff) {
#pragma unroll
        for (int v = 0; v < NV; ++v) Frow[(v * TS + row) * nxp + i_raw] = Fy_lo[v];
      }
    }
    __syncthreads();  // B3

    // ---- P4: upper faces, march face, divergence, correction, update
    double Dl[NV];
    {
      double Fx_hi[NV];
#pragma unroll
      for (int v = 0; v < NV; ++v) Fx_hi[v] = from_right(Fx_lo[v]);
      if (last_x) {
        if (x_per_hi) {
#pragma unroll
          for (int v = 0; v < NV; ++v) Fx_hi[v] = seamF[(row * nwx) * NV + v];
        } else {
#pragma unroll
          for (int v = 0; v < NV; ++v) Fx_hi[v] = 0.0;
          Fx_hi[1] = wall_hi;
        }
      } else if (lane == 63 && xin) {
#pragma unroll
        for (int v = 0; v < NV; ++v) Fx_hi[v] = seamF[(row * nwx + wx + 1) * NV + v];
      }
#pragma unroll
      for (int v = 0; v < NV; ++v) Dl[v] = -(Fx_hi[v] - Fx_lo[v]) * A.inv_dx[0];
    }
    if constexpr (HS) {
      double Fy_hi[NV];
      if (last_row && !first_row) {
#pragma unroll
        for (int v = 0; v < NV; ++v) Fy_hi[v] = Fy_own[v];
      } else {
#pragma unroll
        for (int v = 0; v < NV; ++v) Fy_hi[v] = Frow[(v * TS + row_up) * nxp + i_raw];
      }
#pragma unroll
      for (int v = 0; v < NV; ++v) Dl[v] = fma(-(Fy_hi[v] - Fy_lo[v]), A.inv_dx[1], Dl[v]);
    }
    if constexpr (HM) {
      double sm1[NV], Fm_hi[NV];
#pragma unroll
      for (int v = 0; v < NV; ++v) sm1[v] = mc_slope(q1[v] - q0[v], q2[v] - q1[v]);
      Face<NV> fl, fr;
      make_face<NDIM, DM>(q0, sm0, 1.0, K, fl);
      make_face<NDIM, DM>(q1, sm1, -1.0, K, fr);
      llf<NDIM, DM>(fl, fr, Fm_hi);
#pragma unroll
      for (int v = 0; v < NV; ++v) {
        Dl[v] = fma(-(Fm_hi[v] - Fm_lo[v]), A.inv_dx[DM], Dl[v]);
        Fm_lo[v] = Fm_hi[v];
        sm0[v] = sm1[v];
      }
    }
    double R[NV];
    const unsigned b = rsst_rate<NDIM>(q0, Dl, K, A.form, g, R);
    if (active) {
      bad |= b;
      const long long c = ((long long)k * G.ns + j) * G.nx + i;
      double bgv[NV];
#pragma unroll
      for (int v = 0; v < NV; ++v) bgv[v] = 0.0;
      if constexpr (sizeof(ST) == 4) {
        int bb = 0;
        if (A.bg_axis == 0) bb = i;
        else if (A.bg_axis == 1) bb = (NDIM == 3) ? j : k;
        else if (A.bg_axis == 2) bb = k;
#pragma unroll
        for (int v = 0; v < NV; ++v) bgv[v] = A.bg[v * A.nbg + bb];
      }
      double out[NV];
#pragma unroll
      for (int v = 0; v < NV; ++v) {
        double y = fma(dt, R[v], q0[v]);
        if constexpr (STAGE == 2) y = 0.5 * (un[v] + y);
        const ST st = (ST)(y - bgv[v]);
        uout[v * A.ncell + c] = st;
        out[v] = (double)st + bgv[v];
      }
      if constexpr (STAGE == 2) cmax = fmax(cmax, cell_ctot<NDIM>(out, K));
    }
    if constexpr (HM) {
#pragma unroll
      for (int v = 0; v < NV; ++v) { q0[v] = q1[v]; q1[v] = q2[v]; q2[v] = qn[v]; }
    }
  }

  if (bad) atomicOr((unsigned*)(A.scal + kFlags), bad);

  if constexpr (STAGE == 2) {
    // workgroup maximum of c_tot, then one atomic per workgroup; the last
    // workgroup to finish advances t and sets the next CFL dt
    const double wm = wave_max(cmax);
    if (lane == 0) red[w] = wm;
    __syncthreads();
    if (tid == 0) {
      double m = 0.0;
      for (int q = 0; q < (int)(blockDim.x >> 6); ++q) m = fmax(m, red[q]);
      unsigned long long* mb = (unsigned long long*)(A.scal + kMaxBits);
      unsigned long long* done = (unsigned long long*)(A.scal + kDone);
      atomicMax(mb, (unsigned long long)__double_as_longlong(m));
      __threadfence();
      const unsigned long long prev = atomicAdd(done, 1ull);
      if (prev == (unsigned long long)(gridDim.x - 1)) {
        __threadfence();
        const double cm = __longlong_as_double((long long)atomicAdd(mb, 0ull));
        const double t = A.scal[kTime] + dt;
        double dn = dt;
        if (A.dt_fixed <= 0.0) {
          dn = A.cfl_h / cm;
          if (A.t_end > 0.0) dn = fmin(dn, fmax(A.t_end - t, 0.0));
        }
        A.scal[kTime] = t;
        A.scal[kDtCur] = dn;
        atomicExch(mb, 0ull);
        atomicExch(done, 0ull);
      }
    }
  }
}

// ---------------------------------------------------------------- prime

// CFL time step of a state: dt = cfl * h / max c_tot; also sets t = t0.
template <int NDIM, typename ST>
__global__ void __launch_bounds__(256) prime_kernel(const StageArgs A, const ST* __restrict__ u,
                                                    double t0, int set_t) {
  constexpr int NV = NDIM + 2;
  const Consts K{A.gamma, A.gm1, A.inv_gm1, A.inv_xi, A.f};
  const Geometry& G = A.geo;
  __shared__ double red[4];
  double cm = 0.0;
  unsigned bad = 0;
  for (long long c = (long long)blockIdx.x * blockDim.x + threadIdx.x; c < A.ncell;
       c += (long long)gridDim.x * blockDim.x) {
    double q[NV];
    const int i = (int)(c % G.nx);
    const long long r = c / G.nx;
    const int j = (int)(r % G.ns);
    const int k = (int)(r / G.ns);
#pragma unroll
    for (int v = 0; v < NV; ++v) q[v] = (double)u[v * A.ncell + c];
    if constexpr (sizeof(ST) == 4) {
      int b = 0;
      if (A.bg_axis == 0) b = i;
      else if (A.bg_axis == 1) b = (NDIM == 3) ? j : k;
      else if (A.bg_axis == 2) b = k;
#pragma unroll
      for (int v = 0; v < NV; ++v) q[v] += A.bg[v * A.nbg + b];
    }
    const double ct = cell_ctot<NDIM>(q, K);
    if (!(q[0] > 0.0)) bad |= kBadRho;
    if (!(ct < INFINITY)) bad |= kNonFinite;
    cm = fmax(cm, ct);
  }
  if (bad) atomicOr((unsigned*)(A.scal + kFlags), bad);
  const double wm = wave_max(cm);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = wm;
  __syncthreads();
  if (threadIdx.x == 0) {
    const double m = fmax(fmax(red[0], red[1]), fmax(red[2], red[3]));
    unsigned long long* mb = (unsigned long long*)(A.scal + kMaxBits);
    unsigned long long* done = (unsigned long long*)(A.scal + kDone);
    atomicMax(mb, (unsigned long long)__double_as_longlong(m));
    __threadfence();
    const unsigned long long prev = atomicAdd(done, 1ull);
    if (prev == (unsigned long long)(gridDim.x - 1)) {
      __threadfence();
      const double cmx = __longlong_as_double((long long)atomicAdd(mb, 0ull));
      const double t = set_t ? t0 : A.scal[kTime];
      double dn = A.cfl_h / cmx;
      if (A.t_end > 0.0) dn = fmin(dn, fmax(A.t_end - t, 0.0));
      A.scal[kTime] = t;
      A.scal[kDtCur] = dn;
      atomicExch(mb, 0ull);
      atomicExch(done, 0ull);
    }
  }
}

// ---------------------------------------------------------------- diag

constexpr int kDiagThreads = 256;
constexpr int kDiagBlocks = 1024;

// Per-block partial sums (fixed order: strided per thread, tree per block).
template <int NDIM, typename ST>
__global__ void __launch_bounds__(kDiagThreads) diag_partial_kernel(const StageArgs A,
                                                                    const ST* __restrict__ u,
                                                                    double* __restrict__ part) {
  constexpr int NV = NDIM + 2;
  const Consts K{A.gamma, A.gm1, A.inv_gm1, A.inv_xi, A.f};
  const Geometry& G = A.geo;
  __shared__ double s[8][kDiagThreads];
  double acc[8] = {0, 0, 0, 0, 0, 0, 0, 0};
  for (long long c = (long long)blockIdx.x * blockDim.x + threadIdx.x; c < A.ncell;
       c += (long long)gridDim.x * blockDim.x) {
    double q[NV];
    const int i = (int)(c % G.nx);
    const long long r = c / G.nx;
    const int j = (int)(r % G.ns);
    const int k = (int)(r / G.ns);
#pragma unroll
    for (int v = 0; v < NV; ++v) q[v] = (double)u[v * A.ncell + c];
    if constexpr (sizeof(ST) == 4) {
      int b = 0;
      if (A.bg_axis == 0) b = i;
      else if (A.bg_axis == 1) b = (NDIM == 3) ? j : k;
      else if (A.bg_axis == 2) b = k;
#pragma unroll
      for (int v = 0; v < NV; ++v) q[v] += A.bg[v * A.nbg + b];
    }
    const double rinv = 1.0 / q[0];
    double m2 = 0.0, mv = 0.0;
    acc[0] += q[0];
#pragma unroll
    for (int e = 0; e < NDIM; ++e) {
      acc[1 + e] += q[1 + e];
      m2 = fma(q[1 + e], q[1 + e], m2);
    }
    acc[4] += q[NV - 1];
    acc[5] += 0.5 * m2 * rinv;
    mv = m2 * rinv;
    const double v = sqrt(m2) * rinv;
    const double P = K.gm1 * (q[NV - 1] - 0.5 * mv);
    const double a = sqrt(K.gamma * P * rinv);
    acc[6] = fmax(acc[6], v);
    acc[7] = fmax(acc[7], v / (a * A.inv_xi));
  }
#pragma unroll
  for (int q = 0; q < 8; ++q) s[q][threadIdx.x] = acc[q];
  __syncthreads();
  for (int h = kDiagThreads / 2; h > 0; h >>= 1) {
    if ((int)threadIdx.x < h) {
#pragma unroll
      for (int q = 0; q < 6; ++q) s[q][threadIdx.x] += s[q][threadIdx.x + h];
      s[6][threadIdx.x] = fmax(s[6][threadIdx.x], s[6][threadIdx.x + h]);
      s[7][threadIdx.x] = fmax(s[7][threadIdx.x], s[7][threadIdx.x + h]);
    }
    __syncthreads();
  }
  if (threadIdx.x < 8) part[blockIdx.x * 8 + threadIdx.x] = s[threadIdx.x][0];
}

__global__ void __launch_bounds__(kDiagThreads) diag_final_kernel(const double* __restrict__ part,
                                                                  int np, double vol,
                                                                  double* __restrict__ out) {
  __shared__ double s[8][kDiagThreads];
  double acc[8] = {0, 0, 0, 0, 0, 0, 0, 0};
  for (int b = threadIdx.x; b < np; b += blockDim.x) {
#pragma unroll
    for (int q = 0; q < 6; ++q) acc[q] += part[b * 8 + q];
    acc[6] = fmax(acc[6], part[b * 8 + 6]);
    acc[7] = fmax(acc[7], part[b * 8 + 7]);
  }
#pragma unroll
  for (int q = 0; q < 8; ++q) s[q][threadIdx.x] = acc[q];
  __syncthreads();
  for (int h = kDiagThreads / 2; h > 0; h >>= 1) {
    if ((int)threadIdx.x < h) {
#pragma unroll
      for (int q = 0; q < 6; ++q) s[q][threadIdx.x] += s[q][threadIdx.x + h];
      s[6][threadIdx.x] = fmax(s[6][threadIdx.x], s[6][threadIdx.x + h]);
      s[7][threadIdx.x] = fmax(s[7][threadIdx.x], s[7][threadIdx.x + h]);
    }
    __syncthreads();
  }
  if (threadIdx.x < 8) out[threadIdx.x] = s[threadIdx.x][0] * (threadIdx.x < 6 ? vol : 1.0);
}

// ---------------------------------------------------------------- host side

// 3D workgroups stay at 512 threads so the march state fits in registers.
constexpr int kMaxThreads3D = 512;

Geometry plan_geometry(int ndim, const int n[3]) {
  Geometry G{};
  G.ndim = ndim;
  G.nx = n[0];
  G.ns = (ndim == 3) ? n[1] : 1;
  G.nm = (ndim == 3) ? n[2] : (ndim == 2 ? n[1] : 1);
  G.nwx = (G.nx + 63) / 64;
  if (ndim == 3) {
    int ts = kMaxThreads3D / (64 * G.nwx);
    if (ts > G.ns) ts = G.ns;
    // prefer tilings without a one-row tile (it reads its upper halo late)
    while (ts > 2 && G.ns % ts == 1) --ts;
    G.ts = ts;
  } else {
    G.ts = 1;
  }
  G.ntile_s = (G.ns + G.ts - 1) / G.ts;
  if (ndim == 1) {
    G.km = 1;
  } else {
    // enough workgroups to fill 256 CUs, chunks no shorter than 8 planes
    int km = 32;
    while (km > 8 && (long long)G.ntile_s * ((G.nm + km - 1) / km) < 1024) km >>= 1;
    G.km = km < G.nm ? km : G.nm;
  }
  G.nchunk = (G.nm + G.km - 1) / G.km;
  G.threads = 64 * G.nwx * G.ts;
  const int NV = ndim + 2, PL = NV + 3, nxp = 64 * G.nwx;
  size_t d = 0;
  if (ndim == 3) d += (size_t)(NV + PL + NV) * G.ts * nxp;
  d += (size_t)G.ts * G.nwx * 2 * NV + G.ts * NV + G.ts * G.nwx * PL + G.ts * PL +
       G.ts * G.nwx * NV + 16;
  G.lds_bytes = d * sizeof(double);
  return G;
}

template <int NDIM, int STAGE, typename ST>
static hipError_t launch_stage_t(const StageArgs& a, hipStream_t s) {
  const Geometry& G = a.geo;
  const dim3 grid((unsigned)(G.ntile_s * G.nchunk)), block((unsigned)G.threads);
  auto kern = stage_kernel<NDIM, STAGE, ST, NDIM == 3 ? kMaxThreads3D : 1024>;
  hipError_t e = hipFuncSetAttribute((const void*)kern, hipFuncAttributeMaxDynamicSharedMemorySize,
                                     (int)G.lds_bytes);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(kern, grid, block, G.lds_bytes, s, a);
  return hipGetLastError();
}

template <int NDIM, typename ST>
static hipError_t launch_stage_n(const StageArgs& a, int stage, hipStream_t s) {
  return stage == 1 ? launch_stage_t<NDIM, 1, ST>(a, s) : launch_stage_t<NDIM, 2, ST>(a, s);
}

template <typename ST>
static hipError_t launch_stage_p(const StageArgs& a, int stage, hipStream_t s) {
  switch (a.geo.ndim) {
    case 1: return launch_stage_n<1, ST>(a, stage, s);
    case 2: return launch_stage_n<2, ST>(a, stage, s);
    default: return launch_stage_n<3, ST>(a, stage, s);
  }
}

hipError_t launch_stage(const StageArgs& a, int stage, hipStream_t s) {
  return a.prec ? launch_stage_p<float>(a, stage, s) : launch_stage_p<double>(a, stage, s);
}

template <typename ST>
static hipError_t launch_prime_p(const StageArgs& a, const void* u, double t0, int set_t,
                                 hipStream_t s) {
  long long nb = (a.ncell + 255) / 256;
  if (nb > 2048) nb = 2048;
  const dim3 grid((unsigned)nb), block(256);
  switch (a.geo.ndim) {
    case 1: hipLaunchKernelGGL((prime_kernel<1, ST>), grid, block, 0, s, a, (const ST*)u, t0, set_t); break;
    case 2: hipLaunchKernelGGL((prime_kernel<2, ST>), grid, block, 0, s, a, (const ST*)u, t0, set_t); break;
    default: hipLaunchKernelGGL((prime_kernel<3, ST>), grid, block, 0, s, a, (const ST*)u, t0, set_t); break;
  }
  return hipGetLastError();
}

hipError_t launch_prime(const StageArgs& a, const void* u, double t0, int set_t, hipStream_t s) {
  return a.prec ? launch_prime_p<float>(a, u, t0, set_t, s)
                : launch_prime_p<double>(a, u, t0, set_t, s);
}

int diag_partials(long long ncell) {
  long long nb = (ncell + kDiagThreads - 1) / kDiagThreads;
  return (int)(nb < kDiagBlocks ? nb : kDiagBlocks);
}

template <typename ST>
static hipError_t launch_diag_p(const StageArgs& a, const void* u, double* part, int np,
                                double* out8, hipStream_t s) {
  const dim3 grid((unsigned)np), block(kDiagThreads);
  switch (a.geo.ndim) {
    case 1: hipLaunchKernelGGL((diag_partial_kernel<1, ST>), grid, block, 0, s, a, (const ST*)u, part); break;
    case 2: hipLaunchKernelGGL((diag_partial_kernel<2, ST>), grid, block, 0, s, a, (const ST*)u, part); break;
    default: hipLaunchKernelGGL((diag_partial_kernel<3, ST>), grid, block, 0, s, a, (const ST*)u, part); break;
  }
  double vol = 1.0;
  for (int d = 0; d < a.geo.ndim; ++d) vol /= a.inv_dx[d];
  hipLaunchKernelGGL(diag_final_kernel, dim3(1), dim3(kDiagThreads), 0, s, part, np, vol, out8);
  return hipGetLastError();
}

hipError_t launch_diag(const StageArgs& a, const void* u, double* part, int np, double* out8,
                       hipStream_t s) {
  return a.prec ? launch_diag_p<float>(a, u, part, np, out8, s)
                : launch_diag_p<double>(a, u, part, np, out8, s);
}

}  // namespace rsstk
