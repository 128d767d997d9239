// Device code of one RSST stage over 2D strips, shared by the per-grid 2D
// kernels and the batched persistent kernel.
//
// A workgroup holds ts x rows of nx cells (nwx waves each); row r of the
// workgroup marches y over its own chunk of planes (chunk_base + r).  x
// neighbours and x plus-face states are exchanged through LDS rows with one
// ghost slot at each end (periodic wrap or mirror), and every x face flux is
// formed once, by the cell right of the face, and handed to the cell on its
// left after a third barrier (by DPP within a wave, one LDS seam value per
// wave edge).  y is marched: every y face is formed once and carried to the
// next plane.
#pragma once

#include "rsst_stage.h"

#pragma clang fp contract(off)

namespace rsstk {

// LDS carve-up of a 2D workgroup (doubles): ts rows of nwx waves.
struct Carve2 {
  int u, fp, fxs, red, total;
};

__host__ __device__ inline Carve2 carve2(int ts, int nwx) {
  constexpr int NV = 4, PL = NV + 3;
  const int px = 64 * nwx + 2;
  Carve2 c;
  int o = 0;
  c.u = o;   o += ts * NV * px;   // cell states [row][value][slot], slot 1 + i; 0, nx + 1: x ghosts
  c.fp = o;  o += ts * PL * px;   // x plus-face states, slot 1 + i; slot 0: the left ghost's
  c.fxs = o; o += ts * NV * nwx;  // x flux at the left edge of each wave
  c.red = o; o += 16;
  c.total = o;
  return c;
}

// One stage of R over one group of 2D strips (row r of the workgroup marches
// chunk chunk_base + r), returning the thread's largest c_tot of the stage-2
// output (0 in stage 1) and or-ing non-physical flags into `bad`.  Every row
// of the workgroup runs the same number of march iterations (G.km), so rows
// of different chunks share the workgroup's barriers.
template <int STAGE, typename ST, int FORMX>
__device__ __forceinline__ double stage_body2(const StageArgs& A, double* lds, int chunk_base, double dt,
                                              unsigned& bad) {
  constexpr int NDIM = 2, NV = 4, PL = NV + 3;
  constexpr int FORM = FORMX & 7;
  constexpr int EXT = FORMX & (kExtCmax | kExtVdw);
  constexpr bool HYD = (FORMX & kExtHydro) != 0;
  constexpr bool F32 = sizeof(ST) == 4;
  constexpr int SZ = (int)sizeof(ST);
  const Geometry& G = A.geo;
  const int TS = G.ts, nwx = G.nwx;
  const int PX = 64 * nwx + 2;
  const Carve2 C = carve2(TS, nwx);

  const int tid = threadIdx.x, lane = tid & 63;
  const int w = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int wx = w % nwx, row_raw = w / nwx;
  // waves past the last full row (a row of 3 waves in a 4-wave workgroup)
  // only take part in the barriers
  const bool wave_idle = w >= nwx * TS;
  const int row = wave_idle ? 0 : row_raw;
  const int i_raw = wx * 64 + lane;
  const bool xin = i_raw < G.nx;
  const int i = xin ? i_raw : G.nx - 1;
  const int chunk = chunk_base + row;
  const int k0 = chunk * G.km, k1 = min(k0 + G.km, G.nm);
  const bool active = xin && k0 < G.nm && !wave_idle;
  const bool pub = xin && !wave_idle;  // writes this thread's LDS slots
  const bool last_x = i_raw == G.nx - 1 && !wave_idle;
  const bool first_x = i_raw == 0 && !wave_idle;
  const bool x_per = A.bc_lo[0] == 0;
  const int rm_lo = A.bc_lo[1], rm_hi = A.bc_hi[1];
  const int plane = G.nx * SZ;  // bytes per y row
  const int col = i * SZ;

  // the thread's LDS addresses: its cell slot minus one (its left neighbour),
  // its plus-face slot minus one, and its wave's x seam
  double* const Urow = lds + C.u + row * (NV * PX);
  double* const Frow = lds + C.fp + row * (PL * PX);
  double* const ub = Urow + i;                           // + v PX + {0, 1, 2}: left, own, right
  double* const fb = Frow + i;                           // + q PX + {0, 1}: left neighbour's, own
  double* const xs = lds + C.fxs + row * (NV * nwx) + wx;  // + v nwx

  // FP32 perturbation form: the background in registers, along y (the
  // march axis: bgA plane k, bgB plane k + 2, loaded per plane) or fixed
  // for the march (uniform, along x)
  const bool bg_on_m = F32 && A.bg_axis == 1;
  double bgA[NV], bgB[NV];
  const __amdgpu_buffer_rsrc_t bgr = field_rsrc(A.bg, F32 ? (long long)NV * A.nbg * 8 : 0);
  if constexpr (F32) {
    if (!bg_on_m) load_bg<NV>(bgr, A.nbg, A.bg_axis == 0 ? i : 0, bgA);
  }
  // FP64 state of stored values: FP32 with the background bz; FP64 with the
  // mirror sign and a hydrostatic wall's carried pressure (lever)
  auto fin = [&](const ST (&raw)[NV], int neg, const double (&bz)[NV], double lev, double (&u)[NV]) {
    if constexpr (F32) finish_cell_bgv<NDIM, ST>(raw, neg, bz, u);
    else finish_cell<NDIM, ST>(A, raw, neg, 0, u, lev);
  };

  const Consts K{A.gamma, A.gm1, A.inv_gm1, A.inv_xi, A.f, A.inv_cmax2, A.vdw_a, A.vdw_b};
  const double g[3] = {A.g[0], A.g[1], A.g[2]};
  const double hx = 0.5 * A.inv_dx[0], hy = 0.5 * A.inv_dx[1];
  const Field32 uin = make_field<false>(A.uin, A.ncell, NV, SZ, plane);
  const Field32 unp = make_field<false>(A.un ? A.un : A.uin, A.ncell, NV, SZ, plane);
  // stage 2 writes the new state in place over the step-start state
  const Field32 uout = STAGE == 2 ? unp : make_field<false>(A.uout, A.ncell, NV, SZ, plane);

  double q0[NV], q1[NV], sm0[NV], Fm_lo[NV];
  double cmax = 0.0;
  const int k0l = min(k0, G.nm - 1);  // rows past the grid march in range
  {
    double qa[NV], qb[NV], ha[NV];
    auto ld = [&](int q, double (&u)[NV]) {  // row k0l + q of the thread's column, through the y walls
      bool n;
      const int kk = map_index(k0l + q, G.nm, rm_lo, rm_hi, n);
      ST raw[NV];
      load_cell_raw<NDIM, ST>(uin, kk, col, raw);
      double bz[NV];
      if constexpr (F32) {
        if (bg_on_m) load_bg<NV>(bgr, A.nbg, kk, bz);
        else {
#pragma unroll
          for (int v = 0; v < NV; ++v) bz[v] = bgA[v];
        }
      }
      fin(raw, n ? NDIM : -1, bz, HYD ? hydro_lever(k0l + q, G.nm, rm_lo, rm_hi, A.dx[1], A.g[1]) : 0.0, u);
    };
    ld(-2, qa);
    ld(-1, qb);
    ld(0, q0);
    ld(1, q1);
#pragma unroll
    for (int v = 0; v < NV; ++v) {
      ha[v] = mc_half(qb[v] - qa[v], q0[v] - qb[v]);
      sm0[v] = mc_half(q0[v] - qb[v], q1[v] - q0[v]);
    }
    Face<NV> fl, fr;
    make_face<NDIM, 1, EXT>(qb, ha, true, K, fl);
    make_face<NDIM, 1, EXT>(q0, sm0, false, K, fr);
    flux2<NDIM, 1>(fl, fr, Fm_lo);
  }

  for (int it = 0; it < G.km; ++it) {
    const int kraw = k0 + it;
    const bool kval = kraw < k1;
    const int k = min(kraw, G.nm - 1);  // row used for loads and stores
    // ---- loads for this plane: the row two ahead and the step-start state
    // (stored values now, finished where first used)
    ST q2r[NV], unr[NV];
    bool q2n;
    const int q2k = map_index(k + 2, G.nm, rm_lo, rm_hi, q2n);
    const double q2lev = HYD ? hydro_lever(k + 2, G.nm, rm_lo, rm_hi, A.dx[1], A.g[1]) : 0.0;
    if constexpr (F32) {
      if (bg_on_m) {
        load_bg<NV>(bgr, A.nbg, k, bgA);
        load_bg<NV>(bgr, A.nbg, q2k, bgB);
      }
    }
    load_cell_raw<NDIM, ST>(uin, q2k, col, q2r);
    if constexpr (STAGE == 2) load_cell_raw<NDIM, ST>(unp, k, col, unr);

    // ---- P1: publish the cell state, and the x ghosts
    if (pub) {
#pragma unroll
      for (int v = 0; v < NV; ++v) ub[v * PX + 1] = q0[v];
    }
    if (first_x || last_x) {
      // cell 0: periodic, the ghost right of the last cell; wall, the mirror
      // left of cell 0.  The last cell: periodic, the ghost left of cell 0;
      // wall, the mirror right of the last cell.
      double* ur = Urow + (first_x == x_per ? G.nx + 1 : 0);
#pragma unroll
      for (int v = 0; v < NV; ++v) ur[v * PX] = (v == 1 && !x_per) ? -q0[v] : q0[v];
    }
    __syncthreads();  // B1

    // ---- P2: the x slope and the plus-face state (published)
    double h[NV];
#pragma unroll
    for (int v = 0; v < NV; ++v) h[v] = mc_half(q0[v] - ub[v * PX], ub[v * PX + 2] - q0[v]);
    {
      Face<NV> fp;
      make_face<NDIM, 0, EXT>(q0, h, true, K, fp);
      if (pub) put_face(fb + 1, PX, fp);
      if (x_per && last_x) put_face(Frow, PX, fp);  // the periodic ghost left of cell 0
    }
    __syncthreads();  // B2

    // ---- P3: the x flux at the cell's left face, published at wave edges
    double Fx_lo[NV];
    {
      Face<NV> fm, pl;
      make_face<NDIM, 0, EXT>(q0, h, false, K, fm);
      get_face(fb, PX, pl);  // slot i: the plus face of cell i - 1
      if (!x_per) {
        if (first_x) pl = mirror<NDIM, 0>(fm);
      }
      flux2<NDIM, 0>(pl, fm, Fx_lo);
      if (lane == 0 && !wave_idle) {
#pragma unroll
        for (int v = 0; v < NV; ++v) xs[v * nwx] = Fx_lo[v];
      }
    }
    __syncthreads();  // B3

    // ---- P4: the flux at the cell's right face, the y direction, then the
    // rate, the RK update and the store
    double Dl[NV];
    {
      double Fx_hi[NV];
#pragma unroll
      for (int v = 0; v < NV; ++v) Fx_hi[v] = from_right(Fx_lo[v]);
      if (last_x) {
        if (x_per) {
#pragma unroll
          for (int v = 0; v < NV; ++v) Fx_hi[v] = xs[v * nwx - wx];
        } else {
          Face<NV> fp;
          get_face(fb + 1, PX, fp);
          flux2<NDIM, 0>(fp, mirror<NDIM, 0>(fp), Fx_hi);
        }
      } else if (lane == 63 && xin && !wave_idle) {
#pragma unroll
        for (int v = 0; v < NV; ++v) Fx_hi[v] = xs[v * nwx + 1];
      }
#pragma unroll
      for (int v = 0; v < NV; ++v) Dl[v] = -(Fx_hi[v] - Fx_lo[v]) * hx;
    }
    double q2[NV];
    if (F32 && bg_on_m) fin(q2r, q2n ? NDIM : -1, bgB, 0.0, q2);
    else fin(q2r, q2n ? NDIM : -1, bgA, q2lev, q2);
    {
      double sm1[NV], Fm_hi[NV];
#pragma unroll
      for (int v = 0; v < NV; ++v) sm1[v] = mc_half(q1[v] - q0[v], q2[v] - q1[v]);
      Face<NV> fl, fr;
      make_face<NDIM, 1, EXT>(q0, sm0, true, K, fl);
      make_face<NDIM, 1, EXT>(q1, sm1, false, K, fr);
      flux2<NDIM, 1>(fl, fr, Fm_hi);
#pragma unroll
      for (int v = 0; v < NV; ++v) {
        Dl[v] = fma(-(Fm_hi[v] - Fm_lo[v]), hy, Dl[v]);
        Fm_lo[v] = Fm_hi[v];
        sm0[v] = sm1[v];
      }
    }
    double Rt[NV];
    const unsigned b = rsst_rate<NDIM, FORM, EXT>(q0, Dl, K, g, Rt);
    double un[NV];
    if constexpr (STAGE == 2) fin(unr, -1, bgA, 0.0, un);
    if (active && kval) {
      bad |= b;
      double out[NV];
#pragma unroll
      for (int v = 0; v < NV; ++v) {
        double y = fma(dt, Rt[v], q0[v]);
        if constexpr (STAGE == 2) y = 0.5 * (un[v] + y);
        double bgv = 0.0;
        if constexpr (F32) bgv = bgA[v];
        const ST st = (ST)(y - bgv);
        buf_store<ST>(uout.r, col, uout.soff(v, k), st);
        out[v] = (double)st + bgv;
      }
      if constexpr (STAGE == 2) cmax = fmax(cmax, cell_ctot<NDIM, EXT>(out, K));
    }
#pragma unroll
    for (int v = 0; v < NV; ++v) { q0[v] = q1[v]; q1[v] = q2[v]; }
  }
  return cmax;
}

}  // namespace rsstk
