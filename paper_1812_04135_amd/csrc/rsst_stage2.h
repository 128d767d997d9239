// Device code of one RSST stage over 2D strips, shared by the per-grid 2D
// kernels and the batched persistent kernel.
//
// A workgroup holds ts x rows of nx cells (nwx waves each); row r of the
// workgroup marches y over its own chunk of planes (chunk_base + r), NP
// planes per iteration, so each thread has NP independent cells to
// interleave and the barriers are shared by NP planes.  x neighbours and x
// plus-face states are exchanged through LDS rows with one ghost slot at
// each end (periodic wrap or mirror), and every x face flux is formed once,
// by the cell right of the face, and handed to the cell on its left after a
// third barrier (by DPP within a wave, one LDS seam value per wave edge).
// y is marched: every y face is formed once and carried to the next plane.
#pragma once

#include "rsst_stage.h"

#pragma clang fp contract(off)

namespace rsstk {

// LDS carve-up of a 2D workgroup (doubles): ts rows of nwx waves, np planes
// per iteration.
struct Carve2 {
  int u, fp, fxs, red, total;
};

__host__ __device__ inline Carve2 carve2(int ts, int nwx, int np) {
  constexpr int NV = 4, PL = NV + 3;
  const int px = 64 * nwx + 2, rows = ts * np;
  Carve2 c;
  int o = 0;
  c.u = o;   o += rows * NV * px;   // cell states [row][plane][value][slot], slot 1 + i; 0, nx + 1: ghosts
  c.fp = o;  o += rows * PL * px;   // x plus-face states, slot 1 + i; slot 0: the left ghost's
  c.fxs = o; o += rows * NV * nwx;  // x flux at the left edge of each wave
  c.red = o; o += 16;
  c.total = o;
  return c;
}

// One stage of R over one group of 2D strips (row r of the workgroup marches
// chunk chunk_base + r, NP planes per iteration), returning the thread's
// largest c_tot of the stage-2 output (0 in stage 1) and or-ing
// non-physical flags into `bad`.  Every row of the workgroup runs the same
// number of march iterations, so rows of different chunks share the
// workgroup's barriers; planes past a chunk's end are computed on rows held
// in range and not stored.
template <int STAGE, typename ST, int FORMX, int NP>
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
  const Carve2 C = carve2(TS, nwx, NP);

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

  // the thread's LDS addresses: for plane p of the iteration (at + p UR,
  // + p FR, + p NV nwx), its cell slot minus one (its left neighbour), its
  // plus-face slot minus one, and its wave's x seam
  const int UR = NV * PX, FR = PL * PX;
  double* const Urow = lds + C.u + row * NP * UR;
  double* const Frow = lds + C.fp + row * NP * FR;
  double* const ub = Urow + i;                                 // + p UR + v PX + {0, 1, 2}
  double* const fb = Frow + i;                                 // + p FR + q PX + {0, 1}
  double* const xs = lds + C.fxs + row * NP * (NV * nwx) + wx;  // + (p NV + v) nwx

  // FP32 perturbation form: the background in registers, along y (the march
  // axis: bgc[p] for plane k + p of the iteration, bgn[p] for the planes the
  // iteration loads, k + 2 + p) or fixed for the march (uniform, along x:
  // bgc[0])
  const bool bg_on_m = F32 && A.bg_axis == 1;
  double bgc[NP][NV], bgn[NP][NV];
  const __amdgpu_buffer_rsrc_t bgr = field_rsrc(A.bg, F32 ? (long long)NV * A.nbg * 8 : 0);
  if constexpr (F32) {
    if (!bg_on_m) load_bg<NV>(bgr, A.nbg, A.bg_axis == 0 ? i : 0, bgc[0]);
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
  const Field32 uout = make_field<false>(A.uout, A.ncell, NV, SZ, plane);

  // the march window: planes k and k + 1 (finished), the slope at k and the
  // flux at k - 1/2
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
          for (int v = 0; v < NV; ++v) bz[v] = bgc[0][v];
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

  for (int it = 0; it < G.km; it += NP) {
    const int kraw = k0 + it;
    // ---- loads for this iteration: the NP rows after the window (k + 2 ..
    // k + 1 + NP) and the step-start state of its cells (stored values now,
    // finished where first used)
    int kc[NP];    // row of cell p, held in range
    bool kval[NP]; // cell p is in the chunk
    ST wr[NP][NV], unr[NP][NV];
    bool wn[NP];
    double wlev[NP];
#pragma unroll
    for (int p = 0; p < NP; ++p) {
      kc[p] = min(kraw + p, G.nm - 1);
      kval[p] = kraw + p < k1;
      const int kq = min(kraw, G.nm - 1) + 2 + p;
      const int kk = map_index(kq, G.nm, rm_lo, rm_hi, wn[p]);
      wlev[p] = HYD ? hydro_lever(kq, G.nm, rm_lo, rm_hi, A.dx[1], A.g[1]) : 0.0;
      if constexpr (F32) {
        if (bg_on_m) {
          load_bg<NV>(bgr, A.nbg, kc[p], bgc[p]);
          load_bg<NV>(bgr, A.nbg, kk, bgn[p]);
        }
      }
      load_cell_raw<NDIM, ST>(uin, kk, col, wr[p]);
      if constexpr (STAGE == 2) load_cell_raw<NDIM, ST>(unp, kc[p], col, unr[p]);
    }
    // the cells of this iteration: q[0] = q0, q[1] = q1 (NP = 2)
    double q[NP][NV];
#pragma unroll
    for (int v = 0; v < NV; ++v) {
      q[0][v] = q0[v];
      if constexpr (NP == 2) q[1][v] = q1[v];
    }

    // ---- P1: publish the cell states, and the x ghosts
#pragma unroll
    for (int p = 0; p < NP; ++p) {
      if (pub) {
#pragma unroll
        for (int v = 0; v < NV; ++v) ub[p * UR + v * PX + 1] = q[p][v];
      }
      if (first_x || last_x) {
        // cell 0: periodic, the ghost right of the last cell; wall, the
        // mirror left of cell 0.  The last cell: periodic, the ghost left of
        // cell 0; wall, the mirror right of the last cell.
        double* ur = Urow + p * UR + (first_x == x_per ? G.nx + 1 : 0);
#pragma unroll
        for (int v = 0; v < NV; ++v) ur[v * PX] = (v == 1 && !x_per) ? -q[p][v] : q[p][v];
      }
    }
    __syncthreads();  // B1

    // ---- P2: the x slopes and the plus-face states (published)
    double h[NP][NV];
#pragma unroll
    for (int p = 0; p < NP; ++p) {
#pragma unroll
      for (int v = 0; v < NV; ++v)
        h[p][v] = mc_half(q[p][v] - ub[p * UR + v * PX], ub[p * UR + v * PX + 2] - q[p][v]);
      Face<NV> fp;
      make_face<NDIM, 0, EXT>(q[p], h[p], true, K, fp);
      if (pub) put_face(fb + p * FR + 1, PX, fp);
      if (x_per && last_x) put_face(Frow + p * FR, PX, fp);  // the periodic ghost left of cell 0
    }
    __syncthreads();  // B2

    // ---- P3: the x flux at each cell's left face, published at wave edges
    double Fx_lo[NP][NV];
#pragma unroll
    for (int p = 0; p < NP; ++p) {
      Face<NV> fm, pl;
      make_face<NDIM, 0, EXT>(q[p], h[p], false, K, fm);
      get_face(fb + p * FR, PX, pl);  // slot i: the plus face of cell i - 1
      if (!x_per) {
        if (first_x) pl = mirror<NDIM, 0>(fm);
      }
      flux2<NDIM, 0>(pl, fm, Fx_lo[p]);
      if (lane == 0 && !wave_idle) {
#pragma unroll
        for (int v = 0; v < NV; ++v) xs[(p * NV + v) * nwx] = Fx_lo[p][v];
      }
    }
    __syncthreads();  // B3

    // ---- P4: the flux at each cell's right face, the y direction, then the
    // rate, the RK update and the store
    double Dl[NP][NV];
#pragma unroll
    for (int p = 0; p < NP; ++p) {
      double Fx_hi[NV];
#pragma unroll
      for (int v = 0; v < NV; ++v) Fx_hi[v] = from_right(Fx_lo[p][v]);
      if (last_x) {
        if (x_per) {
#pragma unroll
          for (int v = 0; v < NV; ++v) Fx_hi[v] = xs[(p * NV + v) * nwx - wx];
        } else {
          Face<NV> fp;
          get_face(fb + p * FR + 1, PX, fp);
          flux2<NDIM, 0>(fp, mirror<NDIM, 0>(fp), Fx_hi);
        }
      } else if (lane == 63 && xin && !wave_idle) {
#pragma unroll
        for (int v = 0; v < NV; ++v) Fx_hi[v] = xs[(p * NV + v) * nwx + 1];
      }
#pragma unroll
      for (int v = 0; v < NV; ++v) Dl[p][v] = -(Fx_hi[v] - Fx_lo[p][v]) * hx;
    }
    // the window's next rows, finished: wq[p] is row k + 2 + p
    double wq[NP][NV];
#pragma unroll
    for (int p = 0; p < NP; ++p) {
      if (F32 && bg_on_m) fin(wr[p], wn[p] ? NDIM : -1, bgn[p], 0.0, wq[p]);
      else fin(wr[p], wn[p] ? NDIM : -1, bgc[0], wlev[p], wq[p]);
    }
#pragma unroll
    for (int p = 0; p < NP; ++p) {
      // the slope at k + p + 1 and the flux at k + p + 1/2
      // the rows after cell p: the window is q0, q1, wq[0], ..., wq[NP - 1]
      const double (&qn)[NV] = p == 0 ? q1 : wq[p == 0 ? 0 : p - 1];
      const double (&qnn)[NV] = wq[p];
      double sm1[NV], Fm_hi[NV];
#pragma unroll
      for (int v = 0; v < NV; ++v) sm1[v] = mc_half(qn[v] - q[p][v], qnn[v] - qn[v]);
      Face<NV> fl, fr;
      make_face<NDIM, 1, EXT>(q[p], sm0, true, K, fl);
      make_face<NDIM, 1, EXT>(qn, sm1, false, K, fr);
      flux2<NDIM, 1>(fl, fr, Fm_hi);
#pragma unroll
      for (int v = 0; v < NV; ++v) {
        Dl[p][v] = fma(-(Fm_hi[v] - Fm_lo[v]), hy, Dl[p][v]);
        Fm_lo[v] = Fm_hi[v];
        sm0[v] = sm1[v];
      }
      double Rt[NV];
      const unsigned b = rsst_rate<NDIM, FORM, EXT>(q[p], Dl[p], K, g, Rt);
      double un[NV];
      if constexpr (STAGE == 2) fin(unr[p], -1, bg_on_m ? bgc[p] : bgc[0], 0.0, un);
      if (active && kval[p]) {
        bad |= b;
        double out[NV];
#pragma unroll
        for (int v = 0; v < NV; ++v) {
          double y = fma(dt, Rt[v], q[p][v]);
          if constexpr (STAGE == 2) y = 0.5 * (un[v] + y);
          double bgv = 0.0;
          if constexpr (F32) bgv = bg_on_m ? bgc[p][v] : bgc[0][v];
          const ST st = (ST)(y - bgv);
          buf_store<ST>(uout.r, col, uout.soff(v, kc[p]), st);
          out[v] = (double)st + bgv;
        }
        if constexpr (STAGE == 2) cmax = fmax(cmax, cell_ctot<NDIM, EXT>(out, K));
      }
    }
    // the window moves NP rows
#pragma unroll
    for (int v = 0; v < NV; ++v) {
      if constexpr (NP == 2) {
        q0[v] = wq[0][v];
        q1[v] = wq[1][v];
      } else {
        q0[v] = q1[v];
        q1[v] = wq[0][v];
      }
    }
  }
  return cmax;
}

}  // namespace rsstk
