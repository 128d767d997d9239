// Device code of one RSST stage over a 3D tile (the per-grid 3D kernels).
//
// A tile is TS = 2R stacked y rows of whole x rows, marched along z over one
// chunk of planes.  The workgroup has R thread-rows of nwx waves; each thread
// owns one column i of TWO adjacent rows (j, j + 1), so:
//   * the y face between its two rows is formed once, in registers;
//   * a tile is twice as tall for the same number of waves, which halves the
//     share of cells whose y neighbourhood reaches outside the tile (the
//     tile's edge rows rebuild the face state of the row outside it);
//   * each thread has two independent cells' arithmetic to interleave.
// x neighbours and x face states are exchanged through LDS rows with one
// ghost slot at each end (periodic wrap or mirror), so no lane of a wave is
// special except at the row's two ends.  Every x and y face flux is formed
// once, by the cell above (or right of) the face, and handed to the cell
// below (left) through LDS after a third barrier (x: by DPP within a wave,
// one LDS seam value per wave edge); the y flux at a tile's outer face is
// formed by each of the two tiles that share it, from the same face states
// with the same code, so with the same bits.  z is marched as in the other
// dimensions: every z face is formed once and carried to the next plane.
#pragma once

#include "rsst_stage.h"

#pragma clang fp contract(off)

namespace rsstk {

// Rows per 3D tile (even) for rows of nwx waves: eight waves per workgroup
// (six for rows of three waves), two rows per thread.
__host__ __device__ constexpr int tile_rows3(int nwx) {
  return nwx == 1 ? 16 : (nwx == 2 ? 8 : (nwx <= 4 ? 4 : 2));
}

// LDS carve-up of a 3D workgroup (doubles); ts rows of nwx waves each.
struct Carve3 {
  int u, fp, fyp, fy, fxs, red, total;
};

__host__ __device__ inline Carve3 carve3(int ts, int nwx) {
  constexpr int NV = 5, PL = NV + 3;
  const int nxp = 64 * nwx, px = nxp + 2, r = ts / 2;
  Carve3 c;
  int o = 0;
  // row-major ([row][value][slot]), so that every value of a row is at a
  // fixed offset from the thread's row address
  c.u = o;   o += ts * NV * px;        // cell states, slot 1 + i; slots 0, nx + 1: x ghosts
  c.fp = o;  o += ts * PL * px;        // x plus-face states, slot 1 + i; slot 0: the left ghost's
  c.fyp = o; o += (r - 1) * PL * nxp;  // y plus face of the upper row of thread-rows 0..R-2
  c.fy = o;  o += (r - 1) * NV * nxp;  // y flux at the lower face of thread-rows 1..R-1
  c.fxs = o; o += ts * NV * nwx;       // x flux at the left edge of each wave
  c.red = o; o += 16;
  c.total = o;
  return c;
}

// One stage of R over one 3D tile (rows [tile_s TS, tile_s TS + TS) of the
// z-chunk `chunk`), returning the thread's largest c_tot of the stage-2
// output (0 in stage 1) and or-ing non-physical flags into `bad`.  The last
// tile of a column whose height is not a multiple of TS is moved down to end
// at the last row: its rows below tile_s TS are computed (with the same bits)
// but stored by the tile before it.  NWXC: waves per x row (rows of five to
// eight waves run as rows of eight); BIG: Field64 addressing.
template <int STAGE, typename ST, int FORMX, int NWXC, bool BIG = false>
__device__ __forceinline__ double stage_body3(const StageArgs& A, double* lds, int tile_s, int chunk,
                                              double dt, unsigned& bad) {
  constexpr int NDIM = 3, NV = 5, PL = NV + 3;
  constexpr int FORM = FORMX & 7;
  constexpr int EXT = FORMX & (kExtCmax | kExtVdw);
  constexpr bool HYD = (FORMX & kExtHydro) != 0;
  constexpr bool F32 = sizeof(ST) == 4;
  constexpr int SZ = (int)sizeof(ST);
  constexpr int NXP = 64 * NWXC, PX = NXP + 2;
  constexpr bool ONE = NWXC == 8;  // one thread-row: both tile edges
  constexpr bool kEarlyOut = STAGE == 1 && !ONE && !HYD;
  const Geometry& G = A.geo;
  const int TS = G.ts, R = TS >> 1;
  const Carve3 C = carve3(TS, NWXC);
  double* Us = lds + C.u;     // [TS][NV][PX]
  double* FPs = lds + C.fp;   // [TS][PL][PX]
  double* FYP = lds + C.fyp;  // [R-1][PL][NXP]
  double* FY = lds + C.fy;    // [R-1][NV][NXP]
  double* FXS = lds + C.fxs;  // [TS][NV][NWXC]
  constexpr int UR = NV * PX, FR = PL * PX;  // row pitches of Us, FPs

  const int tid = threadIdx.x, lane = tid & 63;
  const int w = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int wx = w % NWXC, r = w / NWXC;
  const int i_raw = wx * 64 + lane;
  const bool xin = i_raw < G.nx;
  const int i = xin ? i_raw : G.nx - 1;
  const int j_own = tile_s * TS;
  const int j0 = min(j_own, G.ns - TS);
  const int jl = j0 + 2 * r;  // the thread's lower row; its upper row is jl + 1
  const int rl = 2 * r;       // the lower row's index in the tile
  const bool first = r == 0, last = r == R - 1;
  const int k0 = chunk * G.km, k1 = min(k0 + G.km, G.nm);
  const bool own_lo = xin && jl >= j_own, own_hi = xin && jl + 1 >= j_own;
  const bool last_x = i_raw == G.nx - 1;
  const bool x_per = A.bc_lo[0] == 0;
  const int rm_lo = A.bc_lo[2], rm_hi = A.bc_hi[2];
  const int plane = G.nx * G.ns * SZ;  // bytes per z plane
  const int colc[2] = {(jl * G.nx + i) * SZ, ((jl + 1) * G.nx + i) * SZ};
  // the thread's LDS addresses: its lower row's cell slot minus one (its left
  // neighbour) and plus-face slot, the y exchange slots of its thread-row,
  // and its wave's x seam
  double* const ub = Us + rl * UR + i;      // + c UR + v PX + {0, 1, 2}: left, own, right
  double* const fb = FPs + rl * FR + i;     // + c FR + q PX + {0, 1}: left neighbour's, own
  double* const yp = FYP + r * (PL * NXP) + i_raw;  // written by thread-row r; r - 1 reads it
  double* const yf = FY + r * (NV * NXP) + i_raw;   // written by thread-row r + 1 (slot r); r reads it
  double* const xs = FXS + rl * (NV * NWXC) + wx;   // + c NV NWXC + v NWXC

  // FP32 perturbation form: the background is loaded where it is used, not
  // held across the march (ten FP64 values per plane would take 40 VGPRs).
  // bg_at(kk, b): the lower cell's background at plane kk.  Uniform or along
  // z, its index is the same for the whole workgroup and the load goes
  // through the scalar cache into SGPRs; along x it is the thread's column
  // (vector loads, L1 hits).  With a profile along y the upper cell and the
  // rows outside the tile take the indexed path.
  const bool bg_on_m = F32 && A.bg_axis == 2;
  const bool bg_rows = F32 && A.bg_axis == 1;
  auto bg_cell = [&](int c) { return A.bg_axis == 0 ? i : (A.bg_axis == 1 ? jl + c : 0); };
  const __amdgpu_buffer_rsrc_t bgr = field_rsrc(A.bg, F32 ? (long long)NV * A.nbg * 8 : 0);
  auto bg_at = [&](int kk, double (&b)[NV]) {
    if (A.bg_uniform) {
      const int u = __builtin_amdgcn_readfirstlane(A.bg_axis == 2 ? kk : 0);
#pragma unroll
      for (int v = 0; v < NV; ++v) b[v] = A.bg[v * A.nbg + u];
    } else {
      load_bg<NV>(bgr, A.nbg, bg_cell(0), b);
    }
  };
  // FP64 state of stored values: FP32, with the background at profile index b
  // (vector loads where used); FP64, with the mirror sign and the hydrostatic
  // wall's carried pressure (lever)
  auto fin_idx = [&](const ST (&raw)[NV], int neg, int b, double lev, double (&u)[NV]) {
    if constexpr (F32) {
      double bz[NV];
      load_bg<NV>(bgr, A.nbg, b, bz);
      finish_cell_bgv<NDIM, ST>(raw, neg, bz, u);
    } else {
      finish_cell<NDIM, ST>(A, raw, neg, 0, u, lev);
    }
  };
  // FP32: cell c's stored values at plane k with the background bgz (of plane
  // k, or of the plane two ahead for the march loads); a profile along y
  // takes the upper cell's own row
  auto fin_c = [&](const ST (&raw)[NV], int neg, int c, const double (&bgz)[NV], double (&u)[NV]) {
    if constexpr (F32) {
      if (c == 1 && bg_rows) fin_idx(raw, neg, jl + 1, 0.0, u);
      else finish_cell_bgv<NDIM, ST>(raw, neg, bgz, u);
    }
  };

  const Consts K{A.gamma, A.gm1, A.inv_gm1, A.inv_xi, A.f, A.inv_cmax2, A.vdw_a, A.vdw_b};
  const double g[3] = {A.g[0], A.g[1], A.g[2]};
  const double hx = 0.5 * A.inv_dx[0], hy = 0.5 * A.inv_dx[1], hz = 0.5 * A.inv_dx[2];
  const FieldT<BIG> uin = make_field<BIG>(A.uin, A.ncell, NV, SZ, plane);
  const FieldT<BIG> unp = make_field<BIG>(A.un ? A.un : A.uin, A.ncell, NV, SZ, plane);
  // stage 2 writes the new state in place over the step-start state (the
  // callers pass uout == un), so one field serves both
  const FieldT<BIG> uout = make_field<BIG>(A.uout, A.ncell, NV, SZ, plane);

  // y rows just outside the tile: columns, mirror flags, background rows and
  // hydrostatic levers
  int clo1, clo2, chi1, chi2, nlo1, nlo2, nhi1, nhi2, blo1, blo2, bhi1, bhi2;
  double llo1 = 0.0, llo2 = 0.0, lhi1 = 0.0, lhi2 = 0.0;
  {
    bool n;
    int jj;
    if constexpr (HYD) {
      const double dy = A.dx[1], gy = A.g[1];
      const int bl = A.bc_lo[1], bh = A.bc_hi[1];
      llo1 = hydro_lever(j0 - 1, G.ns, bl, bh, dy, gy);
      llo2 = hydro_lever(j0 - 2, G.ns, bl, bh, dy, gy);
      lhi1 = hydro_lever(j0 + TS, G.ns, bl, bh, dy, gy);
      lhi2 = hydro_lever(j0 + TS + 1, G.ns, bl, bh, dy, gy);
    }
    const int bxy = A.bg_axis == 0 ? i : 0;
    jj = map_index(j0 - 1, G.ns, A.bc_lo[1], A.bc_hi[1], n); nlo1 = n ? 2 : -1; clo1 = (jj * G.nx + i) * SZ;
    blo1 = (A.bg_axis == 1) ? jj : bxy;
    jj = map_index(j0 - 2, G.ns, A.bc_lo[1], A.bc_hi[1], n); nlo2 = n ? 2 : -1; clo2 = (jj * G.nx + i) * SZ;
    blo2 = (A.bg_axis == 1) ? jj : bxy;
    jj = map_index(j0 + TS, G.ns, A.bc_lo[1], A.bc_hi[1], n); nhi1 = n ? 2 : -1; chi1 = (jj * G.nx + i) * SZ;
    bhi1 = (A.bg_axis == 1) ? jj : bxy;
    jj = map_index(j0 + TS + 1, G.ns, A.bc_lo[1], A.bc_hi[1], n); nhi2 = n ? 2 : -1; chi2 = (jj * G.nx + i) * SZ;
    bhi2 = (A.bg_axis == 1) ? jj : bxy;
  }
  // The edge thread-rows read the two rows outside their side of the tile
  // one plane ahead, so that load latency hides behind a whole plane of
  // work: o1, o2 are the near and far outside rows of the wave's side (one
  // thread-row: o1, o2 below and o3, o4 above).  Thread-rows between the
  // edges issue the same loads (the rows above the tile, unused), so every
  // wave has the same loads in flight at every point of the march: loads
  // complete in order, and a wait sized for a wave with fewer loads in
  // flight would make the edge rows wait for the next plane's loads.
  const bool o_lo = first;
  const int oc1 = o_lo ? clo1 : chi1, oc2 = o_lo ? clo2 : chi2;
  const int on1 = o_lo ? nlo1 : nhi1, on2 = o_lo ? nlo2 : nhi2;
  const int ob1 = o_lo ? blo1 : bhi1, ob2 = o_lo ? blo2 : bhi2;
  const double ol1 = o_lo ? llo1 : lhi1, ol2 = o_lo ? llo2 : lhi2;
  ST o1[NV], o2[NV], o3[ONE ? NV : 1], o4[ONE ? NV : 1];  // stored values, finished at use
  // an outside row's FP64 state at plane k (k_cur: the plane of this
  // iteration)
  int k_cur = 0;
  auto fin_out = [&](const ST (&raw)[NV], int neg, int b, double lev, double (&u)[NV]) {
    if (F32 && !bg_rows) {
      double bz[NV];
      bg_at(k_cur, bz);
      finish_cell_bgv<NDIM, ST>(raw, neg, bz, u);
    } else {
      fin_idx(raw, neg, b, lev, u);
    }
  };

  double q0[2][NV], q1[2][NV], sm0[2][NV], Fm_lo[2][NV];
  double cmax = 0.0;
  const int k0l = min(k0, G.nm - 1);
#pragma unroll
  for (int c = 0; c < 2; ++c) {
    double qa[NV], qb[NV], ha[NV];
    bool n;
    int kk;
    const int b = A.bg_uniform ? 0 : bg_cell(c);
    auto ld = [&](int q, double (&u)[NV]) {  // plane k0l + q of the cell's column, through the z walls
      const int kk = map_index(k0l + q, G.nm, rm_lo, rm_hi, n);
      ST raw[NV];
      load_cell_raw<NDIM, ST>(uin, kk, colc[c], raw);
      fin_idx(raw, n ? NDIM : -1, bg_on_m ? kk : b,
              HYD ? hydro_lever(k0l + q, G.nm, rm_lo, rm_hi, A.dx[2], A.g[2]) : 0.0, u);
    };
    ld(-2, qa);
    ld(-1, qb);
    ld(0, q0[c]);
    ld(1, q1[c]);
#pragma unroll
    for (int v = 0; v < NV; ++v) {
      ha[v] = mc_half(qb[v] - qa[v], q0[c][v] - qb[v]);
      sm0[c][v] = mc_half(q0[c][v] - qb[v], q1[c][v] - q0[c][v]);
    }
    Face<NV> fl, fr;
    make_face<NDIM, 2, EXT>(qb, ha, true, K, fl);
    make_face<NDIM, 2, EXT>(q0[c], sm0[c], false, K, fr);
    flux2<NDIM, 2>(fl, fr, Fm_lo[c]);
  }
  load_cell_raw<NDIM, ST>(uin, k0l, oc1, o1);
  load_cell_raw<NDIM, ST>(uin, k0l, oc2, o2);
  if constexpr (ONE) {
    load_cell_raw<NDIM, ST>(uin, k0l, chi1, o3);
    load_cell_raw<NDIM, ST>(uin, k0l, chi2, o4);
  }

  for (int it = 0; it < G.km; ++it) {
    const int kraw = k0 + it;
    const bool kval = kraw < k1;
    const int k = min(kraw, G.nm - 1);  // plane used for loads and stores
    // ---- loads for this plane: the plane two ahead and the step-start
    // state (stored values now, finished where first used)
    ST q2r[2][NV], unr[2][NV];
    bool q2n;
    const int q2k = map_index(k + 2, G.nm, rm_lo, rm_hi, q2n);
    const int q2neg = q2n ? NDIM : -1;
    const double q2lev = HYD ? hydro_lever(k + 2, G.nm, rm_lo, rm_hi, A.dx[2], A.g[2]) : 0.0;
    k_cur = k;
#pragma unroll
    for (int c = 0; c < 2; ++c) load_cell_raw<NDIM, ST>(uin, q2k, colc[c], q2r[c]);

    // ---- P1: publish both rows' cell states, and the x ghosts
#pragma unroll
    for (int c = 0; c < 2; ++c) {
      if (xin) {
#pragma unroll
        for (int v = 0; v < NV; ++v) ub[c * UR + v * PX + 1] = q0[c][v];
      }
      if (i_raw == 0 || last_x) {
        // cell 0: periodic, the ghost right of the last cell; wall, the
        // mirror left of cell 0.  The last cell: periodic, the ghost left of
        // cell 0; wall, the mirror right of the last cell.
        double* ur = Us + (rl + c) * UR + ((i_raw == 0) == x_per ? G.nx + 1 : 0);
#pragma unroll
        for (int v = 0; v < NV; ++v) ur[v * PX] = (v == 1 && !x_per) ? -q0[c][v] : q0[c][v];
      }
    }
    __syncthreads();  // B1

    // ---- P2: x plus-face states (published), y face states, the y flux
    // between the thread's rows, and at the tile's outer faces
    double h[2][NV];
#pragma unroll
    for (int c = 0; c < 2; ++c) {
#pragma unroll
      for (int v = 0; v < NV; ++v)
        h[c][v] = mc_half(q0[c][v] - ub[c * UR + v * PX], ub[c * UR + v * PX + 2] - q0[c][v]);
      Face<NV> fp;
      make_face<NDIM, 0, EXT>(q0[c], h[c], true, K, fp);
      if (xin) put_face(fb + c * FR + 1, PX, fp);
      if (x_per && last_x) put_face(FPs + (rl + c) * FR, PX, fp);  // the periodic ghost left of cell 0
    }
    double hl[NV], Fym[NV], Fy_lo[NV], Fy_hi[NV];
    {
      double uD[NV], uU[NV], d[NV], hh[NV];
      if (first) {
        fin_out(o1, on1, bg_on_m ? k : ob1, ol1, uD);
      } else {
#pragma unroll
        for (int v = 0; v < NV; ++v) uD[v] = ub[v * PX + 1 - UR];
      }
      if (last) {
        if constexpr (ONE) fin_out(o3, nhi1, bg_on_m ? k : bhi1, lhi1, uU);
        else fin_out(o1, on1, bg_on_m ? k : ob1, ol1, uU);
      } else {
#pragma unroll
        for (int v = 0; v < NV; ++v) uU[v] = ub[2 * UR + v * PX + 1];
      }
#pragma unroll
      for (int v = 0; v < NV; ++v) {
        d[v] = q0[1][v] - q0[0][v];
        hl[v] = mc_half(q0[0][v] - uD[v], d[v]);
        hh[v] = mc_half(d[v], uU[v] - q0[1][v]);
      }
      {
        Face<NV> a, b;
        make_face<NDIM, 1, EXT>(q0[0], hl, true, K, a);
        make_face<NDIM, 1, EXT>(q0[1], hh, false, K, b);
        flux2<NDIM, 1>(a, b, Fym);
      }
      Face<NV> fyp;
      make_face<NDIM, 1, EXT>(q0[1], hh, true, K, fyp);
      if (!last) put_face(yp, NXP, fyp);
      if (last) {
        // minus state of the row above the tile, and the flux at the
        // tile's upper face
        double u2[NV], h2[NV];
        if constexpr (ONE) fin_out(o4, nhi2, bg_on_m ? k : bhi2, lhi2, u2);
        else fin_out(o2, on2, bg_on_m ? k : ob2, ol2, u2);
#pragma unroll
        for (int v = 0; v < NV; ++v) h2[v] = mc_half(uU[v] - q0[1][v], u2[v] - uU[v]);
        Face<NV> fh;
        make_face<NDIM, 1, EXT>(uU, h2, false, K, fh);
        flux2<NDIM, 1>(fyp, fh, Fy_hi);
      }
      if (first) {
        // plus state of the row below the tile, and the flux at the tile's
        // lower face
        double u2[NV], h2[NV];
        fin_out(o2, on2, bg_on_m ? k : ob2, ol2, u2);
#pragma unroll
        for (int v = 0; v < NV; ++v) h2[v] = mc_half(uD[v] - u2[v], q0[0][v] - uD[v]);
        Face<NV> fh, fm;
        make_face<NDIM, 1, EXT>(uD, h2, true, K, fh);
        make_face<NDIM, 1, EXT>(q0[0], hl, false, K, fm);
        flux2<NDIM, 1>(fh, fm, Fy_lo);
      }
    }
    // the outside rows of the next plane.  Stage 1 issues them as soon as
    // this plane's are finished: the tile that owns those rows read them at
    // the top of the iteration before, so more of them are still in L2 than
    // at the end of this iteration.  Where more is live across P3 and P4
    // (stage 2's step-start state, both outside sides of a one-thread-row
    // tile, the hydrostatic walls' levers) the longer live range would
    // spill, so those issue them last.
    auto load_outside = [&]() {
      const int kn = min(kraw + 1, G.nm - 1);
      load_cell_raw<NDIM, ST>(uin, kn, oc1, o1);
      load_cell_raw<NDIM, ST>(uin, kn, oc2, o2);
      if constexpr (ONE) {
        load_cell_raw<NDIM, ST>(uin, kn, chi1, o3);
        load_cell_raw<NDIM, ST>(uin, kn, chi2, o4);
      }
    };
    if constexpr (kEarlyOut) load_outside();
    __syncthreads();  // B2
    if constexpr (STAGE == 2) {
#pragma unroll
      for (int c = 0; c < 2; ++c) load_cell_raw<NDIM, ST, kUnAux3>(unp, k, colc[c], unr[c]);
    }

    // ---- P3: the x flux at each cell's left face and the y flux at the
    // thread-row's lower face, published for the cell on the other side
    double Fx_lo[2][NV];
#pragma unroll
    for (int c = 0; c < 2; ++c) {
      Face<NV> fm, pl;
      make_face<NDIM, 0, EXT>(q0[c], h[c], false, K, fm);
      get_face(fb + c * FR, PX, pl);  // slot i: the plus face of cell i - 1
      if (!x_per) {
        if (i_raw == 0) pl = mirror<NDIM, 0>(fm);
      }
      flux2<NDIM, 0>(pl, fm, Fx_lo[c]);
      if (lane == 0) {
#pragma unroll
        for (int v = 0; v < NV; ++v) xs[(c * NV + v) * NWXC] = Fx_lo[c][v];
      }
    }
    if (!first) {
      Face<NV> fm, pd;
      make_face<NDIM, 1, EXT>(q0[0], hl, false, K, fm);
      get_face(yp - PL * NXP, NXP, pd);
      flux2<NDIM, 1>(pd, fm, Fy_lo);
#pragma unroll
      for (int v = 0; v < NV; ++v) yf[v * NXP - NV * NXP] = Fy_lo[v];
    }
    __syncthreads();  // B3

    // ---- P4: the fluxes on the far side of each cell, the z direction,
    // then the rate, the RK update and the store
    double Dl[2][NV];
#pragma unroll
    for (int c = 0; c < 2; ++c) {
      double Fx_hi[NV];
#pragma unroll
      for (int v = 0; v < NV; ++v) Fx_hi[v] = from_right(Fx_lo[c][v]);
      if (last_x) {
        if (x_per) {
#pragma unroll
          for (int v = 0; v < NV; ++v) Fx_hi[v] = xs[(c * NV + v) * NWXC - wx];
        } else {
          Face<NV> fp;
          get_face(fb + c * FR + 1, PX, fp);
          flux2<NDIM, 0>(fp, mirror<NDIM, 0>(fp), Fx_hi);
        }
      } else if (lane == 63 && xin) {
#pragma unroll
        for (int v = 0; v < NV; ++v) Fx_hi[v] = xs[(c * NV + v) * NWXC + 1];
      }
#pragma unroll
      for (int v = 0; v < NV; ++v) Dl[c][v] = -(Fx_hi[v] - Fx_lo[c][v]) * hx;
    }
    if (!last) {
#pragma unroll
      for (int v = 0; v < NV; ++v) Fy_hi[v] = yf[v * NXP];
    }
#pragma unroll
    for (int v = 0; v < NV; ++v) {
      Dl[0][v] = fma(-(Fym[v] - Fy_lo[v]), hy, Dl[0][v]);
      Dl[1][v] = fma(-(Fy_hi[v] - Fym[v]), hy, Dl[1][v]);
    }
    double q2[2][NV];
#pragma unroll
    for (int c = 0; c < 2; ++c) {
      if constexpr (F32) {
        double bz[NV];
        bg_at(q2k, bz);
        fin_c(q2r[c], q2neg, c, bz, q2[c]);
      } else {
        fin_idx(q2r[c], q2neg, 0, q2lev, q2[c]);
      }
      double sm1[NV], Fm_hi[NV];
#pragma unroll
      for (int v = 0; v < NV; ++v) sm1[v] = mc_half(q1[c][v] - q0[c][v], q2[c][v] - q1[c][v]);
      Face<NV> fl, fr;
      make_face<NDIM, 2, EXT>(q0[c], sm0[c], true, K, fl);
      make_face<NDIM, 2, EXT>(q1[c], sm1, false, K, fr);
      flux2<NDIM, 2>(fl, fr, Fm_hi);
#pragma unroll
      for (int v = 0; v < NV; ++v) {
        Dl[c][v] = fma(-(Fm_hi[v] - Fm_lo[c][v]), hz, Dl[c][v]);
        Fm_lo[c][v] = Fm_hi[v];
        sm0[c][v] = sm1[v];
      }
      double Rt[NV];
      const unsigned b = rsst_rate<NDIM, FORM, EXT>(q0[c], Dl[c], K, g, Rt);
      double un[NV];
      if constexpr (STAGE == 2) {
        if constexpr (F32) {
          double bz[NV];
          bg_at(k, bz);
          fin_c(unr[c], -1, c, bz, un);
        } else {
          fin_idx(unr[c], -1, 0, 0.0, un);
        }
      }
      if ((c == 0 ? own_lo : own_hi) && kval) {
        bad |= b;
        double out[NV], bgc[NV];
        if constexpr (F32) {
          if (c == 1 && bg_rows) load_bg<NV>(bgr, A.nbg, jl + 1, bgc);
          else bg_at(k, bgc);
        }
#pragma unroll
        for (int v = 0; v < NV; ++v) {
          double y = fma(dt, Rt[v], q0[c][v]);
          if constexpr (STAGE == 2) y = 0.5 * (un[v] + y);
          double bgv = 0.0;
          if constexpr (F32) bgv = bgc[v];
          const ST st = (ST)(y - bgv);
          buf_store<ST, kStoreAux3>(uout.rsrc(v, k), colc[c], uout.soff(v, k), st);
          out[v] = (double)st + bgv;
        }
        if constexpr (STAGE == 2) cmax = fmax(cmax, cell_ctot<NDIM, EXT>(out, K));
      }
#pragma unroll
      for (int v = 0; v < NV; ++v) { q0[c][v] = q1[c][v]; q1[c][v] = q2[c][v]; }
    }
    if constexpr (!kEarlyOut) load_outside();
  }
  return cmax;
}

}  // namespace rsstk
