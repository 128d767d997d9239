// Device code of one RSST stage over a 1D grid: one workgroup holds the whole
// row of nx cells (nwx waves, one lane per cell).  Neighbours come from the
// adjacent lane by DPP and from the adjacent wave through a few LDS seam
// slots; periodic or mirror ends are applied in-row.  Each face state is
// formed once by the cell that owns it; the flux at a wave edge is formed by
// the edge lanes of both waves that share it (the same face states and code,
// so the same bits).  The per-grid 1D kernel stores and reloads the cell;
// the 1D multi-step kernel keeps it in registers across stages (REG).
#pragma once

#include "rsst_stage.h"

#pragma clang fp contract(off)

namespace rsstk {

// LDS carve-up of a 1D workgroup (doubles): the wave-edge seams and the
// reduction slots.
struct Carve1 {
  int seamU, seamUl, seamM, seamP, seamPl, red, total;
};

__host__ __device__ inline Carve1 carve1(int nwx) {
  constexpr int NV = 3, PL = NV + 3;
  Carve1 c;
  int o = 0;
  c.seamU = o;  o += nwx * 2 * NV;  // lane 0 / lane 63 cell states
  c.seamUl = o; o += NV;            // the last cell
  c.seamM = o;  o += nwx * PL;      // lane 0 minus-face states
  c.seamP = o;  o += nwx * PL;      // lane 63 plus-face states
  c.seamPl = o; o += PL;            // the last cell's plus-face state
  c.red = o;    o += 16;
  c.total = o;
  return c;
}

// A 1D cell kept in registers across stages (steps1d_kernel): the stage
// input, the step-start state, the output, and the output's stored value
// (widened).  in and un hold exactly what loading the stored values would
// give, so the results are those of the stored path.
template <int NV>
struct RegCell {
  double in[NV], un[NV], out[NV], st[NV];
};

// One stage of R over the 1D grid, returning the thread's largest c_tot of
// the stage-2 output (0 in stage 1) and or-ing non-physical flags into
// `bad`.  REG: the thread's cell comes from and goes to *rc instead of
// global memory.
template <int STAGE, typename ST, int FORMX, bool REG = false>
__device__ __forceinline__ double stage_body1(const StageArgs& A, double* lds, double dt, unsigned& bad,
                                              RegCell<3>* rc = nullptr) {
  constexpr int NDIM = 1, NV = 3, PL = NV + 3;
  constexpr int FORM = FORMX & 7;
  constexpr int EXT = FORMX & (kExtCmax | kExtVdw);
  constexpr bool F32 = sizeof(ST) == 4;
  constexpr int SZ = (int)sizeof(ST);
  const Geometry& G = A.geo;
  const int nwx = G.nwx;
  const Carve1 C = carve1(nwx);
  double* seamU = lds + C.seamU;    // [nwx][2][NV]
  double* seamUl = lds + C.seamUl;  // [NV]
  double* seamM = lds + C.seamM;    // [nwx][PL]
  double* seamP = lds + C.seamP;    // [nwx][PL]
  double* seamPl = lds + C.seamPl;  // [PL]

  const int tid = threadIdx.x, lane = tid & 63;
  const int wx = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int i_raw = wx * 64 + lane;
  const bool xin = i_raw < G.nx;
  const int i = xin ? i_raw : G.nx - 1;
  const bool last_x = (i_raw == G.nx - 1);
  const bool x_per = A.bc_lo[0] == 0;
  const int col = i * SZ;
  const int plane = G.nx * SZ;

  // FP32 perturbation form: this cell's background values in registers
  double bgA[NV];
  const __amdgpu_buffer_rsrc_t bgr = field_rsrc(A.bg, F32 ? (long long)NV * A.nbg * 8 : 0);
  if constexpr (F32) load_bg<NV>(bgr, A.nbg, A.bg_uniform ? 0 : (A.bg_axis == 0 ? i : 0), bgA);

  const Consts K{A.gamma, A.gm1, A.inv_gm1, A.inv_xi, A.f, A.inv_cmax2, A.vdw_a, A.vdw_b};
  const double g[3] = {A.g[0], A.g[1], A.g[2]};
  const double hx = 0.5 * A.inv_dx[0];
  const Field32 uin = make_field<false>(A.uin, A.ncell, NV, SZ, plane);
  const Field32 unp = make_field<false>(A.un ? A.un : A.uin, A.ncell, NV, SZ, plane);
  // stage 2 writes the new state in place over the step-start state
  const Field32 uout = make_field<false>(A.uout, A.ncell, NV, SZ, plane);

  double q0[NV];
  if constexpr (REG) {
#pragma unroll
    for (int v = 0; v < NV; ++v) q0[v] = rc->in[v];
  } else {
    ST raw[NV];
    load_cell_raw<NDIM, ST>(uin, 0, col, raw);
    if constexpr (F32) finish_cell_bgv<NDIM, ST>(raw, -1, bgA, q0);
    else finish_cell<NDIM, ST>(A, raw, -1, 0, q0);
  }
  ST unr[NV];
  if constexpr (STAGE == 2 && !REG) load_cell_raw<NDIM, ST>(unp, 0, col, unr);

  // ---- P1: publish the cells at the wave edges and the row's end
  {
    double* sw = seamU + wx * 2 * NV;
    if (lane == 0) {
#pragma unroll
      for (int v = 0; v < NV; ++v) sw[v] = q0[v];
    }
    if (lane == 63) {
#pragma unroll
      for (int v = 0; v < NV; ++v) sw[NV + v] = q0[v];
    }
    if (last_x) {
#pragma unroll
      for (int v = 0; v < NV; ++v) seamUl[v] = q0[v];
    }
  }
  __syncthreads();  // B1

  // ---- P2: face states; the flux at the left face from the lane on the left
  double Fx_lo[NV];
  {
    double uL[NV], uR[NV], h[NV];
#pragma unroll
    for (int v = 0; v < NV; ++v) { uL[v] = from_left(q0[v]); uR[v] = from_right(q0[v]); }
    if (lane == 0) {
      if (wx > 0) {
        const double* sw = seamU + ((wx - 1) * 2 + 1) * NV;
#pragma unroll
        for (int v = 0; v < NV; ++v) uL[v] = sw[v];
      } else if (x_per) {
#pragma unroll
        for (int v = 0; v < NV; ++v) uL[v] = seamUl[v];
      } else {
#pragma unroll
        for (int v = 0; v < NV; ++v) uL[v] = q0[v];
        uL[1] = -q0[1];
      }
    }
    if (last_x) {
      if (x_per) {
#pragma unroll
        for (int v = 0; v < NV; ++v) uR[v] = seamU[v];
      } else {
#pragma unroll
        for (int v = 0; v < NV; ++v) uR[v] = q0[v];
        uR[1] = -q0[1];
      }
    } else if (lane == 63 && xin) {
      const double* sw = seamU + (wx + 1) * 2 * NV;
#pragma unroll
      for (int v = 0; v < NV; ++v) uR[v] = sw[v];
    }
#pragma unroll
    for (int v = 0; v < NV; ++v) h[v] = mc_half(q0[v] - uL[v], uR[v] - q0[v]);
    Face<NV> fm, fp;
    make_face<NDIM, 0, EXT>(q0, h, false, K, fm);
    make_face<NDIM, 0, EXT>(q0, h, true, K, fp);
    // the wave-edge faces are redone after the barrier from the seams
    if (lane == 0) put_face(seamM + wx * PL, 1, fm);
    if (lane == 63) put_face(seamP + wx * PL, 1, fp);
    if (last_x) put_face(seamPl, 1, fp);
    const Face<NV> pl = face_from_left(fp);
    flux2<NDIM, 0>(pl, fm, Fx_lo);
  }
  __syncthreads();  // B2

  // ---- P3: the fluxes of the faces at the wave edges, formed by the edge
  // lanes of both waves that share them from the seam face states; then the
  // rate, the RK update and the store
  double Dl[NV];
  {
    double Fx_hi[NV];
#pragma unroll
    for (int v = 0; v < NV; ++v) Fx_hi[v] = from_right(Fx_lo[v]);
    const bool edge_r = last_x || (lane == 63 && xin);
    if (lane == 0 || edge_r) {
      Face<NV> fl, fr;
      if (lane == 0) {  // face at the wave's left edge
        get_face(seamM + wx * PL, 1, fr);
        if (wx > 0) get_face(seamP + (wx - 1) * PL, 1, fl);
        else if (x_per) get_face(seamPl, 1, fl);
        else fl = mirror<NDIM, 0>(fr);
      } else if (last_x) {  // face at the row's end
        get_face(seamPl, 1, fl);
        if (x_per) get_face(seamM, 1, fr);
        else fr = mirror<NDIM, 0>(fl);
      } else {  // face at the wave's right edge
        get_face(seamP + wx * PL, 1, fl);
        get_face(seamM + (wx + 1) * PL, 1, fr);
      }
      double Fe[NV];
      flux2<NDIM, 0>(fl, fr, Fe);
      if (lane == 0) {
#pragma unroll
        for (int v = 0; v < NV; ++v) Fx_lo[v] = Fe[v];
      } else {
#pragma unroll
        for (int v = 0; v < NV; ++v) Fx_hi[v] = Fe[v];
      }
    }
    // A row of 64 m + 1 cells ends in lane 0 of its last wave: that lane
    // took its left face above and forms the row's end face here.
    if (lane == 0 && last_x) {
      Face<NV> fl, fr;
      get_face(seamPl, 1, fl);
      if (x_per) get_face(seamM, 1, fr);
      else fr = mirror<NDIM, 0>(fl);
      flux2<NDIM, 0>(fl, fr, Fx_hi);
    }
#pragma unroll
    for (int v = 0; v < NV; ++v) Dl[v] = -(Fx_hi[v] - Fx_lo[v]) * hx;
  }
  double R[NV];
  const unsigned b = rsst_rate<NDIM, FORM, EXT>(q0, Dl, K, g, R);
  double un[NV];
  if constexpr (STAGE == 2 && REG) {
#pragma unroll
    for (int v = 0; v < NV; ++v) un[v] = rc->un[v];
  } else if constexpr (STAGE == 2) {
    if constexpr (F32) finish_cell_bgv<NDIM, ST>(unr, -1, bgA, un);
    else finish_cell<NDIM, ST>(A, unr, -1, 0, un);
  }
  double cmax = 0.0;
  if (xin) {
    bad |= b;
    double out[NV];
#pragma unroll
    for (int v = 0; v < NV; ++v) {
      double y = fma(dt, R[v], q0[v]);
      if constexpr (STAGE == 2) y = 0.5 * (un[v] + y);
      double bgv = 0.0;
      if constexpr (F32) bgv = bgA[v];
      const ST st = (ST)(y - bgv);
      if constexpr (REG) rc->st[v] = (double)st;
      else buf_store<ST>(uout.r, col, uout.soff(v, 0), st);
      out[v] = (double)st + bgv;
      if constexpr (REG) rc->out[v] = out[v];
    }
    if constexpr (STAGE == 2) cmax = cell_ctot<NDIM, EXT>(out, K);
  }
  return cmax;
}

}  // namespace rsstk
