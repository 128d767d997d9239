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
#include <cstdlib>

#include "rsst_device.h"
#include "rsst_internal.h"

#pragma clang fp contract(off)

namespace rsstk {

// ---------------------------------------------------------------- loads

// Boundary rule on one axis, for an index at most two cells outside [0, n):
// periodic sides wrap; reflecting sides mirror (ghost -1-q takes cell q) and
// flag the normal momentum for negation.  Called with workgroup-uniform
// indices, so it runs on the scalar unit.
__device__ __forceinline__ int map_index(int q, int n, int refl_lo, int refl_hi, bool& neg) {
  neg = false;
  if (q < 0) {
    if (refl_lo) { neg = true; return -1 - q; }
    return q + n;
  }
  if (q >= n) {
    if (refl_hi) { neg = true; return 2 * n - 1 - q; }
    return q - n;
  }
  return q;
}

// Raw buffer access to a field: one resource per field (bounds-checked by
// the hardware against the field's byte size), a workgroup-uniform byte
// offset in an SGPR (plane and variable) and a loop-invariant per-thread
// byte offset in a VGPR (the column), so no vector address arithmetic.
typedef unsigned int u32x2_t __attribute__((ext_vector_type(2)));

__device__ __forceinline__ __amdgpu_buffer_rsrc_t field_rsrc(const void* p, long long bytes) {
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(p), (short)0, (int)bytes, 0x00020000);
}

template <typename ST>
__device__ __forceinline__ double buf_load(__amdgpu_buffer_rsrc_t r, int voff, int soff) {
  if constexpr (sizeof(ST) == 8) {
    const u32x2_t v = __builtin_amdgcn_raw_buffer_load_b64(r, voff, soff, 0);
    return __hiloint2double((int)v.y, (int)v.x);
  } else {
    return (double)__uint_as_float(__builtin_amdgcn_raw_buffer_load_b32(r, voff, soff, 0));
  }
}

template <typename ST>
__device__ __forceinline__ void buf_store(__amdgpu_buffer_rsrc_t r, int voff, int soff, ST x) {
  if constexpr (sizeof(ST) == 8) {
    u32x2_t v;
    v.x = (unsigned)__double2loint(x);
    v.y = (unsigned)__double2hiint(x);
    __builtin_amdgcn_raw_buffer_store_b64(v, r, voff, soff, 0);
  } else {
    __builtin_amdgcn_raw_buffer_store_b32(__float_as_uint(x), r, voff, soff, 0);
  }
}

// Cell state at byte offsets (soff: workgroup-uniform plane offset, voff:
// the thread's column) as FP64; `negv` >= 0 names a momentum component to
// negate (mirror ghost); b: background index (FP32 perturbation form).
template <int NDIM, typename ST>
__device__ __forceinline__ void load_cell(const StageArgs& A, __amdgpu_buffer_rsrc_t r, int soff,
                                          int voff, int negv, int b, double (&u)[NDIM + 2]) {
  constexpr int NV = NDIM + 2;
  const int vstride = (int)(A.ncell * (long long)sizeof(ST));
#pragma unroll
  for (int v = 0; v < NV; ++v) {
    u[v] = buf_load<ST>(r, voff, soff + v * vstride);
    if constexpr (sizeof(ST) == 4) u[v] += A.bg[v * A.nbg + b];
  }
#pragma unroll
  for (int v = 1; v <= NDIM; ++v)
    if (v == negv) u[v] = -u[v];
}

// Index of the background profile for cell (i, j, k) in kernel axes.
template <int NDIM>
__device__ __forceinline__ int bg_index(const StageArgs& A, int i, int j, int k) {
  if (A.bg_axis == 0) return i;
  if (A.bg_axis == 1) return (NDIM == 3) ? j : k;
  if (A.bg_axis == 2) return k;
  return 0;
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

// LDS carve-up of one workgroup (doubles).  3D only: Urow, Prow, Frow.
struct Carve {
  int urow, prow, frow, seamU, seamUl, seamM, seamP, seamPl, seamF, red, total;
};

__host__ __device__ inline Carve carve(int ndim, int ts, int nwx) {
  const int NV = ndim + 2, PL = NV + 3, nxp = 64 * nwx;
  Carve c;
  int o = 0;
  c.urow = o;   if (ndim == 3) o += NV * ts * nxp;        // cell states, per row
  c.prow = o;   if (ndim == 3) o += PL * ts * nxp;        // y plus-face states
  c.frow = o;   if (ndim == 3) o += NV * (ts + 1) * nxp;  // y fluxes at faces r - 1/2
  c.seamU = o;  o += ts * nwx * 2 * NV;                   // lane 0 / lane 63 cell states
  c.seamUl = o; o += ts * NV;                             // last cell of each row
  c.seamM = o;  o += ts * nwx * PL;                       // lane 0 minus-face states
  c.seamP = o;  o += ts * nwx * PL;                       // lane 63 plus-face states
  c.seamPl = o; o += ts * PL;                             // last cell's plus-face state
  c.seamF = o;  o += ts * (nwx + 1) * NV;                 // x fluxes at wave edges
  c.red = o;    o += 16;
  c.total = o;
  return c;
}

// Rows per 3D tile for a row of nwx waves (512 threads at most).
__host__ __device__ constexpr int tile_rows(int nwx) { return nwx == 1 ? 8 : (nwx == 2 ? 4 : 2); }

// NWXC > 0: 3D, rows of exactly NWXC waves (compile-time LDS strides);
// NWXC = 0: 1D/2D, one row per workgroup, nwx from the geometry.
template <int NDIM, int STAGE, typename ST, int FORM, int NWXC>
__global__ void __launch_bounds__(NDIM == 3 ? 512 : 1024) stage_kernel(const StageArgs A) {
  constexpr int NV = NDIM + 2;
  constexpr int PL = NV + 3;          // face payload: U, P, c_tot, V_normal
  constexpr bool HS = (NDIM == 3);    // stacked y rows
  constexpr bool HM = (NDIM >= 2);    // marched last axis
  constexpr int DM = NDIM - 1;        // physical axis of the march
  constexpr int TS = HS ? tile_rows(NWXC) : 1;
  const Geometry& G = A.geo;
  const int nwx = HS ? NWXC : G.nwx;
  constexpr int NXPC = 64 * NWXC;     // 3D row pitch in LDS
  const int nxp = HS ? NXPC : 64 * nwx;

  extern __shared__ double lds[];
  const Carve C = carve(NDIM, TS, nwx);
  double* Urow = lds + C.urow;      // [NV][TS][nxp]
  double* Prow = lds + C.prow;      // [PL][TS][nxp]
  double* Frow = lds + C.frow;      // [NV][TS+1][nxp]
  double* seamU = lds + C.seamU;    // [TS][nwx][2][NV]
  double* seamUl = lds + C.seamUl;  // [TS][NV]
  double* seamM = lds + C.seamM;    // [TS][nwx][PL]
  double* seamP = lds + C.seamP;    // [TS][nwx][PL]
  double* seamPl = lds + C.seamPl;  // [TS][PL]
  double* seamF = lds + C.seamF;    // [TS][nwx+1][NV]
  double* red = lds + C.red;        // [16]

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
  const bool x_per = A.bc_lo[0] == 0;
  const int am = NDIM - 1;
  const int rm_lo = A.bc_lo[am], rm_hi = A.bc_hi[am];
  constexpr int SZ = (int)sizeof(ST);
  const int plane = G.nx * G.ns * SZ;              // bytes per march plane
  const int col = (j * G.nx + i) * SZ;             // this thread's column (bytes)
  const long long fbytes = (long long)NV * A.ncell * SZ;
  const int bgi_xy = (sizeof(ST) == 4) ? bg_index<NDIM>(A, i, j, 0) : 0;
  const bool bg_on_m = (sizeof(ST) == 4) && (A.bg_axis == am) && HM;
  auto bgk = [&](int kk) { return bg_on_m ? kk : bgi_xy; };

  const Consts K{A.gamma, A.gm1, A.inv_gm1, A.inv_xi, A.f};
  const double g[3] = {A.g[0], A.g[1], A.g[2]};
  const double hx = 0.5 * A.inv_dx[0], hy = 0.5 * A.inv_dx[1], hz = 0.5 * A.inv_dx[DM];
  const double dt = (A.dt_fixed > 0.0) ? A.dt_fixed : A.scal[kDtCur];
  const __amdgpu_buffer_rsrc_t uin = field_rsrc(A.uin, fbytes);
  const __amdgpu_buffer_rsrc_t unp = field_rsrc(A.un ? A.un : A.uin, fbytes);
  const __amdgpu_buffer_rsrc_t uout = field_rsrc(A.uout, fbytes);
  const int vstride = (int)(A.ncell * (long long)SZ);

  // y rows just outside the tile (3D): columns and mirror flags, once
  int clo1 = 0, clo2 = 0, chi1 = 0, chi2 = 0, nlo1 = -1, nlo2 = -1, nhi1 = -1, nhi2 = -1;
  int blo1 = 0, blo2 = 0, bhi1 = 0, bhi2 = 0;
  if constexpr (HS) {
    bool n;
    int jj;
    jj = map_index(j0 - 1, G.ns, A.bc_lo[1], A.bc_hi[1], n); nlo1 = n ? 2 : -1; clo1 = (jj * G.nx + i) * SZ;
    blo1 = (A.bg_axis == 1) ? jj : bgi_xy;
    jj = map_index(j0 - 2, G.ns, A.bc_lo[1], A.bc_hi[1], n); nlo2 = n ? 2 : -1; clo2 = (jj * G.nx + i) * SZ;
    blo2 = (A.bg_axis == 1) ? jj : bgi_xy;
    jj = map_index(j0 + ts_eff, G.ns, A.bc_lo[1], A.bc_hi[1], n); nhi1 = n ? 2 : -1; chi1 = (jj * G.nx + i) * SZ;
    bhi1 = (A.bg_axis == 1) ? jj : bgi_xy;
    jj = map_index(j0 + ts_eff + 1, G.ns, A.bc_lo[1], A.bc_hi[1], n); nhi2 = n ? 2 : -1; chi2 = (jj * G.nx + i) * SZ;
    bhi2 = (A.bg_axis == 1) ? jj : bgi_xy;
  }

  double q0[NV], q1[NV], sm0[NV], Fm_lo[NV];
  double cmax = 0.0;
  unsigned bad = 0;

  if constexpr (HM) {
    double qa[NV], qb[NV], ha[NV];
    bool n;
    int kk;
    kk = map_index(k0 - 2, G.nm, rm_lo, rm_hi, n);
    load_cell<NDIM, ST>(A, uin, kk * plane, col, n ? NDIM : -1, bgk(kk), qa);
    kk = map_index(k0 - 1, G.nm, rm_lo, rm_hi, n);
    load_cell<NDIM, ST>(A, uin, kk * plane, col, n ? NDIM : -1, bgk(kk), qb);
    load_cell<NDIM, ST>(A, uin, k0 * plane, col, -1, bgk(k0), q0);
    kk = map_index(k0 + 1, G.nm, rm_lo, rm_hi, n);
    load_cell<NDIM, ST>(A, uin, kk * plane, col, n ? NDIM : -1, bgk(kk), q1);
#pragma unroll
    for (int v = 0; v < NV; ++v) {
      ha[v] = mc_half(qb[v] - qa[v], q0[v] - qb[v]);
      sm0[v] = mc_half(q0[v] - qb[v], q1[v] - q0[v]);
    }
    Face<NV> fl, fr;
    make_face<NDIM, DM>(qb, ha, true, K, fl);
    make_face<NDIM, DM>(q0, sm0, false, K, fr);
    flux2<NDIM, DM>(fl, fr, Fm_lo);
  } else {
    load_cell<NDIM, ST>(A, uin, 0, col, -1, bgi_xy, q0);
  }

  for (int k = k0; k < k1; ++k) {
    const int koff = k * plane;
    // ---- loads for this iteration: the plane two ahead, the step-start state
    double q2[NV], un[NV];
    if constexpr (HM) {
      bool n;
      const int kk = map_index(k + 2, G.nm, rm_lo, rm_hi, n);
      load_cell<NDIM, ST>(A, uin, kk * plane, col, n ? NDIM : -1, bgk(kk), q2);
    }
    if constexpr (STAGE == 2) load_cell<NDIM, ST>(A, unp, koff, col, -1, bgk(k), un);

    // ---- P1: publish this plane's cell state
    if constexpr (HS) {
#pragma unroll
      for (int v = 0; v < NV; ++v) Urow[(v * TS + row) * nxp + i_raw] = q0[v];
    }
    {
      double* sw = seamU + ((row * nwx + wx) * 2) * NV;
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
        for (int v = 0; v < NV; ++v) seamUl[row * NV + v] = q0[v];
      }
    }
    __syncthreads();  // B1

    // ---- P2: x and y face states; lower x flux from the lane on the left
    double Fx_lo[NV];
    {
      double uL[NV], uR[NV], h[NV];
#pragma unroll
      for (int v = 0; v < NV; ++v) { uL[v] = from_left(q0[v]); uR[v] = from_right(q0[v]); }
      if (lane == 0) {
        if (wx > 0) {
          const double* sw = seamU + ((row * nwx + wx - 1) * 2 + 1) * NV;
#pragma unroll
          for (int v = 0; v < NV; ++v) uL[v] = sw[v];
        } else if (x_per) {
#pragma unroll
          for (int v = 0; v < NV; ++v) uL[v] = seamUl[row * NV + v];
        } else {
#pragma unroll
          for (int v = 0; v < NV; ++v) uL[v] = q0[v];
          uL[1] = -q0[1];
        }
      }
      if (last_x) {
        if (x_per) {
          const double* sw = seamU + ((row * nwx) * 2) * NV;
#pragma unroll
          for (int v = 0; v < NV; ++v) uR[v] = sw[v];
        } else {
#pragma unroll
          for (int v = 0; v < NV; ++v) uR[v] = q0[v];
          uR[1] = -q0[1];
        }
      } else if (lane == 63 && xin) {
        const double* sw = seamU + ((row * nwx + wx + 1) * 2) * NV;
#pragma unroll
        for (int v = 0; v < NV; ++v) uR[v] = sw[v];
      }
#pragma unroll
      for (int v = 0; v < NV; ++v) h[v] = mc_half(q0[v] - uL[v], uR[v] - q0[v]);
      Face<NV> fm, fp;
      make_face<NDIM, 0>(q0, h, false, K, fm);
      make_face<NDIM, 0>(q0, h, true, K, fp);
      // the wave-edge faces are redone after the barrier from the seams
      if (lane == 0) put_face(seamM + (row * nwx + wx) * PL, 1, fm);
      if (lane == 63) put_face(seamP + (row * nwx + wx) * PL, 1, fp);
      if (last_x) put_face(seamPl + row * PL, 1, fp);
      const Face<NV> pl = face_from_left(fp);
      flux2<NDIM, 0>(pl, fm, Fx_lo);
    }
    Face<NV> fym;
    if constexpr (HS) {
      double uD[NV], uU[NV], h[NV];
      if (first_row) {
        load_cell<NDIM, ST>(A, uin, koff, clo1, nlo1, bg_on_m ? k : blo1, uD);
      } else {
#pragma unroll
        for (int v = 0; v < NV; ++v) uD[v] = Urow[(v * TS + row - 1) * nxp + i_raw];
      }
      if (last_row) {
        load_cell<NDIM, ST>(A, uin, koff, chi1, nhi1, bg_on_m ? k : bhi1, uU);
      } else {
        const int ru = min(row + 1, TS - 1);  // idle rows past the tile read in range
#pragma unroll
        for (int v = 0; v < NV; ++v) uU[v] = Urow[(v * TS + ru) * nxp + i_raw];
      }
#pragma unroll
      for (int v = 0; v < NV; ++v) h[v] = mc_half(q0[v] - uD[v], uU[v] - q0[v]);
      {
        Face<NV> fyp;
        make_face<NDIM, 1>(q0, h, true, K, fyp);
        put_face(Prow + row * nxp + i_raw, TS * nxp, fyp);
        if (last_row) {
          // minus state of the row above the tile, and the flux at the
          // tile's upper face
          double u2[NV], hh[NV], Fh[NV];
          load_cell<NDIM, ST>(A, uin, koff, chi2, nhi2, bg_on_m ? k : bhi2, u2);
#pragma unroll
          for (int v = 0; v < NV; ++v) hh[v] = mc_half(uU[v] - q0[v], u2[v] - uU[v]);
          Face<NV> fh;
          make_face<NDIM, 1>(uU, hh, false, K, fh);
          flux2<NDIM, 1>(fyp, fh, Fh);
#pragma unroll
          for (int v = 0; v < NV; ++v) Frow[(v * (TS + 1) + ts_eff) * nxp + i_raw] = Fh[v];
        }
      }
      make_face<NDIM, 1>(q0, h, false, K, fym);
      if (first_row) {
        // plus state of the row below the tile, and the flux at the tile's
        // lower face
        double u2[NV], hh[NV], Fh[NV];
        load_cell<NDIM, ST>(A, uin, koff, clo2, nlo2, bg_on_m ? k : blo2, u2);
#pragma unroll
        for (int v = 0; v < NV; ++v) hh[v] = mc_half(uD[v] - u2[v], q0[v] - uD[v]);
        Face<NV> fh;
        make_face<NDIM, 1>(uD, hh, true, K, fh);
        flux2<NDIM, 1>(fh, fym, Fh);
#pragma unroll
        for (int v = 0; v < NV; ++v) Frow[(v * (TS + 1)) * nxp + i_raw] = Fh[v];
      }
    }
    __syncthreads();  // B2

    // ---- P3: x fluxes at the wave edges (lanes 0..nwx of wave 0 of each
    // row), y fluxes at the faces inside the tile
    if (wx == 0 && lane <= nwx) {
      const int e = lane;  // face at the left edge of wave e (e = nwx: row end)
      Face<NV> fl, fr;
      if (e == 0) {
        get_face(seamM + (row * nwx) * PL, 1, fr);
        if (x_per) get_face(seamPl + row * PL, 1, fl);
        else fl = mirror<NDIM, 0>(fr);
      } else if (e == nwx) {
        get_face(seamPl + row * PL, 1, fl);
        if (x_per) get_face(seamM + (row * nwx) * PL, 1, fr);
        else fr = mirror<NDIM, 0>(fl);
      } else {
        get_face(seamP + (row * nwx + e - 1) * PL, 1, fl);
        get_face(seamM + (row * nwx + e) * PL, 1, fr);
      }
      double Fe[NV];
      flux2<NDIM, 0>(fl, fr, Fe);
#pragma unroll
      for (int v = 0; v < NV; ++v) seamF[(row * (nwx + 1) + e) * NV + v] = Fe[v];
    }
    if constexpr (HS) {
      if (row >= 1 && row < ts_eff) {
        Face<NV> pd;
        double Fy[NV];
        get_face(Prow + (row - 1) * nxp + i_raw, TS * nxp, pd);
        flux2<NDIM, 1>(pd, fym, Fy);
#pragma unroll
        for (int v = 0; v < NV; ++v) Frow[(v * (TS + 1) + row) * nxp + i_raw] = Fy[v];
      }
    }
    __syncthreads();  // B3

    // ---- P4: divergence, march face, correction, update
    double Dl[NV];
    {
      double Fx_hi[NV];
#pragma unroll
      for (int v = 0; v < NV; ++v) Fx_hi[v] = from_right(Fx_lo[v]);
      if (lane == 0) {
#pragma unroll
        for (int v = 0; v < NV; ++v) Fx_lo[v] = seamF[(row * (nwx + 1) + wx) * NV + v];
      }
      if (last_x) {
#pragma unroll
        for (int v = 0; v < NV; ++v) Fx_hi[v] = seamF[(row * (nwx + 1) + nwx) * NV + v];
      } else if (lane == 63 && xin) {
#pragma unroll
        for (int v = 0; v < NV; ++v) Fx_hi[v] = seamF[(row * (nwx + 1) + wx + 1) * NV + v];
      }
#pragma unroll
      for (int v = 0; v < NV; ++v) Dl[v] = -(Fx_hi[v] - Fx_lo[v]) * hx;
    }
    if constexpr (HS) {
      const int ru = min(row + 1, TS);
#pragma unroll
      for (int v = 0; v < NV; ++v) {
        const double lo = Frow[(v * (TS + 1) + row) * nxp + i_raw];
        const double hi = Frow[(v * (TS + 1) + ru) * nxp + i_raw];
        Dl[v] = fma(-(hi - lo), hy, Dl[v]);
      }
    }
    if constexpr (HM) {
      double sm1[NV], Fm_hi[NV];
#pragma unroll
      for (int v = 0; v < NV; ++v) sm1[v] = mc_half(q1[v] - q0[v], q2[v] - q1[v]);
      Face<NV> fl, fr;
      make_face<NDIM, DM>(q0, sm0, true, K, fl);
      make_face<NDIM, DM>(q1, sm1, false, K, fr);
      flux2<NDIM, DM>(fl, fr, Fm_hi);
#pragma unroll
      for (int v = 0; v < NV; ++v) {
        Dl[v] = fma(-(Fm_hi[v] - Fm_lo[v]), hz, Dl[v]);
        Fm_lo[v] = Fm_hi[v];
        sm0[v] = sm1[v];
      }
    }
    double R[NV];
    const unsigned b = rsst_rate<NDIM, FORM>(q0, Dl, K, g, R);
    if (active) {
      bad |= b;
      const int bk = bgk(k);
      double out[NV];
#pragma unroll
      for (int v = 0; v < NV; ++v) {
        double y = fma(dt, R[v], q0[v]);
        if constexpr (STAGE == 2) y = 0.5 * (un[v] + y);
        const double bgv = (sizeof(ST) == 4) ? A.bg[v * A.nbg + bk] : 0.0;
        const ST st = (ST)(y - bgv);
        buf_store<ST>(uout, col, koff + v * vstride, st);
        out[v] = (double)st + bgv;
      }
      if constexpr (STAGE == 2) cmax = fmax(cmax, cell_ctot<NDIM>(out, K));
    }
    if constexpr (HM) {
#pragma unroll
      for (int v = 0; v < NV; ++v) { q0[v] = q1[v]; q1[v] = q2[v]; }
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

Geometry plan_geometry(int ndim, const int n[3]) {
  Geometry G{};
  G.ndim = ndim;
  G.nx = n[0];
  G.ns = (ndim == 3) ? n[1] : 1;
  G.nm = (ndim == 3) ? n[2] : (ndim == 2 ? n[1] : 1);
  G.nwx = (G.nx + 63) / 64;
  if (ndim == 3) {
    G.ts = tile_rows(G.nwx);
  } else {
    G.ts = 1;
  }
  G.ntile_s = (G.ns + G.ts - 1) / G.ts;
  if (ndim == 1) {
    G.km = 1;
  } else {
    // at least two workgroups per CU (256 CUs), chunks of 8 to 64 planes
    // (each chunk re-reads 4 planes to start its march); RSST_KM overrides
    // the chunk length (tuning)
    int km = 64;
    while (km > 8 && (long long)G.ntile_s * ((G.nm + km - 1) / km) < 512) km >>= 1;
    if (const char* e = getenv("RSST_KM")) {
      const int v = atoi(e);
      if (v >= 4 && v <= 4096) km = v;
    }
    G.km = km < G.nm ? km : G.nm;
  }
  G.nchunk = (G.nm + G.km - 1) / G.km;
  G.threads = 64 * G.nwx * G.ts;
  G.lds_bytes = (size_t)carve(ndim, G.ts, G.nwx).total * sizeof(double);
  return G;
}

template <int NDIM, int STAGE, typename ST, int FORM, int NWXC>
static hipError_t launch_stage_k(const StageArgs& a, hipStream_t s) {
  const Geometry& G = a.geo;
  const dim3 grid((unsigned)(G.ntile_s * G.nchunk)), block((unsigned)G.threads);
  auto kern = stage_kernel<NDIM, STAGE, ST, FORM, NWXC>;
  hipError_t e = hipFuncSetAttribute((const void*)kern, hipFuncAttributeMaxDynamicSharedMemorySize,
                                     (int)G.lds_bytes);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(kern, grid, block, G.lds_bytes, s, a);
  return hipGetLastError();
}

template <int NDIM, int STAGE, typename ST, int FORM>
static hipError_t launch_stage_t(const StageArgs& a, hipStream_t s) {
  if constexpr (NDIM == 3) {
    switch (a.geo.nwx) {
      case 1: return launch_stage_k<NDIM, STAGE, ST, FORM, 1>(a, s);
      case 2: return launch_stage_k<NDIM, STAGE, ST, FORM, 2>(a, s);
      case 3: return launch_stage_k<NDIM, STAGE, ST, FORM, 3>(a, s);
      default: return launch_stage_k<NDIM, STAGE, ST, FORM, 4>(a, s);
    }
  } else {
    return launch_stage_k<NDIM, STAGE, ST, FORM, 0>(a, s);
  }
}

template <int NDIM, int STAGE, typename ST>
static hipError_t launch_stage_f(const StageArgs& a, hipStream_t s) {
  switch (a.form) {
    case kEuler: return launch_stage_t<NDIM, STAGE, ST, kEuler>(a, s);
    case kPVS: return launch_stage_t<NDIM, STAGE, ST, kPVS>(a, s);
    case kPMS: return launch_stage_t<NDIM, STAGE, ST, kPMS>(a, s);
    case kDVS: return launch_stage_t<NDIM, STAGE, ST, kDVS>(a, s);
    case kDMS: return launch_stage_t<NDIM, STAGE, ST, kDMS>(a, s);
    default: return launch_stage_t<NDIM, STAGE, ST, kPD>(a, s);
  }
}

template <int NDIM, typename ST>
static hipError_t launch_stage_n(const StageArgs& a, int stage, hipStream_t s) {
  return stage == 1 ? launch_stage_f<NDIM, 1, ST>(a, s) : launch_stage_f<NDIM, 2, ST>(a, s);
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
