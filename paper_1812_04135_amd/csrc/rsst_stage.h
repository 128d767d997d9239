// Device code of one RSST stage over a tile, shared by the per-grid kernels
// (rsst_kernels.hip) and the batched persistent kernel (rsst_batch.hip).
// The decomposition is described in rsst_kernels.hip.
#pragma once

#include <type_traits>

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

// Hydrostatic closed wall (bc 2): the ghost at raw index q (outside [0, n))
// mirrors cell k and carries its pressure to the ghost centre along the
// external force, P_g = P_k + rho_k g (x_g - x_k); returns (x_g - x_k) g,
// 0 for any other cell or wall.  x_g - x_k = (2q + 1) dx below the domain
// (q = -1 - k) and (2(q - n) + 1) dx above it.
__device__ __forceinline__ double hydro_lever(int q, int n, int bc_lo, int bc_hi, double dx, double g) {
  if (q < 0) return bc_lo == 2 ? (2.0 * q + 1.0) * dx * g : 0.0;
  if (q >= n) return bc_hi == 2 ? (2.0 * (q - n) + 1.0) * dx * g : 0.0;
  return 0.0;
}

// Raw buffer access: a resource built in scalar registers (base and range,
// see Field32 and Field64) and a loop-invariant per-thread byte offset in a
// VGPR (the column), so no vector address arithmetic.
typedef unsigned int u32x2_t __attribute__((ext_vector_type(2)));

__device__ __forceinline__ __amdgpu_buffer_rsrc_t field_rsrc(const void* p, long long bytes) {
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(p), (short)0, (int)bytes, 0x00020000);
}

// A state: nvar arrays of ncell values, read and written one plane (3D: an
// x-y plane; 2D: a row) and one variable at a time.  Two addressings, the
// same accesses:
//  Field32 (states below 2 GiB): one resource for the whole state and a
//    workgroup-uniform 32-bit offset (plane and variable) in an SGPR;
//  Field64 (any size): per access a resource whose 64-bit base is that plane
//    of that variable and whose range is the plane, so no offset the hardware
//    adds exceeds a plane.  Its scalar address arithmetic costs the 3D kernels
//    about 2%, so the library uses it only for states of 2 GiB or more.
struct Field32 {
  __amdgpu_buffer_rsrc_t r;
  int vbytes;  // bytes of one variable's array
  int pbytes;  // bytes of one plane
  __device__ __forceinline__ __amdgpu_buffer_rsrc_t rsrc(int, int) const { return r; }
  __device__ __forceinline__ int soff(int v, int k) const { return k * pbytes + v * vbytes; }
};

struct Field64 {
  const char* p;     // variable 0, plane 0
  long long vbytes;  // bytes of one variable's array
  int pbytes;        // bytes of one plane
  __device__ __forceinline__ __amdgpu_buffer_rsrc_t rsrc(int v, int k) const {
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<char*>(p + v * vbytes + (long long)k * pbytes), (short)0,
                                             pbytes, 0x00020000);
  }
  __device__ __forceinline__ int soff(int, int) const { return 0; }
};

template <bool BIG>
using FieldT = typename std::conditional<BIG, Field64, Field32>::type;

template <bool BIG>
__device__ __forceinline__ FieldT<BIG> make_field(const void* p, long long ncell, int nv, int sz, int pbytes) {
  if constexpr (BIG) {
    return Field64{(const char*)p, ncell * sz, pbytes};
  } else {
    return Field32{field_rsrc(p, (long long)nv * ncell * sz), (int)(ncell * sz), pbytes};
  }
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

// Cache policy of the 3D stage outputs and of the pointwise step-start reads:
// non-temporal (2), since neither is read again within the stage and a 3D
// state is larger than the caches; the halo reads keep the default policy, so
// L2 holds the rows that neighbouring tiles share (256^3 FP64: 21% fewer
// stage-2 HBM reads).  1D and 2D grids, and the batch, whose states are
// re-read from L2/MALL by the next stage, keep the default policy.
constexpr int kStoreAux3 = 2;  // 3D stage outputs: non-temporal
constexpr int kUnAux3 = 2;     // 3D stage 2's pointwise step-start reads: non-temporal

template <typename ST, int AUX = 0>
__device__ __forceinline__ void buf_store(__amdgpu_buffer_rsrc_t r, int voff, int soff, ST x) {
  if constexpr (sizeof(ST) == 8) {
    u32x2_t v;
    v.x = (unsigned)__double2loint(x);
    v.y = (unsigned)__double2hiint(x);
    __builtin_amdgcn_raw_buffer_store_b64(v, r, voff, soff, AUX);
  } else {
    __builtin_amdgcn_raw_buffer_store_b32(__float_as_uint(x), r, voff, soff, AUX);
  }
}

// The stored values of a cell, as loaded (no conversion): the loads can be
// issued early and their results used a phase later, with no wait in between.
template <typename ST, int AUX = 0>
__device__ __forceinline__ ST buf_load_raw(__amdgpu_buffer_rsrc_t r, int voff, int soff) {
  if constexpr (sizeof(ST) == 8) {
    const u32x2_t v = __builtin_amdgcn_raw_buffer_load_b64(r, voff, soff, AUX);
    return __hiloint2double((int)v.y, (int)v.x);
  } else {
    return __uint_as_float(__builtin_amdgcn_raw_buffer_load_b32(r, voff, soff, AUX));
  }
}

// The stored values of the cell at column byte offset voff of plane k.
template <int NDIM, typename ST, int AUX = 0, typename F>
__device__ __forceinline__ void load_cell_raw(const F& f, int k, int voff, ST (&raw)[NDIM + 2]) {
#pragma unroll
  for (int v = 0; v < NDIM + 2; ++v) raw[v] = buf_load_raw<ST, AUX>(f.rsrc(v, k), voff, f.soff(v, k));
}

// FP64 cell state from its stored values: widening and background (FP32
// perturbation form, b its index), then the mirror negation of momentum
// component `negv` (>= 0) for a ghost across a wall, and for a hydrostatic
// wall's ghost (lever = (x_g - x_k) g != 0) the energy of the carried
// pressure, E + rho lever (de/dP)_rho (rho and |V| unchanged).
template <int NDIM, typename ST>
__device__ __forceinline__ void finish_cell(const StageArgs& A, const ST (&raw)[NDIM + 2], int negv, int b,
                                            double (&u)[NDIM + 2], double lever = 0.0) {
  constexpr int NV = NDIM + 2;
#pragma unroll
  for (int v = 0; v < NV; ++v) u[v] = (double)raw[v];
  if constexpr (sizeof(ST) == 4) {
    // background along the march axis (or uniform): b is the same for the
    // whole workgroup, read through the scalar cache; otherwise per lane
    if (A.bg_uniform) {
      const int bu = __builtin_amdgcn_readfirstlane(b);
#pragma unroll
      for (int v = 0; v < NV; ++v) u[v] += A.bg[v * A.nbg + bu];
    } else {
#pragma unroll
      for (int v = 0; v < NV; ++v) u[v] += A.bg[v * A.nbg + b];
    }
  }
#pragma unroll
  for (int v = 1; v <= NDIM; ++v)
    if (v == negv) u[v] = -u[v];
  if (lever != 0.0) {
    const double dedp = A.eos ? (1.0 - A.vdw_b * u[0]) * A.inv_gm1 : A.inv_gm1;
    u[NDIM + 1] = u[NDIM + 1] + u[0] * lever * dedp;
  }
}

// FP64 cell state from its stored values with the background values bgv
// already in registers (FP32 perturbation form), then the mirror sign.
template <int NDIM, typename ST>
__device__ __forceinline__ void finish_cell_bgv(const ST (&raw)[NDIM + 2], int negv, const double (&bgv)[NDIM + 2],
                                                double (&u)[NDIM + 2]) {
#pragma unroll
  for (int v = 0; v < NDIM + 2; ++v) u[v] = (double)raw[v] + bgv[v];
#pragma unroll
  for (int v = 1; v <= NDIM; ++v)
    if (v == negv) u[v] = -u[v];
}

// The NV background values at profile index idx, as vector loads (their
// wait falls where they are used, not on the LDS counter).
template <int NV>
__device__ __forceinline__ void load_bg(__amdgpu_buffer_rsrc_t r, int nbg, int idx, double (&b)[NV]) {
#pragma unroll
  for (int v = 0; v < NV; ++v) {
    const u32x2_t x = __builtin_amdgcn_raw_buffer_load_b64(r, (v * nbg + idx) * 8, 0, 0);
    b[v] = __hiloint2double((int)x.y, (int)x.x);
  }
}

// Cell state at plane k (workgroup-uniform) and column byte offset voff
// (the thread's) as FP64; `negv` >= 0 names a momentum component to negate
// (mirror ghost); b: background index (FP32 perturbation form).
template <int NDIM, typename ST, typename F>
__device__ __forceinline__ void load_cell(const StageArgs& A, const F& f, int k, int voff, int negv, int b,
                                          double (&u)[NDIM + 2], double lever = 0.0) {
  ST raw[NDIM + 2];
  load_cell_raw<NDIM, ST>(f, k, voff, raw);
  finish_cell<NDIM, ST>(A, raw, negv, b, u, lever);
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

// LDS carve-up of one workgroup (doubles).  3D only: Urow, Prow, Mrow, Frow.
struct Carve {
  int urow, prow, mrow, frow, seamU, seamUl, seamM, seamP, seamPl, red, total;
};

__host__ __device__ inline Carve carve(int ndim, int ts, int nwx) {
  const int NV = ndim + 2, PL = NV + 3, nxp = 64 * nwx;
  Carve c;
  int o = 0;
  c.urow = o;   if (ndim == 3) o += NV * ts * nxp;        // cell states, per row
  // the y face states that another row of the tile reads: the plus state of
  // every row but the last, the minus state of every row but the first
  c.prow = o;   if (ndim == 3) o += PL * (ts - 1) * nxp;
  c.mrow = o;   if (ndim == 3) o += PL * (ts - 1) * nxp;
  c.frow = o;   if (ndim == 3) o += NV * 2 * nxp;         // y fluxes at the tile's two outer faces
  c.seamU = o;  o += ts * nwx * 2 * NV;                   // lane 0 / lane 63 cell states
  c.seamUl = o; o += ts * NV;                             // last cell of each row
  c.seamM = o;  o += ts * nwx * PL;                       // lane 0 minus-face states
  c.seamP = o;  o += ts * nwx * PL;                       // lane 63 plus-face states
  c.seamPl = o; o += ts * PL;                             // last cell's plus-face state
  c.red = o;    o += 16;
  c.total = o;
  return c;
}

// Rows per 3D tile for a row of nwx waves (512 threads at most).  Rows of
// 257-512 cells run as rows of 8 waves, one row per tile.
__host__ __device__ constexpr int tile_rows(int nwx) {
  return nwx == 1 ? 8 : (nwx == 2 ? 4 : (nwx <= 4 ? 2 : 1));
}

// A 1D cell kept in registers across stages (steps1d_kernel): the stage
// input, the step-start state, the output, and the output's stored value
// (widened).  in and un hold exactly what loading the stored values would
// give, so the results are those of the stored path.
template <int NV>
struct RegCell {
  double in[NV], un[NV], out[NV], st[NV];
};

// One stage of R over one tile (3D: TS stacked y rows of one z-chunk) or one
// group of strips (1D/2D: row r of the workgroup marches chunk
// chunk_base + r), returning the thread's largest c_tot of the stage-2
// output (0 in stage 1) and or-ing non-physical flags into `bad`.
// NWXC > 0: 3D, rows of exactly NWXC waves (compile-time LDS strides);
// NWXC = 0: 1D/2D, nwx and the number of row groups from the geometry.
// Every row of the workgroup runs the same number of march iterations
// (G.km), so rows of different chunks share the workgroup's barriers.
// BIG: Field64 addressing (3D states of 2 GiB or more).  REG (1D): the
// thread's cell comes from and goes to *rc instead of global memory.
template <int NDIM, int STAGE, typename ST, int FORMX, int NWXC, bool BIG = false, bool REG = false>
__device__ __forceinline__ double stage_body(const StageArgs& A, double* lds, int tile_s,
                                             int chunk_base, double dt, unsigned& bad,
                                             RegCell<NDIM + 2>* rc = nullptr) {
  static_assert(!REG || NDIM == 1, "register-resident cells: 1D only");
  constexpr int FORM = FORMX & 7;     // correction form
  constexpr int EXT = FORMX & (kExtCmax | kExtVdw);  // xi from eq. cx; van der Waals gas
  constexpr bool HYD = (FORMX & kExtHydro) != 0;     // hydrostatic walls (y, march axis)
  constexpr int NV = NDIM + 2;
  constexpr int PL = NV + 3;          // face payload: U, P, c_tot, V_normal
  constexpr bool HS = (NDIM == 3);    // stacked y rows
  constexpr bool HM = (NDIM >= 2);    // marched last axis
  constexpr int DM = NDIM - 1;        // physical axis of the march
  constexpr int TSC = HS ? tile_rows(NWXC) : 1;
  const Geometry& G = A.geo;
  const int TS = HS ? TSC : G.ts;
  const int nwx = HS ? NWXC : G.nwx;
  constexpr int NXPC = 64 * NWXC;     // 3D row pitch in LDS
  const int nxp = HS ? NXPC : 64 * nwx;

  const Carve C = carve(NDIM, TS, nwx);
  double* Urow = lds + C.urow;      // [NV][TS][nxp]
  double* Prow = lds + C.prow;      // [PL][TS-1][nxp], slot r: row r
  double* Mrow = lds + C.mrow;      // [PL][TS-1][nxp], slot r: row r + 1
  double* Frow = lds + C.frow;      // [NV][2][nxp]: lower and upper outer face
  const int PS = (TS - 1) * nxp;    // stride of one payload value in Prow, Mrow
  double* seamU = lds + C.seamU;    // [TS][nwx][2][NV]
  double* seamUl = lds + C.seamUl;  // [TS][NV]
  double* seamM = lds + C.seamM;    // [TS][nwx][PL]
  double* seamP = lds + C.seamP;    // [TS][nwx][PL]
  double* seamPl = lds + C.seamPl;  // [TS][PL]

  const int tid = threadIdx.x, lane = tid & 63;
  const int w = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int wx = w % nwx, row_raw = w / nwx;
  const int i_raw = wx * 64 + lane;

  // waves past the last full row group (a row of 3 waves in a 4-wave
  // workgroup) only take part in the barriers
  const bool wave_idle = w >= nwx * TS;
  const int row = wave_idle ? 0 : row_raw;  // idle waves read row 0's slots
  // 3D: the tile stores rows [tile_s TS, tile_s TS + TS).  The last tile of a
  // column whose height is not a multiple of TS is moved down to end at the
  // last row: its rows below tile_s TS belong to the tile before it and are
  // computed (the same bits, as every face is formed from the same face
  // states) but not stored.  So a tile holds min(TS, ns) >= 2 rows whenever
  // TS >= 2 (ns >= 4), and its first and last rows are distinct rows that
  // both read their outside rows a plane ahead.
  const int j_own = HS ? tile_s * TS : 0;
  const int j0 = HS ? min(j_own, max(G.ns - TS, 0)) : 0;
  const int ts_eff = HS ? min(TS, G.ns - j0) : TS;
  const bool xin = i_raw < G.nx;
  const int chunk = HS ? chunk_base : chunk_base + row;
  const int k0 = chunk * G.km;
  const int k1 = min(k0 + G.km, G.nm);
  const bool active = xin && row < ts_eff && k0 < G.nm && !wave_idle && j0 + row >= j_own;
  const int i = xin ? i_raw : G.nx - 1;
  const int j = HS ? j0 + min(row, ts_eff - 1) : 0;
  const bool last_x = (i_raw == G.nx - 1);
  const bool first_row = HS && row == 0;
  const bool last_row = HS && row == ts_eff - 1;
  const bool x_per = A.bc_lo[0] == 0;
  const int am = NDIM - 1;
  const int rm_lo = A.bc_lo[am], rm_hi = A.bc_hi[am];
  constexpr int SZ = (int)sizeof(ST);
  const int plane = G.nx * G.ns * SZ;              // bytes per march plane
  const int col = (j * G.nx + i) * SZ;             // this thread's column (bytes)
  const int bgi_xy = (sizeof(ST) == 4 && !A.bg_uniform) ? bg_index<NDIM>(A, i, j, 0) : 0;
  const bool bg_on_m = (sizeof(ST) == 4) && (A.bg_axis == am) && HM;
  auto bgk = [&](int kk) { return bg_on_m ? kk : bgi_xy; };
  // FP32 perturbation form: the background in registers.  Along the march
  // axis: bgA holds plane k and bgB the plane two ahead, loaded at the top of
  // each plane; otherwise (uniform, along x, along y) bgA holds this cell's
  // values for the whole march.  Rows outside a 3D tile with a profile
  // along y take the indexed path.
  constexpr bool F32 = sizeof(ST) == 4;
  const bool bg_rows = F32 && HS && A.bg_axis == 1;
  double bgA[NV], bgB[NV];
  const __amdgpu_buffer_rsrc_t bgr = field_rsrc(A.bg, F32 ? (long long)NV * A.nbg * 8 : 0);
  if constexpr (F32) {
    const int ib = A.bg_uniform ? 0 : bg_index<NDIM>(A, i, j, 0);
    if (!bg_on_m) load_bg<NV>(bgr, A.nbg, ib, bgA);
  }

  const Consts K{A.gamma, A.gm1, A.inv_gm1, A.inv_xi, A.f, A.inv_cmax2, A.vdw_a, A.vdw_b};
  const double g[3] = {A.g[0], A.g[1], A.g[2]};
  const double hx = 0.5 * A.inv_dx[0], hy = 0.5 * A.inv_dx[1], hz = 0.5 * A.inv_dx[DM];
  const FieldT<BIG> uin = make_field<BIG>(A.uin, A.ncell, NV, SZ, plane);
  const FieldT<BIG> unp = make_field<BIG>(A.un ? A.un : A.uin, A.ncell, NV, SZ, plane);
  // stage 2 writes the new state in place over the step-start state (the
  // callers pass uout == un), so one field serves both
  const FieldT<BIG> uout = STAGE == 2 ? unp : make_field<BIG>(A.uout, A.ncell, NV, SZ, plane);

  // y rows just outside the tile (3D): columns and mirror flags, once
  int clo1 = 0, clo2 = 0, chi1 = 0, chi2 = 0, nlo1 = -1, nlo2 = -1, nhi1 = -1, nhi2 = -1;
  int blo1 = 0, blo2 = 0, bhi1 = 0, bhi2 = 0;
  double llo1 = 0.0, llo2 = 0.0, lhi1 = 0.0, lhi2 = 0.0;  // hydrostatic wall levers
  if constexpr (HS) {
    bool n;
    int jj;
    if constexpr (HYD) {
      const double dy = A.dx[1], gy = A.g[1];
      const int bl = A.bc_lo[1], bh = A.bc_hi[1];
      llo1 = hydro_lever(j0 - 1, G.ns, bl, bh, dy, gy);
      llo2 = hydro_lever(j0 - 2, G.ns, bl, bh, dy, gy);
      lhi1 = hydro_lever(j0 + ts_eff, G.ns, bl, bh, dy, gy);
      lhi2 = hydro_lever(j0 + ts_eff + 1, G.ns, bl, bh, dy, gy);
    }
    jj = map_index(j0 - 1, G.ns, A.bc_lo[1], A.bc_hi[1], n); nlo1 = n ? 2 : -1; clo1 = (jj * G.nx + i) * SZ;
    blo1 = (A.bg_axis == 1) ? jj : bgi_xy;
    jj = map_index(j0 - 2, G.ns, A.bc_lo[1], A.bc_hi[1], n); nlo2 = n ? 2 : -1; clo2 = (jj * G.nx + i) * SZ;
    blo2 = (A.bg_axis == 1) ? jj : bgi_xy;
    jj = map_index(j0 + ts_eff, G.ns, A.bc_lo[1], A.bc_hi[1], n); nhi1 = n ? 2 : -1; chi1 = (jj * G.nx + i) * SZ;
    bhi1 = (A.bg_axis == 1) ? jj : bgi_xy;
    jj = map_index(j0 + ts_eff + 1, G.ns, A.bc_lo[1], A.bc_hi[1], n); nhi2 = n ? 2 : -1; chi2 = (jj * G.nx + i) * SZ;
    bhi2 = (A.bg_axis == 1) ? jj : bgi_xy;
  }
  // The edge rows read the two rows outside their side of the tile one
  // plane ahead, so their load latency hides behind a whole plane of work:
  // o1, o2 hold the near and far outside rows of the wave's side (one-row
  // tiles, where a row is both edges: o1, o2 below and o3, o4 above).  The
  // rows between the edges issue the same loads (the rows above the tile,
  // unused), so every wave has the same loads in flight at every point of
  // the march: loads complete in order, and a wait sized for a wave with
  // fewer loads in flight would make the edge rows wait for the loads of
  // the next plane.  For the same reason no load inside the march is
  // consumed in the phase that issues it.
  constexpr bool ONE = HS && TSC == 1;
  constexpr bool pre = HS;
  const bool o_lo = first_row;  // o1, o2 are the rows below (else above)
  const int oc1 = o_lo ? clo1 : chi1, oc2 = o_lo ? clo2 : chi2;
  const int on1 = o_lo ? nlo1 : nhi1, on2 = o_lo ? nlo2 : nhi2;
  const int ob1 = o_lo ? blo1 : bhi1, ob2 = o_lo ? blo2 : bhi2;
  const double ol1 = o_lo ? llo1 : lhi1, ol2 = o_lo ? llo2 : lhi2;
  ST o1[NV], o2[NV], o3[ONE ? NV : 1], o4[ONE ? NV : 1];  // stored values, finished at use

  double q0[NV], q1[NV], sm0[NV], Fm_lo[NV];
  double cmax = 0.0;
  const int k0l = min(k0, G.nm - 1);  // rows past the grid march in range

  if constexpr (HM) {
    double qa[NV], qb[NV], ha[NV];
    bool n;
    int kk;
    kk = map_index(k0l - 2, G.nm, rm_lo, rm_hi, n);
    load_cell<NDIM, ST>(A, uin, kk, col, n ? NDIM : -1, bgk(kk), qa,
                        HYD ? hydro_lever(k0l - 2, G.nm, rm_lo, rm_hi, A.dx[am], A.g[am]) : 0.0);
    kk = map_index(k0l - 1, G.nm, rm_lo, rm_hi, n);
    load_cell<NDIM, ST>(A, uin, kk, col, n ? NDIM : -1, bgk(kk), qb,
                        HYD ? hydro_lever(k0l - 1, G.nm, rm_lo, rm_hi, A.dx[am], A.g[am]) : 0.0);
    load_cell<NDIM, ST>(A, uin, k0l, col, -1, bgk(k0l), q0);
    kk = map_index(k0l + 1, G.nm, rm_lo, rm_hi, n);
    load_cell<NDIM, ST>(A, uin, kk, col, n ? NDIM : -1, bgk(kk), q1,
                        HYD ? hydro_lever(k0l + 1, G.nm, rm_lo, rm_hi, A.dx[am], A.g[am]) : 0.0);
#pragma unroll
    for (int v = 0; v < NV; ++v) {
      ha[v] = mc_half(qb[v] - qa[v], q0[v] - qb[v]);
      sm0[v] = mc_half(q0[v] - qb[v], q1[v] - q0[v]);
    }
    Face<NV> fl, fr;
    make_face<NDIM, DM, EXT>(qb, ha, true, K, fl);
    make_face<NDIM, DM, EXT>(q0, sm0, false, K, fr);
    flux2<NDIM, DM>(fl, fr, Fm_lo);
  } else if constexpr (REG) {
#pragma unroll
    for (int v = 0; v < NV; ++v) q0[v] = rc->in[v];
  } else {
    load_cell<NDIM, ST>(A, uin, 0, col, -1, bgi_xy, q0);
  }
  if constexpr (pre) {
    load_cell_raw<NDIM, ST>(uin, k0l, oc1, o1);
    load_cell_raw<NDIM, ST>(uin, k0l, oc2, o2);
    if constexpr (ONE) {
      load_cell_raw<NDIM, ST>(uin, k0l, chi1, o3);
      load_cell_raw<NDIM, ST>(uin, k0l, chi2, o4);
    }
  }

  for (int it = 0; it < G.km; ++it) {
    const int kraw = k0 + it;
    const bool kval = kraw < k1;
    const int k = min(kraw, G.nm - 1);  // plane used for loads and stores
    // ---- loads for this iteration: the plane two ahead, the step-start state
    // (stored values now, finished where first used, so the loads overlap
    // this plane's work)
    ST q2r[NV], unr[NV];
    int q2k = 0, q2neg = -1;
    double q2lev = 0.0;
    if constexpr (HM) {
      bool n;
      q2k = map_index(min(kraw, G.nm - 1) + 2, G.nm, rm_lo, rm_hi, n);
      q2neg = n ? NDIM : -1;
      if constexpr (HYD) q2lev = hydro_lever(min(kraw, G.nm - 1) + 2, G.nm, rm_lo, rm_hi, A.dx[am], A.g[am]);
    }
    // the background rows first: plane k's is used earliest (P2)
    if constexpr (F32) {
      if (bg_on_m) {
        load_bg<NV>(bgr, A.nbg, k, bgA);
        load_bg<NV>(bgr, A.nbg, q2k, bgB);
      }
    }
    if constexpr (HM) load_cell_raw<NDIM, ST>(uin, q2k, col, q2r);
    if constexpr (STAGE == 2 && !REG) load_cell_raw<NDIM, ST, HS ? kUnAux3 : 0>(unp, k, col, unr);

    // ---- P1: publish this plane's cell state
    if constexpr (HS) {
#pragma unroll
      for (int v = 0; v < NV; ++v) Urow[(v * TS + row) * nxp + i_raw] = q0[v];
    }
    if (!wave_idle) {
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
      make_face<NDIM, 0, EXT>(q0, h, false, K, fm);
      make_face<NDIM, 0, EXT>(q0, h, true, K, fp);
      // the wave-edge faces are redone after the barrier from the seams
      if (!wave_idle) {
        if (lane == 0) put_face(seamM + (row * nwx + wx) * PL, 1, fm);
        if (lane == 63) put_face(seamP + (row * nwx + wx) * PL, 1, fp);
        if (last_x) put_face(seamPl + row * PL, 1, fp);
      }
      const Face<NV> pl = face_from_left(fp);
      flux2<NDIM, 0>(pl, fm, Fx_lo);
    }
    Face<NV> fym;
    if constexpr (HS) {
      double uD[NV], uU[NV], h[NV];
      if (first_row) {
        if (F32 && !bg_rows) finish_cell_bgv<NDIM, ST>(o1, on1, bgA, uD);
        else finish_cell<NDIM, ST>(A, o1, on1, bg_on_m ? k : ob1, uD, ol1);
      } else {
#pragma unroll
        for (int v = 0; v < NV; ++v) uD[v] = Urow[(v * TS + row - 1) * nxp + i_raw];
      }
      if (last_row) {
        if constexpr (ONE) {
          if (F32 && !bg_rows) finish_cell_bgv<NDIM, ST>(o3, nhi1, bgA, uU);
          else finish_cell<NDIM, ST>(A, o3, nhi1, bg_on_m ? k : bhi1, uU, lhi1);
        } else {
          if (F32 && !bg_rows) finish_cell_bgv<NDIM, ST>(o1, on1, bgA, uU);
          else finish_cell<NDIM, ST>(A, o1, on1, bg_on_m ? k : ob1, uU, ol1);
        }
      } else {
        const int ru = min(row + 1, TS - 1);  // idle rows past the tile read in range
#pragma unroll
        for (int v = 0; v < NV; ++v) uU[v] = Urow[(v * TS + ru) * nxp + i_raw];
      }
#pragma unroll
      for (int v = 0; v < NV; ++v) h[v] = mc_half(q0[v] - uD[v], uU[v] - q0[v]);
      {
        Face<NV> fyp;
        make_face<NDIM, 1, EXT>(q0, h, true, K, fyp);
        if (row < ts_eff - 1) put_face(Prow + row * nxp + i_raw, PS, fyp);
        if (last_row) {
          // minus state of the row above the tile, and the flux at the
          // tile's upper face
          double u2[NV], hh[NV], Fh[NV];
          if constexpr (ONE) {
            if (F32 && !bg_rows) finish_cell_bgv<NDIM, ST>(o4, nhi2, bgA, u2);
            else finish_cell<NDIM, ST>(A, o4, nhi2, bg_on_m ? k : bhi2, u2, lhi2);
          } else {
            if (F32 && !bg_rows) finish_cell_bgv<NDIM, ST>(o2, on2, bgA, u2);
            else finish_cell<NDIM, ST>(A, o2, on2, bg_on_m ? k : ob2, u2, ol2);
          }
#pragma unroll
          for (int v = 0; v < NV; ++v) hh[v] = mc_half(uU[v] - q0[v], u2[v] - uU[v]);
          Face<NV> fh;
          make_face<NDIM, 1, EXT>(uU, hh, false, K, fh);
          flux2<NDIM, 1>(fyp, fh, Fh);
#pragma unroll
          for (int v = 0; v < NV; ++v) Frow[(v * 2 + 1) * nxp + i_raw] = Fh[v];
        }
      }
      make_face<NDIM, 1, EXT>(q0, h, false, K, fym);
      if (row >= 1) put_face(Mrow + (row - 1) * nxp + i_raw, PS, fym);
      if (first_row) {
        // plus state of the row below the tile, and the flux at the tile's
        // lower face
        double u2[NV], hh[NV], Fh[NV];
        if (F32 && !bg_rows) finish_cell_bgv<NDIM, ST>(o2, on2, bgA, u2);
        else finish_cell<NDIM, ST>(A, o2, on2, bg_on_m ? k : ob2, u2, ol2);
#pragma unroll
        for (int v = 0; v < NV; ++v) hh[v] = mc_half(uD[v] - u2[v], q0[v] - uD[v]);
        Face<NV> fh;
        make_face<NDIM, 1, EXT>(uD, hh, true, K, fh);
        flux2<NDIM, 1>(fh, fym, Fh);
#pragma unroll
        for (int v = 0; v < NV; ++v) Frow[(v * 2) * nxp + i_raw] = Fh[v];
      }
    }
    if constexpr (pre) {  // the outside rows of the next plane
      const int kn = min(kraw + 1, G.nm - 1);
      load_cell_raw<NDIM, ST>(uin, kn, oc1, o1);
      load_cell_raw<NDIM, ST>(uin, kn, oc2, o2);
      if constexpr (ONE) {
        load_cell_raw<NDIM, ST>(uin, kn, chi1, o3);
        load_cell_raw<NDIM, ST>(uin, kn, chi2, o4);
      }
    }
    __syncthreads();  // B2

    // ---- P3: the fluxes of the faces shared with another wave or row.  The
    // x faces at a wave's edges are formed by the edge lanes of both waves
    // that share them, from the seam face states; the y faces inside the
    // tile by both rows that share them, from the row face states.  A flux is
    // the same function of the same face states wherever it is formed, so
    // its bits do not depend on who forms it, and no third barrier is needed.
    double Dl[NV];
    {
      double Fx_hi[NV];
#pragma unroll
      for (int v = 0; v < NV; ++v) Fx_hi[v] = from_right(Fx_lo[v]);
      const bool edge_r = last_x || (lane == 63 && xin);
      if ((lane == 0 || edge_r) && !wave_idle) {
        Face<NV> fl, fr;
        if (lane == 0) {  // face at the wave's left edge
          get_face(seamM + (row * nwx + wx) * PL, 1, fr);
          if (wx > 0) get_face(seamP + (row * nwx + wx - 1) * PL, 1, fl);
          else if (x_per) get_face(seamPl + row * PL, 1, fl);
          else fl = mirror<NDIM, 0>(fr);
        } else if (last_x) {  // face at the row's end
          get_face(seamPl + row * PL, 1, fl);
          if (x_per) get_face(seamM + (row * nwx) * PL, 1, fr);
          else fr = mirror<NDIM, 0>(fl);
        } else {  // face at the wave's right edge
          get_face(seamP + (row * nwx + wx) * PL, 1, fl);
          get_face(seamM + (row * nwx + wx + 1) * PL, 1, fr);
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
      if (lane == 0 && last_x && !wave_idle) {
        Face<NV> fl, fr;
        get_face(seamPl + row * PL, 1, fl);
        if (x_per) get_face(seamM + (row * nwx) * PL, 1, fr);
        else fr = mirror<NDIM, 0>(fl);
        flux2<NDIM, 0>(fl, fr, Fx_hi);
      }
#pragma unroll
      for (int v = 0; v < NV; ++v) Dl[v] = -(Fx_hi[v] - Fx_lo[v]) * hx;
    }
    if constexpr (HS) {
      double lo[NV], hi[NV];
      if (first_row) {
#pragma unroll
        for (int v = 0; v < NV; ++v) lo[v] = Frow[(v * 2) * nxp + i_raw];
      } else {
        Face<NV> pd;
        get_face(Prow + (row - 1) * nxp + i_raw, PS, pd);
        flux2<NDIM, 1>(pd, fym, lo);
      }
      if (last_row) {
#pragma unroll
        for (int v = 0; v < NV; ++v) hi[v] = Frow[(v * 2 + 1) * nxp + i_raw];
      } else {
        // rows past a ragged tile read in range (their results are not stored)
        const int rp = max(min(row, TS - 2), 0);
        Face<NV> pu, mu;
        get_face(Prow + rp * nxp + i_raw, PS, pu);
        get_face(Mrow + rp * nxp + i_raw, PS, mu);
        flux2<NDIM, 1>(pu, mu, hi);
      }
#pragma unroll
      for (int v = 0; v < NV; ++v) Dl[v] = fma(-(hi[v] - lo[v]), hy, Dl[v]);
    }
    double q2[NV];
    if constexpr (HM) {
      if constexpr (F32) finish_cell_bgv<NDIM, ST>(q2r, q2neg, bg_on_m ? bgB : bgA, q2);
      else finish_cell<NDIM, ST>(A, q2r, q2neg, bgk(q2k), q2, q2lev);
      double sm1[NV], Fm_hi[NV];
#pragma unroll
      for (int v = 0; v < NV; ++v) sm1[v] = mc_half(q1[v] - q0[v], q2[v] - q1[v]);
      Face<NV> fl, fr;
      make_face<NDIM, DM, EXT>(q0, sm0, true, K, fl);
      make_face<NDIM, DM, EXT>(q1, sm1, false, K, fr);
      flux2<NDIM, DM>(fl, fr, Fm_hi);
#pragma unroll
      for (int v = 0; v < NV; ++v) {
        Dl[v] = fma(-(Fm_hi[v] - Fm_lo[v]), hz, Dl[v]);
        Fm_lo[v] = Fm_hi[v];
        sm0[v] = sm1[v];
      }
    }
    double R[NV];
    const unsigned b = rsst_rate<NDIM, FORM, EXT>(q0, Dl, K, g, R);
    double un[NV];
    if constexpr (STAGE == 2 && REG) {
#pragma unroll
      for (int v = 0; v < NV; ++v) un[v] = rc->un[v];
    } else if constexpr (STAGE == 2) {
      if constexpr (F32) finish_cell_bgv<NDIM, ST>(unr, -1, bgA, un);
      else finish_cell<NDIM, ST>(A, unr, -1, bgk(k), un);
    }
    if (active && kval) {
      bad |= b;
      double out[NV];
#pragma unroll
      for (int v = 0; v < NV; ++v) {
        double y = fma(dt, R[v], q0[v]);
        if constexpr (STAGE == 2) y = 0.5 * (un[v] + y);
        double bgv = 0.0;
        if constexpr (F32) bgv = bgA[v];  // plane k (or this cell's invariant values)
        const ST st = (ST)(y - bgv);
        if constexpr (REG) {
          rc->st[v] = (double)st;
        } else {
          buf_store<ST, HS ? kStoreAux3 : 0>(uout.rsrc(v, k), col, uout.soff(v, k), st);
        }
        out[v] = (double)st + bgv;
        if constexpr (REG) rc->out[v] = out[v];
      }
      if constexpr (STAGE == 2) cmax = fmax(cmax, cell_ctot<NDIM, EXT>(out, K));
    }
    if constexpr (HM) {
#pragma unroll
      for (int v = 0; v < NV; ++v) { q0[v] = q1[v]; q1[v] = q2[v]; }
    }
  }

  return cmax;
}

// Tile id -> XCD: dispatch is round-robin over the 8 XCDs, so consecutive
// tiles (which share halo rows) are remapped onto one XCD and its L2.
__device__ __forceinline__ int xcd_tile(int b, int nblk) {
  return ((nblk & 7) == 0) ? (b & 7) * (nblk >> 3) + (b >> 3) : b;
}

// CFL step from the maxima of c_tot that the last stage 2 (or the prime
// kernel) stored per workgroup: dt = cfl h / max, cut at t_end.  Formed by
// every workgroup of stage 1 at its start, the same bits in each (a maximum
// does not depend on its order).  Includes a workgroup barrier; red is not
// written again in stage 1.
__device__ __forceinline__ double cfl_dt_from_blocks(const StageArgs& A, double* red) {
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  double m = 0.0;
  for (int b = threadIdx.x; b < A.nblk; b += blockDim.x) m = fmax(m, A.blkmax[b]);
  m = wave_max(m);
  if (lane == 0) red[w] = m;
  __syncthreads();
  m = 0.0;
  for (int q = 0; q < (int)(blockDim.x >> 6); ++q) m = fmax(m, red[q]);
  const double t = A.scal[kTime];
  double dt = A.cfl_h / m;
  if (A.t_end > 0.0) dt = fmin(dt, fmax(A.t_end - t, 0.0));
  return dt;
}

// Stage 2: the workgroup's largest c_tot of the new state, stored in its own
// slot (plain store: the next stage 1 reads the slots after this kernel has
// ended), and workgroup 0 advances t by the step's dt (t is read by no other
// workgroup of this kernel).
__device__ __forceinline__ void cfl_epilogue(const StageArgs& A, double* red, double cmax, double dt) {
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const double wm = wave_max(cmax);
  if (lane == 0) red[w] = wm;
  __syncthreads();
  if (threadIdx.x == 0) {
    double m = 0.0;
    for (int q = 0; q < (int)(blockDim.x >> 6); ++q) m = fmax(m, red[q]);
    A.blkmax[blockIdx.x] = m;
    if (blockIdx.x == 0) A.scal[kTime] = A.scal[kTime] + dt;
  }
}

}  // namespace rsstk
