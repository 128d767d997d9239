// Device building blocks of the stage kernels shared by every dimension:
// boundary rules, buffer access to states, widening and background, face
// payload moves, the XCD tile map and the CFL reduction.  The stage bodies
// themselves are in rsst_stage1.h (1D), rsst_stage2.h (2D, per-grid and
// batched) and rsst_stage3.h (3D).
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
__device__ __forceinline__ double grid_max_from_blocks(const StageArgs& A, double* red) {
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  double m = 0.0;
  for (int b = threadIdx.x; b < A.nblk; b += blockDim.x) m = fmax(m, A.blkmax[b]);
  m = wave_max(m);
  if (lane == 0) red[w] = m;
  __syncthreads();
  m = 0.0;
  for (int q = 0; q < (int)(blockDim.x >> 6); ++q) m = fmax(m, red[q]);
  return m;
}

__device__ __forceinline__ double cfl_dt_of_max(const StageArgs& A, double m) {
  const double t = A.scal[kTime];
  double dt = A.cfl_h / m;
  if (A.t_end > 0.0) dt = fmin(dt, fmax(A.t_end - t, 0.0));
  return dt;
}

__device__ __forceinline__ double cfl_dt_from_blocks(const StageArgs& A, double* red) {
  return cfl_dt_of_max(A, grid_max_from_blocks(A, red));
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
