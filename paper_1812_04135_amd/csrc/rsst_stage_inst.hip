// Stage kernels of one dimension and storage type, instantiated for every
// form (with and without xi from the sound speed), row width and stage.
// Compiled once per (RSST_INST_NDIM, RSST_INST_ST, RSST_INST_BIG) so the
// library builds in parallel objects; RSST_INST_BIG = 1 builds the 3D
// kernels that address states of 2 GiB or more (Field64).
#include "rsst_stage1.h"
#include "rsst_stage2.h"
#include "rsst_stage3.h"

#pragma clang fp contract(off)

#ifndef RSST_INST_NDIM
#error "RSST_INST_NDIM (1, 2 or 3) must be defined"
#endif
#ifndef RSST_INST_ST
#error "RSST_INST_ST (double or float) must be defined"
#endif
#ifndef RSST_INST_BIG
#define RSST_INST_BIG 0
#endif

namespace rsstk {

// FORM: the correction form, plus kExtCmax when xi follows the sound speed
// (eq. cx), kExtVdw for the van der Waals gas, kExtHydro for hydrostatic walls.
// 3D workgroups are at most 512 threads (8 waves at ~200 VGPRs, two waves per
// SIMD); 1D and 2D rows take up to 1024.
constexpr int kMaxThreads3 = 512;

constexpr bool kBig = RSST_INST_BIG != 0;

template <int NDIM, int STAGE, typename ST, int FORM, int NWXC, bool BIG>
__global__ void __launch_bounds__(NDIM == 3 ? kMaxThreads3 : 1024) stage_kernel(const StageArgs A) {
  extern __shared__ double lds[];
  const Geometry& G = A.geo;
  const int L = xcd_tile(blockIdx.x, gridDim.x);
  const int tile_s = L % G.ntile_s;
  const int chunk_base = (L / G.ntile_s) * (NDIM == 3 ? 1 : G.ts);
  static_assert(NDIM != 2, "2D grids run stage_kernel2d");
  const int red = NDIM == 3 ? carve3(G.ts, NWXC).red : carve1(G.nwx).red;
  // a CFL step's dt: formed by stage 1 from the maxima of the state it
  // reads, recorded for stage 2
  double dt = A.dt_fixed;
  if (!(A.dt_fixed > 0.0)) {
    if constexpr (STAGE == 1) {
      dt = cfl_dt_from_blocks(A, lds + red);
      if (blockIdx.x == 0 && threadIdx.x == 0) A.scal[kDtCur] = dt;
    } else {
      dt = A.scal[kDtCur];
    }
  }
  unsigned bad = 0;
  double cmax;
  if constexpr (NDIM == 3) cmax = stage_body3<STAGE, ST, FORM, NWXC, BIG>(A, lds, tile_s, chunk_base, dt, bad);
  else cmax = stage_body1<STAGE, ST, FORM>(A, lds, dt, bad);
  if (bad) atomicOr((unsigned*)(A.scal + kFlags), bad);
  if constexpr (STAGE == 2) cfl_epilogue(A, lds + red, cmax, dt);
}

// 2D grids: NP planes of y per march iteration (the geometry's np): two for
// large grids with rows of up to eight waves (512 threads at most), else one
// (up to 1024 threads, fewer registers per thread).
template <int STAGE, typename ST, int FORM, int NP>
__global__ void __launch_bounds__(NP == 2 ? 512 : 1024) stage_kernel2d(const StageArgs A) {
  extern __shared__ double lds[];
  const Geometry& G = A.geo;
  const int L = xcd_tile(blockIdx.x, gridDim.x);
  const int chunk_base = L * G.ts;
  const int red = carve2(G.ts, G.nwx, NP).red;
  double dt = A.dt_fixed;
  if (!(A.dt_fixed > 0.0)) {
    if constexpr (STAGE == 1) {
      dt = cfl_dt_from_blocks(A, lds + red);
      if (blockIdx.x == 0 && threadIdx.x == 0) A.scal[kDtCur] = dt;
    } else {
      dt = A.scal[kDtCur];
    }
  }
  unsigned bad = 0;
  const double cmax = stage_body2<STAGE, ST, FORM, NP>(A, lds, chunk_base, dt, bad);
  if (bad) atomicOr((unsigned*)(A.scal + kFlags), bad);
  if constexpr (STAGE == 2) cfl_epilogue(A, lds + red, cmax, dt);
}

// One launch of a stage kernel over the geometry's grid.  The kernel's LDS
// limit is raised only when a larger tile needs it (lds_set: the limit set
// so far per device, owned by the kernel's launcher), so launches of a known
// shape (e.g. under HIP graph capture) make no attribute call.
static hipError_t launch_geo(void (*kern)(StageArgs), int* lds_set, const StageArgs& a, hipStream_t s) {
  const Geometry& G = a.geo;
  const dim3 grid((unsigned)(G.ntile_s * G.nchunk)), block((unsigned)G.threads);
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) dev = 0;
  if ((int)G.lds_bytes > lds_set[dev]) {
    hipError_t e = hipFuncSetAttribute((const void*)kern, hipFuncAttributeMaxDynamicSharedMemorySize,
                                       (int)G.lds_bytes);
    if (e != hipSuccess) return e;
    lds_set[dev] = (int)G.lds_bytes;
  }
  hipLaunchKernelGGL(kern, grid, block, G.lds_bytes, s, a);
  return hipGetLastError();
}

template <int NDIM, int STAGE, typename ST, int FORM, int NWXC>
static hipError_t launch_stage_k(const StageArgs& a, hipStream_t s) {
  static int lds_set[64] = {0};
  return launch_geo(stage_kernel<NDIM, STAGE, ST, FORM, NWXC, kBig>, lds_set, a, s);
}

template <int STAGE, typename ST, int FORM, int NP>
static hipError_t launch_stage_2d(const StageArgs& a, hipStream_t s) {
  static int lds_set[64] = {0};
  return launch_geo(stage_kernel2d<STAGE, ST, FORM, NP>, lds_set, a, s);
}

template <int NDIM, int STAGE, typename ST, int FORM>
static hipError_t launch_stage_t(const StageArgs& a, hipStream_t s) {
  if constexpr (NDIM == 3) {
    switch (a.geo.nwx) {
      case 1: return launch_stage_k<NDIM, STAGE, ST, FORM, 1>(a, s);
      case 2: return launch_stage_k<NDIM, STAGE, ST, FORM, 2>(a, s);
      case 3: return launch_stage_k<NDIM, STAGE, ST, FORM, 3>(a, s);
      case 4: return launch_stage_k<NDIM, STAGE, ST, FORM, 4>(a, s);
      case 8: return launch_stage_k<NDIM, STAGE, ST, FORM, 8>(a, s);
      default: return hipErrorInvalidValue;
    }
  } else if constexpr (NDIM == 2) {
    return a.geo.np == 2 ? launch_stage_2d<STAGE, ST, FORM, 2>(a, s) : launch_stage_2d<STAGE, ST, FORM, 1>(a, s);
  } else {
    return launch_stage_k<NDIM, STAGE, ST, FORM, 0>(a, s);
  }
}

template <int NDIM, int STAGE, typename ST, int X>
static hipError_t launch_stage_x(const StageArgs& a, hipStream_t s) {
  switch (a.form) {
    case kEuler: return launch_stage_t<NDIM, STAGE, ST, kEuler | X>(a, s);
    case kPVS: return launch_stage_t<NDIM, STAGE, ST, kPVS | X>(a, s);
    case kPMS: return launch_stage_t<NDIM, STAGE, ST, kPMS | X>(a, s);
    case kDVS: return launch_stage_t<NDIM, STAGE, ST, kDVS | X>(a, s);
    case kDMS: return launch_stage_t<NDIM, STAGE, ST, kDMS | X>(a, s);
    default: return launch_stage_t<NDIM, STAGE, ST, kPD | X>(a, s);
  }
}

// The van der Waals and hydrostatic-wall kernels exist for FP64 storage only
// (the C ABI rejects the other combinations before any launch); 1D grids
// need no hydrostatic variant (their walls are x walls, allowed only without
// a force along x, where they are mirror walls).
template <int NDIM, int STAGE, typename ST, int H>
static hipError_t launch_stage_g(const StageArgs& a, hipStream_t s) {
  if (a.eos) return launch_stage_x<NDIM, STAGE, ST, kExtVdw | H>(a, s);
  return a.inv_cmax2 > 0.0 ? launch_stage_x<NDIM, STAGE, ST, kExtCmax | H>(a, s)
                           : launch_stage_x<NDIM, STAGE, ST, H>(a, s);
}

template <int NDIM, int STAGE, typename ST>
static hipError_t launch_stage_f(const StageArgs& a, hipStream_t s) {
  if constexpr (sizeof(ST) == 8) {
    if constexpr (NDIM >= 2) {
      if (a.hydro) return launch_stage_g<NDIM, STAGE, ST, kExtHydro>(a, s);
    }
    return launch_stage_g<NDIM, STAGE, ST, 0>(a, s);
  } else {
    if (a.eos || a.hydro) return hipErrorInvalidValue;
    return a.inv_cmax2 > 0.0 ? launch_stage_x<NDIM, STAGE, ST, kExtCmax>(a, s)
                             : launch_stage_x<NDIM, STAGE, ST, 0>(a, s);
  }
}

template <int NDIM, typename ST, bool BIG>
hipError_t launch_stage_n(const StageArgs& a, int stage, hipStream_t s) {
  static_assert(BIG == kBig, "one addressing per object");
  return stage == 1 ? launch_stage_f<NDIM, 1, ST>(a, s) : launch_stage_f<NDIM, 2, ST>(a, s);
}

template hipError_t launch_stage_n<RSST_INST_NDIM, RSST_INST_ST, kBig>(const StageArgs&, int, hipStream_t);

#if RSST_INST_NDIM == 1 && !RSST_INST_BIG
// nsteps whole steps of a 1D grid in one launch.  A 1D grid is one workgroup
// (a row of at most 16 waves), so both stages and the CFL maximum of every
// step run in that workgroup with barriers in between, and each lane keeps
// its own cell in registers from the first load to the last store: the
// stage bodies are those of stage_kernel in their register-resident form
// (stage input, step-start state and output in registers, each equal to
// what storing and reloading would give; neighbours come by DPP and LDS as
// always), each step's dt is formed from the previous step's maximum as
// stage 1 forms it from the stored maxima, and t and dt stay in registers.
// So the state, t and the next dt after each step are bitwise those of the
// per-stage launches.  U is written once, at the end (and the stage buffer
// not at all).  With a CFL step and an end time, the steps after t reaches
// t_end (dt = 0, which would leave U unchanged) are skipped.  a1: stage 1
// (U -> U1), a2: stage 2.
template <typename ST, int FORM>
__global__ void __launch_bounds__(1024) steps1d_kernel(const StageArgs a1, const StageArgs a2, int nsteps) {
  constexpr int NV = 3;
  extern __shared__ double lds[];
  const Geometry& G = a1.geo;
  double* red = lds + carve1(G.nwx).red;
  const bool cfl = !(a1.dt_fixed > 0.0);
  double t = a1.scal[kTime];
  double dt = a1.dt_fixed;
  if (cfl) {  // from the one stored maximum (a 1D grid is one workgroup), as stage 1 forms it
    dt = a1.cfl_h / a1.blkmax[0];
    if (a1.t_end > 0.0) dt = fmin(dt, fmax(a1.t_end - t, 0.0));
  }
  // this lane's cell (lanes past the row hold the last cell and store nothing)
  const int i = min((int)threadIdx.x, G.nx - 1);
  RegCell<NV> c;
  {
    ST raw[NV];
    load_cell_raw<1, ST>(make_field<false>(a1.uin, a1.ncell, NV, (int)sizeof(ST), G.nx * (int)sizeof(ST)), 0,
                         i * (int)sizeof(ST), raw);
    const int b = (sizeof(ST) == 4 && !a1.bg_uniform) ? bg_index<1>(a1, i, 0, 0) : 0;
    finish_cell<1, ST>(a1, raw, -1, b, c.in);
  }
  double stu[NV];  // stored values of the state after the last step
  unsigned bad = 0;
  double mlast = -1.0;
  for (int q = 0; q < nsteps; ++q) {
    if (cfl && a1.t_end > 0.0 && !(dt > 0.0)) break;
#pragma unroll
    for (int v = 0; v < NV; ++v) c.out[v] = c.in[v];
    stage_body1<1, ST, FORM, true>(a1, lds, dt, bad, &c);
    __syncthreads();
#pragma unroll
    for (int v = 0; v < NV; ++v) {
      c.un[v] = c.in[v];
      c.in[v] = c.out[v];
    }
    const double cm = stage_body1<2, ST, FORM, true>(a2, lds, dt, bad, &c);
#pragma unroll
    for (int v = 0; v < NV; ++v) {
      c.in[v] = c.out[v];
      stu[v] = c.st[v];
    }
    const double wm = wave_max(cm);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = wm;
    __syncthreads();
    double m = 0.0;
    for (int w = 0; w < (int)(blockDim.x >> 6); ++w) m = fmax(m, red[w]);
    mlast = m;
    t = t + dt;
    if (cfl) {
      dt = a1.cfl_h / m;
      if (a1.t_end > 0.0) dt = fmin(dt, fmax(a1.t_end - t, 0.0));
    }
    __syncthreads();
  }
  if (mlast >= 0.0 && (int)threadIdx.x < G.nx) {
    ST* u = (ST*)a2.uout;
#pragma unroll
    for (int v = 0; v < NV; ++v) u[v * a2.ncell + i] = (ST)stu[v];
  }
  if (bad) atomicOr((unsigned*)(a1.scal + kFlags), bad);
  if (threadIdx.x == 0) {
    a1.scal[kTime] = t;
    if (mlast >= 0.0) a1.blkmax[0] = mlast;  // the maximum of the state left in U
  }
}

template <typename ST, int FORM>
static hipError_t launch_steps1d_k(const StageArgs& a1, const StageArgs& a2, int nsteps, hipStream_t s) {
  const Geometry& G = a1.geo;
  auto kern = steps1d_kernel<ST, FORM>;
  static int lds_set[64] = {0};
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) dev = 0;
  if ((int)G.lds_bytes > lds_set[dev]) {
    hipError_t e = hipFuncSetAttribute((const void*)kern, hipFuncAttributeMaxDynamicSharedMemorySize,
                                       (int)G.lds_bytes);
    if (e != hipSuccess) return e;
    lds_set[dev] = (int)G.lds_bytes;
  }
  hipLaunchKernelGGL(kern, dim3(1), dim3((unsigned)G.threads), G.lds_bytes, s, a1, a2, nsteps);
  return hipGetLastError();
}

template <typename ST, int X>
static hipError_t launch_steps1d_x(const StageArgs& a1, const StageArgs& a2, int n, hipStream_t s) {
  switch (a1.form) {
    case kEuler: return launch_steps1d_k<ST, kEuler | X>(a1, a2, n, s);
    case kPVS: return launch_steps1d_k<ST, kPVS | X>(a1, a2, n, s);
    case kPMS: return launch_steps1d_k<ST, kPMS | X>(a1, a2, n, s);
    case kDVS: return launch_steps1d_k<ST, kDVS | X>(a1, a2, n, s);
    case kDMS: return launch_steps1d_k<ST, kDMS | X>(a1, a2, n, s);
    default: return launch_steps1d_k<ST, kPD | X>(a1, a2, n, s);
  }
}

template <typename ST>
hipError_t launch_steps1d(const StageArgs& a1, const StageArgs& a2, int nsteps, hipStream_t s) {
  if (a1.geo.ndim != 1 || a1.geo.ntile_s * a1.geo.nchunk != 1) return hipErrorInvalidValue;
  if constexpr (sizeof(ST) == 8) {
    if (a1.eos) return launch_steps1d_x<ST, kExtVdw>(a1, a2, nsteps, s);
  }
  if (a1.eos) return hipErrorInvalidValue;
  return a1.inv_cmax2 > 0.0 ? launch_steps1d_x<ST, kExtCmax>(a1, a2, nsteps, s)
                            : launch_steps1d_x<ST, 0>(a1, a2, nsteps, s);
}

template hipError_t launch_steps1d<RSST_INST_ST>(const StageArgs&, const StageArgs&, int, hipStream_t);
#endif

}  // namespace rsstk
