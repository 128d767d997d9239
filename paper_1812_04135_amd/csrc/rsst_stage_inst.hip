// Stage kernels of one dimension and storage type, instantiated for every
// form (with and without xi from the sound speed), row width and stage.
// Compiled once per (RSST_INST_NDIM, RSST_INST_ST) so the library builds in
// parallel objects.
#include "rsst_stage.h"

#pragma clang fp contract(off)

#ifndef RSST_INST_NDIM
#error "RSST_INST_NDIM (1, 2 or 3) must be defined"
#endif
#ifndef RSST_INST_ST
#error "RSST_INST_ST (double or float) must be defined"
#endif

namespace rsstk {

// FORM: the correction form, plus kExtCmax when xi follows the sound speed
// (eq. cx) or kExtVdw for the van der Waals gas.
#ifndef RSST_LB3
#define RSST_LB3 512
#endif
#ifndef RSST_WPE3
#define RSST_WPE3 1
#endif

template <int NDIM, int STAGE, typename ST, int FORM, int NWXC>
__global__ void __launch_bounds__(NDIM == 3 ? RSST_LB3 : 1024)
    __attribute__((amdgpu_waves_per_eu(NDIM == 3 ? RSST_WPE3 : 1))) stage_kernel(const StageArgs A) {
  extern __shared__ double lds[];
  const Geometry& G = A.geo;
  const int L = xcd_tile(blockIdx.x, gridDim.x);
  const int tile_s = L % G.ntile_s;
  const int chunk_base = (L / G.ntile_s) * (NDIM == 3 ? 1 : G.ts);
  const double dt = (A.dt_fixed > 0.0) ? A.dt_fixed : A.scal[kDtCur];
  unsigned bad = 0;
  const double cmax = stage_body<NDIM, STAGE, ST, FORM, NWXC>(A, lds, tile_s, chunk_base, dt, bad);
  if (bad) atomicOr((unsigned*)(A.scal + kFlags), bad);
  if constexpr (STAGE == 2) {
    const Carve C = carve(NDIM, NDIM == 3 ? tile_rows(NWXC) : G.ts, NDIM == 3 ? NWXC : G.nwx);
    cfl_epilogue(A, lds + C.red, cmax, dt);
  }
}

template <int NDIM, int STAGE, typename ST, int FORM, int NWXC>
static hipError_t launch_stage_k(const StageArgs& a, hipStream_t s) {
  const Geometry& G = a.geo;
  const dim3 grid((unsigned)(G.ntile_s * G.nchunk)), block((unsigned)G.threads);
  auto kern = stage_kernel<NDIM, STAGE, ST, FORM, NWXC>;
  // raise the kernel's LDS limit only when a larger tile needs it, so launches
  // of a known shape (e.g. under HIP graph capture) make no attribute call
  static int lds_set[64] = {0};
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

// The van der Waals kernels exist for FP64 storage only (the C ABI rejects
// the other combinations before any launch).
template <int NDIM, int STAGE, typename ST>
static hipError_t launch_stage_f(const StageArgs& a, hipStream_t s) {
  if constexpr (sizeof(ST) == 8) {
    if (a.eos) return launch_stage_x<NDIM, STAGE, ST, kExtVdw>(a, s);
  }
  if (a.eos) return hipErrorInvalidValue;
  return a.inv_cmax2 > 0.0 ? launch_stage_x<NDIM, STAGE, ST, kExtCmax>(a, s)
                           : launch_stage_x<NDIM, STAGE, ST, 0>(a, s);
}

template <int NDIM, typename ST>
hipError_t launch_stage_n(const StageArgs& a, int stage, hipStream_t s) {
  return stage == 1 ? launch_stage_f<NDIM, 1, ST>(a, s) : launch_stage_f<NDIM, 2, ST>(a, s);
}

template hipError_t launch_stage_n<RSST_INST_NDIM, RSST_INST_ST>(const StageArgs&, int, hipStream_t);

}  // namespace rsstk
