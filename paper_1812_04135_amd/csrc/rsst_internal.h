// Internal interface between the C ABI (rsst_api.hip) and the kernels
// (rsst_kernels.hip).  Not installed; not part of the ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace rsstk {

// Device-side scalars of one solver, in one small allocation.  kDtCur: the
// dt of the step in progress (formed by stage 1, read by stage 2); kTime: t;
// kDtNext: the dt the next stage 1 will form (written on request, for
// reporting).
enum Scalar { kDtCur = 0, kTime = 1, kMaxBits = 2, kDone = 3, kFlags = 4, kDtNext = 5, kNumScalars = 8 };

// Launch geometry of the fused stage kernel.
//   x (axis 0): one lane per cell, a row of nx cells spread over nwx waves;
//   s (axis 1, 3D only): ts rows stacked in one workgroup, exchanged in LDS;
//   m (last axis, 2D/3D): marched by each thread in chunks of km planes.
struct Geometry {
  int ndim;
  int nx, ns, nm;   // extents along x, s, m (ns = 1 unless 3D; nm = 1 in 1D)
  int nwx, ts, km;  // waves per row, rows per tile, planes per chunk
  int np;           // 2D: planes per march iteration (1 or 2)
  int ntile_s, nchunk;
  int threads;
  size_t lds_bytes;
};

struct StageArgs {
  Geometry geo;
  long long ncell;
  int bc_lo[3], bc_hi[3];  // physical axes
  double inv_dx[3];
  double dx[3];      // cell widths (hydrostatic wall ghosts)
  double gamma, gm1, inv_gm1, inv_xi, f;
  double inv_cmax2;  // > 0: xi = [1 + (a/C_max)^4]^(1/4) per state (eq. cx)
  int eos;           // 0 ideal gas, 1 van der Waals (a, b below)
  int hydro;         // a hydrostatic wall on the y or march axis (2D/3D)
  double vdw_a, vdw_b;
  double g[3];
  int form;
  double dt_fixed;   // > 0: use it, else scal[kDtCur]
  double cfl_h;      // cfl * h, h from the dt rule
  double t_end;      // > 0: cut dt at t_end
  double* scal;      // device scalars
  double* blkmax;    // [nblk] largest c_tot of the current state per stage-2 workgroup
  int nblk;          // stage-kernel workgroups (ntile_s * nchunk)
  const void* uin;   // stage input (halo reads)
  const void* un;    // stage 2: state at the start of the step (pointwise)
  void* uout;        // stage output (stage 2: un itself for the in-place step, or another array)
  const double* bg;  // FP32 perturbation form: background [nv][nbg]
  int bg_axis;       // -1 uniform
  int nbg;
  int bg_uniform;    // background index is workgroup-uniform (-1 or the march axis)
  int prec;          // 0 FP64, 1 FP32 perturbation
  int big;           // 3D state of 2 GiB or more (64-bit plane bases)
};

Geometry plan_geometry(int ndim, const int n[3]);

hipError_t launch_stage(const StageArgs& a, int stage, hipStream_t s);
// One instantiation per (NDIM, ST, BIG) lives in its own object
// (rsst_stage_inst.hip); BIG: a 3D state of 2 GiB or more, addressed one
// plane at a time with 64-bit bases.
template <int NDIM, typename ST, bool BIG>
hipError_t launch_stage_n(const StageArgs& a, int stage, hipStream_t s);
// nsteps whole steps of a 1D grid (one workgroup) in one launch; a1 and a2
// are the stage-1 and stage-2 arguments of rsst_stage.
template <typename ST>
hipError_t launch_steps1d(const StageArgs& a1, const StageArgs& a2, int nsteps, hipStream_t s);
hipError_t launch_prime(const StageArgs& a, const void* u, double t0, int set_t, hipStream_t s);
// Writes scal[kDtNext]: the dt the next CFL stage 1 will form from the stored
// per-workgroup maxima (same code, so the same bits), 0 if none is positive.
hipError_t launch_next_dt(const StageArgs& a, hipStream_t s);
hipError_t launch_diag(const StageArgs& a, const void* u, double* partial, int npartial,
                       double* out8, hipStream_t s);
int diag_partials(long long ncell);

}  // namespace rsstk
