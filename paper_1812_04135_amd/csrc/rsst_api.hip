// C ABI of the RSST step library (declared in include/rsst.h).
//
// Host responsibilities only: validate the configuration before any device
// call, own the workspace (the stage buffer U1, the reduction scalars and the
// diagnostic partials), and enqueue the kernels of rsst_kernels.hip.  No
// numerics happen on the host.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>
#include <cstring>
#include <atomic>
#include <new>
#include <vector>

#include "rsst.h"
#include "rsst_adjoint.h"
#include "rsst_internal.h"

using rsstk::Geometry;
using rsstk::StageArgs;

struct rsst_solver {
  rsst_config cfg;
  StageArgs args;
  int device;
  int nv;
  long long ncell;
  size_t elem;       // bytes per stored value
  void* u1;          // stage buffer, owned
  double* scal;      // device scalars, owned
  double* blkmax;    // per-workgroup maxima of c_tot of the current state, owned
  double* part;      // diag partials, owned
  double* diag_out;  // 8 doubles, owned
  int npart;
  bool primed;
  double* adj_work;  // adjoint workspace (flags & RSST_WITH_ADJOINT), owned
};

static int check(hipError_t e) { return e == hipSuccess ? RSST_OK : RSST_E_DEVICE; }

static int validate(const rsst_config* c) {
  if (!c) return RSST_E_ARG;
  if (c->ndim < 1 || c->ndim > 3) return RSST_E_ARG;
  for (int d = 0; d < 3; ++d) {
    if (d < c->ndim) {
      if (c->n[d] < 4) return RSST_E_ARG;
      if (!(c->dx[d] > 0.0) || !std::isfinite(c->dx[d])) return RSST_E_ARG;
      if (c->bc_lo[d] < RSST_PERIODIC || c->bc_lo[d] > RSST_REFLECT_HYDRO) return RSST_E_ARG;
      if (c->bc_hi[d] < RSST_PERIODIC || c->bc_hi[d] > RSST_REFLECT_HYDRO) return RSST_E_ARG;
      if ((c->bc_lo[d] == RSST_PERIODIC) != (c->bc_hi[d] == RSST_PERIODIC)) return RSST_E_ARG;
      if (!std::isfinite(c->g[d])) return RSST_E_ARG;
    } else if (c->n[d] != 1) {
      return RSST_E_ARG;
    }
  }
  if (!(c->gamma > 1.0) || !std::isfinite(c->gamma)) return RSST_E_ARG;
  if (!(c->xi >= 1.0) || !std::isfinite(c->xi)) return RSST_E_ARG;
  if (!(c->cfl > 0.0 && c->cfl <= 1.0)) return RSST_E_ARG;
  if (c->dt_rule != 0 && c->dt_rule != 1) return RSST_E_ARG;
  if (c->form < RSST_EULER || c->form > RSST_PD) return RSST_E_ARG;
  if (c->prec != RSST_FP64 && c->prec != RSST_FP32_PERT) return RSST_E_ARG;
  if (c->prec == RSST_FP32_PERT) {
    if (!c->bg) return RSST_E_ARG;
    if (c->bg_axis < -1 || c->bg_axis >= c->ndim) return RSST_E_ARG;
  }
  if (!(c->t_end >= 0.0) || !std::isfinite(c->t_end)) return RSST_E_ARG;
  if (c->flags & ~RSST_WITH_ADJOINT) return RSST_E_ARG;
  if (!(c->cmax >= 0.0) || !std::isfinite(c->cmax)) return RSST_E_ARG;
  if ((c->flags & RSST_WITH_ADJOINT) && c->cmax > 0.0) return RSST_E_UNSUPPORTED;
  if ((c->flags & RSST_WITH_ADJOINT) && c->prec != RSST_FP64) return RSST_E_UNSUPPORTED;
  if (c->eos != RSST_EOS_IDEAL && c->eos != RSST_EOS_VDW) return RSST_E_ARG;
  {
    // hydrostatic walls: FP64, no adjoint, and along x only where they equal
    // the mirror wall (no force along x: x walls mirror face states in-row)
    bool hydro = false;
    for (int d = 0; d < c->ndim; ++d)
      hydro = hydro || c->bc_lo[d] == RSST_REFLECT_HYDRO || c->bc_hi[d] == RSST_REFLECT_HYDRO;
    if (hydro && (c->prec != RSST_FP64 || (c->flags & RSST_WITH_ADJOINT))) return RSST_E_UNSUPPORTED;
    if ((c->bc_lo[0] == RSST_REFLECT_HYDRO || c->bc_hi[0] == RSST_REFLECT_HYDRO) && c->g[0] != 0.0)
      return RSST_E_UNSUPPORTED;
  }
  if (c->eos == RSST_EOS_VDW) {
    if (!(c->eos_a >= 0.0) || !std::isfinite(c->eos_a)) return RSST_E_ARG;
    if (!(c->eos_b >= 0.0) || !std::isfinite(c->eos_b)) return RSST_E_ARG;
    if (c->prec != RSST_FP64 || c->cmax > 0.0 || (c->flags & RSST_WITH_ADJOINT))
      return RSST_E_UNSUPPORTED;
  }
  // 1D and 2D states are addressed with 32-bit byte offsets; 3D states of
  // 2 GiB or more one x-y plane at a time, with 32-bit offsets inside it
  {
    const int sz = c->prec == RSST_FP32_PERT ? 4 : 8;
    const long long cells = (long long)c->n[0] * c->n[1] * c->n[2];
    if (c->ndim < 3 && cells * (c->ndim + 2) * sz >= (1ll << 31)) return RSST_E_UNSUPPORTED;
    if (c->ndim == 3 && (long long)c->n[0] * c->n[1] * sz >= (1ll << 31)) return RSST_E_UNSUPPORTED;
  }
  // supported launch shapes: whole x rows in one workgroup
  if (c->ndim == 1 && c->n[0] > 1024) return RSST_E_UNSUPPORTED;
  if (c->ndim == 2 && c->n[0] > 1024) return RSST_E_UNSUPPORTED;
  if (c->ndim == 3) {
    if (c->n[0] > 512) return RSST_E_UNSUPPORTED;
  }
  return RSST_OK;
}

// Kernel arguments of a validated configuration (no device call).  The
// state, scalar and maxima pointers are left for the caller to set.
static void fill_args(const rsst_config* cfg, long long ncell, StageArgs& a) {
  std::memset(&a, 0, sizeof(a));
  a.geo = rsstk::plan_geometry(cfg->ndim, cfg->n);
  a.ncell = ncell;
  for (int d = 0; d < 3; ++d) {
    a.bc_lo[d] = cfg->bc_lo[d];
    a.bc_hi[d] = cfg->bc_hi[d];
    a.inv_dx[d] = d < cfg->ndim ? 1.0 / cfg->dx[d] : 0.0;
    a.dx[d] = d < cfg->ndim ? cfg->dx[d] : 0.0;
    if (d >= 1 && d < cfg->ndim && (cfg->bc_lo[d] == RSST_REFLECT_HYDRO || cfg->bc_hi[d] == RSST_REFLECT_HYDRO))
      a.hydro = 1;
    a.g[d] = d < cfg->ndim ? cfg->g[d] : 0.0;
  }
  a.gamma = cfg->gamma;
  a.gm1 = cfg->gamma - 1.0;
  a.inv_gm1 = 1.0 / (cfg->gamma - 1.0);
  a.inv_xi = 1.0 / cfg->xi;
  a.f = 1.0 - 1.0 / (cfg->xi * cfg->xi);
  a.inv_cmax2 = cfg->cmax > 0.0 ? 1.0 / (cfg->cmax * cfg->cmax) : 0.0;
  a.eos = cfg->eos;
  a.vdw_a = cfg->eos == RSST_EOS_VDW ? cfg->eos_a : 0.0;
  a.vdw_b = cfg->eos == RSST_EOS_VDW ? cfg->eos_b : 0.0;
  a.form = cfg->form;
  double hlen;
  if (cfg->dt_rule == 1) {
    hlen = cfg->dx[0];
    for (int d = 1; d < cfg->ndim; ++d) hlen = std::fmin(hlen, cfg->dx[d]);
  } else {
    double sum = 0.0;
    for (int d = 0; d < cfg->ndim; ++d) sum += 1.0 / cfg->dx[d];
    hlen = 1.0 / sum;
  }
  a.cfl_h = cfg->cfl * hlen;
  a.t_end = cfg->t_end;
  a.prec = cfg->prec;
  a.bg = cfg->bg;
  a.bg_axis = cfg->prec == RSST_FP32_PERT ? cfg->bg_axis : -1;
  a.nbg = (a.bg_axis >= 0) ? cfg->n[a.bg_axis] : 1;
  a.bg_uniform = (a.bg_axis == -1 || (cfg->ndim >= 2 && a.bg_axis == cfg->ndim - 1)) ? 1 : 0;
  a.nblk = a.geo.ntile_s * a.geo.nchunk;
  a.big = (cfg->ndim == 3 && (long long)(cfg->ndim + 2) * ncell *
                                 (long long)(cfg->prec == RSST_FP32_PERT ? 4 : 8) >= (1ll << 31)) ? 1 : 0;
}

// ---- rsst_step_noalloc: one step with no allocation ------------------------
// Its scratch (device scalars, per-workgroup CFL maxima, the stage buffer U1)
// lives in one file-scope device array of fixed size instead of a handle's
// workspace.  Each device holds its own copy for the life of the process;
// every call on a device reuses it, so calls that overlap on one device race.
// In host code `scratch` only names the symbol: its device address, per
// device, comes from hipGetSymbolAddress (taken once per device, with that
// device current) and only that address reaches the kernels.
static constexpr size_t kScratchBytes = (size_t)64 << 20;
static __device__ __align__(256) unsigned char scratch[kScratchBytes];
static constexpr int kMaxDevices = 64;
static std::atomic<unsigned char*> g_scratch[kMaxDevices];

static int scratch_on(int dev, unsigned char** out) {
  if (dev < 0 || dev >= kMaxDevices) return RSST_E_DEVICE;
  unsigned char* p = g_scratch[dev].load(std::memory_order_acquire);
  if (!p) {
    void* q = nullptr;
    if (hipGetSymbolAddress(&q, HIP_SYMBOL(scratch)) != hipSuccess || !q) return RSST_E_DEVICE;
    p = (unsigned char*)q;
    g_scratch[dev].store(p, std::memory_order_release);
  }
  *out = p;
  return RSST_OK;
}

// Zeroes the device scalars (a kernel, not a memset node, so a captured call
// replays correctly).
__global__ void __launch_bounds__(64) noalloc_clear_kernel(double* scal) {
  if (threadIdx.x < rsstk::kNumScalars) scal[threadIdx.x] = 0.0;
}

// Copies the non-physical flags of the step into the caller's word.
__global__ void __launch_bounds__(64) noalloc_flags_kernel(const double* scal, uint32_t* flags) {
  if (threadIdx.x == 0) *flags = *(const uint32_t*)(scal + rsstk::kFlags);
}

static size_t round256(size_t x) { return (x + 255) & ~(size_t)255; }

extern "C" {

const char* rsst_strerror(int s) {
  switch (s) {
    case RSST_OK: return "success";
    case RSST_E_ARG: return "invalid argument or configuration";
    case RSST_E_NOMEM: return "device allocation failed";
    case RSST_E_DEVICE: return "HIP runtime call failed";
    case RSST_E_UNSUPPORTED: return "configuration not supported by this build";
    case RSST_E_NONPHYSICAL: return "non-physical state (rho <= 0, P <= 0 or non-finite)";
    case RSST_E_SCRATCH: return "state too large for the fixed scratch of rsst_step_noalloc (64 MiB)";
    default: return "unknown status";
  }
}

const char* rsst_version(void) { return "rsst-gfx950 stage-v20"; }

int rsst_init(const rsst_config* cfg, void* stream, rsst_handle* out) {
  if (!out) return RSST_E_ARG;
  *out = nullptr;
  int st = validate(cfg);
  if (st != RSST_OK) return st;
  hipStream_t s = (hipStream_t)stream;

  rsst_solver* h = new (std::nothrow) rsst_solver();
  if (!h) return RSST_E_NOMEM;
  h->cfg = *cfg;
  h->nv = cfg->ndim + 2;
  h->ncell = (long long)cfg->n[0] * cfg->n[1] * cfg->n[2];
  h->elem = cfg->prec == RSST_FP32_PERT ? sizeof(float) : sizeof(double);
  if (hipGetDevice(&h->device) != hipSuccess) { delete h; return RSST_E_DEVICE; }

  StageArgs& a = h->args;
  fill_args(cfg, h->ncell, a);
  h->npart = rsstk::diag_partials(h->ncell);
  const size_t ubytes = (size_t)h->nv * h->ncell * h->elem;
  if (hipMalloc(&h->u1, ubytes) != hipSuccess) { delete h; return RSST_E_NOMEM; }
  const size_t nscal = rsstk::kNumScalars;
  h->scal = h->blkmax = h->part = h->diag_out = nullptr;
  if (hipMalloc((void**)&h->scal, nscal * sizeof(double)) != hipSuccess ||
      hipMalloc((void**)&h->blkmax, (size_t)a.nblk * sizeof(double)) != hipSuccess ||
      hipMalloc((void**)&h->part, (size_t)h->npart * 8 * sizeof(double)) != hipSuccess ||
      hipMalloc((void**)&h->diag_out, 8 * sizeof(double)) != hipSuccess) {
    (void)hipFree(h->u1); (void)hipFree(h->scal); (void)hipFree(h->blkmax); (void)hipFree(h->part);
    (void)hipFree(h->diag_out);
    delete h;
    return RSST_E_NOMEM;
  }
  h->adj_work = nullptr;
  if (cfg->flags & RSST_WITH_ADJOINT) {
    const size_t nd = rsstk::adjoint_workspace_doubles(cfg->ndim, cfg->n, h->ncell);
    if (hipMalloc((void**)&h->adj_work, nd * sizeof(double)) != hipSuccess) {
      h->adj_work = nullptr;
      rsst_destroy(h);
      return RSST_E_NOMEM;
    }
  }
  // zeroed before any launch on any stream
  const size_t adj_z = h->adj_work ? rsstk::adjoint_zeroed_offset(cfg->ndim, cfg->n, h->ncell) : 0;
  const size_t adj_n = h->adj_work ? rsstk::adjoint_workspace_doubles(cfg->ndim, cfg->n, h->ncell) : 0;
  if (hipMemsetAsync(h->scal, 0, nscal * sizeof(double), s) != hipSuccess ||
      hipMemsetAsync(h->blkmax, 0, (size_t)a.nblk * sizeof(double), s) != hipSuccess ||
      (adj_n > adj_z && hipMemsetAsync(h->adj_work + adj_z, 0, (adj_n - adj_z) * sizeof(double), s) != hipSuccess) ||
      hipStreamSynchronize(s) != hipSuccess) {
    rsst_destroy(h);
    return RSST_E_DEVICE;
  }
  a.scal = h->scal;
  a.blkmax = h->blkmax;
  h->primed = false;
  *out = h;
  return RSST_OK;
}

int rsst_prime(rsst_handle h, const void* U, double t0, void* stream) {
  if (!h || !U || !std::isfinite(t0)) return RSST_E_ARG;
  int st = check(rsstk::launch_prime(h->args, U, t0, 1, (hipStream_t)stream));
  if (st == RSST_OK) h->primed = true;
  return st;
}

int rsst_stage(rsst_handle h, void* U, int stage, double dt_fixed, void* stream) {
  if (!h || !U || !std::isfinite(dt_fixed) || (stage != 1 && stage != 2)) return RSST_E_ARG;
  hipStream_t s = (hipStream_t)stream;
  StageArgs a = h->args;
  a.dt_fixed = dt_fixed > 0.0 ? dt_fixed : 0.0;
  if (stage == 1) {
    if (dt_fixed <= 0.0 && !h->primed) {
      // CFL dt of U at the current device time
      if (rsstk::launch_prime(h->args, U, 0.0, 0, s) != hipSuccess) return RSST_E_DEVICE;
      h->primed = true;
    }
    a.uin = U;
    a.un = nullptr;
    a.uout = h->u1;
  } else {
    a.uin = h->u1;
    a.un = U;
    a.uout = U;
  }
  if (rsstk::launch_stage(a, stage, s) != hipSuccess) return RSST_E_DEVICE;
  // stage 2 stores the maxima of the new state, from which the next CFL dt
  // is formed (after a fixed step too)
  if (stage == 2) h->primed = true;
  return RSST_OK;
}

int rsst_step(rsst_handle h, void* U, double dt_fixed, void* stream) {
  int st = rsst_stage(h, U, 1, dt_fixed, stream);
  if (st != RSST_OK) return st;
  return rsst_stage(h, U, 2, dt_fixed, stream);
}

int rsst_step_out(rsst_handle h, const void* U, void* U1, void* Unext, double dt_fixed, void* stream) {
  if (!h || !U || !U1 || !Unext || !std::isfinite(dt_fixed)) return RSST_E_ARG;
  if (U1 == U || Unext == U || U1 == Unext) return RSST_E_ARG;
  hipStream_t s = (hipStream_t)stream;
  StageArgs a = h->args;
  a.dt_fixed = dt_fixed > 0.0 ? dt_fixed : 0.0;
  if (dt_fixed <= 0.0 && !h->primed) {
    if (rsstk::launch_prime(h->args, U, 0.0, 0, s) != hipSuccess) return RSST_E_DEVICE;
    h->primed = true;
  }
  // the two stages of rsst_step with the caller's buffers in place of the
  // stage buffer and of U
  a.uin = U;
  a.un = nullptr;
  a.uout = U1;
  if (rsstk::launch_stage(a, 1, s) != hipSuccess) return RSST_E_DEVICE;
  a.uin = U1;
  a.un = U;
  a.uout = Unext;
  if (rsstk::launch_stage(a, 2, s) != hipSuccess) return RSST_E_DEVICE;
  h->primed = true;
  return RSST_OK;
}

int rsst_steps_out(rsst_handle h, void* const* U_list, void* const* U1_list, int nsteps, double dt_fixed,
                   void* stream) {
  if (!h || !U_list || !U1_list || nsteps < 0 || !std::isfinite(dt_fixed)) return RSST_E_ARG;
  for (int n = 0; n < nsteps; ++n)
    if (!U_list[n] || !U1_list[n] || !U_list[n + 1]) return RSST_E_ARG;
  for (int n = 0; n < nsteps; ++n) {
    const int st = rsst_step_out(h, U_list[n], U1_list[n], U_list[n + 1], dt_fixed, stream);
    if (st != RSST_OK) return st;
  }
  return RSST_OK;
}

int rsst_steps(rsst_handle h, void* U, int nsteps, double dt_fixed, void* stream) {
  if (nsteps < 0) return RSST_E_ARG;
  if (h && U && std::isfinite(dt_fixed) && nsteps > 0 && h->cfg.ndim == 1) {
    // a 1D grid is one workgroup: every step in one launch (same results)
    hipStream_t s = (hipStream_t)stream;
    StageArgs a1 = h->args, a2 = h->args;
    a1.dt_fixed = a2.dt_fixed = dt_fixed > 0.0 ? dt_fixed : 0.0;
    if (dt_fixed <= 0.0 && !h->primed) {
      if (rsstk::launch_prime(h->args, U, 0.0, 0, s) != hipSuccess) return RSST_E_DEVICE;
      h->primed = true;
    }
    a1.uin = U;
    a1.un = nullptr;
    a1.uout = h->u1;
    a2.uin = h->u1;
    a2.un = U;
    a2.uout = U;
    const hipError_t e = h->elem == sizeof(float) ? rsstk::launch_steps1d<float>(a1, a2, nsteps, s)
                                                  : rsstk::launch_steps1d<double>(a1, a2, nsteps, s);
    if (e != hipSuccess) return RSST_E_DEVICE;
    h->primed = true;
    return RSST_OK;
  }
  for (int q = 0; q < nsteps; ++q) {
    int st = rsst_step(h, U, dt_fixed, stream);
    if (st != RSST_OK) return st;
  }
  return RSST_OK;
}

int rsst_get_time(rsst_handle h, double* t, double* dt_next, void* stream) {
  if (!h) return RSST_E_ARG;
  hipStream_t s = (hipStream_t)stream;
  // the dt the next stage 1 will form, by the same device code (0 before any
  // state has been seen)
  if (rsstk::launch_next_dt(h->args, s) != hipSuccess) return RSST_E_DEVICE;
  double v[rsstk::kNumScalars];
  if (hipStreamSynchronize(s) != hipSuccess ||
      hipMemcpy(v, h->scal, sizeof(v), hipMemcpyDeviceToHost) != hipSuccess)
    return RSST_E_DEVICE;
  if (dt_next) *dt_next = v[rsstk::kDtNext];
  if (t) *t = v[rsstk::kTime];
  return RSST_OK;
}

int rsst_diag(rsst_handle h, const void* U, double out[8], void* stream) {
  if (!h || !U || !out) return RSST_E_ARG;
  hipStream_t s = (hipStream_t)stream;
  if (rsstk::launch_diag(h->args, U, h->part, h->npart, h->diag_out, s) != hipSuccess)
    return RSST_E_DEVICE;
  if (hipMemcpyAsync(out, h->diag_out, 8 * sizeof(double), hipMemcpyDeviceToHost, s) != hipSuccess)
    return RSST_E_DEVICE;
  return check(hipStreamSynchronize(s));
}

int rsst_poll(rsst_handle h, uint32_t* flags) {
  if (!h) return RSST_E_ARG;
  if (hipDeviceSynchronize() != hipSuccess) return RSST_E_DEVICE;
  uint32_t f = 0;
  if (hipMemcpy(&f, h->scal + rsstk::kFlags, sizeof(uint32_t), hipMemcpyDeviceToHost) != hipSuccess)
    return RSST_E_DEVICE;
  if (f) {
    uint32_t z = 0;
    if (hipMemcpy(h->scal + rsstk::kFlags, &z, sizeof(uint32_t), hipMemcpyHostToDevice) != hipSuccess)
      return RSST_E_DEVICE;
  }
  if (flags) *flags = f;
  return f ? RSST_E_NONPHYSICAL : RSST_OK;
}

int rsst_destroy(rsst_handle h) {
  if (!h) return RSST_E_ARG;
  (void)hipDeviceSynchronize();
  (void)hipFree(h->u1);
  (void)hipFree(h->scal);
  (void)hipFree(h->blkmax);
  (void)hipFree(h->part);
  (void)hipFree(h->diag_out);
  if (h->adj_work) (void)hipFree(h->adj_work);
  delete h;
  return RSST_OK;
}

static rsstk::AdjointPlan adjoint_plan(rsst_handle h) {
  const rsst_config& c = h->cfg;
  rsstk::AdjointPlan p{};
  p.ndim = c.ndim;
  for (int d = 0; d < 3; ++d) {
    p.n[d] = c.n[d];
    p.refl_lo[d] = d < c.ndim && c.bc_lo[d] == RSST_REFLECT;
    p.refl_hi[d] = d < c.ndim && c.bc_hi[d] == RSST_REFLECT;
    p.inv_dx[d] = d < c.ndim ? 1.0 / c.dx[d] : 0.0;
    p.g[d] = d < c.ndim ? c.g[d] : 0.0;
  }
  p.gamma = c.gamma;
  p.xi = c.xi;
  p.form = c.form;
  p.ncell = h->ncell;
  p.work = h->adj_work;
  return p;
}

// U1 = U + dt R(U) into the stage buffer: the same stage-1 kernel as the
// forward step.
static hipError_t recompute_u1(rsst_handle h, const void* U, double dt, hipStream_t s) {
  StageArgs a = h->args;
  a.dt_fixed = dt;
  a.uin = U;
  a.un = nullptr;
  a.uout = h->u1;
  return rsstk::launch_stage(a, 1, s);
}

int rsst_adjoint_step(rsst_handle h, const void* U, double* lam, double dt, double* dJdxi, void* stream) {
  if (!h || !U || !lam || !dJdxi || !(dt > 0.0) || !std::isfinite(dt)) return RSST_E_ARG;
  if (!h->adj_work) return RSST_E_UNSUPPORTED;
  hipStream_t s = (hipStream_t)stream;
  if (recompute_u1(h, U, dt, s) != hipSuccess) return RSST_E_DEVICE;
  return check(rsstk::launch_adjoint_step(adjoint_plan(h), (const double*)U, (const double*)h->u1, lam, dt, dJdxi,
                                          false, s));
}

int rsst_adjoint_step_u1(rsst_handle h, const void* U, const void* U1, double* lam, double dt, double* dJdxi,
                         void* stream) {
  if (!h || !U || !U1 || !lam || !dJdxi || !(dt > 0.0) || !std::isfinite(dt)) return RSST_E_ARG;
  if (!h->adj_work) return RSST_E_UNSUPPORTED;
  return check(rsstk::launch_adjoint_step(adjoint_plan(h), (const double*)U, (const double*)U1, lam, dt, dJdxi,
                                          false, (hipStream_t)stream));
}

int rsst_adjoint_run(rsst_handle h, const void* const* U_list, const void* const* U1_list, int nsteps, double* lam,
                     double dt, double* dJdxi, void* stream) {
  if (!h || !U_list || !lam || !dJdxi || nsteps < 0 || !(dt > 0.0) || !std::isfinite(dt)) return RSST_E_ARG;
  if (!h->adj_work) return RSST_E_UNSUPPORTED;
  for (int n = 0; n < nsteps; ++n)
    if (!U_list[n] || (U1_list && !U1_list[n])) return RSST_E_ARG;
  hipStream_t s = (hipStream_t)stream;
  const rsstk::AdjointPlan p = adjoint_plan(h);
  // 2D: each step adds its dJ/dxi share per tile into the run accumulator,
  // folded into dJdxi once after the last step
  const bool defer = p.ndim == 2;
  for (int n = nsteps - 1; n >= 0; --n) {
    const void* U1 = U1_list ? U1_list[n] : h->u1;
    if (!U1_list && recompute_u1(h, U_list[n], dt, s) != hipSuccess) return RSST_E_DEVICE;
    if (rsstk::launch_adjoint_step(p, (const double*)U_list[n], (const double*)U1, lam, dt, dJdxi, defer, s) !=
        hipSuccess)
      return RSST_E_DEVICE;
  }
  if (defer && nsteps > 0 && rsstk::launch_adjoint_xi_fold(p, dJdxi, s) != hipSuccess) return RSST_E_DEVICE;
  return check(hipGetLastError());
}

int rsst_step_noalloc(const rsst_config* cfg, void* U, double dt_fixed, uint32_t* flags, void* stream) {
  if (!U || !std::isfinite(dt_fixed)) return RSST_E_ARG;
  int st = validate(cfg);
  if (st != RSST_OK) return st;
  if ((cfg->flags & RSST_WITH_ADJOINT) || cfg->t_end != 0.0) return RSST_E_UNSUPPORTED;
  const long long ncell = (long long)cfg->n[0] * cfg->n[1] * cfg->n[2];
  const size_t elem = cfg->prec == RSST_FP32_PERT ? sizeof(float) : sizeof(double);
  StageArgs a;
  fill_args(cfg, ncell, a);
  // scratch layout: scalars | CFL maxima | U1, each 256-byte aligned
  const size_t o_blk = round256(rsstk::kNumScalars * sizeof(double));
  const size_t o_u1 = o_blk + round256((size_t)a.nblk * sizeof(double));
  const size_t need = o_u1 + (size_t)(cfg->ndim + 2) * (size_t)ncell * elem;
  if (need > kScratchBytes) return RSST_E_SCRATCH;
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return RSST_E_DEVICE;
  unsigned char* base = nullptr;
  st = scratch_on(dev, &base);
  if (st != RSST_OK) return st;
  hipStream_t s = (hipStream_t)stream;
  a.scal = (double*)base;
  a.blkmax = (double*)(base + o_blk);
  void* u1 = base + o_u1;
  a.dt_fixed = dt_fixed > 0.0 ? dt_fixed : 0.0;
  hipLaunchKernelGGL(noalloc_clear_kernel, dim3(1), dim3(64), 0, s, a.scal);
  if (hipGetLastError() != hipSuccess) return RSST_E_DEVICE;
  // a CFL step: the maxima of U, t = 0
  if (!(dt_fixed > 0.0) && rsstk::launch_prime(a, U, 0.0, 1, s) != hipSuccess) return RSST_E_DEVICE;
  StageArgs a1 = a, a2 = a;
  a1.uin = U;
  a1.un = nullptr;
  a1.uout = u1;
  a2.uin = u1;
  a2.un = U;
  a2.uout = U;
  if (rsstk::launch_stage(a1, 1, s) != hipSuccess || rsstk::launch_stage(a2, 2, s) != hipSuccess)
    return RSST_E_DEVICE;
  if (flags) {
    hipLaunchKernelGGL(noalloc_flags_kernel, dim3(1), dim3(64), 0, s, (const double*)a.scal, flags);
    if (hipGetLastError() != hipSuccess) return RSST_E_DEVICE;
  }
  return RSST_OK;
}

}  // extern "C"

