// Batched RSST: many independent 2D boxes of uneven size, xi and
// background, advanced by one persistent kernel per run, captured in a HIP
// graph and replayed.
//
// Work items are (stage q, box b, strip block p), q = 2 n + stage - 1 for
// step n.  A strip block is `groups` consecutive strips of `strip` rows
// (y, the marched axis) processed side by side by one 256-thread workgroup
// (a box row of nwx <= 4 waves; narrow boxes run 4/nwx strips at once).
// Tickets are handed out in q-major order by one atomic counter, and an item
// only waits on items with smaller tickets:
//   * the strip blocks of its box at q-1 that hold a row within two cells
//     of its own rows (through the boundary rule: a periodic y wraps the
//     first block onto the last ones), or whose rows are within two cells
//     of its own; this orders every read of a row by the previous stage
//     before the in-place stage-2 write of U, and every stage-2 read of U1
//     before the next stage-1 write of it;
//   * for stage 1 of step n > 0, every stage-2 block of step n-1 of its
//     box, whose per-box maximum of c_tot gives the box's CFL dt.
// Every waiting item holds a ticket larger than the ones it waits for, and
// those were taken by running workgroups, so the queue cannot deadlock.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstring>
#include <new>
#include <vector>

#include "rsst.h"
#include "rsst_stage2.h"

#pragma clang fp contract(off)

namespace rsstk {

constexpr int kBatchThreads = 256;  // one box row: at most 4 waves
// Persistent workgroups per CU.  A workgroup is one wave per SIMD, so this is
// also the waves per SIMD the kernel is compiled for (its register budget).
// Measured with 137-VGPR one-plane strips, three per CU were 0-65% slower
// than two on every strip choice (more items in flight, each slower).
constexpr int kBatchPerCU = 2;

struct BoxDev {
  StageArgs s1, s2;  // stage views of the box (pointers into U_all / U1_all)
  double cfl_h;      // cfl * h of the box
  int nblk;          // strip blocks
  int rbase;         // index of the box's first item in a stage
  int groups;        // strips per block
  int pad;
};

// A work item: strip block `blk` of box `box`, and the blocks of the same
// box whose rows its stencil reads or whose stencil reads its rows (the
// order it needs against the previous stage).
constexpr int kMaxDeps = 8;
static_assert(5 + kMaxDeps == RSST_BATCH_PLAN_COLS, "plan table layout");
struct Item {
  int box, blk, ndep;
  int dep[kMaxDeps];
};

struct BatchState {
  unsigned* ticket;              // next ticket
  unsigned long long* maxbits;   // [nbox][max_steps + 1] max c_tot of the input of each step
  unsigned* cnt2;                // [nbox][max_steps] stage-2 blocks done per step
  unsigned* done;                // [2 max_steps][nitem] item done flags
  double* tacc;                  // [nbox] time reached
  unsigned* flags;               // non-physical flags
  int nbox, nitem, nsteps, max_steps;
  unsigned total;                // 2 nsteps nitem tickets
  unsigned long long wait_ticks; // longest dependency wait, in wall-clock ticks (100 MHz)
};

__device__ __forceinline__ unsigned ld_acquire(const unsigned* p) {
  return __hip_atomic_load(p, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT);
}

// Flag bit of a run whose queue gave up on a dependency wait (reported by
// rsst_batch_poll as RSST_E_DEVICE): a wait past its deadline means a
// dependency that will not arrive, so instead of spinning for ever the item
// is skipped (marked done, nothing stored) and every workgroup drains.
constexpr unsigned kQueueTimeout = 8u;

// Spins until *p >= v or the wall clock passes `deadline`; false on timeout.
__device__ __forceinline__ bool wait_at_least(const unsigned* p, unsigned v, unsigned long long deadline) {
  while (ld_acquire(p) < v) {
    if (wall_clock64() > deadline) return false;
    __builtin_amdgcn_s_sleep(2);
  }
  return true;
}

// Clears the per-run counters (graph-safe: a kernel, not a memset node).
__global__ void __launch_bounds__(256) batch_reset_kernel(BatchState S) {
  const long long tid = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  const long long stride = (long long)gridDim.x * blockDim.x;
  if (tid == 0) *S.ticket = 0u;
  for (long long q = tid; q < (long long)S.nbox * (S.max_steps + 1); q += stride) S.maxbits[q] = 0ull;
  for (long long q = tid; q < (long long)S.nbox * S.max_steps; q += stride) S.cnt2[q] = 0u;
  for (long long q = tid; q < 2ll * S.max_steps * S.nitem; q += stride) S.done[q] = 0u;
}

// Per-box maximum of c_tot of the initial state -> maxbits[b][0].
template <typename ST>
__global__ void __launch_bounds__(256) batch_prime_kernel(const BoxDev* __restrict__ boxes, BatchState S,
                                                         int blocks_per_box) {
  constexpr int NV = 4;
  const int b = blockIdx.x / blocks_per_box, part = blockIdx.x % blocks_per_box;
  const StageArgs& A = boxes[b].s1;
  const Consts K{A.gamma, A.gm1, A.inv_gm1, A.inv_xi, A.f};
  const ST* u = (const ST*)A.uin;
  __shared__ double red[4];
  double cm = 0.0;
  for (long long c = (long long)part * blockDim.x + threadIdx.x; c < A.ncell;
       c += (long long)blocks_per_box * blockDim.x) {
    double q[NV];
    const int y = (int)(c / A.geo.nx);
#pragma unroll
    for (int v = 0; v < NV; ++v) {
      q[v] = (double)u[v * A.ncell + c];
      if constexpr (sizeof(ST) == 4) q[v] += A.bg[v * A.nbg + (A.bg_axis == 1 ? y : 0)];
    }
    cm = fmax(cm, cell_ctot<2>(q, K));
  }
  const double wm = wave_max(cm);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = wm;
  __syncthreads();
  if (threadIdx.x == 0) {
    const double m = fmax(fmax(red[0], red[1]), fmax(red[2], red[3]));
    atomicMax(S.maxbits + (long long)b * (S.max_steps + 1), (unsigned long long)__double_as_longlong(m));
  }
}

// Completion of an item: its per-box c_tot maximum (stage 2), the box time,
// then the done flag and the per-step stage-2 count with release order.
struct Pending {
  int b, p, n;
  unsigned q, r;
  bool st2;
  double dt;
};

__device__ __forceinline__ void signal_done(const BatchState& S, const Pending& d, const double* red) {
  if (d.st2) {
    double m = 0.0;
    for (int w = 0; w < kBatchThreads / 64; ++w) m = fmax(m, red[w]);
    atomicMax(S.maxbits + (long long)d.b * (S.max_steps + 1) + d.n + 1,
              (unsigned long long)__double_as_longlong(m));
    if (d.p == 0) S.tacc[d.b] += d.dt;
    __threadfence();
  }
  __hip_atomic_store(S.done + (long long)d.q * S.nitem + d.r, 1u, __ATOMIC_RELEASE,
                     __HIP_MEMORY_SCOPE_AGENT);
  if (d.st2)
    __hip_atomic_fetch_add(S.cnt2 + (long long)d.b * S.max_steps + d.n, 1u, __ATOMIC_RELEASE,
                           __HIP_MEMORY_SCOPE_AGENT);
}

// Thread 0 acts for the workgroup in exactly one region per iteration
// besides the dependency wait: it signals the item just finished and takes
// the next ticket.  Both sit between barriers, so no single-thread region
// ends one iteration and another begins the next; the compiler could
// otherwise join the two across the back edge into a loop that thread 0
// leaves while the rest of its wave goes round without it.
template <typename ST, int FORM>
__global__ void __launch_bounds__(kBatchThreads) __attribute__((amdgpu_waves_per_eu(kBatchPerCU))) batch_kernel(const BoxDev* __restrict__ boxes,
                                                            const Item* __restrict__ items,
                                                            BatchState S) {
  extern __shared__ double lds[];
  __shared__ unsigned tshare, skip;
  __shared__ double red[kBatchThreads / 64];
  const int tid = threadIdx.x;
  Pending prev{-1, 0, 0, 0u, 0u, false, 0.0};
  for (;;) {
    if (tid == 0) {
      if (prev.b >= 0) signal_done(S, prev, red);
      tshare = atomicAdd(S.ticket, 1u);
    }
    __syncthreads();
    const unsigned t = __builtin_amdgcn_readfirstlane(tshare);  // uniform: SGPR box fields
    __syncthreads();
    if (t >= S.total) break;
    const int q = (int)(t / (unsigned)S.nitem), r = (int)(t % (unsigned)S.nitem);
    const Item it = items[r];
    // box and block are workgroup-uniform: said explicitly, every field of
    // the box's stage views stays in scalar registers (otherwise the compiler
    // wraps each buffer access built from them in a per-lane waterfall loop)
    const int b = __builtin_amdgcn_readfirstlane(it.box), p = __builtin_amdgcn_readfirstlane(it.blk), n = q >> 1;
    const bool st2 = (q & 1) != 0;
    const BoxDev& B = boxes[b];
    if (tid == 0) {
      const unsigned long long deadline = wall_clock64() + S.wait_ticks;
      bool ok = true;
      if (!st2 && n > 0)
        ok = wait_at_least(S.cnt2 + (long long)b * S.max_steps + (n - 1), (unsigned)B.nblk, deadline);
      if (q > 0) {
        const unsigned* dq = S.done + (long long)(q - 1) * S.nitem + B.rbase;
        for (int d = 0; d < it.ndep && ok; ++d) ok = wait_at_least(dq + it.dep[d], 1u, deadline);
      }
      if (!ok) atomicOr(S.flags, kQueueTimeout);
      skip = ok ? 0u : 1u;
    }
    __syncthreads();
    const bool skip_item = __builtin_amdgcn_readfirstlane(skip) != 0u;
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
    const unsigned long long mb = __hip_atomic_load(S.maxbits + (long long)b * (S.max_steps + 1) + n,
                                                    __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    const double dt = B.cfl_h / __longlong_as_double((long long)mb);
    unsigned bad = 0;
    double cmax = 0.0;
    if (skip_item) {
      // nothing computed or stored; the item is still signalled done below
    } else if (!st2) {
      cmax = stage_body2<1, ST, FORM, 2>(B.s1, lds, p * B.groups, dt, bad);
    } else {
      cmax = stage_body2<2, ST, FORM, 2>(B.s2, lds, p * B.groups, dt, bad);
    }
    if (bad) atomicOr(S.flags, bad);
    if (st2) {
      const double wm = wave_max(cmax);
      if ((tid & 63) == 0) red[tid >> 6] = wm;
    }
    // every thread's stores are complete device-wide before the signal
    __threadfence();
    __syncthreads();
    prev = Pending{b, p, n, (unsigned)q, (unsigned)r, st2, dt};
  }
}

template <typename ST>
static void* batch_kernel_ptr(int form) {
  switch (form) {
    case kEuler: return (void*)batch_kernel<ST, kEuler>;
    case kPVS: return (void*)batch_kernel<ST, kPVS>;
    case kPMS: return (void*)batch_kernel<ST, kPMS>;
    case kDVS: return (void*)batch_kernel<ST, kDVS>;
    case kDMS: return (void*)batch_kernel<ST, kDMS>;
    default: return (void*)batch_kernel<ST, kPD>;
  }
}

}  // namespace rsstk

using namespace rsstk;

struct rsst_batch_s {
  int nbox, prec, form, max_steps;
  std::vector<rsst_config> cfg;
  std::vector<long long> off;     // element offsets of the boxes in U_all
  long long total_elems;          // size of U_all (elements)
  int strip[4];                   // strip rows per width class (1..4 waves per row)
  // per-build host tables
  std::vector<BoxDev> boxes;
  std::vector<Item> items;
  int nitem;
  size_t lds_bytes;
  // device memory
  void* u1;
  BoxDev* d_boxes;
  Item* d_items;
  int d_items_cap;
  unsigned* d_ticket;
  unsigned long long* d_maxbits;
  unsigned* d_cnt2;
  unsigned* d_done;
  long long d_done_cap;
  double* d_tacc;
  unsigned* d_flags;
  // graph of the last run
  hipStream_t cap_stream;
  hipGraphExec_t exec;
  void* cap_U;
  int cap_steps;
  bool dirty;
  int grid;
  unsigned long long wait_ticks;  // dependency-wait limit of the queue (100 MHz ticks)
};

static int batch_validate(const rsst_config* c, int nbox, const int64_t* off) {
  if (!c || nbox < 1 || !off) return RSST_E_ARG;
  for (int b = 0; b < nbox; ++b) {
    const rsst_config& k = c[b];
    if (k.ndim != 2) return RSST_E_UNSUPPORTED;
    if (k.n[0] < 4 || k.n[1] < 4 || k.n[2] != 1) return RSST_E_ARG;
    if (k.n[0] > 256) return RSST_E_UNSUPPORTED;
    if (!(k.dx[0] > 0) || !(k.dx[1] > 0)) return RSST_E_ARG;
    for (int d = 0; d < 2; ++d) {
      if (k.bc_lo[d] < RSST_PERIODIC || k.bc_lo[d] > RSST_REFLECT_HYDRO) return RSST_E_ARG;
      if (k.bc_hi[d] < RSST_PERIODIC || k.bc_hi[d] > RSST_REFLECT_HYDRO) return RSST_E_ARG;
      if ((k.bc_lo[d] == RSST_PERIODIC) != (k.bc_hi[d] == RSST_PERIODIC)) return RSST_E_ARG;
    }
    if (!(k.gamma > 1.0) || !(k.xi >= 1.0) || !(k.cfl > 0.0 && k.cfl <= 1.0)) return RSST_E_ARG;
    if (k.form != c[0].form || k.prec != c[0].prec) return RSST_E_UNSUPPORTED;
    if (k.form < RSST_EULER || k.form > RSST_PD) return RSST_E_ARG;
    if (k.prec == RSST_FP32_PERT && (!k.bg || (k.bg_axis != -1 && k.bg_axis != 1))) return RSST_E_ARG;
    if (k.t_end != 0.0 || k.cmax != 0.0 || k.flags != 0 || k.eos != RSST_EOS_IDEAL) return RSST_E_UNSUPPORTED;
    for (int d = 0; d < 2; ++d)
      if (k.bc_lo[d] == RSST_REFLECT_HYDRO || k.bc_hi[d] == RSST_REFLECT_HYDRO) return RSST_E_UNSUPPORTED;
    if (off[b] < 0) return RSST_E_ARG;
    const long long bytes = 4ll * k.n[0] * k.n[1] * (k.prec == RSST_FP32_PERT ? 4 : 8);
    if (bytes >= (1ll << 31)) return RSST_E_UNSUPPORTED;
  }
  return RSST_OK;
}

// Row index after the boundary rule of the marched axis (the host copy of
// the device rule: reflecting sides mirror, periodic sides wrap).
static int host_map_row(int q, int n, int refl_lo, int refl_hi) {
  if (q < 0) return refl_lo ? -1 - q : q + n;
  if (q >= n) return refl_hi ? 2 * n - 1 - q : q - n;
  return q;
}

// Strip blocks of one box and their dependency lists, appended to `items`.
// A block is `groups` strips of `km` rows (the rows of one workgroup row
// group); the march runs along y.
static int plan_box(const rsst_config& c, const int strip[4], int b, std::vector<Item>& items, int& km,
                    int& groups, int& nblk) {
  const int nx = c.n[0], nm = c.n[1];
  const int nwx = (nx + 63) / 64;
  groups = 4 / nwx;
  km = strip[nwx - 1] < nm ? strip[nwx - 1] : nm;
  const int nchunk = (nm + km - 1) / km;
  nblk = (nchunk + groups - 1) / groups;
  // rows [k0, k1) of each block; blocks reading each other's rows
  const int rows = groups * km;
  const int rlo = c.bc_lo[1] == RSST_REFLECT, rhi = c.bc_hi[1] == RSST_REFLECT;
  std::vector<std::vector<char>> rel(nblk, std::vector<char>(nblk, 0));
  for (int p = 0; p < nblk; ++p) {
    const int k0 = p * rows, k1 = std::min(k0 + rows, nm);
    for (int k = k0 - 2; k < k1 + 2; ++k) {
      const int o = host_map_row(k, nm, rlo, rhi) / rows;
      rel[p][o] = rel[o][p] = 1;
    }
  }
  for (int p = 0; p < nblk; ++p) {
    Item it{};
    it.box = b;
    it.blk = p;
    for (int o = 0; o < nblk; ++o)
      if (rel[p][o]) {
        if (it.ndep == kMaxDeps) return RSST_E_UNSUPPORTED;
        it.dep[it.ndep++] = o;
      }
    items.push_back(it);
  }
  return RSST_OK;
}

// Stage views, strip blocks and the item table for the current strip rows.
static int batch_build(rsst_batch_s* h, void* U) {
  h->boxes.assign(h->nbox, BoxDev{});
  h->items.clear();
  size_t lds = 0;
  for (int b = 0; b < h->nbox; ++b) {
    const rsst_config& c = h->cfg[b];
    BoxDev& B = h->boxes[b];
    B.rbase = (int)h->items.size();
    int km = 0, groups = 0, nblk = 0;
    const int ps = plan_box(c, h->strip, b, h->items, km, groups, nblk);
    if (ps != RSST_OK) return ps;
    StageArgs a;
    std::memset(&a, 0, sizeof(a));
    Geometry& G = a.geo;
    G.ndim = 2;
    G.nx = c.n[0];
    G.ns = 1;
    G.nm = c.n[1];
    G.nwx = (G.nx + 63) / 64;
    G.ts = groups;
    G.km = km;
    G.np = 2;
    G.ntile_s = 1;
    G.nchunk = (G.nm + G.km - 1) / G.km;
    G.threads = kBatchThreads;
    G.lds_bytes = (size_t)carve2(groups, G.nwx, 2).total * sizeof(double);
    if (G.lds_bytes > lds) lds = G.lds_bytes;
    a.ncell = (long long)G.nx * G.nm;
    for (int d = 0; d < 3; ++d) {
      a.bc_lo[d] = c.bc_lo[d];
      a.bc_hi[d] = c.bc_hi[d];
      a.inv_dx[d] = d < 2 ? 1.0 / c.dx[d] : 0.0;
      a.g[d] = d < 2 ? c.g[d] : 0.0;
    }
    a.gamma = c.gamma;
    a.gm1 = c.gamma - 1.0;
    a.inv_gm1 = 1.0 / (c.gamma - 1.0);
    a.inv_xi = 1.0 / c.xi;
    a.f = 1.0 - 1.0 / (c.xi * c.xi);
    a.form = c.form;
    a.prec = c.prec;
    a.bg = c.bg;
    a.bg_axis = c.prec == RSST_FP32_PERT ? c.bg_axis : -1;
    a.nbg = a.bg_axis >= 0 ? c.n[a.bg_axis] : 1;
    a.bg_uniform = (a.bg_axis == -1 || a.bg_axis == 1) ? 1 : 0;
    const size_t es = c.prec == RSST_FP32_PERT ? 4 : 8;
    char* u = (char*)U + h->off[b] * es;
    char* u1 = (char*)h->u1 + h->off[b] * es;
    B.s1 = a;
    B.s1.uin = u;
    B.s1.un = nullptr;
    B.s1.uout = u1;
    B.s2 = a;
    B.s2.uin = u1;
    B.s2.un = u;
    B.s2.uout = u;
    double hl;
    if (c.dt_rule == 1) hl = std::fmin(c.dx[0], c.dx[1]);
    else hl = 1.0 / (1.0 / c.dx[0] + 1.0 / c.dx[1]);
    B.cfl_h = c.cfl * hl;
    B.groups = groups;
    B.nblk = nblk;
  }
  h->nitem = (int)h->items.size();
  h->lds_bytes = lds;
  return RSST_OK;
}

template <typename ST>
static hipError_t batch_launch_all(rsst_batch_s* h, hipStream_t s, int nsteps) {
  BatchState S;
  S.ticket = h->d_ticket;
  S.maxbits = h->d_maxbits;
  S.cnt2 = h->d_cnt2;
  S.done = h->d_done;
  S.tacc = h->d_tacc;
  S.flags = h->d_flags;
  S.nbox = h->nbox;
  S.nitem = h->nitem;
  S.nsteps = nsteps;
  S.max_steps = h->max_steps;
  S.total = (unsigned)(2ll * nsteps * h->nitem);
  S.wait_ticks = h->wait_ticks;
  hipLaunchKernelGGL(batch_reset_kernel, dim3(256), dim3(256), 0, s, S);
  const int bpb = 8;
  hipLaunchKernelGGL(batch_prime_kernel<ST>, dim3(h->nbox * bpb), dim3(256), 0, s, h->d_boxes, S, bpb);
  void* kern = batch_kernel_ptr<ST>(h->form);
  void* args[] = {(void*)&h->d_boxes, (void*)&h->d_items, (void*)&S};
  hipError_t e = hipLaunchKernel(kern, dim3(h->grid), dim3(kBatchThreads), args, h->lds_bytes, s);
  if (e != hipSuccess) return e;
  return hipGetLastError();
}

static int batch_prepare(rsst_batch_s* h, void* U, int nsteps) {
  const int bs = batch_build(h, U);
  if (bs != RSST_OK) return bs;
  if (h->nitem > h->d_items_cap || 2ll * h->max_steps * h->nitem > h->d_done_cap)
    return RSST_E_UNSUPPORTED;  // strip rows below those sized at init
  if (hipMemcpy(h->d_boxes, h->boxes.data(), sizeof(BoxDev) * h->nbox, hipMemcpyHostToDevice) != hipSuccess)
    return RSST_E_DEVICE;
  if (hipMemcpy(h->d_items, h->items.data(), sizeof(Item) * h->nitem, hipMemcpyHostToDevice) != hipSuccess)
    return RSST_E_DEVICE;
  void* kern = h->prec ? batch_kernel_ptr<float>(h->form) : batch_kernel_ptr<double>(h->form);
  if (hipFuncSetAttribute(kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)h->lds_bytes) != hipSuccess)
    return RSST_E_DEVICE;
  int per_cu = 0, dev = 0, ncu = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kern, kBatchThreads, h->lds_bytes) != hipSuccess)
    return RSST_E_DEVICE;
  if (hipGetDevice(&dev) != hipSuccess ||
      hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
    return RSST_E_DEVICE;
  // at most kBatchPerCU workgroups per CU
  if (per_cu > kBatchPerCU) per_cu = kBatchPerCU;
  h->grid = (per_cu > 0 ? per_cu : 1) * ncu;
  // capture reset + prime + persistent kernel in one graph
  if (h->exec) {
    (void)hipGraphExecDestroy(h->exec);
    h->exec = nullptr;
  }
  hipGraph_t graph = nullptr;
  if (hipStreamBeginCapture(h->cap_stream, hipStreamCaptureModeThreadLocal) != hipSuccess) return RSST_E_DEVICE;
  hipError_t e = h->prec ? batch_launch_all<float>(h, h->cap_stream, nsteps)
                         : batch_launch_all<double>(h, h->cap_stream, nsteps);
  hipError_t e2 = hipStreamEndCapture(h->cap_stream, &graph);
  if (e != hipSuccess || e2 != hipSuccess || !graph) {
    if (graph) (void)hipGraphDestroy(graph);
    return RSST_E_DEVICE;
  }
  e = hipGraphInstantiate(&h->exec, graph, nullptr, nullptr, 0);
  (void)hipGraphDestroy(graph);
  if (e != hipSuccess) return RSST_E_DEVICE;
  h->cap_U = U;
  h->cap_steps = nsteps;
  h->dirty = false;
  return RSST_OK;
}

extern "C" {

int rsst_batch_init(const rsst_config* boxes, int nbox, const int64_t* offsets, int max_steps,
                    void* stream, rsst_batch* out) {
  if (!out) return RSST_E_ARG;
  *out = nullptr;
  if (max_steps < 1) return RSST_E_ARG;
  int st = batch_validate(boxes, nbox, offsets);
  if (st != RSST_OK) return st;
  rsst_batch_s* h = new (std::nothrow) rsst_batch_s();
  if (!h) return RSST_E_NOMEM;
  h->nbox = nbox;
  h->prec = boxes[0].prec;
  h->form = boxes[0].form;
  h->max_steps = max_steps;
  h->cfg.assign(boxes, boxes + nbox);
  h->off.resize(nbox);
  h->total_elems = 0;
  for (int b = 0; b < nbox; ++b) {
    h->off[b] = offsets[b];
    const long long end = offsets[b] + 4ll * boxes[b].n[0] * boxes[b].n[1];
    if (end > h->total_elems) h->total_elems = end;
  }
  h->strip[0] = h->strip[1] = h->strip[2] = h->strip[3] = 16;
  h->wait_ticks = 1000000000ull;  // 10 s
  // size item tables for the shortest strips the tile setter accepts (8 rows)
  long long cap_items = 0;
  for (int b = 0; b < nbox; ++b) {
    const int nwx = (boxes[b].n[0] + 63) / 64, groups = 4 / nwx;
    cap_items += ((boxes[b].n[1] + 7) / 8 + groups - 1) / groups;
  }
  const size_t es = h->prec == RSST_FP32_PERT ? 4 : 8;
  h->d_items_cap = (int)cap_items;
  h->d_done_cap = 2ll * max_steps * cap_items;
  bool ok = hipMalloc(&h->u1, (size_t)h->total_elems * es) == hipSuccess;
  ok = ok && hipMalloc((void**)&h->d_boxes, sizeof(BoxDev) * nbox) == hipSuccess;
  ok = ok && hipMalloc((void**)&h->d_items, sizeof(Item) * (size_t)cap_items) == hipSuccess;
  ok = ok && hipMalloc((void**)&h->d_ticket, sizeof(unsigned)) == hipSuccess;
  ok = ok && hipMalloc((void**)&h->d_maxbits, sizeof(unsigned long long) * (size_t)nbox * (max_steps + 1)) == hipSuccess;
  ok = ok && hipMalloc((void**)&h->d_cnt2, sizeof(unsigned) * (size_t)nbox * max_steps) == hipSuccess;
  ok = ok && hipMalloc((void**)&h->d_done, sizeof(unsigned) * (size_t)h->d_done_cap) == hipSuccess;
  ok = ok && hipMalloc((void**)&h->d_tacc, sizeof(double) * nbox) == hipSuccess;
  ok = ok && hipMalloc((void**)&h->d_flags, sizeof(unsigned)) == hipSuccess;
  ok = ok && hipStreamCreateWithFlags(&h->cap_stream, hipStreamNonBlocking) == hipSuccess;
  if (!ok) {
    rsst_batch_destroy(h);
    return RSST_E_NOMEM;
  }
  hipStream_t s = (hipStream_t)stream;
  if (hipMemsetAsync(h->d_tacc, 0, sizeof(double) * nbox, s) != hipSuccess ||
      hipMemsetAsync(h->d_flags, 0, sizeof(unsigned), s) != hipSuccess ||
      hipStreamSynchronize(s) != hipSuccess) {
    rsst_batch_destroy(h);
    return RSST_E_DEVICE;
  }
  h->dirty = true;
  *out = h;
  return RSST_OK;
}

int rsst_batch_plan(const rsst_config* boxes, int nbox, const int strip_rows[4], int* table, int cap,
                    int* nitem) {
  if (!boxes || nbox < 1 || !strip_rows || !nitem || cap < 0 || (cap > 0 && !table)) return RSST_E_ARG;
  std::vector<int64_t> off(nbox, 0);
  const int st = batch_validate(boxes, nbox, off.data());
  if (st != RSST_OK) return st;
  for (int c = 0; c < 4; ++c)
    if (strip_rows[c] < 8 || strip_rows[c] > 256) return RSST_E_ARG;
  std::vector<Item> items;
  for (int b = 0; b < nbox; ++b) {
    int km = 0, groups = 0, nblk = 0;
    const int ps = plan_box(boxes[b], strip_rows, b, items, km, groups, nblk);
    if (ps != RSST_OK) return ps;
    for (size_t i = items.size() - nblk; i < items.size(); ++i) {
      const Item& it = items[i];
      if ((long long)i >= cap) continue;
      int* row = table + i * RSST_BATCH_PLAN_COLS;
      const int rows = groups * km;
      row[0] = it.box;
      row[1] = it.blk;
      row[2] = it.blk * rows;
      row[3] = std::min((it.blk + 1) * rows, boxes[b].n[1]);
      row[4] = it.ndep;
      for (int d = 0; d < kMaxDeps; ++d) row[5 + d] = d < it.ndep ? it.dep[d] : -1;
    }
  }
  *nitem = (int)items.size();
  return RSST_OK;
}

int rsst_batch_set_tiles(rsst_batch h, const int strip_rows[4]) {
  if (!h || !strip_rows) return RSST_E_ARG;
  for (int c = 0; c < 4; ++c)
    if (strip_rows[c] < 8 || strip_rows[c] > 256) return RSST_E_ARG;
  for (int c = 0; c < 4; ++c) h->strip[c] = strip_rows[c];
  h->dirty = true;
  return RSST_OK;
}

int rsst_batch_get_tiles(rsst_batch h, int strip_rows[4]) {
  if (!h || !strip_rows) return RSST_E_ARG;
  for (int c = 0; c < 4; ++c) strip_rows[c] = h->strip[c];
  return RSST_OK;
}

int rsst_batch_run(rsst_batch h, void* U_all, int nsteps, void* stream) {
  if (!h || !U_all || nsteps < 1 || nsteps > h->max_steps) return RSST_E_ARG;
  hipStream_t s = (hipStream_t)stream;
  if (h->dirty || U_all != h->cap_U || nsteps != h->cap_steps) {
    // rebuilding the tables copies from the host: order after earlier work
    if (hipStreamSynchronize(s) != hipSuccess) return RSST_E_DEVICE;
    int st = batch_prepare(h, U_all, nsteps);
    if (st != RSST_OK) return st;
  }
  return hipGraphLaunch(h->exec, s) == hipSuccess ? RSST_OK : RSST_E_DEVICE;
}

int rsst_batch_times(rsst_batch h, double* t, void* stream) {
  if (!h || !t) return RSST_E_ARG;
  if (hipStreamSynchronize((hipStream_t)stream) != hipSuccess) return RSST_E_DEVICE;
  return hipMemcpy(t, h->d_tacc, sizeof(double) * h->nbox, hipMemcpyDeviceToHost) == hipSuccess
             ? RSST_OK
             : RSST_E_DEVICE;
}

int rsst_batch_set_wait_limit(rsst_batch h, double seconds) {
  if (!h || !(seconds >= 0.0) || !(seconds <= 3600.0)) return RSST_E_ARG;
  h->wait_ticks = (unsigned long long)(seconds * 1e8);
  h->dirty = true;
  return RSST_OK;
}

int rsst_batch_set_times(rsst_batch h, const double* t, uint32_t flags, void* stream) {
  if (!h || !t) return RSST_E_ARG;
  hipStream_t s = (hipStream_t)stream;
  if (hipStreamSynchronize(s) != hipSuccess) return RSST_E_DEVICE;
  if (hipMemcpy(h->d_tacc, t, sizeof(double) * h->nbox, hipMemcpyHostToDevice) != hipSuccess ||
      hipMemcpy(h->d_flags, &flags, sizeof(flags), hipMemcpyHostToDevice) != hipSuccess)
    return RSST_E_DEVICE;
  return RSST_OK;
}

int rsst_batch_poll(rsst_batch h, uint32_t* flags) {
  if (!h) return RSST_E_ARG;
  if (hipDeviceSynchronize() != hipSuccess) return RSST_E_DEVICE;
  uint32_t f = 0;
  if (hipMemcpy(&f, h->d_flags, sizeof(f), hipMemcpyDeviceToHost) != hipSuccess) return RSST_E_DEVICE;
  if (f) {
    uint32_t z = 0;
    if (hipMemcpy(h->d_flags, &z, sizeof(z), hipMemcpyHostToDevice) != hipSuccess) return RSST_E_DEVICE;
  }
  if (flags) *flags = f;
  if (f & kQueueTimeout) return RSST_E_DEVICE;
  return f ? RSST_E_NONPHYSICAL : RSST_OK;
}

int rsst_batch_destroy(rsst_batch h) {
  if (!h) return RSST_E_ARG;
  (void)hipDeviceSynchronize();
  if (h->exec) (void)hipGraphExecDestroy(h->exec);
  if (h->cap_stream) (void)hipStreamDestroy(h->cap_stream);
  (void)hipFree(h->u1);
  (void)hipFree(h->d_boxes);
  (void)hipFree(h->d_items);
  (void)hipFree(h->d_ticket);
  (void)hipFree(h->d_maxbits);
  (void)hipFree(h->d_cnt2);
  (void)hipFree(h->d_done);
  (void)hipFree(h->d_tacc);
  (void)hipFree(h->d_flags);
  delete h;
  return RSST_OK;
}

}  // extern "C"
