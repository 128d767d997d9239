// Fused RSST stage kernels for gfx950 (the kernels themselves are
// instantiated per dimension and storage type in rsst_stage_inst.hip).
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
//     over nwx = ceil(nx/64) waves, so x needs no halo;
//   * 2D and 3D: x neighbours and x plus-face states go through LDS rows
//     with a ghost slot at each end (periodic wrap or mirror); every x flux
//     is formed once, by the cell right of the face, and reaches the cell on
//     its left by DPP within a wave and through one LDS seam value per wave
//     edge after a third barrier (rsst_stage2.h, rsst_stage3.h).  1D keeps
//     its row in one workgroup with DPP neighbours and LDS seams, the
//     wave-edge fluxes formed by both waves (rsst_stage1.h);
//   * 3D: each thread owns two adjacent y rows of its column, and a tile of
//     eight waves stacks 2R rows; the y face between a thread's rows is
//     formed in registers, the one between thread-rows once and handed over
//     in LDS, and the tile's two outer faces by each of the two tiles that
//     share them (the same face states and code, so the same bits), from the
//     rows just outside the tile, which the edge thread-rows read from
//     global memory a plane ahead;
//   * the last axis (z in 3D, y in 2D) is marched: each thread keeps its
//     column's planes in registers, so every z face is computed once and
//     carried to the next plane; large 2D grids march two planes per
//     iteration;
//   * every face state (U +- sigma/2, its pressure, c_tot and normal
//     velocity) is computed once, by the cell that owns it;
//   * workgroup ids are remapped so that consecutive tiles (which share
//     halo rows) run on the same XCD and share its L2.
#include <cstdlib>

#include "rsst_stage1.h"
#include "rsst_stage2.h"
#include "rsst_stage3.h"

#pragma clang fp contract(off)

namespace rsstk {

// ---------------------------------------------------------------- prime

// The largest c_tot of a state per stage-kernel workgroup slot (the grid has
// one workgroup per slot, each taking a strided share of the cells), from
// which the next stage 1 forms the CFL dt; with set_t, also t = t0.
template <int NDIM, typename ST>
__global__ void __launch_bounds__(256) prime_kernel(const StageArgs A, const ST* __restrict__ u,
                                                    double t0, int set_t) {
  constexpr int NV = NDIM + 2;
  const Consts K{A.gamma, A.gm1, A.inv_gm1, A.inv_xi, A.f, A.inv_cmax2, A.vdw_a, A.vdw_b};
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
    const double ct = A.eos ? cell_ctot<NDIM, kExtVdw>(q, K)
                      : (A.inv_cmax2 > 0.0 ? cell_ctot<NDIM, kExtCmax>(q, K) : cell_ctot<NDIM>(q, K));
    if (!(q[0] > 0.0)) bad |= kBadRho;
    if (!(ct < INFINITY)) bad |= kNonFinite;
    cm = fmax(cm, ct);
  }
  if (bad) atomicOr((unsigned*)(A.scal + kFlags), bad);
  const double wm = wave_max(cm);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = wm;
  __syncthreads();
  if (threadIdx.x == 0) {
    A.blkmax[blockIdx.x] = fmax(fmax(red[0], red[1]), fmax(red[2], red[3]));
    if (set_t && blockIdx.x == 0) A.scal[kTime] = t0;
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
  const Consts K{A.gamma, A.gm1, A.inv_gm1, A.inv_xi, A.f, A.inv_cmax2, A.vdw_a, A.vdw_b};
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
    double P, a2;
    if (A.eos) eos_pa2<kExtVdw>(q[0], rinv, q[NV - 1] - 0.5 * mv, K, P, a2);
    else eos_pa2<0>(q[0], rinv, q[NV - 1] - 0.5 * mv, K, P, a2);
    const double ae = A.inv_cmax2 > 0.0 ? a_eff_cmax(a2, K) : sqrt(a2) * A.inv_xi;  // a / xi
    acc[6] = fmax(acc[6], v);
    acc[7] = fmax(acc[7], v / ae);
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
  G.np = 1;
  G.nx = n[0];
  G.ns = (ndim == 3) ? n[1] : 1;
  G.nm = (ndim == 3) ? n[2] : (ndim == 2 ? n[1] : 1);
  G.nwx = (G.nx + 63) / 64;
  if (ndim == 3) {
    // 3D rows of 5-8 waves run as rows of 8 (the waves past the row's end
    // compute on clamped cells and store nothing)
    if (G.nwx > 4) G.nwx = 8;
    // an even number of rows (two per thread), at most the grid's (>= 4)
    G.ts = tile_rows3(G.nwx) < (G.ns & ~1) ? tile_rows3(G.nwx) : (G.ns & ~1);
  } else {
    G.ts = 1;
  }
  G.ntile_s = (G.ns + G.ts - 1) / G.ts;
  if (ndim == 1) {
    G.km = 1;
  } else {
    // chunks of 1 to 128 planes (3D; 2D: 64), halved while the grid has
    // fewer workgroups than the 256 CUs (3D: one workgroup fills a CU) or
    // than two per CU (2D rows of fewer waves).  A plane costs a workgroup
    // about a microsecond and a half however few cells it holds (a wave runs
    // ~1000 dependent instructions per plane), so a small grid is fastest as
    // many short marches, although each chunk re-reads 4 planes and forms one
    // extra face to start.  The environment variable RSST_KM, read when a
    // solver is made, sets the chunk length instead: the results do not
    // depend on it, which a GPU test checks for several lengths
    const long long want = ndim == 3 ? 256 : 512;
    int km = ndim == 3 ? 128 : 64;
    // 2D rows of up to eight waves march two planes per iteration (twice the
    // independent work per thread and half the barriers per plane) when
    // two-plane chunks still give every SIMD two waves (2048 waves); smaller
    // grids run one plane per iteration, in more and shorter marches
    // (measured: the 512^2 bubble 12.4 -> 13.0 Gcell-updates/s with two,
    // the 256^2 adjoint forward 4.3 -> 5.4 ms per 400 steps)
    G.np = (ndim == 2 && G.nwx <= 8 && (long long)((G.nm + 1) / 2) * G.nwx >= 2048) ? 2 : 1;
    const int kmin = G.np;  // a march iteration takes np planes: no shorter chunk
    while (km > kmin && (long long)G.ntile_s * ((G.nm + km - 1) / km) < want) km >>= 1;
    if (const char* e = getenv("RSST_KM")) {
      const int v = atoi(e);
      if (v >= 1 && v <= 4096) km = v;
    }
    G.km = km < G.nm ? km : G.nm;
  }
  G.nchunk = (G.nm + G.km - 1) / G.km;
  G.threads = 64 * G.nwx * (ndim == 3 ? G.ts / 2 : G.ts);
  G.lds_bytes = (size_t)(ndim == 3 ? carve3(G.ts, G.nwx).total
                                    : (ndim == 2 ? carve2(G.ts, G.nwx, G.np).total
                                                 : carve1(G.nwx).total)) *
                sizeof(double);
  return G;
}

template <typename ST>
static hipError_t launch_stage_p(const StageArgs& a, int stage, hipStream_t s) {
  switch (a.geo.ndim) {
    case 1: return launch_stage_n<1, ST, false>(a, stage, s);
    case 2: return launch_stage_n<2, ST, false>(a, stage, s);
    default: return a.big ? launch_stage_n<3, ST, true>(a, stage, s) : launch_stage_n<3, ST, false>(a, stage, s);
  }
}

hipError_t launch_stage(const StageArgs& a, int stage, hipStream_t s) {
  return a.prec ? launch_stage_p<float>(a, stage, s) : launch_stage_p<double>(a, stage, s);
}

template <typename ST>
static hipError_t launch_prime_p(const StageArgs& a, const void* u, double t0, int set_t,
                                 hipStream_t s) {
  const dim3 grid((unsigned)a.nblk), block(256);
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

// The next CFL step's dt, for reporting: one workgroup runs the grid maximum
// and the dt formula of stage 1 over the stored maxima.
__global__ void __launch_bounds__(256) next_dt_kernel(const StageArgs A) {
  __shared__ double red[4];
  const double m = grid_max_from_blocks(A, red);
  if (threadIdx.x == 0) A.scal[kDtNext] = m > 0.0 ? cfl_dt_of_max(A, m) : 0.0;
}

hipError_t launch_next_dt(const StageArgs& a, hipStream_t s) {
  hipLaunchKernelGGL(next_dt_kernel, dim3(1), dim3(256), 0, s, a);
  return hipGetLastError();
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
