// Discrete adjoint of one SSP-RK2 RSST step, FP64, for a fixed dt.
//
// With U1 = U + dt R(U) and U' = (U + U1 + dt R(U1)) / 2 (Sec. 4.1, the
// two-stage scheme), a cotangent lam' = dJ/dU' is pulled back by
//   (a, s1) = VJP(U1, lam'),      mu  = (lam' + dt a) / 2,
//   (b, s2) = VJP(U,  mu),        lam = lam'/2 + mu + dt b,
//   dJ/dxi += dt s1 / 2 + dt s2,
// where VJP(V, w) = (J_R(V)^T w, w . dR/dxi(V)) is the vector-Jacobian
// product of the semi-discrete operator R: MC-limited face states on the
// conservative variables, the LLF flux with c_tot = |V| + a/xi, the flux
// divergence, the RSST correction of the chosen form (eq. pvs_dt and
// App. A) and gravity (App. B).
//
// Derivatives are the branch-frozen ones of the primal values: the MC
// limiter is zero when l r <= 0, else it follows the first minimum among
// (|l+r|/2, 2|l|, 2|r|); the LLF speed is c_L when c_L >= c_R, else c_R;
// d|V| = 0 at |V| = 0.  A reflecting wall is the mirror image S of the
// cell state (normal momentum negated), so the wall face's outer state is
// S of the inner face state and its cotangent returns through S.
//
// On a 1D or 3D grid the VJP runs as the three passes below (a 2D grid
// takes the tiled form of the same passes, rsst_adjoint_tile.hip), each
// writing only its own cells, so the result is deterministic (no atomics):
//   A2 cell   fluxes G = 2 Fhat at the cell's two faces of every axis (a
//             face shared by two cells is formed by both, the same bits),
//             increments Delta, reverse of correction + gravity:
//             Delta_bar, the direct part of U_bar, the f part of xi_bar;
//   A3 face   G_bar from Delta_bar, reverse of the LLF flux into the plus
//             state of the left cell (Pb) and the minus state of the right
//             cell (Mb), the alpha part of xi_bar;
//   A4+A5 cell  U_bar += Pb + Mb, reverse of the MC half slope h = (Pb-Mb):
//             slope cotangents (lb, rb) of the cell, and the -lb of the cell
//             above and +rb of the cell below (formed here as those cells
//             form them); then mu (first VJP) or the new lam (second VJP).
#include <hip/hip_runtime.h>

#include <cstdint>

#include "rsst_adjoint.h"
#include "rsst_adjoint_ops.h"

#pragma clang fp contract(off)

namespace rsstk {

__device__ __forceinline__ void cell_coords(const AdjArgs& A, long long c, int x[3]) {
  x[0] = (int)(c % A.n[0]);
  const long long r = c / A.n[0];
  x[1] = (int)(r % A.n[1]);
  x[2] = (int)(r / A.n[1]);
}

// Neighbour of cell c (coordinates x) at offset o in [-2, 2] along d under
// the boundary rule; neg = the state there is the mirror image of the cell.
__device__ __forceinline__ long long neighbour(const AdjArgs& A, long long c, const int x[3], int d, int o,
                                               bool& neg) {
  const int n = A.n[d];
  int q = x[d] + o;
  neg = false;
  if (q < 0) {
    if (A.refl_lo[d]) { neg = true; q = -1 - q; }
    else q += n;
  } else if (q >= n) {
    if (A.refl_hi[d]) { neg = true; q = 2 * n - 1 - q; }
    else q -= n;
  }
  return c + (long long)(q - x[d]) * A.stride[d];
}

template <int NV>
__device__ __forceinline__ void load(const double* U, long long ncell, long long c, double (&u)[NV]) {
#pragma unroll
  for (int v = 0; v < NV; ++v) u[v] = U[v * ncell + c];
}

template <int NV>
__device__ __forceinline__ void load_nb(const AdjArgs& A, const double* U, long long c, const int x[3], int d,
                                        int o, double (&u)[NV]) {
  bool neg;
  const long long q = neighbour(A, c, x, d, o, neg);
  load<NV>(U, A.ncell, q, u);
  if (neg) u[1 + d] = -u[1 + d];
}

// ---------------------------------------------------------------- passes

template <int NDIM, int D>
__device__ __forceinline__ void face_pair(const AdjArgs& A, const Consts& K, long long c, const int x[3],
                                          Face<NDIM + 2>& L, Face<NDIM + 2>& R, bool& wall_hi) {
  constexpr int NV = NDIM + 2;
  double um[NV], u0[NV], up[NV], upp[NV], h0[NV];
  load_nb<NV>(A, A.V, c, x, D, -1, um);
  load<NV>(A.V, A.ncell, c, u0);
  load_nb<NV>(A, A.V, c, x, D, 1, up);
  half_slope<NDIM>(um, u0, up, h0);
  make_face<NDIM, D>(u0, h0, true, K, L);
  wall_hi = A.refl_hi[D] && x[D] == A.n[D] - 1;
  if (wall_hi) {
    R = mirror<NDIM, D>(L);
  } else {
    double h1[NV];
    load_nb<NV>(A, A.V, c, x, D, 2, upp);
    half_slope<NDIM>(u0, up, upp, h1);
    make_face<NDIM, D>(up, h1, false, K, R);
  }
}

// Minus face state of a cell at a low wall and its mirror (the outer state).
template <int NDIM, int D>
__device__ __forceinline__ void wall_lo_pair(const AdjArgs& A, const Consts& K, long long c, const int x[3],
                                             Face<NDIM + 2>& L, Face<NDIM + 2>& R) {
  constexpr int NV = NDIM + 2;
  double um[NV], u0[NV], up[NV], h0[NV];
  load_nb<NV>(A, A.V, c, x, D, -1, um);
  load<NV>(A.V, A.ncell, c, u0);
  load_nb<NV>(A, A.V, c, x, D, 1, up);
  half_slope<NDIM>(um, u0, up, h0);
  make_face<NDIM, D>(u0, h0, false, K, R);
  L = mirror<NDIM, D>(R);
}

__device__ __forceinline__ void block_partial(double v, double* out) {
  __shared__ double red[kAdjThreads / 64];
  const double w = wave_sum(v);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = w;
  __syncthreads();
  if (threadIdx.x == 0) {
    double s = 0.0;
    for (int q = 0; q < kAdjThreads / 64; ++q) s += red[q];
    out[blockIdx.x] = s;
  }
}

// G at the face below cell c along D (the face i-1/2): the wall pair, or
// the face above the neighbour below, formed as that cell forms it (so the
// two cells sharing a face get the same bits).
template <int NDIM, int D>
__device__ __forceinline__ void flux_below(const AdjArgs& A, const Consts& K, long long c, const int x[3],
                                           double (&G)[NDIM + 2]) {
  constexpr int NV = NDIM + 2;
  Face<NV> L, R;
  if (x[D] == 0 && A.refl_lo[D]) {
    wall_lo_pair<NDIM, D>(A, K, c, x, L, R);
  } else {
    bool neg, wall;
    const long long q = neighbour(A, c, x, D, -1, neg);
    int xq[3] = {x[0], x[1], x[2]};
    xq[D] = x[D] == 0 ? A.n[D] - 1 : x[D] - 1;
    face_pair<NDIM, D>(A, K, q, xq, L, R, wall);
  }
  flux2<NDIM, D>(L, R, G);
}

// The increments of cell c along D from the fluxes of its two faces, both
// formed here (no face pass before the cell pass).
template <int NDIM, int D>
__device__ __forceinline__ void a2_axis(const AdjArgs& A, const Consts& K, long long c, const int x[3],
                                        double (&Dl)[NDIM + 2]) {
  constexpr int NV = NDIM + 2;
  double Gl[NV], Gh[NV];
  flux_below<NDIM, D>(A, K, c, x, Gl);
  Face<NV> L, R;
  bool wall;
  face_pair<NDIM, D>(A, K, c, x, L, R, wall);
  flux2<NDIM, D>(L, R, Gh);
  const double hd = 0.5 * A.inv_dx[D];
#pragma unroll
  for (int v = 0; v < NV; ++v) Dl[v] -= (Gh[v] - Gl[v]) * hd;
}

template <int NDIM, int FORM>
__global__ void __launch_bounds__(kAdjThreads) adj_cell_kernel(AdjArgs A) {
  constexpr int NV = NDIM + 2;
  const long long c = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  double xib = 0.0;
  if (c < A.ncell) {
    int x[3];
    cell_coords(A, c, x);
    const Consts K = adj_consts<NDIM>(A);
    double Dl[NV], u[NV], Rb[NV], Db[NV], ub[NV];
#pragma unroll
    for (int v = 0; v < NV; ++v) {
      Dl[v] = 0.0;
      ub[v] = 0.0;
    }
    a2_axis<NDIM, 0>(A, K, c, x, Dl);
    if constexpr (NDIM >= 2) a2_axis<NDIM, 1>(A, K, c, x, Dl);
    if constexpr (NDIM >= 3) a2_axis<NDIM, 2>(A, K, c, x, Dl);
    load<NV>(A.V, A.ncell, c, u);
    load<NV>(A.W, A.ncell, c, Rb);
    const double fb = rate_vjp<NDIM, FORM>(u, Dl, Rb, A, Db, ub);
    xib = fb * A.dfdxi;
#pragma unroll
    for (int v = 0; v < NV; ++v) {
      A.Db[v * A.ncell + c] = Db[v];
      A.out[v * A.ncell + c] = ub[v];
    }
  }
  block_partial(xib, A.xpart);
}

template <int NDIM, int D>
__device__ __forceinline__ void a3_axis(const AdjArgs& A, const Consts& K, long long c, const int x[3],
                                        double& xib) {
  constexpr int NV = NDIM + 2;
  const double hd = 0.5 * A.inv_dx[D];
  double* Pb = A.Pb + (long long)D * NV * A.ncell;
  double* Mb = A.Mb + (long long)D * NV * A.ncell;
  double d0[NV];
  load<NV>(A.Db, A.ncell, c, d0);
  {
    // face i+1/2: dDelta_i/dG = -hd, dDelta_{i+1}/dG = +hd
    Face<NV> L, R;
    bool wall;
    face_pair<NDIM, D>(A, K, c, x, L, R, wall);
    double Gb[NV], Lb[NV], Rbar[NV];
    if (wall) {
#pragma unroll
      for (int v = 0; v < NV; ++v) Gb[v] = -hd * d0[v];
    } else {
      bool neg;
      const long long q = neighbour(A, c, x, D, 1, neg);
#pragma unroll
      for (int v = 0; v < NV; ++v) Gb[v] = hd * (A.Db[v * A.ncell + q] - d0[v]);
    }
    llf_vjp<NDIM, D>(L, R, Gb, A, Lb, Rbar, xib);
    if (wall) {
      mirror_add<NDIM, D>(Lb, Rbar);
    } else {
      bool neg;
      const long long q = neighbour(A, c, x, D, 1, neg);
#pragma unroll
      for (int v = 0; v < NV; ++v) Mb[v * A.ncell + q] = Rbar[v];
    }
#pragma unroll
    for (int v = 0; v < NV; ++v) Pb[v * A.ncell + c] = Lb[v];
  }
  if (x[D] == 0 && A.refl_lo[D]) {
    // wall face i-1/2: outer state S M_0, inner M_0; dDelta_0/dG = +hd
    Face<NV> L, R;
    wall_lo_pair<NDIM, D>(A, K, c, x, L, R);
    double Gb[NV], Lb[NV], Rbar[NV];
#pragma unroll
    for (int v = 0; v < NV; ++v) Gb[v] = hd * d0[v];
    llf_vjp<NDIM, D>(L, R, Gb, A, Lb, Rbar, xib);
    mirror_add<NDIM, D>(Rbar, Lb);
#pragma unroll
    for (int v = 0; v < NV; ++v) Mb[v * A.ncell + c] = Rbar[v];
  }
}

template <int NDIM>
__global__ void __launch_bounds__(kAdjThreads) adj_face_rev_kernel(AdjArgs A) {
  const long long c = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  double xib = 0.0;
  if (c < A.ncell) {
    int x[3];
    cell_coords(A, c, x);
    const Consts K = adj_consts<NDIM>(A);
    a3_axis<NDIM, 0>(A, K, c, x, xib);
    if constexpr (NDIM >= 2) a3_axis<NDIM, 1>(A, K, c, x, xib);
    if constexpr (NDIM >= 3) a3_axis<NDIM, 2>(A, K, c, x, xib);
  }
  block_partial(xib, A.xpart + A.nblock);
}

// The slope cotangents of cell c along D: lb = (dh/dl) hb, rb = (dh/dr) hb
// with hb = Pb - Mb (the cotangent of its half slope h).
template <int NDIM, int D>
__device__ __forceinline__ void slope_cot(const AdjArgs& A, long long c, const int x[3],
                                          double (&pb)[NDIM + 2], double (&mb)[NDIM + 2],
                                          double (&lb)[NDIM + 2], double (&rb)[NDIM + 2]) {
  constexpr int NV = NDIM + 2;
  const double* Pb = A.Pb + (long long)D * NV * A.ncell;
  const double* Mb = A.Mb + (long long)D * NV * A.ncell;
  double um[NV], u0[NV], up[NV];
  load_nb<NV>(A, A.V, c, x, D, -1, um);
  load<NV>(A.V, A.ncell, c, u0);
  load_nb<NV>(A, A.V, c, x, D, 1, up);
#pragma unroll
  for (int v = 0; v < NV; ++v) {
    pb[v] = Pb[v * A.ncell + c];
    mb[v] = Mb[v * A.ncell + c];
    const double hb = pb[v] - mb[v];
    double dl, dr;
    mc_half_partials(u0[v] - um[v], up[v] - u0[v], dl, dr);
    lb[v] = dl * hb;
    rb[v] = dr * hb;
  }
}

// A4: U_bar += Pb + Mb + lb - rb of the cell itself (a wall's ghost
// neighbour is S of this cell: its share comes back here).
template <int NDIM, int D>
__device__ __forceinline__ void a4_axis(const AdjArgs& A, long long c, const int x[3], double (&ub)[NDIM + 2]) {
  constexpr int NV = NDIM + 2;
  double pb[NV], mb[NV], lb[NV], rb[NV];
  slope_cot<NDIM, D>(A, c, x, pb, mb, lb, rb);
#pragma unroll
  for (int v = 0; v < NV; ++v) ub[v] += pb[v] + mb[v] + lb[v] - rb[v];
  if (x[D] == 0 && A.refl_lo[D]) {
#pragma unroll
    for (int v = 0; v < NV; ++v) ub[v] -= (v == 1 + D) ? -lb[v] : lb[v];
  }
  if (x[D] == A.n[D] - 1 && A.refl_hi[D]) {
#pragma unroll
    for (int v = 0; v < NV; ++v) ub[v] += (v == 1 + D) ? -rb[v] : rb[v];
  }
}

// A5: U_bar gathers -lb of the cell above (its l is U_above - U_this) and
// +rb of the cell below (its r is U_this - U_below), formed here as those
// cells form them.
template <int NDIM, int D>
__device__ __forceinline__ void a5_axis(const AdjArgs& A, long long c, const int x[3], double (&ub)[NDIM + 2]) {
  constexpr int NV = NDIM + 2;
  double pb[NV], mb[NV], lb[NV], rb[NV];
  bool neg;
  if (x[D] + 1 < A.n[D] || !A.refl_hi[D]) {
    const long long q = neighbour(A, c, x, D, 1, neg);
    int xq[3] = {x[0], x[1], x[2]};
    xq[D] = x[D] + 1 < A.n[D] ? x[D] + 1 : 0;
    slope_cot<NDIM, D>(A, q, xq, pb, mb, lb, rb);
#pragma unroll
    for (int v = 0; v < NV; ++v) ub[v] -= lb[v];
  }
  if (x[D] > 0 || !A.refl_lo[D]) {
    const long long q = neighbour(A, c, x, D, -1, neg);
    int xq[3] = {x[0], x[1], x[2]};
    xq[D] = x[D] > 0 ? x[D] - 1 : A.n[D] - 1;
    slope_cot<NDIM, D>(A, q, xq, pb, mb, lb, rb);
#pragma unroll
    for (int v = 0; v < NV; ++v) ub[v] += rb[v];
  }
}

// A4 and A5 of every axis for cell c (A4 of all axes first, then A5, the
// order of the two passes they replace), then mu or the new lam.
template <int NDIM>
__device__ __forceinline__ void gather_cell(const AdjArgs& A, long long c) {
  constexpr int NV = NDIM + 2;
  int x[3];
  cell_coords(A, c, x);
  double ub[NV];
  load<NV>(A.out, A.ncell, c, ub);
  a4_axis<NDIM, 0>(A, c, x, ub);
  if constexpr (NDIM >= 2) a4_axis<NDIM, 1>(A, c, x, ub);
  if constexpr (NDIM >= 3) a4_axis<NDIM, 2>(A, c, x, ub);
  a5_axis<NDIM, 0>(A, c, x, ub);
  if constexpr (NDIM >= 2) a5_axis<NDIM, 1>(A, c, x, ub);
  if constexpr (NDIM >= 3) a5_axis<NDIM, 2>(A, c, x, ub);
  if (A.post == 1) {
#pragma unroll
    for (int v = 0; v < NV; ++v) {
      const long long q = v * A.ncell + c;
      A.mu[q] = 0.5 * (A.lam[q] + A.dt * ub[v]);
    }
  } else if (A.post == 2) {
#pragma unroll
    for (int v = 0; v < NV; ++v) {
      const long long q = v * A.ncell + c;
      A.lam[q] = 0.5 * A.lam[q] + A.mu[q] + A.dt * ub[v];
    }
  } else {
#pragma unroll
    for (int v = 0; v < NV; ++v) A.out[v * A.ncell + c] = ub[v];
  }
}

// The last pass of a VJP; in the second VJP its workgroup 0 also folds the
// xi partials of both VJPs (complete: their passes ended before this one
// began) into dJdxi, after its own cells.
template <int NDIM>
__global__ void __launch_bounds__(kAdjThreads) adj_gather_kernel(AdjArgs A) {
  const long long c = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (c < A.ncell) gather_cell<NDIM>(A, c);
  if (A.post == 2 && blockIdx.x == 0) xi_reduce<kAdjThreads>(A.xp1, A.xp2, A.xm, A.dt, A.dJdxi);
}

template <int NDIM>
static void* cell_kernel_ptr(int form) {
  switch (form) {
    case kEuler: return (void*)adj_cell_kernel<NDIM, kEuler>;
    case kPVS: return (void*)adj_cell_kernel<NDIM, kPVS>;
    case kPMS: return (void*)adj_cell_kernel<NDIM, kPMS>;
    case kDVS: return (void*)adj_cell_kernel<NDIM, kDVS>;
    case kDMS: return (void*)adj_cell_kernel<NDIM, kDMS>;
    default: return (void*)adj_cell_kernel<NDIM, kPD>;
  }
}

template <int NDIM>
static hipError_t vjp_launch(AdjArgs A, int form, hipStream_t s) {
  const dim3 grid(A.nblock), block(kAdjThreads);
  void* args[] = {(void*)&A};
  hipError_t e = hipLaunchKernel(cell_kernel_ptr<NDIM>(form), grid, block, args, 0, s);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(adj_face_rev_kernel<NDIM>, grid, block, 0, s, A);
  hipLaunchKernelGGL(adj_gather_kernel<NDIM>, grid, block, 0, s, A);
  return hipGetLastError();
}

size_t adjoint_workspace_doubles(int ndim, const int n[3], long long ncell) {
  const int nv = ndim + 2;
  if (ndim == 2) {
    // mu; two partial arrays and the run accumulator, one value per tile
    return (size_t)nv * ncell + 3 * (size_t)tile2_nblock(n);
  }
  const long long nblock = (ncell + kAdjThreads - 1) / kAdjThreads;
  // Pb, Mb: ndim fields each; Db, a/b, mu: one each; 4 partial arrays
  return (size_t)nv * ncell * (2 * ndim + 3) + 4 * (size_t)nblock;
}

size_t adjoint_zeroed_offset(int ndim, const int n[3], long long ncell) {
  return ndim == 2 ? (size_t)(ndim + 2) * ncell + 2 * (size_t)tile2_nblock(n) : adjoint_workspace_doubles(ndim, n, ncell);
}

hipError_t launch_adjoint_xi_fold(const AdjointPlan& p, double* dJdxi, hipStream_t s) {
  if (p.ndim != 2) return hipSuccess;
  const int nt = tile2_nblock(p.n);
  return launch_xi_acc_fold(p.work + adjoint_zeroed_offset(2, p.n, p.ncell), nt, dJdxi, s);
}

hipError_t launch_adjoint_step(const AdjointPlan& p, const double* U, const double* U1, double* lam, double dt,
                               double* dJdxi, bool defer, hipStream_t s) {
  const int ndim = p.ndim, nv = ndim + 2;
  const long long n = p.ncell, nf = (long long)nv * n;
  const int nblock = (int)((n + kAdjThreads - 1) / kAdjThreads);
  double* w = p.work;
  AdjArgs A{};
  A.ndim = ndim;
  A.nv = nv;
  for (int d = 0; d < 3; ++d) {
    A.n[d] = p.n[d];
    A.refl_lo[d] = p.refl_lo[d];
    A.refl_hi[d] = p.refl_hi[d];
    A.inv_dx[d] = p.inv_dx[d];
    A.g[d] = p.g[d];
  }
  A.stride[0] = 1;
  A.stride[1] = p.n[0];
  A.stride[2] = (long long)p.n[0] * p.n[1];
  A.ncell = n;
  A.gamma = p.gamma;
  A.gm1 = p.gamma - 1.0;
  A.inv_gm1 = 1.0 / (p.gamma - 1.0);
  A.inv_xi = 1.0 / p.xi;
  A.f = 1.0 - 1.0 / (p.xi * p.xi);
  A.dfdxi = 2.0 / (p.xi * p.xi * p.xi);
  A.lam = lam;
  A.dt = dt;
  A.dJdxi = dJdxi;
  if (ndim == 2) {
    // one tiled launch per VJP; each leaves one partial sum of xi_bar per
    // tile, and a one-workgroup launch after the second folds both sets
    const int nt = tile2_nblock(p.n);
    double* const part1 = w + nf;
    double* const part2 = part1 + nt;
    A.mu = w;
    A.nblock = nt;
    A.xp1 = part1;
    A.xp2 = part2;
    A.xacc = defer ? part2 + nt : nullptr;
    A.V = U1;
    A.W = lam;
    A.xpart = part1;
    A.post = 1;
    hipError_t e = launch_vjp_tile2(A, p.form, s);
    if (e != hipSuccess) return e;
    A.V = U;
    A.W = A.mu;
    A.xpart = part2;
    A.post = 2;
    e = launch_vjp_tile2(A, p.form, s);
    if (e != hipSuccess) return e;
    return hipGetLastError();
  }
  A.Pb = w;
  A.Mb = A.Pb + ndim * nf;
  A.Db = A.Mb + ndim * nf;
  double* ab = A.Db + nf;
  double* mu = ab + nf;
  double* part1 = mu + nf;
  double* part2 = part1 + 2 * nblock;
  A.nblock = nblock;
  A.mu = mu;
  // each VJP leaves partials of the f part then the alpha part (2 nblock
  // each); the second VJP's last pass folds both sets into dJdxi
  A.xp1 = part1;
  A.xp2 = part2;
  A.xm = 2 * nblock;
  auto vjp = [&](const double* V, const double* Wc, double* out, double* part, int post) {
    A.V = V;
    A.W = Wc;
    A.out = out;
    A.xpart = part;
    A.post = post;
    return ndim == 1 ? vjp_launch<1>(A, p.form, s) : vjp_launch<3>(A, p.form, s);
  };
  // (a, s1) = VJP(U1, lam) with mu = (lam + dt a)/2 formed by its last pass
  hipError_t e = vjp(U1, lam, ab, part1, 1);
  if (e != hipSuccess) return e;
  // (b, s2) = VJP(U, mu) with lam = lam/2 + mu + dt b formed by its last pass
  e = vjp(U, mu, ab, part2, 2);
  if (e != hipSuccess) return e;
  return hipGetLastError();
}

}  // namespace rsstk
