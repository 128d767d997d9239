// The vector-Jacobian product of R on a 2D grid as one launch per VJP.
//
// Same product, same arithmetic per cell and per face as the three per-cell
// passes of rsst_adjoint.hip (the cotangent of U comes out with the same
// bits), but each workgroup owns a TX x TY tile of output cells and forms
// everything it needs in LDS, so a VJP is one launch with no full-field
// scratch in HBM:
//   load    U over the tile and four cells around it into LDS (boundary
//           rules applied: periodic wrap, or the mirror image with the
//           normal momentum negated); each thread's own W (and, second VJP,
//           lam) into registers;
//   fluxes  G = 2 Fhat at every face of the cells within two of the tile,
//           keeping the states of the faces the reverse needs;
//   cells   for those cells, the increments Delta, then the reverse of the
//           correction and gravity: Delta_bar (zero outside a wall), and for
//           the tile's own cells the direct part of U_bar and the f part of
//           xi_bar;
//   faces   G_bar = (Delta_bar_right - Delta_bar_left)/(2 dx) at the faces
//           whose states reach a tile cell, the reverse of the LLF flux into
//           the plus state of the left cell and the minus state of the right
//           one (at a wall both return to the inner cell through the mirror),
//           and the alpha part of xi_bar at the faces the tile owns;
//   gather  U_bar of each tile cell: its face-state cotangents, the reverse
//           of its MC half slopes and those of its neighbours on both axes;
//           then mu (first VJP) or the new lam (second VJP).
// 16 x 16 tiles, 1024 threads (four waves per SIMD), 124 KiB of LDS: one
// workgroup per CU.  A face shared by two tiles is formed by both (the same
// bits); the partial sums of xi_bar count each cell and each face once, in
// the tile that owns it (a face i+1/2 belongs to cell i, a low wall face to
// cell 0).  After the second VJP a one-workgroup launch folds both VJPs'
// partial sums into dJ/dxi in a fixed order, or, over a run of steps, the
// second VJP adds its tile's share into a per-tile accumulator folded once
// at the end (no atomics, no cross-workgroup waits).
#include <hip/hip_runtime.h>

#include "rsst_adjoint.h"
#include "rsst_adjoint_ops.h"

#pragma clang fp contract(off)

namespace rsstk {

namespace {

constexpr int kTX = 16, kTY = 16, kTileThreads = 1024;

// Cell index along one axis for a position q of the extended grid, and
// whether the state there is the mirror image (normal momentum negated).
// Positions a workgroup never uses (far outside a wall in a ragged tile) are
// clamped into the grid so every load stays in bounds.
__device__ __forceinline__ int map_pos(int q, int n, int rlo, int rhi, bool& neg) {
  neg = false;
  if (q < 0) {
    if (rlo) {
      neg = true;
      q = -1 - q;
    } else {
      q = q % n + n;
      if (q == n) q = 0;
    }
  } else if (q >= n) {
    if (rhi) {
      neg = true;
      q = 2 * n - 1 - q;
    } else {
      q = q % n;
    }
  }
  return q < 0 ? 0 : (q >= n ? n - 1 : q);
}

// Is position q a cell of the grid (periodic positions all are)?
__device__ __forceinline__ bool real_pos(int q, int n, int rlo, int rhi) {
  return (q >= 0 || !rlo) && (q < n || !rhi);
}

// The left and right states of the face between positions i and i+1 along
// D from the four cells a, b, c, d at i-1 .. i+2 (ghosts already mirrored):
// the plus state of b and the minus state of c, or at a wall the inner
// state and its mirror image.  Selected per value rather than by branch (the
// primitives of a mirror image are those of the state with vn negated, the
// same bits either way).
template <int D>
__device__ __forceinline__ void face_lr(const double (&a)[4], const double (&b)[4], const double (&c)[4],
                                        const double (&d)[4], bool wall_lo, bool wall_hi, const Consts& K,
                                        Face<4>& L, Face<4>& R) {
  double hb[4], hc[4];
  half_slope<2>(a, b, c, hb);
  half_slope<2>(b, c, d, hc);
#pragma unroll
  for (int v = 0; v < 4; ++v) {
    L.u[v] = b[v] + hb[v];
    R.u[v] = c[v] - hc[v];
  }
#pragma unroll
  for (int v = 0; v < 4; ++v) {
    const double m = (v == 1 + D) ? -R.u[v] : R.u[v];
    L.u[v] = wall_lo ? m : L.u[v];
  }
#pragma unroll
  for (int v = 0; v < 4; ++v) {
    const double m = (v == 1 + D) ? -L.u[v] : L.u[v];
    R.u[v] = wall_hi ? m : R.u[v];
  }
  face_prims<2, D>(L, K);
  face_prims<2, D>(R, K);
}

// A face's two states in the cache: u of L and R, then c of L and R, each
// quantity a plane of `stride` faces.
__device__ __forceinline__ void put_face(double* F, int f, int stride, const Face<4>& L, const Face<4>& R) {
#pragma unroll
  for (int v = 0; v < 4; ++v) {
    F[v * stride + f] = L.u[v];
    F[(4 + v) * stride + f] = R.u[v];
  }
  F[8 * stride + f] = L.c;
  F[9 * stride + f] = R.c;
}

// The states as the reverse of the LLF flux reads them (u and c).
__device__ __forceinline__ void get_face(const double* F, int f, int stride, Face<4>& L, Face<4>& R) {
#pragma unroll
  for (int v = 0; v < 4; ++v) {
    L.u[v] = F[v * stride + f];
    R.u[v] = F[(4 + v) * stride + f];
  }
  L.c = F[8 * stride + f];
  R.c = F[9 * stride + f];
}

// dJ/dxi += dt/2 (sum of the first VJP's tile partials) + dt (sum of the
// second's), in a fixed order.
__global__ void __launch_bounds__(kAdjThreads) adj_xi_fold_kernel(const double* p1, const double* p2, int m,
                                                                 double dt, double* dJdxi) {
  xi_reduce<kAdjThreads>(p1, p2, m, dt, dJdxi);
}

// dJ/dxi += sum of a run's per-tile accumulators, in a fixed order; the
// accumulators are left at zero for the next run.
__global__ void __launch_bounds__(kAdjThreads) adj_acc_fold_kernel(double* acc, int m, double* dJdxi) {
  __shared__ double red[kAdjThreads / 64];
  double s = 0.0;
  for (int q = threadIdx.x; q < m; q += kAdjThreads) s += acc[q];
  s = wave_sum(s);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = s;
  __syncthreads();
  for (int q = threadIdx.x; q < m; q += kAdjThreads) acc[q] = 0.0;
  if (threadIdx.x == 0) {
    double t = 0.0;
    for (int q = 0; q < kAdjThreads / 64; ++q) t += red[q];
    *dJdxi += t;
  }
}

template <int TX, int TY>
struct Tile2 {
  // U window: positions (x0-4 .. x0+TX+3, y0-4 .. y0+TY+3), [v][py][px]
  static constexpr int UX = TX + 8, UY = TY + 8;
  // window of the cell phase: positions (x0-2 .. x0+TX+1, y0-2 .. y0+TY+1),
  // [v][ry][rx]: W there, then Delta_bar
  static constexpr int DX = TX + 4, DY = TY + 4;
  // forward fluxes: x faces i = x0-3 .. x0+TX+1 on the rows of that window,
  // [v][ry][k]; y faces j = y0-3 .. y0+TY+1 on its columns, [v][k][rx]
  static constexpr int GXN = TX + 5, GYN = TY + 5;
  // face-state cotangents: x faces i = x0-2 .. x0+TX on the tile's rows,
  // [v][oy][k]; y faces j = y0-2 .. y0+TY on its columns, [v][k][ox]
  static constexpr int LXN = TX + 3, LYN = TY + 3;
  static constexpr int NC = TX * TY;  // tile cells
  static constexpr int NU = 4 * UX * UY;
  static constexpr int ND = 4 * DX * DY;
  static constexpr int NG = 4 * (DY * GXN + GYN * DX);
  static constexpr int NL = 2 * 4 * (TY * LXN + LYN * TX);
  // the states of the faces of the reverse phase, formed in the flux phase:
  // L.u, R.u, L.c, R.c, [q][oy][k] and [q][k][ox] like the cotangents
  static constexpr int NF = 10 * (TY * LXN + LYN * TX);
  // U, Delta_bar, fluxes then face cotangents, face states, direct U_bar of
  // the tile's cells
  static constexpr int NLDS = NU + ND + (NG > NL ? NG : NL) + NF + 4 * NC;
};

template <int FORM, int TX, int TY, int NT>
__global__ void __launch_bounds__(NT) adj_tile2_kernel(AdjArgs A) {
  using T = Tile2<TX, TY>;
  constexpr int UX = T::UX, UY = T::UY, DX = T::DX, DY = T::DY;
  constexpr int GXN = T::GXN, GYN = T::GYN, LXN = T::LXN, LYN = T::LYN, NC = T::NC;
  __shared__ double lds[T::NLDS];
  double* const Us = lds;
  double* const Ds = Us + T::NU;
  double* const Gx = Ds + T::ND;
  double* const Gy = Gx + 4 * DY * GXN;
  double* const Lx = Ds + T::ND;  // after the cell phase, over the fluxes
  double* const Rx = Lx + 4 * TY * LXN;
  double* const Ly = Rx + 4 * TY * LXN;
  double* const Ry = Ly + 4 * LYN * TX;
  double* const FX = Ds + T::ND + (T::NG > T::NL ? T::NG : T::NL);  // face states, x
  double* const FY = FX + 10 * TY * LXN;                             // face states, y
  double* const Bs = FY + 10 * LYN * TX;                             // direct U_bar, [v][cell]
  __shared__ double red[NT / 64];

  const int tid = threadIdx.x;
  // tile of this workgroup: dispatch goes round-robin over the 8 XCDs, so
  // consecutive workgroups take tiles nblock/8 apart and each XCD a
  // contiguous run of tile rows, whose shared halos meet in its own L2
  const int gxt = (A.n[0] + TX - 1) / TX;
  const int tile = ((A.nblock & 7) == 0) ? (blockIdx.x & 7) * (A.nblock >> 3) + (blockIdx.x >> 3) : blockIdx.x;
  const int x0 = (tile % gxt) * TX, y0 = (tile / gxt) * TY;
  const int nx = A.n[0], ny = A.n[1];
  const int rxl = A.refl_lo[0], rxh = A.refl_hi[0], ryl = A.refl_lo[1], ryh = A.refl_hi[1];
  const Consts K = adj_consts<2>(A);
  auto U = [&](int v, int px, int py) -> double { return Us[(v * UY + py) * UX + px]; };
  auto Uc = [&](int px, int py, double (&u)[4]) {
#pragma unroll
    for (int v = 0; v < 4; ++v) u[v] = U(v, px, py);
  };
  auto cell_at = [&](int x, int y, bool& negx, bool& negy) -> long long {
    const int cx = map_pos(x, nx, rxl, rxh, negx);
    const int cy = map_pos(y, ny, ryl, ryh, negy);
    return (long long)cy * nx + cx;
  };

  // ---- load U over its window into LDS; W of this thread's cell-phase
  // item and, for its gather value (cell, v), W and the second VJP's lam
  // wait in registers (all loads in flight together, only U's awaited here)
  static_assert(NT == 4 * NC, "one gather value (cell, v) per thread");
  static_assert(NT >= NC + 4 * (TX + TY), "one cell-phase item per thread");
  const int ge = tid % NC, gv = tid / NC;
  const int gx = x0 + ge % TX, gy = y0 + ge / TX;
  const bool gin = gx < nx && gy < ny;
  const long long gq = gv * A.ncell + (long long)gy * nx + gx;
  // the cell-phase item of this thread: the tile's own cells first, then
  // the two rows and columns around it (corners excluded)
  int crx = 0, cry = 0;
  const bool citem = tid < NC + 4 * (TX + TY);
  if (tid < NC) {
    crx = tid % TX + 2;
    cry = tid / TX + 2;
  } else if (tid < NC + 4 * TX) {
    const int h = tid - NC, band = h / TX;
    crx = h % TX + 2;
    cry = band < 2 ? band : TY + band;
  } else if (citem) {
    const int h = tid - NC - 4 * TX, band = h / TY;
    cry = h % TY + 2;
    crx = band < 2 ? band : TX + band;
  }
  const int cxp = x0 - 2 + crx, cyp = y0 - 2 + cry;
  const bool creal = citem && real_pos(cxp, nx, rxl, rxh) && real_pos(cyp, ny, ryl, ryh);
  for (int t = tid; t < UX * UY; t += NT) {
    if (t < UX * UY) {
      const int px = t % UX, py = t / UX;
      bool negx, negy;
      const long long c = cell_at(x0 - 4 + px, y0 - 4 + py, negx, negy);
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        double val = A.V[v * A.ncell + c];
        if ((v == 1 && negx) || (v == 2 && negy)) val = -val;
        Us[(v * UY + py) * UX + px] = val;
      }
    }
  }
  double Rb[4] = {0.0, 0.0, 0.0, 0.0};
  if (creal) {
    bool negx, negy;
    const long long c = cell_at(cxp, cyp, negx, negy);
#pragma unroll
    for (int v = 0; v < 4; ++v) Rb[v] = A.W[v * A.ncell + c];
  }
  const double w_own = gin ? A.W[gq] : 0.0;
  const double lam_own = (A.post == 2 && gin) ? A.lam[gq] : 0.0;
  __syncthreads();

  // ---- forward fluxes
  for (int t = tid; t < DY * GXN + GYN * DX; t += NT) {
    double a[4], b[4], c[4], d[4], G[4];
    Face<4> L, R;
    if (t < DY * GXN) {
      const int ry = t / GXN, k = t % GXN;  // face i = x0-3+k, row y0-2+ry
      const int i = x0 - 3 + k, py = ry + 2;
      Uc(k, py, a);
      Uc(k + 1, py, b);
      Uc(k + 2, py, c);
      Uc(k + 3, py, d);
      face_lr<0>(a, b, c, d, rxl && i == -1, rxh && i == nx - 1, K, L, R);
      flux2<2, 0>(L, R, G);
#pragma unroll
      for (int v = 0; v < 4; ++v) Gx[(v * DY + ry) * GXN + k] = G[v];
      if (ry >= 2 && ry < TY + 2 && k >= 1 && k <= LXN) put_face(FX, (ry - 2) * LXN + k - 1, TY * LXN, L, R);
    } else {
      const int s = t - DY * GXN;
      const int rx = s % DX, k = s / DX;  // face j = y0-3+k, column x0-2+rx
      const int j = y0 - 3 + k, px = rx + 2;
      Uc(px, k, a);
      Uc(px, k + 1, b);
      Uc(px, k + 2, c);
      Uc(px, k + 3, d);
      face_lr<1>(a, b, c, d, ryl && j == -1, ryh && j == ny - 1, K, L, R);
      flux2<2, 1>(L, R, G);
#pragma unroll
      for (int v = 0; v < 4; ++v) Gy[(v * GYN + k) * DX + rx] = G[v];
      if (rx >= 2 && rx < TX + 2 && k >= 1 && k <= LYN) put_face(FY, (k - 1) * TX + rx - 2, LYN * TX, L, R);
    }
  }
  __syncthreads();

  // ---- cells: Delta_bar over the tile and the two cells around it; the
  // tile's own cells keep their direct U_bar and the f part of xi_bar
  double xib = 0.0;
  const double hdx = 0.5 * A.inv_dx[0], hdy = 0.5 * A.inv_dx[1];
  if (citem) {
    const int t = tid, rx = crx, ry = cry;
    const int x = cxp, y = cyp;
    double Db[4] = {0.0, 0.0, 0.0, 0.0};
    if (creal) {
      double Dl[4] = {0.0, 0.0, 0.0, 0.0}, u[4], ub[4] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const double gl = Gx[(v * DY + ry) * GXN + rx], gh = Gx[(v * DY + ry) * GXN + rx + 1];
        Dl[v] -= (gh - gl) * hdx;
      }
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const double gl = Gy[(v * GYN + ry) * DX + rx], gh = Gy[(v * GYN + ry + 1) * DX + rx];
        Dl[v] -= (gh - gl) * hdy;
      }
      Uc(rx + 2, ry + 2, u);
      const double fb = rate_vjp<2, FORM>(u, Dl, Rb, A, Db, ub);
      if (t < NC) {
#pragma unroll
        for (int v = 0; v < 4; ++v) Bs[v * NC + t] = ub[v];
        if (x < nx && y < ny) xib = fb * A.dfdxi;
      }
    }
#pragma unroll
    for (int v = 0; v < 4; ++v) Ds[(v * DY + ry) * DX + rx] = Db[v];
  }
  __syncthreads();

  // ---- faces: reverse of the LLF flux at every face whose states reach a
  // tile cell
  for (int t = tid; t < TY * LXN + LYN * TX; t += NT) {
    double Gb[4], Lb[4], Rbar[4];
    Face<4> L, R;
    double xf = 0.0;
    if (t < TY * LXN) {
      const int oy = t / LXN, k = t % LXN;  // face i = x0-2+k, row y0+oy
      const int i = x0 - 2 + k, ry = oy + 2;
      const bool wlo = rxl && i == -1, whi = rxh && i == nx - 1;
      get_face(FX, t, TY * LXN, L, R);
#pragma unroll
      for (int v = 0; v < 4; ++v)
        Gb[v] = hdx * (Ds[(v * DY + ry) * DX + k + 1] - Ds[(v * DY + ry) * DX + k]);
      llf_vjp<2, 0>(L, R, Gb, A, Lb, Rbar, xf);
      if (whi) mirror_add<2, 0>(Lb, Rbar);
      if (wlo) mirror_add<2, 0>(Rbar, Lb);
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        Lx[(v * TY + oy) * LXN + k] = Lb[v];
        Rx[(v * TY + oy) * LXN + k] = Rbar[v];
      }
      const bool own = y0 + oy < ny && ((i >= x0 && i < x0 + TX && i < nx) || wlo);
      if (own) xib += xf;
    } else {
      const int s = t - TY * LXN;
      const int ox = s % TX, k = s / TX;  // face j = y0-2+k, column x0+ox
      const int j = y0 - 2 + k, rx = ox + 2;
      const bool wlo = ryl && j == -1, whi = ryh && j == ny - 1;
      get_face(FY, s, LYN * TX, L, R);
#pragma unroll
      for (int v = 0; v < 4; ++v)
        Gb[v] = hdy * (Ds[(v * DY + k + 1) * DX + rx] - Ds[(v * DY + k) * DX + rx]);
      llf_vjp<2, 1>(L, R, Gb, A, Lb, Rbar, xf);
      if (whi) mirror_add<2, 1>(Lb, Rbar);
      if (wlo) mirror_add<2, 1>(Rbar, Lb);
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        Ly[(v * LYN + k) * TX + ox] = Lb[v];
        Ry[(v * LYN + k) * TX + ox] = Rbar[v];
      }
      const bool own = x0 + ox < nx && ((j >= y0 && j < y0 + TY && j < ny) || wlo);
      if (own) xib += xf;
    }
  }
  // the tile's partial sum of xi_bar is complete
  {
    const double w = wave_sum(xib);
    if ((tid & 63) == 0) red[tid >> 6] = w;
  }
  __syncthreads();
  if (tid == 0) {
    double sum = 0.0;
    for (int q = 0; q < NT / 64; ++q) sum += red[q];
    const int b = tile;
    if (A.xacc && A.post == 2) A.xacc[b] += 0.5 * A.dt * A.xp1[b] + A.dt * sum;
    else A.xpart[b] = sum;
  }

  // ---- gather: one value (cell, v) per thread: U_bar from the cell's face
  // cotangents, the reverse of its MC half slopes and those of its
  // neighbours on both axes; then mu or the new lam
  if (gin) {
    const int e = ge, v = gv;
    const int ox = e % TX, oy = e / TX;
    const int x = gx, y = gy;
    const int px = ox + 4, py = oy + 4;
    double ub = Bs[v * NC + e];
    const double* const lx = Lx + (v * TY + oy) * LXN;
    const double* const rxr = Rx + (v * TY + oy) * LXN;
    const double* const ly = Ly + v * LYN * TX + ox;
    const double* const ryr = Ry + v * LYN * TX + ox;
    const double* const urow = Us + (v * UY + py) * UX;
    const double* const ucol = Us + v * UY * UX + px;
    // slope cotangents of the cell at (um, u0, up) with face cotangents (pb, mb)
    auto cot = [](double um, double u0, double up, double pb, double mb, double& lb, double& rb) {
      const double hb = pb - mb;
      double dl, dr;
      mc_half_partials(u0 - um, up - u0, dl, dr);
      lb = dl * hb;
      rb = dr * hb;
    };
    double lb, rb;
    // own slopes, x then y (the cell's plus state is face x, its minus state
    // face x-1)
    {
      const double pb = lx[ox + 2], mb = rxr[ox + 1];
      cot(urow[px - 1], urow[px], urow[px + 1], pb, mb, lb, rb);
      ub += pb + mb + lb - rb;
      if (x == 0 && rxl) ub -= (v == 1) ? -lb : lb;
      if (x == nx - 1 && rxh) ub += (v == 1) ? -rb : rb;
    }
    {
      const double pb = ly[(oy + 2) * TX], mb = ryr[(oy + 1) * TX];
      cot(ucol[(py - 1) * UX], ucol[py * UX], ucol[(py + 1) * UX], pb, mb, lb, rb);
      ub += pb + mb + lb - rb;
      if (y == 0 && ryl) ub -= (v == 2) ? -lb : lb;
      if (y == ny - 1 && ryh) ub += (v == 2) ? -rb : rb;
    }
    // neighbours' slopes: -lb of the cell above, +rb of the cell below
    if (x + 1 < nx || !rxh) {
      cot(urow[px], urow[px + 1], urow[px + 2], lx[ox + 3], rxr[ox + 2], lb, rb);
      ub -= lb;
    }
    if (x > 0 || !rxl) {
      cot(urow[px - 2], urow[px - 1], urow[px], lx[ox + 1], rxr[ox], lb, rb);
      ub += rb;
    }
    if (y + 1 < ny || !ryh) {
      cot(ucol[py * UX], ucol[(py + 1) * UX], ucol[(py + 2) * UX], ly[(oy + 3) * TX], ryr[(oy + 2) * TX], lb,
          rb);
      ub -= lb;
    }
    if (y > 0 || !ryl) {
      cot(ucol[(py - 2) * UX], ucol[(py - 1) * UX], ucol[py * UX], ly[(oy + 1) * TX], ryr[oy * TX], lb, rb);
      ub += rb;
    }
    const double w = w_own;  // W of this value
    if (A.post == 1) A.mu[gq] = 0.5 * (w + A.dt * ub);       // W = lam
    else if (A.post == 2) A.lam[gq] = 0.5 * lam_own + w + A.dt * ub;  // W = mu
    else A.out[gq] = ub;
  }

}

template <int TX, int TY, int NT>
void* tile2_kernel_ptr(int form) {
  switch (form) {
    case kEuler: return (void*)adj_tile2_kernel<kEuler, TX, TY, NT>;
    case kPVS: return (void*)adj_tile2_kernel<kPVS, TX, TY, NT>;
    case kPMS: return (void*)adj_tile2_kernel<kPMS, TX, TY, NT>;
    case kDVS: return (void*)adj_tile2_kernel<kDVS, TX, TY, NT>;
    case kDMS: return (void*)adj_tile2_kernel<kDMS, TX, TY, NT>;
    default: return (void*)adj_tile2_kernel<kPD, TX, TY, NT>;
  }
}

}  // namespace

int tile2_nblock(const int n[3]) { return ((n[0] + kTX - 1) / kTX) * ((n[1] + kTY - 1) / kTY); }

hipError_t launch_vjp_tile2(const AdjArgs& A, int form, hipStream_t s) {
  const dim3 grid(tile2_nblock(A.n)), block(kTileThreads);
  AdjArgs a = A;
  void* args[] = {(void*)&a};
  hipError_t e = hipLaunchKernel(tile2_kernel_ptr<kTX, kTY, kTileThreads>(form), grid, block, args, 0, s);
  if (e != hipSuccess || A.post != 2 || A.xacc) return e;
  hipLaunchKernelGGL(adj_xi_fold_kernel, dim3(1), dim3(kAdjThreads), 0, s, A.xp1, A.xp2, A.nblock, A.dt, A.dJdxi);
  return hipGetLastError();
}

hipError_t launch_xi_acc_fold(double* acc, int m, double* dJdxi, hipStream_t s) {
  hipLaunchKernelGGL(adj_acc_fold_kernel, dim3(1), dim3(kAdjThreads), 0, s, acc, m, dJdxi);
  return hipGetLastError();
}

}  // namespace rsstk
