// Reverse-mode building blocks of the RSST adjoint (FP64): the arguments of
// the vector-Jacobian-product kernels and the pull-backs of the LLF flux,
// the primitives and the corrected rate, shared by the per-cell passes
// (rsst_adjoint.hip) and the tiled 2D VJP (rsst_adjoint_tile.hip).
#pragma once

#include <hip/hip_runtime.h>

#include "rsst_device.h"

#pragma clang fp contract(off)

namespace rsstk {

constexpr int kAdjThreads = 256;

struct AdjArgs {
  int ndim, nv;
  int n[3];
  int refl_lo[3], refl_hi[3];
  long long ncell;
  long long stride[3];  // cells between neighbours along each axis
  double inv_dx[3];
  double gamma, gm1, inv_gm1, inv_xi, f, dfdxi;
  double g[3];
  const double* V;   // primal state [nv][ncell]
  const double* W;   // cotangent of R [nv][ncell]
  double* out;       // J_R^T W [nv][ncell]
  double* Db;        // [nv][ncell]
  double* Pb;        // [ndim][nv][ncell]
  double* Mb;        // [ndim][nv][ncell]
  double* xpart;     // [2][nblock] partial sums of xi_bar
  int nblock;
  // what the last pass does with its result r = J_R^T W (per element):
  // 0: out = r; 1: mu = (lam + dt r)/2; 2: lam = lam/2 + mu + dt r
  int post;
  double* lam;
  double* mu;
  double dt;
  // the second VJP's last pass also folds the xi partials of both VJPs into
  // dJdxi (its workgroup 0, after its own cells)
  const double* xp1;
  const double* xp2;
  int xm;
  double* dJdxi;
  // tiled 2D VJP, second VJP: when set, each tile adds its share of dJ/dxi
  // (dt/2 its first-VJP partial + dt its own) into xacc[tile] instead of a
  // fold into dJdxi (the caller folds the accumulator once, later)
  double* xacc;
};

// ---------------------------------------------------------------- reverse

// dh/dl, dh/dr of the MC half slope h = MC(l, r)/2 with the tie rule above.
__device__ __forceinline__ void mc_half_partials(double l, double r, double& dl, double& dr) {
  dl = 0.0;
  dr = 0.0;
  if (l * r <= 0.0) return;
  const double q1 = fabs(l + r) * 0.5, q2 = 2.0 * fabs(l), q3 = 2.0 * fabs(r);
  if (q1 <= q2 && q1 <= q3) {
    dl = 0.25;
    dr = 0.25;
  } else if (q2 <= q3) {
    dl = 1.0;
  } else {
    dr = 1.0;
  }
}

// Pulls back through the primitives of a state u: the cotangents of the
// velocity vb and the pressure Pb are added into ub (V = m/rho,
// P = (gamma-1)(E - |m|^2/(2 rho))).
template <int NDIM>
__device__ __forceinline__ void prim_pullback(const double (&u)[NDIM + 2], const double (&v)[NDIM], double ri,
                                              double v2, const double (&vb)[NDIM], double Pb, double gm1,
                                              double (&ub)[NDIM + 2]) {
  constexpr int NV = NDIM + 2;
#pragma unroll
  for (int e = 0; e < NDIM; ++e) {
    ub[1 + e] += vb[e] * ri - gm1 * v[e] * Pb;
    ub[0] -= vb[e] * v[e] * ri;
  }
  ub[NV - 1] += gm1 * Pb;
  ub[0] += gm1 * 0.5 * v2 * Pb;
}

// Primitives of a face state and the cotangents of its velocity and
// pressure collected so far (pulled back into the state by prim_pullback).
template <int NDIM>
struct PrimCot {
  double ri, v2, P;
  double v[NDIM];
  double vb[NDIM];
  double Pb;
};

// ub += J_F(u)^T Gb for the Euler flux along D: the parts direct in u go
// into ub, those through V and P into c.vb and c.Pb.
template <int NDIM, int D>
__device__ __forceinline__ void flux_cot(const double (&u)[NDIM + 2], const double (&Gb)[NDIM + 2], double gm1,
                                         double (&ub)[NDIM + 2], PrimCot<NDIM>& c) {
  constexpr int NV = NDIM + 2;
  c.ri = rcp(u[0]);
  c.v2 = 0.0;
#pragma unroll
  for (int e = 0; e < NDIM; ++e) {
    c.v[e] = u[1 + e] * c.ri;
    c.v2 += c.v[e] * c.v[e];
  }
  c.P = gm1 * (u[NV - 1] - 0.5 * u[0] * c.v2);
#pragma unroll
  for (int e = 0; e < NDIM; ++e) c.vb[e] = 0.0;
  c.Pb = 0.0;
  // F = (m_D, m_e v_D + P delta_eD, (E + P) v_D)
  ub[1 + D] += Gb[0];
#pragma unroll
  for (int e = 0; e < NDIM; ++e) {
    ub[1 + e] += Gb[1 + e] * c.v[D];
    c.vb[D] += Gb[1 + e] * u[1 + e];
  }
  c.Pb += Gb[1 + D];
  ub[NV - 1] += Gb[NV - 1] * c.v[D];
  c.Pb += Gb[NV - 1] * c.v[D];
  c.vb[D] += Gb[NV - 1] * (u[NV - 1] + c.P);
}

// Pull-back of a cotangent cb of c_tot = |V| + a/xi of a state with density
// rho and primitives c: into c.vb, c.Pb and the density cotangent rhob;
// xib collects dc/dxi cb.  Nothing is added where cb = 0.
template <int NDIM>
__device__ __forceinline__ void ctot_cot(double rho, double cb, double gamma, double inv_xi, PrimCot<NDIM>& c,
                                         double& rhob, double& xib) {
  const bool on = cb != 0.0;
  const double vabs = sqrt_nr(c.v2);
  const double a = sqrt_nr(gamma * c.P * c.ri);
  const double cv = (on && vabs > 0.0) ? cb * rcp(vabs) : 0.0;
#pragma unroll
  for (int e = 0; e < NDIM; ++e) c.vb[e] += cv * c.v[e];
  const double ab = cb * inv_xi;
  xib += on ? -cb * a * inv_xi * inv_xi : 0.0;
  // a = sqrt(gamma P / rho): da = gamma/(2 a rho) dP - a/(2 rho) drho
  c.Pb += on ? ab * gamma * 0.5 * rcp(a) * c.ri : 0.0;
  rhob -= on ? ab * a * 0.5 * c.ri : 0.0;
}

// Reverse of the corrected rate with gravity at one cell: given Rb, sets
// Db = (dR/dDelta)^T Rb, adds (dR/du)^T Rb into ub and returns dR/df . Rb.
template <int NDIM, int FORM>
__device__ __forceinline__ double rate_vjp(const double (&u)[NDIM + 2], const double (&Dl)[NDIM + 2],
                                           const double (&Rb)[NDIM + 2], const AdjArgs& A,
                                           double (&Db)[NDIM + 2], double (&ub)[NDIM + 2]) {
  constexpr int NV = NDIM + 2;
  const double rho = u[0], ri = rcp(rho);
  double v[NDIM], v2 = 0.0, vdm = 0.0;
#pragma unroll
  for (int e = 0; e < NDIM; ++e) {
    v[e] = u[1 + e] * ri;
    v2 += v[e] * v[e];
    vdm += v[e] * Dl[1 + e];
  }
  const double P = A.gm1 * (u[NV - 1] - 0.5 * rho * v2);
  const double H = (u[NV - 1] + P) * ri;
  const double dP = A.gm1 * (0.5 * v2 * Dl[0] - vdm + Dl[NV - 1]);
#pragma unroll
  for (int q = 0; q < NV; ++q) Db[q] = Rb[q];
  double vb[NDIM];
#pragma unroll
  for (int e = 0; e < NDIM; ++e) vb[e] = 0.0;
  double Pb = 0.0, rhob = 0.0, Hb = 0.0, dPb = 0.0, fb = 0.0;
  if constexpr (FORM == kPVS || FORM == kPMS || FORM == kDVS || FORM == kDMS) {
    constexpr bool VEL = (FORM == kPVS || FORM == kDVS);  // correction vector (1, V, H)
    double s, sb;
    const double igp = rcp(A.gamma * P);
    if constexpr (FORM == kPVS || FORM == kPMS) s = A.f * dP * rho * igp;
    else s = A.f * Dl[0];
    if constexpr (VEL) {
      sb = -Rb[0] - H * Rb[NV - 1];
#pragma unroll
      for (int e = 0; e < NDIM; ++e) {
        sb -= v[e] * Rb[1 + e];
        vb[e] -= s * Rb[1 + e];
      }
      Hb = -s * Rb[NV - 1];
    } else {  // (1, 0, H - |V|^2)
      sb = -Rb[0] - (H - v2) * Rb[NV - 1];
      Hb = -s * Rb[NV - 1];
#pragma unroll
      for (int e = 0; e < NDIM; ++e) vb[e] += 2.0 * s * Rb[NV - 1] * v[e];
    }
    if constexpr (FORM == kPVS || FORM == kPMS) {
      const double k = rho * igp;
      dPb = sb * A.f * k;
      fb = sb * dP * k;
      rhob += sb * A.f * dP * igp;
      Pb -= sb * s * rcp(P);
    } else {
      Db[0] += A.f * sb;
      fb = Dl[0] * sb;
    }
  } else if constexpr (FORM == kPD) {
    dPb = -A.f * A.inv_gm1 * Rb[NV - 1];
    fb = -A.inv_gm1 * dP * Rb[NV - 1];
  }
  if (dPb != 0.0) {
    // dP = (gamma-1)(|V|^2/2 Delta rho - V.Delta m + Delta E)
    Db[0] += A.gm1 * 0.5 * v2 * dPb;
#pragma unroll
    for (int e = 0; e < NDIM; ++e) {
      Db[1 + e] -= A.gm1 * v[e] * dPb;
      vb[e] += A.gm1 * (v[e] * Dl[0] - Dl[1 + e]) * dPb;
    }
    Db[NV - 1] += A.gm1 * dPb;
  }
  // H = (E + P) / rho
  ub[NV - 1] += Hb * ri;
  Pb += Hb * ri;
  rhob -= Hb * H * ri;
  // gravity: R_m += rho g, R_E += m.g
#pragma unroll
  for (int e = 0; e < NDIM; ++e) {
    rhob += A.g[e] * Rb[1 + e];
    ub[1 + e] += A.g[e] * Rb[NV - 1];
  }
  ub[0] += rhob;
  prim_pullback<NDIM>(u, v, ri, v2, vb, Pb, A.gm1, ub);
  return fb;
}


template <int NDIM>
__device__ __forceinline__ void half_slope(const double (&um)[NDIM + 2], const double (&u0)[NDIM + 2],
                                           const double (&up)[NDIM + 2], double (&h)[NDIM + 2]) {
#pragma unroll
  for (int v = 0; v < NDIM + 2; ++v) h[v] = mc_half(u0[v] - um[v], up[v] - u0[v]);
}

template <int NDIM>
__device__ __forceinline__ Consts adj_consts(const AdjArgs& A) {
  return Consts{A.gamma, A.gm1, A.inv_gm1, A.inv_xi, A.f};
}

// Reverse of G = F(L) + F(R) - alpha (R - L): Lb, Rb and the xi part.  The
// cotangent of alpha = max(c_L, c_R) goes to the side that set it (L on a
// tie), pulled back once per face.
template <int NDIM, int D>
__device__ __forceinline__ void llf_vjp(const Face<NDIM + 2>& L, const Face<NDIM + 2>& R, const double (&Gb)[NDIM + 2],
                                        const AdjArgs& A, double (&Lb)[NDIM + 2], double (&Rbar)[NDIM + 2],
                                        double& xib) {
  constexpr int NV = NDIM + 2;
  const bool left = L.c >= R.c;
  const double alpha = left ? L.c : R.c;
  double ab = 0.0;
#pragma unroll
  for (int v = 0; v < NV; ++v) {
    Lb[v] = alpha * Gb[v];
    Rbar[v] = -alpha * Gb[v];
    ab -= Gb[v] * (R.u[v] - L.u[v]);
  }
  PrimCot<NDIM> cl, cr, cs;
  flux_cot<NDIM, D>(L.u, Gb, A.gm1, Lb, cl);
  flux_cot<NDIM, D>(R.u, Gb, A.gm1, Rbar, cr);
  // the side that set alpha
  cs.ri = left ? cl.ri : cr.ri;
  cs.v2 = left ? cl.v2 : cr.v2;
  cs.P = left ? cl.P : cr.P;
  cs.Pb = left ? cl.Pb : cr.Pb;
#pragma unroll
  for (int e = 0; e < NDIM; ++e) {
    cs.v[e] = left ? cl.v[e] : cr.v[e];
    cs.vb[e] = left ? cl.vb[e] : cr.vb[e];
  }
  double rhob = left ? Lb[0] : Rbar[0];
  ctot_cot<NDIM>(left ? L.u[0] : R.u[0], ab, A.gamma, A.inv_xi, cs, rhob, xib);
  if (left) {
    cl.Pb = cs.Pb;
    Lb[0] = rhob;
#pragma unroll
    for (int e = 0; e < NDIM; ++e) cl.vb[e] = cs.vb[e];
  } else {
    cr.Pb = cs.Pb;
    Rbar[0] = rhob;
#pragma unroll
    for (int e = 0; e < NDIM; ++e) cr.vb[e] = cs.vb[e];
  }
  prim_pullback<NDIM>(L.u, cl.v, cl.ri, cl.v2, cl.vb, cl.Pb, A.gm1, Lb);
  prim_pullback<NDIM>(R.u, cr.v, cr.ri, cr.v2, cr.vb, cr.Pb, A.gm1, Rbar);
}

template <int NDIM, int D>
__device__ __forceinline__ void mirror_add(double (&dst)[NDIM + 2], const double (&src)[NDIM + 2]) {
#pragma unroll
  for (int v = 0; v < NDIM + 2; ++v) dst[v] += (v == 1 + D) ? -src[v] : src[v];
}


// dJdxi += dt/2 (sum of the U1 partials) + dt (sum of the U partials), in a
// fixed order, by one workgroup of NT threads (every thread of it calls this).
template <int NT>
__device__ __forceinline__ void xi_reduce(const double* p1, const double* p2, int m, double dt, double* dJdxi) {
  __shared__ double red[2][NT / 64];
  double s1 = 0.0, s2 = 0.0;
  for (int q = threadIdx.x; q < m; q += NT) {
    s1 += p1[q];
    s2 += p2[q];
  }
  s1 = wave_sum(s1);
  s2 = wave_sum(s2);
  if ((threadIdx.x & 63) == 0) {
    red[0][threadIdx.x >> 6] = s1;
    red[1][threadIdx.x >> 6] = s2;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    double a = 0.0, b = 0.0;
    for (int q = 0; q < NT / 64; ++q) {
      a += red[0][q];
      b += red[1][q];
    }
    *dJdxi += 0.5 * dt * a + dt * b;
  }
}

// The tiled 2D VJP (rsst_adjoint_tile.hip): one launch per VJP, one
// workgroup and one partial sum of xi_bar per tile; after the second VJP
// (post = 2) a one-workgroup launch folds both VJPs' partials into dJdxi,
// unless xacc is set.
int tile2_nblock(const int n[3]);
hipError_t launch_vjp_tile2(const AdjArgs& A, int form, hipStream_t s);
// dJdxi += sum of acc[0..m) in a fixed order, then acc = 0 (one workgroup).
hipError_t launch_xi_acc_fold(double* acc, int m, double* dJdxi, hipStream_t s);

}  // namespace rsstk
