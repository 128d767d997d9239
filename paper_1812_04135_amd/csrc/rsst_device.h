// Device building blocks of the RSST stage on gfx950 (CDNA4, wave64).
//
// Everything here is FP64 arithmetic on registers; storage precision is
// handled by the kernels.  Notation follows arXiv:1812.04135:
//   U = (rho, m_1..m_ndim, E), m = rho V, E = e + rho|V|^2/2, e = P/(gamma-1)
//   c_tot = |V| + a/xi, a^2 = gamma P / rho                  (Sec. 4.1)
//   f = 1 - 1/xi^2                                           (eq. pvs_dt)
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

// No implicit contraction: every fused multiply-add below is written as fma(),
// so an expression rounds the same way in every inlined copy (a face computed
// by a tile-edge row and by an interior row gives the same bits).
#pragma clang fp contract(off)

namespace rsstk {

enum Form { kEuler = 0, kPVS = 1, kPMS = 2, kDVS = 3, kDMS = 4, kPD = 5 };

enum Flag : unsigned { kBadRho = 1u, kBadP = 2u, kNonFinite = 4u };

struct Consts {
  double gamma;   // ratio of specific heats
  double gm1;     // gamma - 1
  double inv_gm1; // 1 / (gamma - 1) = (de/dP)_rho of the ideal gas
  double inv_xi;  // 1 / xi
  double f;       // 1 - 1/xi^2
};

// A reconstructed face state: conservative values plus the primitive
// quantities the LLF flux needs.  `vn` is the velocity normal to the face.
template <int NV>
struct Face {
  double u[NV];
  double P;
  double c;
  double vn;
};

// Monotonized-central limited slope.  On the l*r > 0 branch l and r share a
// sign, so |l + r| = |l| + |r| exactly and sign(l + r) = sign(l): the value
// equals sign(l+r) min(|l+r|/2, 2|l|, 2|r|) bit for bit (Sec. 4.1, item 2).
__device__ __forceinline__ double mc_slope(double l, double r) {
  const double al = fabs(l), ar = fabs(r);
  const double q = fmin(0.5 * (al + ar), 2.0 * fmin(al, ar));
  return (l * r > 0.0) ? copysign(q, l) : 0.0;
}

// Primitive recovery of a face state, normal axis D (Sec. 3.2 and 4.1).
template <int NDIM, int D>
__device__ __forceinline__ void face_prims(Face<NDIM + 2>& s, const Consts& K) {
  constexpr int NV = NDIM + 2;
  const double rinv = 1.0 / s.u[0];
  double v2 = 0.0, mv = 0.0, vn = 0.0;
#pragma unroll
  for (int e = 0; e < NDIM; ++e) {
    const double ve = s.u[1 + e] * rinv;
    v2 = fma(ve, ve, v2);
    mv = fma(s.u[1 + e], ve, mv);
    if (e == D) vn = ve;
  }
  s.P = K.gm1 * fma(-0.5, mv, s.u[NV - 1]);
  const double a2 = K.gamma * s.P * rinv;
  s.c = fma(sqrt(a2), K.inv_xi, sqrt(v2));
  s.vn = vn;
}

// Euler flux of a face state along its normal axis D (eq. pvs_dt0).
template <int NDIM, int D>
__device__ __forceinline__ void face_flux(const Face<NDIM + 2>& s, double (&F)[NDIM + 2]) {
  constexpr int NV = NDIM + 2;
  F[0] = s.u[1 + D];
#pragma unroll
  for (int e = 0; e < NDIM; ++e) F[1 + e] = (e == D) ? fma(s.u[1 + e], s.vn, s.P) : s.u[1 + e] * s.vn;
  F[NV - 1] = (s.u[NV - 1] + s.P) * s.vn;
}

// Local Lax-Friedrichs flux between left state L and right state R along D:
// Fhat = (F(L) + F(R))/2 - max(c_L, c_R) (U_R - U_L)/2   (Sec. 4.1, item 4).
template <int NDIM, int D>
__device__ __forceinline__ void llf(const Face<NDIM + 2>& L, const Face<NDIM + 2>& R,
                                    double (&F)[NDIM + 2]) {
  constexpr int NV = NDIM + 2;
  double FL[NV], FR[NV];
  face_flux<NDIM, D>(L, FL);
  face_flux<NDIM, D>(R, FR);
  const double ha = 0.5 * fmax(L.c, R.c);
#pragma unroll
  for (int v = 0; v < NV; ++v) F[v] = fma(-ha, R.u[v] - L.u[v], 0.5 * (FL[v] + FR[v]));
}

// Mirror image of a face state across a wall normal to D.
template <int NDIM, int D>
__device__ __forceinline__ Face<NDIM + 2> mirror(const Face<NDIM + 2>& s) {
  Face<NDIM + 2> m = s;
  m.u[1 + D] = -s.u[1 + D];
  m.vn = -s.vn;
  return m;
}

// Build a face state U0 +- sigma/2 and its primitives.
template <int NDIM, int D>
__device__ __forceinline__ void make_face(const double (&u)[NDIM + 2], const double (&sig)[NDIM + 2],
                                          double sgn, const Consts& K, Face<NDIM + 2>& s) {
#pragma unroll
  for (int v = 0; v < NDIM + 2; ++v) s.u[v] = fma(0.5 * sgn, sig[v], u[v]);
  face_prims<NDIM, D>(s, K);
}

// Corrected time derivative of one cell (eq. pvs_dt, pvs_dt_dpr; App. A.1-A.4)
// plus the external force (App. B).  u: stage-input cell state; Dl: the
// uncorrected increments (Delta rho, Delta m_i, Delta E).  Returns the
// non-physical flags of the cell.
template <int NDIM>
__device__ __forceinline__ unsigned rsst_rate(const double (&u)[NDIM + 2], const double (&Dl)[NDIM + 2],
                                              const Consts& K, int form, const double (&g)[3],
                                              double (&R)[NDIM + 2]) {
  constexpr int NV = NDIM + 2;
  const double rho = u[0];
  const double rinv = 1.0 / rho;
  double v[NDIM];
  double v2 = 0.0, mv = 0.0, vdm = 0.0;
#pragma unroll
  for (int e = 0; e < NDIM; ++e) {
    v[e] = u[1 + e] * rinv;
    v2 = fma(v[e], v[e], v2);
    mv = fma(u[1 + e], v[e], mv);
    vdm = fma(v[e], Dl[1 + e], vdm);
  }
  const double P = K.gm1 * fma(-0.5, mv, u[NV - 1]);
  unsigned bad = 0;
  if (!(rho > 0.0)) bad |= kBadRho;
  if (!(P > 0.0)) bad |= kBadP;
  if (!(fabs(u[NV - 1]) < INFINITY) || !(fabs(P) < INFINITY)) bad |= kNonFinite;
  // Delta P = (gamma-1) (|V|^2/2 Delta rho - V.Delta m + Delta E)
  const double dP = K.gm1 * (fma(0.5 * v2, Dl[0], Dl[NV - 1]) - vdm);
  const double H = (u[NV - 1] + P) * rinv;  // (E + P)/rho
#pragma unroll
  for (int q = 0; q < NV; ++q) R[q] = Dl[q];
  switch (form) {
    case kPVS: {  // coefficients (1, V, H)/a^2 on Delta P
      const double s = K.f * dP * rho / (K.gamma * P);
      R[0] -= s;
#pragma unroll
      for (int e = 0; e < NDIM; ++e) R[1 + e] = fma(-v[e], s, R[1 + e]);
      R[NV - 1] = fma(-H, s, R[NV - 1]);
      break;
    }
    case kPMS: {  // (1, 0, H - |V|^2)/a^2 on Delta P; momentum conservative
      const double s = K.f * dP * rho / (K.gamma * P);
      R[0] -= s;
      R[NV - 1] = fma(-(H - v2), s, R[NV - 1]);
      break;
    }
    case kDVS: {  // (1, V, H) on Delta rho
      const double s = K.f * Dl[0];
      R[0] -= s;
#pragma unroll
      for (int e = 0; e < NDIM; ++e) R[1 + e] = fma(-v[e], s, R[1 + e]);
      R[NV - 1] = fma(-H, s, R[NV - 1]);
      break;
    }
    case kDMS: {  // (1, 0, H - |V|^2) on Delta rho
      const double s = K.f * Dl[0];
      R[0] -= s;
      R[NV - 1] = fma(-(H - v2), s, R[NV - 1]);
      break;
    }
    case kPD: {  // energy only: (de/dP)_rho Delta P
      R[NV - 1] = fma(-K.f * K.inv_gm1, dP, R[NV - 1]);
      break;
    }
    default:
      break;
  }
#pragma unroll
  for (int e = 0; e < NDIM; ++e) {
    R[1 + e] = fma(rho, g[e], R[1 + e]);
    R[NV - 1] = fma(u[1 + e], g[e], R[NV - 1]);
  }
  return bad;
}

// c_tot of a cell state (for the CFL time step).
template <int NDIM>
__device__ __forceinline__ double cell_ctot(const double (&u)[NDIM + 2], const Consts& K) {
  constexpr int NV = NDIM + 2;
  const double rinv = 1.0 / u[0];
  double v2 = 0.0, mv = 0.0;
#pragma unroll
  for (int e = 0; e < NDIM; ++e) {
    const double ve = u[1 + e] * rinv;
    v2 = fma(ve, ve, v2);
    mv = fma(u[1 + e], ve, mv);
  }
  const double P = K.gm1 * fma(-0.5, mv, u[NV - 1]);
  return fma(sqrt(K.gamma * P * rinv), K.inv_xi, sqrt(v2));
}

// ---- cross-lane moves (wave64 DPP) -------------------------------------

// Value held by lane l-1 (lane 0 receives 0).
__device__ __forceinline__ double from_left(double x) {
  const int lo = __builtin_amdgcn_update_dpp(0, __double2loint(x), 0x138, 0xF, 0xF, false);
  const int hi = __builtin_amdgcn_update_dpp(0, __double2hiint(x), 0x138, 0xF, 0xF, false);
  return __hiloint2double(hi, lo);
}

// Value held by lane l+1 (lane 63 receives 0).
__device__ __forceinline__ double from_right(double x) {
  const int lo = __builtin_amdgcn_update_dpp(0, __double2loint(x), 0x130, 0xF, 0xF, false);
  const int hi = __builtin_amdgcn_update_dpp(0, __double2hiint(x), 0x130, 0xF, 0xF, false);
  return __hiloint2double(hi, lo);
}

__device__ __forceinline__ double wave_max(double x) {
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) x = fmax(x, __shfl_xor(x, o, 64));
  return x;
}

}  // namespace rsstk
