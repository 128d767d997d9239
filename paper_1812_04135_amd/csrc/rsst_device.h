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
  double inv_cmax2;  // 1/C_max^2 when xi follows the sound speed (eq. cx), else 0
  double vdw_a;   // van der Waals attraction a (kExtVdw kernels only)
  double vdw_b;   // van der Waals co-volume b
};

// Extension bits of a kernel's template argument, above the form (0..5):
// xi from the sound speed (eq. cx), the van der Waals equation of state in
// place of the ideal gas, and hydrostatic walls on the y or march axis.
enum Ext { kExtCmax = 8, kExtVdw = 16, kExtHydro = 32 };

// A reconstructed face state: conservative values plus the primitive
// quantities the LLF flux needs.  `vn` is the velocity normal to the face.
template <int NV>
struct Face {
  double u[NV];
  double P;
  double c;
  double vn;
};

// Reciprocal: hardware seed (relative error about 2^-24 on gfx950) refined
// by two Newton steps (about 1 ulp).
__device__ __forceinline__ double rcp(double x) {
  double r = __builtin_amdgcn_rcp(x);
  double e = fma(-x, r, 1.0);
  r = fma(r, e, r);
  e = fma(-x, r, 1.0);
  return fma(r, e, r);
}

// Square root of x >= 0: reciprocal-square-root seed (relative error about
// 2^-24 on gfx950) and one coupled Newton step on (s, h) = (x y, y/2), which
// leaves 1.5 e^2, about 2^-47.6; sqrt(0) = 0.
__device__ __forceinline__ double sqrt_nr(double x) {
  const double y = __builtin_amdgcn_rsq(fmax(x, 1e-300));
  const double s = x * y, h = 0.5 * y;
  return fma(fma(-s, s, x), h, s);
}

// Half of the monotonized-central limited slope (Sec. 4.1, item 2):
//   MC(l, r) = 0 if l r <= 0, else sign(l+r) min(|l+r|/2, 2|l|, 2|r|).
// With s = sign(l) (as +-1.0) this is s max(0, min(2|l|, s(l+r)/2, 2 s r)); the
// function returns MC/2 = s max(0, min(|l|, s r, (|l| + s r)/4)), which is
// the offset of the face states from the cell value.  On the l r > 0 branch
// |l| + |r| = |l + r| exactly, so the result equals MC/2 bit for bit.
// Multiplying by s = +-1 is exact and keeps every min/max operand an
// arithmetic result (no NaN-quieting of bit-built operands).
__device__ __forceinline__ double mc_half(double l, double r) {
  const double s = __hiloint2double((__double2hiint(l) & 0x80000000) | 0x3ff00000, 0);
  const double sr = s * r;
  const double al = fabs(l);
  const double h = fmax(fmin(fmin(al, sr), 0.25 * (al + sr)), 0.0);
  return s * h;
}

// 1/sqrt(x), x >= 1: hardware seed refined by two Newton steps.
__device__ __forceinline__ double rsq_nr(double x) {
  double y = __builtin_amdgcn_rsq(x);
  const double hx = 0.5 * x;
  y = y * fma(-hx, y * y, 1.5);
  return y * fma(-hx, y * y, 1.5);
}

// With an upper limit C_max of the sound speed (eq. cx) the rate is
// xi = w^(1/4), w = 1 + (a/C_max)^4, taken from the sound speed of the state
// at hand.  Effective sound speed a/xi = a w^(-1/4), from a^2:
__device__ __forceinline__ double a_eff_cmax(double a2, const Consts& K) {
  const double r2 = a2 * K.inv_cmax2;
  const double y = rsq_nr(fma(r2, r2, 1.0));  // w^(-1/2)
  return sqrt_nr(a2) * sqrt_nr(y);
}

// f = 1 - 1/xi^2 = 1 - w^(-1/2) = r^4 y^2 / (1 + y), y = w^(-1/2): no
// cancellation when a << C_max.
__device__ __forceinline__ double f_cmax(double a2, const Consts& K) {
  const double r2 = a2 * K.inv_cmax2;
  const double r4 = r2 * r2;
  const double y = rsq_nr(1.0 + r4);
  return r4 * (y * y) * rcp(1.0 + y);
}

// Gas pressure P and squared sound speed a^2 from rho, 1/rho and the internal
// energy density e = E - rho|V|^2/2 (Sec. 3.2).  Ideal gas: P = (gamma-1) e,
// a^2 = gamma P / rho.  Van der Waals gas with constant specific heat
// (kExtVdw), e = (P + a rho^2)(1 - b rho)/(gamma-1) - a rho^2, solved for P:
//   P = (gamma-1)(e + a rho^2)/(1 - b rho) - a rho^2,
//   a^2 = gamma (P + a rho^2) / (rho (1 - b rho)) - 2 a rho,
// the isentropic (dP/drho)_S of that gas.  The thermodynamic derivatives of
// eq. pvs_cons_therm give the same a^2; the oracle takes it from there.
template <int X>
__device__ __forceinline__ void eos_pa2(double rho, double ri, double e, const Consts& K, double& P,
                                        double& a2) {
  if constexpr ((X & kExtVdw) != 0) {
    const double q = K.vdw_a * rho * rho;
    const double r1 = rcp(fma(-K.vdw_b, rho, 1.0));
    P = fma(K.gm1 * (e + q), r1, -q);
    a2 = fma(K.gamma * (P + q), ri * r1, -2.0 * K.vdw_a * rho);
  } else {
    P = K.gm1 * e;
    a2 = K.gamma * P * ri;
  }
}

// Primitive recovery of a face state, normal axis D (Sec. 3.2 and 4.1):
// V = m/rho, P and a^2 from the equation of state, c_tot = |V| + a/xi
// (kExtCmax: xi from eq. cx).
template <int NDIM, int D, int X = 0>
__device__ __forceinline__ void face_prims(Face<NDIM + 2>& s, const Consts& K) {
  constexpr int NV = NDIM + 2;
  const double ri = rcp(s.u[0]);
  double v2 = 0.0, vn = 0.0;
#pragma unroll
  for (int e = 0; e < NDIM; ++e) {
    const double ve = s.u[1 + e] * ri;
    v2 = fma(ve, ve, v2);
    if (e == D) vn = ve;
  }
  double a2;
  eos_pa2<X>(s.u[0], ri, fma(-0.5 * s.u[0], v2, s.u[NV - 1]), K, s.P, a2);
  if constexpr ((X & kExtCmax) != 0) s.c = sqrt_nr(v2) + a_eff_cmax(a2, K);
  else s.c = fma(sqrt_nr(a2), K.inv_xi, sqrt_nr(v2));
  s.vn = vn;
}

// Face state U + h (h: half slopes, signed) and its primitives.
template <int NDIM, int D, int X = 0>
__device__ __forceinline__ void make_face(const double (&u)[NDIM + 2], const double (&h)[NDIM + 2],
                                          bool plus, const Consts& K, Face<NDIM + 2>& s) {
#pragma unroll
  for (int v = 0; v < NDIM + 2; ++v) s.u[v] = plus ? u[v] + h[v] : u[v] - h[v];
  face_prims<NDIM, D, X>(s, K);
}

// Twice the local Lax-Friedrichs flux between left state L and right state
// R along D (Sec. 4.1, item 4):
//   G = F(U_L) + F(U_R) - max(c_L, c_R) (U_R - U_L) = 2 Fhat,
// with the Euler flux F_d(U) = (m_d, m_e V_d + P delta_de, (E + P) V_d).
// The factor 1/2 is folded into the 1/dx of the divergence.
template <int NDIM, int D>
__device__ __forceinline__ void flux2(const Face<NDIM + 2>& L, const Face<NDIM + 2>& R,
                                      double (&G)[NDIM + 2]) {
  constexpr int NV = NDIM + 2;
  const double a = fmax(L.c, R.c);
  G[0] = fma(-a, R.u[0] - L.u[0], L.u[1 + D] + R.u[1 + D]);
#pragma unroll
  for (int e = 0; e < NDIM; ++e) {
    const double fl = (e == D) ? fma(L.u[1 + e], L.vn, L.P) : L.u[1 + e] * L.vn;
    const double fr = (e == D) ? fma(R.u[1 + e], R.vn, R.P) : R.u[1 + e] * R.vn;
    G[1 + e] = fma(-a, R.u[1 + e] - L.u[1 + e], fl + fr);
  }
  const double el = (L.u[NV - 1] + L.P) * L.vn, er = (R.u[NV - 1] + R.P) * R.vn;
  G[NV - 1] = fma(-a, R.u[NV - 1] - L.u[NV - 1], el + er);
}

// Mirror image of a face state across a wall normal to D.
template <int NDIM, int D>
__device__ __forceinline__ Face<NDIM + 2> mirror(const Face<NDIM + 2>& s) {
  Face<NDIM + 2> m = s;
  m.u[1 + D] = -s.u[1 + D];
  m.vn = -s.vn;
  return m;
}

// Corrected time derivative of one cell (eq. pvs_dt, pvs_dt_dpr; App. A.1-A.4)
// plus the external force (App. B).  u: stage-input cell state; Dl: the
// uncorrected increments (Delta rho, Delta m_i, Delta E).  Returns the
// non-physical flags of the cell.  kExtCmax: f from the cell's own xi
// (eq. cx); kExtVdw: the van der Waals gas of eos_pa2.
template <int NDIM, int FORM, int X = 0>
__device__ __forceinline__ unsigned rsst_rate(const double (&u)[NDIM + 2], const double (&Dl)[NDIM + 2],
                                              const Consts& K, const double (&g)[3],
                                              double (&R)[NDIM + 2]) {
  constexpr int NV = NDIM + 2;
  constexpr bool VDW = (X & kExtVdw) != 0;
  const double rho = u[0];
  const double ri = rcp(rho);
  double v[NDIM];
  double v2 = 0.0, vdm = 0.0;
#pragma unroll
  for (int e = 0; e < NDIM; ++e) {
    v[e] = u[1 + e] * ri;
    v2 = fma(v[e], v[e], v2);
    vdm = fma(v[e], Dl[1 + e], vdm);
  }
  double P, a2;
  eos_pa2<X>(rho, ri, fma(-0.5 * rho, v2, u[NV - 1]), K, P, a2);
  // van der Waals: 1 - b rho, the factor of (de/dP)_rho = (1 - b rho)/(gamma-1)
  const double omb = VDW ? fma(-K.vdw_b, rho, 1.0) : 1.0;
  unsigned bad = 0;
  if (!(rho > 0.0) || !(omb > 0.0)) bad |= kBadRho;
  if (!(P > 0.0) || (VDW && !(a2 > 0.0))) bad |= kBadP;
  if (!(fabs(u[NV - 1]) < INFINITY) || !(fabs(P) < INFINITY)) bad |= kNonFinite;
#pragma unroll
  for (int q = 0; q < NV; ++q) R[q] = Dl[q];
  if constexpr (FORM != kEuler) {
    const double f = (X & kExtCmax) ? f_cmax(a2, K) : K.f;
    // Delta P = [(de/dP)_rho]^-1 {[|V|^2/2 - (de/drho)_P] Delta rho - V.Delta m + Delta E};
    // ideal gas: (gamma-1) (|V|^2/2 Delta rho - V.Delta m + Delta E)
    double dP;
    if constexpr (VDW) {
      // (de/drho)_P = [2 a rho (1 - b rho) - b (P + a rho^2)]/(gamma-1) - 2 a rho
      const double ar2 = 2.0 * K.vdw_a * rho;
      const double dedr = fma(K.inv_gm1, fma(ar2, omb, -K.vdw_b * fma(K.vdw_a * rho, rho, P)), -ar2);
      dP = K.gm1 * rcp(omb) * (fma(fma(0.5, v2, -dedr), Dl[0], Dl[NV - 1]) - vdm);
    } else {
      dP = K.gm1 * (fma(0.5 * v2, Dl[0], Dl[NV - 1]) - vdm);
    }
    const double H = (u[NV - 1] + P) * ri;  // (E + P)/rho
    if constexpr (FORM == kPVS || FORM == kPMS) {
      // s = f Delta P / a^2 (ideal gas: a^2 = gamma P / rho)
      const double s = VDW ? f * dP * rcp(a2) : f * dP * rho * rcp(K.gamma * P);
      R[0] -= s;
      if constexpr (FORM == kPVS) {
#pragma unroll
        for (int e = 0; e < NDIM; ++e) R[1 + e] = fma(-v[e], s, R[1 + e]);
        R[NV - 1] = fma(-H, s, R[NV - 1]);
      } else {
        R[NV - 1] = fma(-(H - v2), s, R[NV - 1]);
      }
    } else if constexpr (FORM == kDVS || FORM == kDMS) {
      const double s = f * Dl[0];
      R[0] -= s;
      if constexpr (FORM == kDVS) {
#pragma unroll
        for (int e = 0; e < NDIM; ++e) R[1 + e] = fma(-v[e], s, R[1 + e]);
        R[NV - 1] = fma(-H, s, R[NV - 1]);
      } else {
        R[NV - 1] = fma(-(H - v2), s, R[NV - 1]);
      }
    } else {  // PD: energy only, (de/dP)_rho Delta P
      R[NV - 1] = fma(-f * (VDW ? omb * K.inv_gm1 : K.inv_gm1), dP, R[NV - 1]);
    }
  }
#pragma unroll
  for (int e = 0; e < NDIM; ++e) {
    R[1 + e] = fma(rho, g[e], R[1 + e]);
    R[NV - 1] = fma(u[1 + e], g[e], R[NV - 1]);
  }
  return bad;
}

// c_tot of a cell state (for the CFL time step).
template <int NDIM, int X = 0>
__device__ __forceinline__ double cell_ctot(const double (&u)[NDIM + 2], const Consts& K) {
  constexpr int NV = NDIM + 2;
  const double ri = rcp(u[0]);
  double v2 = 0.0;
#pragma unroll
  for (int e = 0; e < NDIM; ++e) {
    const double ve = u[1 + e] * ri;
    v2 = fma(ve, ve, v2);
  }
  double P, a2;
  eos_pa2<X>(u[0], ri, fma(-0.5 * u[0], v2, u[NV - 1]), K, P, a2);
  if constexpr ((X & kExtCmax) != 0) return sqrt_nr(v2) + a_eff_cmax(a2, K);
  else return fma(sqrt_nr(a2), K.inv_xi, sqrt_nr(v2));
}

// ---- cross-lane moves (wave64 DPP) -------------------------------------

// Value held by lane l-1 (lane 0 receives 0: with bound_ctrl set the
// hardware writes 0 where the source lane is outside the wave, so no
// zeroed destination has to be prepared).
__device__ __forceinline__ double from_left(double x) {
  const int lo = __builtin_amdgcn_mov_dpp(__double2loint(x), 0x138, 0xF, 0xF, true);
  const int hi = __builtin_amdgcn_mov_dpp(__double2hiint(x), 0x138, 0xF, 0xF, true);
  return __hiloint2double(hi, lo);
}

// Value held by lane l+1 (lane 63 receives 0).
__device__ __forceinline__ double from_right(double x) {
  const int lo = __builtin_amdgcn_mov_dpp(__double2loint(x), 0x130, 0xF, 0xF, true);
  const int hi = __builtin_amdgcn_mov_dpp(__double2hiint(x), 0x130, 0xF, 0xF, true);
  return __hiloint2double(hi, lo);
}

__device__ __forceinline__ double wave_max(double x) {
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) x = fmax(x, __shfl_xor(x, o, 64));
  return x;
}

// Butterfly sum over the wave: every lane ends with the same value, formed
// in the same order on every run.
__device__ __forceinline__ double wave_sum(double x) {
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) x = x + __shfl_xor(x, o, 64);
  return x;
}

}  // namespace rsstk
