// Plain FP64 CPU oracle for the semi-conservative reduced-speed-of-sound
// technique (RSST) of Iijima, Hotta & Imada (arXiv:1812.04135).
//
// TEST INFRASTRUCTURE ONLY.  This file is the independent reference that the
// GPU path is checked against.  It shares no code, header, table or constant
// with the HIP library, and only the test suite, the smoke check and the CPU
// leg of the benchmark may load it.
//
// What it computes (one explicit time step of the paper's scheme, Sec. 4.1
// "Numerical method", the eight-item implementation list):
//   * cell-centred finite volumes on a structured 1D/2D/3D Cartesian grid;
//   * piecewise-linear (MUSCL) reconstruction of the CONSERVATIVE variables
//     (rho, rho V_i, E) with the monotonized-central (MC) limiter;
//   * local Lax-Friedrichs interface flux whose characteristic speed is
//     c_tot = |V| + a/xi;
//   * flux divergence -> Delta rho, Delta(rho V_i), Delta E   (eq. pvs_dt0);
//   * Delta P from those increments                            (eq. pvs_dt_dpr);
//   * the corrected time derivatives of one of the five forms
//       PVS (eq. pvs_dt), PMS (App. A.2), DVS (App. A.1), DMS (App. A.3),
//       PD (App. A.4), or plain Euler;
//   * the external-force source rho F, rho V.F added after the correction,
//     with Delta P unchanged (App. B);
//   * second-order SSP Runge-Kutta in time, CFL number 0.4 with c_tot.
// Ideal gas: e = P/(gamma-1), a^2 = gamma P / rho, (de/dP)_rho = 1/(gamma-1),
// (de/drho)_P = 0 (Sec. 3.2, after eq. pvs_cons_therm).  General equation of
// state (the formulation of Sec. 3.2 holds for any e(rho, P)): a van der Waals
// gas, whose (de/dP)_rho, (de/drho)_P and a^2 enter through eq. pvs_cons_dpr
// and eq. pvs_cons_therm (see Gas below).
//
// Readings where the paper is silent (each also listed in the design notes):
//   * multi-D time step: dt = C * h / max(c_tot), h = 1/sum_d(1/dx_d)
//     (dt_rule 0) or h = min_d dx_d (dt_rule 1); the same dt for both stages;
//   * |V| in c_tot is the full vector magnitude; the LLF speed at a face is
//     the larger c_tot of the two reconstructed face states;
//   * MC(l,r) = 0 if l*r <= 0, else sign(l+r) min(|l+r|/2, 2|l|, 2|r|);
//   * correction coefficients use the cell-centre primitives of the same
//     stage-input state; sources use the cell-centre rho and rho V;
//   * closed free-slip walls are mirror ghosts (2 layers) with the normal
//     momentum negated; periodic sides wrap;
//   * no positivity floors; a non-physical state is reported, not repaired.
//
// Scalar type is a template parameter: `double` for the plain oracle, and a
// forward-mode dual number for branch-frozen directional derivatives (every
// branch of MC, max and |.| is decided on the primal value; ties take the
// first candidate; d|V| = 0 at |V| = 0).
//
// Layout of every field: structure of arrays [nvar][nz][ny][nx], x fastest,
// nvar = ndim + 2, variables (rho, rho V_1..rho V_ndim, E).

#include <cmath>
#include <cstdint>
#include <cstring>
#include <vector>
#include <algorithm>
#include <omp.h>

extern "C" {

typedef struct {
  int ndim;        // 1, 2 or 3
  int n[3];        // cells per axis (unused axes = 1)
  double dx[3];    // cell width per axis
  double gamma;    // specific heat ratio
  double xi;       // speed-of-sound reduction rate, >= 1
  double cfl;      // Courant number
  int dt_rule;     // 0: h = 1/sum(1/dx), 1: h = min(dx)
  double g[3];     // external force per unit mass
  int bc_lo[3];    // 0 periodic, 1 reflecting (closed free-slip), 2 reflecting
                   // with the ghost pressure extrapolated hydrostatically
  int bc_hi[3];
  int form;        // 0 Euler, 1 PVS, 2 PMS, 3 DVS, 4 DMS, 5 PD
  double cmax;     // > 0: xi from the upper limit of the sound speed (eq. cx)
  int eos;         // 0 ideal gas, 1 van der Waals gas (eos_a, eos_b)
  double eos_a;    // van der Waals attraction a
  double eos_b;    // van der Waals co-volume b
  double p_probe;  // 0, or a relative change applied to every pressure the
                   // run evaluates: measures how much a run amplifies a
                   // one-ulp difference in the equation of state (tests only)
} ora_config;

}  // extern "C"

enum { F_EULER = 0, F_PVS = 1, F_PMS = 2, F_DVS = 3, F_DMS = 4, F_PD = 5 };
enum { BC_PERIODIC = 0, BC_REFLECT = 1, BC_HYDRO = 2 };

// ---------------------------------------------------------------------------
// Scalar types
// ---------------------------------------------------------------------------

template <int N>
struct Dual {
  double v;
  double d[N];
  Dual() : v(0) { for (int i = 0; i < N; ++i) d[i] = 0; }
  Dual(double x) : v(x) { for (int i = 0; i < N; ++i) d[i] = 0; }
};

template <int N> inline Dual<N> operator+(const Dual<N>& a, const Dual<N>& b) {
  Dual<N> r; r.v = a.v + b.v; for (int i = 0; i < N; ++i) r.d[i] = a.d[i] + b.d[i]; return r; }
template <int N> inline Dual<N> operator-(const Dual<N>& a, const Dual<N>& b) {
  Dual<N> r; r.v = a.v - b.v; for (int i = 0; i < N; ++i) r.d[i] = a.d[i] - b.d[i]; return r; }
template <int N> inline Dual<N> operator-(const Dual<N>& a) {
  Dual<N> r; r.v = -a.v; for (int i = 0; i < N; ++i) r.d[i] = -a.d[i]; return r; }
template <int N> inline Dual<N> operator*(const Dual<N>& a, const Dual<N>& b) {
  Dual<N> r; r.v = a.v * b.v; for (int i = 0; i < N; ++i) r.d[i] = a.d[i] * b.v + a.v * b.d[i]; return r; }
template <int N> inline Dual<N> operator/(const Dual<N>& a, const Dual<N>& b) {
  Dual<N> r; r.v = a.v / b.v;
  for (int i = 0; i < N; ++i) r.d[i] = (a.d[i] - r.v * b.d[i]) / b.v;
  return r; }
template <int N> inline Dual<N> operator+(const Dual<N>& a, double b) { return a + Dual<N>(b); }
template <int N> inline Dual<N> operator+(double a, const Dual<N>& b) { return Dual<N>(a) + b; }
template <int N> inline Dual<N> operator-(const Dual<N>& a, double b) { return a - Dual<N>(b); }
template <int N> inline Dual<N> operator-(double a, const Dual<N>& b) { return Dual<N>(a) - b; }
template <int N> inline Dual<N> operator*(const Dual<N>& a, double b) {
  Dual<N> r; r.v = a.v * b; for (int i = 0; i < N; ++i) r.d[i] = a.d[i] * b; return r; }
template <int N> inline Dual<N> operator*(double a, const Dual<N>& b) { return b * a; }
template <int N> inline Dual<N> operator/(const Dual<N>& a, double b) { return a / Dual<N>(b); }
template <int N> inline Dual<N> operator/(double a, const Dual<N>& b) { return Dual<N>(a) / b; }

inline double val(double x) { return x; }
template <int N> inline double val(const Dual<N>& x) { return x.v; }

inline double ssqrt(double x) { return std::sqrt(x); }
template <int N> inline Dual<N> ssqrt(const Dual<N>& x) {
  Dual<N> r; r.v = std::sqrt(x.v);
  // derivative frozen to 0 at the origin (|V| = 0)
  for (int i = 0; i < N; ++i) r.d[i] = (r.v > 0) ? x.d[i] / (2.0 * r.v) : 0.0;
  return r;
}

// ---------------------------------------------------------------------------
// Per-cell pieces
// ---------------------------------------------------------------------------

// Primitive state of one conservative vector (Sec. 3.2: E = e + rho V^2/2,
// ideal gas e = P/(gamma-1); Sec. 2.1: a^2 = gamma P / rho; Sec. 4.1: c_tot).
template <class S>
struct Prim {
  S rho, v[3], P, a2, a, vabs, ctot;
};

// The equation of state.  kind 0: ideal gas with ratio gamma.  kind 1: van der
// Waals gas with constant specific heat at constant volume c_v and gas
// constant (gamma-1) c_v: P = rho R T/(1 - b rho) - a rho^2 and internal
// energy per unit mass c_v T - a rho, so the internal energy per unit volume
// is
//   e(rho, P) = (P + a rho^2)(1 - b rho)/(gamma-1) - a rho^2.
// The paper uses such a gas for tests it does not report, with parameters it
// does not give; a = b = 0 is the ideal gas.
struct Gas {
  double gamma;
  int kind;
  double a, b;
  double probe;  // relative change of every pressure evaluation (0: none)
};

static inline Gas ideal_gas(double gamma) { return Gas{gamma, 0, 0.0, 0.0, 0.0}; }

// Internal energy density e(rho, P).
template <class S>
static S eos_e(const Gas& g, const S& rho, const S& P) {
  if (g.kind == 0) return P / (g.gamma - 1.0);
  return (P + g.a * rho * rho) * (1.0 - g.b * rho) / (g.gamma - 1.0) - g.a * rho * rho;
}

// Pressure P(rho, e): e(rho, P) above solved for P.
template <class S>
static S eos_P(const Gas& g, const S& rho, const S& e) {
  if (g.kind == 0) return (g.gamma - 1.0) * e;
  return (g.gamma - 1.0) * (e + g.a * rho * rho) / (1.0 - g.b * rho) - g.a * rho * rho;
}

// (de/dP)_rho of e(rho, P) above.
template <class S>
static S eos_dedP(const Gas& g, const S& rho) {
  if (g.kind == 0) return S(1.0 / (g.gamma - 1.0));
  return (1.0 - g.b * rho) / (g.gamma - 1.0);
}

// (de/drho)_P of e(rho, P) above (product rule on each factor).
template <class S>
static S eos_dedrho(const Gas& g, const S& rho, const S& P) {
  if (g.kind == 0) return S(0.0);
  return (2.0 * g.a * rho * (1.0 - g.b * rho) - g.b * (P + g.a * rho * rho)) / (g.gamma - 1.0)
         - 2.0 * g.a * rho;
}

// Squared sound speed.  Eq. pvs_cons_therm gives (de/dP)_rho = rho T / P_S and
// (de/drho)_P = (e+P)/rho - rho T a^2 / P_S; eliminating rho T / P_S,
//   a^2 = [(e + P)/rho - (de/drho)_P] / (de/dP)_rho,
// which for the ideal gas is gamma P / rho (written so for that gas).
template <class S>
static S eos_a2(const Gas& g, const S& rho, const S& P) {
  if (g.kind == 0) return g.gamma * P / rho;
  const S e = eos_e(g, rho, P);
  return ((e + P) / rho - eos_dedrho(g, rho, P)) / eos_dedP(g, rho);
}

// Whether the gas state is physical: rho > 0 and P > 0, plus b rho < 1 and
// a^2 > 0 for the van der Waals gas.
template <class S>
static bool eos_ok(const Gas& g, const Prim<S>& p) {
  bool ok = val(p.rho) > 0 && val(p.P) > 0;
  if (g.kind != 0) ok = ok && 1.0 - g.b * val(p.rho) > 0 && val(p.a2) > 0;
  return ok;
}

// The reduction rate: a constant xi (Sec. 4.1), or, with an upper limit
// C_max of the sound speed, xi = [1 + (a/C_max)^4]^(1/4) evaluated from the
// local sound speed a of the state at hand (eq. cx, Sec. 4.1 "Functional
// form of the speed of sound reduction rate").
template <class S>
struct Xi {
  S c;          // the constant rate
  double cmax;  // > 0 selects eq. cx
};

template <class S>
static S xi_at(const Xi<S>& x, const S& a) {
  if (x.cmax > 0.0) {
    S r = a / x.cmax;
    S w = 1.0 + (r * r) * (r * r);
    return ssqrt(ssqrt(w));
  }
  return x.c;
}

template <class S>
static Prim<S> primitives(const S* u, int ndim, const Gas& gas, const Xi<S>& xi) {
  Prim<S> p;
  p.rho = u[0];
  S mv = S(0.0);  // sum_i m_i V_i = rho |V|^2
  S v2 = S(0.0);  // |V|^2
  for (int d = 0; d < 3; ++d) p.v[d] = S(0.0);
  for (int d = 0; d < ndim; ++d) {
    p.v[d] = u[1 + d] / p.rho;
    mv = mv + u[1 + d] * p.v[d];
    v2 = v2 + p.v[d] * p.v[d];
  }
  p.P = eos_P(gas, p.rho, u[ndim + 1] - 0.5 * mv);
  if (gas.probe != 0.0) p.P = p.P * (1.0 + gas.probe);
  p.a2 = eos_a2(gas, p.rho, p.P);
  p.a = ssqrt(p.a2);
  p.vabs = ssqrt(v2);
  p.ctot = p.vabs + p.a / xi_at(xi, p.a);
  return p;
}

// Euler flux along axis d: (m_d, m_e V_d + P delta_de, (E+P) V_d), eq. pvs_dt0.
template <class S>
static void euler_flux(const S* u, const Prim<S>& p, int ndim, int d, S* F) {
  F[0] = u[1 + d];
  for (int e = 0; e < ndim; ++e) {
    F[1 + e] = u[1 + e] * p.v[d];
    if (e == d) F[1 + e] = F[1 + e] + p.P;
  }
  F[ndim + 1] = (u[ndim + 1] + p.P) * p.v[d];
}

// Monotonized-central limited slope from the left and right differences.
// Written as the branch it selects: on the l*r > 0 branch sign(l+r) equals
// sign(l) and sign(r), so sign(l+r)*|l+r|/2 = (l+r)/2, sign(l+r)*2|l| = 2l
// and sign(l+r)*2|r| = 2r.  Ties take the first candidate in that order.
template <class S>
static S mc_slope(const S& l, const S& r) {
  double lv = val(l), rv = val(r);
  if (lv * rv <= 0.0) return S(0.0);
  double q1 = std::fabs(lv + rv) * 0.5, q2 = 2.0 * std::fabs(lv), q3 = 2.0 * std::fabs(rv);
  if (q1 <= q2 && q1 <= q3) return (l + r) * 0.5;
  if (q2 <= q3) return l * 2.0;
  return r * 2.0;
}

// Local Lax-Friedrichs flux at a face between reconstructed states UL, UR
// along axis d, with the RSST speed c_tot = |V| + a/xi (Sec. 4.1).
// Returns false if either face state is non-physical.
template <class S>
static bool llf_flux(const S* UL, const S* UR, int ndim, int d, const Gas& gas,
                     const Xi<S>& xi, S* Fhat) {
  const int nv = ndim + 2;
  Prim<S> pl = primitives(UL, ndim, gas, xi);
  Prim<S> pr = primitives(UR, ndim, gas, xi);
  bool ok = eos_ok(gas, pl) && eos_ok(gas, pr);
  S FL[5], FR[5];
  euler_flux(UL, pl, ndim, d, FL);
  euler_flux(UR, pr, ndim, d, FR);
  S alpha = (val(pl.ctot) >= val(pr.ctot)) ? pl.ctot : pr.ctot;
  for (int k = 0; k < nv; ++k)
    Fhat[k] = 0.5 * (FL[k] + FR[k]) - 0.5 * alpha * (UR[k] - UL[k]);
  return ok;
}

// Corrected time derivative of one cell from its stage-input state u and the
// uncorrected increments D = (Delta rho, Delta m_i, Delta E), plus the
// external force g (App. B: rho g in momentum, rho V.g in energy, Delta P
// unchanged).  f = 1 - 1/xi^2.
//   Delta P = [(de/dP)_rho]^-1 { [|V|^2/2 - (de/drho)_P] Delta rho
//             - V.Delta m + Delta E }                                      eq. pvs_dt_dpr
//           = (gamma-1) ( |V|^2/2 Delta rho - V.Delta m + Delta E )  (ideal gas)
//   PVS: R = D - f (1/a^2, V/a^2, (E+P)/(rho a^2)) Delta P                eq. pvs_dt, pvs_cons_rhs
//   PMS: R = D - f (1/a^2, 0, (E+P-rho V^2)/(rho a^2)) Delta P            App. A.2
//   DVS: R = D - f (1, V, (E+P)/rho) Delta rho                            App. A.1
//   DMS: R = D - f (1, 0, (E+P-rho V^2)/rho) Delta rho                    App. A.3
//   PD : R = D - f (0, 0, (de/dP)_rho) Delta P                            App. A.4
// (E + P = e + P + rho V^2/2 and E + P - rho V^2 = e + P - rho V^2/2.)
template <class S>
static void rsst_correct(const S* u, const S* D, int ndim, const Gas& gas,
                         const Xi<S>& xi, int form, const double* g, S* R) {
  const int nv = ndim + 2;
  const double gamma = gas.gamma;
  Prim<S> p = primitives(u, ndim, gas, xi);
  const S xc = xi_at(xi, p.a);  // the cell's rate
  S f = 1.0 - 1.0 / (xc * xc);
  S v2 = S(0.0);
  for (int d = 0; d < ndim; ++d) v2 = v2 + p.v[d] * p.v[d];
  S vdm = S(0.0);
  for (int d = 0; d < ndim; ++d) vdm = vdm + p.v[d] * D[1 + d];
  S dP;
  if (gas.kind == 0)
    dP = (gamma - 1.0) * (0.5 * v2 * D[0] - vdm + D[nv - 1]);
  else
    dP = ((0.5 * v2 - eos_dedrho(gas, p.rho, p.P)) * D[0] - vdm + D[nv - 1]) / eos_dedP(gas, p.rho);
  S E = u[nv - 1];
  for (int k = 0; k < nv; ++k) R[k] = D[k];
  switch (form) {
    case F_PVS: {
      S s = f * dP / p.a2;
      R[0] = D[0] - s;
      for (int d = 0; d < ndim; ++d) R[1 + d] = D[1 + d] - p.v[d] * s;
      R[nv - 1] = D[nv - 1] - (E + p.P) / p.rho * s;
      break;
    }
    case F_PMS: {
      S s = f * dP / p.a2;
      R[0] = D[0] - s;
      R[nv - 1] = D[nv - 1] - (E + p.P - p.rho * v2) / p.rho * s;
      break;
    }
    case F_DVS: {
      S s = f * D[0];
      R[0] = D[0] - s;
      for (int d = 0; d < ndim; ++d) R[1 + d] = D[1 + d] - p.v[d] * s;
      R[nv - 1] = D[nv - 1] - (E + p.P) / p.rho * s;
      break;
    }
    case F_DMS: {
      S s = f * D[0];
      R[0] = D[0] - s;
      R[nv - 1] = D[nv - 1] - (E + p.P - p.rho * v2) / p.rho * s;
      break;
    }
    case F_PD: {
      if (gas.kind == 0) R[nv - 1] = D[nv - 1] - f * dP / (gamma - 1.0);
      else R[nv - 1] = D[nv - 1] - f * eos_dedP(gas, p.rho) * dP;
      break;
    }
    default:
      break;
  }
  // external force (App. B), after the correction
  for (int d = 0; d < ndim; ++d) {
    R[1 + d] = R[1 + d] + u[0] * g[d];
    R[nv - 1] = R[nv - 1] + u[1 + d] * g[d];
  }
}

// ---------------------------------------------------------------------------
// Grid pieces
// ---------------------------------------------------------------------------

struct Grid {
  int ndim, n[3], nv;
  int64_t ncell;
};


static Gas gas_of(const ora_config* c) {
  Gas g = c->eos == 1 ? Gas{c->gamma, 1, c->eos_a, c->eos_b, 0.0} : ideal_gas(c->gamma);
  g.probe = c->p_probe;
  return g;
}

static Grid make_grid(const ora_config* c) {
  Grid G;
  G.ndim = c->ndim;
  for (int d = 0; d < 3; ++d) G.n[d] = (d < c->ndim) ? c->n[d] : 1;
  G.nv = c->ndim + 2;
  G.ncell = (int64_t)G.n[0] * G.n[1] * G.n[2];
  return G;
}

static inline int64_t cell_index(const Grid& G, int i, int j, int k) {
  return ((int64_t)k * G.n[1] + j) * G.n[0] + i;
}

// Value of variable v at cell index idx[] where at most one axis may lie in
// the two-layer ghost zone.  Periodic sides wrap; reflecting sides mirror
// (ghost -1-k takes cell k) and negate the momentum normal to that side.
// A hydrostatic wall (reading of the closed wall's hydrostatic variant) also
// gives the ghost the pressure of cell k carried to the ghost centre along
// the external force: P_g = P_k + rho_k g_d (x_g - x_k), x_g - x_k = -(2k+1) dx
// below the domain and +(2k+1) dx above it; rho and |V| are the mirrored
// ones, so E changes by (P_g - P_k)(de/dP)_rho.
template <class S>
static S ghosted(const Grid& G, const ora_config* c, const S* U, int v, const int idx[3]) {
  int id[3] = {idx[0], idx[1], idx[2]};
  double sign = 1.0;
  double lever = 0.0;  // (x_g - x_k) g_d for a hydrostatic ghost
  for (int d = 0; d < G.ndim; ++d) {
    const int n = G.n[d];
    if (id[d] < 0) {
      if (c->bc_lo[d] == BC_PERIODIC) id[d] += n;
      else {
        const int k = -1 - id[d];
        if (c->bc_lo[d] == BC_HYDRO) lever = -(2.0 * k + 1.0) * c->dx[d] * c->g[d];
        id[d] = k;
        if (v == 1 + d) sign = -sign;
      }
    } else if (id[d] >= n) {
      if (c->bc_hi[d] == BC_PERIODIC) id[d] -= n;
      else {
        const int k = id[d] - n;
        if (c->bc_hi[d] == BC_HYDRO) lever = (2.0 * k + 1.0) * c->dx[d] * c->g[d];
        id[d] = n - 1 - k;
        if (v == 1 + d) sign = -sign;
      }
    }
  }
  const int64_t ci = cell_index(G, id[0], id[1], id[2]);
  S x = U[(int64_t)v * G.ncell + ci];
  if (v == G.nv - 1 && lever != 0.0) {
    const S rho = U[ci];
    x = x + rho * lever * eos_dedP(gas_of(c), rho);
  }
  return (sign < 0) ? -x : x;
}

// MC slope of every variable at cell idx[] along axis d.
template <class S>
static void slopes_at(const Grid& G, const ora_config* c, const S* U, const int idx[3],
                      int d, S* sig) {
  int im[3] = {idx[0], idx[1], idx[2]}, ip[3] = {idx[0], idx[1], idx[2]};
  im[d] -= 1; ip[d] += 1;
  for (int v = 0; v < G.nv; ++v) {
    S um = ghosted(G, c, U, v, im), u0 = ghosted(G, c, U, v, idx), up = ghosted(G, c, U, v, ip);
    sig[v] = mc_slope(u0 - um, up - u0);
  }
}

// Numerical flux through the face between cell idx[] and its +1 neighbour
// along axis d (the face i+1/2).
template <class S>
static bool face_flux(const Grid& G, const ora_config* c, const S* U, const int idx[3],
                      int d, const Xi<S>& xi, S* Fhat) {
  int ir[3] = {idx[0], idx[1], idx[2]};
  ir[d] += 1;
  S sl[5], sr[5], UL[5], UR[5];
  slopes_at(G, c, U, idx, d, sl);
  slopes_at(G, c, U, ir, d, sr);
  for (int v = 0; v < G.nv; ++v) {
    UL[v] = ghosted(G, c, U, v, idx) + 0.5 * sl[v];
    UR[v] = ghosted(G, c, U, v, ir) - 0.5 * sr[v];
  }
  return llf_flux(UL, UR, G.ndim, d, gas_of(c), xi, Fhat);
}

// Full semi-discrete right-hand side R(U) on every cell.
// Returns the number of non-physical face or cell states met.
template <class S>
static int64_t rate_field(const ora_config* c, const S* U, const Xi<S>& xi, S* R) {
  const Grid G = make_grid(c);
  const int nv = G.nv;
  int64_t bad = 0;
#pragma omp parallel for collapse(2) reduction(+ : bad) schedule(static)
  for (int k = 0; k < G.n[2]; ++k) {
    for (int j = 0; j < G.n[1]; ++j) {
      for (int i = 0; i < G.n[0]; ++i) {
        const int idx[3] = {i, j, k};
        const int64_t ci = cell_index(G, i, j, k);
        S u[5], D[5], Rc[5];
        for (int v = 0; v < nv; ++v) { u[v] = U[(int64_t)v * G.ncell + ci]; D[v] = S(0.0); }
        // Delta = -sum_d (Fhat(i+1/2) - Fhat(i-1/2)) / dx_d, axes in order x, y, z
        for (int d = 0; d < G.ndim; ++d) {
          int il[3] = {i, j, k};
          il[d] -= 1;
          S Fp[5], Fm[5];
          if (!face_flux(G, c, U, idx, d, xi, Fp)) ++bad;
          if (!face_flux(G, c, U, il, d, xi, Fm)) ++bad;
          for (int v = 0; v < nv; ++v) D[v] = D[v] - (Fp[v] - Fm[v]) / c->dx[d];
        }
        const Gas gas = gas_of(c);
        Prim<S> p = primitives(u, G.ndim, gas, xi);
        if (!eos_ok(gas, p)) ++bad;
        rsst_correct(u, D, G.ndim, gas, xi, c->form, c->g, Rc);
        for (int v = 0; v < nv; ++v) R[(int64_t)v * G.ncell + ci] = Rc[v];
      }
    }
  }
  return bad;
}

// Largest c_tot over all cells.
static double max_ctot(const ora_config* c, const double* U) {
  const Grid G = make_grid(c);
  double cmax = 0.0;
#pragma omp parallel for reduction(max : cmax) schedule(static)
  for (int64_t ci = 0; ci < G.ncell; ++ci) {
    double u[5];
    for (int v = 0; v < G.nv; ++v) u[v] = U[(int64_t)v * G.ncell + ci];
    Prim<double> p = primitives(u, G.ndim, gas_of(c), Xi<double>{c->xi, c->cmax});
    if (p.ctot > cmax) cmax = p.ctot;
  }
  return cmax;
}

// dt = C * h / max c_tot  (Sec. 4.1, CFL with c_tot instead of the exact speeds)
static double cfl_dt(const ora_config* c, const double* U) {
  double h;
  if (c->dt_rule == 1) {
    h = c->dx[0];
    for (int d = 1; d < c->ndim; ++d) h = std::min(h, c->dx[d]);
  } else {
    double s = 0.0;
    for (int d = 0; d < c->ndim; ++d) s += 1.0 / c->dx[d];
    h = 1.0 / s;
  }
  return c->cfl * h / max_ctot(c, U);
}

// One second-order SSP Runge-Kutta step with a given dt:
//   U1 = U + dt R(U);   U <- (U + (U1 + dt R(U1))) / 2
template <class S>
static int64_t ssp_rk2(const ora_config* c, S* U, const Xi<S>& xi, double dt) {
  const Grid G = make_grid(c);
  const int64_t len = (int64_t)G.nv * G.ncell;
  std::vector<S> R(len), U1(len);
  int64_t bad = rate_field(c, U, xi, R.data());
  for (int64_t q = 0; q < len; ++q) U1[q] = U[q] + dt * R[q];
  bad += rate_field(c, U1.data(), xi, R.data());
  for (int64_t q = 0; q < len; ++q) U[q] = 0.5 * (U[q] + (U1[q] + dt * R[q]));
  return bad;
}

// ---------------------------------------------------------------------------
// C entry points
// ---------------------------------------------------------------------------

extern "C" {

int ora_version(void) { return 2; }

// OpenMP threads the oracle's loops use.
int ora_threads(void) { return omp_get_max_threads(); }

// Threads for the following calls (timing on one core vs all host cores).
void ora_set_threads(int n) { omp_set_num_threads(n > 0 ? n : 1); }

// Primitive recovery of one cell: out = (rho, V1, V2, V3, P, a2, a, |V|, c_tot)
void ora_prim(int ndim, double gamma, double xi, double cmax, const double* u, double* out) {
  Prim<double> p = primitives(u, ndim, ideal_gas(gamma), Xi<double>{xi, cmax});
  out[0] = p.rho; out[1] = p.v[0]; out[2] = p.v[1]; out[3] = p.v[2];
  out[4] = p.P; out[5] = p.a2; out[6] = p.a; out[7] = p.vabs; out[8] = p.ctot;
}

void ora_flux(int ndim, double gamma, const double* u, int d, double* F) {
  Prim<double> p = primitives(u, ndim, ideal_gas(gamma), Xi<double>{1.0, 0.0});
  euler_flux(u, p, ndim, d, F);
}

// Jacobian dF_d/dU of the Euler flux, row-major [nv][nv], by forward duals.
void ora_flux_jacobian(int ndim, double gamma, const double* u, int d, double* J) {
  const int nv = ndim + 2;
  Dual<5> ud[5];
  for (int k = 0; k < nv; ++k) { ud[k] = Dual<5>(u[k]); ud[k].d[k] = 1.0; }
  Prim<Dual<5>> p = primitives(ud, ndim, ideal_gas(gamma), Xi<Dual<5>>{Dual<5>(1.0), 0.0});
  Dual<5> F[5];
  euler_flux(ud, p, ndim, d, F);
  for (int r = 0; r < nv; ++r)
    for (int k = 0; k < nv; ++k) J[r * nv + k] = F[r].d[k];
}

double ora_mc(double l, double r) { return mc_slope(l, r); }

int ora_llf(int ndim, double gamma, double xi, const double* UL, const double* UR, int d,
            double* F) {
  return llf_flux(UL, UR, ndim, d, ideal_gas(gamma), Xi<double>{xi, 0.0}, F) ? 0 : 1;
}

void ora_correct(int ndim, double gamma, double xi, double cmax, int form, const double* u,
                 const double* D, const double* g, double* R) {
  rsst_correct(u, D, ndim, ideal_gas(gamma), Xi<double>{xi, cmax}, form, g, R);
}

// The equation of state at one (rho, P): out = (e(rho, P), P(rho, e) of that
// e, (de/dP)_rho, (de/drho)_P, a^2).  kind 0 ideal gas, 1 van der Waals.
void ora_eos(double gamma, int kind, double a, double b, double rho, double P, double* out) {
  const Gas g{gamma, kind, a, b, 0.0};
  const double e = eos_e(g, rho, P);
  out[0] = e;
  out[1] = eos_P(g, rho, e);
  out[2] = eos_dedP(g, rho);
  out[3] = eos_dedrho(g, rho, P);
  out[4] = eos_a2(g, rho, P);
}

// ora_prim and ora_correct for a given equation of state (constant xi).
void ora_prim_eos(int ndim, double gamma, int kind, double a, double b, double xi,
                  const double* u, double* out) {
  Prim<double> p = primitives(u, ndim, Gas{gamma, kind, a, b, 0.0}, Xi<double>{xi, 0.0});
  out[0] = p.rho; out[1] = p.v[0]; out[2] = p.v[1]; out[3] = p.v[2];
  out[4] = p.P; out[5] = p.a2; out[6] = p.a; out[7] = p.vabs; out[8] = p.ctot;
}

void ora_correct_eos(int ndim, double gamma, int kind, double a, double b, double xi, int form,
                     const double* u, const double* D, const double* g, double* R) {
  rsst_correct(u, D, ndim, Gas{gamma, kind, a, b, 0.0}, Xi<double>{xi, 0.0}, form, g, R);
}

double ora_cfl_dt(const ora_config* c, const double* U) { return cfl_dt(c, U); }

// R(U) on the whole grid; returns the count of non-physical states met.
int64_t ora_rate(const ora_config* c, const double* U, double* R) {
  return rate_field(c, U, Xi<double>{c->xi, c->cmax}, R);
}

// Advance U by nsteps SSP-RK2 steps.  dt_fixed > 0 uses that dt; otherwise
// each step takes the CFL dt of its input state.  t_end > 0 truncates the
// last step so that t reaches t_end exactly, and stops there.
// On return *t_io holds the new time, *dt_last the last dt used, and the
// return value is the count of non-physical states met (0 on success).
int64_t ora_run(const ora_config* c, double* U, int nsteps, double dt_fixed, double t_end,
                double* t_io, double* dt_last) {
  double t = t_io ? *t_io : 0.0;
  int64_t bad = 0;
  double dt = 0.0;
  for (int s = 0; s < nsteps; ++s) {
    if (t_end > 0.0 && t >= t_end) break;
    dt = (dt_fixed > 0.0) ? dt_fixed : cfl_dt(c, U);
    if (t_end > 0.0 && t + dt > t_end) dt = t_end - t;
    bad += ssp_rk2(c, U, Xi<double>{c->xi, c->cmax}, dt);
    t += dt;
  }
  if (t_io) *t_io = t;
  if (dt_last) *dt_last = dt;
  return bad;
}

// Forward-mode directional derivatives of nsteps steps with a fixed dt.
// U [nv*ncell] is advanced in place.  dU [K][nv*ncell] holds K tangent
// fields, dxi[K] the tangent of xi for each; both are advanced in place.
// K may be at most 8 per call.
int64_t ora_run_tangent(const ora_config* c, double* U, double* dU, const double* dxi, int K,
                        int nsteps, double dt) {
  constexpr int N = 8;
  if (K < 1 || K > N) return -1;
  const Grid G = make_grid(c);
  const int64_t len = (int64_t)G.nv * G.ncell;
  std::vector<Dual<N>> W(len);
  for (int64_t q = 0; q < len; ++q) {
    W[q] = Dual<N>(U[q]);
    for (int k = 0; k < K; ++k) W[q].d[k] = dU[(int64_t)k * len + q];
  }
  Dual<N> xi(c->xi);
  for (int k = 0; k < K; ++k) xi.d[k] = dxi[k];
  int64_t bad = 0;
  const Xi<Dual<N>> law{xi, c->cmax};
  for (int s = 0; s < nsteps; ++s) bad += ssp_rk2(c, W.data(), law, dt);
  for (int64_t q = 0; q < len; ++q) {
    U[q] = W[q].v;
    for (int k = 0; k < K; ++k) dU[(int64_t)k * len + q] = W[q].d[k];
  }
  return bad;
}

// Diagnostics in FP64, summed in cell order:
// out = (sum rho, sum m1, sum m2, sum m3, sum E, sum |m|^2/(2 rho), max |V|,
//        max xi|V|/a with the cell's xi), sums multiplied by the cell volume.
void ora_diag(const ora_config* c, const double* U, double* out) {
  const Grid G = make_grid(c);
  double vol = 1.0;
  for (int d = 0; d < c->ndim; ++d) vol *= c->dx[d];
  double s[6] = {0, 0, 0, 0, 0, 0}, vmax = 0.0, mmax = 0.0;
  for (int64_t ci = 0; ci < G.ncell; ++ci) {
    double u[5];
    for (int v = 0; v < G.nv; ++v) u[v] = U[(int64_t)v * G.ncell + ci];
    const Xi<double> law{c->xi, c->cmax};
    Prim<double> p = primitives(u, G.ndim, gas_of(c), law);
    s[0] += u[0];
    double m2 = 0.0;
    for (int d = 0; d < G.ndim; ++d) { s[1 + d] += u[1 + d]; m2 += u[1 + d] * u[1 + d]; }
    s[4] += u[G.nv - 1];
    s[5] += 0.5 * m2 / u[0];
    vmax = std::max(vmax, p.vabs);
    mmax = std::max(mmax, xi_at(law, p.a) * p.vabs / p.a);
  }
  for (int q = 0; q < 6; ++q) out[q] = s[q] * vol;
  out[6] = vmax;
  out[7] = mmax;
}

}  // extern "C"
