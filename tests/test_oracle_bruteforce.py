"""A second, brute-force transcription of the scheme on tiny grids (pure
Python, scalar loops), against the C++ oracle: 8 cells in 1D, 6 x 5 in 2D,
4 x 4 x 4 in 3D, every form, periodic, mirror and hydrostatic walls, gravity,
the C_max law and the van der Waals gas, two SSP-RK2 steps at a fixed dt.

It is organised differently from the oracle on purpose: the grid is copied
into an array padded with two explicit ghost layers per side (filled by
wrapping or mirroring, Sec. 4.2 and 4.4; a hydrostatic wall's ghost takes its
pressure from the equation of state at the carried pressure), every face flux is computed once into
a face array, and the divergence is assembled from those arrays.  What both
follow is the paper's step: MUSCL with MC on the conservative variables,
LLF with c_tot = |V| + a/xi (Sec. 4.1), the divergence (eq. pvs_dt0), Delta P
(eq. pvs_dt_dpr with eq. pvs_cons_therm), the corrections (eq. pvs_dt, App.
A), gravity after the correction (App. B) and SSP-RK2."""
import math
from itertools import product

import numpy as np
import pytest

import oracle
import workloads as W

G = W.GAMMA


def e_of(rho, P, gas):
    if gas is None:
        return P / (G - 1.0)
    a, b = gas["eos_a"], gas["eos_b"]
    return (P + a * rho * rho) * (1.0 - b * rho) / (G - 1.0) - a * rho * rho


def P_of(rho, e, gas):
    if gas is None:
        return (G - 1.0) * e
    a, b = gas["eos_a"], gas["eos_b"]
    return (G - 1.0) * (e + a * rho * rho) / (1.0 - b * rho) - a * rho * rho


def derivs(rho, P, gas):
    """(de/dP)_rho, (de/drho)_P and a^2 (central differences are not used:
    these are the derivatives of e(rho, P) written out)."""
    if gas is None:
        return 1.0 / (G - 1.0), 0.0, G * P / rho
    a, b = gas["eos_a"], gas["eos_b"]
    dedP = (1.0 - b * rho) / (G - 1.0)
    dedr = (2.0 * a * rho * (1.0 - b * rho) - b * (P + a * rho * rho)) / (G - 1.0) - 2.0 * a * rho
    e = e_of(rho, P, gas)
    return dedP, dedr, ((e + P) / rho - dedr) / dedP


def xi_of(a, xi, cmax):
    return (1.0 + (a / cmax) ** 4) ** 0.25 if cmax > 0 else xi


def prims(u, nd, gas, xi, cmax):
    rho = u[0]
    v = [u[1 + d] / rho for d in range(nd)]
    v2 = sum(x * x for x in v)
    P = P_of(rho, u[nd + 1] - 0.5 * rho * v2, gas)
    a2 = derivs(rho, P, gas)[2]
    a = math.sqrt(a2)
    return rho, v, v2, P, a2, math.sqrt(v2) + a / xi_of(a, xi, cmax)


def mc(l, r):
    if l * r <= 0.0:
        return 0.0
    s = 1.0 if l + r > 0 else -1.0
    return s * min(abs(l + r) / 2.0, 2.0 * abs(l), 2.0 * abs(r))


def padded(U, cfg, gas=None):
    """Copy of U with two ghost layers per side of each used axis.  A
    'hydro' wall's ghost carries the mirrored cell's pressure to the ghost
    centre with the hydrostatic gradient rho g_d (rho and |V| mirrored)."""
    nd = cfg["ndim"]
    n = cfg["n"][:nd]
    nv = nd + 2
    shape = [n[d] + 4 for d in range(nd)]
    Pd = np.zeros([nv] + shape[::-1])
    fields = [U[v].reshape(n[::-1]) for v in range(nv)]
    for gidx in product(*[range(-2, n[d] + 2) for d in range(nd)]):
        src = list(gidx)
        neg = -1
        shift = 0.0  # x_ghost - x_source along the wall's axis
        wall = None
        for d in range(nd):
            if src[d] < 0 or src[d] >= n[d]:
                side = "bc_lo" if src[d] < 0 else "bc_hi"
                if cfg[side][d] == "periodic":
                    src[d] %= n[d]
                else:
                    mirror = -1 - src[d] if src[d] < 0 else 2 * n[d] - 1 - src[d]
                    shift = (gidx[d] - mirror) * cfg["dx"][d]
                    src[d] = mirror
                    neg = d
                    wall = cfg[side][d], d
        vals = [fields[v][tuple(src[::-1])] for v in range(nv)]
        if neg >= 0:
            vals[1 + neg] = -vals[1 + neg]
        if wall is not None and wall[0] == "hydro":
            rho = vals[0]
            v2 = sum((vals[1 + e] / rho) ** 2 for e in range(nd))
            P = P_of(rho, vals[nv - 1] - 0.5 * rho * v2, gas)
            Pg = P + rho * cfg["g"][wall[1]] * shift
            vals[nv - 1] = e_of(rho, Pg, gas) + 0.5 * rho * v2
        for v in range(nv):
            Pd[(v,) + tuple(g + 2 for g in gidx[::-1])] = vals[v]
    return Pd


def rate(U, cfg, gas=None):
    nd = cfg["ndim"]
    n = cfg["n"][:nd]
    nv = nd + 2
    xi, cmax = cfg["xi"], cfg.get("cmax", 0.0)
    form = cfg["form"]
    Pd = padded(U, cfg, gas)

    def at(v, idx):  # idx: cell index per axis (may be -2..n+1)
        return Pd[(v,) + tuple(i + 2 for i in idx[::-1])]

    # fluxes through every face i+1/2, i = -1..n-1, per axis
    flux = []
    for d in range(nd):
        F = {}
        rng = [range(-1, n[e]) if e == d else range(n[e]) for e in range(nd)]
        for idx in product(*rng):
            L, R = list(idx), list(idx)
            R[d] += 1
            uL, uR = [], []
            for v in range(nv):
                def val(c, off):
                    q = list(c)
                    q[d] += off
                    return at(v, q)
                sl = mc(val(L, 0) - val(L, -1), val(L, 1) - val(L, 0))
                sr = mc(val(R, 0) - val(R, -1), val(R, 1) - val(R, 0))
                uL.append(val(L, 0) + 0.5 * sl)
                uR.append(val(R, 0) - 0.5 * sr)
            pl, pr = prims(uL, nd, gas, xi, cmax), prims(uR, nd, gas, xi, cmax)
            alpha = max(pl[5], pr[5])

            def euler(u, p):
                vd, P = p[1][d], p[3]
                f = [u[1 + d]] + [u[1 + e] * vd + (P if e == d else 0.0) for e in range(nd)]
                return f + [(u[nd + 1] + P) * vd]
            fl, fr = euler(uL, pl), euler(uR, pr)
            F[tuple(idx)] = [0.5 * (fl[v] + fr[v]) - 0.5 * alpha * (uR[v] - uL[v]) for v in range(nv)]
        flux.append(F)
    out = np.zeros_like(U)
    for idx in product(*[range(n[d]) for d in range(nd)]):
        lin = 0
        for d in reversed(range(nd)):
            lin = lin * n[d] + idx[d]
        Dl = [0.0] * nv
        for d in range(nd):
            lo = list(idx)
            lo[d] -= 1
            Fp, Fm = flux[d][tuple(idx)], flux[d][tuple(lo)]
            for v in range(nv):
                Dl[v] = Dl[v] - (Fp[v] - Fm[v]) / cfg["dx"][d]
        u = [U[v].reshape(-1)[lin] for v in range(nv)]
        rho, V, v2, P, a2, _ = prims(u, nd, gas, xi, cmax)
        f = 1.0 - 1.0 / xi_of(math.sqrt(a2), xi, cmax) ** 2
        dedP, dedr, _ = derivs(rho, P, gas)
        dP = ((0.5 * v2 - dedr) * Dl[0] - sum(V[e] * Dl[1 + e] for e in range(nd)) + Dl[nv - 1]) / dedP
        E = u[nv - 1]
        H = (E + P) / rho
        R = list(Dl)
        if form in ("pvs", "pms"):
            s = f * dP / a2
            R[0] -= s
            if form == "pvs":
                for e in range(nd):
                    R[1 + e] -= V[e] * s
                R[nv - 1] -= H * s
            else:
                R[nv - 1] -= (H - v2) * s
        elif form in ("dvs", "dms"):
            s = f * Dl[0]
            R[0] -= s
            if form == "dvs":
                for e in range(nd):
                    R[1 + e] -= V[e] * s
                R[nv - 1] -= H * s
            else:
                R[nv - 1] -= (H - v2) * s
        elif form == "pd":
            R[nv - 1] -= f * dedP * dP
        for e in range(nd):
            R[1 + e] += rho * cfg["g"][e]
            R[nv - 1] += u[1 + e] * cfg["g"][e]
        for v in range(nv):
            out[v].reshape(-1)[lin] = R[v]
    return out


def rk2(U, cfg, dt, nsteps, gas=None):
    U = U.copy()
    for _ in range(nsteps):
        U1 = U + dt * rate(U, cfg, gas)
        U = 0.5 * (U + (U1 + dt * rate(U1, cfg, gas)))
    return U


CASES = [
    (1, [8], ["periodic"], [0.0], "pvs"),
    (1, [8], ["reflect"], [-0.7], "pd"),
    (2, [6, 5], ["periodic", "reflect"], [0.0, -0.5], "pms"),
    (2, [6, 5], ["reflect", "periodic"], [0.3, 0.0], "dvs"),
    (2, [6, 5], ["reflect", "reflect"], [0.1, -0.4], "dms"),
    (2, [6, 5], ["periodic", "periodic"], [0.0, 0.0], "euler"),
    (3, [4, 4, 4], ["periodic", "periodic", "reflect"], [0.0, 0.0, -1.0], "pvs"),
    (3, [4, 4, 4], ["reflect", "periodic", "periodic"], [0.2, 0.0, 0.0], "pd"),
    (1, [8], ["hydro"], [-0.7], "pvs"),
    (2, [6, 5], ["periodic", "hydro"], [0.0, -0.8], "pms"),
    (2, [6, 5], ["hydro", "hydro"], [0.3, -0.5], "dvs"),
    (3, [4, 4, 4], ["periodic", "hydro", "hydro"], [0.0, 0.4, -1.0], "pd"),
]


@pytest.mark.parametrize("variant", ["ideal", "cmax", "vdw"])
@pytest.mark.parametrize("nd,n,bc,g,form", CASES, ids=[f"{c[0]}d-{c[4]}-{c[2][0][0]}" for c in CASES])
def test_bruteforce_matches_oracle(nd, n, bc, g, form, variant):
    gas = W.VDW if variant == "vdw" else None
    cfg, U0 = W.random_state(nd, n, seed_k=800 + nd * 10 + len(form), xi=3.0, form=form, bc_lo=bc, g=g,
                             mach=0.3, gas=gas)
    if variant == "cmax":
        cfg["cmax"] = 1.1
    dt = 0.3 * oracle.cfl_dt(cfg, U0)
    Ub = rk2(U0, cfg, dt, 2, gas)
    Uo, _, _ = oracle.run(cfg, U0, 2, dt_fixed=dt)
    s = [np.abs(Uo[0]).max()] + [np.abs(Uo[0]).max()] * nd + [np.abs(Uo[-1]).max()]
    err = max(float(np.abs(Ub[v] - Uo[v]).max() / s[v]) for v in range(nd + 2))
    assert err <= 1e-14, err
