"""Pins of the CPU oracle against what the paper and the mathematics fix.

None of these compares the oracle with itself: each checks a closed form, an
exact special case, an invariant, a textbook definition or a property the
paper states, chosen so that a dropped term, a wrong sign, a wrong index or a
swapped operand anywhere in the oracle fails at least one of them.
"""
import math

import numpy as np
import pytest

import oracle
import workloads as W

GAMMA = 5.0 / 3.0
FORMS = ["pvs", "pms", "dvs", "dms", "pd"]
P_FORMS = ["pvs", "pms", "pd"]
D_FORMS = ["dvs", "dms"]


def rand_cell(rng, ndim, mach=0.4):
    rho = rng.uniform(0.3, 3.0)
    P = rng.uniform(0.2, 5.0)
    a = math.sqrt(GAMMA * P / rho)
    V = rng.uniform(-1, 1, size=ndim) * mach * a
    E = P / (GAMMA - 1) + 0.5 * rho * float(V @ V)
    return np.array([rho, *(rho * V), E]), rho, V, P, a


def pvec(V, gamma=GAMMA):
    """dP = p . dU for the ideal gas (from P = (gamma-1)(E - |m|^2/(2 rho)))."""
    return (gamma - 1) * np.array([0.5 * float(V @ V), *(-V), 1.0])


# ------------------------------------------------------------------ MC limiter

def textbook_mc(l, r):
    if l * r <= 0:
        return 0.0
    return math.copysign(min(abs(l + r) / 2, 2 * abs(l), 2 * abs(r)), l + r)


def minmod3(a, b, c):
    if a > 0 and b > 0 and c > 0:
        return min(a, b, c)
    if a < 0 and b < 0 and c < 0:
        return max(a, b, c)
    return 0.0


def test_mc_enumerated_cases():
    cases = [(0.0, 0.0), (1.0, 0.0), (0.0, -2.0), (1.0, -1.0), (-3.0, 2.0),
             (1.0, 1.0), (1.0, 3.0), (3.0, 1.0), (1.0, 10.0), (10.0, 1.0),
             (-1.0, -3.0), (-3.0, -1.0), (-1.0, -10.0), (2.0, 6.0), (6.0, 2.0),
             (1e-300, 1e-300), (1.0, 1.0 + 2 ** -52)]
    for l, r in cases:
        assert oracle.mc(l, r) == textbook_mc(l, r), (l, r)
    # each branch: central, 2l, 2r
    assert oracle.mc(1.0, 1.5) == 1.25
    assert oracle.mc(1.0, 10.0) == 2.0
    assert oracle.mc(10.0, 1.0) == 2.0
    assert oracle.mc(-1.0, -10.0) == -2.0


def test_mc_random_equals_minmod_form():
    rng = np.random.default_rng(1)
    for _ in range(5000):
        l, r = rng.standard_normal(2) * 10.0 ** rng.integers(-3, 3, size=2)
        assert oracle.mc(l, r) == textbook_mc(l, r)
        assert oracle.mc(l, r) == minmod3((l + r) / 2, 2 * l, 2 * r)


# ------------------------------------------------------------- primitives

@pytest.mark.parametrize("ndim", [1, 2, 3])
def test_primitive_roundtrip(ndim):
    rng = np.random.default_rng(2)
    for _ in range(300):
        u, rho, V, P, a = rand_cell(rng, ndim)
        xi = rng.uniform(1, 30)
        p = oracle.prim(u, ndim, GAMMA, xi)
        np.testing.assert_allclose(p["rho"], rho, rtol=0)
        np.testing.assert_allclose(p["v"], V, rtol=4e-16 * 4, atol=1e-16)
        np.testing.assert_allclose(p["P"], P, rtol=1e-14)
        np.testing.assert_allclose(p["a2"], GAMMA * P / rho, rtol=1e-14)
        np.testing.assert_allclose(p["ctot"], math.sqrt(V @ V) + a / xi, rtol=1e-14)


# ------------------------------------------------------------- Euler flux

@pytest.mark.parametrize("ndim", [1, 2, 3])
def test_flux_jacobian_eigenvalues_are_euler(ndim):
    """Textbook: dF_d/dU of the Euler equations has eigenvalues V_d - a,
    V_d (ndim times) and V_d + a."""
    rng = np.random.default_rng(3)
    for _ in range(50):
        u, rho, V, P, a = rand_cell(rng, ndim, mach=0.8)
        for d in range(ndim):
            J = oracle.flux_jacobian(u, ndim, GAMMA, d)
            ev = np.sort(np.linalg.eigvals(J).real)
            ref = np.sort([V[d] - a, *([V[d]] * ndim), V[d] + a])
            np.testing.assert_allclose(ev, ref, rtol=1e-9, atol=1e-9 * a)


@pytest.mark.parametrize("ndim", [1, 3])
def test_flux_jacobian_matches_finite_difference(ndim):
    rng = np.random.default_rng(4)
    u, *_ = rand_cell(rng, ndim)
    for d in range(ndim):
        J = oracle.flux_jacobian(u, ndim, GAMMA, d)
        for k in range(ndim + 2):
            h = 1e-6 * max(1.0, abs(u[k]))
            up, um = u.copy(), u.copy()
            up[k] += h
            um[k] -= h
            col = (oracle.flux(up, ndim, GAMMA, d) - oracle.flux(um, ndim, GAMMA, d)) / (2 * h)
            np.testing.assert_allclose(J[:, k], col, rtol=1e-6, atol=1e-8)


def test_llf_consistency_and_mirror():
    """LLF(U,U) = F(U) exactly; a mirrored pair gives zero mass and energy flux."""
    rng = np.random.default_rng(5)
    for ndim in (1, 2, 3):
        u, *_ = rand_cell(rng, ndim)
        for d in range(ndim):
            assert np.array_equal(oracle.llf(u, u, ndim, GAMMA, 7.0, d),
                                  oracle.flux(u, ndim, GAMMA, d))
            m = u.copy()
            m[1 + d] = -m[1 + d]
            F = oracle.llf(m, u, ndim, GAMMA, 7.0, d)
            assert F[0] == 0.0 and F[-1] == 0.0


def test_llf_dissipation_speed_is_the_larger_ctot():
    """Local Lax-Friedrichs (Rusanov) flux: the dissipation coefficient is the
    larger local speed of the two states, here c_tot = |V| + a/xi (Sec. 4.1).
    At a contact (V = 0, equal P) the mass flux is -alpha (rho_R - rho_L)/2,
    so alpha can be read off and compared with the closed form a/xi."""
    rng = np.random.default_rng(55)
    for ndim in (1, 2, 3):
        for _ in range(50):
            xi = rng.uniform(1, 20)
            P = rng.uniform(0.5, 2)
            rl, rr = rng.uniform(0.1, 10, size=2)
            UL = np.array([rl] + [0.0] * ndim + [P / (GAMMA - 1)])
            UR = np.array([rr] + [0.0] * ndim + [P / (GAMMA - 1)])
            for d in range(ndim):
                F = oracle.llf(UL, UR, ndim, GAMMA, xi, d)
                alpha = -2 * F[0] / (rr - rl)
                ref = max(math.sqrt(GAMMA * P / rl), math.sqrt(GAMMA * P / rr)) / xi
                assert abs(alpha - ref) <= 1e-13 * ref
                assert abs(F[1 + d] - P) <= 1e-15 * P and F[-1] == 0.0


# ------------------------------------------------------- RSST correction

def corr_matrix(u, ndim, xi, form):
    nv = ndim + 2
    return np.stack([oracle.correct(u, np.eye(nv)[k], ndim, GAMMA, xi, form)
                     for k in range(nv)], axis=1)


def paper_speeds(form, Vd, a, xi, ndim):
    """Eigenvalues printed in the paper: eq. dvs_lambda1/2 for DVS, PVS and PD
    (Sec. 2.1, 3.1, App. A.4); eq. pms_speed for PMS and DMS (App. A.2/A.3);
    plus V_d for the entropy and every transverse component."""
    if form in ("pvs", "dvs", "pd"):
        D = (1 - xi ** -2) ** 2 * Vd ** 2 + 4 * a ** 2 / xi ** 2
        s = [0.5 * ((1 + xi ** -2) * Vd - math.sqrt(D)), 0.5 * ((1 + xi ** -2) * Vd + math.sqrt(D))]
    elif form in ("pms", "dms"):
        D = (1 - xi ** -2) * Vd ** 2 + a ** 2 / xi ** 2
        s = [Vd - math.sqrt(D), Vd + math.sqrt(D)]
    else:
        s = [Vd - a, Vd + a]
    return np.sort(s + [Vd] * ndim)


@pytest.mark.parametrize("form", FORMS + ["euler"])
@pytest.mark.parametrize("ndim", [1, 2, 3])
def test_characteristic_speeds_match_paper(form, ndim):
    """The semi-conservative system dU/dt = M(U) Delta, Delta = -A dU/dx,
    propagates at the eigenvalues of M A; they must be the paper's."""
    rng = np.random.default_rng(6)
    for xi in (1.0, 2.5, 10.0):
        for _ in range(10):
            u, rho, V, P, a = rand_cell(rng, ndim, mach=0.6)
            M = corr_matrix(u, ndim, xi, form)
            for d in range(ndim):
                A = oracle.flux_jacobian(u, ndim, GAMMA, d)
                ref = paper_speeds(form, V[d], a, xi, ndim)
                # characteristic polynomials (well conditioned even where
                # the entropy and transverse speeds coincide)
                cp, cr = np.poly(M @ A), np.poly(ref)
                scale = np.array([a ** k for k in range(ndim + 3)])
                np.testing.assert_allclose(cp / scale, cr / scale, rtol=0, atol=1e-11)
                ev = np.sort(np.linalg.eigvals(M @ A).real)
                np.testing.assert_allclose(ev, ref, rtol=0, atol=1e-6 * a)


# ------------------------------------------ xi from the sound speed (eq. cx)

def test_cmax_effective_sound_speed_limits():
    """Eq. cx: a/xi stays below both a and C_max, tends to a where a << C_max
    and to C_max where a >> C_max (the paper's stated purpose), and grows
    with a."""
    C = 3.0
    prev = 0.0
    for ratio in np.geomspace(1e-3, 1e3, 61):
        a = ratio * C
        rho = 1.3
        P = a * a * rho / GAMMA
        V = np.array([0.2, -0.1])
        u = np.array([rho, *(rho * V), P / (GAMMA - 1) + 0.5 * rho * float(V @ V)])
        p = oracle.prim(u, 2, GAMMA, xi=17.0, cmax=C)
        ae = p["ctot"] - p["vabs"]
        assert ae < min(p["a"], C) * (1 + 1e-15)
        assert ae > prev
        prev = ae
        if ratio <= 1e-3:
            assert abs(ae / p["a"] - 1) <= 1e-12
        if ratio >= 1e3:
            assert abs(ae / C - 1) <= 1e-12


def test_cmax_diagnostics_effective_mach():
    """With xi from eq. cx the effective Mach number is |V| over the
    effective sound speed a/xi(a) (pinned above), for a uniform state."""
    n = [6, 5]
    cfg = W.base_cfg(2, n, xi=9.0)
    cfg["cmax"] = 0.7
    rho, P, V = 1.4, 2.0, np.array([0.3, -0.2])
    shape = tuple(reversed(n))
    U = W.conservative(np.full(shape, rho), [np.full(shape, v) for v in V], np.full(shape, P))
    out = oracle.diag(cfg, U)
    p = oracle.prim(U[:, 0, 0], 2, GAMMA, xi=9.0, cmax=0.7)
    assert abs(out[7] - p["vabs"] / (p["ctot"] - p["vabs"])) <= 1e-14 * out[7]


def test_cmax_huge_reduces_to_euler_bitwise():
    """With C_max far above every sound speed, xi = 1 in every cell and face:
    the RSST forms are the Euler equations bit for bit (Sec. 3.2), whatever
    the constant xi field says."""
    for form in FORMS:
        cfg, U = W.random_state(2, [12, 10], seed_k=30, xi=7.0, form=form,
                                bc_lo=["periodic", "reflect"], g=[0.0, -0.3])
        ce = dict(cfg, form="euler", xi=1.0)
        cc = dict(cfg, cmax=1e150)
        assert np.array_equal(oracle.rate(cc, U), oracle.rate(ce, U)), form
        dt = 0.5 * oracle.cfl_dt(ce, U)
        assert np.array_equal(oracle.run(cc, U, 3, dt_fixed=dt)[0], oracle.run(ce, U, 3, dt_fixed=dt)[0])


@pytest.mark.parametrize("form", FORMS)
def test_cmax_characteristic_speeds(form):
    """About a uniform state the cell's xi is xi(a0) of eq. cx, so the system
    propagates at the paper's speeds with that xi: sound at a0/xi(a0)
    (Sec. 4.1, functional form of the reduction rate)."""
    rng = np.random.default_rng(7)
    ndim = 2
    for ratio in (0.3, 1.0, 4.0):
        for _ in range(5):
            u, rho, V, P, a = rand_cell(rng, ndim, mach=0.3)
            C = a / ratio
            xi_a = (1.0 + ratio ** 4) ** 0.25
            M = np.stack([oracle.correct(u, np.eye(ndim + 2)[k], ndim, GAMMA, 1.0, form, cmax=C)
                          for k in range(ndim + 2)], axis=1)
            for d in range(ndim):
                A = oracle.flux_jacobian(u, ndim, GAMMA, d)
                ref = paper_speeds(form, V[d], a, xi_a, ndim)
                ev = np.sort(np.linalg.eigvals(M @ A).real)
                np.testing.assert_allclose(ev, ref, rtol=0, atol=1e-6 * a)


@pytest.mark.parametrize("ndim", [1, 2, 3])
def test_tendency_identities(ndim):
    """Per-form tendencies derived from the paper's primitive forms:
    P-forms reduce the pressure tendency by xi^2 (eq. pvs_prim, pms_prim,
    pd_prim); D-forms reduce the density tendency (eq. dvs_prim, dms_prim)
    and then the pressure tendency is Delta P - f a^2 Delta rho (eq. dvs_pr);
    the velocity tendency is the Euler one for PVS, DVS and PD; the entropy
    tendency is the Euler one for PVS, PMS, DVS and DMS, and for PD it is
    shifted by -f Delta P / P (from eq. pd_prim with S = ln P - gamma ln rho)."""
    rng = np.random.default_rng(7)
    for _ in range(100):
        u, rho, V, P, a = rand_cell(rng, ndim)
        xi = rng.uniform(1.5, 40)
        f = 1 - xi ** -2
        D = rng.standard_normal(ndim + 2)
        p = pvec(V)
        dP = p @ D
        vtend_euler = (D[1:1 + ndim] - V * D[0]) / rho
        stend_euler = dP / P - GAMMA * D[0] / rho
        scale = np.abs(D).max() * max(1.0, abs(P), a * a)
        for form in FORMS:
            R = oracle.correct(u, D, ndim, GAMMA, xi, form)
            ptend = p @ R
            if form in P_FORMS:
                assert abs(ptend - dP / xi ** 2) <= 1e-13 * scale
            else:
                assert abs(R[0] - D[0] / xi ** 2) <= 1e-14 * scale
                assert abs(ptend - (dP - f * a * a * D[0])) <= 1e-13 * scale
            vt = (R[1:1 + ndim] - V * R[0]) / rho
            if form in ("pvs", "dvs", "pd"):
                np.testing.assert_allclose(vt, vtend_euler, rtol=0, atol=1e-13 * scale)
            st = ptend / P - GAMMA * R[0] / rho
            if form == "pd":
                assert abs(st - (stend_euler - f * dP / P)) <= 1e-12 * scale
            else:
                assert abs(st - stend_euler) <= 1e-12 * scale
            if form in ("pms", "dms", "pd"):
                assert np.array_equal(R[1:1 + ndim], D[1:1 + ndim])
            if form == "pd":
                assert R[0] == D[0]


@pytest.mark.parametrize("form", FORMS)
def test_correction_is_invertible_with_eigenvalue_inverse_xi_squared(form):
    """Steady states coincide with Euler's (Sec. 3.2, last paragraph): the
    correction map I - f c q^T has eigenvalues 1 (nv-1 times) and 1/xi^2."""
    rng = np.random.default_rng(8)
    for ndim in (1, 2, 3):
        u, *_ = rand_cell(rng, ndim)
        xi = 6.0
        M = corr_matrix(u, ndim, xi, form)
        ev = np.sort(np.linalg.eigvals(M).real)
        ref = np.sort([1 / xi ** 2] + [1.0] * (ndim + 1))
        np.testing.assert_allclose(ev, ref, rtol=1e-12, atol=1e-12)


def test_gravity_source_and_unchanged_delta_p():
    """App. B: rho F in momentum, rho V.F in energy, Delta P unchanged, so the
    pressure tendency of a P-form is still Delta P / xi^2."""
    rng = np.random.default_rng(9)
    for ndim in (1, 2, 3):
        u, rho, V, P, a = rand_cell(rng, ndim)
        g = rng.standard_normal(3) * np.array([1, 1, 1])
        g[ndim:] = 0
        D = rng.standard_normal(ndim + 2)
        for form in FORMS:
            R0 = oracle.correct(u, D, ndim, GAMMA, 5.0, form)
            Rg = oracle.correct(u, D, ndim, GAMMA, 5.0, form, g)
            np.testing.assert_allclose(Rg[1:1 + ndim] - R0[1:1 + ndim], rho * g[:ndim], rtol=1e-14)
            np.testing.assert_allclose(Rg[-1] - R0[-1], rho * V @ g[:ndim], rtol=1e-12, atol=1e-15)
            if form in P_FORMS:
                np.testing.assert_allclose(pvec(V) @ Rg, (pvec(V) @ D) / 25.0, rtol=1e-11,
                                           atol=1e-13)


# ------------------------------------------------------------- grid level

def test_xi_one_reduces_to_euler_bitwise():
    """Sec. 3.2 / Sec. 5: at xi = 1 every form is the conservative Euler system."""
    for ndim, n in ((1, [37]), (2, [19, 13]), (3, [9, 7, 6])):
        cfg, U = W.random_state(ndim, n, xi=1.0, g=[0.3, -0.7, 0.2][:ndim])
        cfg["form"] = "euler"
        R0 = oracle.rate(cfg, U)
        for form in FORMS:
            cfg["form"] = form
            assert np.array_equal(oracle.rate(cfg, U), R0), form


@pytest.mark.parametrize("ndim", [1, 2, 3])
def test_uniform_state_is_preserved_bitwise(ndim):
    n = [12, 10, 8][:ndim]
    cfg = W.base_cfg(ndim, n, xi=7.0)
    shape = tuple(reversed(n))
    U = W.conservative(np.full(shape, 1.3), [np.full(shape, 0.2 * (d + 1)) for d in range(ndim)],
                       np.full(shape, 0.9))
    for form in FORMS:
        cfg["form"] = form
        U2, t, _ = oracle.run(cfg, U, 15)
        assert np.array_equal(U2, U), form


def test_uniform_box_in_constant_gravity_falls_exactly():
    """Uniform periodic box under constant g: no flux divergence, Delta P = 0,
    so m = rho (V0 + g t) and E = E0 + rho V0.g t + rho |g|^2 t^2 / 2, which
    SSP-RK2 integrates exactly (the rate is a polynomial of degree 1 in t)."""
    n = [8, 6, 5]
    g = np.array([0.3, -1.0, 0.5])
    rho, P, V0 = 1.7, 2.0, np.array([0.1, 0.05, -0.02])
    shape = tuple(reversed(n))
    U = W.conservative(np.full(shape, rho), [np.full(shape, v) for v in V0], np.full(shape, P))
    cfg = W.base_cfg(3, n, xi=9.0, g=list(g))
    dt = 1e-2
    for form in FORMS:
        cfg["form"] = form
        U2, t, _ = oracle.run(cfg, U, 40, dt_fixed=dt)
        m = rho * (V0 + g * t)
        E = U[-1].flat[0] + rho * V0 @ g * t + 0.5 * rho * g @ g * t * t
        for d in range(3):
            np.testing.assert_allclose(U2[1 + d], m[d], rtol=1e-13, atol=1e-15)
        np.testing.assert_allclose(U2[-1], E, rtol=1e-13)
        np.testing.assert_allclose(U2[0], rho, rtol=1e-15)


def test_cfl_dt_closed_form():
    n = [16, 8, 4]
    cfg = W.base_cfg(3, n, xi=4.0, length=[1.0, 2.0, 0.5])
    shape = tuple(reversed(n))
    rho, P, V = 2.0, 3.0, np.array([0.3, -0.4, 0.0])
    U = W.conservative(np.full(shape, rho), [np.full(shape, v) for v in V], np.full(shape, P))
    c = 0.5 + math.sqrt(GAMMA * P / rho) / 4.0
    h = 1.0 / (16 / 1.0 + 8 / 2.0 + 4 / 0.5)
    assert abs(oracle.cfl_dt(cfg, U) - 0.4 * h / c) <= 1e-15 * (0.4 * h / c)
    cfg["dt_rule"] = 1
    assert abs(oracle.cfl_dt(cfg, U) - 0.4 * (1.0 / 16) / c) <= 1e-15


def test_diagnostics_closed_form_and_brute_force():
    """Volume-weighted sums, kinetic energy, max |V| and max xi |V| / a: a
    uniform state against closed forms, then a two-level state (half the
    cells at each of two known states) against the same closed forms."""
    n = [8, 6, 4]
    L = [1.0, 3.0, 0.5]
    cfg = W.base_cfg(3, n, xi=7.0, length=L)
    shape = tuple(reversed(n))
    vol = L[0] * L[1] * L[2]
    rho, P, V = 1.7, 2.2, np.array([0.25, -0.5, 0.125])
    U = W.conservative(np.full(shape, rho), [np.full(shape, v) for v in V], np.full(shape, P))
    out = oracle.diag(cfg, U)
    a = math.sqrt(GAMMA * P / rho)
    ke = 0.5 * rho * float(V @ V)
    E = P / (GAMMA - 1) + ke
    want = [rho * vol, *(rho * V * vol), E * vol, ke * vol, float(np.linalg.norm(V)),
            7.0 * float(np.linalg.norm(V)) / a]
    np.testing.assert_allclose(out, want, rtol=1e-14, atol=1e-15)
    # two states on alternating x columns: sums are the averages times the volume
    rho2, P2, V2 = 0.4, 0.9, np.array([-1.0, 0.0, 0.75])
    mask = (np.arange(n[0]) % 2 == 1)[None, None, :] * np.ones(shape, dtype=bool)
    r = np.where(mask, rho2, rho)
    p = np.where(mask, P2, P)
    vs = [np.where(mask, V2[d], V[d]) for d in range(3)]
    U = W.conservative(r, vs, p)
    out = oracle.diag(cfg, U)
    a2 = math.sqrt(GAMMA * P2 / rho2)
    ke2 = 0.5 * rho2 * float(V2 @ V2)
    E2 = P2 / (GAMMA - 1) + ke2
    half = 0.5 * vol
    want = [(rho + rho2) * half, *((rho * V + rho2 * V2) * half), (E + E2) * half, (ke + ke2) * half,
            max(np.linalg.norm(V), np.linalg.norm(V2)),
            7.0 * max(np.linalg.norm(V) / a, np.linalg.norm(V2) / a2)]
    np.testing.assert_allclose(out, want, rtol=1e-13, atol=1e-15)


def _sums(cfg, U):
    return np.array([U[v].sum() for v in range(U.shape[0])])


@pytest.mark.parametrize("walls", [False, True])
def test_conservation_per_form(walls):
    """Sec. 5 / App. A: mass is conserved by DVS, DMS (at constant xi, the
    modified law reduces to <rho>) and PD; momentum by PMS, DMS and PD; energy
    only at xi = 1; PVS conserves none of them.  With walls in y, x-momentum
    is still conserved (no tangential wall stress) and mass never crosses."""
    n = [24, 20]
    kw = dict(bc_lo=["periodic", "reflect"]) if walls else {}
    cfg, U = W.random_state(2, n, xi=4.0, seed_k=11, **kw)
    s0 = _sums(cfg, U)
    scale = np.abs(U).reshape(U.shape[0], -1).max(axis=1) * U[0].size
    for form in FORMS + ["euler"]:
        cfg["form"] = form
        U2, _, _ = oracle.run(cfg, U, 30)
        drift = np.abs(_sums(cfg, U2) - s0) / scale
        cons_mass = form in ("dvs", "dms", "pd", "euler")
        cons_mx = form in ("pms", "dms", "pd", "euler")
        cons_my = cons_mx and not walls
        cons_E = form == "euler"
        for idx, cons in ((0, cons_mass), (1, cons_mx), (2, cons_my), (3, cons_E)):
            if cons:
                assert drift[idx] < 1e-14, (form, idx, drift)
            else:
                assert drift[idx] > 1e-9, (form, idx, drift)


@pytest.mark.parametrize("form", FORMS)
def test_isobaric_density_structure(form):
    """Sec. 2.2 / 3.1: with V = 0 and uniform P, a non-uniform density
    (diffused here by the scheme) leaves P and V untouched under the
    pressure-reducing forms, but generates pressure under DVS/DMS with the
    tendency -f a^2 Delta rho of eq. dvs_pr."""
    n = [20, 18]
    cfg, U = W.random_state(2, n, xi=5.0, seed_k=12, mach=0.0, dP=0.0)
    cfg["form"] = form
    assert np.all(U[1:3] == 0)
    P0 = (GAMMA - 1) * U[-1]
    if form in P_FORMS:
        U2, _, _ = oracle.run(cfg, U, 10)
        assert np.array_equal(U2[1:3], U[1:3])
        assert np.array_equal(U2[-1], U[-1])
        assert not np.array_equal(U2[0], U[0])
    else:
        R = oracle.rate(cfg, U)
        cfg_e = dict(cfg, form="euler")
        D = oracle.rate(cfg_e, U)
        f = 1 - 1 / 25.0
        a2 = GAMMA * P0 / U[0]
        Ptend = (GAMMA - 1) * R[-1]  # V = 0: p = (gamma-1)(0, 0, 1)
        np.testing.assert_allclose(Ptend, -f * a2 * D[0], rtol=1e-12,
                                   atol=1e-12 * np.abs(a2 * D[0]).max())
        assert np.abs(Ptend).max() > 1e-6


@pytest.mark.parametrize("ndim", [1, 2])
def test_reflecting_walls_equal_mirrored_periodic_domain(ndim):
    """A closed free-slip wall is a mirror: the walled solution equals the
    periodic solution of the doubled domain with mirrored initial data
    (even in rho, tangential momentum and E, odd in normal momentum)."""
    n = [14, 11][:ndim]
    cfg, U = W.random_state(ndim, n, xi=3.0, seed_k=13,
                            bc_lo=["reflect"] + ["periodic"] * (ndim - 1))
    ax = U.ndim - 1  # x is the last array axis
    M = np.flip(U, axis=ax).copy()
    M[1] = -M[1]
    Ud = np.ascontiguousarray(np.concatenate([U, M], axis=ax))
    cfg_d = dict(cfg)
    cfg_d["n"] = [2 * n[0]] + cfg["n"][1:]
    cfg_d["bc_lo"] = ["periodic"] * 3
    cfg_d["bc_hi"] = ["periodic"] * 3
    Uw, _, _ = oracle.run(cfg, U, 20)
    Up, _, _ = oracle.run(cfg_d, Ud, 20)
    left = Up[(slice(None),) * ax + (slice(0, n[0]),)]
    np.testing.assert_allclose(Uw, left, rtol=1e-14, atol=1e-14)


# ------------------------------------------------------------- linear waves

def _mode(f):
    c = np.fft.rfft(f)[1]
    return abs(c) * 2 / f.size, np.angle(c)


@pytest.mark.parametrize("form,xi", [("euler", 1.0), ("pvs", 10.0), ("pms", 10.0),
                                     ("dvs", 10.0), ("dms", 10.0), ("pd", 10.0)])
def test_sound_wave_travels_at_reduced_speed(form, xi):
    """Linear analysis (Sec. 2.1, 3.1, App. A): at V = 0 every form carries
    sound at +-a/xi and leaves the entropy wave static.  Measure the phase of
    the characteristic variables w+ = dP/(rho a) + dV/xi and of the static
    mode: w0 = drho - dP/a^2 (entropy) for PVS, PMS, DVS, DMS; for PD, whose
    third equation is mass conservation (eq. pd_prim), the static mode is a
    density change at fixed P and V, with left eigenvector (1, 0, -xi^2/a^2)
    in (rho, V, P), so w0 = drho - xi^2 dP/a^2."""
    cfg, U, meta = W.wave1d(xi=xi, form=form)
    a0 = meta["a0"]
    t_q = 0.25 * xi / a0  # a quarter crossing at the reduced speed
    U2, t, _ = oracle.run(cfg, U, 100000, t_end=t_q)
    assert abs(t - t_q) < 1e-14

    def charvars(U):
        rho = U[0]
        V = U[1] / rho
        P = (GAMMA - 1) * (U[2] - 0.5 * rho * V * V)
        dP, drho = P - 1.0, rho - 1.0
        kappa = xi ** 2 if form == "pd" else 1.0
        return dP / a0 + V / xi, drho - kappa * dP / a0 ** 2

    wp0, we0 = charvars(U)
    wp1, we1 = charvars(U2)
    A0, ph0 = _mode(wp0)
    A1, ph1 = _mode(wp1)
    shift = (ph0 - ph1) % (2 * math.pi)
    expect = 2 * math.pi * (a0 / xi) * t
    assert abs(shift - expect) < 0.01 * expect, (shift, expect)
    assert A1 > 0.95 * A0
    Ae0, phe0 = _mode(we0)
    Ae1, phe1 = _mode(we1)
    assert abs((phe1 - phe0 + math.pi) % (2 * math.pi) - math.pi) < 0.01
    assert Ae1 > 0.95 * Ae0


# ------------------------------------------------------ convergence (Sec. 4.2)

def _wave30(N, form):
    cfg, U, meta = W.wave2d_oblique(N, form)
    return cfg, U, meta["theta"]


def _l1_errors(N, form):
    cfg, U, th = _wave30(N, form)
    U2, t, _ = oracle.run(cfg, U, 10 ** 6, t_end=1.0)

    def fields(U):
        rho = U[0]
        vx, vy = U[1] / rho, U[2] / rho
        P = (GAMMA - 1) * (U[3] - 0.5 * rho * (vx * vx + vy * vy))
        return {"S": np.log(P) - GAMMA * np.log(rho),
                "Vperp": -vx * math.sin(th) + vy * math.cos(th), "rho": rho, "P": P}

    f0, f1 = fields(U), fields(U2)
    return {k: float(np.mean(np.abs(f1[k] - f0[k]))) for k in f0}


@pytest.mark.slow
def test_second_order_convergence_as_in_paper():
    """Sec. 4.2: entropy/shear wave at 30 degrees, xi = 5, t = 1.  S and
    V_perp converge at second order in every form; rho and P do so in PVS,
    PMS and PD; P does not converge in DVS and DMS."""
    errs = {f: {N: _l1_errors(N, f) for N in (16, 32, 64)} for f in FORMS}
    for f in FORMS:
        for var in ("S", "Vperp"):
            order = math.log2(errs[f][32][var] / errs[f][64][var])
            assert order > 1.6, (f, var, order)
        if f in P_FORMS:
            for var in ("rho", "P"):
                order = math.log2(errs[f][32][var] / errs[f][64][var])
                assert order > 1.7, (f, var, order)
        else:
            order = math.log2(errs[f][32]["P"] / errs[f][64]["P"])
            assert order < 1.0, (f, "P", order)


# ------------------------------------------------------------- tangents

def test_tangent_matches_central_differences():
    """The dual-number path (used to check the adjoint) against central
    differences of the plain FP64 path, directions in U and in xi."""
    cfg, U = W.random_state(2, [10, 9], xi=4.0, seed_k=14, white=0.0)
    rng = np.random.default_rng(15)
    nsteps, dt = 3, 2e-3
    dU = rng.standard_normal((2, U.size))
    dxi = np.array([0.0, 1.0])
    _, T = oracle.run_tangent(cfg, U, dU, dxi, nsteps, dt)
    for q in range(2):
        h = 1e-6
        up = (U.ravel() + h * dU[q]).reshape(U.shape)
        um = (U.ravel() - h * dU[q]).reshape(U.shape)
        cp, cm = dict(cfg), dict(cfg)
        cp["xi"] += h * dxi[q]
        cm["xi"] -= h * dxi[q]
        Fp, _, _ = oracle.run(cp, up, nsteps, dt_fixed=dt)
        Fm, _, _ = oracle.run(cm, um, nsteps, dt_fixed=dt)
        fd = (Fp - Fm).ravel() / (2 * h)
        np.testing.assert_allclose(T[q], fd, rtol=1e-5, atol=1e-6 * np.abs(fd).max())
