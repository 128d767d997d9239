"""Pins of the oracle's general equation of state (Sec. 3.2, eq. pvs_cons_dpr,
eq. pvs_cons_therm), with the van der Waals gas of the workloads module.

Each check rests on something other than the oracle's own formulas: the ideal
gas as the a = b = 0 case, finite differences of e(rho, P) and P(rho, e), the
first law along an isentrope, the textbook van der Waals sound speed, the
chain rule for the pressure rate, and the linear RSST sound wave, which must
travel at a/xi with the van der Waals a."""
import math

import numpy as np
import pytest

import oracle
import workloads as W

GAMMA = W.GAMMA
VDW = W.VDW
FORMS = ["pvs", "pms", "dvs", "dms", "pd"]
STATES = [(1.0, 1.0), (0.3, 0.05), (2.5, 4.0), (5.0, 0.7), (0.8, 12.0)]


def _P(rho, e, gas):
    """P(rho, e) of the oracle, through its primitive recovery of (rho, 0, e)."""
    return oracle.prim([rho, 0.0, e], 1, GAMMA, 1.0, gas=gas)["P"]


def test_zero_parameters_are_the_ideal_gas():
    gas0 = {"eos": "vdw", "eos_a": 0.0, "eos_b": 0.0}
    for rho, P in STATES:
        a, b = oracle.eos(GAMMA, rho, P), oracle.eos(GAMMA, rho, P, gas0)
        for k in a:
            assert abs(a[k] - b[k]) <= 1e-15 * max(1.0, abs(a[k])), (k, a[k], b[k])
    # and a whole run in every form
    for form in FORMS:
        cfg, U = W.random_state(2, [24, 20], seed_k=601, xi=4.0, form=form,
                                bc_lo=["periodic", "reflect"], g=[0.0, -0.4])
        U1, _, _ = oracle.run(cfg, U, 4)
        U2, _, _ = oracle.run(W.with_gas(cfg, gas0), U, 4)
        assert np.max(np.abs(U1 - U2)) <= 1e-13 * np.max(np.abs(U1))


def test_thermodynamic_derivatives_are_those_of_e():
    """(de/dP)_rho and (de/drho)_P against central differences of e(rho, P),
    and P(rho, e) inverts e(rho, P)."""
    for rho, P in STATES:
        q = oracle.eos(GAMMA, rho, P, VDW)
        assert abs(q["P_of_e"] - P) <= 1e-14 * max(1.0, P)
        hP, hr = 1e-5 * P, 1e-5 * rho
        dedP = (oracle.eos(GAMMA, rho, P + hP, VDW)["e"] - oracle.eos(GAMMA, rho, P - hP, VDW)["e"]) / (2 * hP)
        dedr = (oracle.eos(GAMMA, rho + hr, P, VDW)["e"] - oracle.eos(GAMMA, rho - hr, P, VDW)["e"]) / (2 * hr)
        assert abs(dedP - q["dedP"]) <= 1e-8 * abs(q["dedP"])
        assert abs(dedr - q["dedrho"]) <= 1e-8 * max(abs(q["dedrho"]), abs(q["e"] / rho))


def test_sound_speed_is_the_isentropic_derivative():
    """a^2 of the oracle (from eq. pvs_cons_therm) equals (dP/drho) at constant
    specific entropy: by the first law d(e/rho) = -P d(1/rho) there, i.e.
    de = (e + P)/rho drho, so (dP/drho)_S = (dP/drho)_e + (dP/de)_rho (e + P)/rho,
    here by central differences of the oracle's P(rho, e); and it equals the
    textbook van der Waals form."""
    a_, b_ = VDW["eos_a"], VDW["eos_b"]
    for rho, P in STATES:
        q = oracle.eos(GAMMA, rho, P, VDW)
        e = q["e"]
        hr, he = 1e-5 * rho, 1e-5 * abs(e)
        dPdr = (_P(rho + hr, e, VDW) - _P(rho - hr, e, VDW)) / (2 * hr)
        dPde = (_P(rho, e + he, VDW) - _P(rho, e - he, VDW)) / (2 * he)
        a2_fd = dPdr + dPde * (e + P) / rho
        a2_book = GAMMA * (P + a_ * rho * rho) / (rho * (1.0 - b_ * rho)) - 2.0 * a_ * rho
        assert abs(q["a2"] - a2_book) <= 1e-13 * a2_book
        assert abs(q["a2"] - a2_fd) <= 1e-7 * a2_book
        # and the primitive recovery reports the same a^2
        pr = oracle.prim([rho, 0.0, e], 1, GAMMA, 1.0, gas=VDW)
        assert abs(pr["a2"] - q["a2"]) <= 1e-14 * q["a2"] and abs(pr["P"] - P) <= 1e-14 * max(1, P)


def _pressure_of_u(u, ndim, gas):
    return oracle.prim(u, ndim, GAMMA, 1.0, gas=gas)["P"]


def _rate_along(u, D, ndim, gas, h=1e-6):
    """d/dt P(U) for dU/dt = D, by central differences through the oracle's
    primitive recovery."""
    u, D = np.asarray(u, float), np.asarray(D, float)
    return (_pressure_of_u(u + h * D, ndim, gas) - _pressure_of_u(u - h * D, ndim, gas)) / (2 * h)


@pytest.mark.parametrize("ndim", [1, 2, 3])
def test_delta_p_is_the_pressure_rate_and_the_correction_divides_it_by_xi2(ndim):
    """Delta P of eq. pvs_dt_dpr is the rate of P(U) when U changes at the
    uncorrected rate D (chain rule through e = E - |m|^2/(2 rho) and the
    equation of state).  The P-forms then change P at Delta P / xi^2 (their
    correction moves P alone by -f Delta P: PVS and PMS at constant entropy,
    PD at constant rho), and the D-forms change rho at Delta rho / xi^2."""
    rng = np.random.default_rng(W.seed(602))
    xi = 7.0
    f = 1.0 - 1.0 / xi ** 2
    for _ in range(6):
        rho = rng.uniform(0.5, 3.0)
        V = rng.uniform(-0.5, 0.5, ndim)
        P = rng.uniform(0.3, 3.0)
        e = W.internal_energy(rho, P, GAMMA, VDW)
        u = np.concatenate([[rho], rho * V, [e + 0.5 * rho * V @ V]])
        D = rng.normal(size=ndim + 2)
        dP = _rate_along(u, D, ndim, VDW)
        a2 = oracle.eos(GAMMA, rho, P, VDW)["a2"]
        for form in FORMS:
            R = oracle.correct(u, D, ndim, GAMMA, xi, form, gas=VDW)
            if form in ("pvs", "pms"):
                assert abs((D[0] - R[0]) * a2 / f - dP) <= 1e-7 * (abs(dP) + 1)
            if form in ("pvs", "pms", "pd"):
                assert abs(_rate_along(u, R, ndim, VDW) - dP / xi ** 2) <= 1e-7 * (abs(dP) + 1), form
            else:
                assert abs(R[0] - D[0] / xi ** 2) <= 1e-14 * abs(D[0])
            if form in ("pvs", "dvs"):  # velocity rate unchanged by the correction
                for d in range(ndim):
                    C = R - D
                    assert abs(C[1 + d] - V[d] * C[0]) <= 1e-13 * (abs(C[0]) + 1)


@pytest.mark.parametrize("form", FORMS)
def test_sound_wave_in_vdw_gas_travels_at_reduced_speed(form):
    """A right-going linear sound wave set up with the van der Waals a0
    travels at a0/xi and stays right-going (an ideal-gas a0 would be 4.6%
    slower here and shed a left-going part)."""
    xi = 10.0
    cfg, U, meta = W.wave1d(xi=xi, form=form, gas=VDW)
    a0 = meta["a0"]
    assert abs(a0 - math.sqrt(GAMMA)) > 0.04 * a0
    t_q = 0.25 * xi / a0
    U2, t, _ = oracle.run(cfg, U, 100000, t_end=t_q)

    def wplus(U):
        rho = U[0]
        V = U[1] / rho
        P = np.array([_P(r, E - 0.5 * r * v * v, VDW) for r, v, E in zip(rho, V, U[2])])
        return (P - 1.0) / a0 + V / xi

    def mode(f):
        c = np.fft.rfft(f)[1]
        return abs(c) * 2 / f.size, np.angle(c)

    A0, ph0 = mode(wplus(U))
    A1, ph1 = mode(wplus(U2))
    shift = (ph0 - ph1) % (2 * math.pi)
    expect = 2 * math.pi * (a0 / xi) * t
    assert abs(shift - expect) < 0.01 * expect, (shift, expect)
    assert A1 > 0.95 * A0
