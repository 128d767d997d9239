"""Pins of the hydrostatic wall (the closed free-slip wall of Sec. 4.4 with
the ghost pressure carried along the external force): it is the mirror wall
when the force along the wall's normal is zero, it keeps mass (and tangential
momentum) exactly, and it removes most of the start-up transient that a
mirror wall gives a layer in hydrostatic balance (the first cell's face
pressure then balances gravity)."""
import numpy as np
import pytest

import oracle
import workloads as W


def _column(n, bc, form="euler", xi=1.0):
    cfg = W.base_cfg(2, [8, n], xi=xi, form=form, bc_lo=["periodic", bc], g=[0.0, -1.0])
    y = W.centres(cfg, 1)
    rho0, P0 = W.polytrope(y)
    rho = np.broadcast_to(rho0[:, None], (n, 8))
    P = np.broadcast_to(P0[:, None], (n, 8))
    return cfg, W.conservative(rho, [np.zeros((n, 8))] * 2, P)


@pytest.mark.parametrize("form", ["pvs", "pms", "dvs", "dms", "pd", "euler"])
def test_without_normal_force_it_is_the_mirror_wall(form):
    cfg, U0 = W.random_state(2, [20, 12], seed_k=770, xi=4.0, form=form,
                             bc_lo=["hydro", "reflect"], g=[0.0, -0.6])
    Uh, _, _ = oracle.run(cfg, U0, 5)
    Ur, _, _ = oracle.run(dict(cfg, bc_lo=["reflect", "reflect"], bc_hi=["reflect", "reflect"]), U0, 5)
    assert np.array_equal(Uh, Ur)


@pytest.mark.parametrize("form,xi", [("euler", 1.0), ("pvs", 5.0), ("pms", 5.0)])
def test_layer_at_rest_keeps_mass_and_loses_most_of_the_transient(form, xi):
    """Mass is checked where the form conserves it at xi = 1 (Euler)."""
    out = {}
    for bc in ("reflect", "hydro"):
        cfg, U0 = _column(48, bc, form, xi)
        U, t, _ = oracle.run(cfg, U0, 100)
        out[bc] = float(np.abs(U[2] / U[0]).max())
        if form == "euler":
            assert abs(U[0].sum() - U0[0].sum()) <= 1e-13 * U0[0].sum()
        assert np.abs(U[1]).max() <= 1e-14  # no x momentum appears
    print(f"[walls] {form} xi={xi} max|V_y| after 100 steps: {out}")
    assert out["hydro"] <= 0.2 * out["reflect"], out


@pytest.mark.parametrize("form,xi,cmax", [("pvs", 6.3, 0.0), ("pms", 6.3, 0.0), ("pvs", 1.0, 10.0)])
def test_mirror_walls_reproduce_the_symmetric_periodic_rt_run(form, xi, cmax):
    """The Sec. 4.4 problem is even about x = 1/8 and 3/8; the periodic run
    on [0,1] and the run on [1/8, 3/8] between mirror walls are then the same
    discrete problem (the wall's ghosts are the periodic run's mirror-image
    cells), so they agree to rounding: the mirror wall pinned against
    periodic wrapping, and the strip used as the finer Sec. 4.4 reference."""
    n, nsteps = 64, 80
    cfg, U0, meta = W.rt2d(n, form=form, xi=xi)
    cfs, U0s, ms = W.rt2d(n, form=form, xi=xi, strip=True)
    assert ms["x0"] == 0.125 and cfs["n"][:2] == [n // 4, n] and cfs["dx"][:2] == cfg["dx"][:2]
    if cmax:
        cfg["cmax"] = cfs["cmax"] = cmax
    sl = slice(n // 8, 3 * n // 8)
    assert np.array_equal(U0s, U0[:, :, sl])
    Uf, tf, _ = oracle.run(cfg, U0, nsteps)
    Us, ts, _ = oracle.run(cfs, U0s, nsteps)
    assert abs(tf - ts) <= 1e-14 * tf
    sc = [np.abs(Uf[0]).max(), np.abs(Uf[1:3]).max(), np.abs(Uf[1:3]).max(), np.abs(Uf[3]).max()]
    err = max(float(np.abs(Us[v] - Uf[v][:, sl]).max() / sc[v]) for v in range(4))
    assert err <= 1e-13, err
    # and the periodic run itself is mirror-symmetric about x = 1/8
    mir = Uf[:, :, ::-1]  # x -> 1 - x, then the shift by 1/4 below: x -> 1/4 - x
    mir = np.roll(mir, n // 4, axis=2)
    mir[1] = -mir[1]
    assert float(np.abs(mir - Uf).max() / np.abs(Uf).max()) <= 1e-13
