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
