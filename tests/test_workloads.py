"""Input generators that carry physics of their own (no GPU)."""
import numpy as np

import workloads as W


def test_rt_column_mass_is_hydrostatic():
    """Sec. 4.4: m_c is the column mass above y of the unperturbed profile, so
    m_c(1) = 0 and dm_c/dy = -rho; hence P = Pc - m_c g_y balances gravity."""
    y = np.linspace(0.0, 1.0, 4001)
    m = W.rt_column_mass(y)
    assert m[-1] == 0.0
    rho = 1.0 + 4.5 * (1.0 + np.tanh((y - 0.5) / 0.025))
    # fourth-order central difference of the closed form
    h = 1e-4
    d = (-W.rt_column_mass(y + 2 * h) + 8 * W.rt_column_mass(y + h) - 8 * W.rt_column_mass(y - h)
         + W.rt_column_mass(y - 2 * h)) / (12 * h)
    assert np.abs(d + rho).max() <= 1e-7 * rho.max()
    # total mass of the column
    assert abs(m[0] - np.trapezoid(rho, y)) <= 1e-6 * m[0]


def test_rt_initial_state():
    cfg, U, meta = W.rt2d(32)
    assert cfg["bc_lo"][1] == "reflect" and cfg["g"][1] == -1.0
    assert np.all(U[1] == 0.0) and np.all(U[2] == 0.0)
    P = (5.0 / 3.0 - 1.0) * U[3]
    assert np.allclose(P[:, 0], P[:, 5]) and P[0, 0] > P[-1, 0] > 1000.0
    # light below, heavy above, 1% perturbation along x
    assert U[0][0].mean() < 1.01 and U[0][-1].mean() > 9.9


def test_rt_strip_needs_a_face_at_one_eighth():
    """The Sec. 4.4 strip starts at x = 1/8, which is a cell face only when
    n is a multiple of 8; its grid is n/4 x n with mirror walls in x."""
    import pytest
    with pytest.raises(ValueError):
        W.rt2d(36, strip=True)
    cfg, U0, meta = W.rt2d(32, strip=True)
    assert cfg["n"][:2] == [8, 32] and U0.shape == (4, 32, 8)
    assert cfg["bc_lo"][0] == cfg["bc_hi"][0] == "reflect" and meta["x0"] == 0.125
