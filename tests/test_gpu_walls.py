"""Hydrostatic closed walls on the GPU against the oracle (the FP64 bar of the
other parity tests): walls on the march axis and on the stacked-row axis with
gravity along them, x walls without a force along x, every form, with the
C_max law and the van der Waals gas, and the Sec. 4.4 Rayleigh-Taylor layer."""
import numpy as np
import pytest

import oracle
import workloads as W

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

R = None


def setup_module(module):
    global R
    import paper_1812_04135_amd as lib
    assert torch.cuda.is_available()
    lib.lib()
    R = lib


def _err(Ug, Uo, ndim):
    rho = Uo[0]
    srho = np.abs(rho).max()
    vmax = max(np.abs(Uo[1 + d] / rho).max() for d in range(ndim))
    s = [srho] + [srho * max(1.0, vmax)] * ndim + [np.abs(Uo[-1]).max()]
    return [float(np.abs(Ug[v] - Uo[v]).max() / s[v]) for v in range(ndim + 2)]


def _gpu(cfg, U0, nsteps):
    U = torch.from_numpy(np.ascontiguousarray(U0)).cuda()
    s = R.Solver(cfg)
    s.steps(U, nsteps)
    torch.cuda.synchronize()
    t, _ = s.time()
    flags = s.poll()
    s.close()
    return U.cpu().numpy(), t, flags


CASES = [
    (2, [70, 33], ["periodic", "hydro"], [0.0, -0.6], "pvs", None),
    (2, [37, 20], ["hydro", "hydro"], [0.0, -0.4], "pms", None),
    (2, [64, 16], ["reflect", "hydro"], [0.0, 0.5], "dvs", "vdw"),
    (2, [33, 18], ["periodic", "hydro"], [0.0, -1.0], "pd", "cmax"),
    (3, [37, 9, 8], ["periodic", "periodic", "hydro"], [0.0, 0.0, -1.0], "pvs", None),
    (3, [40, 10, 7], ["hydro", "hydro", "hydro"], [0.0, 0.3, -0.6], "dms", None),
    (3, [130, 9, 6], ["periodic", "hydro", "periodic"], [0.0, -0.5, 0.0], "euler", "vdw"),
    (3, [256, 5, 9], ["periodic", "hydro", "hydro"], [0.0, 0.2, -0.7], "pms", "cmax"),
]


@pytest.mark.parametrize("ndim,n,bc,g,form,extra", CASES,
                         ids=[f"{c[0]}d-{'x'.join(map(str, c[1]))}-{c[4]}-{c[5]}" for c in CASES])
def test_hydro_walls_match_oracle(ndim, n, bc, g, form, extra):
    gas = W.VDW if extra == "vdw" else None
    cfg, U0 = W.random_state(ndim, n, seed_k=780 + sum(n), xi=4.0, form=form, bc_lo=bc, g=g, mach=0.3,
                             gas=gas)
    if extra == "cmax":
        cfg["cmax"] = 1.0
    print(f"[case] hydro {ndim}D n={n} bc={bc} form={form} {extra}", flush=True)
    Ug, tg, flags = _gpu(cfg, U0, 6)
    Uo, to, _ = oracle.run(cfg, U0, 6)
    assert flags == 0 and abs(tg - to) <= 1e-13 * to
    err = _err(Ug, Uo, ndim)
    print(f"[parity] hydro err/scale {['%.2e' % e for e in err]}", flush=True)
    assert max(err) <= 1e-12, err
    # the wall is live: the mirror wall gives another state
    mirror = [b if b != "hydro" else "reflect" for b in bc]
    Um, _, _ = _gpu(dict(cfg, bc_lo=mirror, bc_hi=mirror), U0, 6)
    assert np.abs(Um - Ug).max() > 1e-10


@pytest.mark.parametrize("xi", [1.0, 6.3])
def test_rt_with_hydro_walls_matches_oracle(xi):
    """The Sec. 4.4 layer at 64^2 with hydrostatic walls in y, 150 CFL steps;
    the bar is that of the Rayleigh-Taylor parity test (1e-12, or ten times
    the oracle's own spread under a last-bit change of the input)."""
    cfg, U0, _ = W.rt2d(64, form="pvs", xi=xi)
    cfg = dict(cfg, bc_lo=["periodic", "hydro"], bc_hi=["periodic", "hydro"])
    Ug, tg, flags = _gpu(cfg, U0, 150)
    Uo, to, _ = oracle.run(cfg, U0, 150)
    rng = np.random.default_rng(W.seed(82))
    Up, _, _ = oracle.run(cfg, U0 * (1 + 2.2e-16 * rng.choice([-1.0, 1.0], size=U0.shape)), 150)
    err, spread = _err(Ug, Uo, 2), _err(Up, Uo, 2)
    print(f"[rt-hydro] xi={xi} err/scale={err} spread={spread}", flush=True)
    assert flags == 0 and abs(tg - to) <= 1e-12 * to
    for v in range(4):
        assert err[v] <= max(1e-12, 10 * spread[v]), (v, err[v], spread[v])
