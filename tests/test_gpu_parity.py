"""GPU path (through the C ABI) against the CPU oracle, element by element.

Tolerance (FP64): per variable v, max|U_gpu - U_oracle| <= 1e-12 * s_v with
the natural scales s_rho = max|rho|, s_E = max|E| and s_m = max|rho| * max a
(momentum at Mach 1).  Two independently ordered FP64 codes (FMA contraction
on the GPU, none in the oracle) differ by rounding only; measured against a
momentum perturbation of 1e-4 that rounding random-walks to ~1e-11 over
hundreds of steps, which is why momentum is scaled by rho*a.

FP32 perturbation form: max|U1_gpu - (U_oracle - U0)| <= 1e-5 * s1 per
variable, the oracle run in FP64 from U0 + U1(t=0), with s1 = max|U_oracle - U0|
for rho and E, and for every momentum component the largest perturbation of
any component (momentum is one vector: FP32 rounding of its largest component
feeds absolute errors of that size into all of them).
"""
import math

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
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    lib.lib()  # must load the HIP library, no fallback
    R = lib


GAMMA = 5.0 / 3.0


def scales(U, ndim):
    rho = U[0]
    m2 = sum(U[1 + d] ** 2 for d in range(ndim))
    P = (GAMMA - 1) * (U[-1] - 0.5 * m2 / rho)
    a = np.sqrt(GAMMA * np.abs(P) / rho)
    srho = np.abs(rho).max()
    return [srho] + [srho * a.max()] * ndim + [np.abs(U[-1]).max()]


def parity_err(Ug, Uo, ndim):
    s = scales(Uo, ndim)
    return [float(np.abs(Ug[v] - Uo[v]).max() / s[v]) for v in range(ndim + 2)]


def assert_parity(Ug, Uo, ndim, tol=1e-12, what=""):
    err = parity_err(Ug, Uo, ndim)
    print(f"[parity] {what} err/scale per var = {['%.2e' % e for e in err]}", flush=True)
    assert max(err) <= tol, (what, err)


def pert_errors(Ug, Uo, bg, ndim):
    pert = Uo - bg
    s = [np.abs(pert[v]).max() for v in range(ndim + 2)]
    sm = max(s[1:1 + ndim])
    s = [s[0]] + [sm] * ndim + [s[-1]]
    return [float(np.abs(Ug[v].astype(np.float64) - pert[v]).max() / s[v])
            for v in range(ndim + 2)]


def gpu_run(cfg, U0, nsteps, dt_fixed=0.0, t_end=0.0, prec="fp64", bg=None, bg_axis=-1):
    U = torch.from_numpy(np.ascontiguousarray(U0)).cuda()
    bgt = torch.from_numpy(bg).cuda() if bg is not None else None
    sol = R.Solver(cfg, prec=prec, bg=bgt, bg_axis=bg_axis, t_end=t_end)
    sol.steps(U, nsteps, dt_fixed)
    torch.cuda.synchronize()
    t, dt = sol.time()
    flags = sol.poll()
    out = U.cpu().numpy()
    sol.close()
    return out, t, dt, flags


CASES = [
    # (ndim, n, bc_lo, g, form)
    (1, [37], ["periodic"], None, "pvs"),
    (1, [130], ["reflect"], [-0.3], "pms"),
    (1, [256], ["periodic"], None, "dvs"),
    (1, [64], ["reflect"], [0.5], "dms"),
    (1, [100], ["periodic"], None, "pd"),
    (1, [50], ["reflect"], None, "euler"),
    (2, [70, 45], ["periodic", "periodic"], None, "pvs"),
    (2, [37, 20], ["periodic", "reflect"], [0.0, -0.5], "pms"),
    (2, [64, 16], ["reflect", "periodic"], [0.2, 0.0], "dvs"),
    (2, [130, 12], ["reflect", "reflect"], [0.1, -0.4], "dms"),
    (2, [20, 33], ["periodic", "reflect"], [0.0, -1.0], "pd"),
    (2, [200, 8], ["periodic", "periodic"], None, "euler"),
    (2, [1024, 6], ["periodic", "reflect"], [0.0, -0.3], "pvs"),  # widest 2D row (16 waves)
    (3, [37, 13, 11], ["periodic"] * 3, None, "pvs"),
    (3, [20, 9, 10], ["periodic", "periodic", "reflect"], [0.0, 0.0, -1.0], "pvs"),
    (3, [130, 9, 6], ["reflect", "reflect", "periodic"], [0.3, -0.2, 0.0], "pms"),
    (3, [64, 8, 8], ["periodic", "reflect", "reflect"], [0.0, 0.4, -0.6], "dvs"),
    (3, [17, 6, 5], ["reflect", "periodic", "periodic"], None, "dms"),
    (3, [256, 4, 4], ["periodic"] * 3, [0.0, 0.0, -0.5], "pd"),
    (3, [40, 10, 7], ["reflect"] * 3, None, "euler"),
    (3, [300, 5, 6], ["periodic", "reflect", "reflect"], [0.0, 0.3, -0.5], "pvs"),  # 5 of 8 waves
    (3, [512, 4, 5], ["reflect", "periodic", "periodic"], None, "pms"),  # widest 3D row
    # rows of 64 m + 1 cells: the row's last cell is lane 0 of its last wave,
    # which forms both of its x faces
    (1, [65], ["periodic"], None, "pvs"),
    (1, [129], ["reflect"], [0.2], "pd"),
    (2, [65, 10], ["periodic", "reflect"], [0.0, -0.5], "pvs"),
    (2, [193, 6], ["reflect", "periodic"], None, "pms"),
    (3, [65, 6, 5], ["periodic", "periodic", "reflect"], [0.0, 0.0, -0.5], "pvs"),
    (3, [129, 5, 4], ["reflect", "periodic", "periodic"], None, "dvs"),
    (3, [257, 4, 4], ["periodic"] * 3, None, "pvs"),
    # 2D grids large enough for two planes per march iteration (rows of up to
    # eight waves, two-plane chunks giving 2048 waves): an odd row count (the
    # last chunk's second plane lies past the grid), 64 m + 1 cells, walls
    (2, [449, 515], ["periodic", "reflect"], [0.0, -0.5], "pvs"),
    (2, [512, 520], ["reflect", "periodic"], [0.3, 0.0], "dms"),
]


@pytest.mark.parametrize("ndim,n,bc,g,form", CASES,
                         ids=[f"{c[0]}d-{'x'.join(map(str, c[1]))}-{c[4]}-{c[2][0][0]}{c[2][-1][0]}"
                              for c in CASES])
def test_step_matches_oracle(ndim, n, bc, g, form):
    cfg, U0 = W.random_state(ndim, n, seed_k=200 + sum(n), xi=4.0, form=form, bc_lo=bc,
                             g=g, mach=0.3)
    nsteps = 6
    print(f"[case] {ndim}D n={n} bc={bc} form={form}", flush=True)
    Ug, tg, dtg, flags = gpu_run(cfg, U0, nsteps)
    Uo, to, dto = oracle.run(cfg, U0, nsteps)
    assert flags == 0
    assert abs(tg - to) <= 1e-13 * to
    assert_parity(Ug, Uo, ndim, what=f"{ndim}D {n} {form}")


@pytest.mark.parametrize("form", ["pvs", "pms", "dvs", "dms", "pd", "euler"])
def test_fixed_dt_and_xi_one(form):
    cfg, U0 = W.random_state(2, [48, 40], seed_k=300, xi=1.0 if form == "euler" else 7.0,
                             form=form, bc_lo=["periodic", "reflect"], g=[0.0, -0.7])
    Ug, tg, _, _ = gpu_run(cfg, U0, 5, dt_fixed=1e-3)
    Uo, to, _ = oracle.run(cfg, U0, 5, dt_fixed=1e-3)
    assert abs(tg - 5e-3) < 1e-15
    assert_parity(Ug, Uo, 2, what=f"fixed dt {form}")


def test_t_end_truncates_last_step():
    cfg, U0, meta = W.wave1d(xi=10.0, form="pvs")
    t_end = 0.05 * meta["t_end"]
    Ug, tg, _, _ = gpu_run(cfg, U0, 1000, t_end=t_end)
    Uo, to, _ = oracle.run(cfg, U0, 1000, t_end=t_end)
    assert tg == pytest.approx(t_end, rel=1e-14) and to == pytest.approx(t_end, rel=1e-14)
    assert_parity(Ug, Uo, 1, what="t_end")


def test_linear_wave_full_length():
    """1D periodic wave, 256 cells, xi = 10, to t = 2 reduced crossing times."""
    for xi in (1.0, 10.0):
        cfg, U0, meta = W.wave1d(xi=xi, form="pvs")
        Ug, tg, _, _ = gpu_run(cfg, U0, 100000, t_end=meta["t_end"])
        Uo, to, _ = oracle.run(cfg, U0, 100000, t_end=meta["t_end"])
        assert tg == pytest.approx(meta["t_end"], rel=1e-13)
        assert_parity(Ug, Uo, 1, what=f"wave1d xi={xi}")


def test_bubble2d_full_size_20_steps():
    cfg, U0, meta = W.bubble2d()
    Ug, tg, _, _ = gpu_run(cfg, U0, 20)
    Uo, to, _ = oracle.run(cfg, U0, 20)
    assert abs(tg - to) <= 1e-13 * to
    assert_parity(Ug, Uo, 2, what="bubble2d 512^2 x20")


def test_strat3d_full_size_one_step_from_evolved_state():
    """256^3 stratified box: evolve 5 steps on the GPU, then compare one more
    GPU step with one oracle step from the same state."""
    cfg, U0, meta = W.strat3d()
    U = torch.from_numpy(U0).cuda()
    sol = R.Solver(cfg)
    sol.steps(U, 5)
    torch.cuda.synchronize()
    Us = U.cpu().numpy()
    sol.step(U)
    torch.cuda.synchronize()
    t5 = sol.time()[0]
    Ug = U.cpu().numpy()
    sol.close()
    Uo, _, dto = oracle.run(cfg, Us, 1)
    assert_parity(Ug, Uo, 3, what="strat3d 256^3 one step")


@pytest.mark.parametrize("n,ny,nz", [(32, 16, 24), (300, 5, 8)])
def test_fp32_perturbation_matches_fp64_oracle_3d(n, ny, nz):
    cfg, U0, meta = W.strat3d(n=n, nz=nz, ny=ny, xi=30.0)
    bg = meta["bg"]
    U1 = (U0 - bg[:, :, None, None]).astype(np.float32)
    Ustart = bg[:, :, None, None] + U1.astype(np.float64)
    nsteps = 20
    Ug, tg, _, flags = gpu_run(cfg, U1, nsteps, prec="fp32_pert", bg=bg, bg_axis=2)
    Uo, to, _ = oracle.run(cfg, Ustart, nsteps)
    assert flags == 0
    assert abs(tg - to) <= 1e-6 * to
    err = pert_errors(Ug, Uo, bg[:, :, None, None], 3)
    print(f"[fp32 3d] err/|pert| per var = {['%.2e' % e for e in err]}", flush=True)
    assert max(err) <= 1e-5, err


def test_fp32_perturbation_matches_fp64_oracle_2d_uniform_bg():
    cfg, U0, meta = W.bubble2d(n=96, xi=20.0)
    bg = meta["bg"]
    U1 = (U0 - bg[:, :, None]).astype(np.float32)
    Ustart = bg[:, :, None] + U1.astype(np.float64)
    Ug, tg, _, _ = gpu_run(cfg, U1, 20, prec="fp32_pert", bg=bg, bg_axis=-1)
    Uo, to, _ = oracle.run(cfg, Ustart, 20)
    err = pert_errors(Ug, Uo, bg[:, :, None], 2)
    print(f"[fp32 2d] err/|pert| per var = {['%.2e' % e for e in err]}", flush=True)
    assert max(err) <= 1e-5, err


@pytest.mark.parametrize("ndim,n,axis,wall", [
    (3, [40, 12, 9], 0, None),        # background along x (per-lane profile)
    (3, [36, 22, 7], 1, None),        # along y: the stacked rows' own profile rows
    (3, [70, 9, 14], 1, "reflect"),   # along y, walls on every axis
    (2, [48, 30], 0, "reflect"),      # along x, with y walls
    (1, [90], 0, None),               # along the only axis
])
def test_fp32_perturbation_background_on_any_axis(ndim, n, axis, wall):
    """FP32 perturbation about a background that varies along x or y (the
    stratified box turned so that gravity and the walls lie on that axis),
    20 steps against the FP64 oracle run from U0 + U1(0), at 1e-5 of the
    perturbation."""
    cfg, U0, meta = W.stratified(ndim, n, axis, xi=20.0, seed_k=40 + axis + 3 * ndim, wall_bc=wall)
    bg = meta["bg"]
    bshape = [U0.shape[0]] + [1] * ndim
    bshape[ndim - axis] = n[axis]
    bgb = bg.reshape(bshape)
    U1 = (U0 - bgb).astype(np.float32)
    Ustart = bgb + U1.astype(np.float64)
    nsteps = 20
    print(f"[fp32 bg] {ndim}D n={n} bg_axis={axis} walls={wall}", flush=True)
    Ug, tg, _, flags = gpu_run(cfg, U1, nsteps, prec="fp32_pert", bg=bg, bg_axis=axis)
    Uo, to, _ = oracle.run(cfg, Ustart, nsteps)
    assert flags == 0
    assert abs(tg - to) <= 1e-6 * to
    err = pert_errors(Ug, Uo, bgb, ndim)
    print(f"[fp32 bg] err/|pert| per var = {['%.2e' % e for e in err]}", flush=True)
    assert max(err) <= 1e-5, err


# ------------------------------------------------------------ invariants

def test_uniform_state_bitwise_3d():
    n = [40, 9, 11]
    cfg = W.base_cfg(3, n, xi=5.0, form="pvs")
    shape = tuple(reversed(n))
    U0 = W.conservative(np.full(shape, 1.2), [np.full(shape, 0.1), np.full(shape, -0.05),
                                               np.full(shape, 0.02)], np.full(shape, 0.8))
    Ug, _, _, _ = gpu_run(cfg, U0, 10)
    assert np.array_equal(Ug, U0)


@pytest.mark.parametrize("n,shift", [([100, 14, 12], (5, 3, 37)), ([256, 9, 6], (2, 1, 0)),
                                     ([64, 13, 5], (1, 5, 3)), ([192, 7, 5], (3, 2, 70)),
                                     ([320, 5, 4], (1, 2, 131))])
def test_translation_invariance_bitwise(n, shift):
    """A periodic shift that is not a multiple of any tile or wave moves the
    result bit for bit (tile seams and halos compute the same numbers).  The
    y heights are not multiples of the tile heights (2, 4, 8 rows), so the
    last tile of each column overlaps the one before it, and the rows it
    computes without storing land on rows that another tile stores after the
    shift."""
    cfg, U0 = W.random_state(3, n, seed_k=400 + n[0], xi=3.0)
    print(f"[case] translation {n} shift {shift}", flush=True)
    Ua, _, _, _ = gpu_run(cfg, U0, 3)
    Us = np.ascontiguousarray(np.roll(U0, shift=shift, axis=(1, 2, 3)))
    Ub, _, _, _ = gpu_run(cfg, Us, 3)
    assert np.array_equal(np.roll(Ua, shift=shift, axis=(1, 2, 3)), Ub)


@pytest.mark.parametrize("ndim,n,g", [(2, [96, 40], [0.0, -0.5]), (3, [70, 9, 21], [0.0, 0.0, -0.7])])
def test_chunk_length_changes_no_bit(ndim, n, g, monkeypatch):
    """The march along the last axis is cut into chunks (each starting from
    four re-read planes); the planner's chunk length (RSST_KM, read when a
    solver is made) changes no bit of the result: 1, 2, 3, 8 planes and the
    default, with walls and gravity along the marched axis."""
    bc = ["periodic"] * (ndim - 1) + ["reflect"]
    cfg, U0 = W.random_state(ndim, n, seed_k=410 + ndim, xi=3.0, bc_lo=bc, g=g, mach=0.3)
    ref = None
    for km in (None, "1", "2", "3", "8"):
        if km is None:
            monkeypatch.delenv("RSST_KM", raising=False)
        else:
            monkeypatch.setenv("RSST_KM", km)
        Ug, tg, _, flags = gpu_run(cfg, U0, 4)
        assert flags == 0
        if ref is None:
            ref = (Ug, tg)
        else:
            assert np.array_equal(Ug, ref[0]) and tg == ref[1], (km, np.abs(Ug - ref[0]).max())
    monkeypatch.delenv("RSST_KM", raising=False)


@pytest.mark.parametrize("form", ["dvs", "pd", "euler"])
def test_mass_conservation_on_gpu(form):
    cfg, U0 = W.random_state(2, [96, 64], seed_k=401, xi=4.0 if form != "euler" else 1.0,
                             form=form)
    U = torch.from_numpy(U0).cuda()
    sol = R.Solver(cfg)
    m0 = sol.diag(U)[0]
    sol.steps(U, 50)
    m1 = sol.diag(U)[0]
    sol.close()
    assert abs(m1 - m0) <= 1e-13 * abs(m0)


def test_diag_matches_oracle():
    cfg, U0 = W.random_state(3, [40, 12, 10], seed_k=402, xi=6.0)
    U = torch.from_numpy(U0).cuda()
    sol = R.Solver(cfg)
    d = sol.diag(U)
    sol.close()
    do = oracle.diag(cfg, U0)
    np.testing.assert_allclose(d, do, rtol=1e-13, atol=1e-15)


def test_nonphysical_state_is_latched_and_polled():
    cfg, U0 = W.random_state(2, [32, 16], seed_k=403)
    U0 = U0.copy()
    U0[0, 5, 7] = float("nan")
    U = torch.from_numpy(U0).cuda()
    sol = R.Solver(cfg)
    sol.step(U, dt_fixed=1e-4)
    with pytest.raises(R.RsstError) as e:
        sol.poll()
    assert e.value.code == -5
    assert sol.poll() == 0  # cleared
    sol.close()


# xi from the sound speed (eq. cx): C_max near the median sound speed, so
# xi varies from ~1 to ~2 across each state; every dimension, every form, a
# 256-wide 3D row, walls and gravity.
CMAX_CASES = [
    (1, [90], ["reflect"], [-0.3], "pvs"),
    (1, [64], ["periodic"], None, "pd"),
    (2, [70, 33], ["periodic", "reflect"], [0.0, -0.5], "pvs"),
    (2, [37, 20], ["reflect", "periodic"], [0.2, 0.0], "pms"),
    (2, [64, 16], ["periodic", "periodic"], None, "dvs"),
    (2, [33, 18], ["reflect", "reflect"], [0.1, -0.4], "dms"),
    (2, [20, 33], ["periodic", "reflect"], [0.0, -1.0], "pd"),
    (3, [37, 9, 8], ["periodic", "periodic", "reflect"], [0.0, 0.0, -1.0], "pvs"),
    (3, [256, 4, 5], ["periodic", "reflect", "reflect"], [0.0, 0.3, -0.6], "pms"),
]


@pytest.mark.parametrize("ndim,n,bc,g,form", CMAX_CASES,
                         ids=[f"{c[0]}d-{'x'.join(map(str, c[1]))}-{c[4]}" for c in CMAX_CASES])
def test_cmax_step_matches_oracle(ndim, n, bc, g, form):
    cfg, U0 = W.random_state(ndim, n, seed_k=260 + sum(n), xi=4.0, form=form, bc_lo=bc, g=g, mach=0.3)
    rho = U0[0]
    m2 = sum(U0[1 + d] ** 2 for d in range(ndim))
    a = np.sqrt(GAMMA * (GAMMA - 1) * (U0[-1] - 0.5 * m2 / rho) / rho)
    cfg["cmax"] = float(np.median(a))
    nsteps = 6
    Ug, tg, dtg, flags = gpu_run(cfg, U0, nsteps)
    Uo, to, dto = oracle.run(cfg, U0, nsteps)
    assert flags == 0
    assert abs(tg - to) <= 1e-13 * to
    assert_parity(Ug, Uo, ndim, what=f"cmax {ndim}D {n} {form}")
    # the mode is live: the run differs from the constant-xi run
    Uc, _, _, _ = gpu_run(dict(cfg, cmax=0.0), U0, nsteps)
    assert np.abs(Uc - Ug).max() > 1e-8


def test_cmax_fp32_perturbation_and_diag():
    cfg, U0, meta = W.strat3d(n=32, xi=30.0, nz=24, ny=8)
    cfg["cmax"] = 0.25  # below the sound speed of the lower half of the box
    nsteps = 4
    bg = meta["bg"]
    U1 = (U0 - bg[:, :, None, None]).astype(np.float32)
    Ug, _, _, _ = gpu_run(cfg, U1, nsteps, prec="fp32_pert", bg=bg, bg_axis=2)
    Uo, _, _ = oracle.run(cfg, bg[:, :, None, None] + U1.astype(np.float64), nsteps)
    err = pert_errors(Ug, Uo, bg[:, :, None, None], 3)
    print(f"[parity] cmax fp32 err/pert = {err}", flush=True)
    assert max(err) <= 1e-5
    U = torch.from_numpy(U0).cuda()
    s = R.Solver(cfg)
    d = s.diag(U)
    s.close()
    do = oracle.diag(cfg, U0)
    assert abs(d[7] - do[7]) <= 1e-13 * do[7]
