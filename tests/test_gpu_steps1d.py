"""rsst_steps on a 1D grid runs every step in one launch; its state, time and
next dt must be bitwise those of the same steps taken one rsst_step call at a
time (two stage launches each), for every form, boundary, storage type, the
C_max law and the van der Waals gas, with CFL or fixed steps and an end time."""
import numpy as np
import pytest

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


def _both(cfg, U0, nsteps, dt_fixed=0.0, t_end=0.0, prec="fp64", bg=None, bg_axis=-1, per_step=None):
    """(U, t, dt) after rsst_steps(nsteps) and after per_step single steps."""
    out = []
    bgt = torch.from_numpy(bg).cuda() if bg is not None else None
    for mode in ("steps", "step"):
        U = torch.from_numpy(np.ascontiguousarray(U0)).cuda()
        s = R.Solver(cfg, prec=prec, bg=bgt, bg_axis=bg_axis, t_end=t_end)
        if mode == "steps":
            s.steps(U, nsteps, dt_fixed)
        else:
            for _ in range(per_step if per_step is not None else nsteps):
                s.step(U, dt_fixed)
        torch.cuda.synchronize()
        t, dt = s.time()
        flags = s.poll()
        out.append((U.cpu().numpy(), t, dt, flags))
        s.close()
    return out


def _assert_same(a, b, what):
    (Ua, ta, dta, fa), (Ub, tb, dtb, fb) = a, b
    print(f"[steps1d] {what} t={ta} dt={dta}", flush=True)
    assert fa == fb == 0
    assert np.array_equal(Ua, Ub), (what, np.abs(Ua - Ub).max())
    assert ta == tb and dta == dtb, (what, ta, tb, dta, dtb)


CASES = [
    (70, "periodic", None, "pvs"),
    (90, "reflect", [-0.3], "pms"),
    (64, "periodic", None, "dvs"),
    (130, "reflect", [0.4], "dms"),
    (256, "periodic", None, "pd"),
    (37, "reflect", [-1.0], "euler"),
    (1024, "periodic", [0.2], "pvs"),
]


@pytest.mark.parametrize("n,bc,g,form", CASES, ids=[f"{c[0]}-{c[1]}-{c[3]}" for c in CASES])
def test_steps_equal_single_steps(n, bc, g, form):
    cfg, U0 = W.random_state(1, [n], seed_k=700 + n, xi=5.0, form=form, bc_lo=[bc], g=g, mach=0.3)
    a, b = _both(cfg, U0, 40)
    _assert_same(a, b, f"cfl {n} {bc} {form}")
    a, b = _both(cfg, U0, 25, dt_fixed=2e-4)
    _assert_same(a, b, f"fixed {n} {bc} {form}")


def test_wave_to_end_time_skips_no_op_steps():
    cfg, U0, meta = W.wave1d(xi=10.0, form="pvs")
    a, b = _both(cfg, U0, 100000, t_end=meta["t_end"], per_step=1400)
    _assert_same(a, b, "wave1d to t_end")
    assert a[1] == meta["t_end"] and a[2] == 0.0


def test_cmax_vdw_and_fp32_perturbation():
    cfg, U0 = W.random_state(1, [200], seed_k=720, xi=4.0, form="pvs", bc_lo=["reflect"], g=[-0.5])
    rho = U0[0]
    P = (W.GAMMA - 1) * (U0[2] - 0.5 * U0[1] ** 2 / rho)
    a, b = _both(dict(cfg, cmax=float(np.median(np.sqrt(W.GAMMA * P / rho)))), U0, 30)
    _assert_same(a, b, "cmax")
    cfgv, Uv = W.random_state(1, [200], seed_k=721, xi=4.0, form="pd", gas=W.VDW)
    a, b = _both(cfgv, Uv, 30)
    _assert_same(a, b, "vdw")
    cfgw, Uw, meta = W.wave1d(xi=10.0, form="pms")
    bg = np.ascontiguousarray(np.array([[1.0], [0.0], [1.0 / (W.GAMMA - 1)]]))
    U1 = (Uw - bg).astype(np.float32)
    a, b = _both(cfgw, U1, 60, prec="fp32_pert", bg=bg, bg_axis=-1)
    _assert_same(a, b, "fp32 perturbation")


def test_steps_then_step_continue_the_same_run():
    cfg, U0 = W.random_state(1, [128], seed_k=730, xi=3.0, form="pvs")
    U = torch.from_numpy(U0.copy()).cuda()
    s = R.Solver(cfg)
    s.steps(U, 7)
    s.step(U)
    s.steps(U, 5, 1e-4)
    s.steps(U, 3)
    torch.cuda.synchronize()
    ta, dta = s.time()
    Ua = U.cpu().numpy()
    s.close()
    U = torch.from_numpy(U0.copy()).cuda()
    s = R.Solver(cfg)
    for dt in [0.0] * 8 + [1e-4] * 5 + [0.0] * 3:
        s.step(U, dt)
    torch.cuda.synchronize()
    tb, dtb = s.time()
    Ub = U.cpu().numpy()
    s.close()
    assert np.array_equal(Ua, Ub) and ta == tb and dta == dtb


def test_nonphysical_state_flagged_in_one_launch():
    cfg, U0 = W.random_state(1, [64], seed_k=740, xi=3.0)
    U0 = U0.copy()
    U0[0, 10] = -1.0
    U = torch.from_numpy(U0).cuda()
    s = R.Solver(cfg)
    s.steps(U, 3, 1e-4)
    torch.cuda.synchronize()
    with pytest.raises(R.RsstError) as e:
        s.poll()
    assert e.value.flags & 1
    s.close()


@pytest.mark.parametrize("ndim,n", [(1, [64]), (2, [40, 12]), (3, [37, 9, 8])])
def test_zero_steps_and_steps_past_end_time_change_nothing(ndim, n):
    """nsteps = 0 leaves U, t and dt as they are; after t reaches t_end the
    remaining steps are no-ops (dt = 0), in every dimension."""
    cfg, U0 = W.random_state(ndim, n, seed_k=750 + ndim, xi=3.0)
    U = torch.from_numpy(U0.copy()).cuda()
    s = R.Solver(cfg, t_end=0.01)
    s.steps(U, 0)
    torch.cuda.synchronize()
    assert np.array_equal(U.cpu().numpy(), U0) and s.time()[0] == 0.0
    s.steps(U, 100000 if ndim == 1 else 400)
    t, dt = s.time()
    assert t == pytest.approx(0.01, rel=1e-14) and dt == 0.0
    Ue = U.cpu().numpy()
    s.steps(U, 5)
    s.step(U)
    torch.cuda.synchronize()
    assert np.array_equal(U.cpu().numpy(), Ue) and s.time() == (t, 0.0)
    s.close()
