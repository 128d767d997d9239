"""rsst_step_noalloc (the step that allocates nothing: its scratch is a
fixed device array of the library) against rsst_step on a fresh handle,
through the C ABI: two calls in a row on one device, the second with a
smaller state, each bitwise equal to the handle's step (the same kernels)."""
import numpy as np
import pytest

import workloads as W

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

R = None


def setup_module(module):
    global R
    import paper_1812_04135_amd as lib
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    lib.lib()
    R = lib


def _handle_step(cfg, U0, dt_fixed, prec="fp64", bg=None, bg_axis=-1):
    U = torch.from_numpy(np.ascontiguousarray(U0)).cuda()
    s = R.Solver(cfg, prec=prec, bg=bg, bg_axis=bg_axis)
    s.step(U, dt_fixed)
    torch.cuda.synchronize()
    flags = s.poll()
    out = U.cpu().numpy()
    s.close()
    return out, flags


def _noalloc_step(cfg, U0, dt_fixed, prec="fp64", bg=None, bg_axis=-1):
    U = torch.from_numpy(np.ascontiguousarray(U0)).cuda()
    f = torch.full((1,), 7, dtype=torch.int32, device="cuda")
    c = R.make_config(cfg, prec=prec, bg=bg, bg_axis=bg_axis)
    R.rsst_step_noalloc(c, U, dt_fixed, f)
    torch.cuda.synchronize()
    return U.cpu().numpy(), int(f.item())


CASES = [
    # the first state of each pair is the larger one
    ((3, [64, 40, 33], ["periodic", "periodic", "reflect"], [0.0, 0.0, -0.5], "pvs", 0.0),
     (2, [70, 45], ["periodic", "reflect"], [0.0, -0.5], "pms", 0.0)),
    ((2, [512, 300], ["reflect", "periodic"], None, "dvs", 0.0),
     (1, [65], ["periodic"], None, "pd", 2e-3)),
    ((2, [256, 256], ["periodic", "periodic"], None, "pvs", 1e-3),
     (3, [37, 13, 11], ["periodic"] * 3, None, "euler", 0.0)),
]


@pytest.mark.parametrize("first,second", CASES, ids=["3d-then-2d", "2d-then-1d", "fixeddt-then-3d"])
def test_noalloc_equals_handle_step_twice(first, second):
    for q, (ndim, n, bc, g, form, dt) in enumerate((first, second)):
        cfg, U0 = W.random_state(ndim, n, seed_k=960 + q + sum(n), xi=4.0, form=form, bc_lo=bc, g=g)
        print(f"[noalloc] call {q}: {ndim}D n={n} form={form} dt={dt}", flush=True)
        Uh, fh = _handle_step(cfg, U0, dt)
        Un, fn = _noalloc_step(cfg, U0, dt)
        assert fh == 0 and fn == 0, (fh, fn)
        assert np.array_equal(Un, Uh), float(np.abs(Un - Uh).max())
        assert not np.array_equal(Un, U0)


def test_noalloc_fp32_perturbation_and_too_large():
    cfg, U0, meta = W.strat3d(n=32, xi=30.0, form="pvs")
    bg = torch.from_numpy(meta["bg"]).cuda()
    U1 = (U0 - meta["bg"][:, :, None, None]).astype(np.float32)
    Uh, fh = _handle_step(cfg, U1, 0.0, prec="fp32_pert", bg=bg, bg_axis=2)
    Un, fn = _noalloc_step(cfg, U1, 0.0, prec="fp32_pert", bg=bg, bg_axis=2)
    assert fh == 0 and fn == 0
    assert np.array_equal(Un, Uh)
    # a 3D 128^3 FP64 state needs 80 MiB of scratch: rejected on the host
    big, Ub = W.random_state(3, [8, 8, 8])
    c = R.make_config(big)
    for d in range(3):
        c.n[d] = 128
    U = torch.zeros(5 * 128 ** 3, dtype=torch.float64, device="cuda")
    with pytest.raises(R.RsstError) as e:
        R.rsst_step_noalloc(c, U, 0.0)
    assert e.value.code == R.RSST_E_SCRATCH
