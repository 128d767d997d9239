"""The CFL step on the device (row a2: dt = C h / max c_tot over the cells of
U^n, cut at t_end), as the library forms it: each stage 2 records the largest
c_tot of the new state per workgroup, the next stage 1 reduces those maxima,
and rsst_get_time forms the next dt from them on the host.  Checked against
the oracle's CFL dt of the same state, after CFL steps, after fixed steps,
after a prime with a start time, and at an end time."""
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


CASES = [(1, [90]), (2, [70, 33]), (2, [256, 40]), (3, [37, 9, 8]), (3, [256, 6, 5])]


@pytest.mark.parametrize("ndim,n", CASES, ids=[f"{c[0]}d-{'x'.join(map(str, c[1]))}" for c in CASES])
def test_next_dt_is_the_cfl_dt_of_the_current_state(ndim, n):
    cfg, U0 = W.random_state(ndim, n, seed_k=900 + sum(n), xi=3.0, mach=0.3)
    print(f"[case] cfl {ndim}D {n}", flush=True)
    U = torch.from_numpy(U0.copy()).cuda()
    s = R.Solver(cfg)
    assert s.time() == (0.0, 0.0)  # no state recorded yet
    # a prime sets t and records the maxima of U
    s.prime(U, 0.25)
    t, dt = s.time()
    assert t == 0.25
    assert dt == pytest.approx(oracle.cfl_dt(cfg, U0), rel=1e-13)
    # fixed steps keep the recorded maxima current
    s.steps(U, 3, 1e-4)
    t, dt = s.time()
    Uf = U.cpu().numpy()
    assert t == pytest.approx(0.25 + 3e-4, rel=1e-15)
    assert dt == pytest.approx(oracle.cfl_dt(cfg, Uf), rel=1e-13)
    # a CFL step takes exactly that dt
    s.step(U)
    t2, dt2 = s.time()
    assert t2 == t + dt
    assert dt2 == pytest.approx(oracle.cfl_dt(cfg, U.cpu().numpy()), rel=1e-13)
    assert s.poll() == 0
    s.close()


@pytest.mark.parametrize("ndim,n", [(2, [64, 20]), (3, [40, 10, 7])])
def test_end_time_cuts_the_last_step_and_stops(ndim, n):
    """With t_end, the step that would pass it is cut to end there, the next
    dt is 0, and further steps leave U and t unchanged."""
    cfg, U0 = W.random_state(ndim, n, seed_k=920 + ndim, xi=3.0, mach=0.3)
    dt0 = oracle.cfl_dt(cfg, U0)
    t_end = 2.5 * dt0
    U = torch.from_numpy(U0.copy()).cuda()
    s = R.Solver(cfg, t_end=t_end)
    ts = []
    for _ in range(3):
        s.step(U)
        ts.append(s.time())
    assert ts[-1][0] == pytest.approx(t_end, rel=1e-14) and ts[-1][1] == 0.0
    assert ts[1][0] < t_end and ts[1][1] == pytest.approx(t_end - ts[1][0], rel=1e-12)
    Ue = U.cpu().numpy()
    s.steps(U, 4)
    assert np.array_equal(U.cpu().numpy(), Ue) and s.time() == ts[-1]
    s.close()
