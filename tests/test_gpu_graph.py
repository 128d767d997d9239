"""rsst_step / rsst_steps captured in a HIP graph (torch.cuda.graph) and
replayed several times, with eager work and synchronisations between the
replays, give bitwise the state, time and dt of the same steps run eagerly:
CFL steps (device-side dt and its reduction counters) and fixed steps, in
1D (one launch for all steps), 2D and 3D."""
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


@pytest.mark.parametrize("ndim,n", [(1, [128]), (2, [70, 33]), (3, [37, 9, 8])])
@pytest.mark.parametrize("dt_fixed", [0.0, 2e-4])
def test_graph_replays_equal_eager_steps(ndim, n, dt_fixed):
    cfg, U0 = W.random_state(ndim, n, seed_k=790 + ndim, xi=4.0, form="pvs",
                             bc_lo=["periodic"] * (ndim - 1) + ["reflect"],
                             g=[0.0] * (ndim - 1) + [-0.5])
    nrep, G = 4, 5
    # eager reference: G * nrep steps, one call each
    Ue = torch.from_numpy(U0.copy()).cuda()
    se = R.Solver(cfg)
    ref = []
    for _ in range(nrep):
        for _ in range(G):
            se.step(Ue, dt_fixed)
        torch.cuda.synchronize()
        ref.append((Ue.cpu().numpy(), se.time()))
    se.close()
    # graph: prime outside the capture (first CFL dt), capture G steps, replay
    U = torch.from_numpy(U0.copy()).cuda()
    s = R.Solver(cfg)
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        if dt_fixed == 0.0:
            s.prime(U, 0.0, stream=side)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g, stream=side):
        if ndim == 1:
            s.steps(U, G, dt_fixed, stream=torch.cuda.current_stream())
        else:
            for _ in range(G):
                s.step(U, dt_fixed, stream=torch.cuda.current_stream())
    torch.cuda.synchronize()
    for r in range(nrep):
        g.replay()
        torch.cuda.synchronize()
        _ = (U * 2.0).sum().item()  # eager work between replays
        Ug = U.cpu().numpy()
        tg = s.time()
        assert np.array_equal(Ug, ref[r][0]), (r, np.abs(Ug - ref[r][0]).max())
        assert tg == ref[r][1], (r, tg, ref[r][1])
    s.close()
