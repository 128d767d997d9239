"""A 3D state past 4 GiB: 256 x 256 x 2048 cells in FP64 (5.4 GB; variable 4
starts 4.3 GB into the array), built as 256 copies along z of one random
periodic 256 x 256 x 8 block.  The step is translation invariant bit for bit,
so after two steps every copy equals the block's own two steps, which in turn
match the oracle (1e-12 of the natural scales).  A kernel that wrapped a
32-bit offset would read or write the wrong plane of the wrong variable in
the upper copies."""
import numpy as np
import pytest

import oracle
import workloads as W

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def test_state_past_4_gib():
    import paper_1812_04135_amd as R
    assert torch.cuda.is_available()
    R.lib()
    cfg, Ub = W.random_state(3, [256, 256, 8], seed_k=950, xi=4.0, mach=0.3)
    print("[case] large 256x256x2048 FP64 from a 256x256x8 block", flush=True)
    # the block on the GPU against the oracle
    U = torch.from_numpy(Ub.copy()).cuda()
    s = R.Solver(cfg)
    s.steps(U, 2)
    Ug = U.cpu().numpy()
    assert s.poll() == 0
    dblk = s.diag(U)
    s.close()
    Uo, _, _ = oracle.run(cfg, Ub, 2)
    scale = [np.abs(Uo[0]).max()] * 4 + [np.abs(Uo[4]).max()]
    err = max(float(np.abs(Ug[v] - Uo[v]).max() / scale[v]) for v in range(5))
    print(f"[parity] block err/scale {err:.2e}", flush=True)
    assert err <= 1e-12
    # the tiled state
    reps = 256
    big = dict(cfg, n=[256, 256, 8 * reps])
    Ut = torch.from_numpy(Ub).cuda().repeat(1, reps, 1, 1).contiguous()
    assert Ut.numel() * 8 > 4 * 2 ** 30
    s = R.Solver(big)
    s.steps(Ut, 2)
    torch.cuda.synchronize()
    assert s.poll() == 0
    # the diagnostics of the whole state: sums are reps times the block's
    # (to rounding of the summation order), maxima the block's exactly
    dbig = s.diag(Ut)
    s.close()
    for q in range(6):
        assert abs(dbig[q] - reps * dblk[q]) <= 1e-12 * max(abs(reps * dblk[q]), reps * abs(dblk[0])), (q, dbig[q], dblk[q])
    assert dbig[6] == dblk[6] and dbig[7] == dblk[7]
    ref = torch.from_numpy(Ug).cuda()
    copies = Ut.view(5, reps, 8, 256, 256)
    same = (copies == ref[:, None]).flatten(1).all(dim=1)
    print(f"[large] copies equal to the block per variable: {same.tolist()}", flush=True)
    assert bool(same.all())
    del Ut, copies
    torch.cuda.empty_cache()


def test_fp32_perturbation_state_past_4_gib():
    """The same check in the FP32 perturbation form: 256 x 256 x 4096 cells
    of FP32 perturbations (5.4 GB) about a uniform FP64 background, 512
    copies of one 8-plane block; the block itself against the FP64 oracle
    at the FP32 bar (1e-5 of the perturbation)."""
    import paper_1812_04135_amd as R
    assert torch.cuda.is_available()
    R.lib()
    cfg, Ub = W.random_state(3, [256, 256, 8], seed_k=951, xi=4.0, mach=0.3)
    bg = np.ascontiguousarray(Ub.reshape(5, -1).mean(axis=1)[:, None])  # [nv][1]
    U1 = (Ub - bg[:, :, None, None]).astype(np.float32)
    Ustart = bg[:, :, None, None] + U1.astype(np.float64)
    print("[case] large FP32 256x256x4096 from a 256x256x8 block", flush=True)
    bgt = torch.from_numpy(bg).cuda()
    U = torch.from_numpy(U1.copy()).cuda()
    s = R.Solver(cfg, prec="fp32_pert", bg=bgt, bg_axis=-1)
    s.steps(U, 2)
    Ug = U.cpu().numpy()
    assert s.poll() == 0
    s.close()
    Uo, _, _ = oracle.run(cfg, Ustart, 2)
    pert = Uo - bg[:, :, None, None]
    sc = [np.abs(pert[v]).max() for v in range(5)]
    sc = [sc[0]] + [max(sc[1:4])] * 3 + [sc[4]]
    err = max(float(np.abs(Ug[v].astype(np.float64) - pert[v]).max() / sc[v]) for v in range(5))
    print(f"[parity] FP32 block err/|pert| {err:.2e}", flush=True)
    assert err <= 1e-5
    reps = 512
    big = dict(cfg, n=[256, 256, 8 * reps])
    Ut = torch.from_numpy(U1).cuda().repeat(1, reps, 1, 1).contiguous()
    assert Ut.numel() * 4 > 4 * 2 ** 30
    s = R.Solver(big, prec="fp32_pert", bg=bgt, bg_axis=-1)
    s.steps(Ut, 2)
    torch.cuda.synchronize()
    assert s.poll() == 0
    s.close()
    ref = torch.from_numpy(Ug).cuda()
    same = (Ut.view(5, reps, 8, 256, 256) == ref[:, None]).flatten(1).all(dim=1)
    print(f"[large] FP32 copies equal to the block per variable: {same.tolist()}", flush=True)
    assert bool(same.all())
    del Ut
    torch.cuda.empty_cache()
