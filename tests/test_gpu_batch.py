"""Batched boxes (one persistent launch per run, HIP graph) against
single-box runs of the same library and against the CPU oracle.

Every box of a batch must equal, bit for bit, the same box advanced alone by
rsst_step (same kernels, per-box CFL dt), and the oracle within the
tolerances of test_gpu_parity (FP64: 1e-12 of the natural scales; FP32
perturbation: 1e-5 of the perturbation)."""
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


def _boxes_fp64():
    """Box widths of one to four waves per row, ragged rows and strips, walls
    and periodic y (whose stencil wraps the first strip block onto the last:
    200 x 33 has a one-row last block at 16-row strips)."""
    out = []
    specs = [(16, 12, 3.0, "reflect"), (70, 33, 1.0, "reflect"), (130, 40, 12.0, "periodic"),
             (200, 24, 30.0, "reflect"), (64, 64, 5.0, "periodic"), (37, 9, 2.0, "periodic"),
             (200, 33, 8.0, "periodic"),
             # rows of 64 m + 1 cells (the last cell is lane 0 of the last wave)
             (65, 20, 4.0, "reflect"), (193, 14, 6.0, "periodic")]
    for q, (nx, ny, xi, ybc) in enumerate(specs):
        g = [0.0, -0.5] if ybc == "reflect" else [0.0, 0.0]
        cfg, U = W.random_state(2, [nx, ny], seed_k=500 + q, xi=xi, form="pvs",
                                bc_lo=["periodic", ybc], g=g)
        out.append((cfg, U))
    return out


def _single(cfg, U0, nsteps, prec="fp64", bg=None):
    U = torch.from_numpy(np.ascontiguousarray(U0)).cuda()
    bgt = torch.from_numpy(bg).cuda() if bg is not None else None
    s = R.Solver(cfg, prec=prec, bg=bgt, bg_axis=1 if bg is not None else -1)
    s.steps(U, nsteps)
    torch.cuda.synchronize()
    t = s.time()[0]
    out = U.cpu().numpy()
    s.close()
    return out, t


@pytest.mark.parametrize("tiles", [[16, 16, 16, 16], [8, 24, 32, 8]])
def test_batch_fp64_equals_single_box_runs_and_oracle(tiles):
    boxes = _boxes_fp64()
    nsteps = 7
    B = R.Batch([c for c, _ in boxes], max_steps=16)
    B.set_tiles(tiles)
    U = B.pack([u for _, u in boxes])
    B.run(U, nsteps)
    torch.cuda.synchronize()
    assert B.poll() == 0
    outs = B.unpack(U)
    times = B.times()
    for q, ((cfg, U0), Ub) in enumerate(zip(boxes, outs)):
        Us, ts = _single(cfg, U0, nsteps)
        print(f"[batch] box {q} {cfg['n'][:2]} xi={cfg['xi']} max|batch-single|="
              f"{np.abs(Ub - Us).max():.3e} t={times[q]:.6e}/{ts:.6e}", flush=True)
        assert np.array_equal(Ub, Us), q
        assert times[q] == ts
        Uo, to, _ = oracle.run(cfg, U0, nsteps)
        rho = Uo[0]
        P = (5 / 3 - 1) * (Uo[3] - 0.5 * (Uo[1] ** 2 + Uo[2] ** 2) / rho)
        a = np.sqrt(5 / 3 * P / rho).max()
        sc = [np.abs(rho).max(), np.abs(rho).max() * a, np.abs(rho).max() * a, np.abs(Uo[3]).max()]
        err = max(float(np.abs(Ub[v] - Uo[v]).max() / sc[v]) for v in range(4))
        assert err <= 1e-12, (q, err)
        assert abs(times[q] - to) <= 1e-13 * to


def test_batch_replay_and_second_run_continue():
    """A second run replays the captured graph and continues from the state
    and time the first left."""
    boxes = _boxes_fp64()[:3]
    B = R.Batch([c for c, _ in boxes], max_steps=8)
    U = B.pack([u for _, u in boxes])
    B.run(U, 3)
    B.run(U, 3)
    torch.cuda.synchronize()
    outs = B.unpack(U)
    times = B.times()
    for q, ((cfg, U0), Ub) in enumerate(zip(boxes, outs)):
        Us, ts = _single(cfg, U0, 6)
        assert np.array_equal(Ub, Us), q
        assert abs(times[q] - ts) <= 1e-14 * ts


def test_batch_fp32_perturbation_stratified_boxes():
    rng = np.random.default_rng(W.seed(600))
    boxes = []
    for q, (n, contrast, xi) in enumerate([(64, 3.0, 1.5), (100, 30.0, 10.0), (160, 100.0, 40.0),
                                           (256, 10.0, 5.0)]):
        cfg, U, meta = W.strat2d_box(n, contrast, xi, rng)
        boxes.append((cfg, U, meta["bg"]))
    nsteps = 6
    bgs = [bg for _, _, bg in boxes]
    B = R.Batch([c for c, _, _ in boxes], prec="fp32_pert", bgs=bgs, max_steps=8)
    U1s = [(U - bg[:, :, None]).astype(np.float32) for _, U, bg in boxes]
    U = B.pack(U1s)
    B.run(U, nsteps)
    torch.cuda.synchronize()
    outs = B.unpack(U)
    for q, ((cfg, U0, bg), u1, Ub) in enumerate(zip(boxes, U1s, outs)):
        Us, _ = _single(cfg, u1, nsteps, prec="fp32_pert", bg=bg)
        assert np.array_equal(Ub, Us), q
        Ustart = bg[:, :, None] + u1.astype(np.float64)
        Uo, _, _ = oracle.run(cfg, Ustart, nsteps)
        pert = Uo - bg[:, :, None]
        s = [np.abs(pert[v]).max() for v in range(4)]
        sm = max(s[1:3])
        s = [s[0], sm, sm, s[3]]
        err = max(float(np.abs(Ub[v].astype(np.float64) - pert[v]).max() / s[v]) for v in range(4))
        print(f"[batch fp32] box {q} n={cfg['n'][0]} err/|pert| = {err:.2e}", flush=True)
        assert err <= 1e-5, (q, err)


def test_autotuner_sets_tiles_caches_and_keeps_results(tmp_path):
    """The tuner leaves the caller's state untouched, writes its choice to the
    JSON cache, reuses it on the next call, and the tuned run gives the same
    bits as the default tiles (results do not depend on the strip rows)."""
    from paper_1812_04135_amd import autotune
    boxes = _boxes_fp64()
    cache = str(tmp_path / "tiles.json")
    B = R.Batch([c for c, _ in boxes], max_steps=8)
    U0 = B.pack([u for _, u in boxes])
    U = U0.clone()
    tiles, ms, cached = B.autotune(U, nsteps=4, candidates=(8, 16, 32), reps=1, cache=cache)
    assert not cached and ms > 0
    assert torch.equal(U, U0)
    assert B.tiles() == tiles
    # the tuning runs (on a scratch copy) leave the per-box times and flags as they were
    assert np.all(B.times() == 0.0)
    assert B.poll() == 0
    import json
    db = json.load(open(cache))
    assert db[autotune.batch_key(B)]["strip_rows"] == tiles
    B.set_tiles([16, 16, 16, 16])
    tiles2, _, cached2 = B.autotune(U, cache=cache)
    assert cached2 and tiles2 == tiles and B.tiles() == tiles
    B.run(U, 5)
    torch.cuda.synchronize()
    outs = B.unpack(U)
    times = B.times()
    for q, ((cfg, U0n), Ub) in enumerate(zip(boxes, outs)):
        Us, ts = _single(cfg, U0n, 5)
        assert np.array_equal(Ub, Us), q
        assert times[q] == ts, q


def test_batch_full_size_sampled_boxes():
    """The batched workload at full size (512 stratified boxes, N in 64..256,
    xi in 1..50, FP32 perturbation, 200 steps, one launch): the smallest, the
    median and the largest box against the FP64 oracle over all 200 steps."""
    boxes = W.batch2d(nbox=512)
    cfgs = [c for c, _, _ in boxes]
    nst = 200
    B = R.Batch(cfgs, prec="fp32_pert", bgs=[m["bg"] for _, _, m in boxes], max_steps=nst)
    starts = [(U - m["bg"][:, :, None]).astype(np.float32) for _, U, m in boxes]
    U = B.pack(starts)
    B.run(U, nst)
    torch.cuda.synchronize()
    assert B.poll() == 0
    outs = B.unpack(U)
    sizes = [int(c["n"][0]) for c in cfgs]
    order = np.argsort(sizes, kind="stable")
    for q in (int(order[0]), int(order[len(order) // 2]), int(order[-1])):
        cfg, _, meta = boxes[q]
        bg = meta["bg"][:, :, None]
        Uo, _, _ = oracle.run(cfg, bg + starts[q].astype(np.float64), nst)
        pert = Uo - bg
        s = [np.abs(pert[v]).max() for v in range(4)]
        sm = max(s[1:3])
        s = [s[0], sm, sm, s[3]]
        err = max(float(np.abs(outs[q][v].astype(np.float64) - pert[v]).max() / s[v]) for v in range(4))
        print(f"[batch full] box {q} N={cfg['n'][0]} xi={cfg['xi']:.2f} err/|pert| = {err:.2e}", flush=True)
        assert err <= 1e-5, (q, err)


def test_batch_wait_limit_gives_up_drains_and_recovers():
    """A dependency wait past its limit ends the run with an error instead of
    spinning: with a limit of 0 every wait not satisfied at once gives up, the
    items are skipped but signalled, every workgroup drains and the kernel
    ends; the poll reports the queue flag as RSST_E_DEVICE.  With the limit
    restored the next run is exact again (bitwise the single-box runs)."""
    boxes = _boxes_fp64()
    nsteps = 6
    B = R.Batch([c for c, _ in boxes], max_steps=8)
    B.set_tiles([8, 8, 8, 8])
    U0 = B.pack([u for _, u in boxes])
    U = U0.clone()
    B.set_wait_limit(0.0)
    B.run(U, nsteps)
    torch.cuda.synchronize()
    with pytest.raises(R.RsstError) as e:
        B.poll()
    assert e.value.code == R.RSST_E_DEVICE and (e.value.flags & 8), (e.value.code, e.value.flags)
    assert B.poll() == 0  # cleared
    B.set_wait_limit(10.0)
    U.copy_(U0)
    B.set_times(np.zeros(len(boxes)))
    B.run(U, nsteps)
    torch.cuda.synchronize()
    assert B.poll() == 0
    outs = B.unpack(U)
    times = B.times()
    for q, ((cfg, U0n), Ub) in enumerate(zip(boxes, outs)):
        Us, ts = _single(cfg, U0n, nsteps)
        assert np.array_equal(Ub, Us), q
        assert times[q] == ts, q
