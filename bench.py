#!/usr/bin/env python3
"""Throughput of the RSST time step on one MI355X.

Workload: the 3D stratified convection box, 256^3 cells, FP64, PVS form,
xi = 30, walls in z with gravity, periodic in x and y (synthetic, seeded).
A step is one full SSP-RK2 step (both fused stage kernels) on inputs already
resident in HBM.  Prints one JSON line.

    python bench.py [--steps K] [--warmup W] [--gpus 1] [--no-cpu]
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "Gcell-updates/s & HBM GB/s: FP64 plain vs FP32-pert/batched/adjoint, stated err"
HBM_PEAK_GBS = 8000.0
GAMMA = 5.0 / 3.0


def parity_err(Ug, Uo, ndim):
    import numpy as np
    rho = Uo[0]
    m2 = sum(Uo[1 + d] ** 2 for d in range(ndim))
    P = (GAMMA - 1) * (Uo[-1] - 0.5 * m2 / rho)
    a = np.sqrt(GAMMA * np.abs(P) / rho)
    s = [np.abs(rho).max()] + [np.abs(rho).max() * a.max()] * ndim + [np.abs(Uo[-1]).max()]
    return max(float(np.abs(Ug[v] - Uo[v]).max() / s[v]) for v in range(ndim + 2))


def traffic_from_profile(kernel_tag: str, version: str):
    """HBM bytes per launch from a committed rocprofv3 counter summary, if it
    was taken on this kernel revision; else None."""
    path = os.path.join(ROOT, "profiles", f"traffic_{kernel_tag}.json")
    if not os.path.exists(path):
        return None
    with open(path) as f:
        d = json.load(f)
    if d.get("version") != version:
        return None
    return d.get("bytes_per_launch")


def profile_json(name: str, version: str):
    """A committed per-run byte summary (profiles/<name>.json) if it was taken
    on this library revision; else None."""
    path = os.path.join(ROOT, "profiles", name)
    if not os.path.exists(path):
        return None
    with open(path) as f:
        d = json.load(f)
    return d if d.get("version") == version else None


def alu_view(version: str, value: float):
    """The FP64-ALU side of the headline kernels from the committed SQ counter
    summary (if taken on this revision): VALU wave-instructions per
    cell-update (both stages) and the rate at which they would fill every
    SIMD's issue slots (one wave64 instruction per 4 cycles, 1024 SIMDs at
    2.4 GHz); frac = value / that ceiling."""
    path = os.path.join(ROOT, "profiles", "stage_kernels_strat3d_256_sq_counters.md")
    if not os.path.exists(path):
        return None
    text = open(path).read()
    if f"`{version}`" not in text:
        return None
    per, col = {}, None
    for line in text.splitlines():
        cells = [c.strip() for c in line.split("|")]
        if col is None and "VALU wave-instr per cell" in cells:
            col = cells.index("VALU wave-instr per cell")
        for st in (1, 2):
            if col is not None and line.startswith(f"| `void stage_kernel<3, {st}, double, 1, 4>"):
                per[st] = float(cells[col])
    if len(per) != 2:
        return None
    wi = per[1] + per[2]
    ceiling = 1024 * 2.4e9 / 4 / wi / 1e9
    return {"bound": "alu", "valu_wave_instr_per_cell_update": round(wi, 2),
            "ceiling_Gcell_updates_s": round(ceiling, 2), "frac": round(value / ceiling, 4),
            "source": "profiles/stage_kernels_strat3d_256_sq_counters.md"}


def cpu_model() -> str:
    """The host CPU as /proc/cpuinfo names it, with its family, model and
    stepping numbers (a virtualised host may name only the vendor line) and
    the logical CPU count."""
    info = {}
    try:
        with open("/proc/cpuinfo") as f:
            for ln in f:
                if ":" in ln:
                    k, v = (x.strip() for x in ln.split(":", 1))
                    info.setdefault(k, v)
    except OSError:
        return ""
    name = info.get("model name", "")
    fam, mod, step = info.get("cpu family"), info.get("model"), info.get("stepping")
    extra = f" (family {fam}, model {mod}, stepping {step}" if fam else " ("
    return f"{name}{extra}, {os.cpu_count()} logical CPUs)"


def pert_err(Ug, pert, nv):
    """Max error over the perturbation scale per variable; the momentum
    components share the largest momentum scale."""
    import numpy as np
    sc = [np.abs(pert[v]).max() for v in range(nv)]
    sm = max(sc[1:nv - 1])
    sc = [sc[0]] + [sm] * (nv - 2) + [sc[nv - 1]]
    return max(float(np.abs(Ug[v] - pert[v]).max() / sc[v]) for v in range(nv))


def batch_roofline(version, prec, eff_gbs, cell_updates_s):
    """HBM view of a batched run: algorithmic bytes (5 x 4 values per
    cell-update) over the run time against the 8 TB/s peak, and the HBM bytes
    the committed counters of this revision measured per cell-update."""
    out = {"bound": "hbm", "achieved": round(eff_gbs, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
           "frac": round(eff_gbs / HBM_PEAK_GBS, 4), "traffic_GBs": None}
    t = profile_json("traffic_batch512.json", version)
    if t:
        b = t["bytes_per_cell_update"]["float" if prec == "fp32_pert" else "double"]
        out["traffic_GBs"] = round(b * cell_updates_s / 1e9, 1)
        out["traffic_frac"] = round(b * cell_updates_s / 1e9 / HBM_PEAK_GBS, 4)
        out["traffic_source"] = t["source"]
    return out


def bench_batch(R, W, np, torch, stream, args):
    import oracle
    boxes = W.batch2d(nbox=512)
    cfgs = [c for c, _, _ in boxes]
    ncell = sum(int(c["n"][0]) * int(c["n"][1]) for c in cfgs)
    nst = args.batch_steps
    sizes = [int(c["n"][0]) for c in cfgs]
    order = np.argsort(sizes, kind="stable")
    sample = [int(order[0]), int(order[len(order) // 2]), int(order[-1])]
    res = {}
    for prec in ("fp32_pert", "fp64"):
        if prec == "fp32_pert":
            B = R.Batch(cfgs, prec=prec, bgs=[m["bg"] for _, _, m in boxes], max_steps=nst)
            starts = [(U - m["bg"][:, :, None]).astype(np.float32) for _, U, m in boxes]
        else:
            B = R.Batch(cfgs, prec=prec, max_steps=nst)
            starts = [U for _, U, _ in boxes]
        U0 = B.pack(starts)
        U = torch.empty_like(U0)
        if args.batch_tiles:
            tiles, cached = [int(x) for x in args.batch_tiles.split(",")], False
            B.set_tiles(tiles)
        else:
            tiles, tune_ms, cached = B.autotune(U0, nsteps=40)
        U.copy_(U0)
        B.run(U, nst, stream)  # warm
        ms = []
        for _ in range(args.batch_runs):
            U.copy_(U0)
            a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            a.record(stream)
            B.run(U, nst, stream)
            b.record(stream)
            b.synchronize()
            ms.append(a.elapsed_time(b))
        U.copy_(U0)
        B.run(U, nst, stream)
        torch.cuda.synchronize()
        try:
            B.poll()
            flags = 0
        except R.RsstError as e:
            flags = getattr(e, "flags", -1)
        outs = B.unpack(U)
        errs = []
        for q in sample:
            cfg, Ufull, meta = boxes[q]
            if prec == "fp32_pert":
                bg = meta["bg"][:, :, None]
                Uo, _, _ = oracle.run(cfg, bg + starts[q].astype(np.float64), nst)
                errs.append(pert_err(outs[q].astype(np.float64), Uo - bg, 4))
            else:
                Uo, _, _ = oracle.run(cfg, Ufull, nst)
                errs.append(parity_err(outs[q], Uo, 2))
        best = min(ms)
        es = 4 if prec == "fp32_pert" else 8
        res[f"batch512_{prec}"] = {
            "nbox": len(cfgs), "cells": ncell, "steps": nst, "runs": args.batch_runs,
            "ms_per_run": round(best, 4), "ms_per_run_all": [round(x, 4) for x in ms],
            "Gcell_updates_s": round(ncell * nst / (best * 1e-3) / 1e9, 4),
            "effective_GBs": round(5 * 4 * es * ncell * nst / (best * 1e-3) / 1e9, 1),
            "roofline": batch_roofline(R.rsst_version(), prec, 5 * 4 * es * ncell * nst / (best * 1e-3) / 1e9,
                                       ncell * nst / (best * 1e-3)),
            "strip_rows": tiles, "tiles_from_cache": cached,
            "err_vs_oracle": max(errs), "err_kind": "perturbation scale (1e-5)" if prec == "fp32_pert"
            else "natural scales (1e-12)",
            "err_sample": f"boxes {sample} (smallest, median, largest N) over all {nst} steps",
            "nonphysical_flags": flags}
        B.close()
        del U, U0
        torch.cuda.empty_cache()
    return res


def bench_convergence(R, W, np, torch, stream):
    import math
    res, errs, ms = {}, {}, 0.0
    for N in (64, 128, 256):
        cfg, U0, meta = W.wave2d_oblique(N, "pvs")
        U = torch.from_numpy(U0).cuda()
        s = R.Solver(cfg, t_end=meta["t_end"])
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record(stream)
        s.steps(U, 40 * N)
        b.record(stream)
        b.synchronize()
        ms += a.elapsed_time(b)
        t, _ = s.time()
        s.close()
        th = meta["theta"]

        def fields(V):
            rho = V[0]
            vx, vy = V[1] / rho, V[2] / rho
            P = (GAMMA - 1) * (V[3] - 0.5 * rho * (vx * vx + vy * vy))
            return {"S": np.log(P) - GAMMA * np.log(rho), "Vperp": -vx * math.sin(th) + vy * math.cos(th),
                    "rho": rho, "P": P}
        f0, f1 = fields(U0), fields(U.cpu().numpy())
        errs[N] = {k: float(np.mean(np.abs(f1[k] - f0[k]))) for k in f0}
        res[f"t_reached_{N}"] = t
    res["L1"] = {str(N): errs[N] for N in errs}
    res["order_64_256"] = {k: round(0.5 * math.log2(errs[64][k] / errs[256][k]), 3) for k in errs[64]}
    res["gpu_ms_all_runs"] = round(ms, 2)
    return res


def run_to(s, U, t_end):
    """CFL steps until t = t_end (the last one cut); returns the step count."""
    n = 0
    while True:
        t, dt = s.time()
        if t >= t_end:
            return n
        if dt > 0 and t + 600 * dt < t_end:
            s.steps(U, 500)
            n += 500
        else:
            s.step(U)
            n += 1


def bench_rt(R, W, np, torch, stream, n=256):
    """Sec. 4.4 Rayleigh-Taylor at n^2 to t = 2.5: xi = 1 against the RSST at
    xi = 6.3 (PVS and PMS), at C_max = 10 (PVS, xi from each state's sound
    speed), and at xi = 6.3 with hydrostatic walls: steps, GPU time, max |V_y|
    and the L1 distance of the density field from the xi = 1 run."""
    out, ref = {}, None
    for form, xi, extra in (("pvs", 1.0, ""), ("pvs", 6.3, ""), ("pms", 6.3, ""), ("pvs", 1.0, "cmax10"),
                            ("pvs", 6.3, "hydro")):
        cfg, U0, meta = W.rt2d(n, form=form, xi=xi)
        if extra == "cmax10":
            cfg["cmax"] = 10.0
        elif extra == "hydro":
            cfg = dict(cfg, bc_lo=["periodic", "hydro"], bc_hi=["periodic", "hydro"])
        U = torch.from_numpy(U0).cuda()
        s = R.Solver(cfg, t_end=meta["t_end"])
        torch.cuda.synchronize()
        w0 = time.perf_counter()
        steps = run_to(s, U, meta["t_end"])
        torch.cuda.synchronize()
        wall = time.perf_counter() - w0
        s.close()
        Un = U.cpu().numpy()
        key = f"{form}_cmax10" if extra == "cmax10" else f"{form}_xi{xi:g}" + (f"_{extra}" if extra else "")
        out[key] = {"steps": steps, "wall_s": round(wall, 3), "max_abs_Vy": float(np.abs(Un[2] / Un[0]).max())}
        if ref is None:
            ref = Un[0]
        else:
            out[key]["L1_rho_vs_xi1"] = float(np.mean(np.abs(Un[0] - ref)))
            out[key]["step_saving_vs_xi1"] = round(out["pvs_xi1"]["steps"] / steps, 3)
    out["grid"] = [n, n]
    out["t_end"] = 2.5
    return out


def bench_rt_paper(R, W, np, torch, stream, n=1024, refs=(2048, 4096), log=None):
    """Sec. 4.4 at the paper's scale: 1024^2 to t = 2.5 with xi = 6.3 (PVS and
    PMS), C_max = 10 (PVS) and xi = 1: steps, GPU time, max |V_y| at
    t = 0.25, 0.5, ..., 2.5, and the L1 distance of the density at t = 2.5
    from the xi = 1 run on the same grid and from xi = 1 references on finer
    grids (the paper's is 4096^2).  A reference runs on the strip x in
    [1/8, 3/8] between mirror walls, which is the periodic problem restricted
    to it (the problem is even about both ends): its rows stay within the
    1024 cells of the 2D kernels and it costs a quarter of the full grid.
    Its density, averaged over blocks of (N/n)^2 cells, is compared with the
    1024^2 runs' on the same strip."""
    times = [0.25 * (k + 1) for k in range(10)]
    out = {}

    def run(N, form, xi, cmax=0.0, strip=False):
        cfg, U0, meta = W.rt2d(N, form=form, xi=xi, strip=strip)
        if cmax > 0:
            cfg["cmax"] = cmax
        U = torch.from_numpy(U0).cuda()
        s = R.Solver(cfg, t_end=meta["t_end"])
        vy, steps, wall = [], 0, 0.0
        for te in times:
            torch.cuda.synchronize()
            w0 = time.perf_counter()
            # run_to with this time as the end: the solver's end time stays
            # 2.5, so each leg lands on te by cutting its own last step
            s2 = steps
            while True:
                t, dt = s.time()
                if t >= te - 1e-12 * te:
                    break
                if dt > 0 and t + 600 * dt < te:
                    s.steps(U, 500)
                    steps += 500
                else:
                    s.step(U, min(dt, te - t) if dt > 0 else 0.0)
                    steps += 1
            torch.cuda.synchronize()
            wall += time.perf_counter() - w0
            vy.append(float((U[2] / U[0]).abs().max()))
            if log:
                log(f"[rt{N}{' strip' if strip else ''}] {form} xi={xi} cmax={cmax}: t={s.time()[0]:.4f} steps {steps} "
                    f"(+{steps - s2}) max|Vy|={vy[-1]:.4f} wall {wall:.1f} s")
        s.close()
        rho = U[0].cpu().numpy()
        return rho, {"steps": steps, "gpu_wall_s": round(wall, 2),
                     "max_abs_Vy": [round(x, 6) for x in vy], "_rho": rho}

    ref = None
    for form, xi, cmax in (("pvs", 1.0, 0.0), ("pvs", 6.3, 0.0), ("pms", 6.3, 0.0), ("pvs", 1.0, 10.0)):
        key = f"{form}_cmax10" if cmax else f"{form}_xi{xi:g}"
        rho, out[key] = run(n, form, xi, cmax)
        if ref is None:
            ref = rho
        else:
            out[key]["L1_rho_vs_xi1"] = float(np.mean(np.abs(rho - ref)))
            out[key]["step_saving_vs_xi1"] = round(out["pvs_xi1"]["steps"] / out[key]["steps"], 3)
    sl = slice(n // 8, 3 * n // 8)
    coarse = {k: v.pop("_rho") for k, v in out.items()}
    for N in refs:
        f = N // n
        rho, info = run(N, "pvs", 1.0, strip=True)
        info.pop("_rho", None)
        avg = rho.reshape(n, f, n // 4, f).mean(axis=(1, 3))
        info["grid"] = [N // 4, N]
        info["domain"] = "x in [1/8, 3/8] between mirror walls (the periodic problem restricted to it)"
        info["L1_rho_of_1024_runs"] = {k: float(np.mean(np.abs(r[:, sl] - avg))) for k, r in coarse.items()}
        out[f"ref{N}_pvs_xi1"] = info
        if log:
            log(f"[rt ref{N}] " + json.dumps(info))
    out["grid"] = [n, n]
    out["times"] = times
    return out


def adjoint_roofline(version, step_ms):
    """HBM bytes of one backward step (the segment's forward re-run, the
    stage-1 recompute and two VJPs) from the committed counters of this
    revision, over the measured backward time per step, against 8 TB/s."""
    t = profile_json("traffic_adjoint_bubble256.json", version)
    if not t:
        return None
    gbs = t["bytes_per_backward_step"] / (step_ms * 1e-3) / 1e9
    return {"bound": "latency", "achieved": round(gbs, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": round(gbs / HBM_PEAK_GBS, 4), "bytes_per_backward_step": round(t["bytes_per_backward_step"]),
            "source": t["source"]}


def bench_adjoint(R, W, np, torch, stream, args):
    """Gradient of the final kinetic energy of the 256^2 bubble (xi = 10,
    400 fixed-dt steps) w.r.t. the initial density field and xi, with the
    trajectory kept in HBM (and, for comparison, checkpoints every 20 steps
    with the segments re-run), with central differences on 32 directions as
    its error."""
    from paper_1812_04135_amd.rollout import kinetic_energy, rollout
    cfg, U0np, meta = W.adjoint2d(n=256, ndir=32)
    nsteps, K = args.adjoint_steps, 20
    dev = "cuda"
    g = 5.0 / 3.0
    vx, vy, P = (torch.from_numpy(meta[k]).to(dev) for k in ("vx", "vy", "P"))
    rho0 = torch.from_numpy(meta["rho"]).to(dev)

    def cons(r):
        return torch.stack([r, r * vx, r * vy, P / (g - 1.0) + 0.5 * r * (vx * vx + vy * vy)]).contiguous()

    s = R.Solver(cfg)
    U = cons(rho0)
    s.prime(U)
    _, dt = s.time()
    ncell = U0np[0].size

    def J_at(r):
        with torch.no_grad():
            u = cons(r)
            s.steps(u, nsteps, dt)
            return float(kinetic_energy(u, cfg))

    # forward alone (same steps, same dt), then forward + backward
    J_at(rho0)
    torch.cuda.synchronize()
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    a.record(stream)
    u = cons(rho0)
    s.steps(u, nsteps, dt)
    b.record(stream)
    b.synchronize()
    fwd_ms = a.elapsed_time(b)
    # one untimed forward + backward of each kind first (loads the adjoint
    # kernels; every checkpointed backward captures its own segment graphs,
    # so that cost stays in its timing)
    # (the trajectory's warm-up is full length: the runtime's first long
    # launch sequence has run up to 8x slower than the next ones)
    for k, m in ((1, nsteps), (K, 2 * K)):
        rw = rho0.clone().requires_grad_(True)
        kinetic_energy(rollout(cons(rw), torch.tensor(cfg["xi"], dtype=torch.float64, requires_grad=True),
                               cfg, m, dt, checkpoint_every=k), cfg).backward()

    def timed_backward(k):
        rho = rho0.clone().requires_grad_(True)
        xi = torch.tensor(cfg["xi"], dtype=torch.float64, requires_grad=True)
        u0 = cons(rho)
        torch.cuda.synchronize()
        f0, f1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        f0.record(stream)
        UN = rollout(u0, xi, cfg, nsteps, dt, checkpoint_every=k)
        f1.record(stream)
        f1.synchronize()
        timed_backward.fwd_ms = f0.elapsed_time(f1)
        J = kinetic_energy(UN, cfg)
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        J.backward()
        e1.record(stream)
        e1.synchronize()
        return e0.elapsed_time(e1), rho.grad, xi.grad, J

    # the whole trajectory kept in HBM ("auto" picks it: 2 x 400 states of
    # 2 MiB), then checkpoints every K steps with the segments re-run
    from paper_1812_04135_amd.rollout import trajectory_or_interval
    kind = trajectory_or_interval(rho0, nsteps, "auto")
    bwd_ms, grad, xi_grad, J = timed_backward("auto")
    roll_fwd_ms = timed_backward.fwd_ms
    ck_ms, ck_grad, _, _ = timed_backward(K)
    same_bits = bool(torch.equal(grad, ck_grad))
    # central differences over a sweep of steps: truncation error falls as
    # h^2 and forward rounding grows as 1/h, so the sweep shows where the
    # floor sits; h = 1e-6 stays the reported figure
    sweep = {}
    hs = tuple(float(x) for x in args.fd_h.split(",") if x.strip()) or (1e-6,)
    for h in hs:
        e = []
        for q in range(meta["dirs"].shape[0]):
            d = torch.from_numpy(meta["dirs"][q]).to(dev)
            fd = (J_at(rho0 + h * d) - J_at(rho0 - h * d)) / (2 * h)
            ad = float((grad * d).sum())
            e.append(abs(fd - ad) / abs(ad))
        sweep[h] = np.array(e)
    s.close()
    href = 1e-6 if 1e-6 in sweep else hs[0]
    errs = sweep[href]
    adj_step_ms = bwd_ms / nsteps
    return {"adjoint_bubble256_fp64": {
        "steps": nsteps, "dt": dt, "J": float(J.detach()),
        "dJ_dxi": float(xi_grad),
        "backward_kept": "trajectory" if kind == 1 else f"checkpoints every {kind}",
        "trajectory_bytes": 2 * nsteps * U.numel() * 8,
        "forward_ms": round(fwd_ms, 3), "rollout_forward_ms": round(roll_fwd_ms, 3),
        "backward_ms": round(bwd_ms, 3),
        "backward_ms_per_step": round(adj_step_ms, 5),
        "Gcell_updates_s": round(ncell * nsteps / (bwd_ms * 1e-3) / 1e9, 4),
        "backward_over_forward": round(bwd_ms / fwd_ms, 3),
        "checkpoint_every": K, "backward_checkpointed_ms": round(ck_ms, 3),
        "checkpointed_over_forward": round(ck_ms / fwd_ms, 3),
        "checkpointed_same_dJdU0_bits": same_bits,
        "roofline": adjoint_roofline(R.rsst_version(), adj_step_ms),
        "fd_rel_err_median": float(np.median(errs)), "fd_rel_err_max": float(errs.max()),
        "fd_within_bar": bool(errs.max() <= 1e-4),
        "fd_h_sweep": {f"{h:g}": {"median": float(np.median(e)), "max": float(e.max())}
                       for h, e in sweep.items()},
        "fd": f"central differences, h = {href:g}, 32 smooth density directions; "
              "bar: every direction within 1e-4 relative (the full-size GPU test's)"}}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--cpu-steps", type=int, default=4)
    ap.add_argument("--no-batch", action="store_true", help="skip the batched 512-box workload")
    ap.add_argument("--batch-steps", type=int, default=200)
    ap.add_argument("--batch-runs", type=int, default=3)
    ap.add_argument("--no-adjoint", action="store_true", help="skip the adjoint workload")
    ap.add_argument("--no-rt", action="store_true", help="skip the Rayleigh-Taylor workload")
    ap.add_argument("--no-conv", action="store_true", help="skip the linear-wave convergence runs")
    ap.add_argument("--adjoint-steps", type=int, default=400)
    ap.add_argument("--only", choices=["batch", "adjoint", "rt1024"], default=None,
                    help="run only that secondary workload and print its JSON (for profiling)")
    ap.add_argument("--fd-h", default="1e-3,1e-4,1e-5,1e-6,1e-7",
                    help="finite-difference steps of the adjoint leg's check (comma-separated; "
                         "the errors at 1e-6 are the reported ones when it is in the list)")
    ap.add_argument("--rt-refs", default="2048,4096",
                    help="grids of the xi = 1 references of --only rt1024 (comma-separated, "
                         "multiples of 1024; empty for none)")
    ap.add_argument("--batch-tiles", default=None,
                    help="strip rows per width class, e.g. 32,64,96,96 (skips the autotuner)")
    ap.add_argument("--copy-ref", action="store_true",
                    help="only run a plain device copy of one 256^3 FP64 state (5 x 134 MB), "
                         "the reference kernel for scaling HBM byte counters")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py: this build measures one GPU only (the step is single-device; "
              "multi-GPU domain decomposition is a design note, not built)", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import paper_1812_04135_amd as R
    import workloads as W

    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    if args.only:
        stream = torch.cuda.current_stream()
        if args.only == "rt1024":
            refs = tuple(int(x) for x in args.rt_refs.split(",") if x.strip())
            if any(N % 1024 for N in refs):
                ap.error("--rt-refs: each grid must be a multiple of 1024")
            res = bench_rt_paper(R, W, np, torch, stream, refs=refs,
                                 log=lambda m: print(m, file=sys.stderr, flush=True))
        else:
            leg = bench_batch if args.only == "batch" else bench_adjoint
            res = leg(R, W, np, torch, stream, args)
        print(json.dumps(res), flush=True)
        return
    if args.copy_ref:
        x = torch.ones(5 * 256 ** 3, dtype=torch.float64, device=dev)
        y = torch.empty_like(x)
        for _ in range(5):
            y.copy_(x)
        torch.cuda.synchronize()
        print(json.dumps({"copy_ref_bytes_read": x.numel() * 8, "copy_ref_bytes_written": x.numel() * 8}))
        return
    cfg, U0, meta = W.strat3d(n=256, xi=30.0, form="pvs")
    nv, ncell = U0.shape[0], U0[0].size
    U = torch.from_numpy(U0).to(dev)
    sol = R.Solver(cfg)
    stream = torch.cuda.current_stream()

    for _ in range(args.warmup):
        sol.step(U)
    torch.cuda.synchronize()

    K = args.steps
    ev = [[torch.cuda.Event(enable_timing=True) for _ in range(3)] for _ in range(K)]
    e_start, e_end = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    w0 = time.perf_counter()
    e_start.record(stream)
    for q in range(K):
        ev[q][0].record(stream)
        sol.stage(U, 1)
        ev[q][1].record(stream)
        sol.stage(U, 2)
        ev[q][2].record(stream)
    e_end.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - w0
    total_ms = e_start.elapsed_time(e_end)
    s1 = sum(ev[q][0].elapsed_time(ev[q][1]) for q in range(K)) / K
    s2 = sum(ev[q][1].elapsed_time(ev[q][2]) for q in range(K)) / K
    ms_step = total_ms / K
    gcell = ncell / (ms_step * 1e-3) / 1e9
    try:
        sol.poll()
        flags = 0
    except R.RsstError as e:
        flags = getattr(e, "flags", -1)

    bytes_s1 = 2 * nv * 8 * ncell
    bytes_s2 = 3 * nv * 8 * ncell
    ach2 = bytes_s2 / (s2 * 1e-3) / 1e9
    ach1 = bytes_s1 / (s1 * 1e-3) / 1e9
    eff = 5 * nv * 8 * ncell / (ms_step * 1e-3) / 1e9
    version = R.rsst_version()
    traffic = traffic_from_profile("stage2_strat3d_256_fp64", version)
    # a plain device copy of one 256^3 FP64 state (read + write), the second
    # denominator next to the published HBM peak
    xa = torch.empty(nv * ncell, dtype=torch.float64, device=dev).fill_(1.0)
    xb = torch.empty_like(xa)
    for _ in range(3):
        xb.copy_(xa)
    c0, c1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    c0.record(stream)
    for _ in range(10):
        xb.copy_(xa)
    c1.record(stream)
    torch.cuda.synchronize()
    copy_gbs = 2 * xa.numel() * 8 * 10 / (c0.elapsed_time(c1) * 1e-3) / 1e9
    del xa, xb

    out = {
        "metric": METRIC,
        "value": round(gcell, 4),
        "unit": "Gcell-updates/s",
        "n_gpus": 1,
        "steps": K,
        "warmup": args.warmup,
        "ms_per_step": round(ms_step, 5),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": "strat3d: 3D stratified polytropic box 256^3, PVS, xi=30, "
                               "gravity -z, walls z, periodic x/y, FP64",
                   "grid": [256, 256, 256], "form": "pvs", "xi": 30.0, "cfl": 0.4},
        "roofline": {"bound": "hbm", "achieved": round(ach2, 1), "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": round(ach2 / HBM_PEAK_GBS, 4),
                     "traffic": traffic, "kernel": "stage_kernel<3,2,double> (RK stage 2)",
                     "alg_bytes_per_launch": bytes_s2, "avg_ms": round(s2, 5),
                     "copy_GBs": round(copy_gbs, 1), "frac_of_copy": round(ach2 / copy_gbs, 4),
                     "traffic_GBs": round(traffic / (s2 * 1e-3) / 1e9, 1) if traffic else None,
                     # the whole step (both stage kernels, 5 nvar 8 B per cell-update)
                     # against the same peak, next to the dominant kernel's figure above
                     "step": {"achieved": round(eff, 1), "frac": round(eff / HBM_PEAK_GBS, 4),
                              "ms": round(ms_step, 5)},
                     "alu_view": alu_view(version, gcell)},
        "stage1": {"avg_ms": round(s1, 5), "achieved_GBs": round(ach1, 1),
                   "alg_bytes_per_launch": bytes_s1},
        "effective_GBs_step": round(eff, 1),
        "wall_s": round(wall, 3),
        "nonphysical_flags": flags,
        "library": version,
    }

    # ---- secondary workloads (same GPU, same library), each with its error
    sec = {}

    def timed(sol, U, nsteps, warm=3):
        for _ in range(warm):
            sol.step(U)
        torch.cuda.synchronize()
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record(stream)
        for _ in range(nsteps):
            sol.step(U)
        b.record(stream)
        torch.cuda.synchronize()
        return a.elapsed_time(b) / nsteps

    # FP32 perturbation about the FP64 polytrope, same 256^3 box
    bg = torch.from_numpy(meta["bg"]).to(dev)
    U1_0 = (U0 - meta["bg"][:, :, None, None]).astype(np.float32)
    U32 = torch.from_numpy(U1_0).to(dev)
    s32 = R.Solver(cfg, prec="fp32_pert", bg=bg, bg_axis=2)
    ms32 = timed(s32, U32, K)
    s32.close()
    sec["strat3d_fp32_pert"] = {
        "ms_per_step": round(ms32, 5), "Gcell_updates_s": round(ncell / (ms32 * 1e-3) / 1e9, 4),
        "effective_GBs": round(5 * nv * 4 * ncell / (ms32 * 1e-3) / 1e9, 1),
        "speedup_vs_fp64": round(ms_step / ms32, 3)}

    # the same 256^3 box with xi from the sound speed (eq. cx), C_max = 0.1
    # (a runs from 0.18 at the top to 0.84 at the bottom): time per step and
    # the CFL step it allows against the constant xi = 30
    cfg_c = dict(cfg, cmax=0.1)
    Uc = torch.from_numpy(U0).to(dev)
    sc = R.Solver(cfg_c)
    msc = timed(sc, Uc, K)
    sc.prime(torch.from_numpy(U0).to(dev))
    _, dtc = sc.time()
    sc.close()
    s30 = R.Solver(cfg)
    s30.prime(torch.from_numpy(U0).to(dev))
    _, dt30 = s30.time()
    s30.close()
    sec["strat3d_cmax_fp64"] = {"cmax": 0.1, "ms_per_step": round(msc, 5),
                                "Gcell_updates_s": round(ncell / (msc * 1e-3) / 1e9, 4),
                                "speed_vs_constant_xi": round(ms_step / msc, 3),
                                "cfl_dt": dtc, "cfl_dt_constant_xi30": dt30}

    # the same 256^3 box as a van der Waals gas (same rho and P, so the same
    # hydrostatic balance; E from that gas's internal energy): the cost of
    # the general equation of state in the step
    cfg_v, U0v, _ = W.strat3d(n=256, xi=30.0, form="pvs", gas=W.VDW)
    Uv = torch.from_numpy(U0v).to(dev)
    sv = R.Solver(cfg_v)
    msv = timed(sv, Uv, K)
    sv.close()
    del Uv
    sec["strat3d_vdw_fp64"] = {"eos": dict(W.VDW), "ms_per_step": round(msv, 5),
                               "Gcell_updates_s": round(ncell / (msv * 1e-3) / 1e9, 4),
                               "speed_vs_ideal_gas": round(ms_step / msv, 3)}

    # 2D bubble 512^2 FP64 (L2/MALL resident; launch-latency sensitive)
    cfg2, U2_0, meta2 = W.bubble2d()
    U2 = torch.from_numpy(U2_0).to(dev)
    s2 = R.Solver(cfg2)
    ms2 = timed(s2, U2, 200)
    s2.close()
    n2 = U2_0[0].size
    nv2 = U2_0.shape[0]
    sec["bubble2d_512_fp64"] = {"ms_per_step": round(ms2, 5),
                                "Gcell_updates_s": round(n2 / (ms2 * 1e-3) / 1e9, 4),
                                "effective_GBs": round(5 * nv2 * 8 * n2 / (ms2 * 1e-3) / 1e9, 1)}
    # the same bubble as an FP32 perturbation about the uniform ambient state
    bg2 = torch.from_numpy(meta2["bg"]).to(dev)
    U2p0 = (U2_0 - meta2["bg"][:, :, None]).astype(np.float32)
    U2p = torch.from_numpy(U2p0).to(dev)
    s2p = R.Solver(cfg2, prec="fp32_pert", bg=bg2, bg_axis=-1)
    ms2p = timed(s2p, U2p, 200)
    s2p.close()
    sec["bubble2d_512_fp32_pert"] = {"ms_per_step": round(ms2p, 5),
                                     "Gcell_updates_s": round(n2 / (ms2p * 1e-3) / 1e9, 4),
                                     "effective_GBs": round(5 * nv2 * 4 * n2 / (ms2p * 1e-3) / 1e9, 1),
                                     "speedup_vs_fp64": round(ms2 / ms2p, 3)}
    # FP64 diagnostics (sums, kinetic energy, maxima) of the 256^3 state
    td = time.perf_counter()
    for _ in range(20):
        sol.diag(U)
    sec["diag_strat3d_256_ms"] = round((time.perf_counter() - td) / 20 * 1e3, 4)

    # 1D wave, 256 cells, xi = 10, the whole run to t_end (2 reduced crossings):
    # one untimed run (first launch of the kernel), then three timed ones
    cfg1, U1w, meta1 = W.wave1d(xi=10.0)
    rates = []
    for rep in range(4):
        Uw = torch.from_numpy(U1w).to(dev)
        s1 = R.Solver(cfg1, t_end=meta1["t_end"])
        s1.prime(Uw)
        torch.cuda.synchronize()
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record(stream)
        s1.steps(Uw, 1300)
        b.record(stream)
        torch.cuda.synchronize()
        t1, _ = s1.time()
        s1.close()
        if rep > 0:
            rates.append(round(1300 / (a.elapsed_time(b) * 1e-3), 1))
    sec["wave1d_256_xi10"] = {"steps": 1300, "t_reached": t1, "t_end": meta1["t_end"],
                              "steps_per_s": float(np.median(rates)), "steps_per_s_all": rates,
                              "timing": "median of 3 runs after one untimed run"}
    # batched sweep: 512 stratified 2D boxes (N in 64..256, contrast 3..100,
    # xi 1..50), 200 steps with per-box CFL dt in one persistent launch
    # replayed from a HIP graph; FP32 perturbation (the workload) and FP64
    if not args.no_batch:
        sec.update(bench_batch(R, W, np, torch, stream, args))
    if not args.no_adjoint:
        sec.update(bench_adjoint(R, W, np, torch, stream, args))
    # Sec. 4.2 linear wave at 30 degrees (PVS, xi = 5) to t = 1 at N = 64,
    # 128, 256: L1 errors against the initial snapshot and their orders
    if not args.no_conv:
        sec["wave2d_convergence_pvs"] = bench_convergence(R, W, np, torch, stream)
    if not args.no_rt:
        sec["rt2d_256"] = bench_rt(R, W, np, torch, stream)
    out["secondary"] = sec

    if not args.no_cpu:
        import oracle
        # the CPU oracle on a bounded sample: cpu_steps full 256^3 steps from
        # the initial state, which also gives the GPU error on that sample
        t0 = time.perf_counter()
        Uo, _, _ = oracle.run(cfg, U0, args.cpu_steps)
        cpu_s = time.perf_counter() - t0
        Ug = torch.from_numpy(U0).to(dev)
        s = R.Solver(cfg)
        s.steps(Ug, args.cpu_steps)
        torch.cuda.synchronize()
        err = parity_err(Ug.cpu().numpy(), Uo, 3)
        s.close()
        # FP32 perturbation on the same sample, against the same FP64 oracle
        # run from U0 + fp32(U - U0)
        Ustart = meta["bg"][:, :, None, None] + U1_0.astype(np.float64)
        Uo32, _, _ = oracle.run(cfg, Ustart, args.cpu_steps)
        Ug32 = torch.from_numpy(U1_0).to(dev)
        s = R.Solver(cfg, prec="fp32_pert", bg=bg, bg_axis=2)
        s.steps(Ug32, args.cpu_steps)
        torch.cuda.synchronize()
        pert = Uo32 - meta["bg"][:, :, None, None]
        g32 = Ug32.cpu().numpy().astype(np.float64)
        sc = [np.abs(pert[v]).max() for v in range(nv)]
        sm = max(sc[1:4])
        sc = [sc[0], sm, sm, sm, sc[4]]
        err32 = max(float(np.abs(g32[v] - pert[v]).max() / sc[v]) for v in range(nv))
        s.close()
        out["secondary"]["strat3d_fp32_pert"]["err_vs_oracle_pert"] = err32
        # C_max mode: one step of the 256^3 box against the oracle
        Uoc, _, _ = oracle.run(cfg_c, U0, 1)
        Ugc = torch.from_numpy(U0).to(dev)
        s = R.Solver(cfg_c)
        s.step(Ugc)
        torch.cuda.synchronize()
        s.close()
        out["secondary"]["strat3d_cmax_fp64"]["err_vs_oracle"] = parity_err(Ugc.cpu().numpy(), Uoc, 3)
        out["secondary"]["strat3d_cmax_fp64"]["err_steps"] = 1
        # van der Waals gas: one step of the 256^3 box against the oracle
        Uov, _, _ = oracle.run(cfg_v, U0v, 1)
        Ugv = torch.from_numpy(U0v).to(dev)
        s = R.Solver(cfg_v)
        s.step(Ugv)
        torch.cuda.synchronize()
        s.close()
        out["secondary"]["strat3d_vdw_fp64"]["err_vs_oracle"] = parity_err(Ugv.cpu().numpy(), Uov, 3)
        out["secondary"]["strat3d_vdw_fp64"]["err_steps"] = 1
        del Ugv, Uov
        # the bubble's FP32 perturbation over 5 steps against the FP64 oracle
        Uo2, _, _ = oracle.run(cfg2, meta2["bg"][:, :, None] + U2p0.astype(np.float64), 5)
        g2 = torch.from_numpy(U2p0).to(dev)
        s = R.Solver(cfg2, prec="fp32_pert", bg=bg2, bg_axis=-1)
        s.steps(g2, 5)
        torch.cuda.synchronize()
        s.close()
        out["secondary"]["bubble2d_512_fp32_pert"]["err_vs_oracle_pert"] = pert_err(
            g2.cpu().numpy().astype(np.float64), Uo2 - meta2["bg"][:, :, None], 4)
        out["secondary"]["bubble2d_512_fp32_pert"]["err_steps"] = 5
        # the same oracle on one core, on a smaller bounded sample: one step
        # of a 256 x 256 x 32 slab of the box (same columns, bottom 32 planes)
        nth = oracle.threads()
        oracle.set_threads(1)
        cfg1 = dict(cfg)
        cfg1["n"] = [256, 256, 32]
        U1c = np.ascontiguousarray(U0[:, :32])
        t1 = time.perf_counter()
        oracle.run(cfg1, U1c, 1)
        one_s = time.perf_counter() - t1
        oracle.set_threads(nth)
        model = cpu_model()
        out["cpu_baseline"] = {"value": round(ncell * args.cpu_steps / cpu_s / 1e9, 6),
                               "unit": "Gcell-updates/s", "cores": nth, "cpu_model": model,
                               "kind": "oracle",
                               "sample": f"{args.cpu_steps} full steps of the 256^3 box "
                                         f"({cpu_s:.1f} s)",
                               "one_core": {"value": round(256 * 256 * 32 / one_s / 1e9, 6),
                                            "cores": 1,
                                            "sample": f"1 step of a 256x256x32 slab ({one_s:.1f} s)"}}
        out["err_vs_oracle"] = {"max_err_over_scale": err, "steps": args.cpu_steps,
                                "tolerance": 1e-12}
    sol.close()
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
