"""Differentiable multi-step RSST rollout for PyTorch (FP64).

RSSTRollout.apply(U0, xi, cfg, nsteps, dt, checkpoint_every) runs nsteps
fixed-dt SSP-RK2 steps of the library from U0 and returns the final state.
Its backward pulls the incoming gradient back through every step with the
hand-written adjoint, giving dJ/dU0 and dJ/dxi.

Two ways to keep what the backward needs:
  * the whole trajectory (checkpoint_every = 1, or "auto" where the states
    and stage values of every step fit in half of the free device memory):
    the forward steps out of place (rsst_steps_out, one call) into preallocated
    buffers, keeping each state U_n and stage value U1_n, and the backward
    is one rsst_adjoint_run call over them, no step recomputed;
  * checkpoints (checkpoint_every = K > 1): the forward keeps the state at
    every K-th step; the backward re-runs each segment from its checkpoint
    (out of place, keeping the stage values) and runs its adjoint steps in
    reverse.  Each segment's backward is captured once as a HIP graph and
    replayed for the other segments of the same length.
Both give the same bits of dJ/dU0; dJ/dxi agrees to rounding (a trajectory
run sums it per tile over the whole run).

The time step is frozen: dt is an input, not the CFL rule, so the gradient
is that of the map U0 -> U_N at fixed dt.  Every step, forward and adjoint,
runs in the library's kernels; this module orders the calls and owns the
trajectory and checkpoint tensors.
"""
from __future__ import annotations

import torch

from . import Solver


class RSSTRollout(torch.autograd.Function):
    @staticmethod
    def forward(ctx, U0, xi, cfg, nsteps, dt, checkpoint_every="auto", use_graph=True):
        if U0.dtype != torch.float64 or not U0.is_cuda:
            raise TypeError("RSSTRollout: U0 must be a float64 CUDA tensor")
        nsteps = int(nsteps)
        K = trajectory_or_interval(U0, nsteps, checkpoint_every)
        c = dict(cfg)
        c["xi"] = float(xi)
        solver = Solver(c, adjoint=True)
        ctx.solver, ctx.nsteps, ctx.dt, ctx.K = solver, nsteps, float(dt), K
        ctx.use_graph = bool(use_graph)
        ctx.xi_needs_grad = isinstance(xi, torch.Tensor) and xi.requires_grad
        if K == 1:
            # the whole trajectory: states U_0..U_{N-1} and stage values
            # U1_0..U1_{N-1}; U_N goes to its own tensor (the output)
            shape = (max(nsteps, 1),) + tuple(U0.shape)
            traj = torch.empty(shape, dtype=torch.float64, device=U0.device)
            stage1 = torch.empty(shape, dtype=torch.float64, device=U0.device)
            out = U0.detach().contiguous().clone()
            if nsteps > 0:
                traj[0].copy_(out)
                solver.steps_out([traj[n] for n in range(nsteps)] + [out], [stage1[n] for n in range(nsteps)], dt)
            ctx.traj, ctx.stage1, ctx.ckpts = traj, stage1, None
            return out
        U = U0.detach().contiguous().clone()
        ckpts = [U.clone()]
        for n in range(nsteps):
            solver.step(U, dt)
            if (n + 1) % K == 0 and n + 1 < nsteps:
                ckpts.append(U.clone())
        ctx.ckpts, ctx.traj, ctx.stage1 = ckpts, None, None
        return U

    @staticmethod
    def _segment(solver, states, stage1, lam, dxi, dt, m):
        """Re-run m - 1 steps from states[0] into states[1..], keeping each
        step's stage value in stage1[..], then pull lam back through the m
        steps (the last one recomputes its stage value; states[0] must
        already hold the checkpoint)."""
        for i in range(1, m):
            solver.step_out(states[i - 1], stage1[i - 1], states[i], dt)
        for n in reversed(range(m)):
            solver.adjoint_step(states[n], lam, dt, dxi, U1=stage1[n] if n < m - 1 else None)

    @staticmethod
    def backward(ctx, gU):
        solver, K, dt, nsteps = ctx.solver, ctx.K, ctx.dt, ctx.nsteps
        lam = gU.detach().to(torch.float64).contiguous().clone()
        dxi = torch.zeros(1, dtype=torch.float64, device=lam.device)
        if K == 1:
            solver.adjoint_run([ctx.traj[n] for n in range(nsteps)], [ctx.stage1[n] for n in range(nsteps)],
                               lam, dt, dxi)
            torch.cuda.synchronize()
            solver.close()
            ctx.traj = ctx.stage1 = None
            gxi = dxi.reshape(()) if ctx.xi_needs_grad else None
            return lam, gxi, None, None, None, None, None
        nseg = len(ctx.ckpts)
        states = [torch.empty_like(lam) for _ in range(min(K, nsteps))]
        stage1 = [torch.empty_like(lam) for _ in range(min(K, nsteps) - 1)]
        graphs = {}
        for seg in reversed(range(nseg)):
            n0, n1 = seg * K, min((seg + 1) * K, nsteps)
            m = n1 - n0
            states[0].copy_(ctx.ckpts[seg])
            if not ctx.use_graph or nseg < 3:
                RSSTRollout._segment(solver, states, stage1, lam, dxi, dt, m)
                continue
            if m not in graphs:
                # first segment of this length runs eagerly (it also sets up
                # the kernels), later ones replay a HIP graph of the same
                # launches: forward re-run and adjoint steps
                RSSTRollout._segment(solver, states, stage1, lam, dxi, dt, m)
                g = torch.cuda.CUDAGraph()
                lam_in = lam.clone()
                dxi_in = dxi.clone()
                torch.cuda.synchronize()
                with torch.cuda.graph(g):
                    RSSTRollout._segment(solver, states, stage1, lam, dxi, dt, m)
                # capturing does not run the work: restore the cotangents
                lam.copy_(lam_in)
                dxi.copy_(dxi_in)
                graphs[m] = g
                continue
            graphs[m].replay()
        torch.cuda.synchronize()
        graphs.clear()
        solver.close()
        ctx.ckpts = None
        gxi = dxi.reshape(()) if ctx.xi_needs_grad else None
        return lam, gxi, None, None, None, None, None


def trajectory_or_interval(U0, nsteps, checkpoint_every):
    """1 (keep the whole trajectory) or the checkpoint interval K > 1.
    "auto": the trajectory where its 2 nsteps + 1 states fit in half of the
    free device memory, else every 20 steps."""
    if checkpoint_every != "auto":
        return max(1, int(checkpoint_every))
    free, _ = torch.cuda.mem_get_info(U0.device)
    need = (2 * int(nsteps) + 1) * U0.numel() * 8
    return 1 if need <= free // 2 else 20


def rollout(U0, xi, cfg, nsteps, dt, checkpoint_every="auto", use_graph=True):
    """Final state of nsteps fixed-dt steps from U0 (differentiable in U0
    and, if xi is a tensor that requires grad, in xi).  checkpoint_every: 1
    keeps the whole trajectory, K > 1 a checkpoint every K steps, "auto"
    the trajectory where it fits in half of the free device memory.
    use_graph: replay the backward of each checkpoint segment from a HIP
    graph (same kernels, fewer host launches)."""
    return RSSTRollout.apply(U0, xi, cfg, nsteps, dt, checkpoint_every, use_graph)


def kinetic_energy(U, cfg):
    """Domain integral of |m|^2 / (2 rho), the final-state functional of the
    adjoint workload."""
    ndim = int(cfg["ndim"])
    vol = 1.0
    for d in range(ndim):
        vol *= float(cfg["dx"][d])
    m2 = sum(U[1 + d] ** 2 for d in range(ndim))
    return 0.5 * (m2 / U[0]).sum() * vol
