"""Differentiable SSP-RK3 + CSWENO trajectories (argument marshalling over the
C ABI's tape and vector-Jacobian-product calls).

The limiter is differentiated with each stage's troubled-cell set frozen and
dt frozen per step (both are decisions, not smooth functions of the state).
Memory is bounded by step checkpointing: the forward keeps the state every
`checkpoint_every` steps; the backward recomputes one segment at a time,
recording a tape per step, and runs the step adjoints in reverse.
"""
from __future__ import annotations

import torch


class _Trajectory(torch.autograd.Function):
    @staticmethod
    def forward(ctx, u0, solver, nsteps, checkpoint_every):
        u = u0.detach().clone().contiguous()
        ckpts = []
        for s in range(nsteps):
            if s % checkpoint_every == 0:
                ckpts.append(u.clone())
            solver.ssprk3_step(u)
        ctx.solver = solver
        ctx.nsteps = nsteps
        ctx.every = checkpoint_every
        ctx.ckpts = ckpts
        return u

    @staticmethod
    def backward(ctx, grad):
        S = ctx.solver
        ybar = grad.detach().clone().contiguous()
        nseg = len(ctx.ckpts)
        tapes = [S.new_tape() for _ in range(min(ctx.every, ctx.nsteps))]
        for seg in range(nseg - 1, -1, -1):
            first = seg * ctx.every
            last = min(ctx.nsteps, first + ctx.every)
            u = ctx.ckpts[seg].clone()
            for i, s in enumerate(range(first, last)):
                S.ssprk3_step_tape(u, tapes[i])
            for i in range(last - first - 1, -1, -1):
                ybar = S.ssprk3_step_vjp(tapes[i], ybar)
        return ybar, None, None, None


def trajectory(solver, u0, nsteps, checkpoint_every=10):
    """u(T) after nsteps SSP-RK3 steps with the limiter, differentiable in u0."""
    return _Trajectory.apply(u0, solver, nsteps, checkpoint_every)


def record(solver, u0, nsteps):
    """Forward with one tape per step (decisions recorded): (u_T, tapes)."""
    u = u0.detach().clone().contiguous()
    tapes = []
    for _ in range(nsteps):
        t = solver.new_tape()
        solver.ssprk3_step_tape(u, t)
        tapes.append(t)
    return u, tapes


def replay(solver, u0, tapes):
    """Forward with every step's dt and troubled sets taken from tapes."""
    u = u0.detach().clone().contiguous()
    for t in tapes:
        tt = t.clone()
        solver.ssprk3_step_tape(u, tt, replay=True)
    return u
