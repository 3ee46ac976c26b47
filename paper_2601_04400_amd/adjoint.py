"""Differentiable rollout of the RK3 solver: torch.autograd.Function whose
backward runs the hand-written discrete adjoint kernels with checkpointing.

Section 2 trains through m unrolled solver steps and infers physical
parameters by reverse-mode differentiation; here the forward pass keeps a
copy of the state every `every` steps, and the backward pass replays each
segment from its checkpoint, recording the stage-start states of every step
of the segment (shk_rk3_step_record), and then runs the reverse steps from
those records (shk_rk3_step_adjoint_tape).  Memory: nsteps/every checkpoints
plus 3 * every recorded states.
"""
import torch


class _Rollout(torch.autograd.Function):
    @staticmethod
    def forward(ctx, U0, params, grid, nsteps, dt, every):
        U = U0.detach().clone()
        if not torch.is_tensor(dt):
            dt = torch.full((grid.shape[0],), float(dt), dtype=torch.float64, device=U.device)
        ckpts = [U.clone()]
        for s in range(nsteps):
            grid.step(U, dt)
            if (s + 1) % every == 0 and s + 1 < nsteps:
                ckpts.append(U.clone())
        ctx.grid, ctx.nsteps, ctx.dt, ctx.every = grid, nsteps, dt, every
        ctx.ckpts = ckpts
        return U

    @staticmethod
    def backward(ctx, U_bar):
        g, dt, every, nsteps = ctx.grid, ctx.dt, ctx.every, ctx.nsteps
        Ub = U_bar.detach().to(dtype=torch.float64).contiguous().clone()
        pb = g.param_bar()
        tapes = torch.empty((min(every, nsteps), 3) + tuple(g.shape), dtype=torch.float64, device=Ub.device)
        if not torch.is_tensor(dt):
            dt = g._dt_tensor(dt)
        for c in range(len(ctx.ckpts) - 1, -1, -1):
            first = c * every
            count = min(every, nsteps - first)
            U = ctx.ckpts[c].clone()
            g.steps_record(U, tapes, count, dt)
            g.steps_adjoint_tape(tapes, count, dt, Ub, pb)
        return Ub, pb, None, None, None, None


def rollout(grid, U0, params, nsteps, dt, every=20):
    """U after `nsteps` fixed-dt RK3 steps from U0, differentiable with
    respect to U0 and `params` = tensor [nbatch, 5] of (gamma, inflow rho, u,
    v, p).  `params` carries no values into the solver: it must equal the
    grid's own description and only receives the gradient."""
    return _Rollout.apply(U0, params, grid, nsteps, dt, every)
