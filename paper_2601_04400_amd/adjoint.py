"""Differentiable rollout of the RK3 solver: torch.autograd.Function whose
backward runs the hand-written discrete adjoint kernels with checkpointing.

Section 2 trains through m unrolled solver steps and infers physical
parameters by reverse-mode differentiation; here the forward pass keeps a
copy of the state every `every` steps, and the backward pass replays each
segment from its checkpoint, recording the stage-start states of every step
of the segment (shk_rk3_step_record), and then runs the reverse steps from
those records (shk_rk3_step_adjoint_tape).  Memory: nsteps/every checkpoints
plus 3 * every recorded states.

The replay of a segment only reads its checkpoint, so by default it runs on
a replica of the grid (own workspace, second HIP stream) one segment ahead
of the reverse pass, into the other of two tape buffers: the replay of
segment c - 1 overlaps the reverse steps of segment c.  Events order each
reverse segment after its replay and each replay after the reverse segment
that last read its tape buffer.  The kernels and their inputs are the same
as in the serial order, so the gradients are identical bit for bit.
"""
import torch


class _Rollout(torch.autograd.Function):
    @staticmethod
    def forward(ctx, U0, params, grid, nsteps, dt, every, overlap, trace):
        U = U0.detach().clone()
        if not torch.is_tensor(dt):
            dt = torch.full((grid.shape[0],), float(dt), dtype=torch.float64, device=U.device)
        ckpts = [U.clone()]
        for s in range(nsteps):
            grid.step(U, dt)
            if (s + 1) % every == 0 and s + 1 < nsteps:
                ckpts.append(U.clone())
        ctx.grid, ctx.nsteps, ctx.dt, ctx.every, ctx.overlap, ctx.trace = grid, nsteps, dt, every, overlap, trace
        ctx.ckpts = ckpts
        return U

    @staticmethod
    def backward(ctx, U_bar):
        g, dt, every, nsteps = ctx.grid, ctx.dt, ctx.every, ctx.nsteps
        Ub = U_bar.detach().to(dtype=torch.float64).contiguous().clone()
        pb = g.param_bar()
        if not torch.is_tensor(dt):
            dt = g._dt_tensor(dt)
        nseg = len(ctx.ckpts)
        if not ctx.overlap or nseg < 2:
            tapes = torch.empty((min(every, nsteps), 3) + tuple(g.shape), dtype=torch.float64, device=Ub.device)
            for c in range(nseg - 1, -1, -1):
                count = min(every, nsteps - c * every)
                U = ctx.ckpts[c].clone()
                g.steps_record(U, tapes, count, dt)
                g.steps_adjoint_tape(tapes, count, dt, Ub, pb)
        else:
            _reverse_overlapped(g, ctx.ckpts, nsteps, every, dt, Ub, pb, ctx.trace)
        return Ub, pb, None, None, None, None, None, None


def _mark(trace, stream, label):
    """Timing event on `stream` appended to trace (a list) as (label, event)."""
    if trace is not None:
        e = torch.cuda.Event(enable_timing=True)
        e.record(stream)
        trace.append((label, e))


def _reverse_overlapped(g, ckpts, nsteps, every, dt, Ub, pb, trace=None):
    main = torch.cuda.current_stream(Ub.device)
    rep, side = g.replica()
    tapes, work = g.replay_buffers(min(every, nsteps))
    for t in list(ckpts) + [dt]:
        t.record_stream(side)
    side.wait_stream(main)  # checkpoints, dt and earlier users of the buffers are done
    freed = [None, None]  # per tape buffer: the reverse segment that read it last is done
    ready = {}

    def replay(c):
        k = c % 2
        if freed[k] is not None:
            side.wait_event(freed[k])
        with torch.cuda.stream(side):
            _mark(trace, side, f"replay {c} start")
            work.copy_(ckpts[c])
            rep.steps_record(work, tapes[k], min(every, nsteps - c * every), dt)
            _mark(trace, side, f"replay {c} end")
            ready[c] = torch.cuda.Event()
            ready[c].record(side)

    nseg = len(ckpts)
    replay(nseg - 1)
    for c in range(nseg - 1, -1, -1):
        if c > 0:
            replay(c - 1)
        _mark(trace, main, f"reverse {c} issued")
        main.wait_event(ready.pop(c))
        k = c % 2
        _mark(trace, main, f"reverse {c} start")
        g.steps_adjoint_tape(tapes[k], min(every, nsteps - c * every), dt, Ub, pb)
        _mark(trace, main, f"reverse {c} end")
        freed[k] = torch.cuda.Event()
        freed[k].record(main)


def rollout(grid, U0, params, nsteps, dt, every=20, overlap=True, trace=None):
    """U after `nsteps` fixed-dt RK3 steps from U0, differentiable with
    respect to U0 and `params` = tensor [nbatch, 5] of (gamma, inflow rho, u,
    v, p).  `params` carries no values into the solver: it must equal the
    grid's own description and only receives the gradient.  overlap: replay
    segments on a replica grid concurrently with the reverse pass.  trace: a
    list that, in the overlapped backward pass, receives (label, timing
    event) pairs at the start and end of every replay and reverse segment."""
    return _Rollout.apply(U0, params, grid, nsteps, dt, every, overlap, trace)
