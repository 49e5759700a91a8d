"""Differentiation form: gradient of the final kinetic energy w.r.t. the initial velocity.

``Rollout`` is a ``torch.autograd.Function`` around `steps` TVD-RK3 steps of the library.
The forward pass keeps the state every `checkpoint_every` steps; the backward pass
recomputes each segment's states from its checkpoint and runs ``dfdg_rk3_step_vjp``
(the hand-written adjoint of the residual and the self-adjoint mass solve) in reverse.
All arithmetic runs in the library's kernels; this module only orders the calls.
"""
import torch


class Rollout(torch.autograd.Function):
    @staticmethod
    def forward(ctx, U0, solver, dt, steps, checkpoint_every):
        U = U0.detach().clone()
        ckpts = {0: U.clone()}
        solver.reset_history()
        for n in range(steps):
            solver.rk3_step(U, dt)
            if (n + 1) % checkpoint_every == 0 and n + 1 < steps:
                ckpts[n + 1] = U.clone()
        ctx.solver, ctx.dt, ctx.steps, ctx.every, ctx.ckpts = solver, dt, steps, checkpoint_every, ckpts
        return U

    @staticmethod
    def backward(ctx, Ubar):
        s, dt, steps, every = ctx.solver, ctx.dt, ctx.steps, ctx.every
        Ubar = Ubar.detach().clone().contiguous()
        for s0 in sorted(ctx.ckpts, reverse=True):
            s1 = min(s0 + every, steps)
            states = [ctx.ckpts[s0]]
            for _ in range(s0, s1 - 1):
                u = states[-1].clone()
                s.rk3_step(u, dt)
                states.append(u)
            for n in range(s1 - 1, s0 - 1, -1):
                s.rk3_step_vjp(states[n - s0], Ubar, dt)
        return Ubar, None, None, None, None


def final_energy(solver, U0, dt, steps, checkpoint_every=10):
    """E = 1/2 ||u_N||^2 (the basis is orthonormal), differentiable w.r.t. U0."""
    UN = Rollout.apply(U0, solver, dt, steps, checkpoint_every)
    return 0.5 * (UN * UN).sum()
