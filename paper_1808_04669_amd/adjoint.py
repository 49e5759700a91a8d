"""Differentiation form: gradient of the final kinetic energy w.r.t. the initial velocity.

``Rollout`` is a ``torch.autograd.Function`` around `steps` TVD-RK3 steps of the library.
The forward pass keeps the state and the solver's warm-start history every
`checkpoint_every` steps (and all stage states of the last segment, which the reverse
sweep needs first); the backward pass recomputes each other segment from its checkpoint
with ``dfdg_rk3_step_stages`` (the same solves as the forward pass, keeping the
stage states of every step of the segment) and runs ``dfdg_rk3_step_vjp_stages`` (the
hand-written adjoint of the residual and the self-adjoint mass solve) in reverse, so a
step costs three forward and three adjoint stage solves in the reverse sweep.
All arithmetic runs in the library's kernels; this module only orders the calls.
"""
import torch


class Rollout(torch.autograd.Function):
    @staticmethod
    def forward(ctx, U0, solver, dt, steps, checkpoint_every):
        U = U0.detach().clone()
        solver.reset_history()
        ckpts = {0: (U.clone(), solver.history_save())}
        last = ((steps - 1) // checkpoint_every) * checkpoint_every  # start of the last segment
        tail = ([], [])  # states and stage states of the last segment, kept from this pass
        for n in range(steps):
            if n >= last:
                U1, U2 = torch.empty_like(U), torch.empty_like(U)
                tail[0].append(U.clone())
                solver.rk3_step_stages(U, dt, U1, U2)
                tail[1].append((U1, U2))
            else:
                solver.rk3_step(U, dt)
            if (n + 1) % checkpoint_every == 0 and n + 1 < steps:
                ckpts[n + 1] = (U.clone(), solver.history_save())
        ctx.solver, ctx.dt, ctx.steps, ctx.every, ctx.ckpts = solver, dt, steps, checkpoint_every, ckpts
        ctx.tail = (last, tail)
        return U

    @staticmethod
    def backward(ctx, Ubar):
        s, dt, steps, every = ctx.solver, ctx.dt, ctx.steps, ctx.every
        Ubar = Ubar.detach().clone().contiguous()
        s.reset_adjoint_history()
        for s0 in sorted(ctx.ckpts, reverse=True):
            s1 = min(s0 + every, steps)
            # recompute the segment from its checkpoint (state and warm-start history, so
            # that the solves repeat the forward ones), keeping every step's stage states
            if s0 == ctx.tail[0]:
                states, stages = ctx.tail[1]
            else:
                U_ck, hist = ctx.ckpts[s0]
                s.history_restore(hist)
                states, stages = [U_ck], []
                for _ in range(s0, s1):
                    u = states[-1].clone()
                    U1, U2 = torch.empty_like(u), torch.empty_like(u)
                    s.rk3_step_stages(u, dt, U1, U2)
                    states.append(u)
                    stages.append((U1, U2))
            for n in range(s1 - 1, s0 - 1, -1):
                U1, U2 = stages[n - s0]
                s.rk3_step_vjp_stages(states[n - s0], U1, U2, Ubar, dt)
        s.reset_history()
        return Ubar, None, None, None, None


def final_energy(solver, U0, dt, steps, checkpoint_every=10):
    """E = 1/2 ||u_N||^2 (the basis is orthonormal), differentiable w.r.t. U0."""
    UN = Rollout.apply(U0, solver, dt, steps, checkpoint_every)
    return 0.5 * (UN * UN).sum()
