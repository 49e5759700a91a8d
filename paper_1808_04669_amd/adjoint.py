"""Differentiation form: gradient of the final kinetic energy w.r.t. the initial velocity.

``Rollout`` is a ``torch.autograd.Function`` around `steps` TVD-RK3 steps of the library.
The forward pass keeps the state and the solver's warm-start history every
`checkpoint_every` steps (and all stage states of the last segment, which the reverse
sweep needs first); the backward pass recomputes each other segment from its checkpoint
with ``dfdg_rk3_step_stages`` (the same solves as the forward pass, keeping the stage
states of every step of the segment) and runs ``dfdg_rk3_step_vjp_stages`` (the
hand-written adjoint of the residual and the self-adjoint mass solve) in reverse, so a
step costs three forward and three adjoint stage solves in the reverse sweep.

With a second solver context (`recompute_solver`: same mesh and parameters, its own HIP
stream), the recomputation of the next earlier segment runs on that context, from a
helper thread, while the reverse sweep of the current segment runs on the first one; the
two streams share the GPU.  Both contexts restore the same checkpointed history, so the
gradient is the same bit for bit.
All arithmetic runs in the library's kernels; this module only orders the calls.
"""
from concurrent.futures import ThreadPoolExecutor

import torch


def _recompute(solver, ckpt, dt, n_steps):
    """States U^{s0..s0+n-1} and stage states of a segment, from its checkpoint."""
    U_ck, hist = ckpt
    solver.history_restore(hist)
    states, stages = [U_ck], []
    for _ in range(n_steps):
        u = states[-1].clone()
        U1, U2 = torch.empty_like(u), torch.empty_like(u)
        solver.rk3_step_stages(u, dt, U1, U2)
        states.append(u)
        stages.append((U1, U2))
    return states, stages


class Rollout(torch.autograd.Function):
    @staticmethod
    def forward(ctx, U0, solver, dt, steps, checkpoint_every, recompute_solver=None):
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
        ctx.recompute = recompute_solver
        return U

    @staticmethod
    def backward(ctx, Ubar):
        s, dt, steps, every = ctx.solver, ctx.dt, ctx.steps, ctx.every
        Ubar = Ubar.detach().clone().contiguous()
        s.reset_adjoint_history()
        order = sorted(ctx.ckpts, reverse=True)
        seg_len = {s0: min(s0 + every, steps) - s0 for s0 in order}

        def sweep(s0, states, stages):
            for n in range(seg_len[s0] - 1, -1, -1):
                U1, U2 = stages[n]
                s.rk3_step_vjp_stages(states[n], U1, U2, Ubar, dt)

        r = ctx.recompute
        if r is None:
            for s0 in order:
                if s0 == ctx.tail[0]:
                    states, stages = ctx.tail[1]
                else:
                    states, stages = _recompute(s, ctx.ckpts[s0], dt, seg_len[s0])
                sweep(s0, states, stages)
        else:
            main = s.stream  # where the reverse sweep runs

            def helper(s0):
                with torch.cuda.stream(r.stream):
                    states, stages = _recompute(r, ctx.ckpts[s0], dt, seg_len[s0])
                    done = torch.cuda.Event()
                    done.record(r.stream)
                return states, stages, done

            with ThreadPoolExecutor(max_workers=1) as ex:
                cur = ctx.tail[1] if order[0] == ctx.tail[0] else _recompute(s, ctx.ckpts[order[0]], dt,
                                                                              seg_len[order[0]])
                for i, s0 in enumerate(order):
                    fut = ex.submit(helper, order[i + 1]) if i + 1 < len(order) else None
                    sweep(s0, *cur)
                    if fut is not None:
                        states, stages, done = fut.result()
                        main.wait_event(done)
                        for t in states[1:] + [x for pair in stages for x in pair]:
                            t.record_stream(main)  # made on the helper stream, used on this one
                        cur = (states, stages)
            r.reset_history()
        s.reset_history()
        return Ubar, None, None, None, None, None


class KineticEnergy(torch.autograd.Function):
    """E = 1/2 int |u|^2 of a state (dfdg_diagnostics), with its cotangent from
    dfdg_energy_vjp."""

    @staticmethod
    def forward(ctx, U, solver):
        ctx.solver = solver
        ctx.save_for_backward(U)
        return torch.tensor(solver.diagnostics(U)["energy"], dtype=torch.float64, device=U.device)

    @staticmethod
    def backward(ctx, gE):
        (U,) = ctx.saved_tensors
        return ctx.solver.energy_vjp(U, float(gE)), None


def final_energy(solver, U0, dt, steps, checkpoint_every=10, recompute_solver=None):
    """E = 1/2 ||u_N||^2 (the basis is orthonormal), differentiable w.r.t. U0.
    recompute_solver: optional second context (same mesh and parameters, another stream)
    that recomputes checkpoint segments concurrently with the reverse sweep."""
    UN = Rollout.apply(U0, solver, dt, steps, checkpoint_every, recompute_solver)
    return KineticEnergy.apply(UN, solver)
