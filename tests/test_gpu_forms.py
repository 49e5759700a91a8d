"""GPU tests of the two extra forms: mixed precision and the adjoint."""
import numpy as np
import pytest
import torch

from inputs import RandomStreamField, double_shear_layer, eval_broken_poly, random_broken_poly
from oracle.adjoint import energy_and_gradient, residual_jacobian

pytestmark = pytest.mark.gpu

from gpu_util import make_pair, rel_l2, transfer, values_to_lib  # noqa: E402


def _log(*a):
    print(*a, flush=True)


# ---------------------------------------------------------------------------------------
# mixed precision: FP32 residual and inner iterations, FP64 refinement / recovery; both
# refinements (Krylov: FP64 PCG with the FP32 cycle; restarted: FP32 PCG + FP64 refinement)
# ---------------------------------------------------------------------------------------
@pytest.mark.parametrize("solver", ["krylov", "restarted"])
@pytest.mark.parametrize("k,N,precond", [(1, 6, "jacobi"), (2, 8, "jacobi"), (3, 5, "jacobi"), (2, 16, "amg"),
                                         (3, 10, "amg")])
def test_mixed_mass_solve_parity(k, N, precond, solver):
    orc, s, _, _ = make_pair(N, k, order="random", seed=1, precision="mixed", ir_rtol=1e-11, inner_rtol=1e-3,
                             precond=precond, mixed_solver=solver)
    coef = random_broken_poly(s.T, k, seed=7)
    F = values_to_lib(s, lambda pts: eval_broken_poly(coef, pts))
    U, info = s.mass_solve(F)
    _log("mixed mass", k, N, "refinements", info.refinements, "inner its", info.iterations, "res", info.rel_residual)
    assert info.status == 0 and info.refinements >= 1 and info.rel_residual <= 1e-11
    from oracle.quadrature import triangle_rule
    rule = triangle_rule(2 * k)
    U_orc = orc.mass_solve(orc.space.assemble(orc.space.load_vector(eval_broken_poly(coef, rule[0]), rule)))
    err = rel_l2(orc, s, U, U_orc)
    _log("  rel L2", err)
    assert err < 1e-9
    d = s.diagnostics(U)
    assert d["max_div"] < 1e-11 * np.sqrt(d["enstrophy"])


@pytest.mark.parametrize("solver", ["krylov", "restarted"])
@pytest.mark.parametrize("k,N,steps,precond", [(2, 8, 6, "jacobi"), (3, 6, 4, "jacobi"), (2, 16, 4, "amg")])
def test_mixed_trajectory_within_1e6_of_oracle(k, N, steps, precond, solver):
    orc, s, _, _ = make_pair(N, k, order="morton", precision="mixed", ir_rtol=1e-10, inner_rtol=1e-3,
                             precond=precond, mixed_solver=solver)
    U0 = orc.project(lambda x, y: double_shear_layer(x, y, sharpness=20.0))
    U = transfer(orc, U0, s)
    dt = 0.1 / N / k ** 2
    Uo = U0
    for _ in range(steps):
        info = s.rk3_step(U, dt)
        assert info.status == 0
        Uo = orc.rk3_step(Uo, dt)
    err = rel_l2(orc, s, U, Uo)
    d = s.diagnostics(U)
    _log("mixed rk3", k, N, "rel L2", err, "diag", d)
    assert err < 1e-6
    assert d["max_div"] < 1e-11


# ---------------------------------------------------------------------------------------
# adjoint
# ---------------------------------------------------------------------------------------
def _div_free_dirs(orc, n, seed=1):
    rng = np.random.default_rng(seed)
    out = []
    for _ in range(n):
        d = orc.mass_solve(rng.standard_normal(orc.space.ndof))
        out.append(d / np.sqrt(d @ (orc.M @ d)))
    return out


@pytest.mark.parametrize("k,N", [(1, 5), (2, 6), (3, 4)])
def test_residual_vjp_parity(k, N):
    """y . (J_L(u) d) through dfdg_dg_residual_vjp equals the oracle's Jacobian product."""
    orc, s, _, _ = make_pair(N, k, nu=0.01, order="random", seed=2)
    U0 = orc.project(RandomStreamField(seed=1, kmax=3))
    U = transfer(orc, U0, s)
    J = residual_jacobian(orc, U0)
    for y_g, d_g in zip(_div_free_dirs(orc, 2, seed=5), _div_free_dirs(orc, 2, seed=6)):
        y, d = transfer(orc, y_g, s), transfer(orc, d_g, s)
        gpu = torch.dot(s.residual_vjp(U, y), d).item()
        ref = float(y_g @ (J @ d_g))
        _log("vjp", k, N, gpu, ref)
        assert abs(gpu - ref) < 1e-10 * (abs(ref) + 1e-3)


def test_rk3_step_vjp_matches_finite_differences():
    orc, s, _, _ = make_pair(6, 2, nu=1e-3, order="morton", cg_rtol=1e-14)
    U0 = transfer(orc, orc.project(RandomStreamField(seed=0, kmax=3)), s)
    dt = 0.1 / 6 / 4
    w = transfer(orc, _div_free_dirs(orc, 1, seed=9)[0], s)
    for d_g in _div_free_dirs(orc, 3, seed=4):
        d = transfer(orc, d_g, s)
        h = 1e-6

        def step(u):
            v = u.clone()
            s.reset_history()
            s.rk3_step(v, dt)
            return v

        fd = torch.dot(w, step(U0 + h * d) - step(U0 - h * d)).item() / (2 * h)
        Ub = w.clone()
        s.rk3_step_vjp(U0, Ub, dt)
        adj = torch.dot(Ub, d).item()
        _log("step vjp", adj, fd)
        assert abs(adj - fd) < 1e-6 * abs(fd) + 1e-10


@pytest.mark.parametrize("precond", ["jacobi", "amg"])
def test_step_vjp_with_given_stages_equals_recomputing_vjp(precond):
    """rk3_step_vjp_stages(U^n, U1, U2) with the stage states left by rk3_step_stages gives
    the same cotangent as rk3_step_vjp (which recomputes them), and rk3_step_stages
    advances U exactly like rk3_step; several steps in a row exercise the warm-started
    adjoint solves."""
    orc, s, _, _ = make_pair(12, 2, nu=1e-3, order="random", seed=2, cg_rtol=1e-13, precond=precond,
                             extrapolate=2)
    U = transfer(orc, orc.project(RandomStreamField(seed=1, kmax=4)), s)
    dt = 0.1 / 12 / 4
    states, stages = [U.clone()], []
    s.reset_history()
    for _ in range(4):
        u = states[-1].clone()
        v = states[-1].clone()
        U1, U2 = torch.empty_like(u), torch.empty_like(u)
        s.rk3_step_stages(u, dt, U1, U2)
        states.append(u)
        stages.append((U1, U2))
    s.reset_history()
    ref = states[0].clone()
    for _ in range(4):
        s.rk3_step(ref, dt)
    assert (ref - states[-1]).norm().item() < 1e-11 * ref.norm().item()
    w = transfer(orc, _div_free_dirs(orc, 1, seed=5)[0], s)
    Ya, Yb = w.clone(), w.clone()
    s.reset_adjoint_history()
    for n in range(3, -1, -1):
        s.rk3_step_vjp_stages(states[n], stages[n][0], stages[n][1], Ya, dt)
        s.rk3_step_vjp(states[n], Yb, dt)
    err = (Ya - Yb).norm().item() / Yb.norm().item()
    _log("vjp stages vs recompute", precond, err)
    assert err < 1e-10
    with pytest.raises(Exception):
        s.rk3_step_vjp_stages(states[0], stages[0][0], stages[0][1], states[0], dt)  # Ubar aliases U^n


def test_history_restore_repeats_the_trajectory_bitwise():
    """With the state and the warm-start history restored at a checkpoint, the next steps
    repeat the original ones bit for bit (the kernels are deterministic and the PCG start
    is the same), which the checkpointed reverse sweep relies on."""
    _, s, xyz, _ = make_pair(16, 2, nu=1e-3, order="morton", oracle=False, cg_rtol=1e-12, precond="amg",
                             extrapolate=2)
    f = RandomStreamField(seed=3, kmax=4)

    def vals(pts):  # [T, 2, nq] values of f at reference points of every element
        x = xyz[:, None, 0, :] + (pts[None, :, 0, None] * (xyz[:, None, 1, :] - xyz[:, None, 0, :])
                                  + pts[None, :, 1, None] * (xyz[:, None, 2, :] - xyz[:, None, 0, :]))
        u1, u2 = f(x[..., 0], x[..., 1])
        return np.stack([u1, u2], axis=1)

    U = s.mass_solve(values_to_lib(s, vals))[0]
    dt = 0.1 / 16 / 4
    s.reset_history()
    for _ in range(4):
        s.rk3_step(U, dt)
    snap, U_ck = s.history_save(), U.clone()
    assert snap[1] == (4, 4, 4)
    its_a = [list(s.rk3_step(U, dt).iterations) for _ in range(3)]
    s.reset_history()  # a cold step in between must not matter after the restore
    V = U_ck.clone()
    s.rk3_step(V, dt)
    s.history_restore(snap)
    V = U_ck.clone()
    its_b = [list(s.rk3_step(V, dt).iterations) for _ in range(3)]
    _log("history restore", its_a, its_b)
    assert its_a == its_b
    assert torch.equal(U, V)
    from paper_1808_04669_amd.dfdg import HISTORY_DEPTH
    with pytest.raises(Exception):
        s.history_restore((snap[0], (HISTORY_DEPTH + 1, 0, 0)))


def test_pipelined_reverse_sweep_equals_sequential():
    """The reverse sweep with a second context recomputing segments on its own stream
    gives the same gradient bit for bit as the sequential sweep (both restore the same
    checkpointed warm-start history)."""
    from paper_1808_04669_amd import Solver
    from paper_1808_04669_amd.adjoint import final_energy
    orc, s, xyz, per = make_pair(16, 2, nu=1e-3, order="morton", cg_rtol=1e-12, precond="amg", extrapolate=2)
    r = Solver(xyz, per, 2, nu=1e-3, cg_rtol=1e-12, precond="amg", extrapolate=2, stream=torch.cuda.Stream())
    U0 = transfer(orc, orc.project(RandomStreamField(seed=2, kmax=4)), s)
    dt = 0.1 / 16 / 4
    grads = []
    for rec in (None, r):
        U = U0.clone().requires_grad_(True)
        final_energy(s, U, dt, 12, checkpoint_every=4, recompute_solver=rec).backward()
        torch.cuda.synchronize()
        grads.append(U.grad.clone())
    _log("pipelined vs sequential", (grads[0] - grads[1]).abs().max().item())
    assert torch.equal(grads[0], grads[1])


@pytest.mark.parametrize("precond", ["jacobi", "amg"])
def test_energy_gradient_vs_oracle_and_fd(precond):
    """Gradient of the final kinetic energy w.r.t. U0 through checkpointed RK3 steps."""
    from paper_1808_04669_amd.adjoint import final_energy
    N, k, steps, every = 6, 2, 6, 2
    orc, s, _, _ = make_pair(N, k, nu=1e-3, order="random", seed=3, cg_rtol=1e-14, precond=precond, extrapolate=2)
    U0o = orc.project(RandomStreamField(seed=0, kmax=3))
    dt = 0.1 / N / k ** 2
    E_o, g_o = energy_and_gradient(orc, U0o, dt, steps, checkpoint_every=every)
    U0 = transfer(orc, U0o, s).requires_grad_(True)
    E = final_energy(s, U0, dt, steps, checkpoint_every=every)
    E.backward()
    g = U0.grad
    _log("E gpu", E.item(), "E oracle", E_o)
    assert abs(E.item() - E_o) < 1e-10 * E_o
    for d_g in _div_free_dirs(orc, 4, seed=11):
        d = transfer(orc, d_g, s)
        gpu = torch.dot(g, d).item()
        ref = float(g_o @ d_g)
        h = 1e-6
        with torch.no_grad():
            fd = (final_energy(s, U0.detach() + h * d, dt, steps, every)
                  - final_energy(s, U0.detach() - h * d, dt, steps, every)).item() / (2 * h)
        _log("  dE.d gpu", gpu, "oracle", ref, "fd", fd)
        assert abs(gpu - ref) < 1e-8 * abs(ref) + 1e-12
        assert abs(gpu - fd) < 1e-6 * abs(fd) + 1e-10


def test_energy_and_its_cotangent_from_the_library():
    """The objective of the adjoint form: dfdg_diagnostics' energy is 1/2 U . U (orthonormal
    broken basis), and dfdg_energy_vjp gives Ebar U exactly (also in place)."""
    from paper_1808_04669_amd.adjoint import KineticEnergy
    orc, s, _, _ = make_pair(6, 2, order="random", seed=3)
    U = transfer(orc, orc.project(RandomStreamField(seed=0, kmax=3)), s)
    E = KineticEnergy.apply(U, s).item()
    ref = 0.5 * torch.dot(U, U).item()
    assert abs(E - ref) < 1e-14 * ref and abs(E - orc.energy(orc.project(RandomStreamField(seed=0, kmax=3)))) < 1e-12 * ref
    Ub = s.energy_vjp(U, 2.5)
    assert torch.equal(Ub, 2.5 * U)
    V = U.clone()
    s.energy_vjp(V, -0.5, V)
    assert torch.equal(V, -0.5 * U)
    from paper_1808_04669_amd.dfdg import DfdgError
    with pytest.raises(DfdgError):
        s.energy_vjp(U, float("nan"))


def test_adaptive_warm_start_order():
    """Adaptive warm starts (the extrapolation order chosen on the device per solve by a
    one-step backtest): identical runs are bitwise equal, the trajectory equals a
    fixed-order one to the solve tolerance, and once the history is full the initial
    residuals are no larger than those of the plain previous-multiplier start."""
    from gpu_util import project_field
    from inputs import taylor_green_2d
    runs = {}
    for name, order in (("a", "adaptive"), ("b", "adaptive"), ("o0", 0), ("o2", 2)):
        _, s, xyz, _ = make_pair(32, 2, nu=1e-3, order="morton", oracle=False, cg_rtol=1e-13, precond="amg",
                                 extrapolate=order)
        U, vmax = project_field(s, xyz, lambda x, y: taylor_green_2d(x, y))
        dt = 0.1 / 32 / (4 * vmax)
        its, r0 = [], []
        for _ in range(12):
            info = s.rk3_step(U, dt)
            assert info.status == 0
            its.append(list(info.iterations))
            r0.append(list(info.initial_rel_residual))
        runs[name] = (U, its, np.array(r0))
        _log("warm start", name, "iterations", its[-3:], "initial residual", runs[name][2][-3:].mean())
    Ua, itsa, r0a = runs["a"]
    Ub, itsb, _ = runs["b"]
    assert torch.equal(Ua, Ub) and itsa == itsb
    U2 = runs["o2"][0]
    assert (Ua - U2).norm().item() < 1e-11 * U2.norm().item()
    # steps 7..12: six kept multipliers per stage, every order up to 4 can be backtested
    assert r0a[6:].mean() <= runs["o0"][2][6:].mean()
