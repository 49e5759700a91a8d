"""GPU parity of the tetrahedral path (d = 3) against the oracle, on periodic Kuhn-split
cubes small enough for the oracle's sparse direct solve, and properties that hold at any
size on larger meshes: the exact ABC flow's convergence order, symmetry and idempotence of
the mass solve, constant fields, divergence and normal jumps.

Tolerances: the FP64 targets (relative L2 1e-10 for velocities with the facet PCG at rtol
1e-13; 1e-11 entrywise for the residual; max |div u| and normal jumps below 1e-11).
"""
import numpy as np
import pytest
import torch

from inputs import (RandomVectorPotentialField, abc_flow, eval_broken_poly_3d, random_broken_poly_3d,
                    taylor_green_3d)
from oracle.quadrature import tet_rule

pytestmark = pytest.mark.gpu

from gpu_util import (broken_residual_on_oracle_basis, gpu_vals, make_pair, phys_points,  # noqa: E402
                      project_field, rel_l2, to_dev, transfer, values_to_lib)


def _log(*a):
    print(*a, flush=True)


@pytest.mark.parametrize("precond", ["jacobi", "block_jacobi", "amg", "amg_fp64_cycle", "jacobi_mf", "amg_mf"])
@pytest.mark.parametrize("k,N,order", [(1, 2, "lex"), (1, 3, "random"), (2, 2, "random"), (2, 3, "morton"),
                                       (1, 4, "morton")])
def test_mass_solve_parity_3d(k, N, order, precond):
    """Divergence-free mass inversion of a random broken functional on tetrahedra
    (Theorems 1-2)."""
    _log("mass solve 3d", k, N, order, precond)
    kw = {"amg_fp64_cycle": dict(precond="amg", mg_fp32=False), "jacobi_mf": dict(precond="jacobi", matrix_free=True),
          "amg_mf": dict(precond="amg", matrix_free=True)}.get(precond, dict(precond=precond))
    orc, s, _, _ = make_pair(N, k, order=order, seed=N, dim=3, cg_rtol=1e-13, **kw)
    coef = random_broken_poly_3d(s.T, k, seed=10 + k)
    F = values_to_lib(s, lambda pts: eval_broken_poly_3d(coef, pts))
    U, info = s.mass_solve(F)
    assert info.status == 0 and info.rel_residual <= 1e-13 and info.iterations > 0
    rule = tet_rule(2 * k)
    R = orc.space.load_vector(eval_broken_poly_3d(coef, rule[0]), rule)
    U_orc = orc.mass_solve(orc.space.assemble(R))
    err = rel_l2(orc, s, U, U_orc)
    d = s.diagnostics(U)
    _log("  iters", info.iterations, "rel L2", err, d)
    assert err < 1e-10
    scale = np.sqrt(d["enstrophy"])
    assert d["max_div"] < 1e-11 * scale and d["max_normal_jump"] < 1e-11 * scale
    assert abs(d["energy"] - orc.energy(U_orc)) < 1e-10 * orc.energy(U_orc)
    assert abs(d["enstrophy"] - orc.enstrophy(U_orc)) < 1e-9 * orc.enstrophy(U_orc)


@pytest.mark.parametrize("k,N", [(1, 3), (2, 2), (2, 3)])
@pytest.mark.parametrize("nu", [0.0, 0.05])
def test_residual_parity_3d(k, N, nu):
    """L(u)(v) on every broken test function for a divergence-free u (eqs. (adv),
    (viscous)) on tetrahedra."""
    _log("residual 3d", k, N, nu)
    orc, s, _, _ = make_pair(N, k, nu=nu, order="random", seed=N, dim=3)
    U_orc = orc.project(RandomVectorPotentialField(seed=k + N, kmax=2))
    U = transfer(orc, U_orc, s)
    R_gpu = broken_residual_on_oracle_basis(orc, s, s.residual(U))
    R_orc = orc.res.broken(orc.space.local_coeffs(U_orc))
    err = np.abs(R_gpu - R_orc).max() / np.abs(R_orc).max()
    _log("  max rel", err)
    assert err < 1e-11


@pytest.mark.parametrize("k", [1, 2])
def test_residual_parity_broken_field_3d(k):
    """The residual of a discontinuous random field, where the upwind choice matters at
    every face point."""
    orc, s, _, _ = make_pair(2, k, nu=0.02, order="random", seed=3, dim=3)
    coef = random_broken_poly_3d(s.T, k, seed=21)
    U = values_to_lib(s, lambda pts: eval_broken_poly_3d(coef, pts))
    rule = tet_rule(2 * k)
    cU = orc.space.broken_project(eval_broken_poly_3d(coef, rule[0]), rule)
    R_orc = orc.res.broken(cU)
    R_gpu = broken_residual_on_oracle_basis(orc, s, s.residual(U))
    err = np.abs(R_gpu - R_orc).max() / np.abs(R_orc).max()
    _log("broken residual 3d", k, err)
    assert err < 1e-11


@pytest.mark.parametrize("k,N,nu,field,steps,precond,mf", [
    (2, 3, 1.0 / 1600, "tg", 3, "jacobi", False),   # the 3D Taylor-Green workload's parameters, small mesh
    (2, 4, 1.0 / 1600, "tg", 3, "amg", False),
    (2, 4, 1.0 / 1600, "tg", 3, "amg", True),
    (1, 4, 0.0, "abc", 3, "jacobi", True),
    (2, 2, 1e-2, "rand", 2, "amg", False),
])
def test_rk3_trajectory_parity_3d(k, N, nu, field, steps, precond, mf):
    """TVD-RK3 trajectories (eq. (rk3)) on tetrahedra from the oracle's projected field."""
    _log("rk3 3d", k, N, nu, field, precond, "matrix free" if mf else "")
    orc, s, _, _ = make_pair(N, k, nu=nu, order="morton", dim=3, cg_rtol=1e-13, precond=precond,
                             extrapolate="adaptive", matrix_free=mf)
    f = {"tg": taylor_green_3d, "abc": abc_flow, "rand": RandomVectorPotentialField(seed=1, kmax=2)}[field]
    U0 = orc.project(f)
    U = transfer(orc, U0, s)
    dt = 0.1 / N / k ** 2
    Uo = U0
    for _ in range(steps):
        info = s.rk3_step(U, dt)
        assert info.status == 0
        Uo = orc.rk3_step(Uo, dt)
    err = rel_l2(orc, s, U, Uo)
    d = s.diagnostics(U)
    _log("  rel L2", err, "iters", list(info.iterations), d)
    assert err < 1e-10
    assert d["max_div"] < 1e-11 and d["max_normal_jump"] < 1e-11
    assert abs(d["energy"] - orc.energy(Uo)) < 1e-10 * orc.energy(Uo)
    assert abs(d["enstrophy"] - orc.enstrophy(Uo)) < 1e-9 * orc.enstrophy(Uo)


@pytest.mark.parametrize("k", [1, 2])
def test_diagnostics_parity_broken_field_3d(k):
    """dfdg_diagnostics on a random broken field against the oracle's: energy, enstrophy
    (vector curl), max |div u| at the residual volume rule's points, normal jump at the face
    rule's points."""
    orc, s, _, _ = make_pair(2, k, order="random", seed=4, dim=3)
    coef = random_broken_poly_3d(s.T, k, seed=31 + k)
    U = values_to_lib(s, lambda pts: eval_broken_poly_3d(coef, pts))
    rule = tet_rule(2 * k + 2)
    cU = orc.space.broken_project(eval_broken_poly_3d(coef, rule[0]), rule)
    d = s.diagnostics(U)
    pts, _ = s.residual_rule()
    ref = {"energy": orc.energy_local(cU), "enstrophy": orc.enstrophy_local(cU),
           "max_div": orc.divergence_max_local(cU, pts), "max_normal_jump": orc.normal_jump_max_local(cU)}
    _log("diagnostics 3d", k, d, ref)
    for key, v in ref.items():
        assert abs(d[key] - v) < 1e-11 * abs(v), (key, d[key], v)


def test_constant_field_exact_and_steady_3d():
    """A constant velocity is projected exactly and its residual vanishes (16^3, BDM_2)."""
    for nu in (0.0, 1e-3):
        _, s, xyz, _ = make_pair(16, 2, nu=nu, oracle=False, dim=3, cg_rtol=1e-12, precond="jacobi")
        U, _ = project_field(s, xyz, lambda x, y, z: (np.ones_like(x), 2.0 * np.ones_like(y), -0.5 * np.ones_like(z)))
        pts = np.array([[0.2, 0.3, 0.1], [0.1, 0.1, 0.6]])
        v = s.eval(U, pts).cpu().numpy()
        assert np.abs(v[0] - 1).max() < 1e-11 and np.abs(v[1] - 2).max() < 1e-11 and np.abs(v[2] + 0.5).max() < 1e-11
        L = s.residual(U)
        _log("constant field nu", nu, "max |L|", L.abs().max().item())
        assert L.abs().max().item() < 1e-11 * 5.25
        del s


def test_abc_flow_convergence_on_the_gpu():
    """The exact ABC flow (steady Euler solution): L2 error after a few steps on N = 4, 8,
    16 (BDM_2) decays at about order k + 1 = 3 -- a pin at sizes the oracle cannot reach."""
    errs = []
    for N in (4, 8, 16):
        _, s, xyz, _ = make_pair(N, 2, oracle=False, dim=3, cg_rtol=1e-13, precond="jacobi", extrapolate=2)
        U, vmax = project_field(s, xyz, abc_flow)
        dt = 0.02 / N
        for _ in range(4):
            assert s.rk3_step(U, dt).status == 0
        rule = tet_rule(8)
        g = gpu_vals(s, U, rule[0])  # [T, 3, q]
        x = phys_points(xyz, rule[0])
        ex = np.stack(abc_flow(x[..., 0], x[..., 1], x[..., 2]), axis=1)
        J = np.transpose(xyz[:, 1:] - xyz[:, :1], (0, 2, 1))
        det = np.linalg.det(J)
        errs.append(float(np.sqrt(np.einsum("q,t,tcq->", rule[1], det, (g - ex) ** 2))))
        del s
    rates = np.log2(np.array(errs[:-1]) / np.array(errs[1:]))
    _log("ABC errors", errs, "rates", rates)
    assert rates[-1] > 2.6


@pytest.mark.parametrize("precond", ["jacobi", "amg"])
def test_mass_solve_symmetric_idempotent_and_divergence_free_at_32(precond):
    """32^3 BDM_2 (the 3D Taylor-Green mesh, 196608 tetrahedra): g.P f = f.P g, P(P f) = P f,
    and a Taylor-Green trajectory (nu = 1/1600) stays divergence free with continuous
    normal components to 1e-11 while its energy decays."""
    _, s, xyz, _ = make_pair(32, 2, nu=1.0 / 1600, oracle=False, dim=3, cg_rtol=1e-12, precond=precond,
                             extrapolate=2)
    _log("32^3: T", s.T, "E", s.E, "n_bdm", s.n_bdm)
    g0 = torch.Generator(device="cpu").manual_seed(0)
    f = torch.randn(s.n_broken, generator=g0, dtype=torch.float64).to(s.device)
    g = torch.randn(s.n_broken, generator=g0, dtype=torch.float64).to(s.device)
    Pf, i1 = s.mass_solve(f)
    Pg, _ = s.mass_solve(g)
    _log("  cold random solve: iterations", i1.iterations)
    a, b = torch.dot(g, Pf).item(), torch.dot(f, Pg).item()
    assert abs(a - b) < 1e-9 * abs(a)
    PPf, _ = s.mass_solve(Pf)
    assert (PPf - Pf).norm().item() < 1e-9 * Pf.norm().item()
    U, vmax = project_field(s, xyz, taylor_green_3d)
    e0 = s.diagnostics(U)["energy"]
    dt = 0.1 / 32 / (4 * vmax)
    for _ in range(3):
        info = s.rk3_step(U, dt)
        assert info.status == 0
    d = s.diagnostics(U)
    _log("  TG 3 steps: iterations", list(info.iterations), d)
    assert d["max_div"] < 1e-11 and d["max_normal_jump"] < 1e-11
    assert d["energy"] < e0
    assert abs(e0 - 0.125) < 1e-6  # 1/2 ||u0||^2 = 1/2 (1/8 + 1/8) for the 3D Taylor-Green field


@pytest.mark.parametrize("precond", ["jacobi", "amg"])
def test_matrix_free_products_equal_the_assembled_matrix(precond):
    """The matrix-free products sum_T C_T W_T C_T^T p give the solves of the assembled S
    (12^3 BDM_2: same iteration count within one, velocities within 1e-12), and replaying
    their iterations from captured graphs repeats the eager launches bit for bit."""
    outs = {}
    for mf in (False, True):
        for graphs in ((True, False) if mf else (True,)):
            _, s, xyz, _ = make_pair(12, 2, nu=1e-3, oracle=False, dim=3, cg_rtol=1e-12, precond=precond,
                                     matrix_free=mf, graphs=graphs, extrapolate=2)
            g0 = torch.Generator(device="cpu").manual_seed(1)
            f = torch.randn(s.n_broken, generator=g0, dtype=torch.float64).to(s.device)
            Pf, info = s.mass_solve(f)
            U, _ = project_field(s, xyz, taylor_green_3d)
            its = [list(s.rk3_step(U, 0.002).iterations) for _ in range(3)]
            outs[(mf, graphs)] = (Pf.clone(), info.iterations, U.clone(), its)
            del s
    (P0, i0, U0, _), (P1, i1, U1, its1) = outs[(False, True)], outs[(True, True)]
    _log(precond, "assembled", i0, "matrix free", i1, "diff", ((P1 - P0).norm() / P0.norm()).item())
    assert abs(i1 - i0) <= 1
    assert ((P1 - P0).norm() / P0.norm()).item() < 1e-12
    assert ((U1 - U0).norm() / U0.norm()).item() < 1e-12
    P2, i2, U2, its2 = outs[(True, False)]
    assert torch.equal(P1, P2) and i1 == i2 and torch.equal(U1, U2) and its1 == its2


def test_time_kernel_and_binding_3d():
    """The measurement entry point runs the 7-slot SpMV and the tetrahedral residual."""
    _, s, xyz, _ = make_pair(8, 2, oracle=False, dim=3, precond="jacobi")
    U, _ = project_field(s, xyz, taylor_green_3d)
    s.residual(U)
    ms, b = s.time_kernel(0, reps=5)
    assert ms > 0 and b == s.E * (7 * 36 * 8 + 7 * 4 + 4 * 6 * 8)
    ms, b = s.time_kernel(2, reps=5)
    assert ms > 0 and b > 0
    _, smf, _, _ = make_pair(8, 2, oracle=False, dim=3, precond="jacobi", matrix_free=True)
    ms, b = smf.time_kernel(0, reps=5)
    assert ms > 0 and b == smf.T * (72 + 80 + 4 * 40 + 4 * 6 * 16 + 4 * 6 * 8) + smf.E * (8 + 6 * 6 * 8)
    assert s.to_tcp(U).shape == (3, 10, s.T)
    assert to_dev(s, np.zeros((s.T, 3, 2))).numel() == 6 * s.T
