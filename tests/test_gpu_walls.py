"""GPU parity with the oracle on channels with walls: periodic in x, no-flow walls at y = 0
and y = 1 (eq. (euler-3) with g = 0; with viscosity the free-slip scheme of Sec. 3, whose
viscous facet terms run over interior facets only).  The velocity space is BDM_k in
H_0(div) (eq. (space-3)): the hybrid-mixed solve enforces u.n = 0 on the walls through the
multipliers of the boundary facets."""
import numpy as np
import pytest
import torch

from inputs import RandomStreamField, channel_shear_layer, double_shear_layer, eval_broken_poly, random_broken_poly
from oracle.quadrature import triangle_rule

pytestmark = pytest.mark.gpu

from gpu_util import (broken_residual_on_oracle_basis, make_pair, project_field, rel_l2, transfer,  # noqa: E402
                      values_to_lib)


def _log(*a):
    print(*a, flush=True)


@pytest.mark.parametrize("precond", ["jacobi", "amg"])
@pytest.mark.parametrize("k,N,order", [(1, 4, "lex"), (2, 6, "morton"), (3, 5, "random"), (2, 12, "morton")])
def test_mass_solve_parity_with_walls(k, N, order, precond):
    orc, s, _, _ = make_pair(N, k, order=order, seed=N, walls=True, cg_rtol=1e-13, precond=precond)
    assert (s.mesh.facets()[:, 2] < 0).sum() == 2 * N
    coef = random_broken_poly(s.T, k, seed=30 + k)
    F = values_to_lib(s, lambda pts: eval_broken_poly(coef, pts))
    U, info = s.mass_solve(F)
    assert info.status == 0 and info.rel_residual <= 1e-13
    rule = triangle_rule(2 * k)
    U_orc = orc.mass_solve(orc.space.assemble(orc.space.load_vector(eval_broken_poly(coef, rule[0]), rule)))
    err = rel_l2(orc, s, U, U_orc)
    d = s.diagnostics(U)
    _log("walls mass solve", k, N, precond, "iters", info.iterations, "rel L2", err, d)
    assert err < 1e-10
    scale = np.sqrt(d["enstrophy"])
    # divergence-free, and the normal jump (on a wall: u.n itself) at rounding level
    assert d["max_div"] < 1e-11 * scale and d["max_normal_jump"] < 1e-11 * scale
    assert abs(d["energy"] - orc.energy(U_orc)) < 1e-10 * orc.energy(U_orc)


@pytest.mark.parametrize("k,N", [(1, 5), (2, 4), (3, 4)])
@pytest.mark.parametrize("nu", [0.0, 0.05])
def test_residual_parity_with_walls(k, N, nu):
    orc, s, _, _ = make_pair(N, k, nu=nu, order="random", seed=N, walls=True)
    U_orc = orc.project(RandomStreamField(seed=k + N, kmax=3))
    U = transfer(orc, U_orc, s)
    R_gpu = broken_residual_on_oracle_basis(orc, s, s.residual(U))
    R_orc = orc.res.broken(orc.space.local_coeffs(U_orc))
    err = np.abs(R_gpu - R_orc).max() / np.abs(R_orc).max()
    _log("walls residual", k, N, nu, err)
    assert err < 1e-11


@pytest.mark.parametrize("k,N,nu,steps,precond", [(1, 8, 1e-2, 6, "jacobi"), (2, 8, 0.0, 5, "amg"),
                                                  (3, 6, 1e-3, 3, "amg")])
def test_rk3_trajectory_parity_with_walls(k, N, nu, steps, precond):
    """TVD-RK3 on the channel: a shear layer against the walls (free-slip for nu > 0)."""
    orc, s, _, _ = make_pair(N, k, nu=nu, walls=True, cg_rtol=1e-13, precond=precond, extrapolate="adaptive")
    U0 = orc.project(lambda x, y: double_shear_layer(x, y, sharpness=20.0))
    U = transfer(orc, U0, s)
    dt = 0.1 / N / k ** 2
    Uo = U0
    for _ in range(steps):
        assert s.rk3_step(U, dt).status == 0
        Uo = orc.rk3_step(Uo, dt)
    err = rel_l2(orc, s, U, Uo)
    d = s.diagnostics(U)
    _log("walls rk3", k, N, nu, err, d)
    assert err < 1e-10
    assert d["max_div"] < 1e-11 and d["max_normal_jump"] < 1e-11


def test_channel_shear_layer_at_256_keeps_walls_and_energy():
    """Five steps of the 256x256 BDM_2 shear layer in the channel (the benchmark's size),
    from a field tangent to the walls: no flow through the walls, divergence-free to the
    absolute 1e-11 of the periodic benchmark and energy non-increasing.  (Projecting the
    torus's shear layer instead, whose u2 crosses the walls, leaves a divergence of
    rounding times the removed pressure, growing like N^2: 2.5e-11 at 256.)"""
    _, s, xyz, _ = make_pair(256, 2, oracle=False, walls=True, cg_rtol=1e-12, precond="amg", extrapolate="adaptive")
    U, vmax = project_field(s, xyz, channel_shear_layer)
    dt = 0.1 / 256 / (4 * vmax)
    e0 = s.diagnostics(U)["energy"]
    its = []
    for _ in range(5):
        info = s.rk3_step(U, dt)
        assert info.status == 0
        its.append(list(info.iterations))
    d = s.diagnostics(U)
    _log("channel 256 BDM_2", its, d)
    assert d["max_div"] < 1e-11 and d["max_normal_jump"] < 1e-11
    assert d["energy"] <= e0


def _div_free_dirs(orc, n, seed):
    rng = np.random.default_rng(seed)
    out = []
    for _ in range(n):
        d = orc.mass_solve(rng.standard_normal(orc.space.ndof))
        out.append(d / np.sqrt(d @ (orc.M @ d)))
    return out


@pytest.mark.parametrize("k,N", [(1, 5), (2, 4), (3, 3)])
def test_residual_vjp_parity_with_walls(k, N):
    """y . (J_L(u) d) through the residual's vector-Jacobian product equals the oracle's
    Jacobian product on the channel (no wall facet terms on either side)."""
    from oracle.adjoint import residual_jacobian
    orc, s, _, _ = make_pair(N, k, nu=0.01, order="random", seed=3, walls=True)
    U0 = orc.project(RandomStreamField(seed=2, kmax=3))
    U = transfer(orc, U0, s)
    J = residual_jacobian(orc, U0)
    for y_g, d_g in zip(_div_free_dirs(orc, 2, seed=7), _div_free_dirs(orc, 2, seed=8)):
        y, d = transfer(orc, y_g, s), transfer(orc, d_g, s)
        gpu = torch.dot(s.residual_vjp(U, y), d).item()
        ref = float(y_g @ (J @ d_g))
        _log("walls vjp", k, N, gpu, ref)
        assert abs(gpu - ref) < 1e-10 * (abs(ref) + 1e-3)


def test_rk3_step_vjp_with_walls_matches_finite_differences():
    orc, s, _, _ = make_pair(6, 2, nu=1e-3, walls=True, cg_rtol=1e-14)
    U0 = transfer(orc, orc.project(RandomStreamField(seed=0, kmax=3)), s)
    dt = 0.1 / 6 / 4
    w = transfer(orc, _div_free_dirs(orc, 1, seed=9)[0], s)
    for d_g in _div_free_dirs(orc, 2, seed=4):
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
        _log("walls step vjp", adj, fd)
        assert abs(adj - fd) < 1e-6 * abs(fd) + 1e-10


@pytest.mark.parametrize("precond", ["jacobi", "amg"])
@pytest.mark.parametrize("k,N,mf", [(1, 3, False), (2, 2, False), (2, 3, True)])
def test_walls_3d_mass_solve_parity(k, N, mf, precond):
    """Tetrahedral channel (walls at z = 0, 1): mass inversion against the oracle, also
    with the matrix-free product (boundary faces have one side in the face pass)."""
    orc, s, _, _ = make_pair(N, k, dim=3, order="random", seed=N, walls=True, cg_rtol=1e-13, precond=precond,
                             matrix_free=mf)
    assert (s.mesh.facets()[:, 2] < 0).sum() == 4 * N * N
    from gpu_util import to_dev
    from oracle.quadrature import poly_basis_nd
    Fb = np.random.default_rng(k).standard_normal((orc.mesh.T, 3, orc.space.nm))
    U_orc = orc.mass_solve(orc.space.assemble(Fb))
    pts, _ = s.proj_rule()
    vals, _ = poly_basis_nd(k, pts)
    # the functional Fb on the oracle's local basis, as values of a broken field whose
    # L2 products with m_a e_c are Fb (reference-orthonormal m_a: the field sum_a Fb m_a / det J)
    F = s.load_vector(to_dev(s, np.einsum("tca,qa->tcq", Fb / orc.mesh.detJ[:, None, None], vals)))
    U, info = s.mass_solve(F)
    assert info.status == 0 and info.rel_residual <= 1e-13
    err = rel_l2(orc, s, U, U_orc)
    d = s.diagnostics(U)
    _log("walls 3d mass solve", k, N, mf, precond, "iters", info.iterations, "rel L2", err, d)
    assert err < 1e-10
    scale = np.sqrt(d["enstrophy"])
    assert d["max_div"] < 1e-11 * scale and d["max_normal_jump"] < 1e-11 * scale


@pytest.mark.parametrize("k,N,nu,steps", [(1, 3, 0.0, 3), (2, 2, 1e-2, 2)])
def test_walls_3d_rk3_trajectory_parity(k, N, nu, steps):
    from inputs import taylor_green_3d
    orc, s, _, _ = make_pair(N, k, dim=3, nu=nu, walls=True, cg_rtol=1e-13, precond="amg", extrapolate="adaptive")
    U0 = orc.project(taylor_green_3d)
    U = transfer(orc, U0, s)
    R_gpu = broken_residual_on_oracle_basis(orc, s, s.residual(U))
    R_orc = orc.res.broken(orc.space.local_coeffs(U0))
    rerr = np.abs(R_gpu - R_orc).max() / np.abs(R_orc).max()
    dt = 0.1 / N / k ** 2
    Uo = U0
    for _ in range(steps):
        assert s.rk3_step(U, dt).status == 0
        Uo = orc.rk3_step(Uo, dt)
    err = rel_l2(orc, s, U, Uo)
    _log("walls 3d residual", rerr, "rk3", k, N, nu, err)
    assert rerr < 1e-11 and err < 1e-10


@pytest.mark.parametrize("precond", ["jacobi", "amg"])
def test_walls_grid_stride_and_mixed(precond):
    """The facet kernels' grid-stride path (facet_blocks = 1: one block walks all rows,
    boundary rows included) gives the single-pass result; the mixed-precision form on the
    channel stays within 1e-6 of FP64."""
    orc, s, xyz, _ = make_pair(16, 2, order="random", seed=3, walls=True, cg_rtol=1e-13, precond=precond,
                               facet_blocks=1)
    coef = random_broken_poly(s.T, 2, seed=61)
    F = values_to_lib(s, lambda pts: eval_broken_poly(coef, pts))
    U, info = s.mass_solve(F)
    rule = triangle_rule(4)
    U_orc = orc.mass_solve(orc.space.assemble(orc.space.load_vector(eval_broken_poly(coef, rule[0]), rule)))
    err = rel_l2(orc, s, U, U_orc)
    _log("walls grid stride", precond, info.iterations, err)
    assert info.status == 0 and err < 1e-10
    out = {}
    for prec in ("fp64", "mixed"):
        _, sm, xyz2, _ = make_pair(32, 2, nu=1e-3, oracle=False, walls=True, cg_rtol=1e-10, precond=precond,
                                   precision=prec, ir_rtol=1e-10)
        V, vmax = project_field(sm, xyz2, channel_shear_layer)
        for _ in range(3):
            assert sm.rk3_step(V, 0.1 / 32 / (4 * vmax)).status == 0
        out[prec] = V
        del sm
    errm = ((out["mixed"] - out["fp64"]).norm() / out["fp64"].norm()).item()
    _log("walls mixed vs fp64", precond, errm)
    assert errm < 1e-6
