"""GPU parity with the oracle on the square with an inflow boundary at x = 0 and an outflow
boundary at x = 1, periodic in y (Sec. 2.5): the state is a lift carrying the inflow's
normal velocity plus an increment closed at the inflow; outflow facets have no multiplier
(p = 0) and keep the outgoing convective flux."""
import numpy as np
import pytest
import torch

from inputs import RandomStreamField, eval_broken_poly, random_broken_poly
from oracle.quadrature import triangle_rule

pytestmark = pytest.mark.gpu

from gpu_util import (broken_residual_on_oracle_basis, make_pair, project_field, rel_l2, transfer,  # noqa: E402
                      values_to_lib)


def _log(*a):
    print(*a, flush=True)


def _lift(x, y):  # uniform: u.n = -0.8 on the inflow boundary
    return 0.8 + 0 * x, 0.15 + 0 * y


@pytest.mark.parametrize("precond", ["jacobi", "amg"])
@pytest.mark.parametrize("k,N", [(1, 5), (2, 4), (3, 3), (2, 16)])
def test_inout_mass_solve_parity(k, N, precond):
    orc, s, _, _ = make_pair(N, k, order="random", seed=N, inout=True, cg_rtol=1e-13, precond=precond)
    assert s.mesh.open.sum() == N
    coef = random_broken_poly(s.T, k, seed=50 + k)
    F = values_to_lib(s, lambda pts: eval_broken_poly(coef, pts))
    U, info = s.mass_solve(F)
    assert info.status == 0 and info.rel_residual <= 1e-13
    rule = triangle_rule(2 * k)
    U_orc = orc.mass_solve(orc.space.assemble(orc.space.load_vector(eval_broken_poly(coef, rule[0]), rule)))
    err = rel_l2(orc, s, U, U_orc)
    d = s.diagnostics(U)
    _log("inout mass solve", k, N, precond, "iters", info.iterations, "rel L2", err, d)
    assert err < 1e-10
    scale = np.sqrt(d["enstrophy"])
    assert d["max_div"] < 1e-11 * scale and d["max_normal_jump"] < 1e-11 * scale


@pytest.mark.parametrize("k,N", [(1, 5), (2, 4), (3, 3)])
@pytest.mark.parametrize("nu", [0.0, 0.05])
def test_inout_residual_parity(k, N, nu):
    """Residual of a state with inflow, outflow and backflow (the random part exceeds the
    mean flow in places) on every broken test function."""
    orc, s, _, _ = make_pair(N, k, nu=nu, order="random", seed=N, inout=True, inflow=_lift)
    U_orc = orc.project(RandomStreamField(seed=k + N, kmax=3))
    U = transfer(orc, U_orc, s)
    R_gpu = broken_residual_on_oracle_basis(orc, s, s.residual(U))
    R_orc = orc.res.broken(orc.state_local(U_orc))
    err = np.abs(R_gpu - R_orc).max() / np.abs(R_orc).max()
    _log("inout residual", k, N, nu, err)
    assert err < 1e-11


@pytest.mark.parametrize("k,N,nu,steps,precond", [(1, 8, 1e-2, 5, "jacobi"), (2, 6, 0.0, 4, "amg"),
                                                  (3, 5, 1e-3, 3, "amg")])
def test_inout_rk3_trajectory_parity(k, N, nu, steps, precond):
    orc, s, _, _ = make_pair(N, k, nu=nu, inout=True, inflow=_lift, cg_rtol=1e-13, precond=precond,
                             extrapolate="adaptive")
    U0 = orc.project(RandomStreamField(seed=7, kmax=2, norm=0.3))
    U = transfer(orc, U0, s)  # the full state: lift + increment
    dt = 0.1 / N / k ** 2
    Uo = U0
    for _ in range(steps):
        assert s.rk3_step(U, dt).status == 0
        Uo = orc.rk3_step(Uo, dt)
    err = rel_l2(orc, s, U, Uo)
    _log("inout rk3", k, N, nu, err)
    assert err < 1e-10


@pytest.mark.parametrize("k,N", [(1, 5), (2, 4)])
def test_inout_residual_vjp_parity(k, N):
    from oracle.adjoint import residual_jacobian
    orc, s, _, _ = make_pair(N, k, nu=0.01, order="random", seed=4, inout=True, inflow=_lift)
    U0 = orc.project(RandomStreamField(seed=3, kmax=2))
    U = transfer(orc, U0, s)
    J = residual_jacobian(orc, U0)
    rng = np.random.default_rng(12)
    for _ in range(2):
        y_g, d_g = (orc.mass_solve(rng.standard_normal(orc.space.ndof)) for _ in range(2))
        y, d = (s.load_vector(values_to_lib_raw(orc, s, v)) for v in (y_g, d_g))
        gpu = torch.dot(s.residual_vjp(U, y), d).item()
        ref = float(y_g @ (J @ d_g))
        _log("inout vjp", k, N, gpu, ref)
        assert abs(gpu - ref) < 1e-10 * (abs(ref) + 1e-3)


def values_to_lib_raw(orc, s, V):
    """Values at the projection points of an increment V alone (no lift)."""
    from gpu_util import to_dev
    pts, _ = s.proj_rule()
    return to_dev(s, orc.space.eval_ref(V, pts))


def test_uniform_flow_steady_at_256_bdm2():
    """u = (1, 0) through the 256x256 BDM_2 square, inflow at x = 0, outflow at x = 1: five
    TVD-RK3 steps keep it to rounding (an exact steady solution)."""
    _, s, xyz, _ = make_pair(256, 2, oracle=False, inout=True, cg_rtol=1e-12, precond="amg", extrapolate="adaptive")
    U = values_to_lib(s, lambda pts: np.stack([np.ones((s.T, len(pts))), np.zeros((s.T, len(pts)))], axis=1))
    U0 = U.clone()
    for _ in range(5):
        assert s.rk3_step(U, 0.1 / 256 / 4).status == 0
    err = ((U - U0).norm() / U0.norm()).item()
    _log("uniform flow 256", err)
    assert err < 1e-12


def test_inflow_outflow_shear_layer_at_256_bdm2():
    """A perturbed stream through the 256x256 BDM_2 square for 10 steps: the uniform lift
    (1, 0) plus 0.2 times the channel shear layer turned by 90 degrees (divergence-free,
    u1 = 0 on x = 0 and x = 1).  Converged solves, divergence at rounding, interior normal
    jumps at rounding (the diagnostic's maximum is the inflow's |u.n| = 1, a closed
    boundary facet's u.n), and the inflow's normal velocity unchanged."""
    from inputs import channel_shear_layer
    _, s, xyz, _ = make_pair(256, 2, oracle=False, inout=True, cg_rtol=1e-12, precond="amg", extrapolate="adaptive")
    lift = values_to_lib(s, lambda pts: np.stack([np.ones((s.T, len(pts))), np.zeros((s.T, len(pts)))], axis=1))

    def turned(x, y):
        u, v = channel_shear_layer(y, x)
        return 0.2 * v, 0.2 * u

    P, vmax = project_field(s, xyz, turned)
    U = lift + P
    U_init = U.clone()
    its = []
    for _ in range(10):
        info = s.rk3_step(U, 0.1 / 256 / (4 * (1 + vmax)))
        assert info.status == 0
        its.append(list(info.iterations))
    d = s.diagnostics(U)
    _log("inout 256", its, d)
    assert d["max_div"] < 1e-11 and abs(d["max_normal_jump"] - 1.0) < 1e-11
    # the inflow's normal velocity is the initial state's: the change of u1 at the midpoints
    # of the facets on x = 0 vanishes (local facet f joins reference vertices f+1 and f+2)
    from gpu_util import gpu_vals
    refmid = np.array([[0.5, 0.5], [0.0, 0.5], [0.5, 0.0]])
    dv = gpu_vals(s, U - U_init, refmid)  # [T, 2, 3]
    fac = s.mesh.facets()
    inflow = np.nonzero((fac[:, 2] < 0) & ~s.mesh.open)[0]
    assert inflow.size == 256
    change = np.abs(dv[fac[inflow, 0], 0, fac[inflow, 1]]).max()
    _log("inflow normal velocity change", change, "state change", float((U - U_init).abs().max()))
    assert change < 1e-12


def _lift3(x, y, z):
    return 0.8 + 0 * x, 0.15 + 0 * y, -0.1 + 0 * z


@pytest.mark.parametrize("precond,mf", [("jacobi", False), ("amg", False), ("amg", True)])
@pytest.mark.parametrize("k,N", [(1, 3), (2, 2)])
def test_inout_3d_mass_solve_parity(k, N, precond, mf):
    """Tetrahedra, inflow at x = 0 and outflow at x = 1: mass inversion against the oracle,
    also with the matrix-free product (the outflow rows' identity blocks in the face pass)."""
    from gpu_util import to_dev
    from oracle.quadrature import poly_basis_nd
    orc, s, _, _ = make_pair(N, k, dim=3, order="random", seed=N, inout=True, cg_rtol=1e-13, precond=precond,
                             matrix_free=mf)
    assert s.mesh.open.sum() == 2 * N * N
    Fb = np.random.default_rng(k).standard_normal((orc.mesh.T, 3, orc.space.nm))
    U_orc = orc.mass_solve(orc.space.assemble(Fb))
    pts, _ = s.proj_rule()
    vals, _ = poly_basis_nd(k, pts)
    F = s.load_vector(to_dev(s, np.einsum("tca,qa->tcq", Fb / orc.mesh.detJ[:, None, None], vals)))
    U, info = s.mass_solve(F)
    assert info.status == 0 and info.rel_residual <= 1e-13
    err = rel_l2(orc, s, U, U_orc)
    _log("inout 3d mass solve", k, N, precond, mf, "iters", info.iterations, "rel L2", err)
    assert err < 1e-10


@pytest.mark.parametrize("k,N,nu,steps", [(1, 3, 0.0, 3), (2, 2, 1e-2, 2)])
def test_inout_3d_residual_and_rk3_parity(k, N, nu, steps):
    from inputs import abc_flow
    orc, s, _, _ = make_pair(N, k, dim=3, nu=nu, inout=True, inflow=_lift3, cg_rtol=1e-13, precond="amg",
                             extrapolate="adaptive")
    U0 = orc.project(lambda x, y, z: tuple(0.3 * c for c in abc_flow(x, y, z)))
    U = transfer(orc, U0, s)
    R_gpu = broken_residual_on_oracle_basis(orc, s, s.residual(U))
    R_orc = orc.res.broken(orc.state_local(U0))
    rerr = np.abs(R_gpu - R_orc).max() / np.abs(R_orc).max()
    dt = 0.1 / N / k ** 2
    Uo = U0
    for _ in range(steps):
        assert s.rk3_step(U, dt).status == 0
        Uo = orc.rk3_step(Uo, dt)
    err = rel_l2(orc, s, U, Uo)
    _log("inout 3d residual", rerr, "rk3", k, N, nu, err)
    assert rerr < 1e-11 and err < 1e-10


@pytest.mark.parametrize("precond", ["jacobi", "amg"])
def test_inout_grid_stride_and_mixed(precond):
    """Grid-stride facet kernels (facet_blocks = 1) with outflow rows, against the oracle;
    the mixed-precision form of a stream through the square within 1e-6 of FP64."""
    orc, s, _, _ = make_pair(16, 2, order="random", seed=5, inout=True, cg_rtol=1e-13, precond=precond,
                             facet_blocks=1)
    coef = random_broken_poly(s.T, 2, seed=62)
    F = values_to_lib(s, lambda pts: eval_broken_poly(coef, pts))
    U, info = s.mass_solve(F)
    rule = triangle_rule(4)
    U_orc = orc.mass_solve(orc.space.assemble(orc.space.load_vector(eval_broken_poly(coef, rule[0]), rule)))
    err = rel_l2(orc, s, U, U_orc)
    _log("inout grid stride", precond, info.iterations, err)
    assert info.status == 0 and err < 1e-10
    from inputs import channel_shear_layer
    out = {}
    for prec in ("fp64", "mixed"):
        _, sm, xyz2, _ = make_pair(32, 2, nu=1e-3, oracle=False, inout=True, cg_rtol=1e-10, precond=precond,
                                   precision=prec, ir_rtol=1e-10)
        lift = values_to_lib(sm, lambda pts: np.stack([np.ones((sm.T, len(pts))), np.zeros((sm.T, len(pts)))], axis=1))

        def turned(x, y):
            u, v = channel_shear_layer(y, x)
            return 0.2 * v, 0.2 * u

        P, vmax = project_field(sm, xyz2, turned)
        V = lift + P
        for _ in range(3):
            assert sm.rk3_step(V, 0.1 / 32 / (4 * (1 + vmax))).status == 0
        out[prec] = V
        del sm
    errm = ((out["mixed"] - out["fp64"]).norm() / out["fp64"].norm()).item()
    _log("inout mixed vs fp64", precond, errm)
    assert errm < 1e-6


def test_inout_rk3_step_vjp_matches_finite_differences():
    """The RK3-step vector-Jacobian product with inflow and outflow (mass inversions closed
    at the inflow, open at the outflow; outgoing flux in the residual's transpose) against
    central differences along increments."""
    orc, s, _, _ = make_pair(6, 2, nu=1e-3, inout=True, inflow=_lift, cg_rtol=1e-14)
    U0 = transfer(orc, orc.project(RandomStreamField(seed=1, kmax=2, norm=0.3)), s)
    dt = 0.1 / 6 / 4
    rng = np.random.default_rng(21)

    def incr():
        d = orc.mass_solve(rng.standard_normal(orc.space.ndof))
        return s.load_vector(values_to_lib_raw(orc, s, d / np.sqrt(d @ (orc.M @ d))))

    w = incr()
    for _ in range(2):
        d = incr()
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
        _log("inout step vjp", adj, fd)
        assert abs(adj - fd) < 1e-6 * abs(fd) + 1e-10
