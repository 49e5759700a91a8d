"""GPU parity of the reduced local space of eq. (FE4) (local_space="fe4": the locally
divergence-free element basis from stream-function curls, without the pressure w; remark
"More efficient implementation", Sec. 2.4) with the oracle, on meshes with distorted
vertices (every element its own Gram matrix), periodic and with walls, and with the FE3
route at the benchmark size."""
import numpy as np
import pytest
import torch

from inputs import RandomStreamField, double_shear_layer, eval_broken_poly, random_broken_poly
from oracle.quadrature import triangle_rule

pytestmark = pytest.mark.gpu

from gpu_util import make_pair, project_field, rel_l2, transfer, values_to_lib  # noqa: E402


def _log(*a):
    print(*a, flush=True)


@pytest.mark.parametrize("walls", [False, True])
@pytest.mark.parametrize("precond", ["jacobi", "amg"])
@pytest.mark.parametrize("k,N", [(1, 6), (2, 5), (3, 4), (2, 16)])
def test_fe4_mass_solve_parity(k, N, precond, walls):
    orc, s, _, _ = make_pair(N, k, order="random", seed=N, walls=walls, distort=0.15, cg_rtol=1e-13,
                             precond=precond, local_space="fe4")
    coef = random_broken_poly(s.T, k, seed=40 + k)
    F = values_to_lib(s, lambda pts: eval_broken_poly(coef, pts))
    U, info = s.mass_solve(F)
    assert info.status == 0 and info.rel_residual <= 1e-13
    rule = triangle_rule(2 * k)
    U_orc = orc.mass_solve(orc.space.assemble(orc.space.load_vector(eval_broken_poly(coef, rule[0]), rule)))
    err = rel_l2(orc, s, U, U_orc)
    d = s.diagnostics(U)
    _log("fe4 mass solve", k, N, precond, walls, "iters", info.iterations, "rel L2", err, d)
    assert err < 1e-10
    scale = np.sqrt(d["enstrophy"])
    assert d["max_div"] < 1e-11 * scale and d["max_normal_jump"] < 1e-11 * scale


@pytest.mark.parametrize("k,N,nu,steps,precond,walls", [(1, 8, 1e-2, 5, "jacobi", False), (2, 6, 0.0, 4, "amg", False),
                                                        (3, 5, 1e-3, 3, "amg", False), (2, 6, 1e-3, 4, "amg", True)])
def test_fe4_rk3_trajectory_parity(k, N, nu, steps, precond, walls):
    orc, s, _, _ = make_pair(N, k, nu=nu, walls=walls, distort=0.15, cg_rtol=1e-13, precond=precond,
                             extrapolate="adaptive", local_space="fe4")
    U0 = orc.project(RandomStreamField(seed=k + N, kmax=3))
    U = transfer(orc, U0, s)
    dt = 0.1 / N / k ** 2
    Uo = U0
    for _ in range(steps):
        assert s.rk3_step(U, dt).status == 0
        Uo = orc.rk3_step(Uo, dt)
    err = rel_l2(orc, s, U, Uo)
    _log("fe4 rk3", k, N, nu, walls, err)
    assert err < 1e-10


def test_fe4_equals_fe3_at_256_bdm2():
    """Five TVD-RK3 steps of the 256x256 BDM_2 double shear layer: the two local spaces
    give the same trajectory to rounding and the same iteration counts."""
    out, its = {}, {}
    for ls in ("fe3", "fe4"):
        _, s, xyz, _ = make_pair(256, 2, oracle=False, cg_rtol=1e-12, precond="amg", extrapolate="adaptive",
                                 local_space=ls)
        U, vmax = project_field(s, xyz, double_shear_layer)
        dt = 0.1 / 256 / (4 * vmax)
        its[ls] = []
        for _ in range(5):
            info = s.rk3_step(U, dt)
            assert info.status == 0
            its[ls].append(list(info.iterations))
        d = s.diagnostics(U)
        assert d["max_div"] < 1e-11 and d["max_normal_jump"] < 1e-11
        out[ls] = U
        del s
    err = ((out["fe4"] - out["fe3"]).norm() / out["fe3"].norm()).item()
    _log("fe4 vs fe3 at 256", err, its)
    assert err < 1e-11
    assert abs(sum(map(sum, its["fe4"])) - sum(map(sum, its["fe3"]))) <= 3


def test_fe4_mixed_precision_against_fp64():
    out = {}
    for prec in ("fp64", "mixed"):
        _, s, xyz, _ = make_pair(64, 2, nu=1e-3, oracle=False, distort=0.15, cg_rtol=1e-10, precond="amg",
                                 precision=prec, ir_rtol=1e-10, local_space="fe4")
        U, vmax = project_field(s, xyz, double_shear_layer)
        for _ in range(3):
            assert s.rk3_step(U, 0.1 / 64 / (4 * vmax)).status == 0
        out[prec] = U
        del s
    err = ((out["mixed"] - out["fp64"]).norm() / out["fp64"].norm()).item()
    _log("fe4 mixed vs fp64", err)
    assert err < 1e-6
    assert torch.isfinite(out["mixed"]).all()
