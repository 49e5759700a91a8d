"""GPU parity against the oracle on a 64x64 mesh (BDM_2, 8192 triangles, 12288 facets).

At this size every element kernel runs 64 blocks and every facet kernel 48, so the XCD
block remapping is not the identity, and the multigrid hierarchy has several levels.  Each
case also runs with the facet kernels capped at 13 blocks (``facet_blocks``), so that every
thread walks about four facet rows in the grid-stride loop that meshes above 262144 facets
take; the results must match the oracle the same way.

Tolerances: the FP64 targets, relative L2 1e-10 for velocities (facet PCG at rtol 1e-13),
1e-11 entrywise for the residual, and the diagnostics of Example 2 of Sec. 4 (energy,
enstrophy) plus max |div u| and the normal jump.
"""
import numpy as np
import pytest

from inputs import RandomStreamField, double_shear_layer, eval_broken_poly, random_broken_poly
from oracle.quadrature import triangle_rule

pytestmark = pytest.mark.gpu

from gpu_util import (broken_residual_on_oracle_basis, make_pair, rel_l2, transfer,  # noqa: E402
                      values_to_lib)

N, K = 64, 2
_ORC = {}


def _log(*a):
    print(*a, flush=True)


def _oracle(nu):
    if nu not in _ORC:
        from inputs import periodic_split_square
        from oracle import Oracle
        xyz, per = periodic_split_square(N)
        _ORC[nu] = Oracle(xyz, per, K, nu=nu)
    return _ORC[nu]


def _solver(nu=0.0, **kw):
    _, s, _, _ = make_pair(N, K, nu=nu, oracle=False, **kw)
    return s


@pytest.mark.parametrize("nu", [0.0, 1e-3])
def test_residual_parity_64(nu):
    """L(u)(v) for every broken test function (eqs. (adv), (viscous)) of a divergence-free u."""
    orc = _oracle(nu)
    s = _solver(nu=nu)
    U_orc = orc.project(RandomStreamField(seed=3, kmax=6))
    U = transfer(orc, U_orc, s)
    R_gpu = broken_residual_on_oracle_basis(orc, s, s.residual(U))
    R_orc = orc.res.broken(orc.space.local_coeffs(U_orc))
    err = np.abs(R_gpu - R_orc).max() / np.abs(R_orc).max()
    _log("residual 64x64 nu", nu, "max rel", err)
    assert err < 1e-11


@pytest.mark.parametrize("facet_blocks,fine_smooth", [(0, 1), (13, 1), (0, 2), (0, 3)])
@pytest.mark.parametrize("precond", ["amg", "jacobi"])
def test_mass_solve_parity_64(precond, facet_blocks, fine_smooth):
    """Divergence-free mass inversion of a random broken functional (Theorems 1-2); with
    the multigrid, also for two and three smoothing steps of the finest prolongator (rows of
    up to 8 entries packed in FP16, then the general padded rows)."""
    if precond == "jacobi" and fine_smooth > 1:
        pytest.skip("the prolongator steps belong to the multigrid")
    orc = _oracle(0.0)
    s = _solver(precond=precond, cg_rtol=1e-13, facet_blocks=facet_blocks, mg_fine_smooth=fine_smooth)
    coef = random_broken_poly(s.T, K, seed=17)
    F = values_to_lib(s, lambda pts: eval_broken_poly(coef, pts))
    U, info = s.mass_solve(F)
    assert info.status == 0 and info.rel_residual <= 1e-13
    rule = triangle_rule(2 * K)
    U_orc = orc.mass_solve(orc.space.assemble(orc.space.load_vector(eval_broken_poly(coef, rule[0]), rule)))
    err = rel_l2(orc, s, U, U_orc)
    d = s.diagnostics(U)
    _log("mass solve 64x64", precond, facet_blocks, fine_smooth, "iters", info.iterations, "rel L2", err, d)
    assert err < 1e-10
    assert d["max_div"] < 1e-11 and d["max_normal_jump"] < 1e-11
    assert abs(d["energy"] - orc.energy(U_orc)) < 1e-10 * orc.energy(U_orc)
    assert abs(d["enstrophy"] - orc.enstrophy(U_orc)) < 1e-10 * orc.enstrophy(U_orc)


@pytest.mark.parametrize("facet_blocks", [0, 13])
def test_rk3_parity_64(facet_blocks):
    """Three TVD-RK3 steps (eq. (rk3)) of the double shear layer, adaptive warm starts and
    the multigrid cycle, from the oracle's projected initial field; diagnostics compared."""
    orc = _oracle(0.0)
    s = _solver(precond="amg", cg_rtol=1e-13, extrapolate="adaptive", facet_blocks=facet_blocks)
    U0 = orc.project(double_shear_layer)
    U = transfer(orc, U0, s)
    dt = 0.1 / N / (K * K)
    Uo = U0
    for _ in range(3):
        info = s.rk3_step(U, dt)
        assert info.status == 0
        Uo = orc.rk3_step(Uo, dt)
    err = rel_l2(orc, s, U, Uo)
    d = s.diagnostics(U)
    _log("rk3 64x64 facet_blocks", facet_blocks, "rel L2", err, "iters", list(info.iterations), d)
    assert err < 1e-10
    assert d["max_div"] < 1e-11 and d["max_normal_jump"] < 1e-11
    assert abs(d["energy"] - orc.energy(Uo)) < 1e-10 * orc.energy(Uo)
    assert abs(d["enstrophy"] - orc.enstrophy(Uo)) < 1e-9 * orc.enstrophy(Uo)


@pytest.mark.parametrize("k,n", [(1, 5), (2, 64), (3, 6)])
def test_diagnostics_parity_broken_field(k, n):
    """dfdg_diagnostics on a random broken field (outside BDM_k, so every diagnostic is of
    order one) against the oracle's: energy and enstrophy are exact integrals on both
    sides; max |div u| is taken at the residual's volume-rule points and the normal jump at
    the facet rule's Gauss-Legendre points (exact for degree 3k), the same point sets."""
    from inputs import periodic_split_square
    from oracle import Oracle
    xyz, per = periodic_split_square(n, "random", seed=n)
    orc = Oracle(xyz, per, k)
    _, s, _, _ = make_pair(n, k, order="random", seed=n, oracle=False)
    coef = random_broken_poly(s.T, k, seed=31 + k)
    U = values_to_lib(s, lambda pts: eval_broken_poly(coef, pts))
    rule = triangle_rule(2 * k + 2)
    cU = orc.space.broken_project(eval_broken_poly(coef, rule[0]), rule)
    d = s.diagnostics(U)
    pts, _ = s.residual_rule()
    ref = {"energy": orc.energy_local(cU), "enstrophy": orc.enstrophy_local(cU),
           "max_div": orc.divergence_max_local(cU, pts), "max_normal_jump": orc.normal_jump_max_local(cU)}
    _log("diagnostics broken field", k, n, d, ref)
    for key, v in ref.items():
        assert abs(d[key] - v) < 1e-12 * abs(v) * 10, (key, d[key], v)
