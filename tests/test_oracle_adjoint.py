"""Pins of the oracle's reverse-mode gradient: Jacobian of L and dE/dU0 vs central
finite differences of the forward oracle."""
import numpy as np
import pytest

from inputs import RandomStreamField, periodic_split_square
from oracle import Oracle
from oracle.adjoint import energy_and_gradient, residual_jacobian


def _setup(N=5, k=2, nu=1e-3, walls=False):
    xyz, per = periodic_split_square(N, "random", seed=1)
    orc = Oracle(xyz, np.array([1.0, 0.0]) if walls else per, k, nu=nu)
    U0 = orc.project(RandomStreamField(seed=0, kmax=3))
    return orc, U0


def _directions(orc, n, seed=1):
    rng = np.random.default_rng(seed)
    out = []
    for _ in range(n):
        d = orc.mass_solve(rng.standard_normal(orc.space.ndof))  # in V^{k,-1}
        out.append(d / np.sqrt(d @ (orc.M @ d)))
    return out


@pytest.mark.parametrize("walls", [False, True])
@pytest.mark.parametrize("k", [1, 2, 3])
def test_residual_jacobian_matches_finite_differences(k, walls):
    """Also on the channel with walls at y = 0, 1, where the space has no normal moments on
    the wall facets."""
    orc, U0 = _setup(N=4, k=k, nu=0.01, walls=walls)
    assert orc.mesh.bnd.any() == walls
    J = residual_jacobian(orc, U0)
    for d in _directions(orc, 3):
        h = 1e-6
        fd = (orc.L(U0 + h * d) - orc.L(U0 - h * d)) / (2 * h)
        assert np.abs(J @ d - fd).max() < 1e-6 * np.abs(fd).max()


def test_energy_gradient_matches_finite_differences():
    orc, U0 = _setup()
    dt, steps = 0.01, 5
    E, g = energy_and_gradient(orc, U0, dt, steps, checkpoint_every=2)

    def energy(U):
        return orc.energy(orc.run(U, dt, steps))

    assert abs(E - energy(U0)) < 1e-14 * E
    for d in _directions(orc, 4, seed=3):
        h = 1e-6
        fd = (energy(U0 + h * d) - energy(U0 - h * d)) / (2 * h)
        assert abs(g @ d - fd) < 1e-6 * abs(fd) + 1e-12, (g @ d, fd)


def _lift3(x, y, z):
    return 0.8 + 0 * x, 0.15 + 0 * y, -0.1 + 0 * z


@pytest.mark.parametrize("kind,k", [("periodic", 1), ("periodic", 2), ("walls", 1), ("walls", 2), ("inout", 1)])
def test_residual_jacobian_matches_finite_differences_3d(kind, k):
    """Tetrahedra: the periodic cube, the channel with walls at z = 0, 1 (no normal moments
    on the wall faces), and the cube with an inflow at x = 0 (a constant lift) and an outflow
    at x = 1 (the outgoing flux and its kink at u.n = 0)."""
    from inputs import (RandomVectorPotentialField, channel_kuhn_cube, inout_kuhn_cube, outflow_at_right,
                        periodic_kuhn_cube)
    gen = {"periodic": periodic_kuhn_cube, "walls": channel_kuhn_cube, "inout": inout_kuhn_cube}[kind]
    xyz, per = gen(2, "random", 2)
    kw = dict(outflow=outflow_at_right, inflow=_lift3) if kind == "inout" else {}
    orc = Oracle(xyz, per, k, nu=0.01, **kw)
    assert orc.mesh.bnd.any() == (kind != "periodic")
    U0 = orc.project(RandomVectorPotentialField(seed=1, kmax=2, norm=0.5))
    J = residual_jacobian(orc, U0)
    for d in _directions(orc, 2, seed=4):
        h = 1e-6
        fd = (orc.L(U0 + h * d) - orc.L(U0 - h * d)) / (2 * h)
        assert np.abs(J @ d - fd).max() < 1e-6 * np.abs(fd).max()
