"""Pins of the oracle with walls: the channel periodic in x with no-flow walls at y = 0 and
y = 1 (eq. (euler-3) with g = 0; velocity space BDM_k in H_0(div), eq. (space-3); the
free-slip Navier-Stokes scheme of Sec. 3 sums its viscous facet terms over interior
facets only)."""
import numpy as np
import pytest
import scipy.linalg as sla

from inputs import periodic_split_square
from oracle import Oracle
from oracle.quadrature import triangle_rule
from oracle.scheme import hybrid_solve_dense

WALLS = np.array([1.0, 0.0])  # periodic in x, walls in y


def _oracle(N, k, nu=0.0):
    xyz, _ = periodic_split_square(N, "morton", seed=1)
    return Oracle(xyz, WALLS, k, nu=nu)


@pytest.mark.parametrize("N,k", [(2, 1), (3, 1), (2, 2), (3, 2), (2, 3)])
def test_divergence_free_dimension_on_the_channel(N, k):
    """dim{v in BDM_k, v.n = 0 on the walls, div v = 0} (SVD null space of the divergence)
    equals the count from the de Rham sequence of the periodic channel: such fields are the
    curls of continuous P^{k+1} stream functions that vanish on one wall and are constant
    on the other (that constant is the flux through the channel), i.e. the interior
    Lagrange nodes plus one."""
    o = _oracle(N, k)
    m = o.mesh
    assert m.T == 2 * N * N and m.bnd.sum() == 2 * N and m.E == 3 * N * N + N
    Z = sla.null_space(o.B.toarray())
    verts = N * (N - 1)                       # vertices off the walls
    edges = 3 * N * N - N                     # edges off the walls
    nodes = verts + k * edges + 2 * N * N * (k * (k - 1) // 2)
    assert Z.shape[1] == nodes + 1


@pytest.mark.parametrize("k", [1, 2, 3])
def test_mass_solve_equals_svd_nullspace_projection_with_walls(k):
    o = _oracle(3, k)
    Z = sla.null_space(o.B.toarray())
    M = o.M.toarray()
    f = np.random.default_rng(7).standard_normal(o.space.ndof)
    u = o.mass_solve(f)
    ub = Z @ np.linalg.solve(Z.T @ M @ Z, Z.T @ f)
    assert np.abs(u - ub).max() < 1e-12 * np.abs(ub).max()
    # divergence-free and no flow through the walls (the normal jump there is u.n itself)
    assert o.divergence_max(u) < 1e-11 * np.abs(u).max() * 3
    assert o.normal_jump_max(u) < 1e-11 * np.abs(u).max() * 3


@pytest.mark.parametrize("k", [1, 2, 3])
def test_hybrid_equals_mixed_with_walls(k):
    """Theorem 2 with walls: multipliers on the boundary facets enforce u.n = 0 there."""
    o = _oracle(2, k)
    Fb = np.random.default_rng(3).standard_normal((o.mesh.T, 2, o.space.nm))
    cu_h = hybrid_solve_dense(o, Fb)
    cu_m = o.space.local_coeffs(o.mass_solve(o.space.assemble(Fb)))
    assert np.abs(cu_h - cu_m).max() < 1e-11 * np.abs(cu_m).max()


@pytest.mark.parametrize("k", [1, 2, 3])
def test_channel_flow_projected_exactly_and_steady(k):
    """u = (c, 0) has u.n = 0 on the walls: it lies in the space, its projection is exact,
    and it is a steady solution (L(u) = 0: no gradients, no jumps, no boundary terms)."""
    o = _oracle(3, k, nu=0.01)
    U = o.project(lambda x, y: (0.7 + 0 * x, 0 * y))
    v = o.eval_ref(U, triangle_rule(4)[0])
    assert np.abs(v[:, 0] - 0.7).max() < 1e-13 and np.abs(v[:, 1]).max() < 1e-13
    assert np.abs(o.L(U)).max() < 1e-12


@pytest.mark.parametrize("k", [1, 2, 3])
def test_projection_removes_flow_through_the_walls(k):
    """A field crossing the walls is projected to one without normal flow there; a
    divergence-free field tangential at the walls is kept to the projection's accuracy."""
    o = _oracle(4, k)
    U = o.project(lambda x, y: (np.cos(2 * np.pi * y), 0.5 + 0.2 * np.sin(2 * np.pi * x)))
    assert o.normal_jump_max(U) < 1e-12 and o.divergence_max(U) < 1e-11


def test_convective_energy_identity_with_walls():
    """U . L_0(U) = -1/2 sum over interior facets of int |u.n| |u+ - u-|^2 <= 0: no
    boundary term, since u.n = 0 on the walls (the energy identity of Sec. 2.2)."""
    o = _oracle(4, 2)
    rng = np.random.default_rng(5)
    U = o.mass_solve(rng.standard_normal(o.space.ndof))
    e = float(U @ o.L(U))
    assert e <= 1e-13 * abs(e) + 1e-14
    assert e < -1e-8  # a random field jumps: strictly dissipative


def test_viscous_form_symmetric_and_dissipative_with_walls():
    """The interior-facet SIPG form is symmetric, and for k = 2 dissipative, on the
    channel (eq. (viscous) with the free-slip condition natural)."""
    o0, o1 = _oracle(3, 2, nu=0.0), _oracle(3, 2, nu=0.1)
    rng = np.random.default_rng(8)
    U, V = (o1.mass_solve(f) for f in rng.standard_normal((2, o1.space.ndof)))
    # L(u) - L_0(u) = -nu B_h(u, .): the convective parts are the same and cancel
    bUV = float(V @ (o1.L(U) - o0.L(U)))
    bVU = float(U @ (o1.L(V) - o0.L(V)))
    assert abs(bUV - bVU) < 1e-10 * max(abs(bUV), 1e-30)
    assert float(U @ (o1.L(U) - o0.L(U))) < 0


def test_channel_shear_layer_input_is_divergence_free_and_tangent():
    """The channel's shear-layer input: div u = 0 (complex-step derivatives, exact to
    rounding) and u.n = u2 = 0 on both walls."""
    from inputs import channel_shear_layer
    rng = np.random.default_rng(5)
    x, y = rng.random(200), rng.random(200)
    h = 1e-30
    du1dx = channel_shear_layer(x + 1j * h, y)[0].imag / h
    du2dy = channel_shear_layer(x, y + 1j * h)[1].imag / h
    assert np.abs(du1dx + du2dy).max() < 1e-14
    for yw in (0.0, 1.0):
        assert np.abs(channel_shear_layer(x, np.full_like(x, yw))[1]).max() < 1e-17


def _oracle3(N, k, nu=0.0):
    from inputs import channel_kuhn_cube
    xyz, per = channel_kuhn_cube(N, "random", seed=2)
    return Oracle(xyz, per, k, nu=nu)


@pytest.mark.parametrize("k", [1, 2])
def test_walls_3d_mass_solve_svd_and_theorem2(k):
    """Tetrahedral channel (periodic in x, y; walls at z = 0, 1): the mass inversion equals
    the SVD null-space projection, and the hybrid-mixed velocity the mixed one (Theorem 2);
    no flow through the walls."""
    o = _oracle3(2, k)
    assert o.mesh.bnd.sum() == 16
    Z = sla.null_space(o.B.toarray())
    M = o.M.toarray()
    f = np.random.default_rng(4).standard_normal(o.space.ndof)
    u = o.mass_solve(f)
    ub = Z @ np.linalg.solve(Z.T @ M @ Z, Z.T @ f)
    assert np.abs(u - ub).max() < 1e-11 * np.abs(ub).max()
    assert o.normal_jump_max(u) < 1e-11 * np.abs(u).max() * 3
    Fb = np.random.default_rng(5).standard_normal((o.mesh.T, 3, o.space.nm))
    cu_h = hybrid_solve_dense(o, Fb)
    cu_m = o.space.local_coeffs(o.mass_solve(o.space.assemble(Fb)))
    assert np.abs(cu_h - cu_m).max() < 1e-10 * np.abs(cu_m).max()


@pytest.mark.parametrize("k", [1, 2])
def test_walls_3d_channel_flow_steady_and_energy(k):
    """u = (a, b, 0) is tangent to the walls: projected exactly and steady; a random
    divergence-free field loses energy through the upwind jumps only (no wall term)."""
    o = _oracle3(2, k, nu=0.01)
    U = o.project(lambda x, y, z: (0.7 + 0 * x, -0.3 + 0 * y, 0 * z))
    assert np.abs(o.L(U)).max() < 1e-12
    o0 = _oracle3(2, k)
    V = o0.mass_solve(np.random.default_rng(6).standard_normal(o0.space.ndof))
    e = float(V @ o0.L(V))
    assert e < 0
