"""Pins of the oracle with inflow and outflow boundaries (Sec. 2.5): the unit square with
an inflow boundary at x = 0 (u.n given), an outflow boundary at x = 1 (p = 0, u.n free),
periodic in y.  The state is a fixed lift carrying the inflow data plus an increment in
the space whose normal moments vanish on the inflow boundary; on the outflow boundary the
convective term keeps the outgoing flux, -int max(u.n, 0) (u . v)."""
import numpy as np
import pytest
import scipy.linalg as sla

from inputs import RandomStreamField, inout_split_square, outflow_at_right
from oracle import Oracle
from oracle.quadrature import facet_rule, poly_basis_nd
from oracle.scheme import hybrid_solve_dense, hybrid_system_dense


def _oracle(N, k, nu=0.0, inflow=None, order="random"):
    xyz, per = inout_split_square(N, order, seed=3)
    return Oracle(xyz, per, k, nu=nu, outflow=outflow_at_right, inflow=inflow)


def test_boundary_facets_classified():
    o = _oracle(3, 1)
    m = o.mesh
    assert m.bnd.sum() == 6 and m.open.sum() == 3
    xm = m.PA.mean(axis=1)[:, 0]
    assert np.all(np.abs(xm[m.open] - 1.0) < 1e-12) and np.all(np.abs(xm[m.bnd & ~m.open]) < 1e-12)


def _broken_constraints(o):
    """Constraint rows on the broken coefficients [T][d][nm] (the oracle's local basis),
    written from the definitions: normal moments continuous across interior facets, zero on
    the inflow boundary, free on the outflow boundary; divergence zero on every element."""
    m, k, sp_ = o.mesh, o.k, o.space
    nu, nf, T = sp_.nu, sp_.nf, m.T
    s, w = facet_rule(2, k)  # exact for the degree-2k moment integrands
    xa, xb = m.facet_points(s)
    va, _ = poly_basis_nd(k, xa)
    vb, _ = poly_basis_nd(k, xb)
    s1 = np.asarray(s, dtype=float).reshape(-1)
    leg = np.stack([w * np.polynomial.legendre.legval(2 * s1 - 1, np.eye(nf)[j]) for j in range(nf)], axis=1)
    rows = []
    for F in range(m.E):
        if m.open[F]:
            continue
        for j in range(nf):
            r = np.zeros(T * nu)
            for c in range(2):
                a = m.fA_elem[F] * nu + c * sp_.nm
                r[a:a + sp_.nm] += m.normal[F, c] * (leg[:, j] @ va[F])
                if not m.bnd[F]:
                    b = m.fB_elem[F] * nu + c * sp_.nm
                    r[b:b + sp_.nm] -= m.normal[F, c] * (leg[:, j] @ vb[F])
            rows.append(r)
    K, nU, nW = hybrid_system_dense(o)
    D = -K[nU:nU + nW, :nU]
    return np.vstack(rows + [D])


@pytest.mark.parametrize("k", [1, 2, 3])
def test_mass_solve_equals_constrained_projection(k):
    """The mass inversion equals the M-orthogonal projection onto the null space (SVD) of
    the constraints written out on the broken space."""
    o = _oracle(3, k)
    Z = sla.null_space(_broken_constraints(o))
    Fb = np.random.default_rng(k).standard_normal((o.mesh.T, 2, o.space.nm))
    Mb = np.kron(np.diag(o.mesh.detJ), np.eye(o.space.nu))  # orthonormal reference modes
    ub = Z @ np.linalg.solve(Z.T @ Mb @ Z, Z.T @ Fb.reshape(-1))
    u = o.space.local_coeffs(o.mass_solve(o.space.assemble(Fb))).reshape(-1)
    assert np.abs(u - ub).max() < 1e-11 * np.abs(ub).max()


@pytest.mark.parametrize("k", [1, 2, 3])
def test_hybrid_equals_mixed_with_outflow(k):
    """Theorem 2 with no multiplier on the outflow boundary (there p = 0)."""
    o = _oracle(2, k)
    Fb = np.random.default_rng(3 + k).standard_normal((o.mesh.T, 2, o.space.nm))
    cu_h = hybrid_solve_dense(o, Fb)
    cu_m = o.space.local_coeffs(o.mass_solve(o.space.assemble(Fb)))
    assert np.abs(cu_h - cu_m).max() < 1e-11 * np.abs(cu_m).max()


@pytest.mark.parametrize("nu", [0.0, 0.01])
@pytest.mark.parametrize("k", [1, 2, 3])
def test_uniform_flow_is_steady(k, nu):
    """u = (c, 0) entering at x = 0 and leaving at x = 1 is an exact steady solution: the
    increment space gets no right-hand side (the residual acts on the inflow's normal
    component only), so RK3 keeps the state."""
    o = _oracle(3, k, nu=nu, inflow=lambda x, y: (0.8 + 0 * x, 0 * y))
    U = np.zeros(o.space.ndof)
    assert np.abs(o.mass_solve(o.L(U))).max() < 1e-12  # rounding of the k = 3 local bases
    U1 = o.rk3_step(U, 0.01)
    assert np.abs(U1).max() < 1e-12


def _oracle3(N, k, nu=0.0, inflow=None):
    from inputs import inout_kuhn_cube
    xyz, per = inout_kuhn_cube(N, "random", seed=3)
    return Oracle(xyz, per, k, nu=nu, outflow=outflow_at_right, inflow=inflow)


@pytest.mark.parametrize("k", [1, 2])
def test_tetrahedra_hybrid_equals_mixed_and_uniform_flow_steady(k):
    """On the Kuhn cube with inflow at x = 0 and outflow at x = 1 (periodic in y, z):
    Theorem 2 without outflow multipliers, and u = (c, 0, 0) is steady."""
    o = _oracle3(2, k)
    assert o.mesh.open.sum() == 8 and o.mesh.bnd.sum() == 16
    Fb = np.random.default_rng(k).standard_normal((o.mesh.T, 3, o.space.nm))
    cu_h = hybrid_solve_dense(o, Fb)
    cu_m = o.space.local_coeffs(o.mass_solve(o.space.assemble(Fb)))
    assert np.abs(cu_h - cu_m).max() < 1e-10 * np.abs(cu_m).max()
    o = _oracle3(2, k, nu=0.01, inflow=lambda x, y, z: (0.8 + 0 * x, 0 * y, 0 * z))
    U = np.zeros(o.space.ndof)
    assert np.abs(o.mass_solve(o.L(U))).max() < 1e-12


@pytest.mark.parametrize("dim", [2, 3])
def test_energy_balance_closed_form(dim):
    """u . L_0(u) = -(1/2 sum_interior int |u.n| |[u]|^2 + 1/2 int_out |u.n| |u|^2
    - 1/2 int_in (u.n) |u|^2) for u = lift + increment (div u = 0 element-wise; the facet
    integrals with the residual's facet rule)."""
    k = 2
    if dim == 2:
        o = _oracle(4, k, inflow=lambda x, y: (0.6 + 0 * x, 0 * y + 0.2))
        U = o.project(RandomStreamField(seed=2, kmax=2))
    else:
        o = _oracle3(2, k, inflow=lambda x, y, z: (0.6 + 0 * x, 0 * y + 0.2, 0 * z - 0.1))
        U = o.mass_solve(np.random.default_rng(3).standard_normal(o.space.ndof))
    cU = o.state_local(U)
    lhs = float(np.sum(o.res.broken(cU) * cU))
    m = o.mesh
    s, w = facet_rule(dim, k)
    xa, xb = m.facet_points(s)
    va, _ = poly_basis_nd(k, xa)
    vb, _ = poly_basis_nd(k, xb)
    uA = np.einsum("eca,era->erc", cU[m.fA_elem], va)
    uB = np.einsum("eca,era->erc", cU[m.fB_elem], vb)
    un = np.einsum("erc,ec->er", uA, m.normal)
    wq = w[None, :] * m.flen[:, None]
    interior = 0.5 * np.sum(wq * np.abs(0.5 * (un + np.einsum("erc,ec->er", uB, m.normal)))
                            * np.sum((uA - uB) ** 2, axis=2), axis=1)
    outflow = 0.5 * np.sum(wq * np.abs(un) * np.sum(uA ** 2, axis=2), axis=1)
    inflow = -0.5 * np.sum(wq * un * np.sum(uA ** 2, axis=2), axis=1)
    rhs = -(interior[~m.bnd].sum() + outflow[m.open].sum() + inflow[m.bnd & ~m.open].sum())
    assert abs(lhs - rhs) < 1e-12 * abs(rhs)
    assert inflow[m.bnd & ~m.open].sum() > 0  # the inflow carries energy in


def test_residual_jacobian_with_outflow_matches_finite_differences():
    """The Jacobian of L at a state with inflow and outflow (the outflow term's max(u.n, 0)
    included) against central differences of the forward residual."""
    from oracle.adjoint import residual_jacobian
    o = _oracle(3, 2, nu=0.01, inflow=lambda x, y: (0.7 + 0 * x, 0 * y))
    U0 = o.project(RandomStreamField(seed=4, kmax=2))
    J = residual_jacobian(o, U0)
    rng = np.random.default_rng(9)
    for _ in range(3):
        d = o.mass_solve(rng.standard_normal(o.space.ndof))
        h = 1e-6
        fd = (o.L(U0 + h * d) - o.L(U0 - h * d)) / (2 * h)
        assert np.abs(J @ d - fd).max() < 1e-6 * np.abs(fd).max()
