"""Pins of the oracle's diagnostics and its broken L2 projection against plain calculus.

Energy and enstrophy are the quantities Example 2 of Sec. 4 reports (energy 1/2 ||u||^2,
enstrophy ||curl u||^2); max |div u| and the normal jump are the divergence-free checks.
Each pin computes the expected value without the oracle: closed-form integrals of
polynomials over the unit square, exact curls and divergences of polynomial fields, and
the Taylor-Green vortex's enstrophy 4 pi^2 on the unit torus.
"""
import numpy as np
import pytest

from inputs import eval_broken_poly, periodic_split_square, random_broken_poly, taylor_green_2d
from oracle import Oracle
from oracle.quadrature import poly_basis, triangle_rule

TWO_PI = 2.0 * np.pi


# ---- polynomials in (x, y) as coefficient arrays C[i, j] of x^i y^j -------------------------
def _pmul(A, B):
    out = np.zeros((A.shape[0] + B.shape[0] - 1, A.shape[1] + B.shape[1] - 1))
    for i in range(A.shape[0]):
        for j in range(A.shape[1]):
            out[i:i + B.shape[0], j:j + B.shape[1]] += A[i, j] * B
    return out


def _dx(C):
    return (C * np.arange(C.shape[0])[:, None])[1:, :] if C.shape[0] > 1 else np.zeros((1, C.shape[1]))


def _dy(C):
    return (C * np.arange(C.shape[1])[None, :])[:, 1:] if C.shape[1] > 1 else np.zeros((C.shape[0], 1))


def _padd(A, B):
    out = np.zeros((max(A.shape[0], B.shape[0]), max(A.shape[1], B.shape[1])))
    out[:A.shape[0], :A.shape[1]] += A
    out[:B.shape[0], :B.shape[1]] += B
    return out


def _int_unit_square(C):
    i = np.arange(C.shape[0])[:, None]
    j = np.arange(C.shape[1])[None, :]
    return float((C / ((i + 1) * (j + 1))).sum())


def _peval(C, x, y):
    return sum(C[i, j] * x ** i * y ** j for i in range(C.shape[0]) for j in range(C.shape[1]))


def _periodic_bdm_poly(k, seed):
    """A random global polynomial field of degree k whose normal component matches across
    the periodic boundary of the unit square (u1(0, y) = u1(1, y), u2(x, 0) = u2(x, 1)), so
    that it lies in the periodic BDM_k space: u1 = p(y) + x(1-x) q(x, y) and
    u2 = r(x) + y(1-y) s(x, y) with deg p, r <= k and deg q, s <= k - 2."""
    rng = np.random.default_rng(seed)
    U1 = np.zeros((k + 1, k + 1))
    U2 = np.zeros((k + 1, k + 1))
    U1[0, :] = rng.standard_normal(k + 1)
    U2[:, 0] = rng.standard_normal(k + 1)
    if k >= 2:
        bump = np.array([[0.0], [1.0], [-1.0]])  # x - x^2
        for d in range(k - 1):
            for q in range(d + 1):
                Q = np.zeros((d - q + 1, q + 1))
                Q[d - q, q] = rng.standard_normal()
                U1 = _padd(U1, _pmul(bump, Q))
                S = np.zeros((d - q + 1, q + 1))
                S[d - q, q] = rng.standard_normal()
                U2 = _padd(U2, _pmul(bump.T, S))
    return U1, U2


def _bdm_coefficients(o, U1, U2):
    """Global BDM_k coefficients of a field in BDM_k: its L2 projection onto BDM_k (the full
    space, not the divergence-free one), solved with the BDM mass matrix."""
    import scipy.sparse.linalg as spla
    rule = triangle_rule(2 * o.k + 2)
    x = o.phys_points(rule[0])
    f = np.stack([_peval(U1, x[..., 0], x[..., 1]), _peval(U2, x[..., 0], x[..., 1])], axis=1)
    rhs = o.space.assemble(o.space.load_vector(f, rule))
    return spla.spsolve(o.M.tocsc(), rhs)


@pytest.mark.parametrize("k", [1, 2, 3])
@pytest.mark.parametrize("N", [2, 3])
def test_diagnostics_of_a_polynomial_field_in_bdm(k, N):
    """Energy, enstrophy, max |div u| and the normal jump of a global polynomial field in
    the periodic BDM_k space, against closed-form integrals over the unit square."""
    xyz, per = periodic_split_square(N, "random", seed=N)
    o = Oracle(xyz, per, k)
    U1, U2 = _periodic_bdm_poly(k, seed=10 * k + N)
    U = _bdm_coefficients(o, U1, U2)
    energy = 0.5 * (_int_unit_square(_pmul(U1, U1)) + _int_unit_square(_pmul(U2, U2)))
    curl = _padd(_dx(U2), -_dy(U1))
    div = _padd(_dx(U1), _dy(U2))
    enstrophy = _int_unit_square(_pmul(curl, curl))
    assert abs(o.energy(U) - energy) < 1e-12 * energy
    assert abs(o.energy_local(o.space.local_coeffs(U)) - energy) < 1e-12 * energy
    assert abs(o.enstrophy(U) - enstrophy) < 1e-11 * max(enstrophy, 1.0)
    assert o.normal_jump_max(U) < 1e-12
    pts = np.array([[0.1, 0.2], [0.7, 0.1], [0.3, 0.3], [0.05, 0.9]])
    x = o.phys_points(pts)
    dmax = float(np.abs(_peval(div, x[..., 0], x[..., 1])).max())
    assert abs(o.divergence_max(U, pts) - dmax) < 1e-11 * max(dmax, 1.0)


@pytest.mark.parametrize("k", [1, 2])
def test_taylor_green_enstrophy_converges_to_4pi2(k):
    """The projected Taylor-Green vortex (curl = 4 pi sin 2 pi x sin 2 pi y on the unit
    torus) has enstrophy tending to (4 pi)^2 / 4 = 4 pi^2 as the mesh is refined.  The
    element-wise curl ignores the tangential jumps, which limits the rate to 2 for every k
    (observed 1.95-1.97 on the finest pair)."""
    errs = []
    for N in (8, 16, 32):
        xyz, per = periodic_split_square(N)
        o = Oracle(xyz, per, k)
        U = o.project(taylor_green_2d)
        errs.append(abs(o.enstrophy(U) - 4 * np.pi ** 2))
    rates = np.log2(np.array(errs[:-1]) / np.array(errs[1:]))
    assert rates[-1] > 1.8, (errs, rates)
    assert errs[-1] < 0.02 * 4 * np.pi ** 2


@pytest.mark.parametrize("k", [1, 2, 3])
def test_broken_project_reproduces_polynomials_and_is_orthogonal(k):
    """The element-wise L2 projection onto [P^k]^2 returns broken polynomials of degree k
    unchanged, and leaves a degree-(k+1) field with an error orthogonal to every degree-k
    polynomial on every element."""
    xyz, per = periodic_split_square(3, "random", seed=1)
    o = Oracle(xyz, per, k)
    rule = triangle_rule(2 * k + 2)
    coef = random_broken_poly(o.mesh.T, k, seed=5)
    cU = o.space.broken_project(eval_broken_poly(coef, rule[0]), rule)
    pts = np.random.default_rng(2).uniform(0, 0.5, size=(9, 2))
    vals, _ = poly_basis(k, pts[:, 0], pts[:, 1])
    got = np.einsum("tca,pa->tcp", cU, vals)
    assert np.abs(got - eval_broken_poly(coef, pts)).max() < 1e-12 * np.abs(coef).max() * 10
    # degree k+1 data: the error is orthogonal to the monomials of degree <= k
    coef1 = random_broken_poly(o.mesh.T, k + 1, seed=6)
    fine = triangle_rule(2 * k + 4)
    cU1 = o.space.broken_project(eval_broken_poly(coef1, fine[0]), fine)
    v1, _ = poly_basis(k, fine[0][:, 0], fine[0][:, 1])
    err = eval_broken_poly(coef1, fine[0]) - np.einsum("tca,qa->tcq", cU1, v1)
    xi, eta = fine[0][:, 0], fine[0][:, 1]
    for d in range(k + 1):
        for q in range(d + 1):
            m = xi ** (d - q) * eta ** q
            moment = np.einsum("q,tcq,q->tc", fine[1], err, m)
            assert np.abs(moment).max() < 1e-12 * np.abs(coef1).max() * 10


def test_broken_diagnostics_of_piecewise_fields():
    """Normal jumps and divergence of broken fields with hand-computable values: a
    piecewise constant field c_t (jump (c_A - c_B) . n) and the piecewise linear field
    (a_t x, b_t y) (divergence a_t + b_t)."""
    xyz, per = periodic_split_square(3, "random", seed=4)
    o = Oracle(xyz, per, 2)
    m = o.mesh
    rng = np.random.default_rng(7)
    rule = triangle_rule(6)
    c = rng.standard_normal((m.T, 2))
    vals = np.repeat(c[:, :, None], len(rule[1]), axis=2)
    cU = o.space.broken_project(vals, rule)
    jumps = np.abs(np.einsum("ec,ec->e", c[m.fA_elem] - c[m.fB_elem], m.normal))
    assert abs(o.normal_jump_max_local(cU) - jumps.max()) < 1e-12
    assert o.divergence_max_local(cU) < 1e-12
    assert abs(o.energy_local(cU) - 0.5 * float((m.area[:, None] * c ** 2).sum())) < 1e-12
    assert o.enstrophy_local(cU) < 1e-24
    a, b = rng.standard_normal(m.T), rng.standard_normal(m.T)
    x = o.phys_points(rule[0])
    lin = np.stack([a[:, None] * x[..., 0], b[:, None] * x[..., 1]], axis=1)
    cL = o.space.broken_project(lin, rule)
    assert abs(o.divergence_max_local(cL) - np.abs(a + b).max()) < 1e-12
    # (a x, b y) has zero curl; adding (-w y, w x) per element gives curl 2 w
    w = rng.standard_normal(m.T)
    rot = lin + np.stack([-w[:, None] * x[..., 1], w[:, None] * x[..., 0]], axis=1)
    cR = o.space.broken_project(rot, rule)
    assert abs(o.enstrophy_local(cR) - float((m.area * (2 * w) ** 2).sum())) < 1e-11
