"""Pins of the oracle's divergence-free mass inversion (Theorems 1 and 2)."""
import numpy as np
import pytest
import scipy.linalg as sla

from inputs import periodic_split_square, random_broken_poly, eval_broken_poly
from oracle import Oracle
from oracle.quadrature import triangle_rule
from oracle.scheme import hybrid_solve_dense


def _oracle(N, k, order="morton"):
    xyz, per = periodic_split_square(N, order, seed=1)
    return Oracle(xyz, per, k)


@pytest.mark.parametrize("k", [1, 2, 3])
def test_mass_solve_equals_svd_nullspace_projection(k):
    """u = Z (Z^T M Z)^{-1} Z^T f with Z a brute-force SVD basis of ker(div)."""
    o = _oracle(3, k)
    Z = sla.null_space(o.B.toarray())
    M = o.M.toarray()
    f = np.random.default_rng(7).standard_normal(o.space.ndof)
    u = o.mass_solve(f)
    ub = Z @ np.linalg.solve(Z.T @ M @ Z, Z.T @ f)
    assert np.abs(u - ub).max() < 1e-12 * np.abs(ub).max()
    assert o.divergence_max(u) < 1e-11 * np.abs(u).max() * 3


@pytest.mark.parametrize("k", [1, 2, 3])
def test_hybrid_equals_mixed(k):
    """Theorem 2: the hybrid-mixed velocity (FE3) equals the mixed one (FE2)."""
    o = _oracle(2, k, "lex")
    Fb = np.random.default_rng(3).standard_normal((o.mesh.T, 2, o.space.nm))
    cu_h = hybrid_solve_dense(o, Fb)
    cu_m = o.space.local_coeffs(o.mass_solve(o.space.assemble(Fb)))
    assert np.abs(cu_h - cu_m).max() < 1e-11 * np.abs(cu_m).max()


@pytest.mark.parametrize("k", [1, 2])
def test_mass_solve_symmetric_and_idempotent(k):
    o = _oracle(4, k)
    rng = np.random.default_rng(11)
    f, g = rng.standard_normal((2, o.space.ndof))
    Pf, Pg = o.mass_solve(f), o.mass_solve(g)
    # symmetric: g . P f = f . P g
    assert abs(g @ Pf - f @ Pg) < 1e-12 * abs(g @ Pf) + 1e-12
    # idempotent on V^{k,-1}: solving with the functional (u, .) returns u
    assert np.abs(o.mass_solve(o.M @ Pf) - Pf).max() < 1e-12 * np.abs(Pf).max()


@pytest.mark.parametrize("k", [1, 2, 3])
def test_projection_of_divergence_free_polynomial_is_exact(k):
    """A constant field is in V^{k,-1}: its L2 projection reproduces it."""
    o = _oracle(3, k)
    U = o.project(lambda x, y: (0.25 + 0 * x, -1.5 + 0 * y))
    rule = triangle_rule(4)
    v = o.eval_ref(U, rule[0])
    assert np.abs(v[:, 0] - 0.25).max() < 1e-13
    assert np.abs(v[:, 1] + 1.5).max() < 1e-13


def test_broken_load_vector_of_random_polynomial():
    """The load vector of a broken polynomial equals its exact element integrals."""
    o = _oracle(2, 2)
    coef = random_broken_poly(o.mesh.T, 2, seed=5)
    rule = triangle_rule(4)
    f = eval_broken_poly(coef, rule[0])
    R = o.space.load_vector(f, rule)
    rule2 = triangle_rule(9)
    R2 = o.space.load_vector(eval_broken_poly(coef, rule2[0]), rule2)
    assert np.abs(R - R2).max() < 1e-14 * np.abs(R).max() * 10
