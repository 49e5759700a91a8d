"""Pins of the oracle's quadrature, mesh and BDM space against closed forms."""
from math import factorial

import numpy as np
import pytest
import scipy.linalg as sla

from inputs import periodic_split_square
from oracle import Oracle
from oracle.mesh import OracleMesh
from oracle.quadrature import gauss_legendre_01, monomials, poly_basis, triangle_rule


@pytest.mark.parametrize("deg", range(0, 12))
def test_triangle_rule_exact(deg):
    pts, w = triangle_rule(deg)
    for p in range(deg + 1):
        q = deg - p
        exact = factorial(p) * factorial(q) / factorial(p + q + 2)
        got = np.sum(w * pts[:, 0] ** p * pts[:, 1] ** q)
        assert abs(got - exact) < 1e-15 * max(1, 1 / exact) * 10


@pytest.mark.parametrize("n", range(1, 8))
def test_gauss_legendre_exact(n):
    s, w = gauss_legendre_01(n)
    for j in range(2 * n):
        assert abs(np.sum(w * s ** j) - 1.0 / (j + 1)) < 1e-15
    # symmetric about 1/2 (the upwind facet rule relies on it)
    assert np.allclose(np.sort(s), np.sort(1 - s), atol=1e-15)


@pytest.mark.parametrize("k", [1, 2, 3, 4])
def test_poly_basis_orthonormal_and_hierarchical(k):
    pts, w = triangle_rule(2 * k)
    v, _ = poly_basis(k, pts[:, 0], pts[:, 1])
    G = np.einsum("q,qa,qb->ab", w, v, v)
    # orthonormal up to the rounding of the Cholesky factor of an ill-conditioned Gram matrix
    assert np.abs(G - np.eye(len(G))).max() < 1e-10
    # the first dim P^{k-1} functions are polynomials of degree k-1: they are
    # orthogonal to every degree-k monomial-free remainder, i.e. spanned by
    # monomials of degree <= k-1
    m, _ = monomials(k, pts[:, 0], pts[:, 1])
    npk1 = k * (k + 1) // 2
    coef = np.linalg.lstsq(m[:, :npk1], v[:, :npk1], rcond=None)[0]
    assert np.abs(m[:, :npk1] @ coef - v[:, :npk1]).max() < 1e-12


@pytest.mark.parametrize("N", [1, 2, 3, 5])
def test_periodic_mesh_counts(N):
    xyz, per = periodic_split_square(N)
    m = OracleMesh(xyz, per)
    assert m.T == 2 * N * N
    assert m.E == 3 * N * N            # Euler: V - E + T = 0 on the torus, V = N^2
    assert np.allclose(m.area.sum(), 1.0)
    assert np.allclose(m.hT, 1.0 / N)  # (2|T|)^(1/2) is the grid spacing
    # every element's three facets are distinct facets
    for t in range(m.T):
        assert len(set(m.elem_facet[t])) == 3
    # A and B copies of every facet coincide after the periodic shift
    assert np.all(np.abs(np.abs(m.shiftB) - np.round(np.abs(m.shiftB))) < 1e-14)


@pytest.mark.parametrize("k", [1, 2, 3])
@pytest.mark.parametrize("N", [2, 3])
def test_bdm_conforming_and_dimensions(k, N):
    xyz, per = periodic_split_square(N, "random", seed=N)
    o = Oracle(xyz, per, k)
    sp = o.space
    T, E = o.mesh.T, o.mesh.E
    assert sp.ndof == E * (k + 1) + T * (k + 1) * (k - 1)
    U = np.random.default_rng(k).standard_normal(sp.ndof)
    assert o.normal_jump_max(U) < 1e-13 * np.abs(U).max() * N
    # de Rham: dim V^{k,-1} = dim BDM_k - (dim Q^{k-1} - 1) = N^2 (k+1)^2 + 1 (2D torus)
    Z = sla.null_space(o.B.toarray())
    assert Z.shape[1] == N * N * (k + 1) ** 2 + 1
    assert Z.shape[1] == sp.ndof - (sp.npres - 1)
