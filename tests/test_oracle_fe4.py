"""Pins of the oracle's reduced local spaces (remark "More efficient implementation",
Sec. 2.4, eq. (FE4), and the V^{k,0} + Q^0 variant the paper ran): the stream-function
basis spans exactly the null space of the element divergence (SVD), and both variants
give the velocity of the global mixed solve (eq. (FE2), conforming basis, SuperLU)."""
import numpy as np
import pytest
import scipy.linalg as sla

from inputs import periodic_split_square
from oracle import Oracle
from oracle.fe4 import (constant_divergence_field, curl_basis, fe4_facet_matrix, fe4_solve_dense,
                        vk0_q0_solve_dense)
from oracle.scheme import hybrid_system_dense


def _oracle(N, k, walls=False, order="random"):
    xyz, per = periodic_split_square(N, order, seed=2)
    return Oracle(xyz, np.array([1.0, 0.0]) if walls else per, k)


def _element_divergence(o):
    K, nU, nW = hybrid_system_dense(o)
    nu, npr = o.space.nu, o.space.np_
    return [-K[nU + t * npr:nU + (t + 1) * npr, t * nu:(t + 1) * nu] for t in range(o.mesh.T)]


@pytest.mark.parametrize("k", [1, 2, 3])
def test_curl_basis_spans_the_divergence_null_space(k):
    """dim = dim P^{k+1} - 1 = n_u - n_p; D_T Z_T = 0; and the orthogonal projector onto
    span Z_T equals the one onto the SVD null space of D_T."""
    o = _oracle(2, k)
    D = _element_divergence(o)
    nu, npr = o.space.nu, o.space.np_
    assert (k + 2) * (k + 3) // 2 - 1 == nu - npr
    for t in range(o.mesh.T):
        Z = curl_basis(o, t)
        assert Z.shape == (nu, nu - npr) and np.linalg.matrix_rank(Z) == nu - npr
        assert np.abs(D[t] @ Z).max() < 1e-11 * np.abs(D[t]).max() * np.abs(Z).max()
        N = sla.null_space(D[t])
        Q, _ = np.linalg.qr(Z)
        assert np.abs(Q @ Q.T - N @ N.T).max() < 1e-11


@pytest.mark.parametrize("k", [1, 2, 3])
def test_constant_divergence_field(k):
    """The field added for V^{k,0} has divergence exactly 1: its divergence moments are
    those of the constant 1 (|T| times the reference constant mode's value sqrt 2 on that
    mode, zero on the others)."""
    o = _oracle(2, k)
    D = _element_divergence(o)
    for t in range(o.mesh.T):
        d = D[t] @ constant_divergence_field(o, t)[:, 0]
        # D rows are moments against the reference-orthonormal modes times det J
        one = np.zeros(o.space.np_)
        one[0] = o.mesh.detJ[t] * np.sqrt(2.0) / 2  # int_T 1 m_0: m_0 = sqrt 2 on the reference, area 1/2
        assert np.abs(d - one).max() < 1e-12 * abs(one[0])


@pytest.mark.parametrize("walls", [False, True])
@pytest.mark.parametrize("k", [1, 2, 3])
def test_fe4_velocity_equals_mixed(k, walls):
    """eq. (FE4) on the locally divergence-free space gives the velocity of eq. (FE2)."""
    o = _oracle(3, k, walls)
    Fb = np.random.default_rng(k).standard_normal((o.mesh.T, 2, o.space.nm))
    cu4 = fe4_solve_dense(o, Fb)
    cum = o.space.local_coeffs(o.mass_solve(o.space.assemble(Fb)))
    assert np.abs(cu4 - cum).max() < 1e-11 * np.abs(cum).max()


@pytest.mark.parametrize("walls", [False, True])
@pytest.mark.parametrize("k", [1, 2])
def test_vk0_q0_velocity_equals_mixed(k, walls):
    """The paper's V^{k,0} + Q^0 form of eq. (FE3) gives the same velocity too."""
    o = _oracle(3, k, walls)
    Fb = np.random.default_rng(10 + k).standard_normal((o.mesh.T, 2, o.space.nm))
    cu0 = vk0_q0_solve_dense(o, Fb)
    cum = o.space.local_coeffs(o.mass_solve(o.space.assemble(Fb)))
    assert np.abs(cu0 - cum).max() < 1e-11 * np.abs(cum).max()


@pytest.mark.parametrize("k", [1, 2, 3])
def test_fe4_facet_matrix_equals_fe3_condensation(k):
    """The multiplier system of (FE4) is the one of (FE3): the local divergence-free
    projector is the same operator, whichever local unknowns compute it."""
    o = _oracle(2, k)
    K, nU, nW = hybrid_system_dense(o)
    nx = nU + nW
    S3 = K[:nx, nx:].T @ np.linalg.solve(K[:nx, :nx], K[:nx, nx:])
    S4 = fe4_facet_matrix(o)
    assert np.abs(S4 - S3).max() < 1e-11 * np.abs(S3).max()
