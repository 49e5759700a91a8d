"""Quadrature rules of the oracle (its own; nothing is shared with the GPU library).

The paper does not state its quadrature.  The reading used throughout is that
polynomial integrands are integrated exactly; the only non-polynomial integrand
on the path, the pointwise upwind flux on a facet, is integrated with the
Gauss-Legendre rule of ceil((3k+1)/2) points (exact for degree 3k), which is
stated as part of the method so that any two implementations agree.
"""
import numpy as np
from scipy.special import roots_jacobi


def gauss_legendre_01(n):
    """n-point Gauss-Legendre nodes and weights on [0, 1] (weights sum to 1)."""
    x, w = np.polynomial.legendre.leggauss(n)
    return 0.5 * (x + 1.0), 0.5 * w


def facet_rule_points(k):
    """Number of Gauss-Legendre points of the facet rule: exact for degree 3k."""
    return (3 * k + 2) // 2


def triangle_rule(degree):
    """Collapsed (Duffy) Gauss rule on the reference triangle {xi, eta >= 0, xi + eta <= 1}.

    Gauss-Legendre in a and Gauss-Jacobi (alpha=1, beta=0) in b, with
    xi = (1+a)(1-b)/4, eta = (1+b)/2; the Jacobian (1-b)/8 is carried by the
    Jacobi weight and the factor 1/8.  Exact for total degree ``degree``.
    Returns (points[nq, 2], weights[nq]); the weights sum to 1/2.
    """
    n = (degree + 2) // 2
    a, wa = np.polynomial.legendre.leggauss(n)
    b, wb = roots_jacobi(n, 1.0, 0.0)
    A, B = np.meshgrid(a, b, indexing="ij")
    xi = 0.25 * (1.0 + A) * (1.0 - B)
    eta = 0.5 * (1.0 + B)
    w = np.outer(wa, wb) / 8.0
    return np.stack([xi.ravel(), eta.ravel()], axis=1), w.ravel()


def monomials(k, xi, eta):
    """Monomials xi^(d-q) eta^q (d = 0..k, q = 0..d) and their reference gradients.

    Returns vals[..., n] and grads[..., 2, n] with grads[..., r, a] = d m_a / d xi_r.
    """
    xi = np.asarray(xi, dtype=np.result_type(xi, float))
    eta = np.asarray(eta, dtype=np.result_type(eta, float))
    vals, gx, gy = [], [], []
    for d in range(k + 1):
        for q in range(d + 1):
            p = d - q
            vals.append(xi ** p * eta ** q)
            gx.append(p * xi ** max(p - 1, 0) * eta ** q if p > 0 else np.zeros_like(xi))
            gy.append(q * xi ** p * eta ** max(q - 1, 0) if q > 0 else np.zeros_like(xi))
    vals = np.stack(vals, axis=-1)
    grads = np.stack([np.stack(gx, axis=-1), np.stack(gy, axis=-1)], axis=-2)
    return vals, grads


def legendre01(j, s):
    """Legendre polynomial P_j(2s - 1) on [0, 1] (unnormalised)."""
    c = np.zeros(j + 1)
    c[j] = 1.0
    return np.polynomial.legendre.legval(2.0 * np.asarray(s) - 1.0, c)


def _monomial_gram(k):
    """Exact Gram matrix of the monomials on the reference triangle.

    int xi^p eta^q = p! q! / (p + q + 2)!.
    """
    from math import factorial
    exps = [(d - q, q) for d in range(k + 1) for q in range(d + 1)]
    n = len(exps)
    G = np.empty((n, n))
    for i, (p1, q1) in enumerate(exps):
        for j, (p2, q2) in enumerate(exps):
            p, q = p1 + p2, q1 + q2
            G[i, j] = factorial(p) * factorial(q) / factorial(p + q + 2)
    return G


_QCACHE = {}


def poly_basis(k, xi, eta):
    """Reference-orthonormal scalar basis of P^k, hierarchical by degree.

    The monomials are orthonormalised on the reference triangle through the
    Cholesky factor of their exact Gram matrix, G = L L^T, basis = m^T L^{-T};
    the first dim P^j functions span P^j.  Returns vals[..., n], grads[..., 2, n].
    """
    if k not in _QCACHE:
        L = np.linalg.cholesky(_monomial_gram(k))
        _QCACHE[k] = np.linalg.inv(L).T
    Q = _QCACHE[k]
    v, g = monomials(k, xi, eta)
    return v @ Q, g @ Q
