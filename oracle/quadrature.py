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


# ---- three dimensions ----------------------------------------------------------------------
def tet_rule(degree):
    """Collapsed (Duffy) Gauss rule on the reference tetrahedron {xi, eta, zeta >= 0,
    xi + eta + zeta <= 1}: Gauss-Legendre in a, Gauss-Jacobi (1, 0) in b and (2, 0) in c,
    with xi = (1+a)(1-b)(1-c)/8, eta = (1+b)(1-c)/4, zeta = (1+c)/2; the Jacobian
    (1-b)(1-c)^2/64 is carried by the Jacobi weights and the factor 1/64.  Exact for total
    degree ``degree``.  Returns (points[nq, 3], weights[nq]); the weights sum to 1/6."""
    n = (degree + 2) // 2
    a, wa = np.polynomial.legendre.leggauss(n)
    b, wb = roots_jacobi(n, 1.0, 0.0)
    c, wc = roots_jacobi(n, 2.0, 0.0)
    A, B, C = np.meshgrid(a, b, c, indexing="ij")
    xi = 0.125 * (1.0 + A) * (1.0 - B) * (1.0 - C)
    eta = 0.25 * (1.0 + B) * (1.0 - C)
    zeta = 0.5 * (1.0 + C)
    w = np.einsum("i,j,k->ijk", wa, wb, wc) / 64.0
    return np.stack([xi.ravel(), eta.ravel(), zeta.ravel()], axis=1), w.ravel()


def simplex_rule(d, degree):
    """triangle_rule (d = 2) or tet_rule (d = 3): exact for total degree ``degree``."""
    return triangle_rule(degree) if d == 2 else tet_rule(degree)


def monomials3(k, xi, eta, zeta):
    """Monomials xi^p eta^q zeta^r of total degree <= k (ordered by degree d, then q + r,
    then r) and their reference gradients: vals[..., n], grads[..., 3, n]."""
    xi, eta, zeta = (np.asarray(v, dtype=np.result_type(v, float)) for v in (xi, eta, zeta))

    def pw(x, e):
        return x ** e if e > 0 else np.ones_like(x)

    def dpw(x, e):
        return e * x ** (e - 1) if e > 0 else np.zeros_like(x)

    vals, g0, g1, g2 = [], [], [], []
    for d in range(k + 1):
        for qr in range(d + 1):
            for r in range(qr + 1):
                p, q = d - qr, qr - r
                vals.append(pw(xi, p) * pw(eta, q) * pw(zeta, r))
                g0.append(dpw(xi, p) * pw(eta, q) * pw(zeta, r))
                g1.append(pw(xi, p) * dpw(eta, q) * pw(zeta, r))
                g2.append(pw(xi, p) * pw(eta, q) * dpw(zeta, r))
    vals = np.stack(vals, axis=-1)
    grads = np.stack([np.stack(g0, axis=-1), np.stack(g1, axis=-1), np.stack(g2, axis=-1)], axis=-2)
    return vals, grads


def _monomial_gram3(k):
    """Exact Gram matrix of the monomials on the reference tetrahedron:
    int xi^p eta^q zeta^r = p! q! r! / (p + q + r + 3)!."""
    from math import factorial
    exps = [(d - qr, qr - r, r) for d in range(k + 1) for qr in range(d + 1) for r in range(qr + 1)]
    G = np.empty((len(exps), len(exps)))
    for i, (p1, q1, r1) in enumerate(exps):
        for j, (p2, q2, r2) in enumerate(exps):
            p, q, r = p1 + p2, q1 + q2, r1 + r2
            G[i, j] = factorial(p) * factorial(q) * factorial(r) / factorial(p + q + r + 3)
    return G


_QCACHE3 = {}


def poly_basis3(k, xi, eta, zeta):
    """Reference-orthonormal scalar basis of P^k on the reference tetrahedron, hierarchical
    by degree (monomials orthonormalised through the Cholesky factor of their exact Gram
    matrix).  Returns vals[..., n], grads[..., 3, n]."""
    if k not in _QCACHE3:
        L = np.linalg.cholesky(_monomial_gram3(k))
        _QCACHE3[k] = np.linalg.inv(L).T
    Q = _QCACHE3[k]
    v, g = monomials3(k, xi, eta, zeta)
    return v @ Q, g @ Q


def poly_basis_nd(k, pts):
    """poly_basis (pts[..., 2]) or poly_basis3 (pts[..., 3]) at reference points."""
    pts = np.asarray(pts)
    if pts.shape[-1] == 2:
        return poly_basis(k, pts[..., 0], pts[..., 1])
    return poly_basis3(k, pts[..., 0], pts[..., 1], pts[..., 2])


def _s21(a):
    """Barycentric orbit (a, a, 1 - 2a) as reference points (xi, eta) of its 3 members."""
    b = 1.0 - 2.0 * a
    return [(a, a), (a, b), (b, a)]


def _s111(a, b):
    """Orbit of (a, b, 1 - a - b) under the 6 vertex permutations, as (xi, eta) points."""
    c = 1.0 - a - b
    out = []
    for x, y in ((a, b), (b, a), (a, c), (c, a), (b, c), (c, b)):
        out.append((x, y))
    return out


# Fully symmetric rules on the reference triangle with positive weights (Dunavant's
# degree-4 and degree-6 rules; 6 and 12 points): orbit structure and published values to
# about 12 digits, refined below by solving the moment equations.
_SYM_RULES = {
    4: [("s21", (0.445948490915965,), 0.223381589678011), ("s21", (0.091576213509771,), 0.109951743655322)],
    6: [("s21", (0.249286745170910,), 0.116786275726379), ("s21", (0.063089014491502,), 0.050844906370207),
        ("s111", (0.053145049844817, 0.310352451033784), 0.082851075618374)],
}
_SYMCACHE = {}


def symmetric_triangle_rule(degree):
    """The fully symmetric rule of degree 4 (6 points) or 6 (12 points) with positive
    weights on the reference triangle: orbit parameters and weights solved from the moment
    equations sum_q w_q xi_q^p eta_q^r = p! r! / (p + r + 2)! (p + r <= degree) by least
    squares from the published values.  Its point set is invariant under the 6 permutations
    of the triangle's vertices.  Returns (points[nq, 2], weights[nq]) with weights summing
    to 1/2."""
    if degree in _SYMCACHE:
        return _SYMCACHE[degree]
    from math import factorial
    from scipy.optimize import least_squares
    spec = _SYM_RULES[degree]
    x0 = []
    for kind, par, w in spec:
        x0 += list(par) + [w]
    exps = [(p, r) for p in range(degree + 1) for r in range(degree + 1 - p)]
    exact = np.array([factorial(p) * factorial(r) / factorial(p + r + 2) for p, r in exps])

    def build(x):
        pts, ws, i = [], [], 0
        for kind, par, _ in spec:
            if kind == "s21":
                pp = _s21(x[i])
                i += 1
            else:
                pp = _s111(x[i], x[i + 1])
                i += 2
            pts += pp
            ws += [0.5 * x[i]] * len(pp)  # published weights are relative to the area
            i += 1
        return np.array(pts), np.array(ws)

    def resid(x):
        pts, ws = build(x)
        return np.array([(ws * pts[:, 0] ** p * pts[:, 1] ** r).sum() for p, r in exps]) / exact - 1.0

    sol = least_squares(resid, np.array(x0), xtol=1e-15, ftol=1e-15, gtol=1e-15, method="lm")
    pts, ws = build(sol.x)
    assert np.abs(resid(sol.x)).max() < 1e-14 and np.all(ws > 0)
    _SYMCACHE[degree] = (pts, ws)
    return pts, ws


def facet_rule(d, k):
    """The facet rule of the residual's facet integrals (including the pointwise upwind
    flux, the only non-polynomial integrand), on the reference facet with weights summing
    to 1 (multiply by the facet measure): d = 2: Gauss-Legendre with ceil((3k+1)/2) points
    on [0, 1] (exact for degree 3k), points[nq, 1]; d = 3: the fully symmetric triangle rule
    of degree max(4, 3k) (k <= 2), points[nq, 2]."""
    if d == 2:
        s, w = gauss_legendre_01(facet_rule_points(k))
        return s[:, None], w
    if k > 2:
        raise ValueError("three-dimensional facet rules are defined for k <= 2")
    pts, w = symmetric_triangle_rule(4 if k == 1 else 6)
    return pts, 2.0 * w


def facet_moment_rule(d, k):
    """Rule for the BDM facet moments (exact for degree 2k) on the reference facet, weights
    summing to 1, and the moment basis of P^k on the facet at its points: d = 2: k+1
    Gauss-Legendre points and orthonormal Legendre polynomials sqrt(2j+1) P_j(2s-1); d = 3:
    the collapsed triangle rule of degree 2k and poly_basis on the reference triangle.
    Returns (points[nq, d-1], weights[nq], basis[nq, n_f])."""
    if d == 2:
        s, w = gauss_legendre_01(k + 1)
        basis = np.stack([np.sqrt(2 * j + 1) * legendre01(j, s) for j in range(k + 1)], axis=1)
        return s[:, None], w, basis
    pts, w = triangle_rule(2 * k)
    basis, _ = poly_basis(k, pts[:, 0], pts[:, 1])
    return pts, 2.0 * w, basis
