"""Reduced local velocity spaces of the hybrid-mixed mass inversion (test infrastructure).

Two variants of eq. (FE3) from the remark "More efficient implementation" (Sec. 2.4),
written out densely for tiny triangle meshes:

* eq. (FE4): the broken velocity is restricted to the locally divergence-free space
  V^{k,-1} (div v = 0 on every element) and the equations of w and z are dropped.
  The local basis is built as the paper says it can be: in 2D the divergence-free
  [P^k(T)]^2 fields are the curls of the stream functions in P^{k+1}(T), modulo
  constants.
* the variant the paper's own runs used: velocity in V^{k,0} (div v constant on every
  element) with w in the piecewise constants Q^0.

Both restate the assembly of ``hybrid_system_dense`` on smaller unknown sets; the
velocities must equal that of eq. (FE2) (Theorem 2 with V^{k,-1} or V^{k,0} in place
of the broken [P^k]^d).  Triangles only.
"""
import numpy as np
import scipy.linalg as sla

from .quadrature import poly_basis_nd, simplex_rule
from .scheme import hybrid_system_dense


def _fit_local(orc, t, values_at, degree_extra=2):
    """Local coefficients [d*nm, ncol] of vector fields given at reference points.

    values_at(pts) -> [Q, d, ncol] physical components at the points of a rule exact
    for degree 2k + degree_extra; the fields must lie in [P^k(T)]^d (the fit is exact,
    and the residual is checked)."""
    k, nm = orc.k, orc.space.nm
    pts, _ = simplex_rule(2, 2 * k + degree_extra)
    vk, _ = poly_basis_nd(k, pts)  # [Q, nm]
    vals = values_at(pts)  # [Q, 2, ncol]
    Q, d, ncol = vals.shape
    coef, *_ = np.linalg.lstsq(vk, vals.reshape(Q, d * ncol), rcond=None)  # [nm, d*ncol]
    resid = vk @ coef - vals.reshape(Q, d * ncol)
    assert np.abs(resid).max() < 1e-10 * max(1.0, np.abs(vals).max()), "field not in [P^k]^d"
    return coef.reshape(nm, d, ncol).transpose(1, 0, 2).reshape(d * nm, ncol)


def curl_basis(orc, t):
    """Columns spanning the locally divergence-free [P^k(T)]^2 of element t: curl psi =
    (d psi/dy, -d psi/dx) for the non-constant reference modes psi of P^{k+1}."""
    if orc.d != 2:
        raise ValueError("stream-function bases are two-dimensional")
    Ji = orc.mesh.Jinv[t]  # [r][c] = d xi_r / d x_c

    def curls(pts):
        _, dk1 = poly_basis_nd(orc.k + 1, pts)  # [Q, r, nm1]
        grad = np.einsum("qrb,rc->qcb", dk1[:, :, 1:], Ji)  # physical gradient
        return np.stack([grad[:, 1, :], -grad[:, 0, :]], axis=1)

    return _fit_local(orc, t, curls)


def constant_divergence_field(orc, t):
    """Local coefficients of v = (x - x_0, 0) on element t (x_0 its first vertex):
    div v = 1, the direction that V^{k,0} adds to V^{k,-1}."""
    J = np.linalg.inv(orc.mesh.Jinv[t])  # [c][r] = d x_c / d xi_r

    def field(pts):
        x = pts @ J[0]  # x - x_0 as a function of the reference point
        return np.stack([x, np.zeros_like(x)], axis=1)[:, :, None]

    return _fit_local(orc, t, field)


def _blocks(orc):
    K, nU, nW = hybrid_system_dense(orc)
    return K[:nU, :nU], K[:nU, nU:nU + nW], K[:nU, nU + nW:], nU, nW


def fe4_system_dense(orc):
    """Dense eq. (FE4): unknowns (coefficients of the curl basis per element, facet
    multipliers).  Returns (K4, Z): K4 = [[Z^T M Z, Z^T C^T], [C Z, 0]] with the
    block-diagonal Z of the element curl bases (the multiplier's sign as in (FE3); it
    does not change the velocity)."""
    M, _, Ct, nU, _ = _blocks(orc)
    Z = sla.block_diag(*[curl_basis(orc, t) for t in range(orc.mesh.T)])
    A = Z.T @ M @ Z
    B = Z.T @ Ct
    nL = Ct.shape[1]
    K4 = np.block([[A, B], [B.T, np.zeros((nL, nL))]])
    return K4, Z


def fe4_solve_dense(orc, Fbroken):
    """Velocity local coefficients cU[T, 2, nm] of eq. (FE4) for the functional Fbroken
    on the broken local basis (least squares: the system is singular by the constant
    multiplier only)."""
    K4, Z = fe4_system_dense(orc)
    rhs = np.zeros(K4.shape[0])
    rhs[:Z.shape[1]] = Z.T @ Fbroken.reshape(-1)
    sol = np.linalg.lstsq(K4, rhs, rcond=None)[0]
    return (Z @ sol[:Z.shape[1]]).reshape(orc.mesh.T, 2, orc.space.nm)


def fe4_facet_matrix(orc):
    """Facet Schur complement of eq. (FE4): (C Z) (Z^T M Z)^{-1} (C Z)^T."""
    M, _, Ct, _, _ = _blocks(orc)
    Z = sla.block_diag(*[curl_basis(orc, t) for t in range(orc.mesh.T)])
    CZ = Ct.T @ Z
    return CZ @ np.linalg.solve(Z.T @ M @ Z, CZ.T)


def vk0_q0_solve_dense(orc, Fbroken):
    """Velocity cU[T, 2, nm] of eq. (FE3) with velocity in V^{k,0} (curl basis plus the
    constant-divergence field per element) and w in Q^0 (the constant pressure mode of
    each element)."""
    M, Dt, Ct, nU, nW = _blocks(orc)
    T, npr = orc.mesh.T, orc.space.np_
    V0 = sla.block_diag(*[np.hstack([curl_basis(orc, t), constant_divergence_field(orc, t)])
                          for t in range(T)])
    D0t = Dt[:, np.arange(T) * npr]  # the constant mode of every element's pressure
    A, B, Cc = V0.T @ M @ V0, V0.T @ D0t, V0.T @ Ct
    nv, nl = A.shape[0], Cc.shape[1]
    K0 = np.block([[A, B, Cc],
                   [B.T, np.zeros((T, T)), np.zeros((T, nl))],
                   [Cc.T, np.zeros((nl, T)), np.zeros((nl, nl))]])
    rhs = np.zeros(K0.shape[0])
    rhs[:nv] = V0.T @ Fbroken.reshape(-1)
    sol = np.linalg.lstsq(K0, rhs, rcond=None)[0]
    return (V0 @ sol[:nv]).reshape(T, 2, orc.space.nm)
