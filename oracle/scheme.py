"""Mass matrices, the global mixed solve, TVD-RK3 and diagnostics of the oracle.

The divergence-free mass inversion is done as the mixed Poisson problem of
Sec. 2.4, eq. (FE2): find (u, w) in BDM_k x Q^{k-1} with
  (u, v) - (w, div v) = F(v)   for all v in BDM_k,
  (div u, z)          = 0      for all z in Q^{k-1},
where Q^{k-1} is broken P^{k-1} with zero mean (enforced by one Lagrange
multiplier).  Theorem 1 states that u is the mass inversion of F on the
divergence-free space.  The saddle matrix does not depend on the time step
(Remark "Equivalence with the velocity-pressure formulation"), so it is
factored once with SuperLU and reused.
"""
import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from .bdm import BDMSpace, n_mono
from .mesh import OracleMesh
from .quadrature import (facet_moment_rule, facet_rule, gauss_legendre_01, poly_basis, poly_basis_nd,
                         simplex_rule)
from .residual import Residual


class Oracle:
    """Plain FP64 reference solver on a periodic simplex mesh.

    xyz[T, 3, 2]: counter-clockwise triangles, or xyz[T, 4, 3]: positively oriented
    tetrahedra; period[d] or None.
    """

    def __init__(self, xyz, period, k, nu=0.0, alpha=2.0, outflow=None, inflow=None):
        self.mesh = OracleMesh(xyz, period, outflow)
        self.k = k
        self.d = self.mesh.d
        self.space = BDMSpace(self.mesh, k)
        self.res = Residual(self.space, nu=nu, alpha=alpha)
        self._assemble()
        self._lu = None
        # Inflow data (Sec. 2.5): the state is u = lift + U with U in the space whose normal
        # moments vanish on the closed boundary (walls and inflow), the lift a fixed
        # divergence-free polynomial field of degree <= k (``inflow(x, y)``) carrying the
        # inflow's normal velocity; the stages change U only.
        self.cLift = None if inflow is None else self._broken_exact(inflow)

    def _broken_exact(self, field):
        """Local coefficients [T, d, nm] of a polynomial field of degree <= k (element-wise
        L2 projection with the reference-orthonormal modes: exact)."""
        rule = simplex_rule(self.d, 2 * self.k + 2)
        x = self.phys_points(rule[0])
        R = self.space.load_vector(np.stack(field(*[x[..., i] for i in range(self.d)]), axis=1), rule)
        return R / self.mesh.detJ[:, None, None]

    def state_local(self, U):
        """Local coefficients of the state: lift (if any) + U."""
        c = self.space.local_coeffs(U)
        return c if self.cLift is None else c + self.cLift

    # ---- matrices ----------------------------------------------------------------
    def _assemble(self):
        sp_, m, k, d = self.space, self.mesh, self.k, self.d
        pts, w = simplex_rule(d, 2 * k)
        vals, dref = poly_basis_nd(k, pts)                           # [q, nm], [q, d, nm]
        nm, npr = sp_.nm, sp_.np_
        # element mass in the local basis (block-diagonal over components)
        Mref = np.einsum("q,qa,qb->ab", w, vals, vals)
        Mphi = np.zeros((sp_.nu, sp_.nu))
        for c in range(d):
            Mphi[c * nm:(c + 1) * nm, c * nm:(c + 1) * nm] = Mref
        ML = np.einsum("t,tai,ab,tbj->tij", m.detJ, sp_.A, Mphi, sp_.A)
        # divergence against the pressure basis z_p (the first dim P^{k-1} of the local basis)
        z = vals[:, :npr]
        div_phi = np.einsum("qra,trc->tqca", dref, m.Jinv)         # d m_a/dx_c at q
        Dphi = np.einsum("q,t,qp,tqca->tpca", w, m.detJ, z, div_phi).reshape(m.T, npr, sp_.nu)
        BL = np.einsum("tpa,tai->tpi", Dphi, sp_.A)                # (z_p, div beta_i)_T
        cmean = np.einsum("q,t,qp->tp", w, m.detJ, z)              # int_T z_p
        T = m.T
        rows = np.repeat(sp_.dofs, sp_.nu, axis=1).ravel()
        cols = np.tile(sp_.dofs, (1, sp_.nu)).ravel()
        keep = (rows >= 0) & (cols >= 0)  # zero boundary moments (walls) are not unknowns
        self.M = sp.csr_matrix((ML.ravel()[keep], (rows[keep], cols[keep])), shape=(sp_.ndof, sp_.ndof))
        prow = (np.arange(T)[:, None] * npr + np.arange(npr)[None, :])
        brow = np.repeat(prow, sp_.nu, axis=1).ravel()
        bcol = np.tile(sp_.dofs, (1, npr)).ravel()
        keep = bcol >= 0
        self.B = sp.csr_matrix((BL.ravel()[keep], (brow[keep], bcol[keep])), shape=(sp_.npres, sp_.ndof))
        self.c = cmean.ravel()

    def saddle_matrix(self):
        n, p = self.space.ndof, self.space.npres
        if self.mesh.open.any():
            # an outflow boundary fixes the pressure (p = 0 there, Sec. 2.5): no mean constraint;
            # the unused mean multiplier keeps the unknowns' layout (an identity row)
            K = sp.bmat([[self.M, -self.B.T, None], [-self.B, None, None], [None, None, sp.identity(1)]],
                        format="csc")
            return K
        c = sp.csr_matrix(self.c.reshape(-1, 1))
        K = sp.bmat([[self.M, -self.B.T, None],
                     [-self.B, None, c],
                     [None, c.T, None]], format="csc")
        assert K.shape == (n + p + 1, n + p + 1)
        return K

    def factor(self):
        if self._lu is None:
            self._lu = spla.splu(self.saddle_matrix())
        return self._lu

    def mass_solve(self, F, return_pressure=False):
        """Divergence-free mass inversion of the functional F (values on the BDM basis)."""
        n, p = self.space.ndof, self.space.npres
        rhs = np.zeros(n + p + 1, dtype=F.dtype)
        rhs[:n] = F
        lu = self.factor()
        if np.iscomplexobj(rhs):
            sol = lu.solve(rhs.real) + 1j * lu.solve(rhs.imag)
        else:
            sol = lu.solve(rhs)
        if return_pressure:
            return sol[:n], sol[n:n + p]
        return sol[:n]

    # ---- data transfer ----------------------------------------------------------------
    def project(self, field, degree=None):
        """L2 projection of the vector field ``field(x, y) -> (u1, u2)`` onto V^{k,-1}.

        The right-hand side int u0 . psi uses a rule of degree 2k+10 (2D) or 2k+6 (3D) by
        default.
        """
        k = self.k
        rule = simplex_rule(self.d, (2 * k + 10 if self.d == 2 else 2 * k + 6) if degree is None else degree)
        x = self.phys_points(rule[0])
        u = field(*[x[..., i] for i in range(self.d)])
        R = self.space.load_vector(np.stack(u, axis=1), rule)
        return self.mass_solve(self.space.assemble(R))

    def phys_points(self, ref_pts):
        """Physical coordinates [T, P, 2] of reference points (unwrapped per element)."""
        m = self.mesh
        return m.xyz[:, None, 0, :] + np.einsum("tir,pr->tpi", m.J, ref_pts)

    def eval_ref(self, U, ref_pts):
        if self.cLift is None:
            return self.space.eval_ref(U, ref_pts)
        vals, _ = poly_basis_nd(self.k, ref_pts)
        return np.einsum("tca,pa->tcp", self.state_local(U), vals)

    # ---- time stepping (eq. (rk3), mass-matrix form) ------------------------------
    def L(self, U):
        if self.cLift is None:
            return self.res(U)
        return self.space.assemble(self.res.broken(self.state_local(U)))

    def rk3_step(self, U, dt):
        """One TVD-RK3 step: each stage solves M u^(s) = (combination of M u + dt L(u))."""
        M = self.M
        MU = M @ U
        U1 = self.mass_solve(MU + dt * self.L(U))
        U2 = self.mass_solve(0.75 * MU + 0.25 * (M @ U1 + dt * self.L(U1)))
        return self.mass_solve(MU / 3.0 + 2.0 / 3.0 * (M @ U2 + dt * self.L(U2)))

    def rk4_step(self, U, dt):
        """One step of the classical four-stage RK4 (Sec. 4, Example 1b) for M du/dt = L(u):
        k_i = M^{-1} L(u_i) by the divergence-free mass inversion of L(u_i), u_1 = u^n,
        u_2 = u^n + dt/2 k_1, u_3 = u^n + dt/2 k_2, u_4 = u^n + dt k_3,
        u^{n+1} = u^n + dt/6 (k_1 + 2 k_2 + 2 k_3 + k_4)."""
        k1 = self.mass_solve(self.L(U))
        k2 = self.mass_solve(self.L(U + 0.5 * dt * k1))
        k3 = self.mass_solve(self.L(U + 0.5 * dt * k2))
        k4 = self.mass_solve(self.L(U + dt * k3))
        return U + dt / 6.0 * (k1 + 2.0 * k2 + 2.0 * k3 + k4)

    def fe_step(self, U, dt):
        """One forward-Euler step, eq. (FE): (u^{n+1}, v) = (u^n, v) + dt L(u^n)(v) for all v
        in the divergence-free space (the time stepping of Example 5)."""
        return self.mass_solve(self.M @ U + dt * self.L(U))

    def run(self, U, dt, steps, callback=None, step=None):
        step = self.rk3_step if step is None else step
        for n in range(steps):
            U = step(U, dt)
            if callback is not None:
                callback(n + 1, U)
        return U

    # ---- diagnostics ------------------------------------------------------------------
    # Each diagnostic is written on the element-local coefficients cU[T, 2, nm] of a broken
    # field (any piecewise polynomial of degree <= k, in or outside BDM_k); the global-vector
    # versions convert first.  Example 2 of Sec. 4 reports the energy and the enstrophy.
    def energy(self, U):
        """Kinetic energy 1/2 ||u_h||^2."""
        return 0.5 * float(U @ (self.M @ U))

    def energy_local(self, cU):
        """1/2 ||u_h||^2 of a broken field (degree-2k rule: exact)."""
        pts, w = simplex_rule(self.d, 2 * self.k)
        vals, _ = poly_basis_nd(self.k, pts)
        u = np.einsum("tca,qa->tcq", cU, vals)
        return 0.5 * float(np.einsum("q,t,tcq->", w, self.mesh.detJ, u * u))

    def l2_diff(self, valsA, valsB, rule):
        """L2 norm of the difference of two fields given at the points of ``rule``."""
        _, w = rule
        d = valsA - valsB
        return float(np.sqrt(np.einsum("q,t,tcq->", w, self.mesh.detJ, d * d)))

    def l2_error_to(self, U, field, degree=None):
        rule = simplex_rule(self.d, (2 * self.k + 10 if self.d == 2 else 2 * self.k + 6) if degree is None
                            else degree)
        uh = self.eval_ref(U, rule[0])
        x = self.phys_points(rule[0])
        u = field(*[x[..., i] for i in range(self.d)])
        return self.l2_diff(uh, np.stack(u, axis=1), rule)

    def _phys_gradients(self, cU, pts):
        """g[t, q, c, j] = d u_c / d x_j of a broken field at reference points pts[Q, d]."""
        _, dref = poly_basis_nd(self.k, pts)
        return np.einsum("tca,qra,trj->tqcj", cU, dref, self.mesh.Jinv)

    def divergence_max(self, U, pts=None):
        """max over elements and points of |div u_h| (pointwise; by default at the points
        of the degree-2k rule)."""
        return self.divergence_max_local(self.space.local_coeffs(U), pts)

    def divergence_max_local(self, cU, pts=None):
        if pts is None:
            pts, _ = simplex_rule(self.d, 2 * self.k)
        g = self._phys_gradients(cU, np.asarray(pts, dtype=float))
        return float(np.abs(np.einsum("tqcc->tq", g)).max())

    def normal_jump_max(self, U):
        """max over facet quadrature points of |u_A . n - u_B . n|."""
        return self.normal_jump_max_local(self.space.local_coeffs(U))

    def normal_jump_max_local(self, cU):
        """max over the facet rule's points (the rule of the residual's facet integrals) of
        the normal jump |u_A . n - u_B . n| of a broken field."""
        m = self.mesh
        s, _ = facet_rule(self.d, self.k)
        xa, xb = m.facet_points(s)
        va, _ = poly_basis_nd(self.k, xa)
        vb, _ = poly_basis_nd(self.k, xb)
        uA = np.einsum("eca,era->erc", cU[m.fA_elem], va)
        uB = np.einsum("eca,era->erc", cU[m.fB_elem], vb)
        uB = np.where(m.bnd[:, None, None], 0.0, uB)  # walls: the jump is u . n itself
        jn = np.abs(np.einsum("erc,ec->er", uA - uB, m.normal))
        return float(np.where(m.open[:, None], 0.0, jn).max())  # outflow: u . n is free

    def enstrophy(self, U):
        """||curl_h u_h||^2 with the element-wise curl du2/dx - du1/dy."""
        return self.enstrophy_local(self.space.local_coeffs(U))

    def enstrophy_local(self, cU):
        """||curl_h u_h||^2 of a broken field (degree-2k rule: the squared curl has degree
        2k - 2, so the integral is exact).  2D: curl = du2/dx - du1/dy; 3D: the vector
        curl (du3/dy - du2/dz, du1/dz - du3/dx, du2/dx - du1/dy)."""
        pts, w = simplex_rule(self.d, 2 * self.k)
        g = self._phys_gradients(cU, pts)
        if self.d == 2:
            om2 = (g[:, :, 1, 0] - g[:, :, 0, 1]) ** 2
        else:
            om2 = ((g[:, :, 2, 1] - g[:, :, 1, 2]) ** 2 + (g[:, :, 0, 2] - g[:, :, 2, 0]) ** 2
                   + (g[:, :, 1, 0] - g[:, :, 0, 1]) ** 2)
        return float(np.einsum("q,t,tq->", w, self.mesh.detJ, om2))


def hybrid_system_dense(orc):
    """Dense matrix of the hybrid-mixed system of eq. (FE3) (tiny meshes only).

    Unknown order: broken velocity [T][d][nm] (local basis), broken pressure
    [T][npr], facet multipliers [E][n_f] in a basis of P^k on the facet, in the facet
    parameter (side A's direction): Legendre P_j(2s-1) on an edge, the reference
    triangle's orthonormal basis (poly_basis) on a face.  Rows: the three equations of
    (FE3), signed so that the matrix is symmetric.  An outflow facet has no multiplier (the
    pressure is zero there, Sec. 2.5): its rows and columns stay zero.  Returns (K, nU, nW).
    """
    m, sp_, k, d = orc.mesh, orc.space, orc.k, orc.d
    T, E, nu, npr, nf = m.T, m.E, sp_.nu, sp_.np_, sp_.nf
    pts, w = simplex_rule(d, 2 * k)
    vals, dref = poly_basis_nd(k, pts)
    nm = sp_.nm
    Mref = np.einsum("q,qa,qb->ab", w, vals, vals)
    z = vals[:, :npr]
    nU, nW, nL = T * nu, T * npr, E * nf
    K = np.zeros((nU + nW + nL, nU + nW + nL))
    s, ws, lbasis = facet_moment_rule(d, k)  # weights summing to 1
    if d == 2:
        lbasis = np.stack([np.polynomial.legendre.legval(2 * s[:, 0] - 1, np.eye(nf)[j]) for j in range(nf)], axis=1)
    for t in range(T):
        iu = slice(t * nu, (t + 1) * nu)
        iw = slice(nU + t * npr, nU + (t + 1) * npr)
        for c in range(d):
            K[iu, iu][c * nm:(c + 1) * nm, c * nm:(c + 1) * nm] = m.detJ[t] * Mref
        div_phi = np.einsum("qra,rc->qca", dref, m.Jinv[t])
        D = np.einsum("q,qp,qca->pca", w, z, div_phi).reshape(npr, nu) * m.detJ[t]
        K[iw, iu] = -D
        K[iu, iw] = -D.T
        for f in range(d + 1):
            xh, F = m.element_facet_points(np.array([t]), np.array([f]), s)
            F = int(F[0])
            if m.open[F]:
                continue
            v, _ = poly_basis_nd(k, xh[0])                             # [R, nm]
            isA = (m.fA_elem[F] == t) and (m.fA_loc[F] == f)
            nT = m.normal[F] if isA else -m.normal[F]
            for j in range(nf):
                mom = (ws * lbasis[:, j]) @ v * m.flen[F]                # int_F l_j m_a dS
                row = nU + nW + F * nf + j
                for c in range(d):
                    K[t * nu + c * nm: t * nu + (c + 1) * nm, row] += mom * nT[c]
                    K[row, t * nu + c * nm: t * nu + (c + 1) * nm] += mom * nT[c]
    return K, nU, nW


def hybrid_solve_dense(orc, Fbroken):
    """Hybrid-mixed solve of eq. (FE3), written out densely (tiny meshes only).

    Unknowns: broken [P^k]^d velocity (local basis per element), broken
    P^{k-1} pressure w, facet multiplier lambda in P^k(F) (basis of hybrid_system_dense).
    Fbroken[T, d, nm] holds the functional on the broken local basis.  The system is singular only by the constant (w, lambda) = (c, c);
    it is solved in the least-squares sense.  Returns the velocity's local
    coefficients cU[T, 2, nm].
    """
    K, nU, _ = hybrid_system_dense(orc)
    rhs = np.zeros(K.shape[0])
    rhs[:nU] = Fbroken.reshape(-1)
    sol = np.linalg.lstsq(K, rhs, rcond=None)[0]
    return sol[:nU].reshape(orc.mesh.T, orc.d, orc.space.nm)
