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
from .quadrature import gauss_legendre_01, facet_rule_points, poly_basis, triangle_rule
from .residual import Residual


class Oracle:
    """Plain FP64 reference solver on a periodic triangle mesh.

    xyz[T, 3, 2]: counter-clockwise element vertices; period[2] or None.
    """

    def __init__(self, xyz, period, k, nu=0.0, alpha=2.0):
        self.mesh = OracleMesh(xyz, period)
        self.k = k
        self.space = BDMSpace(self.mesh, k)
        self.res = Residual(self.space, nu=nu, alpha=alpha)
        self._assemble()
        self._lu = None

    # ---- matrices ----------------------------------------------------------------
    def _assemble(self):
        sp_, m, k = self.space, self.mesh, self.k
        pts, w = triangle_rule(2 * k)
        vals, dref = poly_basis(k, pts[:, 0], pts[:, 1])            # [q, nm], [q, 2, nm]
        nm, npr = sp_.nm, sp_.np_
        # element mass in the local basis (block-diagonal over components)
        Mref = np.einsum("q,qa,qb->ab", w, vals, vals)
        Mphi = np.zeros((sp_.nu, sp_.nu))
        Mphi[:nm, :nm] = Mref
        Mphi[nm:, nm:] = Mref
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
        self.M = sp.csr_matrix((ML.ravel(), (rows, cols)), shape=(sp_.ndof, sp_.ndof))
        prow = (np.arange(T)[:, None] * npr + np.arange(npr)[None, :])
        brow = np.repeat(prow, sp_.nu, axis=1).ravel()
        bcol = np.tile(sp_.dofs, (1, npr)).ravel()
        self.B = sp.csr_matrix((BL.ravel(), (brow, bcol)), shape=(sp_.npres, sp_.ndof))
        self.c = cmean.ravel()

    def saddle_matrix(self):
        n, p = self.space.ndof, self.space.npres
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

        The right-hand side int u0 . psi uses a rule of degree 2k+10 by default.
        """
        k = self.k
        rule = triangle_rule(2 * k + 10 if degree is None else degree)
        x = self.phys_points(rule[0])
        u1, u2 = field(x[..., 0], x[..., 1])
        R = self.space.load_vector(np.stack([u1, u2], axis=1), rule)
        return self.mass_solve(self.space.assemble(R))

    def phys_points(self, ref_pts):
        """Physical coordinates [T, P, 2] of reference points (unwrapped per element)."""
        m = self.mesh
        return m.xyz[:, None, 0, :] + np.einsum("tir,pr->tpi", m.J, ref_pts)

    def eval_ref(self, U, ref_pts):
        return self.space.eval_ref(U, ref_pts)

    # ---- time stepping (eq. (rk3), mass-matrix form) ------------------------------
    def L(self, U):
        return self.res(U)

    def rk3_step(self, U, dt):
        """One TVD-RK3 step: each stage solves M u^(s) = (combination of M u + dt L(u))."""
        M = self.M
        MU = M @ U
        U1 = self.mass_solve(MU + dt * self.L(U))
        U2 = self.mass_solve(0.75 * MU + 0.25 * (M @ U1 + dt * self.L(U1)))
        return self.mass_solve(MU / 3.0 + 2.0 / 3.0 * (M @ U2 + dt * self.L(U2)))

    def run(self, U, dt, steps, callback=None):
        for n in range(steps):
            U = self.rk3_step(U, dt)
            if callback is not None:
                callback(n + 1, U)
        return U

    # ---- diagnostics ------------------------------------------------------------------
    def energy(self, U):
        """Kinetic energy 1/2 ||u_h||^2."""
        return 0.5 * float(U @ (self.M @ U))

    def l2_diff(self, valsA, valsB, rule):
        """L2 norm of the difference of two fields given at the points of ``rule``."""
        _, w = rule
        d = valsA - valsB
        return float(np.sqrt(np.einsum("q,t,tcq->", w, self.mesh.detJ, d * d)))

    def l2_error_to(self, U, field, degree=None):
        rule = triangle_rule(2 * self.k + 10 if degree is None else degree)
        uh = self.eval_ref(U, rule[0])
        x = self.phys_points(rule[0])
        u1, u2 = field(x[..., 0], x[..., 1])
        return self.l2_diff(uh, np.stack([u1, u2], axis=1), rule)

    def divergence_max(self, U):
        """max over elements and points of |div u_h| (pointwise, degree-2k rule points)."""
        pts, _ = triangle_rule(2 * self.k)
        _, dref = poly_basis(self.k, pts[:, 0], pts[:, 1])
        cU = self.space.local_coeffs(U)
        g = np.einsum("tca,qra,trc->tq", cU, dref, self.mesh.Jinv)
        return float(np.abs(g).max())

    def normal_jump_max(self, U):
        """max over facet quadrature points of |u_A . n - u_B . n|."""
        m = self.mesh
        s, _ = gauss_legendre_01(facet_rule_points(self.k))
        xa, xb = m.facet_points(s)
        cU = self.space.local_coeffs(U)
        va, _ = poly_basis(self.k, xa[..., 0], xa[..., 1])
        vb, _ = poly_basis(self.k, xb[..., 0], xb[..., 1])
        uA = np.einsum("eca,era->erc", cU[m.fA_elem], va)
        uB = np.einsum("eca,era->erc", cU[m.fB_elem], vb)
        return float(np.abs(np.einsum("erc,ec->er", uA - uB, m.normal)).max())

    def enstrophy(self, U):
        """||curl_h u_h||^2 with the element-wise curl du2/dx - du1/dy."""
        rule = triangle_rule(2 * self.k)
        pts, w = rule
        _, dref = poly_basis(self.k, pts[:, 0], pts[:, 1])
        cU = self.space.local_coeffs(U)
        g = np.einsum("tca,qra,trj->tqcj", cU, dref, self.mesh.Jinv)
        om = g[:, :, 1, 0] - g[:, :, 0, 1]
        return float(np.einsum("q,t,tq->", w, self.mesh.detJ, om * om))


def hybrid_system_dense(orc):
    """Dense matrix of the hybrid-mixed system of eq. (FE3) (tiny meshes only).

    Unknown order: broken velocity [T][2][nm] (local basis), broken pressure
    [T][npr], facet multipliers [E][k+1] in the Legendre basis P_j(2s-1) of the
    facet parameter s (side A's direction).  Rows: the three equations of (FE3),
    signed so that the matrix is symmetric.  Returns (K, nU, nW).
    """
    m, sp_, k = orc.mesh, orc.space, orc.k
    T, E, nu, npr, nf = m.T, m.E, sp_.nu, sp_.np_, sp_.nf
    pts, w = triangle_rule(2 * k)
    vals, dref = poly_basis(k, pts[:, 0], pts[:, 1])
    nm = sp_.nm
    Mref = np.einsum("q,qa,qb->ab", w, vals, vals)
    z = vals[:, :npr]
    nU, nW, nL = T * nu, T * npr, E * nf
    K = np.zeros((nU + nW + nL, nU + nW + nL))
    s, ws = gauss_legendre_01(k + 1)
    for t in range(T):
        iu = slice(t * nu, (t + 1) * nu)
        iw = slice(nU + t * npr, nU + (t + 1) * npr)
        K[iu, iu][:nm, :nm] = m.detJ[t] * Mref
        K[iu, iu][nm:, nm:] = m.detJ[t] * Mref
        div_phi = np.einsum("qra,rc->qca", dref, m.Jinv[t])
        D = np.einsum("q,qp,qca->pca", w, z, div_phi).reshape(npr, nu) * m.detJ[t]
        K[iw, iu] = -D
        K[iu, iw] = -D.T
        for f in range(3):
            xh, F = m.element_facet_points(np.array([t]), np.array([f]), s)
            F = int(F[0])
            v, _ = poly_basis(k, xh[0, :, 0], xh[0, :, 1])          # [R, nm]
            isA = (m.fA_elem[F] == t) and (m.fA_loc[F] == f)
            nT = m.normal[F] if isA else -m.normal[F]
            for j in range(nf):
                lj = np.polynomial.legendre.legval(2 * s - 1, np.eye(nf)[j])
                mom = (ws * lj) @ v * m.flen[F]                       # [nm]
                row = nU + nW + F * nf + j
                for c in range(2):
                    K[t * nu + c * nm: t * nu + (c + 1) * nm, row] += mom * nT[c]
                    K[row, t * nu + c * nm: t * nu + (c + 1) * nm] += mom * nT[c]
    return K, nU, nW


def hybrid_solve_dense(orc, Fbroken):
    """Hybrid-mixed solve of eq. (FE3), written out densely (tiny meshes only).

    Unknowns: broken [P^k]^2 velocity (monomial basis per element), broken
    P^{k-1} pressure w, facet multiplier lambda in P^k(F) (Legendre basis in the
    facet parameter).  Fbroken[T, 2, nm] holds the functional on the broken
    local basis.  The system is singular only by the constant (w, lambda) = (c, c);
    it is solved in the least-squares sense.  Returns the velocity's local
    coefficients cU[T, 2, nm].
    """
    K, nU, _ = hybrid_system_dense(orc)
    rhs = np.zeros(K.shape[0])
    rhs[:nU] = Fbroken.reshape(-1)
    sol = np.linalg.lstsq(K, rhs, rcond=None)[0]
    return sol[:nU].reshape(orc.mesh.T, 2, orc.space.nm)
