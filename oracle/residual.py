"""The DG operator L(u)(v) = -C_h(u; u, v) - B_h(u, v) on broken test functions.

C_h is the upwind convective form (Sec. 2.2, eq. (adv)); B_h the symmetric
interior penalty viscous form with penalty nu alpha k^2 / h (Sec. 3,
eq. (viscous)).  Readings of the paper used here:

* the upwind value is chosen pointwise at each facet quadrature point, from the
  side whose outward normal satisfies u . n >= 0, with u . n the two-sided
  average (identical to either side for H(div) velocities);
* jumps of vectors and tensors are the tensor jumps [[u (x) n]] = u+ (x) n+ + u- (x) n-,
  (grad u)_ij = du_i/dx_j and ":" the Frobenius product;
* h in the penalty is h_F = min(h_T+, h_T-) with h_T = (d! |T|)^(1/d);
* walls (boundary facets): u . n = 0 there, so the convective boundary term vanishes, and
  the viscous facet terms run over interior facets only (eq. (viscous), free-slip
  condition (ns-4) natural): boundary facets contribute nothing.

The residual is returned on the broken local basis Phi_(c,a) of every element:
R[t, c, a] = L(u)(m_a e_c restricted to element t), m_a the local polynomial basis.  The
code is the same for triangles and tetrahedra (d = 2, 3): only the rules differ.  It works for complex
coefficients too (the upwind switch then uses the real part), which the adjoint
module uses for complex-step derivatives.
"""
import numpy as np

from .quadrature import facet_rule, poly_basis_nd, simplex_rule


def _phys_grad(dref, Jinv):
    """d m_a/dx_j = sum_r d m_a/dxi_r * Jinv[r, j]; dref[..., r, a], Jinv[..., r, j]."""
    return np.einsum("...ra,...rj->...ja", dref, Jinv)


class Residual:
    def __init__(self, space, nu=0.0, alpha=2.0, chunk=8192):
        self.space = space
        self.mesh = space.mesh
        self.k = space.k
        self.nu = float(nu)
        self.alpha = float(alpha)
        self.chunk = chunk
        k = self.k
        m = self.mesh
        # volume rule: degree 3k+2 (>= 3k-1 needed by (u (x) u) : grad v)
        self.vpts, self.vw = simplex_rule(m.d, 3 * k + 2)
        self.vm, self.vdm = poly_basis_nd(k, self.vpts)
        # facet rule, weights summing to 1 (times the facet measure below)
        self.fs, self.fw = facet_rule(m.d, k)
        xa, xb = m.facet_points(self.fs)
        self.fmA, self.fdmA = poly_basis_nd(k, xa)  # [E,R,nm], [E,R,d,nm]
        self.fmB, self.fdmB = poly_basis_nd(k, xb)
        self.sigma = self.alpha * k * k / m.hF  # penalty per facet

    # ---------------------------------------------------------------------------------
    def volume(self, cU, out):
        """Element integrals: + int_T (u (x) u) : grad v  -  nu int_T grad u : grad v."""
        m = self.mesh
        for t0 in range(0, m.T, self.chunk):
            sl = slice(t0, min(t0 + self.chunk, m.T))
            c = cU[sl]
            Jinv = m.Jinv[sl]
            u = np.einsum("tca,qa->tqc", c, self.vm)
            gref = np.einsum("tca,qra->tqcr", c, self.vdm)
            grad = np.einsum("tqcr,trj->tqcj", gref, Jinv)          # du_c/dx_j
            conv = np.einsum("tqi,tqj->tqij", u, u)                  # u (x) u
            flux = conv - self.nu * grad
            gv = np.einsum("qra,trj->tqja", self.vdm, Jinv)          # d m_a/dx_j
            out[sl] += np.einsum("q,t,tqcj,tqja->tca", self.vw, m.detJ[sl], flux, gv)

    def facet_terms(self, cUA, cUB):
        """Facet integrals of -C_h (upwind) and -B_h (consistency, symmetry, penalty).

        cUA[E, 2, nm], cUB[E, 2, nm]: coefficients of the two sides of every facet.
        Returns the contributions (RA, RB) to the test functions of sides A and B.
        """
        m = self.mesh
        A, B = m.fA_elem, m.fB_elem
        n = m.normal                      # A's outward normal, [E, d]
        nA, nB = n, -n
        uA = np.einsum("eca,era->erc", cUA, self.fmA)
        uB = np.einsum("eca,era->erc", cUB, self.fmB)
        gA = np.einsum("eca,ersa,esj->ercj", cUA, self.fdmA, m.Jinv[A])
        gB = np.einsum("eca,ersa,esj->ercj", cUB, self.fdmB, m.Jinv[B])
        # test-function gradients on each side
        tgA = np.einsum("ersa,esj->erja", self.fdmA, m.Jinv[A])
        tgB = np.einsum("ersa,esj->erja", self.fdmB, m.Jinv[B])
        wq = self.fw[None, :] * m.flen[:, None]  # [E, R]

        # ---- convection: -sum_T int_{dT} (u . n_T)(u^up . v) -----------------------
        un_A = 0.5 * np.einsum("erc,ec->er", uA + uB, nA)      # u . n_A
        upwind_is_A = np.real(un_A) >= 0.0                     # outflow side of A
        uup = np.where(upwind_is_A[..., None], uA, uB)
        un_B = -un_A
        convA = -np.einsum("er,er,erc,era->eca", wq, un_A, uup, self.fmA)
        convB = -np.einsum("er,er,erc,era->eca", wq, un_B, uup, self.fmB)

        # ---- viscosity (interior facets) ------------------------------------------
        avg_grad = 0.5 * (gA + gB)                                              # {grad u}
        jump_u = (np.einsum("erc,ej->ercj", uA, nA) + np.einsum("erc,ej->ercj", uB, nB))  # [[u (x) n]]
        sig = self.sigma[:, None]
        nu = self.nu
        # +nu {grad u} : [[v (x) n]] with v = m_a e_c on side X: sum_j {grad u}_cj n_Xj m_a
        viscA = nu * np.einsum("er,ercj,ej,era->eca", wq, avg_grad, nA, self.fmA)
        viscB = nu * np.einsum("er,ercj,ej,era->eca", wq, avg_grad, nB, self.fmB)
        # +nu {grad v} : [[u (x) n]] with {grad v}_cj = 1/2 d m_a/dx_j on side X
        viscA += nu * np.einsum("er,ercj,erja->eca", wq, jump_u, 0.5 * tgA)
        viscB += nu * np.einsum("er,ercj,erja->eca", wq, jump_u, 0.5 * tgB)
        # -nu alpha k^2/h [[u (x) n]] : [[v (x) n]]
        viscA -= nu * np.einsum("er,er,ercj,ej,era->eca", wq, sig, jump_u, nA, self.fmA)
        viscB -= nu * np.einsum("er,er,ercj,ej,era->eca", wq, sig, jump_u, nB, self.fmB)
        inner = (~m.bnd).astype(float)[:, None, None]  # boundary facets: no terms, except
        # on an outflow boundary: -int max(u.n, 0) (u . v) with the own trace (the exterior
        # state of backflow is zero; no viscous facet terms on any boundary)
        opn = m.open.astype(float)[:, None, None]
        uAn = np.einsum("erc,ec->er", uA, nA)
        out = np.where(np.real(uAn) > 0.0, uAn, 0.0)
        convO = -np.einsum("er,er,erc,era->eca", wq, out, uA, self.fmA)
        return (convA + viscA) * inner + convO * opn, (convB + viscB) * inner

    def facets(self, cU, out):
        m = self.mesh
        RA, RB = self.facet_terms(cU[m.fA_elem], cU[m.fB_elem])
        np.add.at(out, m.fA_elem, RA)
        np.add.at(out, m.fB_elem, RB)

    def broken(self, cU):
        """R[T, 2, nm] = L(u)(Phi_(c,a)) for the field with local coefficients cU."""
        out = np.zeros(cU.shape, dtype=cU.dtype)
        self.volume(cU, out)
        self.facets(cU, out)
        return out

    def __call__(self, U):
        """L(u) on the global BDM basis for the global coefficient vector U."""
        return self.space.assemble(self.broken(self.space.local_coeffs(U)))
