"""Global H(div)-conforming BDM_k basis of the oracle (Sec. 2.1, eq. (space-3)), d = 2, 3.

On each element the velocity is expanded in the basis Phi_(c,a) = m_a(xhat) e_c of
[P^k]^d, where m_a are the reference-orthonormal polynomials of ``quadrature.poly_basis``
(``poly_basis3`` on tetrahedra) and e_c the Cartesian unit vectors.  The BDM_k degrees of
freedom are facet-averaged normal moments (1/|F|) int_F l_j (v . n_F) dS against a basis
l_j of P^k on the facet (orthonormal Legendre polynomials on an edge, orthonormal
polynomials of the reference triangle on a face), with the facet's global normal and
parameter, plus interior functions with zero normal moments.  With N_T the element's
moment matrix, the local basis is Phi [pinv(N_T) | null(N_T)]: functions carrying one facet
moment each, followed by a basis of the moment-free (interior) functions.  Two elements
that share a facet DOF then have the same normal trace there, so the assembled functions
are in H(div).  On a mesh with walls (boundary facets) the normal moments of the boundary
facets are not degrees of freedom: they are zero, so the space is BDM_k in H_0(div) of eq.
(space-3) (no flow through the walls); local DOFs there map to -1.  The same holds on an
inflow boundary for the space of increments (the normal velocity is given there, Sec.
2.5); on an outflow boundary (mesh.open) the normal moments are degrees of freedom of the
one element that has the facet.
"""
import numpy as np

from .quadrature import facet_moment_rule, poly_basis_nd, simplex_rule


def n_mono(k, d=2):
    """dim P^k in d variables."""
    if k < 0:
        return 0
    if d == 1:
        return k + 1
    if d == 2:
        return (k + 1) * (k + 2) // 2
    return (k + 1) * (k + 2) * (k + 3) // 6


class BDMSpace:
    """Global BDM_k velocity and broken P^{k-1} pressure on an OracleMesh."""

    def __init__(self, mesh, k):
        if k < 1:
            raise ValueError("k >= 1")
        self.mesh = mesh
        self.k = k
        d = self.d = mesh.d
        self.nm = n_mono(k, d)           # scalar polynomials of degree <= k
        self.nu = d * self.nm            # local velocity functions
        self.np_ = n_mono(k - 1, d)      # local pressure functions (degree <= k-1)
        self.nf = n_mono(k, d - 1)       # moments per facet
        self.nfac = d + 1                # facets per element
        self.nint = self.nu - self.nfac * self.nf
        T, E = mesh.T, mesh.E
        bnd = getattr(mesh, "bnd", np.zeros(E, dtype=bool))
        carry = ~bnd | getattr(mesh, "open", np.zeros(E, dtype=bool))
        # slot of each facet among the facets that carry moments (-1: closed boundary facet)
        self.fslot = np.full(E, -1, dtype=np.int64)
        self.fslot[carry] = np.arange(int(carry.sum()))
        self.Eint = int(carry.sum())
        self.ndof = self.Eint * self.nf + T * self.nint
        self.npres = T * self.np_
        self._build_local_bases()

    def _build_local_bases(self):
        m, k, T, d = self.mesh, self.k, self.mesh.T, self.d
        s, w, lbasis = facet_moment_rule(d, k)  # exact for the degree-2k moment integrands
        nr = self.nfac * self.nf
        N = np.zeros((T, nr, self.nu))
        tt = np.arange(T)
        for f in range(self.nfac):
            xh, F = m.element_facet_points(tt, np.full(T, f), s)
            vals, _ = poly_basis_nd(k, xh)  # [T, R, nm]
            n = m.normal[F]  # [T, d]
            for j in range(self.nf):
                # facet-averaged moment (1/|F|) int_F l_j v.n dS = sum_r w_r l_j(s_r) v.n
                mom = np.einsum("r,r,tra->ta", w, lbasis[:, j], vals)
                for c in range(d):
                    N[:, f * self.nf + j, c * self.nm:(c + 1) * self.nm] = mom * n[:, c:c + 1]
        self.N = N
        pinv = np.linalg.pinv(N)                      # [T, nu, nr]
        _, _, vh = np.linalg.svd(N, full_matrices=True)
        null = np.transpose(vh[:, nr:, :], (0, 2, 1))  # [T, nu, nint]
        self.A = np.concatenate([pinv, null], axis=2)  # [T, nu, nu]
        # local -> global numbering
        dofs = np.empty((T, self.nu), dtype=np.int64)
        for f in range(self.nfac):
            sl = self.fslot[m.elem_facet[:, f]]
            for j in range(self.nf):
                dofs[:, f * self.nf + j] = np.where(sl >= 0, sl * self.nf + j, -1)
        dofs[:, nr:] = self.Eint * self.nf + tt[:, None] * self.nint + np.arange(self.nint)[None, :]
        self.dofs = dofs
        # gather/scatter index: -1 (a zero boundary moment) goes to a trailing zero slot
        self.dofs_x = np.where(dofs >= 0, dofs, self.ndof)

    # ---- coefficient conversions -------------------------------------------------
    def local_coeffs(self, U):
        """Local coefficients cU[T, d, nm] of the global BDM vector U (any dtype)."""
        Ux = np.concatenate([U, np.zeros(1, dtype=U.dtype)])
        c = np.einsum("tab,tb->ta", self.A, Ux[self.dofs_x])
        return c.reshape(self.mesh.T, self.d, self.nm)

    def assemble(self, R):
        """Functional on the global basis from its values R[T, d, nm] on the local Phi."""
        Rl = np.einsum("tab,ta->tb", self.A, R.reshape(self.mesh.T, self.nu))
        out = np.zeros(self.ndof + 1, dtype=Rl.dtype)
        np.add.at(out, self.dofs_x.ravel(), Rl.ravel())
        return out[:self.ndof]

    def eval_ref(self, U, ref_pts):
        """Values [T, d, P] of the BDM function U at reference points ref_pts[P, d]."""
        vals, _ = poly_basis_nd(self.k, ref_pts)  # [P, nm]
        return np.einsum("tca,pa->tcp", self.local_coeffs(U), vals)

    def load_vector(self, f_at_q, rule):
        """R[T, d, nm] = int_T f . Phi_(c,a) for f given at the points of ``rule``."""
        pts, w = rule
        vals, _ = poly_basis_nd(self.k, pts)
        return np.einsum("q,t,tcq,qa->tca", w, self.mesh.detJ, f_at_q, vals)

    def broken_project(self, f_at_q, rule):
        """Local coefficients cU[T, d, nm] of the element-wise L2 projection onto [P^k]^d.

        Reproduces broken polynomial data of degree <= k exactly when the rule is exact
        for degree 2k.
        """
        pts, w = rule
        vals, _ = poly_basis_nd(self.k, pts)
        Mref = np.einsum("q,qa,qb->ab", w, vals, vals)
        rhs = np.einsum("q,tcq,qa->tca", w, f_at_q, vals)
        T, dd = f_at_q.shape[0], f_at_q.shape[1]
        return np.linalg.solve(Mref, rhs.reshape(-1, self.nm).T).T.reshape(T, dd, self.nm)

    def volume_rule(self, degree):
        return simplex_rule(self.d, degree)
