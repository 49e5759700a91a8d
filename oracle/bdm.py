"""Global H(div)-conforming BDM_k basis of the oracle (Sec. 2.1, eq. (space-3)).

On each element the velocity is expanded in the basis Phi_(c,a) = m_a(xi, eta) e_c
of [P^k]^2, where m_a are the reference-orthonormal polynomials of
``quadrature.poly_basis`` and e_c the Cartesian unit vectors.  The BDM_k degrees
of freedom are the facet-averaged normal moments (1/|F|) int_F l_j (v . n_F) ds
against orthonormal Legendre polynomials l_j, j = 0..k, on each facet (with the
facet's global normal and parameter), plus interior functions
with zero normal moments.  With N_T the element's moment matrix, the local
basis is Phi [pinv(N_T) | null(N_T)]: functions carrying one facet moment each,
followed by a basis of the moment-free (interior) functions.  Two elements that
share a facet DOF then have the same normal trace there, so the assembled
functions are in H(div).
"""
import numpy as np

from .quadrature import gauss_legendre_01, legendre01, poly_basis, triangle_rule


def n_mono(k):
    return (k + 1) * (k + 2) // 2


class BDMSpace:
    """Global BDM_k velocity and broken P^{k-1} pressure on an OracleMesh."""

    def __init__(self, mesh, k):
        if k < 1:
            raise ValueError("k >= 1")
        self.mesh = mesh
        self.k = k
        self.nm = n_mono(k)          # scalar polynomials of degree <= k
        self.nu = 2 * self.nm        # local velocity functions
        self.np_ = n_mono(k - 1)     # local pressure functions (degree <= k-1)
        self.nf = k + 1              # moments per facet
        self.nint = self.nu - 3 * self.nf
        T, E = mesh.T, mesh.E
        self.ndof = E * self.nf + T * self.nint
        self.npres = T * self.np_
        self._build_local_bases()

    def _build_local_bases(self):
        m, k, T = self.mesh, self.k, self.mesh.T
        s, w = gauss_legendre_01(k + 1)  # exact for the degree-2k moment integrands
        N = np.zeros((T, 3 * self.nf, self.nu))
        tt = np.arange(T)
        for f in range(3):
            xh, F = m.element_facet_points(tt, np.full(T, f), s)
            vals, _ = poly_basis(k, xh[..., 0], xh[..., 1])  # [T, R, nm]
            n = m.normal[F]  # [T, 2]
            for j in range(self.nf):
                lj = np.sqrt(2 * j + 1) * legendre01(j, s)  # orthonormal on [0, 1]
                # facet-averaged moment (1/|F|) int_F l_j v.n ds = sum_r w_r l_j(s_r) v.n
                mom = np.einsum("r,r,tra->ta", w, lj, vals)
                for c in range(2):
                    N[:, f * self.nf + j, c * self.nm:(c + 1) * self.nm] = mom * n[:, c:c + 1]
        self.N = N
        pinv = np.linalg.pinv(N)                      # [T, nu, 3nf]
        _, _, vh = np.linalg.svd(N, full_matrices=True)
        null = np.transpose(vh[:, 3 * self.nf:, :], (0, 2, 1))  # [T, nu, nint]
        self.A = np.concatenate([pinv, null], axis=2)  # [T, nu, nu]
        # local -> global numbering
        dofs = np.empty((T, self.nu), dtype=np.int64)
        for f in range(3):
            F = m.elem_facet[:, f]
            for j in range(self.nf):
                dofs[:, f * self.nf + j] = F * self.nf + j
        E = m.E
        dofs[:, 3 * self.nf:] = E * self.nf + tt[:, None] * self.nint + np.arange(self.nint)[None, :]
        self.dofs = dofs

    # ---- coefficient conversions -------------------------------------------------
    def local_coeffs(self, U):
        """Local coefficients cU[T, 2, nm] of the global BDM vector U (any dtype)."""
        c = np.einsum("tab,tb->ta", self.A, U[self.dofs])
        return c.reshape(self.mesh.T, 2, self.nm)

    def assemble(self, R):
        """Functional on the global basis from its values R[T, 2, nm] on the local Phi."""
        Rl = np.einsum("tab,ta->tb", self.A, R.reshape(self.mesh.T, self.nu))
        out = np.zeros(self.ndof, dtype=Rl.dtype)
        np.add.at(out, self.dofs.ravel(), Rl.ravel())
        return out

    def eval_ref(self, U, ref_pts):
        """Values [T, 2, P] of the BDM function U at reference points ref_pts[P, 2]."""
        vals, _ = poly_basis(self.k, ref_pts[:, 0], ref_pts[:, 1])  # [P, nm]
        return np.einsum("tca,pa->tcp", self.local_coeffs(U), vals)

    def load_vector(self, f_at_q, rule):
        """R[T, 2, nm] = int_T f . Phi_(c,a) for f given at the points of ``rule``."""
        pts, w = rule
        vals, _ = poly_basis(self.k, pts[:, 0], pts[:, 1])
        return np.einsum("q,t,tcq,qa->tca", w, self.mesh.detJ, f_at_q, vals)

    def broken_project(self, f_at_q, rule):
        """Local coefficients cU[T, 2, nm] of the element-wise L2 projection onto [P^k]^2.

        Reproduces broken polynomial data of degree <= k exactly when the rule is exact
        for degree 2k.
        """
        pts, w = rule
        vals, _ = poly_basis(self.k, pts[:, 0], pts[:, 1])
        Mref = np.einsum("q,qa,qb->ab", w, vals, vals)
        rhs = np.einsum("q,tcq,qa->tca", w, f_at_q, vals)
        return np.linalg.solve(Mref, rhs.reshape(-1, self.nm).T).T.reshape(f_at_q.shape[0], 2, self.nm)

    def volume_rule(self, degree):
        return triangle_rule(degree)
