"""Oracle mesh topology: affine maps, facets and periodic facet matching.

Notation follows Sec. 2.1 of the paper: T_h the triangulation of Omega in R^d (d = 2, 3),
F_h its facets; on a periodic mesh every facet is interior and has two sides.  A period
component 0 makes the domain non-periodic in that direction: its boundary facets (one side
only) carry the no-flow condition u . n = 0 of eq. (euler-3) with g = 0.
"""
from math import factorial

import numpy as np


def local_facet_vertices(d, f):
    """Local vertices of local facet f: in 2D the counter-clockwise edge (f+1)%3 -> (f+2)%3;
    in 3D the face opposite vertex f, its other vertices in increasing order."""
    if d == 2:
        return ((f + 1) % 3, (f + 2) % 3)
    return tuple(v for v in range(4) if v != f)


class OracleMesh:
    """Simplex mesh given by per-element vertex coordinates xyz[T, d+1, d] (positively
    oriented: counter-clockwise triangles, tetrahedra with det J > 0).

    Facets of different elements are identified when their barycentres agree modulo the
    period.  For each facet the first element found is side A, the second side B; the
    facet normal n is A's outward normal and the facet parameter s (s in [0, 1] in 2D,
    (s, t) in the reference triangle in 3D) runs along A's local facet vertices:
    x = a_0 + sum_r s_r (a_{r+1} - a_0).  Where a period component is 0, facets left
    without a partner are boundary facets: bnd[F] is set and side B repeats side A (the
    operators give boundary facets their own terms).  A boundary facet is closed (a wall,
    or an inflow boundary: the normal velocity is given there) unless ``outflow(mid)``,
    called with the boundary facets' barycentres [n, d], marks it open (an outflow
    boundary of Sec. 2.5, where the pressure is zero and u.n is free): open[F].
    """

    def __init__(self, xyz, period=None, outflow=None):
        xyz = np.asarray(xyz, dtype=float)
        self.xyz = xyz
        self.T, nv, self.d = xyz.shape
        if nv != self.d + 1 or self.d not in (2, 3):
            raise ValueError("oracle mesh: xyz must be [T, 3, 2] triangles or [T, 4, 3] tetrahedra")
        d = self.d
        self.period = None if period is None else np.asarray(period, dtype=float)
        v0 = xyz[:, 0]
        J = np.stack([xyz[:, r + 1] - v0 for r in range(d)], axis=-1)  # J[t, i, r] = dx_i/dxi_r
        self.J = J
        self.detJ = np.linalg.det(J)
        if np.any(self.detJ <= 0):
            raise ValueError("oracle mesh: elements must be positively oriented and non-degenerate")
        self.Jinv = np.linalg.inv(J)  # Jinv[t, r, i] = dxi_r/dx_i
        self.area = self.detJ / factorial(d)  # element measure |T|
        # h_T = (d! |T|)^(1/d): the mesh-size reading used in the penalty
        self.hT = self.detJ ** (1.0 / d)
        self._match_facets()
        self.open = np.zeros(self.E, dtype=bool)
        if outflow is not None and self.bnd.any():
            F = np.nonzero(self.bnd)[0]
            self.open[F] = np.asarray(outflow(self.PA[F].mean(axis=1)), dtype=bool)

    def _key(self, mid):
        d = self.d
        m = mid.copy()
        per = self.period if self.period is not None else np.zeros(d)
        ext = np.abs(self.xyz).reshape(-1, d).max(axis=0) + 1.0
        scale = np.where(per > 0, per, ext)
        m = np.where(per > 0, np.mod(m, np.where(per > 0, per, 1.0)), m)
        q = np.round(m / scale * 2 ** 30).astype(np.int64)
        q = np.where(per > 0, np.mod(q, 2 ** 30), q)
        return [tuple(r) for r in q]

    def _match_facets(self):
        T, d = self.T, self.d
        nfac = d + 1
        # facet vertex coordinates pv[t, f, j, :] (j over the facet's d vertices)
        pv = np.stack([np.stack([self.xyz[:, v] for v in local_facet_vertices(d, f)], axis=1)
                       for f in range(nfac)], axis=1)
        mid = pv.mean(axis=2)
        keys = self._key(mid.reshape(-1, d))
        first = {}
        sideA, sideB = [], []
        for idx, key in enumerate(keys):
            t, f = divmod(idx, nfac)
            if key in first:
                a = first.pop(key)
                sideA.append(a)
                sideB.append((t, f))
            else:
                first[key] = (t, f)
        walls = self.period is not None and np.any(self.period == 0)
        if first and not walls:
            raise ValueError("oracle mesh: %d unmatched facets (non-periodic boundary)" % len(first))
        nb = len(first)
        for key in sorted(first, key=lambda k_: first[k_]):  # boundary facets: side B := side A
            sideA.append(first[key])
            sideB.append(first[key])
        sideA = np.array(sideA)
        sideB = np.array(sideB)
        self.E = len(sideA)
        self.bnd = np.zeros(self.E, dtype=bool)
        if nb:
            self.bnd[self.E - nb:] = True
        self.fA_elem, self.fA_loc = sideA[:, 0], sideA[:, 1]
        self.fB_elem, self.fB_loc = sideB[:, 0], sideB[:, 1]
        self.elem_facet = np.empty((T, nfac), dtype=np.int64)
        self.elem_facet[self.fB_elem, self.fB_loc] = np.arange(self.E)
        self.elem_facet[self.fA_elem, self.fA_loc] = np.arange(self.E)
        # facet geometry in A's coordinates
        PA = pv[self.fA_elem, self.fA_loc]  # [E, d, d]
        self.PA = PA
        self.P0 = PA[:, 0]
        self.P1 = PA[:, 1]
        if d == 2:
            t = self.P1 - self.P0
            self.flen = np.linalg.norm(t, axis=1)
            self.normal = np.stack([t[:, 1], -t[:, 0]], axis=1) / self.flen[:, None]
        else:
            c = np.cross(PA[:, 1] - PA[:, 0], PA[:, 2] - PA[:, 0])
            nrm = np.linalg.norm(c, axis=1)
            self.flen = 0.5 * nrm  # facet measure (the area of a face)
            n = c / nrm[:, None]
            opp = self.xyz[self.fA_elem, self.fA_loc]  # the vertex opposite the face
            sgn = np.sign(np.einsum("ec,ec->e", n, PA[:, 0] - opp))
            self.normal = n * sgn[:, None]
        # translation carrying A's copy of the facet onto B's copy
        self.shiftB = mid[self.fB_elem, self.fB_loc] - mid[self.fA_elem, self.fA_loc]
        self.hF = np.minimum(self.hT[self.fA_elem], self.hT[self.fB_elem])

    def to_ref(self, t, x):
        """Reference coordinates of physical points x[..., d] in elements t[...]."""
        return np.einsum("...ri,...i->...r", self.Jinv[t], x - self.xyz[t, 0])

    def _facet_phys(self, F, s):
        """Physical points [len(F), R, d] of facet parameters s[R, d-1] (A's copy)."""
        s = np.asarray(s, dtype=float)
        if s.ndim == 1:
            s = s[:, None]
        P = self.PA[F]  # [n, d, d]
        x = P[:, None, 0, :] + np.einsum("rj,njc->nrc", s, P[:, 1:, :] - P[:, :1, :])
        return x

    def facet_points(self, s):
        """Points of parameter s on every facet, in A's and in B's reference coordinates.

        s[R] (2D) or s[R, d-1]; returns (xhatA[E, R, d], xhatB[E, R, d]).
        """
        x = self._facet_phys(np.arange(self.E), s)
        xa = self.to_ref(self.fA_elem[:, None], x)
        xb = self.to_ref(self.fB_elem[:, None], x + self.shiftB[:, None, :])
        return xa, xb

    def element_facet_points(self, t, f, s):
        """Points of facet parameter s on local facet f of element t (facet orientation).

        Used for the BDM moments: the parameter is the facet's global one (A's
        direction), expressed in element t's own coordinates.
        """
        F = self.elem_facet[t, f]
        x = self._facet_phys(F, s)
        isB = (self.fB_elem[F] == t) & (self.fB_loc[F] == f)
        x = x + np.where(isB[:, None, None], self.shiftB[F][:, None, :], 0.0)
        return self.to_ref(t[:, None], x), F
