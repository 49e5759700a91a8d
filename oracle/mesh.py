"""Oracle mesh topology: affine maps, facets and periodic facet matching.

Notation follows Sec. 2.1 of the paper: T_h the triangulation, F_h its facets;
on a periodic mesh every facet is interior and has two sides.
"""
import numpy as np


class OracleMesh:
    """Triangle mesh given by per-element vertex coordinates (counter-clockwise).

    Local facet f of a triangle joins its vertices (f+1)%3 -> (f+2)%3, traversed
    counter-clockwise.  Facets of different elements are identified when their
    midpoints agree modulo the period.  For each facet the first element found
    is side A, the second side B; the facet normal n is A's outward normal and
    the facet parameter s in [0, 1] runs along A's traversal direction.
    """

    def __init__(self, xyz, period=None):
        xyz = np.asarray(xyz, dtype=float)
        self.xyz = xyz
        self.T = xyz.shape[0]
        self.period = None if period is None else np.asarray(period, dtype=float)
        v0 = xyz[:, 0]
        J = np.stack([xyz[:, 1] - v0, xyz[:, 2] - v0], axis=-1)  # J[t, i, r] = dx_i/dxi_r
        self.J = J
        self.detJ = np.linalg.det(J)
        if np.any(self.detJ <= 0):
            raise ValueError("oracle mesh: elements must be counter-clockwise and non-degenerate")
        self.Jinv = np.linalg.inv(J)  # Jinv[t, r, i] = dxi_r/dx_i
        self.area = 0.5 * self.detJ
        # h_T = (d! |T|)^(1/d): the mesh-size reading used in the penalty.
        self.hT = np.sqrt(2.0 * self.area)
        self._match_facets()

    def _key(self, mid):
        m = mid.copy()
        if self.period is not None:
            m = np.mod(m, self.period)
            scale = self.period
        else:
            scale = np.ones(2)
        q = np.round(m / scale * 2 ** 30).astype(np.int64)
        if self.period is not None:
            q = np.mod(q, 2 ** 30)
        return [tuple(r) for r in q]

    def _match_facets(self):
        T = self.T
        p0 = np.stack([self.xyz[:, (f + 1) % 3] for f in range(3)], axis=1)  # [T,3,2]
        p1 = np.stack([self.xyz[:, (f + 2) % 3] for f in range(3)], axis=1)
        mid = 0.5 * (p0 + p1)
        keys = self._key(mid.reshape(-1, 2))
        first = {}
        sideA, sideB = [], []
        for idx, key in enumerate(keys):
            t, f = divmod(idx, 3)
            if key in first:
                a = first.pop(key)
                sideA.append(a)
                sideB.append((t, f))
            else:
                first[key] = (t, f)
        if first:
            raise ValueError("oracle mesh: %d unmatched facets (non-periodic boundary)" % len(first))
        sideA = np.array(sideA)
        sideB = np.array(sideB)
        self.E = len(sideA)
        self.fA_elem, self.fA_loc = sideA[:, 0], sideA[:, 1]
        self.fB_elem, self.fB_loc = sideB[:, 0], sideB[:, 1]
        # element -> facet map
        self.elem_facet = np.empty((T, 3), dtype=np.int64)
        self.elem_facet[self.fA_elem, self.fA_loc] = np.arange(self.E)
        self.elem_facet[self.fB_elem, self.fB_loc] = np.arange(self.E)
        # facet geometry in A's coordinates
        P0 = p0[self.fA_elem, self.fA_loc]
        P1 = p1[self.fA_elem, self.fA_loc]
        t = P1 - P0
        self.flen = np.linalg.norm(t, axis=1)
        self.normal = np.stack([t[:, 1], -t[:, 0]], axis=1) / self.flen[:, None]
        self.P0 = P0
        self.P1 = P1
        # translation carrying A's copy of the facet onto B's copy
        self.shiftB = mid[self.fB_elem, self.fB_loc] - mid[self.fA_elem, self.fA_loc]
        self.hF = np.minimum(self.hT[self.fA_elem], self.hT[self.fB_elem])

    def to_ref(self, t, x):
        """Reference coordinates of physical points x[..., 2] in elements t[...]."""
        return np.einsum("...ri,...i->...r", self.Jinv[t], x - self.xyz[t, 0])

    def facet_points(self, s):
        """Points of parameter s[R] on every facet, in A's and in B's coordinates.

        Returns (xhatA[E, R, 2], xhatB[E, R, 2]).
        """
        x = self.P0[:, None, :] + s[None, :, None] * (self.P1 - self.P0)[:, None, :]
        xa = self.to_ref(self.fA_elem[:, None], x)
        xb = self.to_ref(self.fB_elem[:, None], x + self.shiftB[:, None, :])
        return xa, xb

    def element_facet_points(self, t, f, s):
        """Points of facet parameter s on local facet f of element t (facet orientation).

        Used for the BDM moments: the parameter is the facet's global one (A's
        direction), expressed in element t's own coordinates.
        """
        F = self.elem_facet[t, f]
        x = self.P0[F][:, None, :] + s[None, :, None] * (self.P1 - self.P0)[F][:, None, :]
        isB = (self.fB_elem[F] == t) & (self.fB_loc[F] == f)
        x = x + np.where(isB[:, None, None], self.shiftB[F][:, None, :], 0.0)
        return self.to_ref(t[:, None], x), F
