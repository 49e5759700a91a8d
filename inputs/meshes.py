"""Periodic simplicial meshes of the unit square, as plain vertex-coordinate data.

The mesh is handed to both implementations as an array ``xyz[T, 3, 2]`` holding,
for each triangle, the coordinates of its three vertices (counter-clockwise),
"unwrapped" so that each triangle is a genuine triangle in the plane, plus the
period vector.  Facet matching across the periodic boundary is each consumer's
own business.

Every square ``[i/N, (i+1)/N] x [j/N, (j+1)/N]`` is split along the diagonal from
``(i, j)`` to ``(i+1, j+1)`` into a lower and an upper triangle, so the mesh is
translation invariant and conforming across the periodic boundary.
"""
import numpy as np


def _morton_key(i, j, bits):
    key = np.zeros_like(i, dtype=np.int64)
    for b in range(bits):
        key |= ((i >> b) & 1).astype(np.int64) << (2 * b)
        key |= ((j >> b) & 1).astype(np.int64) << (2 * b + 1)
    return key


def element_order(N, order="morton", seed=0):
    """Permutation of the N*N squares: 'lex' (row-major), 'morton' or 'random'."""
    i, j = np.meshgrid(np.arange(N), np.arange(N), indexing="xy")
    i = i.ravel()
    j = j.ravel()
    if order == "lex":
        perm = np.arange(N * N)
    elif order == "morton":
        bits = max(1, int(np.ceil(np.log2(max(N, 2)))))
        perm = np.argsort(_morton_key(i, j, bits), kind="stable")
    elif order == "random":
        perm = np.random.default_rng(seed).permutation(N * N)
    else:
        raise ValueError(f"unknown order {order!r}")
    return i[perm], j[perm]


def periodic_split_square(N, order="morton", seed=0):
    """Return (xyz[T,3,2] float64, period[2]) for the N x N split periodic unit square.

    T = 2 N^2 triangles; lower triangle (i,j),(i+1,j),(i+1,j+1) and upper
    triangle (i,j),(i+1,j+1),(i,j+1) of each square, both counter-clockwise.
    The lower/upper pair of one square are consecutive.
    """
    if N < 1:
        raise ValueError("N must be >= 1")
    i, j = element_order(N, order, seed)
    h = 1.0 / N
    x0 = i * h
    y0 = j * h
    x1 = (i + 1) * h
    y1 = (j + 1) * h
    T = 2 * N * N
    xyz = np.empty((T, 3, 2))
    lo = xyz[0::2]
    up = xyz[1::2]
    lo[:, 0, 0], lo[:, 0, 1] = x0, y0
    lo[:, 1, 0], lo[:, 1, 1] = x1, y0
    lo[:, 2, 0], lo[:, 2, 1] = x1, y1
    up[:, 0, 0], up[:, 0, 1] = x0, y0
    up[:, 1, 0], up[:, 1, 1] = x1, y1
    up[:, 2, 0], up[:, 2, 1] = x0, y1
    return xyz, np.array([1.0, 1.0])


def channel_split_square(N, order="morton", seed=0):
    """The N x N split unit square as a channel: periodic in x, walls at y = 0 and y = 1
    (period[1] = 0).  Same triangles as periodic_split_square."""
    xyz, _ = periodic_split_square(N, order, seed)
    return xyz, np.array([1.0, 0.0])


def _morton_key3(i, j, k, bits):
    key = np.zeros_like(i, dtype=np.int64)
    for b in range(bits):
        key |= ((i >> b) & 1).astype(np.int64) << (3 * b)
        key |= ((j >> b) & 1).astype(np.int64) << (3 * b + 1)
        key |= ((k >> b) & 1).astype(np.int64) << (3 * b + 2)
    return key


def periodic_kuhn_cube(N, order="morton", seed=0):
    """Return (xyz[T,4,3] float64, period[3]) for the N x N x N periodic unit cube, every
    cube split into the 6 Kuhn tetrahedra that share its main diagonal.

    The cube with lowest corner c = (i, j, k)/N gives, for every permutation s of the axes,
    the tetrahedron c, c + h e_s0, c + h (e_s0 + e_s1), c + h (1, 1, 1) (h = 1/N); for odd
    permutations the middle two vertices are swapped so that every element is positively
    oriented (det J = h^3).  The split is translation invariant, hence conforming across the
    periodic boundary.  T = 6 N^3; the six tetrahedra of one cube are consecutive, and the
    cubes are ordered 'lex', 'morton' or 'random'.
    """
    if N < 1:
        raise ValueError("N must be >= 1")
    i, j, k = np.meshgrid(np.arange(N), np.arange(N), np.arange(N), indexing="ij")
    i, j, k = i.ravel(), j.ravel(), k.ravel()
    if order == "lex":
        perm = np.lexsort((i, j, k))
    elif order == "morton":
        bits = max(1, int(np.ceil(np.log2(max(N, 2)))))
        perm = np.argsort(_morton_key3(i, j, k, bits), kind="stable")
    elif order == "random":
        perm = np.random.default_rng(seed).permutation(N ** 3)
    else:
        raise ValueError(f"unknown order {order!r}")
    i, j, k = i[perm], j[perm], k[perm]
    h = 1.0 / N
    corner = np.stack([i, j, k], axis=1) * h  # [C, 3]
    perms = [(0, 1, 2), (0, 2, 1), (1, 0, 2), (1, 2, 0), (2, 0, 1), (2, 1, 0)]
    odd = [False, True, True, False, False, True]
    eye = np.eye(3)
    xyz = np.empty((6 * N ** 3, 4, 3))
    for p, (s, o) in enumerate(zip(perms, odd)):
        v1 = eye[s[0]]
        v2 = eye[s[0]] + eye[s[1]]
        verts = [np.zeros(3), v1, v2, np.ones(3)]
        if o:
            verts[1], verts[2] = verts[2], verts[1]
        for a in range(4):
            xyz[p::6, a, :] = corner + h * verts[a]
    return xyz, np.array([1.0, 1.0, 1.0])


def distort_split_square(xyz, period, N, amplitude=0.15, seed=0):
    """Move every vertex of an N x N split-square mesh (periodic or channel) by a seeded uniform
    displacement in [-amplitude, amplitude] * h per coordinate, the same for every triangle
    that shares the vertex (periodic images included), so the mesh stays conforming and its
    triangles become all different.  Vertices on a wall (a direction with period 0) keep
    that coordinate.  amplitude <= 0.2 keeps every triangle counter-clockwise."""
    xyz = np.asarray(xyz, dtype=float)
    lat = np.rint(xyz * N).astype(np.int64)  # lattice indices of the vertices
    rng = np.random.default_rng(seed)
    disp = rng.uniform(-amplitude, amplitude, size=(N + 1, N + 1, 2)) / N
    out = xyz.copy()
    for d in range(2):
        idx = [lat[..., 0], lat[..., 1]]
        for e in range(2):
            if period[e] > 0:
                idx[e] = np.mod(idx[e], N)  # periodic images share the displacement
        move = disp[idx[0], idx[1], d]
        if period[d] == 0:
            wall = (lat[..., d] == 0) | (lat[..., d] == N)
            move = np.where(wall, 0.0, move)
        out[..., d] += move
    return out


def inout_split_square(N, order="morton", seed=0):
    """The N x N split unit square with an inflow boundary at x = 0 and an outflow
    boundary at x = 1, periodic in y (period[0] = 0).  Same triangles as
    periodic_split_square; ``outflow_at_right`` marks the outflow facets."""
    xyz, _ = periodic_split_square(N, order, seed)
    return xyz, np.array([0.0, 1.0])


def outflow_at_right(mid):
    """Boundary-facet barycentres [n, d] -> True on the outflow boundary x = 1."""
    return np.asarray(mid)[:, 0] > 0.5


def channel_kuhn_cube(N, order="morton", seed=0):
    """The N^3 Kuhn-split unit cube as a channel: periodic in x and y, walls at z = 0 and
    z = 1 (period[2] = 0).  Same tetrahedra as periodic_kuhn_cube."""
    xyz, _ = periodic_kuhn_cube(N, order, seed)
    return xyz, np.array([1.0, 1.0, 0.0])


def inout_kuhn_cube(N, order="morton", seed=0):
    """The N^3 Kuhn-split unit cube with an inflow boundary at x = 0 and an outflow
    boundary at x = 1, periodic in y and z (period[0] = 0); ``outflow_at_right`` marks the
    outflow faces."""
    xyz, _ = periodic_kuhn_cube(N, order, seed)
    return xyz, np.array([0.0, 1.0, 1.0])
