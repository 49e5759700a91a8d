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
