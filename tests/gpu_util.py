"""Helpers shared by the GPU tests: oracle/library pairs and exact data transfer
(triangle and tetrahedral meshes; the dimension follows the library context)."""
import numpy as np
import torch

from inputs import (channel_kuhn_cube, channel_split_square, distort_split_square, inout_kuhn_cube,
                    inout_split_square, outflow_at_right,
                    periodic_kuhn_cube, periodic_split_square)
from oracle import Oracle
from oracle.quadrature import poly_basis_nd, simplex_rule


def make_pair(N, k, nu=0.0, order="morton", seed=0, oracle=True, dim=2, walls=False, distort=0.0, inout=False,
              inflow=None, **kw):
    """Oracle and library solver on the same mesh: the periodic unit square (or cube), or
    with walls=True the channel periodic in x with walls at y = 0 and 1, or with inout=True
    the square periodic in y with an inflow boundary at x = 0 (the oracle's lift: the
    polynomial field ``inflow``) and an outflow boundary at x = 1; distort > 0 moves the
    triangle mesh's vertices by up to that fraction of h (seeded)."""
    from paper_1808_04669_amd import Solver
    gen = ((inout_split_square if dim == 2 else inout_kuhn_cube) if inout
           else (channel_split_square if dim == 2 else channel_kuhn_cube) if walls
           else (periodic_split_square if dim == 2 else periodic_kuhn_cube))
    xyz, per = gen(N, order, seed)
    if distort > 0:
        xyz = distort_split_square(xyz, per, N, distort, seed=seed + 101)
    out = outflow_at_right if inout else None
    orc = Oracle(xyz, per, k, nu=nu, outflow=out, inflow=inflow) if oracle else None
    s = Solver(xyz, per, k, nu=nu, device="cuda:0", outflow=out, **kw)
    return orc, s, xyz, per


def to_dev(s, vals):
    """[T, d, nq] numpy values -> flat device array in the library layout [d][nq][T]."""
    return torch.from_numpy(np.ascontiguousarray(np.transpose(vals, (1, 2, 0)))).to(s.device).reshape(-1)


def transfer(orc, U_orc, s):
    """Library coefficients of the oracle's piecewise polynomial (exact: orthonormal basis,
    projection rule of degree >= 2k)."""
    pts, _ = s.proj_rule()
    return s.load_vector(to_dev(s, orc.eval_ref(U_orc, pts)))


def values_to_lib(s, field_vals_fn):
    pts, _ = s.proj_rule()
    return s.load_vector(to_dev(s, field_vals_fn(pts)))


def gpu_vals(s, U, ref_pts):
    return s.eval(U, ref_pts).cpu().numpy().transpose(2, 0, 1)  # [T, d, P]


def rel_l2(orc, s, U_gpu, U_orc):
    rule = simplex_rule(orc.d, 2 * orc.k + 2)
    g = gpu_vals(s, U_gpu, rule[0])
    o = orc.eval_ref(U_orc, rule[0])
    return orc.l2_diff(g, o, rule) / orc.l2_diff(o, 0 * o, rule)


def broken_residual_on_oracle_basis(orc, s, L_gpu):
    """R[T, d, nm] = L(u)(m_a e_c) from the library's L(u)(psi_i e_c), using
    m_a e_c = sum_i (m_a, psi_i) psi_i e_c (the library basis is orthonormal)."""
    pts, _ = s.proj_rule()
    vals, _ = poly_basis_nd(orc.k, pts)  # [nq, nm]
    T, P, d = s.T, s.P, s.dim
    Lv = L_gpu.view(d, P, T)
    out = np.empty((T, d, orc.space.nm))
    for a in range(orc.space.nm):
        f = np.zeros((T, d, len(pts)))
        for c in range(d):
            f[:, c, :] = vals[:, a][None, :]
        G = s.load_vector(to_dev(s, f)).view(d, P, T)
        out[:, :, a] = (G * Lv).sum(dim=1).T.cpu().numpy()
    return out


def phys_points(xyz, pts):
    """Physical points [T, nq, d] of reference points pts[nq, d] in every element."""
    return xyz[:, None, 0, :] + np.einsum("tir,qr->tqi", np.transpose(xyz[:, 1:] - xyz[:, :1], (0, 2, 1)), pts)


def project_field(s, xyz, field):
    """L2 projection (on the GPU, dfdg_project) of a closed-form field u(x, y[, z]) sampled
    at the library's projection points; also returns max |u| at those points."""
    pts, _ = s.proj_rule()
    x = phys_points(xyz, pts)
    u = field(*[x[..., i] for i in range(s.dim)])  # d arrays [T, nq]
    vmax = float(np.sqrt(sum(c ** 2 for c in u)).max())
    fq = torch.from_numpy(np.ascontiguousarray(np.stack([c.T for c in u]))).to(s.device).reshape(-1)
    U, info = s.project(fq)
    assert info.status == 0
    return U, vmax
