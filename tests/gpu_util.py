"""Helpers shared by the GPU tests: oracle/library pairs and exact data transfer."""
import numpy as np
import torch

from inputs import periodic_split_square
from oracle import Oracle
from oracle.quadrature import poly_basis, triangle_rule


def make_pair(N, k, nu=0.0, order="morton", seed=0, oracle=True, **kw):
    from paper_1808_04669_amd import Solver
    xyz, per = periodic_split_square(N, order, seed)
    orc = Oracle(xyz, per, k, nu=nu) if oracle else None
    s = Solver(xyz, per, k, nu=nu, device="cuda:0", **kw)
    return orc, s, xyz, per


def to_dev(s, vals):
    """[T, 2, nq] numpy values -> flat device array in the library layout [2][nq][T]."""
    return torch.from_numpy(np.ascontiguousarray(np.transpose(vals, (1, 2, 0)))).to(s.device).reshape(-1)


def transfer(orc, U_orc, s):
    """Library coefficients of the oracle's piecewise polynomial (exact: orthonormal basis,
    projection rule of degree 2k+4)."""
    pts, _ = s.proj_rule()
    return s.load_vector(to_dev(s, orc.eval_ref(U_orc, pts)))


def values_to_lib(s, field_vals_fn):
    pts, _ = s.proj_rule()
    return s.load_vector(to_dev(s, field_vals_fn(pts)))


def gpu_vals(s, U, ref_pts):
    return s.eval(U, ref_pts).cpu().numpy().transpose(2, 0, 1)  # [T, 2, P]


def rel_l2(orc, s, U_gpu, U_orc):
    rule = triangle_rule(2 * orc.k + 2)
    g = gpu_vals(s, U_gpu, rule[0])
    o = orc.eval_ref(U_orc, rule[0])
    return orc.l2_diff(g, o, rule) / orc.l2_diff(o, 0 * o, rule)


def broken_residual_on_oracle_basis(orc, s, L_gpu):
    """R[T, 2, nm] = L(u)(m_a e_c) from the library's L(u)(psi_i e_c), using
    m_a e_c = sum_i (m_a, psi_i) psi_i e_c (the library basis is orthonormal)."""
    pts, _ = s.proj_rule()
    vals, _ = poly_basis(orc.k, pts[:, 0], pts[:, 1])  # [nq, nm]
    T, P = s.T, s.P
    Lv = L_gpu.view(2, P, T)
    out = np.empty((T, 2, orc.space.nm))
    for a in range(orc.space.nm):
        f = np.zeros((T, 2, len(pts)))
        f[:, 0, :] = vals[:, a][None, :]
        f[:, 1, :] = vals[:, a][None, :]
        G = s.load_vector(to_dev(s, f)).view(2, P, T)
        out[:, :, a] = (G * Lv).sum(dim=1).T.cpu().numpy()
    return out


def project_field(s, xyz, field):
    """L2 projection (on the GPU, dfdg_project) of a closed-form field u(x, y) -> (u1, u2)
    sampled at the library's projection points; also returns max |u| at those points."""
    pts, _ = s.proj_rule()
    x = xyz[:, None, 0, :] + (pts[None, :, 0, None] * (xyz[:, None, 1, :] - xyz[:, None, 0, :])
                              + pts[None, :, 1, None] * (xyz[:, None, 2, :] - xyz[:, None, 0, :]))
    u1, u2 = field(x[..., 0], x[..., 1])  # [T, nq]
    vmax = float(np.sqrt(u1 ** 2 + u2 ** 2).max())
    fq = torch.from_numpy(np.ascontiguousarray(np.stack([u1.T, u2.T]))).to(s.device).reshape(-1)
    U, info = s.project(fq)
    assert info.status == 0
    return U, vmax
