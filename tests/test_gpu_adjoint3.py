"""GPU parity of the adjoint form on tetrahedra: the residual's vector-Jacobian product
against the oracle's Jacobian (periodic cube, channel with walls, inflow/outflow cube), and
the TVD-RK3 step's VJP against central differences of the library's own steps."""
import numpy as np
import pytest
import torch

from inputs import RandomVectorPotentialField

pytestmark = pytest.mark.gpu

from gpu_util import make_pair, to_dev, transfer  # noqa: E402


def _log(*a):
    print(*a, flush=True)


def _lift3(x, y, z):
    return 0.8 + 0 * x, 0.15 + 0 * y, -0.1 + 0 * z


def _increments(orc, s, n, seed):
    """Seeded increments in the divergence-free space (closed at an inflow), on the
    oracle's basis and as library coefficients (no lift), unit in L2."""
    rng = np.random.default_rng(seed)
    pts, _ = s.proj_rule()
    out = []
    for _ in range(n):
        d = orc.mass_solve(rng.standard_normal(orc.space.ndof))
        d = d / np.sqrt(d @ (orc.M @ d))
        out.append((d, s.load_vector(to_dev(s, orc.space.eval_ref(d, pts)))))
    return out


def _pair(kind, N, k, nu, **kw):
    extra = dict(walls=True) if kind == "walls" else dict(inout=True, inflow=_lift3) if kind == "inout" else {}
    return make_pair(N, k, nu=nu, dim=3, order="random", seed=N, **extra, **kw)


@pytest.mark.parametrize("kind,k,N", [("periodic", 1, 3), ("periodic", 2, 2), ("walls", 1, 2), ("walls", 2, 2),
                                      ("inout", 1, 2), ("inout", 2, 2)])
def test_residual_vjp_parity_3d(kind, k, N):
    """y . (J_L(u) d) through dfdg_dg_residual_vjp equals the oracle's Jacobian product."""
    from oracle.adjoint import residual_jacobian
    _log("vjp 3d", kind, k, N)
    orc, s, _, _ = _pair(kind, N, k, nu=0.01)
    U0 = orc.project(RandomVectorPotentialField(seed=1, kmax=2, norm=0.5))
    U = transfer(orc, U0, s)
    J = residual_jacobian(orc, U0)
    for (y_g, y), (d_g, d) in zip(_increments(orc, s, 2, 5), _increments(orc, s, 2, 6)):
        gpu = torch.dot(s.residual_vjp(U, y), d).item()
        ref = float(y_g @ (J @ d_g))
        _log("  ", gpu, ref)
        assert abs(gpu - ref) < 1e-10 * (abs(ref) + 1e-3)


@pytest.mark.parametrize("kind", ["periodic", "inout"])
def test_rk3_step_vjp_3d_matches_finite_differences(kind):
    """One TVD-RK3 step's VJP on tetrahedra against central differences of the step along
    divergence-free increments."""
    _log("step vjp 3d", kind)
    orc, s, _, _ = _pair(kind, 3, 1, nu=1e-3, cg_rtol=1e-14)
    U0 = transfer(orc, orc.project(RandomVectorPotentialField(seed=2, kmax=2, norm=0.5)), s)
    dt = 0.1 / 3 / 4
    (_, w), *dirs = _increments(orc, s, 3, 9)
    for _, d in dirs:
        h = 1e-6

        def step(u):
            v = u.clone()
            s.reset_history()
            assert s.rk3_step(v, dt).status == 0
            return v

        fd = torch.dot(w, step(U0 + h * d) - step(U0 - h * d)).item() / (2 * h)
        Ub = w.clone()
        assert s.rk3_step_vjp(U0, Ub, dt).status == 0
        adj = torch.dot(Ub, d).item()
        _log("  ", adj, fd)
        assert abs(adj - fd) < 1e-6 * abs(fd) + 1e-10
