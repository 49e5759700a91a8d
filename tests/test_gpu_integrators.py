"""GPU parity of the other time integrators of the paper against the oracle: the classical
four-stage RK4 (Sec. 4, Example 1b, Table 2) and forward Euler (eq. (FE); Example 5), on
triangles and tetrahedra; the mixed-precision RK4 against FP64; and the warm-start history
belonging to one integrator at a time."""
import numpy as np
import pytest
import torch

from inputs import RandomStreamField, abc_flow, taylor_green_2d, taylor_green_3d

pytestmark = pytest.mark.gpu

from gpu_util import make_pair, project_field, rel_l2, transfer  # noqa: E402


def _log(*a):
    print(*a, flush=True)


@pytest.mark.parametrize("dim,k,N,nu,steps,precond,method", [
    (2, 2, 8, 1e-2, 4, "jacobi", "rk4"),
    (2, 3, 6, 1e-3, 3, "amg", "rk4"),
    (3, 1, 3, 0.0, 3, "jacobi", "rk4"),
    (3, 2, 2, 1.0 / 1600, 2, "amg", "rk4"),
    (2, 2, 8, 1e-2, 6, "amg", "fe"),
    (3, 2, 3, 1.0 / 1600, 4, "jacobi", "fe"),
])
def test_integrator_parity(dim, k, N, nu, steps, precond, method):
    _log(method, dim, k, N, nu, precond)
    orc, s, _, _ = make_pair(N, k, nu=nu, dim=dim, cg_rtol=1e-13, precond=precond, extrapolate="adaptive")
    f = {2: RandomStreamField(seed=4, kmax=3), 3: abc_flow if k == 1 else taylor_green_3d}[dim]
    U0 = orc.project(f)
    U = transfer(orc, U0, s)
    dt = 0.1 / N / k ** 2
    Uo = U0
    for _ in range(steps):
        info = s.rk4_step(U, dt) if method == "rk4" else s.fe_step(U, dt)
        assert info.status == 0
        Uo = orc.rk4_step(Uo, dt) if method == "rk4" else orc.fe_step(Uo, dt)
    err = rel_l2(orc, s, U, Uo)
    d = s.diagnostics(U)
    _log("  rel L2", err, d)
    assert err < 1e-10
    assert d["max_div"] < 1e-11 and d["max_normal_jump"] < 1e-11


def test_mixed_rk4_against_fp64():
    """The mixed-precision form of RK4 (FP32 residual and inner PCG, FP64 refinement to
    1e-10) stays within 1e-6 of the FP64 path (64x64 BDM_2 Taylor-Green, nu = 1e-3)."""
    out = {}
    for prec in ("fp64", "mixed"):
        _, s, xyz, _ = make_pair(64, 2, nu=1e-3, oracle=False, cg_rtol=1e-10, precond="amg", precision=prec,
                                 ir_rtol=1e-10)
        U, vmax = project_field(s, xyz, taylor_green_2d)
        for _ in range(5):
            assert s.rk4_step(U, 0.1 / 64 / (4 * vmax)).status == 0
        out[prec] = U
        del s
    err = ((out["mixed"] - out["fp64"]).norm() / out["fp64"].norm()).item()
    _log("mixed RK4 vs FP64", err)
    assert err < 1e-6


def test_switching_integrators_starts_a_fresh_history():
    """RK4 after TVD-RK3 on one context gives the same bits as RK4 on a fresh context from
    the same state (the history is the integrator's), and back again."""
    _, a, xyz, _ = make_pair(16, 2, nu=1e-3, oracle=False, cg_rtol=1e-12, precond="amg", extrapolate="adaptive")
    _, b, _, _ = make_pair(16, 2, nu=1e-3, oracle=False, cg_rtol=1e-12, precond="amg", extrapolate="adaptive")
    U, vmax = project_field(a, xyz, taylor_green_2d)
    dt = 0.1 / 16 / (4 * vmax)
    for _ in range(3):
        a.rk3_step(U, dt)
    V = U.clone()
    ia = [list(a.rk4_step(U, dt).iterations) for _ in range(2)]
    ib = [list(b.rk4_step(V, dt).iterations) for _ in range(2)]
    torch.cuda.synchronize()
    _log("rk4 iterations after rk3", ia, "fresh", ib)
    assert ia == ib and torch.equal(U, V)
    a.fe_step(U, dt)
    b.reset_history()
    b.fe_step(V, dt)
    assert torch.equal(U, V)
    assert np.isfinite(a.diagnostics(U)["energy"])
