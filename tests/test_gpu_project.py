"""Start values of the forward stage solves projected onto earlier solutions
(extrapolate="project"): the element of the span of up to 24 earlier solutions closest in
the S-norm to the new solution, from an S-orthogonal basis grown by two Gram-Schmidt passes
and rebuilt from the latest 8 solutions when full.  Start values change the iterations, not
the converged solution: trajectories equal the oracle's and the extrapolating modes' to the
solver tolerance, on triangles and tetrahedra, periodic, with walls and with inflow/outflow,
for TVD-RK3, RK4 and forward Euler."""
import numpy as np
import pytest
import torch

from inputs import RandomStreamField, RandomVectorPotentialField, double_shear_layer

pytestmark = pytest.mark.gpu

from gpu_util import make_pair, project_field, rel_l2, transfer  # noqa: E402


def _log(*a):
    print(*a, flush=True)


@pytest.mark.parametrize("dim,k,N,kind,precond", [
    (2, 2, 8, "periodic", "amg"), (2, 1, 10, "periodic", "jacobi"), (2, 3, 5, "walls", "amg"),
    (2, 2, 6, "inout", "amg"), (3, 1, 3, "periodic", "amg"), (3, 2, 2, "walls", "jacobi"),
    (3, 2, 2, "inout", "amg_mf"),
])
def test_project_rk3_trajectory_parity(dim, k, N, kind, precond):
    """Twelve steps (36 solves: the basis fills and is rebuilt) against the oracle (on
    tetrahedra also with the matrix-free product of the facet system)."""
    _log("project rk3", dim, k, N, kind, precond)
    mf = precond.endswith("_mf")
    precond = precond.replace("_mf", "")
    lift = {2: lambda x, y: (0.8 + 0 * x, 0.15 + 0 * y),
            3: lambda x, y, z: (0.8 + 0 * x, 0.15 + 0 * y, -0.1 + 0 * z)}[dim]
    extra = dict(walls=True) if kind == "walls" else dict(inout=True, inflow=lift) if kind == "inout" else {}
    orc, s, _, _ = make_pair(N, k, nu=1e-3, dim=dim, order="random", seed=N, cg_rtol=1e-13, precond=precond,
                             extrapolate="project", matrix_free=mf, **extra)
    f = RandomStreamField(seed=3, kmax=2, norm=0.5) if dim == 2 else RandomVectorPotentialField(seed=3, kmax=2, norm=0.5)
    U0 = orc.project(f)
    U = transfer(orc, U0, s)
    dt = 0.1 / N / k ** 2
    Uo = U0
    its = []
    for _ in range(12):
        info = s.rk3_step(U, dt)
        assert info.status == 0 and info.max_rel_residual <= 1e-13
        its.append(list(info.iterations))
        Uo = orc.rk3_step(Uo, dt)
    err = rel_l2(orc, s, U, Uo)
    _log("  its", its, "rel L2", err)
    assert err < 1e-10


@pytest.mark.parametrize("method", ["rk4", "fe"])
def test_project_other_integrators(method):
    orc, s, _, _ = make_pair(8, 2, nu=1e-2, cg_rtol=1e-13, precond="amg", extrapolate="project")
    U0 = orc.project(RandomStreamField(seed=4, kmax=3))
    U = transfer(orc, U0, s)
    dt = 0.1 / 8 / 4
    Uo = U0
    for _ in range(8):
        info = s.rk4_step(U, dt) if method == "rk4" else s.fe_step(U, dt)
        assert info.status == 0
        Uo = orc.rk4_step(Uo, dt) if method == "rk4" else orc.fe_step(Uo, dt)
    err = rel_l2(orc, s, U, Uo)
    _log("project", method, err)
    assert err < 1e-10


def test_project_saves_iterations_and_keeps_the_trajectory_at_64():
    """64x64 BDM_2 double shear layer, 40 steps at rtol 1e-12: the projected start values
    need fewer PCG iterations than the adaptive extrapolation, and the two trajectories agree
    to the solver tolerance; reset_history empties the basis (a step after it repeats the
    step of a fresh context bit for bit)."""
    out = {}
    for ex in ("adaptive", "project"):
        _, s, xyz, _ = make_pair(64, 2, oracle=False, cg_rtol=1e-12, precond="amg", extrapolate=ex)
        U, vmax = project_field(s, xyz, double_shear_layer)
        dt = 0.1 / 64 / (4 * vmax)
        its = []
        for _ in range(40):
            info = s.rk3_step(U, dt)
            assert info.status == 0
            its.append(np.mean(info.iterations))
        out[ex] = (U, float(np.mean(its[10:])), s, dt)
    dif = ((out["project"][0] - out["adaptive"][0]).norm() / out["adaptive"][0].norm()).item()
    _log("iterations per stage: adaptive", out["adaptive"][1], "project", out["project"][1], "difference", dif)
    assert dif < 1e-9
    assert out["project"][1] < out["adaptive"][1] - 1.0
    # reset: the next step equals a fresh context's step from the same state
    U, _, s, dt = out["project"]
    s.reset_history()
    A = U.clone()
    ia = s.rk3_step(A, dt)
    _, f, _, _ = make_pair(64, 2, oracle=False, cg_rtol=1e-12, precond="amg", extrapolate="project")
    B = U.clone()
    ib = f.rk3_step(B, dt)
    assert list(ia.iterations) == list(ib.iterations) and torch.equal(A, B)
