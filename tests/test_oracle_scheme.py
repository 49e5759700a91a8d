"""Pins of the full oracle scheme: convergence orders, temporal order, energy."""
import json
import os

import numpy as np
import pytest

from inputs import periodic_split_square, taylor_green_2d, double_shear_layer
from oracle import Oracle

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _tg_errors(k, Ns, nu, tend=0.1, cfl=0.05):
    errs = []
    for N in Ns:
        xyz, per = periodic_split_square(N)
        o = Oracle(xyz, per, k, nu=nu)
        U = o.project(taylor_green_2d)
        n = int(np.ceil(tend / (cfl / N / k ** 2)))
        U = o.run(U, tend / n, n)
        errs.append(o.l2_error_to(U, lambda x, y: taylor_green_2d(x, y, tend, nu)))
    return np.array(errs)


@pytest.mark.parametrize("k,Ns", [(1, (8, 16, 32)), (2, (4, 8, 16))])
@pytest.mark.parametrize("nu", [0.0, 0.01])
def test_taylor_green_spatial_order(k, Ns, nu):
    """Sec. 4 Example 1a: optimal (k+1)-th order L2 convergence (Table 1 pattern)."""
    with open(os.path.join(GOLDEN, "table1_eoc.json")) as f:
        table = json.load(f)
    paper = table["euler" if nu == 0 else "navier_stokes_re100"][str(k)]
    errs = _tg_errors(k, Ns, nu)
    rates = np.log2(errs[:-1] / errs[1:])
    # finest-pair rate within 0.25 of the paper's finest-mesh EOC
    assert abs(rates[-1] - paper[-1]) < 0.25, (errs, rates)


def test_rk3_temporal_order():
    """Sec. 4 Example 1b / Table 2: TVD-RK3 converges at third order in time."""
    with open(os.path.join(GOLDEN, "table2_eoc.json")) as f:
        paper = json.load(f)["tvd_rk3_eoc"]
    xyz, per = periodic_split_square(4)
    o = Oracle(xyz, per, 2, nu=0.02)
    U0 = o.project(taylor_green_2d)
    # add a non-stationary component so the Euler part of the flow evolves
    U0 = U0 + 0.5 * o.project(lambda x, y: (np.sin(2 * np.pi * y), 0 * x))
    tend = 0.2
    ref = o.run(U0, tend / 1024, 1024)
    errs = []
    for n in (16, 32, 64):
        d = o.run(U0, tend / n, n) - ref
        errs.append(np.sqrt(d @ (o.M @ d)))
    rates = np.log2(np.array(errs[:-1]) / np.array(errs[1:]))
    assert abs(rates[-1] - paper[-1]) < 0.2, (errs, rates)


def _temporal_errors(step_name, ns):
    xyz, per = periodic_split_square(4)
    o = Oracle(xyz, per, 2, nu=0.02)
    U0 = o.project(taylor_green_2d)
    U0 = U0 + 0.5 * o.project(lambda x, y: (np.sin(2 * np.pi * y), 0 * x))
    tend = 0.2
    step = getattr(o, step_name)
    ref = o.run(U0, tend / 512, 512, step=o.rk4_step)
    errs = []
    for n in ns:
        d = o.run(U0, tend / n, n, step=step) - ref
        errs.append(np.sqrt(d @ (o.M @ d)))
    return np.array(errs)


def test_rk4_temporal_order():
    """Sec. 4 Example 1b / Table 2: the classical RK4 converges at fourth order in time."""
    with open(os.path.join(GOLDEN, "table2_eoc.json")) as f:
        paper = json.load(f)["rk4_eoc"]
    errs = _temporal_errors("rk4_step", (8, 16, 32))
    rates = np.log2(errs[:-1] / errs[1:])
    assert abs(rates[-1] - paper[-1]) < 0.2, (errs, rates)


def test_forward_euler_first_order_and_rk_consistency():
    """Forward Euler (eq. (FE), Example 5) converges at first order; one forward-Euler step
    equals the first TVD-RK3 stage, and all three integrators agree to their orders."""
    errs = _temporal_errors("fe_step", (64, 128, 256))
    rates = np.log2(errs[:-1] / errs[1:])
    assert abs(rates[-1] - 1.0) < 0.1, (errs, rates)
    xyz, per = periodic_split_square(3)
    o = Oracle(xyz, per, 2, nu=0.01)
    U = o.project(taylor_green_2d)
    dt = 1e-3
    stage1 = o.mass_solve(o.M @ U + dt * o.L(U))
    assert np.abs(o.fe_step(U, dt) - stage1).max() == 0.0
    a, b = o.rk3_step(U, dt), o.rk4_step(U, dt)
    assert np.abs(a - b).max() < 1e-7 * np.abs(a).max()


def test_inviscid_energy_non_increasing():
    """Sec. 2.2 energy stability; Sec. 4 Example 2: energy decays monotonically."""
    xyz, per = periodic_split_square(8)
    o = Oracle(xyz, per, 2, nu=0.0)
    U = o.project(lambda x, y: double_shear_layer(x, y, sharpness=30.0))
    dt = 0.1 / 8 / 4
    E = [o.energy(U)]
    for _ in range(15):
        U = o.rk3_step(U, dt)
        E.append(o.energy(U))
    dE = np.diff(E)
    assert np.all(dE <= 1e-14 * E[0]), dE
    assert E[-1] < E[0]
    assert o.divergence_max(U) < 1e-10


def test_viscous_taylor_green_energy_decay():
    """Navier-Stokes TG: kinetic energy decays like exp(-16 pi^2 nu t)."""
    nu = 0.01
    xyz, per = periodic_split_square(8)
    o = Oracle(xyz, per, 2, nu=nu)
    U = o.project(taylor_green_2d)
    E0 = o.energy(U)
    tend, n = 0.1, 20
    U = o.run(U, tend / n, n)
    ratio = o.energy(U) / E0
    assert abs(ratio - np.exp(-16 * np.pi ** 2 * nu * tend)) < 2e-3
