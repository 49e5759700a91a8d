"""Reverse-mode gradient of the final kinetic energy through the oracle's TVD-RK3.

The Jacobian of L(u) (upwind side frozen: the derivative almost everywhere) is
assembled as a sparse matrix on the global BDM basis from element and facet blocks
obtained by complex-step differentiation of the oracle's own residual terms (exact to
round-off for these polynomial integrands).  The time stepping is the paper-literal
mass-matrix form (eq. (rk3)) with the mixed solve S (eq. (FE2)), which is symmetric, so
the reverse sweep applies S to the cotangents.  Pinned against central finite
differences of the forward oracle in tests/test_oracle_adjoint.py.
"""
import numpy as np
import scipy.sparse as sp

H_CS = 1e-30


def residual_jacobian(orc, U):
    """Sparse d L / d U on the global BDM basis at the state U."""
    space, res, m = orc.space, orc.res, orc.mesh
    T, nm, nu = m.T, space.nm, space.nu
    cU = orc.state_local(U)  # with the inflow lift, if any (Sec. 2.5)
    # element (volume) blocks Jv[t, out, in] in the local basis
    Jv = np.zeros((T, nu, nu))
    for j in range(nu):
        c, a = divmod(j, nm)
        cz = cU.astype(complex)
        cz[:, c, a] += 1j * H_CS
        out = np.zeros(cz.shape, dtype=complex)
        res.volume(cz, out)
        Jv[:, :, j] = out.imag.reshape(T, nu) / H_CS
    # facet blocks: derivatives of (RA, RB) w.r.t. side A's and side B's coefficients
    E = m.E
    cA, cB = cU[m.fA_elem], cU[m.fB_elem]
    JAA, JBA, JAB, JBB = (np.zeros((E, nu, nu)) for _ in range(4))
    for j in range(nu):
        c, a = divmod(j, nm)
        za = cA.astype(complex)
        za[:, c, a] += 1j * H_CS
        RA, RB = res.facet_terms(za, cB.astype(complex))
        JAA[:, :, j] = RA.imag.reshape(E, nu) / H_CS
        JBA[:, :, j] = RB.imag.reshape(E, nu) / H_CS
        zb = cB.astype(complex)
        zb[:, c, a] += 1j * H_CS
        RA, RB = res.facet_terms(cA.astype(complex), zb)
        JAB[:, :, j] = RA.imag.reshape(E, nu) / H_CS
        JBB[:, :, j] = RB.imag.reshape(E, nu) / H_CS
    # dofs_x sends the normal moments on walls (not in BDM_k with u.n = 0) to a trailing
    # slot that is cut off below
    Aloc, dofs = space.A, space.dofs_x
    rows, cols, vals = [], [], []

    def add(blocks, te_out, te_in):
        # global block = A_out^T J A_in
        G = np.einsum("eai,eab,ebj->eij", Aloc[te_out], blocks, Aloc[te_in])
        rows.append(np.repeat(dofs[te_out], nu, axis=1).ravel())
        cols.append(np.tile(dofs[te_in], (1, nu)).ravel())
        vals.append(G.ravel())

    tt = np.arange(T)
    add(Jv, tt, tt)
    add(JAA, m.fA_elem, m.fA_elem)
    add(JBA, m.fB_elem, m.fA_elem)
    add(JAB, m.fA_elem, m.fB_elem)
    add(JBB, m.fB_elem, m.fB_elem)
    n = space.ndof
    J = sp.csr_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))), shape=(n + 1, n + 1))
    return J[:n, :n]


def energy_and_gradient(orc, U0, dt, steps, checkpoint_every=10):
    """E = 1/2 ||u_N||^2 after `steps` TVD-RK3 steps and dE/dU0 (global BDM coefficients).

    Forward states are stored every `checkpoint_every` steps; each segment's step states
    are recomputed in the reverse sweep.
    """
    M = orc.M
    ckpt = {0: U0.copy()}
    U = U0.copy()
    for n in range(steps):
        U = orc.rk3_step(U, dt)
        if (n + 1) % checkpoint_every == 0:
            ckpt[n + 1] = U.copy()
    E = 0.5 * float(U @ (M @ U))
    Ubar = M @ U
    seg_starts = sorted(k for k in ckpt if k < steps)
    for s0 in reversed(seg_starts):
        s1 = min(s0 + checkpoint_every, steps)
        states = [ckpt[s0]]
        for n in range(s0, s1 - 1):
            states.append(orc.rk3_step(states[-1], dt))
        for n in range(s1 - 1, s0 - 1, -1):
            Ubar = step_vjp(orc, states[n - s0], Ubar, dt)
    return E, Ubar


def step_vjp(orc, Un, Ubar3, dt):
    """Cotangent of U^n from that of U^{n+1} for one oracle rk3_step (form of eq. (rk3))."""
    M = orc.M
    MU = M @ Un
    U1 = orc.mass_solve(MU + dt * orc.L(Un))
    U2 = orc.mass_solve(0.75 * MU + 0.25 * (M @ U1 + dt * orc.L(U1)))
    w3 = orc.mass_solve(Ubar3)
    Ubar = (M @ w3) / 3.0
    J2 = residual_jacobian(orc, U2)
    Ubar2 = 2.0 / 3.0 * (M @ w3 + dt * (J2.T @ w3))
    w2 = orc.mass_solve(Ubar2)
    Ubar = Ubar + 0.75 * (M @ w2)
    J1 = residual_jacobian(orc, U1)
    Ubar1 = 0.25 * (M @ w2 + dt * (J1.T @ w2))
    w1 = orc.mass_solve(Ubar1)
    J0 = residual_jacobian(orc, Un)
    return Ubar + M @ w1 + dt * (J0.T @ w1)
