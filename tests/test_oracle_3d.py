"""Pins of the oracle on periodic tetrahedral meshes (the method is posed for d = 2, 3,
Sec. 2; the three-dimensional characterisation of the divergence-free space, Sec. 2.4).

Each pin is independent of the oracle's own arithmetic: closed-form integrals on the
reference tetrahedron and triangle, Euler's formula on the 3-torus, the de Rham count of the
divergence-free BDM_k functions from the Lagrange and Nedelec (second kind) dimensions, a
brute-force SVD null-space projection, the dense hybrid-mixed system (Theorem 2), the
convective energy identity, and the convergence order on the ABC flow, an exact solution.
"""
from itertools import permutations
from math import factorial

import numpy as np
import pytest
import scipy.linalg as sla

from inputs import (RandomVectorPotentialField, abc_flow, eval_broken_poly_3d, periodic_kuhn_cube,
                    random_broken_poly_3d, taylor_green_3d)
from oracle import Oracle
from oracle.mesh import OracleMesh
from oracle.quadrature import (facet_rule, poly_basis3, poly_basis_nd, symmetric_triangle_rule, tet_rule,
                               triangle_rule)
from oracle.scheme import hybrid_solve_dense


def _oracle(N, k, nu=0.0, order="morton", seed=1):
    xyz, per = periodic_kuhn_cube(N, order, seed)
    return Oracle(xyz, per, k, nu=nu)


@pytest.mark.parametrize("deg", range(0, 9))
def test_tet_rule_exact(deg):
    pts, w = tet_rule(deg)
    for p in range(deg + 1):
        for q in range(deg + 1 - p):
            r = deg - p - q
            exact = factorial(p) * factorial(q) * factorial(r) / factorial(deg + 3)
            got = np.sum(w * pts[:, 0] ** p * pts[:, 1] ** q * pts[:, 2] ** r)
            assert abs(got - exact) < 1e-14 * exact


@pytest.mark.parametrize("deg", [4, 6])
def test_symmetric_facet_rule_exact_and_permutation_invariant(deg):
    """The face rule of the 3D residual: exact for its degree, positive weights, and the
    same point set (with the same weights) in every parametrisation of the face."""
    pts, w = symmetric_triangle_rule(deg)
    assert np.all(w > 0) and abs(w.sum() - 0.5) < 1e-15
    for p in range(deg + 1):
        for q in range(deg + 1 - p):
            exact = factorial(p) * factorial(q) / factorial(p + q + 2)
            assert abs(np.sum(w * pts[:, 0] ** p * pts[:, 1] ** q) - exact) < 1e-14 * exact
    bary = np.stack([pts[:, 0], pts[:, 1], 1 - pts[:, 0] - pts[:, 1]], axis=1)
    key = {tuple(np.round(b, 12)): wi for b, wi in zip(bary, w)}
    for perm in permutations(range(3)):
        for b, wi in zip(bary[:, perm], w):
            assert abs(key[tuple(np.round(b, 12))] - wi) < 1e-15
    # the k = 1, 2 facet rules of the residual are these, weights normalised to sum 1
    for k, dg in ((1, 4), (2, 6)):
        fp, fw = facet_rule(3, k)
        if dg == deg:
            assert np.allclose(fp, pts) and np.allclose(fw, 2 * w) and abs(fw.sum() - 1) < 1e-15


@pytest.mark.parametrize("k", [1, 2, 3])
def test_poly_basis3_orthonormal_and_hierarchical(k):
    pts, w = tet_rule(2 * k)
    v, g = poly_basis3(k, pts[:, 0], pts[:, 1], pts[:, 2])
    assert np.abs(np.einsum("q,qa,qb->ab", w, v, v) - np.eye(v.shape[1])).max() < 1e-10
    npk1 = k * (k + 1) * (k + 2) // 6
    # the first dim P^{k-1} functions have degree <= k-1: they integrate exactly against
    # one another with a rule of degree 2k-2
    p2, w2 = tet_rule(2 * k - 2)
    v2, _ = poly_basis3(k, p2[:, 0], p2[:, 1], p2[:, 2])
    G = np.einsum("q,qa,qb->ab", w2, v2[:, :npk1], v2[:, :npk1])
    assert np.abs(G - np.eye(npk1)).max() < 1e-10
    # gradients: finite differences
    x0 = np.array([0.21, 0.17, 0.3])
    h = 1e-6
    _, gx = poly_basis3(k, *x0)
    for r in range(3):
        e = np.zeros(3)
        e[r] = h
        fd = (poly_basis3(k, *(x0 + e))[0] - poly_basis3(k, *(x0 - e))[0]) / (2 * h)
        assert np.abs(fd - gx[r]).max() < 1e-6 * np.abs(gx).max()


def _count_entities(xyz):
    """Vertices, edges, faces and tetrahedra of a periodic Kuhn mesh, identified modulo the
    period by their barycentres (independently of the oracle's facet matching)."""
    def key(p):
        return tuple(np.round(np.mod(p, 1.0) * 2 ** 20).astype(np.int64) % 2 ** 20)
    V, Ed, F = set(), set(), set()
    for tet in xyz:
        for a in range(4):
            V.add(key(tet[a]))
            for b in range(a + 1, 4):
                Ed.add(key(0.5 * (tet[a] + tet[b])))
                for c in range(b + 1, 4):
                    F.add(key((tet[a] + tet[b] + tet[c]) / 3.0))
    return len(V), len(Ed), len(F), len(xyz)


@pytest.mark.parametrize("N", [2, 3])
def test_kuhn_mesh_counts_and_euler(N):
    xyz, per = periodic_kuhn_cube(N, "random", seed=N)
    m = OracleMesh(xyz, per)
    V, Ed, F, T = _count_entities(xyz)
    assert (V, Ed, F, T) == (N ** 3, 7 * N ** 3, 12 * N ** 3, 6 * N ** 3)
    assert V - Ed + F - T == 0  # Euler characteristic of the 3-torus
    assert m.T == T and m.E == F
    assert abs(m.area.sum() - 1.0) < 1e-13
    assert np.allclose(m.hT, 1.0 / N)  # (6 |T|)^(1/3) is the grid spacing
    assert all(len(set(m.elem_facet[t])) == 4 for t in range(m.T))
    # outward normals: the face barycentre minus the element barycentre points along n
    for e in range(m.E):
        t, f = m.fA_elem[e], m.fA_loc[e]
        c = xyz[t].mean(axis=0)
        fb = np.delete(xyz[t], f, axis=0).mean(axis=0)
        assert np.dot(fb - c, m.normal[e]) > 0
    assert np.allclose(np.abs(m.flen - 0.5 / N ** 2 * np.array([1.0, np.sqrt(2)]).reshape(2, 1)).min(axis=0), 0)


def _de_rham_dimension(xyz, k):
    """dim {v in BDM_k : div v = 0} on a periodic mesh from the exact sequence
    Lagrange_{k+2} -> Nedelec(2nd kind)_{k+1} -> BDM_k -> P^{k-1} on the 3-torus
    (Betti numbers 1, 3, 3, 1): dim NED - dim LAG + 1."""
    V, Ed, F, T = _count_entities(xyz)
    lag = V + Ed * (k + 1) + F * k * (k + 1) // 2 + T * (k - 1) * k * (k + 1) // 6
    ned = Ed * (k + 2) + F * k * (k + 2) + T * (k - 1) * k * (k + 2) // 2
    return ned - lag + 1


@pytest.mark.parametrize("k", [1, 2])
def test_bdm3_conforming_dimensions_and_de_rham(k):
    xyz, per = periodic_kuhn_cube(2, "random", seed=3)
    o = Oracle(xyz, per, k)
    sp = o.space
    T, E = o.mesh.T, o.mesh.E
    nf = (k + 1) * (k + 2) // 2
    assert sp.ndof == E * nf + T * (3 * (k + 1) * (k + 2) * (k + 3) // 6 - 4 * nf)
    U = np.random.default_rng(k).standard_normal(sp.ndof)
    assert o.normal_jump_max(U) < 1e-12 * np.abs(U).max() * 8
    Z = sla.null_space(o.B.toarray())
    assert Z.shape[1] == _de_rham_dimension(xyz, k)
    assert Z.shape[1] == sp.ndof - (sp.npres - 1)


@pytest.mark.parametrize("k", [1, 2])
def test_mass_solve_3d_equals_svd_nullspace_projection(k):
    o = _oracle(2, k)
    Z = sla.null_space(o.B.toarray())
    M = o.M.toarray()
    f = np.random.default_rng(7).standard_normal(o.space.ndof)
    u = o.mass_solve(f)
    ub = Z @ np.linalg.solve(Z.T @ M @ Z, Z.T @ f)
    assert np.abs(u - ub).max() < 1e-11 * np.abs(ub).max()
    assert o.divergence_max(u) < 1e-10 * np.abs(u).max()


@pytest.mark.parametrize("k", [1, 2])
def test_hybrid_equals_mixed_3d(k):
    """Theorem 2 on tetrahedra: the hybrid-mixed velocity (FE3) equals the mixed one (FE2)."""
    o = _oracle(2, k, order="lex")
    Fb = np.random.default_rng(3).standard_normal((o.mesh.T, 3, o.space.nm))
    cu_h = hybrid_solve_dense(o, Fb)
    cu_m = o.space.local_coeffs(o.mass_solve(o.space.assemble(Fb)))
    assert np.abs(cu_h - cu_m).max() < 1e-10 * np.abs(cu_m).max()


@pytest.mark.parametrize("k", [1, 2])
def test_constant_field_steady_and_projected_exactly_3d(k):
    o = _oracle(2, k, nu=0.2)
    U = o.project(lambda x, y, z: (0.4 + 0 * x, -1.1 + 0 * y, 0.3 + 0 * z))
    pts, _ = tet_rule(3)
    v = o.eval_ref(U, pts)
    assert np.abs(v[:, 0] - 0.4).max() < 1e-12 and np.abs(v[:, 2] - 0.3).max() < 1e-12
    cU = o.space.local_coeffs(U)
    vol = np.zeros_like(cU)
    o.res.volume(cU, vol)
    assert np.abs(vol).max() > 0.1
    assert np.abs(o.res.broken(cU)).max() < 1e-12 * np.abs(vol).max()


@pytest.mark.parametrize("k", [1, 2])
def test_convective_energy_identity_3d(k):
    """C_h(u;u,u) = 1/2 sum_F int_F |u.n| |u+ - u-|^2 for u in V^{k,-1} (Sec. 2.2, with the
    factor 1/2 the derivation gives); the facet integral is written out here."""
    o = _oracle(2, k)
    U = o.project(RandomVectorPotentialField(seed=2, kmax=2))
    lhs = U @ o.L(U)
    m = o.mesh
    s, w = facet_rule(3, k)
    xa, xb = m.facet_points(s)
    cU = o.space.local_coeffs(U)
    va, _ = poly_basis_nd(k, xa)
    vb, _ = poly_basis_nd(k, xb)
    uA = np.einsum("eca,era->erc", cU[m.fA_elem], va)
    uB = np.einsum("eca,era->erc", cU[m.fB_elem], vb)
    un = np.einsum("erc,ec->er", uA, m.normal)
    diss = 0.5 * np.einsum("r,e,er,er->", w, m.flen, np.abs(un), ((uA - uB) ** 2).sum(-1))
    assert diss > 0
    assert abs(lhs + diss) < 1e-11 * diss


def test_viscous_form_symmetric_3d():
    o1 = _oracle(2, 1, nu=1.0, order="lex")
    o0 = _oracle(2, 1, nu=0.0, order="lex")
    n = o1.space.ndof
    A = np.zeros((n, n))
    for j in range(n):
        e = np.zeros(n)
        e[j] = 1.0
        A[:, j] = o1.L(e) - o0.L(e)
    assert np.abs(A - A.T).max() < 1e-13 * np.abs(A).max()


def test_diagnostics_3d_of_a_linear_field():
    """Energy, enstrophy (vector curl) and divergence of the linear field u = G x, whose curl
    is the constant (G32 - G23, G13 - G31, G21 - G12) and divergence the trace of G, on a
    broken projection (exact for polynomials of degree <= k)."""
    xyz, per = periodic_kuhn_cube(2, "random", seed=5)
    o = Oracle(xyz, per, 2)
    G = np.random.default_rng(4).standard_normal((3, 3))
    rule = tet_rule(6)
    x = o.phys_points(rule[0])
    vals = np.einsum("ij,tqj->tiq", G, x)
    cU = o.space.broken_project(vals, rule)
    curl = np.array([G[2, 1] - G[1, 2], G[0, 2] - G[2, 0], G[1, 0] - G[0, 1]])
    assert abs(o.enstrophy_local(cU) - (curl ** 2).sum()) < 1e-12 * (curl ** 2).sum()
    assert abs(o.divergence_max_local(cU) - abs(np.trace(G))) < 1e-12
    # energy: 1/2 int |G x|^2 over the elements as placed (unwrapped): per element the
    # second moments of the tetrahedron, int x x^T = |T| (c c^T + (sum_v v v^T - 4 c c^T)/20)
    E = 0.0
    for tet in xyz:
        c = tet.mean(axis=0)
        vol = abs(np.linalg.det((tet[1:] - tet[0]).T)) / 6
        M2 = vol * (np.outer(c, c) + (np.einsum("vi,vj->ij", tet, tet) - 4 * np.outer(c, c)) / 20)
        E += 0.5 * np.trace(G @ M2 @ G.T)
    assert abs(o.energy_local(cU) - E) < 1e-12 * E


@pytest.mark.parametrize("k", [1, 2])
def test_broken_load_vector_and_projection_3d(k):
    o = _oracle(2, k)
    coef = random_broken_poly_3d(o.mesh.T, k, seed=5)
    rule = tet_rule(2 * k)
    cU = o.space.broken_project(eval_broken_poly_3d(coef, rule[0]), rule)
    pts = np.random.default_rng(1).uniform(0, 0.3, size=(7, 3))
    v, _ = poly_basis3(k, pts[:, 0], pts[:, 1], pts[:, 2])
    assert np.abs(np.einsum("tca,pa->tcp", cU, v) - eval_broken_poly_3d(coef, pts)).max() < 1e-11


def test_abc_flow_convergence_order():
    """The ABC flow is an exact Euler solution (steady): after a short run the L2 error of
    BDM_1 on N = 4, 8 decays at about order k + 1 = 2."""
    errs = []
    for N in (4, 8):
        o = _oracle(N, 1)
        U = o.project(abc_flow)
        tend, n = 0.02, 4
        U = o.run(U, tend / n, n)
        errs.append(o.l2_error_to(U, abc_flow))
    rate = np.log2(errs[0] / errs[1])
    assert rate > 1.7, (errs, rate)


def test_inviscid_energy_non_increasing_3d():
    o = _oracle(3, 1)
    U = o.project(taylor_green_3d)
    E = [o.energy(U)]
    for _ in range(6):
        U = o.rk3_step(U, 0.1 / 3 / 2)
        E.append(o.energy(U))
    assert np.all(np.diff(E) <= 1e-14 * E[0]) and E[-1] < E[0]
    assert o.divergence_max(U) < 1e-10
