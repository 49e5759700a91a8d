"""CPU tests of the C ABI library: symbols, host validation, and the host set-up
(reference basis, facet matching, condensed facet matrix) against the oracle."""
import ctypes
import os
import re

import numpy as np
import pytest

from inputs import periodic_split_square
from oracle import Oracle
from oracle.mesh import OracleMesh
from oracle.quadrature import triangle_rule
from oracle.scheme import hybrid_system_dense

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
lib_mod = pytest.importorskip("paper_1808_04669_amd.dfdg")


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(lib_mod.LIB_PATH):
        from paper_1808_04669_amd import build
        build.build()
    return lib_mod.load_library()


P_ = ctypes.c_void_p


def _mesh(lib, xyz, per):
    xyz = np.ascontiguousarray(xyz, dtype=np.float64)
    per = np.ascontiguousarray(per, dtype=np.float64)
    h = P_()
    rc = lib.dfdg_mesh_create(2, xyz.shape[0], xyz.ctypes.data_as(P_), per.ctypes.data_as(P_), ctypes.byref(h))
    return rc, h


def _ctx(lib, mesh, **kw):
    p = lib_mod.Params()
    lib.dfdg_params_default(ctypes.byref(p))
    for k, v in kw.items():
        setattr(p, k, v)
    h = P_()
    rc = lib.dfdg_ctx_create(mesh, ctypes.byref(p), None, ctypes.byref(h))
    return rc, h


def test_header_symbols_exported(lib):
    with open(os.path.join(ROOT, "include", "dfdg.h")) as f:
        hdr = f.read()
    declared = set(re.findall(r"\b(dfdg_[a-z0-9_]+)\s*\(", hdr))
    assert declared, "no declarations found"
    for name in declared:
        assert hasattr(lib, name), name
    assert declared == set(lib_mod.EXPORTED)


def test_mesh_validation(lib):
    xyz, per = periodic_split_square(3)
    assert _mesh(lib, xyz, per)[0] == 0
    # clockwise element
    bad = xyz.copy()
    bad[0, [1, 2]] = bad[0, [2, 1]]
    assert _mesh(lib, bad, per)[0] == -2
    # non-periodic (period too large: boundary facets have no partner)
    assert _mesh(lib, xyz, np.array([2.0, 2.0]))[0] == -2
    # non-finite coordinates, bad period, bad dim
    nanx = xyz.copy()
    nanx[1, 1, 1] = np.nan
    assert _mesh(lib, nanx, per)[0] == -1
    assert _mesh(lib, xyz, np.array([-1.0, 1.0]))[0] == -1
    assert _mesh(lib, xyz, np.array([np.inf, 1.0]))[0] == -1
    h = P_()
    assert lib.dfdg_mesh_create(4, 4, xyz.ctypes.data_as(P_), per.ctypes.data_as(P_), ctypes.byref(h)) == -1
    assert lib.dfdg_mesh_create(2, 4, None, per.ctypes.data_as(P_), ctypes.byref(h)) == -1
    assert b"partner" in lib.dfdg_mesh_last_error() or True


@pytest.mark.parametrize("N,order", [(1, "lex"), (2, "morton"), (3, "random"), (8, "morton")])
def test_facet_matching_agrees_with_oracle(lib, N, order):
    xyz, per = periodic_split_square(N, order, seed=4)
    rc, h = _mesh(lib, xyz, per)
    assert rc == 0
    T, E = ctypes.c_int(), ctypes.c_int()
    lib.dfdg_mesh_counts(h, ctypes.byref(T), ctypes.byref(E))
    assert (T.value, E.value) == (2 * N * N, 3 * N * N)
    f = np.empty((E.value, 4), dtype=np.int32)
    lib.dfdg_mesh_facets(h, f.ctypes.data_as(P_))
    lib.dfdg_mesh_destroy(h)
    om = OracleMesh(xyz, per)
    lib_pairs = {frozenset([(a, b), (c, d)]) for a, b, c, d in f}
    orc_pairs = {frozenset([(a, b), (c, d)]) for a, b, c, d in
                 zip(om.fA_elem, om.fA_loc, om.fB_elem, om.fB_loc)}
    assert lib_pairs == orc_pairs
    assert np.all(f[:, 0] != f[:, 2])


def test_param_validation_and_unbound_calls(lib):
    xyz, per = periodic_split_square(2)
    rc, m = _mesh(lib, xyz, per)
    for kw in [dict(k=0), dict(k=4), dict(nu=-1.0), dict(alpha=0.0), dict(precision=7),
               dict(cg_rtol=0.0), dict(cg_maxit=0), dict(precond=5), dict(extrapolate=7), dict(extrapolate=-1),
               dict(extrapolate=6, precision=1), dict(graphs=2), dict(mg_fp32=3), dict(mg_fine_fp16=2)]:
        assert _ctx(lib, m, **kw)[0] == -1, kw
    # projected start values (FP64): accepted, with 65 vectors of n_lambda doubles more workspace
    rc, c0 = _ctx(lib, m, k=2, extrapolate=5)
    rc6, c6 = _ctx(lib, m, k=2, extrapolate=6)
    assert rc == 0 and rc6 == 0
    b0, b6 = ctypes.c_size_t(), ctypes.c_size_t()
    assert lib.dfdg_ctx_workspace_bytes(c0, ctypes.byref(b0)) == 0
    assert lib.dfdg_ctx_workspace_bytes(c6, ctypes.byref(b6)) == 0
    assert 65 * 36 * 8 <= b6.value - b0.value <= 65 * 36 * 8 + 256 * 80 + 8 * 512 * 32 + 8 * 24 * 24 + 3 * 8 * 24
    lib.dfdg_ctx_destroy(c0)
    lib.dfdg_ctx_destroy(c6)
    rc, c = _ctx(lib, m, k=2)
    assert rc == 0
    s = lib_mod.Sizes()
    assert lib.dfdg_ctx_sizes(c, ctypes.byref(s)) == 0
    T, E = 8, 12
    assert (s.T, s.E, s.P, s.n_f, s.n_p) == (T, E, 6, 3, 3)
    assert s.n_broken == 2 * 6 * T and s.n_lambda == 3 * E
    assert s.n_bdm == E * 3 + T * 3 * 1
    nb = ctypes.c_size_t()
    assert lib.dfdg_ctx_workspace_bytes(c, ctypes.byref(nb)) == 0 and nb.value > 0
    # misaligned / too small workspaces are rejected before any device call
    assert lib.dfdg_ctx_bind_workspace(c, P_(0x1001), nb.value) == -3
    assert lib.dfdg_ctx_bind_workspace(c, P_(0x100000), 16) == -3
    # entry points refuse to run without a workspace
    assert lib.dfdg_dg_residual(c, P_(0x100000), P_(0x100000)) == -3
    assert lib.dfdg_rk3_step(c, P_(0x100000), ctypes.c_double(0.1), None) == -3
    assert lib.dfdg_energy_vjp(c, P_(0x100000), ctypes.c_double(1.0), P_(0x100000)) == -3
    assert lib.dfdg_dg_residual_vjp(c, P_(0x100000), P_(0x100000), P_(0x100000)) == -3
    assert b"workspace" in lib.dfdg_last_error(c)
    lib.dfdg_ctx_destroy(c)
    lib.dfdg_mesh_destroy(m)


@pytest.mark.parametrize("k", [1, 2, 3])
def test_reference_basis_orthonormal(lib, k):
    """The Dubiner basis is L2-orthonormal on the reference triangle (checked with the
    oracle's own quadrature) and hierarchical; gradients match finite differences."""
    pts, w = triangle_rule(2 * k + 2)
    P = (k + 1) * (k + 2) // 2
    vals = np.empty((len(pts), P))
    grads = np.empty((len(pts), 2, P))
    pc = np.ascontiguousarray(pts)
    assert lib.dfdg_debug_basis(k, len(pts), pc.ctypes.data_as(P_), vals.ctypes.data_as(P_),
                                grads.ctypes.data_as(P_)) == 0
    G = np.einsum("q,qa,qb->ab", w, vals, vals)
    assert np.abs(G - np.eye(P)).max() < 1e-13
    h = 1e-6
    for d in range(2):
        e = np.zeros(2)
        e[d] = h
        vp = np.empty_like(vals)
        vm = np.empty_like(vals)
        a = np.ascontiguousarray(pts + e)
        b = np.ascontiguousarray(pts - e)
        lib.dfdg_debug_basis(k, len(pts), a.ctypes.data_as(P_), vp.ctypes.data_as(P_), None)
        lib.dfdg_debug_basis(k, len(pts), b.ctypes.data_as(P_), vm.ctypes.data_as(P_), None)
        assert np.abs((vp - vm) / (2 * h) - grads[:, d, :]).max() < 1e-6
    # value at the top vertex (collapsed-coordinate singularity) is finite
    top = np.array([[0.0, 1.0]])
    v1 = np.empty((1, P))
    lib.dfdg_debug_basis(k, 1, top.ctypes.data_as(P_), v1.ctypes.data_as(P_), None)
    assert np.all(np.isfinite(v1))


@pytest.mark.parametrize("k", [1, 2, 3])
def test_residual_volume_rule_exact(lib, k):
    """The residual's volume rule integrates every monomial xi^a eta^b of total degree
    <= 3k-1 exactly over the reference triangle (closed form a! b! / (a+b+2)!), has its
    points inside the triangle and positive weights, and has 3 / 7 points for k = 1 / 2."""
    from math import factorial
    n = ctypes.c_int(0)
    assert lib.dfdg_debug_residual_rule(k, ctypes.byref(n), None, None) == 0
    pts = np.empty((n.value, 2))
    w = np.empty(n.value)
    assert lib.dfdg_debug_residual_rule(k, ctypes.byref(n), pts.ctypes.data_as(P_), w.ctypes.data_as(P_)) == 0
    assert n.value == {1: 3, 2: 7, 3: 25}[k]
    assert np.all(w > 0) and np.all(pts > 0) and np.all(pts.sum(1) < 1)
    for a in range(3 * k):
        for b in range(3 * k - a):
            exact = factorial(a) * factorial(b) / factorial(a + b + 2)
            assert abs(np.sum(w * pts[:, 0] ** a * pts[:, 1] ** b) - exact) < 1e-15
    # one degree higher is not integrated exactly by the symmetric rules (they are minimal)
    if k < 3:
        d = 3 * k
        errs = [abs(np.sum(w * pts[:, 0] ** a * pts[:, 1] ** (d - a))
                    - factorial(a) * factorial(d - a) / factorial(d + 2)) for a in range(d + 1)]
        assert max(errs) > 1e-8
    assert lib.dfdg_debug_residual_rule(0, ctypes.byref(n), None, None) != 0


@pytest.mark.parametrize("k", [1, 2, 3])
@pytest.mark.parametrize("N", [2, 3])
def test_facet_matrix_equals_oracle_condensation(lib, k, N):
    """The library's facet matrix S equals the static condensation of the oracle's dense
    hybrid-mixed system (eq. (FE3)) onto the multipliers, after the change of facet basis
    (library: sqrt(2m+1) P_m(2s-1) / sqrt|F|; oracle: P_m(2s-1); same facet parameter)."""
    xyz, per = periodic_split_square(N, "random", seed=N + k)
    rc, m = _mesh(lib, xyz, per)
    rc, c = _ctx(lib, m, k=k)
    assert rc == 0
    s = lib_mod.Sizes()
    lib.dfdg_ctx_sizes(c, ctypes.byref(s))
    E, NF = s.E, s.n_f
    cols = np.empty((5, E), dtype=np.int32)
    vals = np.empty((5, NF, NF, E))
    assert lib.dfdg_debug_facet_matrix(c, cols.ctypes.data_as(P_), vals.ctypes.data_as(P_)) == 0
    lib.dfdg_ctx_destroy(c)
    fac = np.empty((E, 4), dtype=np.int32)
    lib.dfdg_mesh_facets(m, fac.ctypes.data_as(P_))
    lib.dfdg_mesh_destroy(m)
    S = np.zeros((E * NF, E * NF))
    for sl in range(5):
        for F in range(E):
            S[F * NF:(F + 1) * NF, cols[sl, F] * NF:(cols[sl, F] + 1) * NF] += vals[sl, :, :, F]
    orc = Oracle(xyz, per, k)
    K, nU, nW = hybrid_system_dense(orc)
    nx = nU + nW
    Kxx, Kxl = K[:nx, :nx], K[:nx, nx:]
    So = Kxl.T @ np.linalg.solve(Kxx, Kxl)
    # map oracle facets (side A order) to library facets (side L order): same first element
    om = orc.mesh
    key = {(a, b): F for F, (a, b) in enumerate(zip(om.fA_elem, om.fA_loc))}
    perm = np.array([key[(fac[F, 0], fac[F, 1])] for F in range(E)])
    scale = np.sqrt(2 * np.arange(NF) + 1)[None, :] / np.sqrt(om.flen[perm])[:, None]  # [E, NF]
    idx = (perm[:, None] * NF + np.arange(NF)[None, :]).ravel()
    So_lib = So[np.ix_(idx, idx)] * np.outer(scale.ravel(), scale.ravel())
    assert np.abs(S - So_lib).max() < 1e-11 * np.abs(So_lib).max()
    assert np.abs(S - S.T).max() < 1e-13 * np.abs(S).max()


def _lib_facet_matrix(lib, xyz, per, **kw):
    """Dense facet matrix of a library context and the mesh's facet table."""
    rc, m = _mesh(lib, xyz, per)
    assert rc == 0
    rc, c = _ctx(lib, m, **kw)
    assert rc == 0
    s = lib_mod.Sizes()
    lib.dfdg_ctx_sizes(c, ctypes.byref(s))
    E, NF = s.E, s.n_f
    cols = np.empty((5, E), dtype=np.int32)
    vals = np.empty((5, NF, NF, E))
    assert lib.dfdg_debug_facet_matrix(c, cols.ctypes.data_as(P_), vals.ctypes.data_as(P_)) == 0
    lib.dfdg_ctx_destroy(c)
    fac = np.empty((E, 4), dtype=np.int32)
    lib.dfdg_mesh_facets(m, fac.ctypes.data_as(P_))
    lib.dfdg_mesh_destroy(m)
    S = np.zeros((E * NF, E * NF))
    for sl in range(5):
        for F in range(E):
            S[F * NF:(F + 1) * NF, cols[sl, F] * NF:(cols[sl, F] + 1) * NF] += vals[sl, :, :, F]
    return S, fac


def _to_lib_facets(orc, S_orc, fac):
    """An oracle facet matrix in the library's facet numbering and facet basis."""
    om, NF = orc.mesh, orc.space.nf
    key = {(a, b): F for F, (a, b) in enumerate(zip(om.fA_elem, om.fA_loc))}
    perm = np.array([key[(fac[F, 0], fac[F, 1])] for F in range(fac.shape[0])])
    scale = np.sqrt(2 * np.arange(NF) + 1)[None, :] / np.sqrt(om.flen[perm])[:, None]
    idx = (perm[:, None] * NF + np.arange(NF)[None, :]).ravel()
    return S_orc[np.ix_(idx, idx)] * np.outer(scale.ravel(), scale.ravel())


@pytest.mark.parametrize("walls", [False, True])
@pytest.mark.parametrize("k", [1, 2, 3])
def test_fe4_facet_matrix_equals_oracle_fe4(lib, k, walls):
    """local_space = DFDG_LOCAL_FE4 (eq. (FE4): Piola images of the orthonormalised
    reference curls, per-element Gram inverse) gives the facet matrix of the oracle's FE4
    (its own stream-function basis per element) and of the library's FE3 route, on a mesh
    with distorted vertices, so that every element has its own Gram matrix."""
    from inputs import channel_split_square, distort_split_square
    from oracle.fe4 import fe4_facet_matrix
    N = 3
    xyz, per = (channel_split_square if walls else periodic_split_square)(N, "random", seed=k)
    xyz = distort_split_square(xyz, per, N, 0.15, seed=7 + k)
    S4, fac = _lib_facet_matrix(lib, xyz, per, k=k, local_space=1)
    S3, _ = _lib_facet_matrix(lib, xyz, per, k=k, local_space=0)
    orc = Oracle(xyz, per, k)
    So = _to_lib_facets(orc, fe4_facet_matrix(orc), fac)
    assert np.abs(S4 - So).max() < 1e-11 * np.abs(So).max()
    assert np.abs(S4 - S3).max() < 1e-12 * np.abs(S3).max()
    assert np.abs(S4 - S4.T).max() < 1e-13 * np.abs(S4).max()


@pytest.mark.parametrize("k", [1, 2, 3])
def test_facet_matrix_with_outflow_equals_oracle_condensation(lib, k):
    """Inflow at x = 0 (closed), outflow at x = 1 (open), periodic in y: the library's S
    equals the oracle's condensed FE3 system, which has no multiplier on the outflow facets,
    with identity blocks on those rows; S is then definite."""
    from inputs import inout_split_square, outflow_at_right
    N = 3
    xyz, per = inout_split_square(N, "random", seed=k)
    rc, m = _mesh(lib, xyz, per)
    assert rc == 0
    E = ctypes.c_int()
    T = ctypes.c_int()
    lib.dfdg_mesh_counts(m, ctypes.byref(T), ctypes.byref(E))
    fac = np.empty((E.value, 4), dtype=np.int32)
    lib.dfdg_mesh_facets(m, fac.ctypes.data_as(P_))
    b = fac[:, 2] < 0
    mid = 0.5 * (xyz[fac[:, 0], (fac[:, 1] + 1) % 3] + xyz[fac[:, 0], (fac[:, 1] + 2) % 3])
    opn = (b & outflow_at_right(mid)).astype(np.int32)
    assert opn.sum() == N and b.sum() == 2 * N
    bad = np.zeros(E.value, dtype=np.int32)
    bad[np.nonzero(~b)[0][0]] = 1  # an interior facet cannot be an outflow facet
    assert lib.dfdg_mesh_set_outflow(m, bad.ctypes.data_as(P_)) == -1
    assert lib.dfdg_mesh_set_outflow(m, opn.ctypes.data_as(P_)) == 0
    rc, c = _ctx(lib, m, k=k)
    assert rc == 0
    s = lib_mod.Sizes()
    lib.dfdg_ctx_sizes(c, ctypes.byref(s))
    NF = s.n_f
    cols = np.empty((5, E.value), dtype=np.int32)
    vals = np.empty((5, NF, NF, E.value))
    assert lib.dfdg_debug_facet_matrix(c, cols.ctypes.data_as(P_), vals.ctypes.data_as(P_)) == 0
    lib.dfdg_ctx_destroy(c)
    lib.dfdg_mesh_destroy(m)
    S = np.zeros((E.value * NF, E.value * NF))
    for sl in range(5):
        for F in range(E.value):
            S[F * NF:(F + 1) * NF, cols[sl, F] * NF:(cols[sl, F] + 1) * NF] += vals[sl, :, :, F]
    orc = Oracle(xyz, per, k, outflow=outflow_at_right)
    K, nU, nW = hybrid_system_dense(orc)
    nx = nU + nW
    So = _to_lib_facets(orc, K[:nx, nx:].T @ np.linalg.solve(K[:nx, :nx], K[:nx, nx:]), fac)
    for F in np.nonzero(opn)[0]:
        So[F * NF:(F + 1) * NF, F * NF:(F + 1) * NF] = np.eye(NF)
    assert np.abs(S - So).max() < 1e-11 * np.abs(So).max()
    assert np.linalg.eigvalsh(S)[0] > 1e-8 * np.abs(S).max()


def test_local_space_parameter(lib):
    xyz, per = periodic_split_square(2)
    rc, m = _mesh(lib, xyz, per)
    assert _ctx(lib, m, local_space=2)[0] == -1
    lib.dfdg_mesh_destroy(m)
    from inputs import periodic_kuhn_cube
    xyz3, per3 = periodic_kuhn_cube(2)
    h = P_()
    assert lib.dfdg_mesh_create(3, xyz3.shape[0], np.ascontiguousarray(xyz3).ctypes.data_as(P_),
                                np.ascontiguousarray(per3, dtype=float).ctypes.data_as(P_), ctypes.byref(h)) == 0
    assert _ctx(lib, h, local_space=1)[0] == -8  # tetrahedra: FE3 only
    lib.dfdg_mesh_destroy(h)


@pytest.mark.parametrize("k,N", [(1, 3), (2, 4), (3, 3)])
def test_facet_matrix_with_walls_equals_oracle_condensation(lib, k, N):
    """On the channel (period (1, 0): walls at y = 0, 1) the boundary facets have one side
    (element R = -1); the facet matrix still equals the condensation of the oracle's dense
    FE3 system, whose boundary multipliers enforce u.n = 0, and keeps the constant
    multiplier as its only kernel."""
    from inputs import channel_split_square
    xyz, per = channel_split_square(N, "random", seed=N + k)
    rc, m = _mesh(lib, xyz, per)
    assert rc == 0
    rc, c = _ctx(lib, m, k=k)
    assert rc == 0
    s = lib_mod.Sizes()
    lib.dfdg_ctx_sizes(c, ctypes.byref(s))
    E, NF = s.E, s.n_f
    cols = np.empty((5, E), dtype=np.int32)
    vals = np.empty((5, NF, NF, E))
    assert lib.dfdg_debug_facet_matrix(c, cols.ctypes.data_as(P_), vals.ctypes.data_as(P_)) == 0
    lib.dfdg_ctx_destroy(c)
    fac = np.empty((E, 4), dtype=np.int32)
    lib.dfdg_mesh_facets(m, fac.ctypes.data_as(P_))
    lib.dfdg_mesh_destroy(m)
    assert E == 3 * N * N + N and (fac[:, 2] < 0).sum() == 2 * N and (fac[:, 3] < 0).sum() == 2 * N
    S = np.zeros((E * NF, E * NF))
    for sl in range(5):
        for F in range(E):
            S[F * NF:(F + 1) * NF, cols[sl, F] * NF:(cols[sl, F] + 1) * NF] += vals[sl, :, :, F]
    orc = Oracle(xyz, per, k)
    K, nU, nW = hybrid_system_dense(orc)
    nx = nU + nW
    So = K[:nx, nx:].T @ np.linalg.solve(K[:nx, :nx], K[:nx, nx:])
    om = orc.mesh
    key = {(a, b): F for F, (a, b) in enumerate(zip(om.fA_elem, om.fA_loc))}
    perm = np.array([key[(fac[F, 0], fac[F, 1])] for F in range(E)])
    assert np.array_equal(om.bnd[perm], fac[:, 2] < 0)
    scale = np.sqrt(2 * np.arange(NF) + 1)[None, :] / np.sqrt(om.flen[perm])[:, None]
    idx = (perm[:, None] * NF + np.arange(NF)[None, :]).ravel()
    So_lib = So[np.ix_(idx, idx)] * np.outer(scale.ravel(), scale.ravel())
    assert np.abs(S - So_lib).max() < 1e-11 * np.abs(So_lib).max()
    w = np.linalg.eigvalsh(S)
    assert abs(w[0]) < 1e-10 * w[-1] < w[1]


def test_mesh_periods(lib):
    """A period component 0 means walls (triangles and tetrahedra); negative periods are
    rejected."""
    xyz, _ = periodic_split_square(3)
    assert _mesh(lib, xyz, np.array([1.0, -1.0]))[0] == -1
    rc, m = _mesh(lib, xyz, np.array([0.0, 0.0]))  # walls on all four sides
    assert rc == 0
    E = ctypes.c_int()
    T = ctypes.c_int()
    lib.dfdg_mesh_counts(m, ctypes.byref(T), ctypes.byref(E))
    assert E.value == 3 * 9 + 2 * 3  # 3 N^2 + 2 N facets on the square with four walls
    lib.dfdg_mesh_destroy(m)
    from inputs import periodic_kuhn_cube
    xyz3, _ = periodic_kuhn_cube(2)
    h = P_()
    per3 = np.array([1.0, 1.0, 0.0])
    assert lib.dfdg_mesh_create(3, xyz3.shape[0], np.ascontiguousarray(xyz3).ctypes.data_as(P_),
                                per3.ctypes.data_as(P_), ctypes.byref(h)) == 0
    E3 = ctypes.c_int()
    T3 = ctypes.c_int()
    lib.dfdg_mesh_counts(h, ctypes.byref(T3), ctypes.byref(E3))
    fac = np.empty((E3.value, 4), dtype=np.int32)
    lib.dfdg_mesh_facets(h, fac.ctypes.data_as(P_))
    assert T3.value == 48 and (fac[:, 2] < 0).sum() == 16  # two walls of 2 x 2 squares, 2 faces each
    lib.dfdg_mesh_destroy(h)
    per3[2] = -1.0
    assert lib.dfdg_mesh_create(3, xyz3.shape[0], np.ascontiguousarray(xyz3).ctypes.data_as(P_),
                                per3.ctypes.data_as(P_), ctypes.byref(h)) == -1


@pytest.mark.parametrize("k,N", [(1, 24), (2, 20), (3, 12)])
def test_multigrid_hierarchy(lib, k, N):
    """Aggregation coarsens the facet system by at least a factor 2 per level down to a
    dense coarsest level of at most 1000 rows; the Chebyshev bound rho(D^{-1} S) of the
    finest level exceeds 1 (the diagonal of an SPD matrix lies inside its spectrum), stays
    below the Gershgorin bound of the oracle-checked facet matrix and is within 2 % of its
    spectral radius."""
    xyz, per = periodic_split_square(N, "morton")
    rc, m = _mesh(lib, xyz, per)
    rc, c = _ctx(lib, m, k=k, precond=2)
    assert rc == 0
    s = lib_mod.Sizes()
    lib.dfdg_ctx_sizes(c, ctypes.byref(s))
    E, NF = s.E, s.n_f
    L = ctypes.c_int()
    rows = np.zeros(16, dtype=np.int64)
    nnz = np.zeros(16, dtype=np.int64)
    rho = np.zeros(16)
    assert lib.dfdg_debug_multigrid(c, 16, ctypes.byref(L), rows.ctypes.data_as(P_), nnz.ctypes.data_as(P_),
                                    rho.ctypes.data_as(P_)) == 0
    nl = L.value
    cols = np.empty((5, E), dtype=np.int32)
    vals = np.empty((5, NF, NF, E))
    lib.dfdg_debug_facet_matrix(c, cols.ctypes.data_as(P_), vals.ctypes.data_as(P_))
    lib.dfdg_ctx_destroy(c)
    lib.dfdg_mesh_destroy(m)
    assert nl >= 2 and rows[0] == E * NF
    assert all(2 * rows[l + 1] <= rows[l] for l in range(nl - 1))
    assert rows[nl - 1] <= 1000 and all(rows[l] > 1000 for l in range(nl - 1))
    # Gershgorin bound of D^{-1} S from the BSR blocks
    S = np.zeros((E * NF, E * NF))
    for sl in range(5):
        for F in range(E):
            S[F * NF:(F + 1) * NF, cols[sl, F] * NF:(cols[sl, F] + 1) * NF] += vals[sl, :, :, F]
    d = np.diag(S)
    gersh = (np.abs(S).sum(axis=1) / d).max()
    assert 1.0 < rho[0] <= gersh * (1 + 1e-12)
    assert abs(rho[0] - np.abs(np.linalg.eigvals(S / d[:, None])).max()) < 0.02 * rho[0]


def test_binding_covers_the_entry_points():
    """Every hot-path entry point of the C ABI has its method on the Python binding."""
    methods = {"dfdg_project": "project", "dfdg_load_vector": "load_vector", "dfdg_dg_residual": "residual",
               "dfdg_hdiv_mass_solve": "mass_solve", "dfdg_rk3_step": "rk3_step",
               "dfdg_rk4_step": "rk4_step", "dfdg_fe_step": "fe_step",
               "dfdg_rk3_step_stages": "rk3_step_stages", "dfdg_reset_history": "reset_history",
               "dfdg_reset_adjoint_history": "reset_adjoint_history", "dfdg_history_save": "history_save",
               "dfdg_history_restore": "history_restore", "dfdg_dg_residual_vjp": "residual_vjp",
               "dfdg_rk3_step_vjp": "rk3_step_vjp", "dfdg_rk3_step_vjp_stages": "rk3_step_vjp_stages",
               "dfdg_energy_vjp": "energy_vjp",
               "dfdg_diagnostics": "diagnostics", "dfdg_eval": "eval", "dfdg_time_kernel": "time_kernel",
               "dfdg_proj_rule": "proj_rule"}
    for sym, meth in methods.items():
        assert sym in lib_mod.EXPORTED, sym
        assert callable(getattr(lib_mod.Solver, meth, None)), meth
