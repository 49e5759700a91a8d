"""Thin ctypes binding of libdfdg.so (the C ABI in include/dfdg.h).

Only argument marshalling lives here: every step of the method runs in the HIP
kernels of the library.  PyTorch provides device memory (the workspace and the
vectors) and the stream.  Loading fails loudly if the library is missing; there
is no fallback path.
"""
import ctypes
import os
import time

import numpy as np
import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libdfdg.so")

DFDG_OK = 0
STATUS = {0: "OK", -1: "E_INVALID_ARG", -2: "E_MESH", -3: "E_WORKSPACE", -4: "E_HIP",
          -5: "E_NOT_CONVERGED", -6: "E_NONFINITE", -7: "E_BREAKDOWN", -8: "E_UNSUPPORTED"}
FP64, MIXED = 0, 1
JACOBI, BLOCK_JACOBI, AMG = 0, 1, 2
HISTORY_DEPTH = 6  # DFDG_HISTORY_DEPTH: earlier multipliers kept per stage
EXTRAPOLATE_ADAPTIVE = 5  # extrapolate="adaptive": order chosen per solve by a one-step backtest
EXTRAPOLATE_PROJECT = 6  # extrapolate="project": projection onto earlier solutions (S-norm)


class DfdgError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"dfdg {STATUS.get(code, code)}: {msg}")
        self.code = code


class Params(ctypes.Structure):
    _fields_ = [("k", ctypes.c_int), ("nu", ctypes.c_double), ("alpha", ctypes.c_double),
                ("precision", ctypes.c_int), ("cg_rtol", ctypes.c_double), ("cg_maxit", ctypes.c_int),
                ("precond", ctypes.c_int), ("ir_rtol", ctypes.c_double), ("inner_rtol", ctypes.c_double),
                ("extrapolate", ctypes.c_int), ("graphs", ctypes.c_int), ("mg_fp32", ctypes.c_int),
                ("mg_fine_fp16", ctypes.c_int), ("facet_blocks", ctypes.c_int), ("matrix_free", ctypes.c_int),
                ("mixed_solver", ctypes.c_int),
                ("mg_fine_smooth", ctypes.c_int),
                ("local_space", ctypes.c_int)]


class Sizes(ctypes.Structure):
    _fields_ = [("T", ctypes.c_int32), ("E", ctypes.c_int32), ("k", ctypes.c_int32), ("P", ctypes.c_int32),
                ("n_f", ctypes.c_int32), ("n_p", ctypes.c_int32), ("n_broken", ctypes.c_int64),
                ("n_lambda", ctypes.c_int64), ("n_bdm", ctypes.c_int64), ("nq_proj", ctypes.c_int32),
                ("dim", ctypes.c_int32)]


class SolveInfo(ctypes.Structure):
    _fields_ = [("iterations", ctypes.c_int), ("refinements", ctypes.c_int),
                ("rel_residual", ctypes.c_double), ("status", ctypes.c_int),
                ("initial_rel_residual", ctypes.c_double)]


class StepInfo(ctypes.Structure):
    _fields_ = [("iterations", ctypes.c_int * 3), ("max_refinements", ctypes.c_int),
                ("max_rel_residual", ctypes.c_double), ("status", ctypes.c_int),
                ("initial_rel_residual", ctypes.c_double * 3)]


class Rk4Info(ctypes.Structure):
    _fields_ = [("iterations", ctypes.c_int * 4), ("max_rel_residual", ctypes.c_double), ("status", ctypes.c_int)]


class Diag(ctypes.Structure):
    _fields_ = [("energy", ctypes.c_double), ("enstrophy", ctypes.c_double), ("max_div", ctypes.c_double),
                ("max_normal_jump", ctypes.c_double)]


_lib = None

# name -> (restype, argtypes)
_P = ctypes.c_void_p
_SIGS = {
    "dfdg_mesh_create": (ctypes.c_int, [ctypes.c_int, ctypes.c_int, _P, _P, ctypes.POINTER(_P)]),
    "dfdg_mesh_destroy": (None, [_P]),
    "dfdg_mesh_last_error": (ctypes.c_char_p, []),
    "dfdg_mesh_counts": (ctypes.c_int, [_P, ctypes.POINTER(ctypes.c_int), ctypes.POINTER(ctypes.c_int)]),
    "dfdg_mesh_facets": (ctypes.c_int, [_P, _P]),
    "dfdg_mesh_set_outflow": (ctypes.c_int, [_P, _P]),
    "dfdg_params_default": (None, [ctypes.POINTER(Params)]),
    "dfdg_ctx_create": (ctypes.c_int, [_P, ctypes.POINTER(Params), _P, ctypes.POINTER(_P)]),
    "dfdg_ctx_set_stream": (ctypes.c_int, [_P, _P]),
    "dfdg_ctx_sizes": (ctypes.c_int, [_P, ctypes.POINTER(Sizes)]),
    "dfdg_ctx_workspace_bytes": (ctypes.c_int, [_P, ctypes.POINTER(ctypes.c_size_t)]),
    "dfdg_ctx_bind_workspace": (ctypes.c_int, [_P, _P, ctypes.c_size_t]),
    "dfdg_last_error": (ctypes.c_char_p, [_P]),
    "dfdg_ctx_destroy": (None, [_P]),
    "dfdg_proj_rule": (ctypes.c_int, [_P, _P, _P]),
    "dfdg_load_vector": (ctypes.c_int, [_P, _P, _P]),
    "dfdg_project": (ctypes.c_int, [_P, _P, _P, ctypes.POINTER(SolveInfo)]),
    "dfdg_dg_residual": (ctypes.c_int, [_P, _P, _P]),
    "dfdg_hdiv_mass_solve": (ctypes.c_int, [_P, _P, _P, _P, ctypes.POINTER(SolveInfo)]),
    "dfdg_rk3_step": (ctypes.c_int, [_P, _P, ctypes.c_double, ctypes.POINTER(StepInfo)]),
    "dfdg_rk3_step_stages": (ctypes.c_int, [_P, _P, ctypes.c_double, _P, _P, ctypes.POINTER(StepInfo)]),
    "dfdg_rk4_step": (ctypes.c_int, [_P, _P, ctypes.c_double, ctypes.POINTER(Rk4Info)]),
    "dfdg_fe_step": (ctypes.c_int, [_P, _P, ctypes.c_double, ctypes.POINTER(SolveInfo)]),
    "dfdg_reset_history": (ctypes.c_int, [_P]),
    "dfdg_reset_adjoint_history": (ctypes.c_int, [_P]),
    "dfdg_history_bytes": (ctypes.c_int, [_P, ctypes.POINTER(ctypes.c_size_t)]),
    "dfdg_history_save": (ctypes.c_int, [_P, _P, _P]),
    "dfdg_history_restore": (ctypes.c_int, [_P, _P, _P]),
    "dfdg_dg_residual_vjp": (ctypes.c_int, [_P, _P, _P, _P]),
    "dfdg_rk3_step_vjp": (ctypes.c_int, [_P, _P, _P, ctypes.c_double, ctypes.POINTER(StepInfo)]),
    "dfdg_rk3_step_vjp_stages": (ctypes.c_int, [_P, _P, _P, _P, _P, ctypes.c_double, ctypes.POINTER(StepInfo)]),
    "dfdg_energy_vjp": (ctypes.c_int, [_P, _P, ctypes.c_double, _P]),
    "dfdg_diagnostics": (ctypes.c_int, [_P, _P, ctypes.POINTER(Diag)]),
    "dfdg_diagnostics_noalloc": (ctypes.c_int, [_P, _P, ctypes.POINTER(Diag)]),
    "dfdg_eval": (ctypes.c_int, [_P, _P, ctypes.c_int, _P, _P]),
    "dfdg_time_kernel": (ctypes.c_int, [_P, ctypes.c_int, ctypes.c_int, ctypes.POINTER(ctypes.c_float),
                                        ctypes.POINTER(ctypes.c_double)]),
    "dfdg_debug_basis": (ctypes.c_int, [ctypes.c_int, ctypes.c_int, _P, _P, _P]),
    "dfdg_debug_residual_rule": (ctypes.c_int, [ctypes.c_int, _P, _P, _P]),
    "dfdg_debug_facet_matrix": (ctypes.c_int, [_P, _P, _P]),
    "dfdg_debug_basis3": (ctypes.c_int, [ctypes.c_int, ctypes.c_int, _P, _P, _P]),
    "dfdg_debug_rule3": (ctypes.c_int, [ctypes.c_int, ctypes.c_int, _P, _P, _P]),
    "dfdg_debug_multigrid": (ctypes.c_int, [_P, ctypes.c_int, ctypes.POINTER(ctypes.c_int), _P, _P, _P]),
    "dfdg_debug_multigrid_matrix": (ctypes.c_int, [_P, ctypes.c_int, ctypes.c_int, _P, _P, _P, _P, _P, _P]),
    "dfdg_debug_vcycle": (ctypes.c_int, [_P, _P, _P]),
    "dfdg_debug_facet_rhs": (ctypes.c_int, [_P, _P]),
}
EXPORTED = tuple(_SIGS)


def load_library(path=LIB_PATH):
    """Load libdfdg.so and declare every entry point (raises if anything is missing)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise ImportError(f"libdfdg.so not found at {path}: build it with `python -m paper_1808_04669_amd.build`")
    lib = ctypes.CDLL(path)
    for name, (res, args) in _SIGS.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr())


def rule3(k, which):
    """dfdg_debug_rule3: (points, weights) of the tetrahedral path's volume (which = 0),
    face (1) or projection (2) rule."""
    lib = load_library()
    n = ctypes.c_int()
    rc = lib.dfdg_debug_rule3(int(k), int(which), ctypes.byref(n), None, None)
    if rc != DFDG_OK:
        raise DfdgError(rc, "dfdg_debug_rule3")
    d = 2 if which == 1 else 3
    pts = np.empty((n.value, d))
    w = np.empty(n.value)
    lib.dfdg_debug_rule3(int(k), int(which), ctypes.byref(n), pts.ctypes.data_as(_P), w.ctypes.data_as(_P))
    return pts, w


class Mesh:
    """A simplex mesh (host object of the library): xyz[T, 3, 2] triangles or xyz[T, 4, 3]
    tetrahedra; period[dim] > 0 periodic, 0 boundary facets in that direction, closed
    (walls, inflow) unless ``outflow(barycentres[n, dim]) -> bool[n]`` marks them as an
    outflow boundary."""

    def __init__(self, xyz, period, outflow=None):
        lib = load_library()
        xyz = np.ascontiguousarray(xyz, dtype=np.float64)
        per = np.ascontiguousarray(period, dtype=np.float64)
        self.dim = xyz.shape[2]
        if xyz.ndim != 3 or xyz.shape[1] != self.dim + 1 or per.shape != (self.dim,):
            raise ValueError("xyz must be [T, 3, 2] or [T, 4, 3] and period [dim]")
        h = ctypes.c_void_p()
        rc = lib.dfdg_mesh_create(self.dim, xyz.shape[0], xyz.ctypes.data_as(_P), per.ctypes.data_as(_P),
                                  ctypes.byref(h))
        if rc != DFDG_OK:
            raise DfdgError(rc, lib.dfdg_mesh_last_error().decode())
        self._h = h
        self._lib = lib
        T, E = ctypes.c_int(), ctypes.c_int()
        lib.dfdg_mesh_counts(h, ctypes.byref(T), ctypes.byref(E))
        self.T, self.E = T.value, E.value
        self.open = np.zeros(self.E, dtype=bool)
        if outflow is not None:
            fac = self.facets()
            b = np.nonzero(fac[:, 2] < 0)[0]
            if b.size:
                L, f = fac[b, 0], fac[b, 1]
                if self.dim == 2:  # local facet f: the edge (f+1) -> (f+2)
                    mid = 0.5 * (xyz[L, (f + 1) % 3] + xyz[L, (f + 2) % 3])
                else:  # local face f: the face opposite vertex f
                    mid = (xyz[L].sum(axis=1) - xyz[L, f]) / 3.0
                self.open[b] = np.asarray(outflow(mid), dtype=bool)
            marks = np.ascontiguousarray(self.open, dtype=np.int32)
            rc = lib.dfdg_mesh_set_outflow(h, marks.ctypes.data_as(_P))
            if rc != DFDG_OK:
                raise DfdgError(rc, lib.dfdg_mesh_last_error().decode())

    def facets(self):
        out = np.empty((self.E, 4), dtype=np.int32)
        self._lib.dfdg_mesh_facets(self._h, out.ctypes.data_as(_P))
        return out

    def __del__(self):
        if getattr(self, "_h", None):
            self._lib.dfdg_mesh_destroy(self._h)
            self._h = None


class Solver:
    """One discretisation context on one GPU: mesh + parameters + bound workspace.

    Vectors are torch float64 CUDA tensors of length n_broken (velocity-like,
    layout [d][P][T]) or n_lambda (facet multipliers, [E][n_f]).
    """

    def __init__(self, xyz, period, k, nu=0.0, alpha=2.0, precision="fp64", cg_rtol=1e-12, cg_maxit=20000,
                 precond="jacobi", ir_rtol=1e-10, inner_rtol=1e-4, extrapolate=0, graphs=True, mg_fp32=True,
                 mg_fine_fp16=True, facet_blocks=0, matrix_free=False, mixed_solver="krylov", local_space="fe3",
                 outflow=None, mg_fine_smooth=None, device="cuda:0", stream=None):
        lib = load_library()
        self._lib = lib
        self.device = torch.device(device)
        t0 = time.perf_counter()
        self.mesh = Mesh(xyz, period, outflow)
        t1 = time.perf_counter()
        p = Params()
        lib.dfdg_params_default(ctypes.byref(p))
        p.k, p.nu, p.alpha = int(k), float(nu), float(alpha)
        p.precision = {"fp64": FP64, "mixed": MIXED}[precision]
        p.cg_rtol, p.cg_maxit = float(cg_rtol), int(cg_maxit)
        p.precond = {"jacobi": JACOBI, "block_jacobi": BLOCK_JACOBI, "amg": AMG}[precond]
        p.ir_rtol, p.inner_rtol = float(ir_rtol), float(inner_rtol)
        p.extrapolate = {"adaptive": EXTRAPOLATE_ADAPTIVE, "project": EXTRAPOLATE_PROJECT}.get(extrapolate, extrapolate)
        p.extrapolate = int(p.extrapolate)
        p.graphs = 1 if graphs else 0
        p.mg_fp32 = 1 if mg_fp32 else 0
        p.mg_fine_fp16 = 1 if mg_fine_fp16 else 0
        p.facet_blocks = int(facet_blocks)
        p.matrix_free = 1 if matrix_free else 0
        p.mixed_solver = {"krylov": 1, "restarted": 0}[mixed_solver]
        p.local_space = {"fe3": 0, "fe4": 1}[local_space]
        if mg_fine_smooth is not None:
            p.mg_fine_smooth = int(mg_fine_smooth)
        self.params = p
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        h = ctypes.c_void_p()
        rc = lib.dfdg_ctx_create(self.mesh._h, ctypes.byref(p), ctypes.c_void_p(self.stream.cuda_stream),
                                 ctypes.byref(h))
        if rc != DFDG_OK:
            raise DfdgError(rc, lib.dfdg_last_error(None).decode())
        t2 = time.perf_counter()
        self._h = h
        s = Sizes()
        self._check(lib.dfdg_ctx_sizes(h, ctypes.byref(s)))
        self.sizes = s
        self.T, self.E, self.k, self.P, self.dim = s.T, s.E, s.k, s.P, s.dim
        self.n_broken, self.n_lambda, self.n_bdm, self.nq_proj = s.n_broken, s.n_lambda, s.n_bdm, s.nq_proj
        nb = ctypes.c_size_t()
        self._check(lib.dfdg_ctx_workspace_bytes(h, ctypes.byref(nb)))
        self.workspace = torch.empty(nb.value + 256, dtype=torch.uint8, device=self.device)
        base = self.workspace.data_ptr()
        off = (-base) % 256
        self._check(lib.dfdg_ctx_bind_workspace(h, ctypes.c_void_p(base + off), nb.value))
        t3 = time.perf_counter()
        # wall-clock seconds of the set-up calls: mesh (facet matching), context (host set-up:
        # tabulations, geometry, element condensation, facet matrix, multigrid hierarchy),
        # workspace (allocation, upload, device-side packing)
        self.setup_seconds = {"mesh": t1 - t0, "context": t2 - t1, "workspace": t3 - t2}

    # ---- helpers ------------------------------------------------------------------
    def _check(self, rc):
        if rc != DFDG_OK:
            raise DfdgError(rc, self._lib.dfdg_last_error(self._h if hasattr(self, "_h") else None).decode())

    def _vec(self, t, n, name):
        if not (isinstance(t, torch.Tensor) and t.dtype == torch.float64 and t.device == self.device
                and t.is_contiguous() and t.numel() == n):
            raise ValueError(f"{name}: expected a contiguous float64 tensor of {n} elements on {self.device}")
        return _ptr(t)

    def new_vector(self, kind="broken"):
        n = self.n_broken if kind == "broken" else self.n_lambda
        return torch.zeros(n, dtype=torch.float64, device=self.device)

    def proj_rule(self):
        pts = np.empty((self.nq_proj, self.dim))
        w = np.empty(self.nq_proj)
        self._check(self._lib.dfdg_proj_rule(self._h, pts.ctypes.data_as(_P), w.ctypes.data_as(_P)))
        return pts, w

    def set_stream(self, stream):
        """Move the context to another torch stream (dfdg_ctx_set_stream waits for the work
        still queued on the previous one)."""
        self._check(self._lib.dfdg_ctx_set_stream(self._h, ctypes.c_void_p(stream.cuda_stream)))
        self.stream = stream

    def residual_rule(self):
        """Points [n, d] and weights [n] of the residual's volume rule (also the points of
        max |div u| in the diagnostics)."""
        if self.dim == 3:
            return rule3(self.k, 0)
        n = ctypes.c_int()
        self._check(self._lib.dfdg_debug_residual_rule(self.k, ctypes.byref(n), None, None))
        pts = np.empty((n.value, 2))
        w = np.empty(n.value)
        self._check(self._lib.dfdg_debug_residual_rule(self.k, ctypes.byref(n), pts.ctypes.data_as(_P),
                                                       w.ctypes.data_as(_P)))
        return pts, w

    # ---- entry points -----------------------------------------------------------------
    def load_vector(self, f_at_q, F=None):
        F = self.new_vector() if F is None else F
        fq = f_at_q.contiguous()
        self._check(self._lib.dfdg_load_vector(self._h, self._vec(fq, self.dim * self.nq_proj * self.T, "f_at_q"),
                                               self._vec(F, self.n_broken, "F")))
        return F

    def project(self, f_at_q, U=None):
        U = self.new_vector() if U is None else U
        info = SolveInfo()
        fq = f_at_q.contiguous()
        self._check(self._lib.dfdg_project(self._h, self._vec(fq, self.dim * self.nq_proj * self.T, "f_at_q"),
                                           self._vec(U, self.n_broken, "U"), ctypes.byref(info)))
        return U, info

    def residual(self, U, L=None):
        L = self.new_vector() if L is None else L
        self._check(self._lib.dfdg_dg_residual(self._h, self._vec(U, self.n_broken, "U"),
                                               self._vec(L, self.n_broken, "L")))
        return L

    def mass_solve(self, F, U=None, lam=None):
        U = self.new_vector() if U is None else U
        info = SolveInfo()
        lp = None if lam is None else self._vec(lam, self.n_lambda, "lambda")
        self._check(self._lib.dfdg_hdiv_mass_solve(self._h, self._vec(F, self.n_broken, "F"),
                                                   self._vec(U, self.n_broken, "U"), lp, ctypes.byref(info)))
        return U, info

    def rk3_step(self, U, dt):
        info = StepInfo()
        self._check(self._lib.dfdg_rk3_step(self._h, self._vec(U, self.n_broken, "U"), ctypes.c_double(dt),
                                            ctypes.byref(info)))
        return info

    def rk4_step(self, U, dt):
        """One classical RK4 step in place (dfdg_rk4_step)."""
        info = Rk4Info()
        self._check(self._lib.dfdg_rk4_step(self._h, self._vec(U, self.n_broken, "U"), ctypes.c_double(dt),
                                            ctypes.byref(info)))
        return info

    def fe_step(self, U, dt):
        """One forward-Euler step in place (dfdg_fe_step)."""
        info = SolveInfo()
        self._check(self._lib.dfdg_fe_step(self._h, self._vec(U, self.n_broken, "U"), ctypes.c_double(dt),
                                           ctypes.byref(info)))
        return info

    def rk3_step_stages(self, U, dt, U1, U2):
        """rk3_step that also leaves the states entering stages 2 and 3 in U1 and U2."""
        info = StepInfo()
        self._check(self._lib.dfdg_rk3_step_stages(self._h, self._vec(U, self.n_broken, "U"), ctypes.c_double(dt),
                                                   self._vec(U1, self.n_broken, "U1"),
                                                   self._vec(U2, self.n_broken, "U2"), ctypes.byref(info)))
        return info

    def reset_history(self):
        self._check(self._lib.dfdg_reset_history(self._h))

    def reset_adjoint_history(self):
        self._check(self._lib.dfdg_reset_adjoint_history(self._h))

    def history_save(self):
        """Snapshot of the forward warm-start history: (device tensor, counts)."""
        nb = ctypes.c_size_t()
        self._check(self._lib.dfdg_history_bytes(self._h, ctypes.byref(nb)))
        buf = torch.empty(nb.value // 8, dtype=torch.float64, device=self.device)
        counts = (ctypes.c_int * 3)()
        self._check(self._lib.dfdg_history_save(self._h, _ptr(buf), counts))
        return buf, tuple(counts)

    def history_restore(self, snap):
        buf, counts = snap
        c = (ctypes.c_int * 3)(*counts)
        self._check(self._lib.dfdg_history_restore(self._h, self._vec(buf, buf.numel(), "history"), c))

    def residual_vjp(self, U, Lbar, Ubar=None):
        Ubar = self.new_vector() if Ubar is None else Ubar
        self._check(self._lib.dfdg_dg_residual_vjp(self._h, self._vec(U, self.n_broken, "U"),
                                                   self._vec(Lbar, self.n_broken, "Lbar"),
                                                   self._vec(Ubar, self.n_broken, "Ubar")))
        return Ubar

    def rk3_step_vjp(self, Un, Ubar, dt):
        """In place: Ubar (cotangent of U^{n+1}) becomes the cotangent of U^n."""
        info = StepInfo()
        self._check(self._lib.dfdg_rk3_step_vjp(self._h, self._vec(Un, self.n_broken, "Un"),
                                                self._vec(Ubar, self.n_broken, "Ubar"), ctypes.c_double(dt),
                                                ctypes.byref(info)))
        return info

    def energy_vjp(self, U, Ebar, Ubar=None):
        """dfdg_energy_vjp: the cotangent Ebar U of the kinetic energy 1/2 U . U."""
        Ubar = self.new_vector() if Ubar is None else Ubar
        self._check(self._lib.dfdg_energy_vjp(self._h, self._vec(U, self.n_broken, "U"), ctypes.c_double(Ebar),
                                              self._vec(Ubar, self.n_broken, "Ubar")))
        return Ubar

    def rk3_step_vjp_stages(self, Un, U1, U2, Ubar, dt):
        """rk3_step_vjp with the stage states given (from rk3_step_stages)."""
        info = StepInfo()
        self._check(self._lib.dfdg_rk3_step_vjp_stages(self._h, self._vec(Un, self.n_broken, "Un"),
                                                       self._vec(U1, self.n_broken, "U1"),
                                                       self._vec(U2, self.n_broken, "U2"),
                                                       self._vec(Ubar, self.n_broken, "Ubar"), ctypes.c_double(dt),
                                                       ctypes.byref(info)))
        return info

    def diagnostics(self, U):
        d = Diag()
        self._check(self._lib.dfdg_diagnostics(self._h, self._vec(U, self.n_broken, "U"), ctypes.byref(d)))
        return {"energy": d.energy, "enstrophy": d.enstrophy, "max_div": d.max_div,
                "max_normal_jump": d.max_normal_jump}

    def diagnostics_noalloc(self, U):
        """dfdg_diagnostics_noalloc: the diagnostics with the library's static scratch."""
        d = Diag()
        self._check(self._lib.dfdg_diagnostics_noalloc(self._h, self._vec(U, self.n_broken, "U"), ctypes.byref(d)))
        return {"energy": d.energy, "enstrophy": d.enstrophy, "max_div": d.max_div,
                "max_normal_jump": d.max_normal_jump}

    def eval(self, U, ref_pts):
        ref = np.ascontiguousarray(ref_pts, dtype=np.float64)
        n = ref.shape[0]
        if ref.shape != (n, self.dim):
            raise ValueError(f"ref_pts must be [n, {self.dim}]")
        out = torch.empty(self.dim * n * self.T, dtype=torch.float64, device=self.device)
        self._check(self._lib.dfdg_eval(self._h, self._vec(U, self.n_broken, "U"), n, ref.ctypes.data_as(_P),
                                        _ptr(out)))
        return out.view(self.dim, n, self.T)

    def mg_levels(self):
        """Rows of the multigrid levels (empty unless precond="amg")."""
        L = ctypes.c_int()
        rows = np.zeros(16, dtype=np.int64)
        nnz = np.zeros(16, dtype=np.int64)
        rho = np.zeros(16)
        self._check(self._lib.dfdg_debug_multigrid(self._h, 16, ctypes.byref(L), rows.ctypes.data_as(_P),
                                                   nnz.ctypes.data_as(_P), rho.ctypes.data_as(_P)))
        return [int(r) for r in rows[:L.value]]

    def mg_matrix(self, level, which):
        """dfdg_debug_multigrid_matrix as a scipy CSR matrix (which: 0 A_level, 1 P, 2 the
        dense coarsest pseudo-inverse)."""
        import scipy.sparse as sp
        n, m, nz = ctypes.c_int64(), ctypes.c_int64(), ctypes.c_int64()
        self._check(self._lib.dfdg_debug_multigrid_matrix(self._h, int(level), int(which), ctypes.byref(n),
                                                           ctypes.byref(m), ctypes.byref(nz), None, None, None))
        ptr = np.empty(n.value + 1, dtype=np.int64)
        col = np.empty(nz.value, dtype=np.int32)
        val = np.empty(nz.value)
        self._check(self._lib.dfdg_debug_multigrid_matrix(self._h, int(level), int(which), ctypes.byref(n),
                                                           ctypes.byref(m), ctypes.byref(nz), ptr.ctypes.data_as(_P),
                                                           col.ctypes.data_as(_P), val.ctypes.data_as(_P)))
        return sp.csr_matrix((val, col, ptr), shape=(n.value, m.value))

    def vcycle(self, b):
        """dfdg_debug_vcycle: one V-cycle of the context's multigrid applied to b."""
        z = torch.empty_like(b)
        self._check(self._lib.dfdg_debug_vcycle(self._h, self._vec(b, self.n_lambda, "b"),
                                                self._vec(z, self.n_lambda, "z")))
        return z

    def facet_rhs(self):
        """dfdg_debug_facet_rhs: the facet right-hand side of the last solve."""
        g = torch.empty(self.n_lambda, dtype=torch.float64, device=self.device)
        self._check(self._lib.dfdg_debug_facet_rhs(self._h, self._vec(g, self.n_lambda, "g")))
        return g

    def time_kernel(self, which, reps=50):
        ms = ctypes.c_float()
        b = ctypes.c_double()
        self._check(self._lib.dfdg_time_kernel(self._h, int(which), int(reps), ctypes.byref(ms), ctypes.byref(b)))
        return ms.value, b.value

    # ---- layout helpers -----------------------------------------------------------------
    def to_tcp(self, U):
        """View [d, P, T] of a broken vector."""
        return U.view(self.dim, self.P, self.T)

    def __del__(self):
        if getattr(self, "_h", None):
            self._lib.dfdg_ctx_destroy(self._h)
            self._h = None
