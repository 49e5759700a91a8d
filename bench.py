"""Benchmark: velocity DOF-stages per second of the explicit divergence-free DG hot path.

Workload (default): inviscid double shear layer on the 256x256 periodic split unit square
(131072 triangles), BDM_2 velocity + P1 pressure + P2 facet multipliers, FP64, TVD-RK3 at
CFL 0.1, facet PCG to relative residual 1e-12, 200 steps.  Synthetic data (the closed-form
initial field), projected on the GPU.  One step = one TVD-RK3 step = three passes of the
hot path (residual -> condensation -> facet PCG -> recovery).

Prints one JSON line.  Extra objects: "roofline" (PCG SpMV kernel, timed live with HIP
events), "cpu_baseline" (the CPU oracle on a bounded sample), "accuracy" (FP64 and mixed
GPU paths vs the oracle on that sample), "random_numbering" (the same workload on a
randomly numbered mesh), "mixed" (mixed-precision form vs FP64 on the 512x512 BDM_3
double shear layer), "adjoint" (gradient of the final kinetic energy on the 128x128
BDM_2 random field: reverse sweep and whole gradient over the forward rollout).
"""
import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
COUNTERS = os.path.join(ROOT, "profiles", "k_pcg_spmv_dsl256_bdm2_counters.md")
COUNTERS_3D = os.path.join(ROOT, "profiles", "k_pcg_spmv_tg3d32_bdm2_counters.md")
KERNEL_SRC = os.path.join(ROOT, "paper_1808_04669_amd", "csrc", "dfdg_kernels.hip")


def measured_traffic(path=COUNTERS):
    """HBM bytes per k_pcg_spmv launch from the committed counter runs, or None when the
    kernel source changed since they were taken."""
    import hashlib
    try:
        with open(path) as f:
            txt = f.read()
        with open(KERNEL_SRC, "rb") as f:
            sha = hashlib.sha256(f.read()).hexdigest()[:16]
    except OSError:
        return None
    vals = dict(line.split(": ", 1) for line in txt.splitlines() if line.startswith(("traffic_bytes", "kernel_source")))
    if vals.get("kernel_source_sha256", "").strip() != sha:
        return None
    return float(vals["traffic_bytes_per_launch"])


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--N", type=int, default=256)
    ap.add_argument("--k", type=int, default=2)
    ap.add_argument("--rtol", type=float, default=1e-12)
    ap.add_argument("--precond", default="amg", choices=["jacobi", "block_jacobi", "amg"])
    ap.add_argument("--extrapolate", default="project",
                    help="warm-start extrapolation order 0..4, adaptive (chosen per solve), or project "
                         "(projection onto earlier solutions)")
    ap.add_argument("--order", default="morton")
    ap.add_argument("--no-mg-fp16", action="store_true",
                    help="finest-level multigrid smoothing reads S in FP32 instead of FP16")
    ap.add_argument("--no-cpu-baseline", action="store_true",
                    help="skip the oracle timing and the accuracy check against the oracle")
    ap.add_argument("--no-mixed", action="store_true", help="skip the mixed-precision comparison")
    ap.add_argument("--no-adjoint", action="store_true", help="skip the adjoint timing")
    ap.add_argument("--no-random-order", action="store_true", help="skip the randomly numbered mesh run")
    ap.add_argument("--no-3d", action="store_true", help="skip the 3D Taylor-Green run")
    ap.add_argument("--mg-fine-smooth", type=int, default=None,
                    help="damped-Jacobi steps of the finest multigrid prolongator")
    ap.add_argument("--no-local-spaces", action="store_true",
                    help="skip the FE3 / FE4 local-space comparison")
    ap.add_argument("--local-steps", type=int, default=50)
    ap.add_argument("--only-3d", action="store_true",
                    help="run only the 3D Taylor-Green leg and print its object (profiling)")
    ap.add_argument("--three-d-variants", default="amg,amg_matrix_free,jacobi_matrix_free",
                    help="comma list of the extra 3D solver variants to run beside Jacobi PCG")
    ap.add_argument("--three-d-N", type=int, default=32)
    ap.add_argument("--three-d-steps", type=int, default=50)
    ap.add_argument("--mixed-N", type=int, default=512)
    ap.add_argument("--mixed-k", type=int, default=3)
    ap.add_argument("--mixed-steps", type=int, default=20)
    ap.add_argument("--mixed-ir-rtol", type=float, default=1e-10)
    ap.add_argument("--mixed-inner-rtol", type=float, default=1e-3)
    ap.add_argument("--adjoint-N", type=int, default=128)
    ap.add_argument("--adjoint-steps", type=int, default=100)
    ap.add_argument("--cpu-sample-N", type=int, default=64)
    ap.add_argument("--cpu-sample-steps", type=int, default=3)
    ap.add_argument("--copy-calib-mb", type=int, default=0,
                    help="run one plain device copy of this many MB first (counter calibration)")
    return ap.parse_args()


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def project_field(s, field):
    """GPU L2 projection of a closed-form field sampled at the library's projection points
    (triangles or tetrahedra); returns U, max |u| at those points and the solve info."""
    import torch
    pts, _ = s.proj_rule()
    xyz = s._xyz
    J = np.transpose(xyz[:, 1:] - xyz[:, :1], (0, 2, 1))
    x = xyz[:, None, 0, :] + np.einsum("tir,qr->tqi", J, pts)
    u = field(*[x[..., i] for i in range(s.dim)])  # d arrays [T, nq]
    vmax = float(np.sqrt(sum(c ** 2 for c in u)).max())
    fq = torch.from_numpy(np.ascontiguousarray(np.stack([c.T for c in u]))).to(s.device).reshape(-1)
    del x, u
    U, info = s.project(fq)
    return U, vmax, info


def make_solver(N, k, precision, args, order=None, rtol=None, nu=0.0, **kw):
    from inputs import periodic_split_square
    from paper_1808_04669_amd import Solver
    xyz, per = periodic_split_square(N, order or args.order)
    # the projected start values run in FP64 contexts; mixed ones extrapolate
    ex = kw.pop("extrapolate", args.extrapolate)
    if precision == "mixed" and ex == "project":
        ex = "adaptive"
    s = Solver(xyz, per, k, nu=nu, precision=precision, cg_rtol=rtol or args.rtol, precond=args.precond,
               extrapolate=ex,
               **{"mg_fine_fp16": not args.no_mg_fp16, "mg_fine_smooth": args.mg_fine_smooth, **kw})
    s._xyz = xyz
    return s


def timed_run(s, U, dt, steps, warmup, start_residuals=None):
    """Times `steps` TVD-RK3 steps after `warmup` untimed ones; returns the seconds and the
    PCG iterations per stage. The stages' start-value relative residuals are appended to
    `start_residuals` when given."""
    import torch
    its = []
    for _ in range(warmup):
        s.rk3_step(U, dt)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        info = s.rk3_step(U, dt)
        its.append(list(info.iterations))
        if start_residuals is not None:
            start_residuals.extend(info.initial_rel_residual)
    torch.cuda.synchronize()
    return time.perf_counter() - t0, np.array(its)


def cpu_baseline(args):
    """The oracle (global mixed BDM solve with SuperLU) on the same workload at a reduced
    size; returns the timing and the oracle's final state (for the accuracy check)."""
    from inputs import double_shear_layer, periodic_split_square
    from oracle import Oracle
    N, k = args.cpu_sample_N, args.k
    xyz, per = periodic_split_square(N, args.order)
    orc = Oracle(xyz, per, k, nu=0.0)
    t0 = time.perf_counter()
    orc.factor()
    t_factor = time.perf_counter() - t0
    U0 = orc.project(double_shear_layer)
    vmax = sample_vmax(orc, U0)
    dt = 0.1 / N / (k ** 2 * vmax)
    U = U0
    t0 = time.perf_counter()
    for _ in range(args.cpu_sample_steps):
        U = orc.rk3_step(U, dt)
    t = time.perf_counter() - t0
    n_u = orc.space.ndof
    try:
        threads = len(os.sched_getaffinity(0))
    except Exception:
        threads = os.cpu_count()
    out = {"value": n_u * 3 * args.cpu_sample_steps / t, "unit": "velocity DOF-stages/s", "cores": 1,
           "kind": "oracle",
           "sample": (f"double shear layer, BDM_{k}, {N}x{N} split mesh ({2 * N * N} triangles, N_u={n_u}), "
                      f"{args.cpu_sample_steps} TVD-RK3 steps timed after a {t_factor:.1f} s SuperLU factorisation "
                      f"(excluded, like the GPU set-up); SuperLU and the NumPy residual run on one core "
                      f"({threads} host threads visible)")}
    return out, (orc, U0, U, dt)


def sample_vmax(orc, U):
    from oracle.quadrature import triangle_rule
    pts, _ = triangle_rule(2 * orc.k + 2)
    v = orc.eval_ref(U, pts)  # [T, 2, nq]
    return float(np.sqrt((v ** 2).sum(axis=1)).max())


def accuracy_vs_oracle(args, orc, U0_orc, U_orc, dt):
    """Relative L2 difference between the GPU paths and the oracle after the same steps on
    the sample mesh, both starting from the oracle's projected initial field (a piecewise
    polynomial, which the library takes over exactly through its orthonormal basis)."""
    import torch
    from oracle.quadrature import triangle_rule
    pts, w = triangle_rule(2 * orc.k + 2)
    o = orc.eval_ref(U_orc, pts)
    out = {}
    for prec in ("fp64", "mixed"):
        kw = dict(ir_rtol=args.mixed_ir_rtol, inner_rtol=args.mixed_inner_rtol) if prec == "mixed" else {}
        s = make_solver(args.cpu_sample_N, orc.k, prec, args, **kw)
        qp, _ = s.proj_rule()
        vals = np.ascontiguousarray(np.transpose(orc.eval_ref(U0_orc, qp), (1, 2, 0)))  # [2, nq, T]
        U = s.load_vector(torch.from_numpy(vals).to(s.device).reshape(-1))
        for _ in range(args.cpu_sample_steps):
            s.rk3_step(U, dt)
        g = s.eval(U, pts).cpu().numpy().transpose(2, 0, 1)
        out[prec] = orc.l2_diff(g, o, (pts, w)) / orc.l2_diff(o, 0 * o, (pts, w))
        if prec == "fp64":
            out["max_div_fp64"] = s.diagnostics(U)["max_div"]
        del s
    return {"rel_l2_fp64_vs_oracle": out["fp64"], "rel_l2_mixed_vs_oracle": out["mixed"],
            "max_div_fp64": out["max_div_fp64"], "max_div_oracle": orc.divergence_max(U_orc),
            "sample": f"{args.cpu_sample_N}x{args.cpu_sample_N} mesh, BDM_{orc.k}, {args.cpu_sample_steps} steps"}


def mixed_vs_fp64(args):
    """Mixed-precision form against the FP64 path on the 512x512 BDM_3 double shear layer
    (facet solves to relative residual 1e-10 in both)."""
    import torch
    from inputs import double_shear_layer
    N, k, steps = args.mixed_N, args.mixed_k, args.mixed_steps
    res, start_res = {}, {}
    for prec in ("fp64", "fp64_plain", "mixed", "mixed_restarted"):
        kw = dict(ir_rtol=args.mixed_ir_rtol, inner_rtol=args.mixed_inner_rtol) if prec.startswith("mixed") else {}
        if prec == "fp64_plain":
            kw["mg_fp32"] = False
        if prec == "mixed_restarted":
            kw["mixed_solver"] = "restarted"
        s = make_solver(N, k, "mixed" if prec.startswith("mixed") else "fp64", args, rtol=args.mixed_ir_rtol, **kw)
        U, vmax, _ = project_field(s, double_shear_layer)
        dt = 0.1 / N / (k ** 2 * vmax)
        r0 = []
        t, its = timed_run(s, U, dt, steps, 2, r0)
        start_res[prec] = float(np.exp(np.mean(np.log(np.maximum(r0, 1e-300)))))
        res[prec] = (t, its, U, s.n_bdm, s.diagnostics(U), s.setup_seconds)
        del s
        torch.cuda.empty_cache()
    t64, it64, U64, n_u, d64, su64 = res["fp64"]
    tpl, itpl, _, _, _, _ = res["fp64_plain"]
    tm, itm, Um, _, dm, sum_ = res["mixed"]
    tr, itr, Ur, _, dr, _ = res["mixed_restarted"]
    return {"workload": f"double shear layer {N}x{N} split mesh, BDM_{k}, {steps} TVD-RK3 steps, "
                        f"FP64 PCG rtol {args.mixed_ir_rtol:g} vs mixed (FP32 residual, FP32 inner iterations, "
                        f"FP64 refinement to {args.mixed_ir_rtol:g})",
            "value": n_u * 3 * steps / tm, "fp64_value": n_u * 3 * steps / t64, "unit": "velocity DOF-stages/s",
            "speedup_vs_fp64": t64 / tm, "rel_l2_vs_fp64_gpu": ((Um - U64).norm() / U64.norm()).item(),
            "fp64_plain_value": n_u * 3 * steps / tpl, "speedup_vs_fp64_plain": tpl / tm,
            "restarted_value": n_u * 3 * steps / tr, "restarted_speedup_vs_fp64_plain": tpl / tr,
            "restarted_rel_l2_vs_fp64_gpu": ((Ur - U64).norm() / U64.norm()).item(),
            "note": ("mixed: FP32 residual, FP64 PCG refining to the FP64 tolerance with the multigrid "
                     "cycle in FP32 (FP16 S on the finest level) as the inner FP32 iterations; "
                     "mixed_restarted: FP32 residual, FP32 inner PCG on an FP32 S to inner rtol, "
                     "restarted FP64 refinement; fp64: FP64 residual, FP64 PCG with the FP32 cycle "
                     "(the benchmark path); fp64_plain: everything in FP64"),
            "iterations_per_stage": {"fp64": float(it64.mean()), "fp64_plain": float(itpl.mean()),
                                     "mixed": float(itm.mean()), "mixed_restarted_inner_total": float(itr.mean())},
            "max_div": {"fp64": d64["max_div"], "mixed": dm["max_div"], "mixed_restarted": dr["max_div"]},
            "max_normal_jump": {"fp64": d64["max_normal_jump"], "mixed": dm["max_normal_jump"],
                                "mixed_restarted": dr["max_normal_jump"]},
            "start_rel_residual_geomean": start_res,
            "setup_s": {"fp64": su64, "mixed": sum_}}


def three_d(args):
    """The 3D periodic Taylor-Green vortex on the 32^3 Kuhn-split cube (196608 tetrahedra),
    BDM_2, nu = 1/1600, FP64, Jacobi-preconditioned facet PCG, TVD-RK3 at CFL 0.1: velocity
    DOF-stages/s, the 7-slot facet SpMV against the HBM peak (its 793 MB matrix is three
    times the Infinity Cache), set-up time, and the FP64 error against the oracle on the
    same workload at N = 4 (where its sparse direct solve still runs)."""
    import torch
    from inputs import periodic_kuhn_cube, taylor_green_3d
    from paper_1808_04669_amd import Solver
    N, k, nu, steps = args.three_d_N, 2, 1.0 / 1600, args.three_d_steps
    xyz, per = periodic_kuhn_cube(N, args.order)
    # other solver variants on the same workload: the multigrid-preconditioned PCG, and
    # matrix-free products of the facet system in both
    variants = {}
    all_variants = (("amg", dict(precond="amg")), ("amg_matrix_free", dict(precond="amg", matrix_free=True)),
                    ("jacobi_matrix_free", dict(precond="jacobi", matrix_free=True)))
    wanted = [v for v in args.three_d_variants.split(",") if v]
    for name, kw in all_variants:
        if name not in wanted:
            continue
        sa = Solver(xyz, per, k, nu=nu, cg_rtol=args.rtol, extrapolate=args.extrapolate,
                    mg_fine_smooth=args.mg_fine_smooth, **kw)
        sa._xyz = xyz
        Ua, vmax, _ = project_field(sa, taylor_green_3d)
        dt = 0.1 * (1.0 / N) / (k ** 2 * vmax)
        ta, itsa = timed_run(sa, Ua, dt, steps, 2)
        v = {"value": sa.n_bdm * 3 * steps / ta, "ms_per_step": 1e3 * ta / steps,
             "pcg_iterations_per_stage": float(itsa.mean()), "setup_s": sa.setup_seconds,
             "diagnostics_final": sa.diagnostics(Ua)}
        if kw["precond"] == "amg":
            v["levels_rows"] = sa.mg_levels()
            ms_vc, b_vc = sa.time_kernel(4, reps=20)
            v["vcycle"] = {"us": round(ms_vc * 1e3, 3), "GB/s": round(b_vc / ms_vc / 1e6, 1)}
        ms_sp, b_sp = sa.time_kernel(0, reps=20)
        v["spmv"] = {"us": round(ms_sp * 1e3, 3), "bytes": b_sp, "GB/s": round(b_sp / ms_sp / 1e6, 1)}
        variants[name] = v
        log("3d variant", name, v)
        del sa, Ua
        torch.cuda.empty_cache()
    s = Solver(xyz, per, k, nu=nu, cg_rtol=args.rtol, precond="jacobi", extrapolate=args.extrapolate)
    s._xyz = xyz
    U, vmax, pinfo = project_field(s, taylor_green_3d)
    dt = 0.1 * (1.0 / N) / (k ** 2 * vmax)
    t, its = timed_run(s, U, dt, steps, 2)
    d = s.diagnostics(U)
    ms_spmv, b_spmv = s.time_kernel(0, reps=50)
    ms_res, b_res = s.time_kernel(2, reps=50)
    spmv_gbs = b_spmv / (ms_spmv * 1e-3) / 1e9
    out = {"workload": f"3D periodic Taylor-Green, {N}^3 Kuhn-split cube ({s.T} tetrahedra), BDM_{k}, "
                       f"nu=1/1600, FP64, Jacobi PCG rtol {args.rtol:g}, TVD-RK3 CFL 0.1, {steps} steps",
           "value": s.n_bdm * 3 * steps / t, "unit": "velocity DOF-stages/s", "ms_per_step": 1e3 * t / steps,
           "N_u": s.n_bdm, "T": s.T, "E": s.E, "dt": dt, "projection_iterations": pinfo.iterations,
           "pcg_iterations_per_stage": {"mean": float(its.mean()), "max": int(its.max()), "min": int(its.min())},
           "diagnostics_final": d, "setup_s": s.setup_seconds,
           "spmv": {"kernel": "k_pcg_spmv<6, 7> (7-slot face BSR SpMV + p update + (p,Sp) partials)",
                    "avg_launch_us": round(ms_spmv * 1e3, 3), "bytes_per_launch": b_spmv,
                    "achieved_GBs": round(spmv_gbs, 1), "frac": round(spmv_gbs / HBM_PEAK_GBS, 4),
                    "traffic": measured_traffic(COUNTERS_3D)},
           "residual": {"avg_launch_us": round(ms_res * 1e3, 3), "bytes_per_launch": b_res,
                        "GBs": round(b_res / (ms_res * 1e-3) / 1e9, 1)},
           "variants": variants}
    del s
    torch.cuda.empty_cache()
    if not args.no_cpu_baseline:
        out["accuracy"] = three_d_accuracy(args)
    return out


def three_d_accuracy(args):
    """Relative L2 difference between the GPU FP64 path and the oracle after 3 steps of the
    3D Taylor-Green workload on the 4^3 Kuhn mesh (BDM_2, nu = 1/1600), both from the
    oracle's projected initial field."""
    import torch
    from inputs import periodic_kuhn_cube, taylor_green_3d
    from oracle import Oracle
    from oracle.quadrature import tet_rule
    from paper_1808_04669_amd import Solver
    N, k, nu, steps = 4, 2, 1.0 / 1600, 3
    xyz, per = periodic_kuhn_cube(N, args.order)
    orc = Oracle(xyz, per, k, nu=nu)
    U0 = orc.project(taylor_green_3d)
    dt = 0.1 / N / k ** 2
    Uo = U0
    for _ in range(steps):
        Uo = orc.rk3_step(Uo, dt)
    s = Solver(xyz, per, k, nu=nu, cg_rtol=1e-13, precond="jacobi", extrapolate=2)
    qp, _ = s.proj_rule()
    vals = np.ascontiguousarray(np.transpose(orc.eval_ref(U0, qp), (1, 2, 0)))
    U = s.load_vector(torch.from_numpy(vals).to(s.device).reshape(-1))
    for _ in range(steps):
        s.rk3_step(U, dt)
    pts, w = tet_rule(2 * k + 2)
    g = s.eval(U, pts).cpu().numpy().transpose(2, 0, 1)
    o = orc.eval_ref(Uo, pts)
    return {"rel_l2_fp64_vs_oracle": orc.l2_diff(g, o, (pts, w)) / orc.l2_diff(o, 0 * o, (pts, w)),
            "max_div_fp64": s.diagnostics(U)["max_div"], "max_div_oracle": orc.divergence_max(Uo),
            "sample": f"{N}^3 Kuhn mesh, BDM_{k}, nu=1/1600, {steps} steps"}


def local_spaces(args):
    """The two element-local spaces of the condensation on the headline workload: FE3
    (broken velocity + P^{k-1} pressure, projector I - D^T (D D^T)^{-1} D) and FE4 (locally
    divergence-free velocity, projector Z (Z^T Z)^{-1} Z^T), same steps from the same state:
    time per step, the two element kernels they differ in, and the difference of the results."""
    from inputs import double_shear_layer
    N, k = args.N, args.k
    out, Us = {}, {}
    for ls in ("fe3", "fe4"):
        s = make_solver(N, k, "fp64", args, local_space=ls)
        U, vmax, _ = project_field(s, double_shear_layer)
        dt = 0.1 * (1.0 / N) / (k ** 2 * vmax)
        t, its = timed_run(s, U, dt, args.local_steps, 2)
        d = s.diagnostics(U)
        rec = {"ms_per_step": 1e3 * t / args.local_steps, "pcg_iterations_per_stage": float(its.mean()),
               "max_div": d["max_div"], "max_normal_jump": d["max_normal_jump"],
               "setup_s": s.setup_seconds}
        for name, which in (("k_cond_rhs", 5), ("k_recover", 6)):
            ms, b = s.time_kernel(which, reps=100)
            rec[name] = {"us": round(ms * 1e3, 3), "bytes": b, "GB/s": round(b / ms / 1e6, 1)}
        out[ls] = rec
        Us[ls] = U
        del s
    out["rel_diff_fe4_fe3"] = float(((Us["fe4"] - Us["fe3"]).norm() / Us["fe3"].norm()).item())
    out["steps"] = args.local_steps
    return out


def adjoint_cost(args):
    """Gradient of the final kinetic energy through checkpointed TVD-RK3 steps (random
    divergence-free field, nu = 1e-3): time of the plain forward rollout, of the forward
    pass with checkpoints and of the reverse sweep."""
    import torch
    from inputs import RandomStreamField
    from paper_1808_04669_amd.adjoint import final_energy
    N, k, steps, every = args.adjoint_N, 2, args.adjoint_steps, 10
    # extrapolated start values: the checkpointed recomputation repeats the original solves
    # bit for bit (the projection basis is not part of the saved history)
    s = make_solver(N, k, "fp64", args, nu=1e-3, extrapolate="adaptive")
    U0, vmax, _ = project_field(s, RandomStreamField(seed=0, kmax=8))
    dt = 0.1 / N / (k ** 2 * vmax)
    U = U0.clone()
    s.reset_history()
    s.rk3_step(U, dt)  # first use: graph capture
    s.reset_history()  # both timed runs start from a fresh state without warm-start history
    torch.cuda.synchronize()
    t_fwd, _ = timed_run(s, U0.clone(), dt, steps, 0)
    # second context on its own stream: recomputes checkpoint segments during the sweep
    r = make_solver(N, k, "fp64", args, nu=1e-3, stream=torch.cuda.Stream(), extrapolate="adaptive")
    times = {}
    for name, rec in (("sequential", None), ("pipelined", r)):
        U0r = U0.clone().requires_grad_(True)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        E = final_energy(s, U0r, dt, steps, checkpoint_every=every, recompute_solver=rec)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        E.backward()
        torch.cuda.synchronize()
        t2 = time.perf_counter()
        times[name] = (t1 - t0, t2 - t1, U0r.grad)
    tf, tb, g = times["pipelined"]
    same = bool(torch.equal(g, times["sequential"][2]))
    return {"workload": f"random stream-function field (|k|<=8, seed 0), {N}x{N} split mesh, BDM_{k}, nu=1e-3, "
                        f"{steps} TVD-RK3 steps, checkpoints every {every} steps, FP64",
            "forward_s": t_fwd, "forward_with_checkpoints_s": tf, "backward_s": tb,
            "backward_over_forward": tb / t_fwd, "gradient_over_forward": (tf + tb) / t_fwd,
            "sequential_backward_over_forward": times["sequential"][1] / t_fwd,
            "sequential_gradient_over_forward": sum(times["sequential"][:2]) / t_fwd,
            "pipelined_equals_sequential": same,
            "note": ("backward: reverse sweep with a second solver context recomputing the next checkpoint "
                     "segment on its own stream; sequential: one context"),
            "final_energy": E.item(), "grad_norm": g.norm().item()}


def main():
    args = parse()
    if args.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU only; --gpus must be 1"}))
        sys.exit(2)
    import torch
    from inputs import double_shear_layer
    if args.copy_calib_mb > 0:
        n = args.copy_calib_mb * (1 << 20) // 8
        a = torch.ones(n, dtype=torch.float64, device="cuda:0")
        b = torch.empty_like(a)
        torch.cuda.synchronize()
        b.copy_(a)
        torch.cuda.synchronize()
        log(f"copy calibration: {n * 8} bytes read, {n * 8} bytes written")
        del a, b
    if args.only_3d:
        print(json.dumps({"three_d": three_d(args)}), flush=True)
        return
    N, k = args.N, args.k
    s = make_solver(N, k, "fp64", args)
    U, vmax, pinfo = project_field(s, double_shear_layer)
    dt = 0.1 * (1.0 / N) / (k ** 2 * vmax)
    log(f"workload: N={N} k={k} T={s.T} E={s.E} N_u={s.n_bdm} dt={dt:.4e} projection iters={pinfo.iterations}")
    r0 = []
    t, its = timed_run(s, U, dt, args.steps, args.warmup, r0)
    value = s.n_bdm * 3 * args.steps / t
    d = s.diagnostics(U)
    log(f"fp64: {t:.3f} s for {args.steps} steps, mean PCG iterations/stage {its.mean():.1f}, diag {d}")

    # roofline of the dominant kernel: the facet SpMV of the PCG, timed live on the ctx stream
    ms_spmv, bytes_spmv = s.time_kernel(0, reps=200)
    ms_upd, bytes_upd = s.time_kernel(1, reps=200)
    ms_res, bytes_res = s.time_kernel(2, reps=200)
    ms_vc, bytes_vc = s.time_kernel(4, reps=50) if args.precond == "amg" else (None, None)
    achieved = bytes_spmv / (ms_spmv * 1e-3) / 1e9
    roof = {"kernel": "k_pcg_spmv (facet BSR SpMV + p update + (p,Sp) partials)", "bound": "hbm",
            "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": measured_traffic(),
            "avg_launch_us": round(ms_spmv * 1e3, 3), "bytes_per_launch": bytes_spmv,
            "others": {"k_pcg_update": {"us": round(ms_upd * 1e3, 3), "GB/s": round(bytes_upd / ms_upd / 1e6, 1)},
                       "k_residual": {"us": round(ms_res * 1e3, 3), "GB/s": round(bytes_res / ms_res / 1e6, 1)}}}
    # the pair the residual + SpMV roofline target is stated for: one launch of each
    pair = (bytes_spmv + bytes_res) / ((ms_spmv + ms_res) * 1e-3) / 1e9
    roof["residual_plus_spmv"] = {"GB/s": round(pair, 1), "frac": round(pair / HBM_PEAK_GBS, 4)}
    if ms_vc is not None:
        roof["others"]["vcycle"] = {"us": round(ms_vc * 1e3, 3), "GB/s": round(bytes_vc / ms_vc / 1e6, 1)}
    out = {"metric": "velocity DOF-stages/sec at stated L2 err vs FP64 oracle; mixed/FP64 speedup",
           "value": value, "unit": "velocity DOF-stages/s", "n_gpus": 1, "steps": args.steps,
           "warmup": args.warmup, "ms_per_step": 1e3 * t / args.steps, "higher_is_better": True,
           "scaling": "weak", "vs_baseline": None, "dtype": "f64", "data": "synthetic",
           "config": {"workload": f"2D periodic double shear layer {N}x{N} split mesh ({s.T} triangles), "
                                  f"BDM_{k}+P{k - 1}+P{k} facet, FP64, TVD-RK3 CFL 0.1, PCG rtol {args.rtol:g}",
                      "N": N, "k": k, "N_u": s.n_bdm, "T": s.T, "E": s.E, "precond": args.precond,
                      "extrapolate": args.extrapolate, "order": args.order},
           "pcg_iterations_per_stage": {"mean": float(its.mean()), "max": int(its.max()), "min": int(its.min())},
           "start_rel_residual_geomean": float(np.exp(np.mean(np.log(np.maximum(r0, 1e-300))))),
           "diagnostics_final": d,
           "setup_s": s.setup_seconds,
           "roofline": roof}
    if not args.no_random_order:
        sr = make_solver(N, k, "fp64", args, order="random")
        Ur, _, _ = project_field(sr, double_shear_layer)
        tr, itr = timed_run(sr, Ur, dt, min(args.steps, 50), 1)
        out["random_numbering"] = {"value": sr.n_bdm * 3 * min(args.steps, 50) / tr,
                                   "steps": min(args.steps, 50),
                                   "pcg_iterations_per_stage": float(itr.mean())}
        log("random numbering", out["random_numbering"])
        del sr
    if not args.no_local_spaces:
        out["local_spaces"] = local_spaces(args)
        log("local spaces", out["local_spaces"])
    if not args.no_mixed:
        out["mixed"] = mixed_vs_fp64(args)
        log("mixed", out["mixed"])
    if not args.no_adjoint:
        out["adjoint"] = adjoint_cost(args)
        log("adjoint", out["adjoint"])
    if not args.no_3d:
        out["three_d"] = three_d(args)
        log("3d", out["three_d"])
    if not args.no_cpu_baseline:
        out["cpu_baseline"], (orc, U0_orc, U_orc, dt_s) = cpu_baseline(args)
        log("cpu baseline", out["cpu_baseline"])
        out["accuracy"] = accuracy_vs_oracle(args, orc, U0_orc, U_orc, dt_s)
        log("accuracy", out["accuracy"])
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
