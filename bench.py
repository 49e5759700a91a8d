"""Benchmark: velocity DOF-stages per second of the explicit divergence-free DG hot path.

Workload (default): inviscid double shear layer on the 256x256 periodic split unit square
(131072 triangles), BDM_2 velocity + P1 pressure + P2 facet multipliers, FP64, TVD-RK3 at
CFL 0.1, facet PCG to relative residual 1e-12, 200 steps.  Synthetic data (the closed-form
initial field), projected on the GPU.  One step = one TVD-RK3 step = three passes of the
hot path (residual -> condensation -> facet PCG -> recovery).

Prints one JSON line.  Extra objects: "roofline" (PCG SpMV kernel, timed live with HIP
events), "cpu_baseline" (the CPU oracle on a bounded sample), "accuracy" (FP64 GPU vs the
oracle on a reduced copy of the workload), "mixed" (mixed-precision form, optional).
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
KERNEL_SRC = os.path.join(ROOT, "paper_1808_04669_amd", "csrc", "dfdg_kernels.hip")


def measured_traffic():
    """HBM bytes per k_pcg_spmv launch from the committed counter runs, or None when the
    kernel source changed since they were taken."""
    import hashlib
    try:
        with open(COUNTERS) as f:
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
    ap.add_argument("--extrapolate", type=int, default=2)
    ap.add_argument("--order", default="morton")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-accuracy", action="store_true")
    ap.add_argument("--mixed", action="store_true", help="also time the mixed-precision form")
    ap.add_argument("--cpu-sample-N", type=int, default=64)
    ap.add_argument("--cpu-sample-steps", type=int, default=3)
    ap.add_argument("--copy-calib-mb", type=int, default=0,
                    help="run one plain device copy of this many MB first (counter calibration)")
    return ap.parse_args()


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def project_field(s, field):
    import torch
    pts, _ = s.proj_rule()
    xyz = s._xyz
    x = xyz[:, None, 0, :] + (pts[None, :, 0, None] * (xyz[:, None, 1, :] - xyz[:, None, 0, :])
                              + pts[None, :, 1, None] * (xyz[:, None, 2, :] - xyz[:, None, 0, :]))
    u1, u2 = field(x[..., 0], x[..., 1])  # [T, nq]
    vmax = float(np.sqrt(u1 ** 2 + u2 ** 2).max())
    fq = torch.from_numpy(np.ascontiguousarray(np.stack([u1.T, u2.T]))).to(s.device).reshape(-1)
    U, info = s.project(fq)
    return U, vmax, info


def make_solver(N, k, precision, args, order=None):
    from inputs import periodic_split_square
    from paper_1808_04669_amd import Solver
    xyz, per = periodic_split_square(N, order or args.order)
    s = Solver(xyz, per, k, nu=0.0, precision=precision, cg_rtol=args.rtol, precond=args.precond,
               extrapolate=args.extrapolate, ir_rtol=1e-10, inner_rtol=1e-3)
    s._xyz = xyz
    return s


def timed_run(s, U, dt, steps, warmup):
    import torch
    its = []
    for _ in range(warmup):
        s.rk3_step(U, dt)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        info = s.rk3_step(U, dt)
        its.append(list(info.iterations))
    torch.cuda.synchronize()
    return time.perf_counter() - t0, np.array(its)


def cpu_baseline(args):
    """The oracle (global mixed BDM solve with SuperLU) on the same workload at N = 64."""
    from inputs import double_shear_layer, periodic_split_square
    from oracle import Oracle
    N, k = args.cpu_sample_N, args.k
    xyz, per = periodic_split_square(N)
    orc = Oracle(xyz, per, k, nu=0.0)
    t0 = time.perf_counter()
    orc.factor()
    t_factor = time.perf_counter() - t0
    U = orc.project(double_shear_layer)
    dt = 0.1 / N / k ** 2
    t0 = time.perf_counter()
    for _ in range(args.cpu_sample_steps):
        U = orc.rk3_step(U, dt)
    t = time.perf_counter() - t0
    n_u = orc.space.ndof
    try:
        threads = len(os.sched_getaffinity(0))
    except Exception:
        threads = os.cpu_count()
    return {"value": n_u * 3 * args.cpu_sample_steps / t, "unit": "velocity DOF-stages/s", "cores": 1,
            "kind": "oracle",
            "sample": (f"double shear layer, BDM_{k}, {N}x{N} split mesh ({2 * N * N} triangles, N_u={n_u}), "
                       f"{args.cpu_sample_steps} TVD-RK3 steps timed after a {t_factor:.1f} s SuperLU factorisation "
                       f"(excluded, like the GPU set-up); SuperLU and the NumPy residual run on one core "
                       f"({threads} host threads visible)")}


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
    N, k = args.N, args.k
    s = make_solver(N, k, "fp64", args)
    U, vmax, pinfo = project_field(s, double_shear_layer)
    dt = 0.1 * (1.0 / N) / (k ** 2 * vmax)
    log(f"workload: N={N} k={k} T={s.T} E={s.E} N_u={s.n_bdm} dt={dt:.4e} projection iters={pinfo.iterations}")
    t, its = timed_run(s, U, dt, args.steps, args.warmup)
    value = s.n_bdm * 3 * args.steps / t
    d = s.diagnostics(U)
    log(f"fp64: {t:.3f} s for {args.steps} steps, mean PCG iterations/stage {its.mean():.1f}, diag {d}")

    # roofline of the dominant kernel: the facet SpMV of the PCG, timed live on the ctx stream
    ms_spmv, bytes_spmv = s.time_kernel(0, reps=200)
    ms_upd, bytes_upd = s.time_kernel(1, reps=200)
    ms_res, bytes_res = s.time_kernel(2, reps=50)
    achieved = bytes_spmv / (ms_spmv * 1e-3) / 1e9
    roof = {"kernel": "k_pcg_spmv (facet BSR SpMV + p update + (p,Sp) partials)", "bound": "hbm",
            "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": measured_traffic(),
            "avg_launch_us": round(ms_spmv * 1e3, 3), "bytes_per_launch": bytes_spmv,
            "others": {"k_pcg_update": {"us": round(ms_upd * 1e3, 3), "GB/s": round(bytes_upd / ms_upd / 1e6, 1)},
                       "k_residual": {"us": round(ms_res * 1e3, 3), "GB/s": round(bytes_res / ms_res / 1e6, 1)}}}
    out = {"metric": "velocity DOF-stages/sec at stated L2 err vs FP64 oracle; mixed/FP64 speedup",
           "value": value, "unit": "velocity DOF-stages/s", "n_gpus": 1, "steps": args.steps,
           "warmup": args.warmup, "ms_per_step": 1e3 * t / args.steps, "higher_is_better": True,
           "scaling": "weak", "vs_baseline": None, "dtype": "f64", "data": "synthetic",
           "config": {"workload": f"2D periodic double shear layer {N}x{N} split mesh ({s.T} triangles), "
                                  f"BDM_{k}+P{k - 1}+P{k} facet, FP64, TVD-RK3 CFL 0.1, PCG rtol {args.rtol:g}",
                      "N": N, "k": k, "N_u": s.n_bdm, "T": s.T, "E": s.E, "precond": args.precond,
                      "extrapolate": args.extrapolate, "order": args.order},
           "pcg_iterations_per_stage": {"mean": float(its.mean()), "max": int(its.max()), "min": int(its.min())},
           "diagnostics_final": d,
           "roofline": roof}
    if args.mixed:
        sm = make_solver(N, k, "mixed", args)
        Um, _, _ = project_field(sm, double_shear_layer)
        tm, itm = timed_run(sm, Um, dt, args.steps, args.warmup)
        diff = (Um - U).norm().item() / U.norm().item()
        out["mixed"] = {"value": sm.n_bdm * 3 * args.steps / tm, "speedup_vs_fp64": t / tm,
                        "rel_l2_vs_fp64_gpu": diff, "inner_iterations_mean": float(itm.mean())}
        log(f"mixed: {tm:.3f} s, speedup {t / tm:.3f}, rel diff vs fp64 {diff:.3e}")
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(args)
        log("cpu baseline", out["cpu_baseline"])
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
