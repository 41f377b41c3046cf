#!/usr/bin/env python3
"""Benchmark of the recycling Krylov hot path on one MI355X.

Workload (default "porous256_ir"): the 256^3 (16.8M unknowns) sphere-pack
porous-medium pressure system with 1000:1 conductivity contrast, constant A,
20 right-hand sides b_t from a seeded AR(1) walk.  Each system is solved to a
1e-8 relative true residual by the hybrid method (rGCROT(30,20) with
harmonic-Ritz recycle updates for the first 3 systems, then rBiCGStab with
that recycle space), with the two-level Schwarz-Jacobi preconditioner.

  timed path : FP32 stencil / preconditioner / projections / BiCGStab
               updates inside FP64 iterative refinement (krs_ir_solve)
  comparison : the same hybrid sequence entirely in FP64 (krs_hybrid_solve)

A "step" is one system of the sequence (one whole pass of the hot path).
Inputs are resident in HBM before the timed region.  Prints one JSON line.
"""
import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

PEAK_HBM_GBS = 8000.0
N_SWITCH = 3
M, K = 30, 20


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def build_inputs(n, steps, warmup, dev, torch):
    import workloads as W
    t0 = time.time()
    prob = W.porous_problem(n, seed_cfg=4)
    gen = W.rhs_ar1(prob, warmup + steps, seed_cfg=4)
    bs = [torch.from_numpy(next(gen)).to(dev) for _ in range(warmup + steps)]
    log(f"[bench] inputs: {prob.name} N={prob.n} ({time.time() - t0:.1f}s)")
    return prob, bs


def cpu_baseline(prob, mv_per_solve):
    """Oracle (plain NumPy FP64) time of one preconditioned operator
    application A M^-1 v on the same system, scaled by the matvecs per solve."""
    from oracle import precond, stencil
    v = np.random.default_rng(1).standard_normal(prob.n)
    t0 = time.perf_counter()
    z = precond.schwarz_jacobi(prob.bands, prob.shape, prob.periodic, v, tile=8)
    stencil.apply(prob.bands, prob.shape, prob.periodic, z)
    dt = time.perf_counter() - t0
    return {"value": 1.0 / (dt * mv_per_solve), "unit": "solves/s", "cores": 1, "kind": "oracle",
            "sample": (f"one oracle application of A M^-1 (Schwarz-Jacobi + stencil) on the "
                       f"{prob.shape[0]}^3 system took {dt:.2f} s on 1 host thread; scaled by the "
                       f"GPU run's {mv_per_solve:.0f} operator applications per solve")}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--n", type=int, default=256, help="grid size per axis")
    ap.add_argument("--inner-tol", type=float, default=1e-5)
    ap.add_argument("--no-fp64", action="store_true")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="only run a plain 1 GiB device copy (reference for HBM counters)")
    args = ap.parse_args()
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py measures one GPU: the method here runs on a single MI355X; "
              "--gpus must be 1", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_1501_03358_amd import krs

    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    if args.calibrate_copy:
        # a plain copy of known size: reads 2^30 bytes, writes 2^30 bytes per launch
        a = torch.ones(1 << 28, dtype=torch.float32, device=dev)
        b = torch.empty_like(a)
        for _ in range(5):
            b.copy_(a)
        torch.cuda.synchronize()
        print(json.dumps({"calibration": "copy", "bytes_read": 1 << 30, "bytes_written": 1 << 30,
                          "launches": 5}))
        return
    prob, bs = build_inputs(args.n, args.steps, args.warmup, dev, torch)
    ctx = krs.Context(dev)
    b64 = torch.from_numpy(prob.bands).to(dev)
    b32 = b64.float()
    A64 = krs.Matrix(ctx, prob.shape, prob.periodic, b64)
    A32 = krs.Matrix(ctx, prob.shape, prob.periodic, b32)
    pc = dict(tile=8, overlap=1, local_sweeps=5, omega_local=6 / 7, global_sweeps=1,
              omega_global=6 / 7)
    M32 = krs.Precond(ctx, A32, "schwarz", **pc)
    M64 = krs.Precond(ctx, A64, "schwarz", **pc)
    ws_ir = torch.empty(krs.workspace_size(krs.SOLVER_IR, prob.n, M, K, torch.float32),
                        dtype=torch.uint8, device=dev)
    ws64 = torch.empty(krs.workspace_size(krs.SOLVER_RGCROT, prob.n, M, K, torch.float64),
                       dtype=torch.uint8, device=dev)
    xs = [torch.zeros(prob.n, dtype=torch.float64, device=dev) for _ in range(args.steps)]
    x64s = [torch.zeros(prob.n, dtype=torch.float64, device=dev) for _ in range(args.steps)]

    def ir_step(rec, t, b, x):
        inner = krs.SOLVER_RGCROT if t < N_SWITCH else krs.SOLVER_RBICGSTAB
        o = krs.make_opts(m=M, k=K, tol=1e-8, inner_solver=inner, inner_tol=args.inner_tol,
                          max_matvecs=4000)
        return krs.ir_solve(ctx, A64, A32, M32, rec, b, x, o, ws_ir)

    # warmup: throwaway recycle space, warmup right-hand sides
    wrec = krs.Recycle(ctx, prob.n, K, torch.float32)
    for w in range(args.warmup):
        xw = torch.zeros(prob.n, dtype=torch.float64, device=dev)
        rc, st = ir_step(wrec, w, bs[w], xw)
        log(f"[bench] warmup {w}: status {rc} outer {st.outer} its {st.iterations} "
            f"{st.time_ms:.0f} ms")
    del wrec

    # ---- timed: FP32 inner solves inside FP64 refinement -------------------
    rec32 = krs.Recycle(ctx, prob.n, K, torch.float32)
    krs.timing_reset(ctx)
    krs.timing_enable(ctx, True)
    lat, its, mvs, byt, outer, statuses = [], 0, 0, 0.0, [], []
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for t in range(args.steps):
        s0 = time.perf_counter()
        rc, st = ir_step(rec32, t, bs[args.warmup + t], xs[t])
        lat.append((time.perf_counter() - s0) * 1e3)
        its += st.iterations
        mvs += st.matvecs
        byt += st.bytes_model
        outer.append(st.outer)
        statuses.append(rc)
        log(f"[bench] fp32+ir step {t}: status {rc} outer {st.outer} inner its {st.iterations} "
            f"rel_res {st.rel_res_true:.2e} {lat[-1]:.0f} ms")
    torch.cuda.synchronize()
    t_ir = time.perf_counter() - t0
    krs.timing_enable(ctx, False)
    kt = krs.timing_read(ctx)

    # ---- comparison: the same sequence all in FP64 -------------------------
    fp64 = None
    if not args.no_fp64:
        rec64 = krs.Recycle(ctx, prob.n, K, torch.float64)
        its64 = 0
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        for t in range(args.steps):
            o = krs.make_opts(m=M, k=K, tol=1e-8, max_matvecs=4000)
            rc, st = krs.hybrid_solve(ctx, A64, M64, rec64, t, N_SWITCH, bs[args.warmup + t],
                                      x64s[t], o, ws64)
            its64 += st.iterations
            log(f"[bench] fp64 step {t}: status {rc} its {st.iterations} "
                f"rel_res {st.rel_res_true:.2e} {st.time_ms:.0f} ms")
        torch.cuda.synchronize()
        t64 = time.perf_counter() - t1
        diffs = [float(torch.linalg.vector_norm(xs[t] - x64s[t]) /
                       torch.linalg.vector_norm(x64s[t])) for t in range(args.steps)]
        fp64 = {"solves_per_s": args.steps / t64, "ms_per_step": 1e3 * t64 / args.steps,
                "iterations": its64, "max_rel_diff_fp32ir_vs_fp64": max(diffs)}
        del rec64

    # ---- roofline of the dominant kernel class ------------------------------
    dom = max(kt, key=lambda c: kt[c][1])
    n_l, ms_l, by_l = kt[dom]
    achieved = by_l / (ms_l * 1e-3) / 1e9 if ms_l > 0 else 0.0
    kernels = {c: {"launches": v[0], "ms": round(v[1], 3),
                   "GB_s": round(v[2] / (v[1] * 1e-3) / 1e9, 1) if v[1] > 0 else None}
               for c, v in kt.items() if v[0] > 0}

    cpu = None
    if not args.no_cpu:
        log("[bench] timing the CPU oracle sample ...")
        cpu = cpu_baseline(prob, mvs / args.steps)

    value = args.steps / t_ir
    out = {
        "metric": "solves/s to 1e-8 relative residual (FP32+FP64-IR hybrid rGCROT->rBiCGStab)",
        "value": value, "unit": "solves/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": 1e3 * t_ir / args.steps, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f32+f64", "data": "synthetic",
        "config": {"workload": f"porous{args.n}_ir", "grid": f"{args.n}^3",
                   "unknowns": prob.n, "time_steps": args.steps,
                   "solver": f"hybrid rGCROT({M},{K}) x{N_SWITCH} -> rBiCGStab(k={K})",
                   "precond": "Schwarz-Jacobi 8^3 tiles overlap 1, 5 local + 1 global sweeps",
                   "tol": 1e-8, "inner_tol": args.inner_tol},
        "all_converged": all(s == 0 for s in statuses),
        "iterations_per_s": its / t_ir, "inner_iterations": its,
        "outer_steps": outer,
        "hbm_GB_s_model": byt / t_ir / 1e9,
        "latency_ms": {"p50": float(np.percentile(lat, 50)), "p99": float(np.percentile(lat, 99))},
        "fp64": fp64,
        "speedup_vs_fp64": (value / fp64["solves_per_s"]) if fp64 else None,
        "roofline": {"bound": "hbm", "kernel": dom, "achieved": achieved, "peak": PEAK_HBM_GBS,
                     "unit": "GB/s", "frac": achieved / PEAK_HBM_GBS, "traffic": None,
                     "launches": n_l, "avg_launch_us": 1e3 * ms_l / max(n_l, 1)},
        "kernels": kernels,
        "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
