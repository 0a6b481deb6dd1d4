#!/usr/bin/env python3
"""Benchmark of S_N source iteration with heterogeneous DSA on one MI355X.

Workload (default): 2D 256 x 256 Q1-DG, level-symmetric S8 (40 directions),
16 x 16-cell tiles seeded void / thin / thick 20 / 50 / 30 %, vacuum
boundaries, q = 1 on thin tiles; thick threshold eta = 1 (19,712 thick cells).

A step is one source iteration through the C ABI: transport sweep of all 40
directions, FP64 scalar-flux moment, residual, heterogeneous DSA (SIP on the
thick cells, block-Jacobi PCG to 1e-2) and update.  K steps are timed from
phi = 0 after W warm-up steps.  `value` is the grind time of one whole step in
ns per (cell x direction), FP64 sweep.  Also reported: the same for the FP32
sweep form, sweep-only grind times, time to a 1e-8 residual for both forms,
the FP32 form's error against the FP64 forms and the CPU oracle, the sweep
kernel's roofline fraction (HIP events on the library's stream), the CPU
oracle's time on the same workload, and the 3D 128^3 S12 sweep grind time.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "sweep grind time ns/(cell·dir) + time-to-1e-8, FP32 vs FP64 sweep, 1 MI355X"
# relative tolerance of the thick-region CG inside source iteration: on c2 the
# source-iteration count (45 to 1e-8) is the same for 1e-1 .. 1e-4, so the
# diffusion correction is solved to 1e-2 rather than over-solved
CG_RTOL = 1e-2
HBM_PEAK_GBS = 8000.0


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def sweep_bytes_per_call(nc, ndirs, nn, s):
    """Algorithmic bytes of the sweep kernels of one sweep: psi written once
    (nc*ndirs*nn*s) plus the per-cell inputs read once (nn source values and
    sigma_t in the sweep precision)."""
    return nc * ndirs * nn * s + nc * (nn + 1) * s


def traffic_from_profiles(kernel_key):
    """HBM bytes per launch measured with rocprofv3 counters, if the summary in
    profiles/ was taken on the current kernel source (else None)."""
    from paper_2001_09196_amd.profile_summary import kernel_source_sha
    path = os.path.join(ROOT, "profiles", "traffic.json")
    if not os.path.exists(path):
        return None
    try:
        with open(path) as f:
            data = json.load(f)
        ent = data.get(kernel_key)
        if not ent:
            return None
        if ent.get("kernel_src_sha256") != kernel_source_sha():
            return None
        return float(ent["bytes_per_launch"])
    except Exception:
        return None


COPY_PROBE_BYTES = 1 << 31


def copy_probe():
    """Three copies of a 2 GiB FP64 buffer: each reads and writes exactly
    COPY_PROBE_BYTES, which scales the FETCH_SIZE / WRITE_SIZE counters."""
    import torch
    a = torch.empty(COPY_PROBE_BYTES // 8, dtype=torch.float64, device="cuda")
    a.fill_(1.0)
    b = torch.empty_like(a)
    torch.cuda.synchronize()
    for _ in range(3):
        b.copy_(a)
    torch.cuda.synchronize()
    log(f"copy probe: 3 x {COPY_PROBE_BYTES} bytes")


def sweeps_only(name, prec_name, n):
    """n sweeps of one workload from a seeded random phi (counter passes)."""
    import torch

    import sninputs
    from paper_2001_09196_amd import SN_FP32, SN_FP64, Context, sn_sweep
    dev = torch.device("cuda:0")
    p = sninputs.config(name)
    prec, dt = (SN_FP64, torch.float64) if prec_name == "fp64" else (SN_FP32, torch.float32)
    st = torch.tensor(p.sigma_t, dtype=torch.float64, device=dev)
    ss = torch.tensor(p.sigma_s, dtype=torch.float64, device=dev)
    q = torch.tensor(p.q, dtype=torch.float64, device=dev)
    phi = torch.rand((p.ncells, p.nn), dtype=torch.float64, device=dev, generator=torch.Generator(dev).manual_seed(0))
    with Context(p.dim, p.nx, p.ny, p.nz, p.h, p.omega, p.w, st, ss, eta=p.eta) as ctx:
        psi = torch.empty((p.ncells, p.ndirs, p.nn), dtype=dt, device=dev)
        for _ in range(n):
            sn_sweep(ctx, phi, q, None, False, prec, psi)
        torch.cuda.synchronize()
    log(f"{n} sweeps of {name} in {prec_name}")


def main():
    ap = argparse.ArgumentParser(description=__doc__.splitlines()[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-3d", action="store_true", help="skip the 128^3 S12 sweep measurement")
    ap.add_argument("--copy-probe", action="store_true",
                    help="only run a plain 2 GiB device copy three times (calibrates rocprofv3 byte counters)")
    ap.add_argument("--sweeps-only", type=int, default=0, metavar="N",
                    help="only run N sweeps of --config in --prec (for rocprofv3 counter passes)")
    ap.add_argument("--config", default="c2", help="workload of --sweeps-only (c1..c5)")
    ap.add_argument("--prec", default="fp64", choices=("fp64", "fp32"), help="sweep precision of --sweeps-only")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU only: this build has no multi-GPU path "
              "(the sharding design is described in DESIGN.md)", file=sys.stderr)
        sys.exit(2)
    if args.copy_probe:
        copy_probe()
        return
    if args.sweeps_only:
        sweeps_only(args.config, args.prec, args.sweeps_only)
        return

    import numpy as np
    import torch

    import sninputs
    from paper_2001_09196_amd import (SN_FP32, SN_FP64, Context, sn_source_iterate, sn_sweep)
    from paper_2001_09196_amd.binding import sn_kernel_timing, sn_set_kernel_timing

    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    p = sninputs.config("c2")
    nc, D, nn = p.ncells, p.ndirs, p.nn
    cd = nc * D
    st = torch.tensor(p.sigma_t, dtype=torch.float64, device=dev)
    ss = torch.tensor(p.sigma_s, dtype=torch.float64, device=dev)
    q = torch.tensor(p.q, dtype=torch.float64, device=dev)
    ctx = Context(p.dim, p.nx, p.ny, p.nz, p.h, p.omega, p.w, st, ss, eta=p.eta)
    log(f"c2: {nc} cells x {D} dirs, {ctx.thick_count} thick cells")

    def run_steps(k, prec, timing=False, sweeps_only=True):
        phi = torch.zeros((nc, nn), dtype=torch.float64, device=dev)
        if timing:
            sn_set_kernel_timing(ctx, True, sweeps_only=sweeps_only)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        r = sn_source_iterate(ctx, q, None, phi, tol=0.0, max_it=k, use_dsa=True, prec=prec, cg_rtol=CG_RTOL,
                              cg_maxit=1000)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        kt = None
        if timing:
            kt = sn_kernel_timing(ctx)
            sn_set_kernel_timing(ctx, False)
        return (t1 - t0), r, kt

    # ---- timed steps, FP64 sweep (the reported value) ----
    # HIP events bracket the sweep kernel (the roofline's kernel) in every
    # timed step; each recorded event holds the next kernel back by a few
    # microseconds, so the DSA's share of the step is timed in a separate
    # run of the same steps that does not enter the reported value.
    run_steps(max(args.warmup, 1), SN_FP64)
    dt64, r64, kt64 = run_steps(args.steps, SN_FP64, timing=True)
    _, _, kt64_all = run_steps(args.steps, SN_FP64, timing=True, sweeps_only=False)
    ms_step = dt64 / args.steps * 1e3
    value = ms_step * 1e6 / cd
    log(f"fp64 step: {ms_step:.3f} ms = {value:.5f} ns/(cell*dir); CG its {r64['cg_hist'].tolist()}")
    # ---- same for the FP32 sweep form ----
    run_steps(max(args.warmup, 1), SN_FP32)
    dt32, r32, kt32 = run_steps(args.steps, SN_FP32, timing=True)
    ms_step32 = dt32 / args.steps * 1e3
    log(f"fp32 step: {ms_step32:.3f} ms")

    # ---- sweep-only grind time (event-timed sweep kernels) ----
    phi0 = torch.rand((nc, nn), dtype=torch.float64, device=dev, generator=torch.Generator(dev).manual_seed(0))
    grind = {}
    sweep_ms = {}
    for name, prec, dt in (("fp64", SN_FP64, torch.float64), ("fp32", SN_FP32, torch.float32)):
        psi = torch.empty((nc, D, nn), dtype=dt, device=dev)
        for _ in range(3):
            sn_sweep(ctx, phi0, q, None, False, prec, psi)
        reps = 20
        sn_set_kernel_timing(ctx, True)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(reps):
            sn_sweep(ctx, phi0, q, None, False, prec, psi)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        kt = sn_kernel_timing(ctx)
        sn_set_kernel_timing(ctx, False)
        sweep_ms[name] = kt["sweep_ms"] / kt["sweep_count"]
        grind[name] = {"sweep_kernel_ns": sweep_ms[name] * 1e6 / cd,
                       "sn_sweep_call_ns": (t1 - t0) / reps * 1e9 / cd}
        del psi
        log(f"sweep {name}: kernel {sweep_ms[name]*1e3:.1f} us, grind {grind[name]['sweep_kernel_ns']:.5f} ns")

    # ---- time to 1e-8 ----
    def solve(prec, tol=1e-8):
        best = None
        for _ in range(3):
            phi = torch.zeros((nc, nn), dtype=torch.float64, device=dev)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            r = sn_source_iterate(ctx, q, None, phi, tol=tol, max_it=2000, use_dsa=True, prec=prec, cg_rtol=CG_RTOL,
                                  cg_maxit=1000)
            torch.cuda.synchronize()
            t = time.perf_counter() - t0
            if best is None or t < best[0]:
                best = (t, r, phi.clone())
        return best

    # ---- thick-region preconditioners: block Jacobi against multigrid ----
    def dsa_compare(precond, k=6):
        phi = torch.zeros((nc, nn), dtype=torch.float64, device=dev)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        sn_source_iterate(ctx, q, None, phi, tol=0.0, max_it=1, use_dsa=True, prec=SN_FP64, cg_rtol=CG_RTOL,
                          cg_maxit=1000, precond=precond)     # first use builds the hierarchy
        torch.cuda.synchronize()
        first = time.perf_counter() - t0
        phi.zero_()
        sn_set_kernel_timing(ctx, True)
        r = sn_source_iterate(ctx, q, None, phi, tol=0.0, max_it=k, use_dsa=True, prec=SN_FP64, cg_rtol=CG_RTOL,
                              cg_maxit=1000, precond=precond)
        kt = sn_kernel_timing(ctx)
        sn_set_kernel_timing(ctx, False)
        return {"dsa_ms": kt["dsa_ms"] / max(kt["dsa_count"], 1), "cg_iters": r["cg_hist"].tolist(),
                "first_call_s": first}

    precond_cmp = {"block_jacobi": dsa_compare(0), "multigrid": dsa_compare(1)}
    log(f"c2 DSA: block Jacobi {precond_cmp['block_jacobi']['dsa_ms']:.3f} ms "
        f"{precond_cmp['block_jacobi']['cg_iters']}, multigrid {precond_cmp['multigrid']['dsa_ms']:.3f} ms "
        f"{precond_cmp['multigrid']['cg_iters']}")

    t64, s64, phi64 = solve(SN_FP64)
    t32, s32, phi32 = solve(SN_FP32)
    err32_vs64 = float(torch.linalg.norm(phi32 - phi64) / torch.linalg.norm(phi64))
    log(f"time to 1e-8: fp64 {t64*1e3:.1f} ms ({s64['iters']} it, rc {s64['rc']}), "
        f"fp32 {t32*1e3:.1f} ms ({s32['iters']} it, rc {s32['rc']}), fp32 vs fp64 {err32_vs64:.2e}")

    # ---- roofline of the dominant kernel (per step) ----
    sweep_per_step = kt64["sweep_ms"] / max(kt64["sweep_count"], 1)
    dsa_per_step = kt64_all["dsa_ms"] / max(kt64_all["dsa_count"], 1)
    bytes_sweep = sweep_bytes_per_call(nc, D, nn, 8)
    roofline = {"kernel": "sweep2d_kernel<double> (one launch per sweep)", "bound": "hbm",
                "achieved": bytes_sweep / (sweep_per_step * 1e-3) / 1e9, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "algorithmic_bytes_per_launch": bytes_sweep, "avg_launch_ms": sweep_per_step,
                "traffic": traffic_from_profiles("sweep2d_fp64_c2")}
    roofline["frac"] = roofline["achieved"] / roofline["peak"]
    log(f"per step: sweep {sweep_per_step:.3f} ms, dsa {dsa_per_step:.3f} ms of {ms_step:.3f} ms")

    out = {
        "metric": METRIC,
        "value": value,
        "unit": "ns/(cell*dir)",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_step,
        "higher_is_better": False,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": "c2: 2D 256x256 Q1 upwind-DG, S8 (40 dirs), seeded 16x16 tiles void/thin/thick "
                               "20/50/30%, vacuum; one step = sweep + FP64 moment + residual + thick-only DSA "
                               "(SIP, block-Jacobi PCG rtol 1e-2) + update",
                   "cells": nc, "dirs": D, "thick_cells": ctx.thick_count, "eta": p.eta},
        "roofline": roofline,
        "step_breakdown_ms": {"sweep": sweep_per_step, "dsa": dsa_per_step,
                              "cg_iters_per_dsa": float(np.mean(r64["cg_hist"]))},
        "fp32_form": {"ms_per_step": ms_step32, "value": ms_step32 * 1e6 / cd, "dtype": "f32 sweep, f64 moment/DSA",
                      "speedup_vs_fp64_step": ms_step / ms_step32},
        "sweep_grind_ns": grind,
        "time_to_1e-8": {"fp64": {"seconds": t64, "iters": s64["iters"], "rc": s64["rc"],
                                  "cg_iters_total": int(np.sum(s64["cg_hist"]))},
                         "fp32": {"seconds": t32, "iters": s32["iters"], "rc": s32["rc"],
                                  "cg_iters_total": int(np.sum(s32["cg_hist"]))},
                         "fp32_speedup": t64 / t32, "fp32_vs_fp64_rel_l2": err32_vs64},
        "dsa_preconditioners_c2": precond_cmp,
    }
    del ctx

    # ---- pure-scatterer thick tiles (sigma_a = 0): where multigrid matters ----
    try:
        out["dsa_preconditioners_c2s"] = pure_scatterer_compare(log)
    except Exception as e:  # report, do not hide
        out["dsa_preconditioners_c2s"] = {"error": repr(e)}

    # ---- 3D: 128^3, S12 (168 dirs) sweep grind time and HBM fraction ----
    if not args.no_3d:
        try:
            out["sweep3d_c5"] = bench_3d(log)
        except Exception as e:  # report, do not hide
            out["sweep3d_c5"] = {"error": repr(e)}

    # ---- 3D solves to 1e-8 in both forms (C3, C5) ----
    if not args.no_3d:
        try:
            out["time_to_1e-8_3d"] = bench_to_tolerance_3d(log)
        except Exception as e:  # report, do not hide
            out["time_to_1e-8_3d"] = {"error": repr(e)}

    # ---- CPU oracle on the same workload (bounded: one solve to 1e-8) ----
    if not args.no_cpu_baseline:
        import oracle
        nth = oracle.num_threads()
        t0 = time.perf_counter()
        ro = oracle.source_iterate(p, tol=1e-8, max_it=2000, use_dsa=True, cg_rtol=CG_RTOL)
        tcpu = time.perf_counter() - t0
        its = ro["iters"]
        ref = torch.tensor(ro["phi"], dtype=torch.float64, device=dev)
        e64 = float(torch.linalg.norm(phi64 - ref) / torch.linalg.norm(ref))
        e32 = float(torch.linalg.norm(phi32 - ref) / torch.linalg.norm(ref))
        out["cpu_baseline"] = {"value": tcpu / its * 1e9 / cd, "unit": "ns/(cell*dir)", "cores": nth,
                               "kind": "oracle",
                               "sample": f"c2 solve to 1e-8 from phi=0: {its} source iterations "
                                         f"(+1 sweep for ||b||) in {tcpu:.2f} s; value = time per iteration",
                               "time_to_1e-8_s": tcpu}
        out["time_to_1e-8"]["fp64_vs_oracle_rel_l2"] = e64
        out["time_to_1e-8"]["fp32_vs_oracle_rel_l2"] = e32
        log(f"oracle: {tcpu:.2f} s for {its} iterations on {nth} threads; gpu fp64 err {e64:.2e}, fp32 {e32:.2e}")
    print(json.dumps(out), flush=True)


def pure_scatterer_compare(log):
    """c2s (c2 with sigma_s = sigma_t in the thick tiles): FP64 source iteration
    to 1e-8 with each thick-region preconditioner."""
    import torch

    import sninputs
    from paper_2001_09196_amd import SN_FP64, Context, sn_source_iterate
    dev = torch.device("cuda:0")
    p = sninputs.config("c2s")
    st = torch.tensor(p.sigma_t, dtype=torch.float64, device=dev)
    ss = torch.tensor(p.sigma_s, dtype=torch.float64, device=dev)
    q = torch.tensor(p.q, dtype=torch.float64, device=dev)
    res = {"workload": "c2s: c2 with pure-scatterer thick tiles (sigma_t = sigma_s = 1e3)"}
    with Context(p.dim, p.nx, p.ny, p.nz, p.h, p.omega, p.w, st, ss, eta=p.eta) as ctx:
        for name, pc in (("block_jacobi", 0), ("multigrid", 1)):
            phi = torch.zeros((p.ncells, p.nn), dtype=torch.float64, device=dev)
            sn_source_iterate(ctx, q, None, phi, tol=0.0, max_it=1, use_dsa=True, prec=SN_FP64, cg_rtol=CG_RTOL,
                              cg_maxit=5000, precond=pc)      # builds the hierarchy on first use
            phi.zero_()
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            r = sn_source_iterate(ctx, q, None, phi, tol=1e-8, max_it=2000, use_dsa=True, prec=SN_FP64,
                                  cg_rtol=CG_RTOL, cg_maxit=5000, precond=pc)
            torch.cuda.synchronize()
            t = time.perf_counter() - t0
            res[name] = {"time_to_1e-8_s": t, "iters": r["iters"], "rc": r["rc"],
                         "cg_iters_total": int(r["cg_hist"].sum()),
                         "cg_iters_mean": float(r["cg_hist"].mean())}
            log(f"c2s {name}: {t*1e3:.1f} ms to 1e-8, {r['iters']} SI iterations, "
                f"CG {int(r['cg_hist'].sum())} total")
    return res


def bench_3d(log):
    import torch

    import sninputs
    from paper_2001_09196_amd import SN_FP32, SN_FP64, Context, sn_sweep
    from paper_2001_09196_amd.binding import sn_kernel_timing, sn_set_kernel_timing
    dev = torch.device("cuda:0")
    p = sninputs.config("c5")
    nc, D, nn = p.ncells, p.ndirs, p.nn
    cd = nc * D
    st = torch.tensor(p.sigma_t, dtype=torch.float64, device=dev)
    ss = torch.tensor(p.sigma_s, dtype=torch.float64, device=dev)
    q = torch.tensor(p.q, dtype=torch.float64, device=dev)
    phi0 = torch.rand((nc, nn), dtype=torch.float64, device=dev, generator=torch.Generator(dev).manual_seed(0))
    res = {"workload": "c5: 3D 128^3 Q1-DG, S12 (168 dirs), seeded 16^3 tiles", "cells": nc, "dirs": D}
    with Context(p.dim, p.nx, p.ny, p.nz, p.h, p.omega, p.w, st, ss, eta=p.eta) as ctx:
        for name, prec, dt, s in (("fp32", SN_FP32, torch.float32, 4), ("fp64", SN_FP64, torch.float64, 8)):
            psi = torch.empty((nc, D, nn), dtype=dt, device=dev)
            sn_sweep(ctx, phi0, q, None, False, prec, psi)
            reps = 5
            sn_set_kernel_timing(ctx, True)
            for _ in range(reps):
                sn_sweep(ctx, phi0, q, None, False, prec, psi)
            kt = sn_kernel_timing(ctx)
            sn_set_kernel_timing(ctx, False)
            ms = kt["sweep_ms"] / kt["sweep_count"]
            b = sweep_bytes_per_call(nc, D, nn, s)
            res[name] = {"sweep_ms": ms, "grind_ns": ms * 1e6 / cd, "algorithmic_bytes": b,
                         "achieved_GBs": b / (ms * 1e-3) / 1e9, "hbm_frac": b / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS,
                         "traffic": traffic_from_profiles(f"sweep3d_{name}_c5")}
            log(f"c5 sweep {name}: {ms:.3f} ms, grind {ms*1e6/cd:.5f} ns, {res[name]['achieved_GBs']:.0f} GB/s")
            del psi
            torch.cuda.empty_cache()
        # source iterations: fused sweep + moment (psi never stored) and DSA
        from paper_2001_09196_amd import sn_source_iterate
        for pc_name, pc in (("block_jacobi", 0), ("multigrid", 1)):
            phi = torch.zeros((nc, nn), dtype=torch.float64, device=dev)
            t0 = time.perf_counter()
            sn_source_iterate(ctx, q, None, phi, tol=0.0, max_it=1, use_dsa=True, prec=SN_FP64, cg_rtol=CG_RTOL,
                              cg_maxit=2000, precond=pc)
            torch.cuda.synchronize()
            first = time.perf_counter() - t0
            phi.zero_()
            sn_set_kernel_timing(ctx, True)
            r = sn_source_iterate(ctx, q, None, phi, tol=0.0, max_it=4, use_dsa=True, prec=SN_FP64, cg_rtol=CG_RTOL,
                                  cg_maxit=2000, precond=pc)
            kt = sn_kernel_timing(ctx)
            sn_set_kernel_timing(ctx, False)
            res.setdefault("dsa_preconditioners", {})[pc_name] = {
                "dsa_ms": kt["dsa_ms"] / max(kt["dsa_count"], 1), "cg_iters": r["cg_hist"].tolist(),
                "first_call_s": first}
            log(f"c5 DSA {pc_name}: {res['dsa_preconditioners'][pc_name]['dsa_ms']:.3f} ms, CG {r['cg_hist'].tolist()}, "
                f"first call {first:.2f} s")
            del phi
        for name, prec in (("fp32", SN_FP32), ("fp64", SN_FP64)):
            k = 4
            phi = torch.zeros((nc, nn), dtype=torch.float64, device=dev)
            sn_source_iterate(ctx, q, None, phi, tol=0.0, max_it=1, use_dsa=True, prec=prec, cg_rtol=CG_RTOL,
                              cg_maxit=2000)
            phi.zero_()
            sn_set_kernel_timing(ctx, True)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            r = sn_source_iterate(ctx, q, None, phi, tol=0.0, max_it=k, use_dsa=True, prec=prec, cg_rtol=CG_RTOL,
                                  cg_maxit=2000)
            torch.cuda.synchronize()
            t1 = time.perf_counter()
            kt = sn_kernel_timing(ctx)
            sn_set_kernel_timing(ctx, False)
            fused = kt["sweep_ms"] / max(kt["sweep_count"], 1)
            res[name]["si_step_ms"] = (t1 - t0) / k * 1e3
            res[name]["fused_sweep_moment_ms"] = fused
            res[name]["fused_grind_ns"] = fused * 1e6 / cd
            res[name]["dsa_ms"] = kt["dsa_ms"] / max(kt["dsa_count"], 1)
            res[name]["cg_iters"] = r["cg_hist"].tolist()
            log(f"c5 SI {name}: step {res[name]['si_step_ms']:.2f} ms, fused sweep+moment {fused:.3f} ms, "
                f"dsa {res[name]['dsa_ms']:.3f} ms, CG {r['cg_hist'].tolist()}")
            del phi
    return res


def bench_to_tolerance_3d(log):
    """C3 and C5 solved to 1e-8 from phi = 0 in both forms (one timed solve
    each, after a first call that builds the context's workspace): seconds,
    source iterations, FP32 form against FP64, and for C3 both against the
    oracle's converged flux at its stored sample points."""
    import numpy as np
    import torch

    import sninputs
    from paper_2001_09196_amd import SN_FP32, SN_FP64, Context, sn_source_iterate
    dev = torch.device("cuda:0")
    gold_path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "tests", "golden", "c3_phi.json")
    out = {}
    for name in ("c3", "c5"):
        p = sninputs.config(name)
        nc, nn = p.ncells, p.nn
        st = torch.tensor(p.sigma_t, dtype=torch.float64, device=dev)
        ss = torch.tensor(p.sigma_s, dtype=torch.float64, device=dev)
        q = torch.tensor(p.q, dtype=torch.float64, device=dev)
        res = {"workload": f"{name}: {p.nx}x{p.ny}x{p.nz}, {p.ndirs} dirs", "cg_rtol": CG_RTOL}
        phis = {}
        with Context(p.dim, p.nx, p.ny, p.nz, p.h, p.omega, p.w, st, ss, eta=p.eta) as ctx:
            for form, prec in (("fp64", SN_FP64), ("fp32", SN_FP32)):
                phi = torch.zeros((nc, nn), dtype=torch.float64, device=dev)
                sn_source_iterate(ctx, q, None, phi, tol=0.0, max_it=1, use_dsa=True, prec=prec, cg_rtol=CG_RTOL,
                                  cg_maxit=2000)
                phi.zero_()
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                r = sn_source_iterate(ctx, q, None, phi, tol=1e-8, max_it=2000, use_dsa=True, prec=prec,
                                      cg_rtol=CG_RTOL, cg_maxit=2000)
                torch.cuda.synchronize()
                res[form] = {"seconds": time.perf_counter() - t0, "iters": r["iters"], "rc": r["rc"],
                             "cg_iters_total": int(r["cg_hist"][:r["iters"]].sum())}
                phis[form] = phi
                log(f"{name} to 1e-8 {form}: {res[form]['seconds']:.3f} s, {r['iters']} iterations")
        res["fp32_speedup"] = res["fp64"]["seconds"] / res["fp32"]["seconds"]
        res["fp32_vs_fp64_rel_l2"] = float(torch.linalg.norm(phis["fp32"] - phis["fp64"]) /
                                           torch.linalg.norm(phis["fp64"]))
        if name == "c3" and os.path.exists(gold_path):
            gold = json.load(open(gold_path))
            res["oracle_samples"] = (f"{len(gold['sample_index'])} values of the oracle's flux solved to residual "
                                     f"{gold['res_last']:.1e}; the gap below is the 1e-8 stop of these solves")
            idx = torch.tensor(gold["sample_index"], dtype=torch.long, device=dev)
            ref = torch.tensor(gold["sample_value"], dtype=torch.float64, device=dev)
            for form in ("fp64", "fp32"):
                got = phis[form].reshape(-1)[idx]
                res[form]["vs_oracle_samples_rel_l2"] = float(torch.linalg.norm(got - ref) / torch.linalg.norm(ref))
        out[name] = res
        del phis
        torch.cuda.empty_cache()
    return out


if __name__ == "__main__":
    main()
