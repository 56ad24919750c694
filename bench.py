#!/usr/bin/env python3
"""Benchmark of the rotating-GPE ground-state solver on one MI355X.

Workload: 2-D 512^2 grid on [-16, 16]^2, V = (x^2 + y^2)/2, beta = 1000, Omega = 0.9, seeded
vortex-seed start (seed 103), PCG with the symmetric combined preconditioner, stop at
||H phi - lambda phi||_inf <= 1e-8.  One step = one full solve from the resident start (every
stage of the hot path: transforms, H apply, preconditioner, reductions, direction, line search,
retraction, convergence control, precision switch).

Printed (one JSON line on stdout): the mixed FP32/FP64 time-to-1e-8 as `value`, beside the FP64
time-to-1e-8, H_phi applies/s, PCG iterations/s, the dominant kernel's roofline figure measured
with HIP events, and the CPU oracle timed on the host (bounded sample, extrapolated).
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "time-to-1e-8 residual + H_phi applies/s, 2D 512^2 Omega=0.9: mixed vs FP64"
HBM_PEAK_GBS = 8000.0


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def time_solves(torch, plan, V, starts, **opts):
    reps = []
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for phi in starts:
        reps.append(plan.pcg_solve(V, phi, **opts))
    torch.cuda.synchronize()
    return time.perf_counter() - t0, reps


def applies_per_s(torch, plan, phi, V, reps, batched=False):
    out = torch.empty_like(phi)
    f = plan.apply_H_batched if batched else plan.apply_H
    for _ in range(3):
        f(phi, V, out)
    s = torch.cuda.current_stream()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(s)
    for _ in range(reps):
        f(phi, V, out)
    e1.record(s)
    e1.synchronize()
    sec = e0.elapsed_time(e1) / 1e3
    count = reps * (phi.shape[0] if batched else 1)
    return count / sec, sec / reps


def cpu_baseline(prob, V, phi0, iters, gpu_fp64_iters):
    """The FP64 oracle, as it stands, on the same workload for a bounded number of iterations."""
    from oracle import gpe_oracle as O
    try:
        from threadpoolctl import threadpool_limits
        ctx = threadpool_limits(1)
    except Exception:  # pragma: no cover
        ctx = None
    t0 = time.perf_counter()
    res = O.pcg(prob, V, phi0, tol_res=1e-8, max_iter=iters)
    sec = time.perf_counter() - t0
    if ctx is not None:
        ctx.unregister() if hasattr(ctx, "unregister") else None
    done = max(1, res.iters)
    it_s = done / sec
    return {
        "value": gpu_fp64_iters / it_s,
        "unit": "s",
        "cores": 1,
        "kind": "oracle",
        "sample": (f"numpy FP64 oracle, PCG_C on the same 512^2 workload, first {done} iterations "
                   f"({sec:.1f} s, {it_s:.2f} it/s, 1 thread), extrapolated to the GPU FP64 solve's "
                   f"{gpu_fp64_iters} iterations to 1e-8"),
        "iters_per_s": it_s,
    }


def main():
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--cpu-iters", type=int, default=40)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--profile-iters", type=int, default=30)
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only (asked for --gpus {args.gpus}); the solver is a single-GPU "
              "path and nothing here uses a second device", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    from gpe_inputs import workload_2d
    from paper_1611_02045_amd import gpe

    if not torch.cuda.is_available():
        log("no GPU available")
        sys.exit(1)
    gpe.lib()
    prob, V_np, phi0_np = workload_2d(512)
    plan = gpe.Plan.from_problem(prob, "f64")
    V = torch.from_numpy(V_np).to("cuda")
    phi0 = torch.from_numpy(phi0_np).to("cuda")
    tol = 1e-8
    mixed = dict(tol=tol, precision="mixed", max_iter=50000)
    fp64 = dict(tol=tol, precision="fp64", max_iter=50000)

    log(f"[bench] warmup {args.warmup} mixed + 1 fp64 solve(s)")
    for _ in range(args.warmup):
        plan.pcg_solve(V, phi0.clone(), **mixed)
    plan.pcg_solve(V, phi0.clone(), **fp64)

    # timed region: exactly K mixed-precision solves, starts resident in HBM
    starts = [phi0.clone() for _ in range(args.steps)]
    torch.cuda.synchronize()
    log(f"[bench] timing {args.steps} mixed solves")
    sec_mixed, reps_mixed = time_solves(torch, plan, V, starts, **mixed)
    t_mixed = sec_mixed / args.steps
    log(f"[bench] mixed: {t_mixed:.4f} s/solve, iters {[r['iters'] for r in reps_mixed]}")

    starts = [phi0.clone() for _ in range(args.steps)]
    sec_fp64, reps_fp64 = time_solves(torch, plan, V, starts, **fp64)
    t_fp64 = sec_fp64 / args.steps
    log(f"[bench] fp64:  {t_fp64:.4f} s/solve, iters {[r['iters'] for r in reps_fp64]}")

    # H_phi applies/s (single field and a batch of 32 fields, FP64 and FP32)
    log("[bench] H applies")
    plan32 = gpe.Plan.from_problem(prob, "f32")
    V32, phi32 = V.float(), phi0.to(torch.complex64)
    ap64, _ = applies_per_s(torch, plan, phi0, V, 400)
    ap32, _ = applies_per_s(torch, plan32, phi32, V32, 400)
    batch = 32
    bphi64 = phi0.unsqueeze(0).repeat(batch, 1, 1).contiguous()
    bphi32 = phi32.unsqueeze(0).repeat(batch, 1, 1).contiguous()
    apb64, tb64 = applies_per_s(torch, plan, bphi64, V, 20, batched=True)
    apb32, tb32 = applies_per_s(torch, plan32, bphi32, V32, 20, batched=True)

    # per-kernel event timings of the solver iteration (FP32 fields: the bulk of a mixed solve)
    log("[bench] kernel profile")
    prof32 = plan.profile(V, phi0, iters=args.profile_iters, precision="mixed")
    prof64 = plan.profile(V, phi0, iters=args.profile_iters, precision="fp64")
    n32 = sum(r["iters_fp32"] for r in reps_mixed) / len(reps_mixed)
    n64 = sum(r["iters"] - r["iters_fp32"] for r in reps_mixed) / len(reps_mixed)
    weight = {"fp32": n32, "fp64": n64}
    totals = []
    for tag, prof in (("fp32", prof32), ("fp64", prof64)):
        for name, ms, by in prof:
            totals.append((weight[tag] * ms, tag, name, ms, by))
    totals.sort(reverse=True)
    _, tag, name, ms, by = totals[0]
    achieved = by / (ms * 1e-3) / 1e9
    roofline = {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": achieved / HBM_PEAK_GBS, "traffic": None,
                "kernel": f"{name} ({tag})", "bytes_per_launch": by, "avg_ms": ms}

    cpu = None
    if not args.no_cpu:
        log(f"[bench] CPU oracle sample ({args.cpu_iters} iterations)")
        cpu = cpu_baseline(prob, V_np, phi0_np, args.cpu_iters, int(reps_fp64[0]["iters"]))

    r0 = reps_mixed[0]
    out = {
        "metric": METRIC,
        "value": t_mixed,
        "unit": "s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": t_mixed * 1e3,
        "higher_is_better": False,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "mixed fp32/fp64 (fp32 fields, fp64 scalars, fp64 refinement)",
        "data": "synthetic (seeded vortex-seed start, analytic trap)",
        "config": {"workload": "2D 512^2 rotating GPE on [-16,16]^2, V=(x^2+y^2)/2, beta=1000, Omega=0.9, "
                               "PCG + symmetric combined preconditioner, ||r||_inf <= 1e-8",
                   "grid": [512, 512], "beta": 1000.0, "omega": 0.9, "tol": tol, "seed": 103},
        "time_to_tol_fp64_s": t_fp64,
        "speedup_mixed_vs_fp64": t_fp64 / t_mixed,
        "iters_mixed": {"total": r0["iters"], "fp32": r0["iters_fp32"]},
        "iters_fp64": reps_fp64[0]["iters"],
        "pcg_iters_per_s": {"mixed": r0["iters"] / t_mixed, "fp64": reps_fp64[0]["iters"] / t_fp64},
        "h_applies_per_s": {"fp64": ap64, "fp32": ap32, "fp64_batch32": apb64, "fp32_batch32": apb32},
        "h_apply_batch32_hbm_gbs": {
            "fp64": 11 * 8 * 512 * 512 * batch / tb64 / 1e9, "fp32": 11 * 4 * 512 * 512 * batch / tb32 / 1e9},
        "final": {"E_mixed": r0["E"], "res_mixed": r0["res_inf"], "E_fp64": reps_fp64[0]["E"],
                  "res_fp64": reps_fp64[0]["res_inf"]},
        "kernels": {"fp32": [{"name": n, "avg_ms": m, "bytes": b, "GB_s": b / (m * 1e-3) / 1e9} for n, m, b in prof32],
                    "fp64": [{"name": n, "avg_ms": m, "bytes": b, "GB_s": b / (m * 1e-3) / 1e9} for n, m, b in prof64]},
        "roofline": roofline,
        "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
