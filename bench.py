#!/usr/bin/env python3
"""Benchmark of the rotating-GPE ground-state solver on one MI355X.

Workload: 2-D 512^2 grid on [-16, 16]^2, V = (x^2 + y^2)/2, beta = 1000, Omega = 0.9, four seeded
vortex-seed starts (seeds 103, 107, 109, 113), PCG with the symmetric combined preconditioner, stop
at ||H phi - lambda phi||_inf <= 1e-8.  One step = one full solve of each of the four starts from
its resident copy (every stage of the hot path: transforms, H apply, preconditioner, reductions,
direction, line search, retraction, convergence control, precision switch).  At Omega = 0.9 the
iteration count to 1e-8 depends strongly on the start (soft vortex-lattice modes), hence several.

Printed (one JSON line on stdout): the mixed FP32/FP64 time-to-1e-8 per solve as `value`, beside
the FP64 time-to-1e-8, the four starts solved together as one batched solve (mixed and FP64),
H_phi applies/s, PCG iterations/s, the dominant kernel's roofline figure (kernel-only HIP event
timings), and the CPU oracle timed on the host (bounded sample, extrapolated).
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
                   f"({sec:.1f} s, {it_s:.2f} it/s, 1 thread), extrapolated to the GPU FP64 solves' "
                   f"mean {gpu_fp64_iters:.0f} iterations to 1e-8"),
        "iters_per_s": it_s,
    }


def mean(xs):
    return float(sum(xs)) / len(xs)


def kernel_rows(prof):
    return [{"name": n, "avg_ms": m, "bytes": b, "GB_s": b / (m * 1e-3) / 1e9} for n, m, b in prof]


def source_digest():
    """Digest of the HIP sources: counter figures taken from an older build no longer apply."""
    import glob
    import hashlib
    h = hashlib.sha256()
    for f in sorted(glob.glob(os.path.join(ROOT, "paper_1611_02045_amd", "csrc", "*"))):
        with open(f, "rb") as fh:
            h.update(os.path.basename(f).encode())
            h.update(fh.read())
    return h.hexdigest()[:16]


def measured_traffic(kernel):
    """HBM bytes per launch of `kernel` from the committed counter summary, if it was taken from
    these exact sources (else None)."""
    path = os.path.join(ROOT, "profiles", "hbm_traffic_2d_512.md")
    try:
        with open(path) as fh:
            for line in fh:
                if line.startswith("traffic-json:"):
                    rec = json.loads(line.split(":", 1)[1])
                    if rec.get("source_digest") == source_digest() and kernel in rec.get("kernels", {}):
                        return rec["kernels"][kernel]["hbm_bytes_per_launch"]
    except OSError:
        pass
    return None


def main():
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=2)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--cpu-iters", type=int, default=40)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--profile-iters", type=int, default=30)
    ap.add_argument("--batched", action="store_true",
                    help="also solve the four starts as one batched solve (mixed and FP64)")
    ap.add_argument("--profile-only", action="store_true",
                    help="only the per-kernel profile of the iteration and a 512 MiB copy (for counter runs)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only (asked for --gpus {args.gpus}); the solver is a single-GPU "
              "path and nothing here uses a second device", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    from gpe_inputs import SEEDS_2D_512_SET, workload_2d_set
    from paper_1611_02045_amd import gpe

    if not torch.cuda.is_available():
        log("no GPU available")
        sys.exit(1)
    gpe.lib()
    prob, V_np, starts_np = workload_2d_set(512)
    phi0_np = starts_np[0]
    plan = gpe.Plan.from_problem(prob, "f64")
    V = torch.from_numpy(V_np).to("cuda")
    starts0 = [torch.from_numpy(x).to("cuda") for x in starts_np]
    phi0 = starts0[0]
    tol = 1e-8
    mixed = dict(tol=tol, precision="mixed", max_iter=200000)
    fp64 = dict(tol=tol, precision="fp64", max_iter=200000)

    def step_inputs():
        return [x.clone() for x in starts0]

    if args.profile_only:
        prof32 = plan.profile(V, phi0, iters=args.profile_iters, precision="mixed")
        prof64 = plan.profile(V, phi0, iters=args.profile_iters, precision="fp64")
        # a plain copy of known size, to scale the HBM byte counters
        a = torch.empty(512 << 20, dtype=torch.uint8, device="cuda").fill_(1)
        b = torch.empty_like(a)
        b.copy_(a)
        torch.cuda.synchronize()
        print(json.dumps({"profile_only": True, "copy_bytes": a.numel(),
                          "kernels": {"fp32": kernel_rows(prof32), "fp64": kernel_rows(prof64)}}), flush=True)
        return

    log(f"[bench] warmup {args.warmup} step(s) of {len(starts0)} mixed solves + 1 fp64 solve")
    for _ in range(args.warmup):
        time_solves(torch, plan, V, step_inputs(), **mixed)
    plan.pcg_solve(V, phi0.clone(), **fp64)

    # timed region: exactly K steps, each the mixed-precision solves of every start, starts resident in HBM
    inputs = [step_inputs() for _ in range(args.steps)]
    torch.cuda.synchronize()
    log(f"[bench] timing {args.steps} step(s) of mixed solves")
    sec_mixed, reps_mixed = time_solves(torch, plan, V, [x for st in inputs for x in st], **mixed)
    n_solves = len(reps_mixed)
    t_mixed = sec_mixed / n_solves
    log(f"[bench] mixed: {t_mixed:.4f} s/solve, iters {[r['iters'] for r in reps_mixed]}")

    inputs = [step_inputs() for _ in range(args.steps)]
    sec_fp64, reps_fp64 = time_solves(torch, plan, V, [x for st in inputs for x in st], **fp64)
    t_fp64 = sec_fp64 / len(reps_fp64)
    log(f"[bench] fp64:  {t_fp64:.4f} s/solve, iters {[r['iters'] for r in reps_fp64]}")

    # the same starts as one batched solve (per-instance convergence masks)
    batched = None if not args.batched else {}
    for tag, opts in ((("mixed", mixed), ("fp64", fp64)) if args.batched else ()):
        phis = step_inputs()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        _, reps = gpe.pcg_solve_batched([prob] * len(phis), [V] * len(phis), phis, "f64", **opts)
        torch.cuda.synchronize()
        batched[tag] = {"seconds": time.perf_counter() - t0, "iters": [r["iters"] for r in reps],
                        "status": [r["status"] for r in reps]}
        log(f"[bench] batched {tag}: {batched[tag]['seconds']:.3f} s, iters {batched[tag]['iters']}")

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
    kname = f"{name} ({tag})"
    roofline = {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": achieved / HBM_PEAK_GBS, "traffic": measured_traffic(kname),
                "kernel": kname, "bytes_per_launch": by, "avg_ms": ms,
                "timing": "HIP start/stop events recorded by each launch (kernel execution only)"}

    it_fp64 = [r["iters"] for r in reps_fp64]
    cpu = None
    if not args.no_cpu:
        log(f"[bench] CPU oracle sample ({args.cpu_iters} iterations)")
        cpu = cpu_baseline(prob, V_np, phi0_np, args.cpu_iters, mean(it_fp64))

    it_mixed = [r["iters"] for r in reps_mixed]
    it_fp64 = [r["iters"] for r in reps_fp64]
    out = {
        "metric": METRIC,
        "value": t_mixed,
        "unit": "s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": sec_mixed / args.steps * 1e3,
        "higher_is_better": False,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "mixed fp32/fp64 (fp32 fields, fp64 scalars, fp64 refinement)",
        "data": "synthetic (seeded vortex-seed starts, analytic trap)",
        "config": {"workload": "2D 512^2 rotating GPE on [-16,16]^2, V=(x^2+y^2)/2, beta=1000, Omega=0.9, "
                               "PCG + symmetric combined preconditioner, ||r||_inf <= 1e-8, value = mean "
                               "seconds per solve over the seeded starts",
                   "grid": [512, 512], "beta": 1000.0, "omega": 0.9, "tol": tol,
                   "seeds": list(SEEDS_2D_512_SET)},
        "time_to_tol_fp64_s": t_fp64,
        "speedup_mixed_vs_fp64": t_fp64 / t_mixed,
        "iters_mixed": {"per_solve": it_mixed, "fp32": [r["iters_fp32"] for r in reps_mixed]},
        "iters_fp64": it_fp64,
        "batched_4_starts": batched,
        "pcg_iters_per_s": {"mixed": sum(it_mixed) / sec_mixed, "fp64": sum(it_fp64) / sec_fp64},
        "h_applies_per_s": {"fp64": ap64, "fp32": ap32, "fp64_batch32": apb64, "fp32_batch32": apb32},
        "h_apply_batch32_hbm_gbs": {
            "fp64": 11 * 8 * 512 * 512 * batch / tb64 / 1e9, "fp32": 11 * 4 * 512 * 512 * batch / tb32 / 1e9},
        "final": {"E_mixed": [r["E"] for r in reps_mixed[:len(starts0)]],
                  "res_mixed": max(r["res_inf"] for r in reps_mixed),
                  "E_fp64": [r["E"] for r in reps_fp64[:len(starts0)]],
                  "res_fp64": max(r["res_inf"] for r in reps_fp64)},
        "kernels": {"fp32": kernel_rows(prof32), "fp64": kernel_rows(prof64)},
        "roofline": roofline,
        "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
