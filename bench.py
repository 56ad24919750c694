#!/usr/bin/env python3
"""Benchmark of the rotating-GPE ground-state solver on one MI355X.

Workload: 2-D 512^2 grid on [-16, 16]^2, V = (x^2 + y^2)/2, beta = 1000, Omega = 0.9, eight seeded
vortex-seed starts (the several initial data the paper runs per parameter set, keeping the lowest
energy), PCG with the symmetric combined preconditioner, stop at ||H phi - lambda phi||_inf <= 1e-8
for every start.  One step = the eight starts solved together from resident copies as one batched
PCG solve with per-instance convergence masks, run by the library as two parts of four on two
streams (every stage of the hot path: transforms, H apply,
preconditioner, reductions, direction, line search, retraction, convergence control, precision
switch).  At Omega = 0.9 the iteration count to 1e-8 depends strongly on the start (soft
vortex-lattice modes): a step lasts as long as its slowest start.

Printed (one JSON line on stdout): the mixed FP32/FP64 time-to-1e-8 of a step as `value`, beside the
FP64 step time, each start solved alone (mixed and FP64), the same starts on nested grids 64^2 ->
512^2 (the paper's multigrid preparation of initial data), the 64-instance sweep of mixed grids,
H_phi applies/s, PCG iterations/s, the
dominant kernel's roofline figure (kernel-only HIP event timings of the step's configuration, HBM
traffic from the committed counter summary) and the CPU oracle timed on the host (bounded sample,
extrapolated).
"""
from __future__ import annotations

import argparse
import json
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
    """HBM bytes per launch of `kernel` (step configuration) from the committed counter summary, if
    it was taken from these exact sources (else None)."""
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


def applies_per_s_graph(torch, plan, phi, V, reps=1000):
    """H_phi applies/s of a captured graph of `reps` applies (one field), replayed once; the output of
    the replay is checked against an eager apply."""
    out = torch.empty_like(phi)
    ref = plan.apply_H(phi, V)  # also sizes the plan's scratch before capture
    torch.cuda.synchronize()
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.stream(side):
        with torch.cuda.graph(graph, stream=side):
            for _ in range(reps):
                plan.apply_H(phi, V, out, stream=side)
    torch.cuda.synchronize()
    graph.replay()  # warm
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    s = torch.cuda.current_stream()
    e0.record(s)
    graph.replay()
    e1.record(s)
    e1.synchronize()
    if not torch.equal(out, ref):
        raise RuntimeError("graph-replayed H apply differs from the eager apply")
    return reps / (e0.elapsed_time(e1) / 1e3)


def cpu_model():
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    import platform
    return platform.processor() or "unknown"


def _oracle_sample_job(args):
    """One worker of the all-cores oracle sample: `iters` FP64 PCG_C iterations from one start (BLAS
    and OpenMP held to one thread per process)."""
    sys.path.insert(0, ROOT)
    from oracle import gpe_oracle as O
    prob, V, phi0, iters = args
    try:
        from threadpoolctl import threadpool_limits
        threadpool_limits(1)
    except Exception:  # pragma: no cover
        pass
    t0 = time.perf_counter()
    res = O.pcg(prob, V, phi0, tol_res=1e-8, max_iter=iters)
    return max(1, res.iters), time.perf_counter() - t0


def cpu_all_cores(prob, V, starts, iters, gpu_fp64_iters):
    """The oracle on the host's cores: the eight starts in concurrent worker processes, one start each
    (at most as many as the cores this process may use, 16 at most), `iters` iterations each; the step
    extrapolated as the starts solved concurrently (the slowest start's GPU FP64 iteration count at the
    measured per-process rate)."""
    import multiprocessing as mp
    import os
    avail = len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else (os.cpu_count() or 1)
    procs = max(1, min(len(starts), avail, 16))
    jobs = [(prob, V, starts[k], iters) for k in range(procs)]
    ctx = mp.get_context("spawn")
    # the workers inherit one BLAS / OpenMP thread each (set before they start: numpy reads it on import)
    keys = ("OMP_NUM_THREADS", "OPENBLAS_NUM_THREADS", "MKL_NUM_THREADS")
    saved = {k: os.environ.get(k) for k in keys}
    for k in keys:
        os.environ[k] = "1"
    try:
        t0 = time.perf_counter()
        with ctx.Pool(procs) as pool:
            out = pool.map(_oracle_sample_job, jobs)
        wall = time.perf_counter() - t0
    finally:
        for k, v in saved.items():
            if v is None:
                os.environ.pop(k, None)
            else:
                os.environ[k] = v
    per_proc = [n / sec for n, sec in out]
    rate = min(per_proc)
    return {"processes": procs, "cores_available": avail, "iters_each": iters,
            "iters_per_s_total": sum(n for n, _ in out) / wall, "iters_per_s_per_process": rate,
            "step_s": max(gpu_fp64_iters[:procs]) / rate if procs == len(starts) else None,
            "note": "each start on its own process; the step extrapolated as the starts solved concurrently"}


def cpu_baseline(prob, V, phi0, iters, gpu_fp64_iters_total):
    """The FP64 oracle, as it stands, on the GPU machine's host: PCG iterations/s and H_phi applies/s on
    the 512^2 workload (bounded samples), the 1-D 256-point configuration solved to 1e-10 and the
    2-D 256^2 and 3-D 128^3 configurations sampled, all on one thread (numpy's transforms are
    single-threaded; BLAS is held to one thread so that the figure does not depend on the box's
    core count)."""
    from gpe_inputs import workload_1d, workload_2d, workload_3d
    from oracle import gpe_oracle as O
    try:
        from threadpoolctl import threadpool_limits
        ctx = threadpool_limits(1)
    except Exception:  # pragma: no cover
        ctx = None

    def timed(fn):
        t0 = time.perf_counter()
        r = fn()
        return r, time.perf_counter() - t0

    res, sec = timed(lambda: O.pcg(prob, V, phi0, tol_res=1e-8, max_iter=iters))
    done = max(1, res.iters)
    it_s = done / sec
    phi = phi0 / O.norm(prob, phi0)
    _, ha = timed(lambda: [O.hamiltonian(prob, V, phi) for _ in range(10)])
    p1, V1, f1 = workload_1d()
    r1, s1 = timed(lambda: O.pcg(p1, V1, f1, tol_res=1e-10, max_iter=5000))
    p2, V2, f2 = workload_2d(256)
    r2, s2 = timed(lambda: O.pcg(p2, V2, f2, tol_res=1e-8, max_iter=40))
    p3, V3, f3 = workload_3d(128)
    r3, s3 = timed(lambda: O.pcg(p3, V3, f3, tol_res=1e-8, max_iter=3))
    if ctx is not None and hasattr(ctx, "unregister"):
        ctx.unregister()
    return {
        "value": gpu_fp64_iters_total / it_s,
        "unit": "s",
        "cores": 1,
        "kind": "oracle",
        "sample": (f"numpy FP64 oracle on {cpu_model()} (1 thread), PCG_C on the first 512^2 start, {done} iterations "
                   f"({sec:.1f} s, {it_s:.2f} it/s), extrapolated to one step: the {gpu_fp64_iters_total} iterations "
                   f"the eight starts take to 1e-8 in FP64 on the GPU, solved one after another"),
        "cpu_model": cpu_model(),
        "iters_per_s": it_s,
        "h_applies_per_s_512": 10.0 / ha,
        "c1_1d_256_to_1e-10": {"s": s1, "iters": r1.iters, "E": r1.E, "status": r1.status},
        "c2_2d_256_iters_per_s": r2.iters / s2,
        "c3_3d_128_iters_per_s": max(1, r3.iters) / s3,
    }


def main():
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=2)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--cpu-iters", type=int, default=40)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-single", action="store_true", help="skip the one-start-at-a-time solves")
    ap.add_argument("--no-nested", action="store_true", help="skip the nested-grid solves")
    ap.add_argument("--no-sweep", action="store_true", help="skip the 64-instance sweep")
    ap.add_argument("--no-configs", action="store_true", help="skip the 1-D, 2-D 256^2 and 3-D single solves")
    ap.add_argument("--no-diff", action="store_true", help="skip the differentiation workload")
    ap.add_argument("--paper-table", action="store_true",
                    help="also solve the paper's fast-rotation table (eta = 1000, 5000, 10000 x Omega = 1 ... 4.5 on "
                         "640^2 points of [-20, 20]^2, its stopping rule |E_n+1 - E_n| <= 1e-14), about a minute")
    ap.add_argument("--no-step-rules", action="store_true",
                    help="skip the Armijo / full / Wolfe line search and Fletcher-Reeves solves")
    ap.add_argument("--tol-coarse", type=float, default=1e-5, help="residual tolerance of the coarse nested grids")
    ap.add_argument("--profile-iters", type=int, default=30)
    ap.add_argument("--profile-only", action="store_true",
                    help="only the per-kernel profile of the step's iteration and a 512 MiB copy (counter runs)")
    ap.add_argument("--profile-more", action="store_true",
                    help="only the per-kernel profiles of the 3-D 128^3 iteration and of the sweep's grid groups "
                         "(profiler runs)")
    ap.add_argument("--profile-plane", action="store_true",
                    help="only the whole-plane and directional-pass H applies of the plane comparison, 5 "
                         "launches each (profiler runs)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only (asked for --gpus {args.gpus}); the solver is a single-GPU "
              "path and nothing here uses a second device", file=sys.stderr)
        sys.exit(2)

    import torch

    from gpe_inputs import SEEDS_2D_512_SET, harmonic_potential, workload_2d_set
    from paper_1611_02045_amd import gpe

    if not torch.cuda.is_available():
        log("no GPU available")
        sys.exit(1)
    gpe.lib()
    prob, V_np, starts_np = workload_2d_set(512)
    S = len(starts_np)
    V = torch.from_numpy(V_np).to("cuda")
    starts0 = [torch.from_numpy(x).to("cuda") for x in starts_np]
    tol = 1e-8
    mixed = dict(tol=tol, precision="mixed", max_iter=200000)
    fp64 = dict(tol=tol, precision="fp64", max_iter=200000)
    probs, Vs = [prob] * S, [V] * S

    def profile(precision, count=S):
        # `count` instances: the eight starts, repeated
        ss = [starts0[k % S] for k in range(count)]
        return gpe.pcg_profile_batched([prob] * count, [V] * count, ss, "f64", iters=args.profile_iters,
                                       precision=precision)

    def above_mall():
        """Configurations whose working set exceeds the 256 MB Infinity Cache (MALL), so that their
        HBM figures are DRAM figures: the step's iteration with 24 FP32 instances (8 FP32 fields + V
        per instance: 24 x 17 MiB = 408 MiB), the FP64 iteration of the 8 starts (8 x 34 MiB =
        272 MiB), and H applies over 64 FP32 fields (phi, H phi and the intermediate: 384 MiB) and 32
        FP64 fields (384 MiB), timed per pass with HIP events on the launch stream."""
        out = {"iteration_fp32_x24": kernel_rows(profile("mixed", 3 * S))}
        pl32 = gpe.Plan.from_problem(prob, "f32")
        pl64 = gpe.Plan.from_problem(prob, "f64")
        for tag, pl, dt, n in (("apply_fp32_x64", pl32, torch.complex64, 64), ("apply_fp64_x32", pl64, torch.complex128, 32)):
            bphi = starts0[0].to(dt).unsqueeze(0).repeat(n, 1, 1).contiguous()
            Vd = V.float() if dt == torch.complex64 else V
            rate, sec = applies_per_s(torch, pl, bphi, Vd, 10, batched=True)
            rb = 4 if dt == torch.complex64 else 8
            # the two passes' bytes: x reads phi and the shared V once, writes W; y reads phi and W,
            # writes H phi: (10 n + 1) s N
            out[tag] = {"applies_per_s": rate, "s_per_launch_pair": sec,
                        "GB_s": (10 * n + 1) * rb * 512 * 512 / sec / 1e9}
            del bphi
        return out

    def plane_rates(reps=20, profile_run=False):
        """The whole-plane H apply against the directional passes (both forced through
        gpe_set_apply_kernel) on planes that fit one workgroup's LDS: 128^2 complex64 (one CU per
        plane) for 1, 256 and 1024 fields, 64^2 complex128 for 1 and 1024 fields, and 3-D 128^3
        complex64 (128 planes per field, then the z pass) for 2 fields.  Seconds per launch from
        torch events around `reps` launches on the current stream (the applies' stream); bytes per
        field as the two kernels move them: 2-D 5sN (plane) and 11sN (passes), 3-D 11sN and 17sN,
        with the shared V counted once per launch."""
        gen = torch.Generator(device="cuda")
        gen.manual_seed(2024)
        res = {}
        for dim, n, dt, counts in ((2, (128, 128), "f32", (1, 256, 1024)), (2, (64, 64), "f64", (1, 1024)),
                                   (3, (128, 128, 128), "f32", (2,))):
            pp = type(prob)(dim, n, tuple(8.0 for _ in n), 1000.0, 0.9)
            pl = gpe.Plan.from_problem(pp, dt)
            cd, rd, sb = (torch.complex64, torch.float32, 4) if dt == "f32" else (torch.complex128, torch.float64, 8)
            shape = tuple(reversed(n))
            Vd = torch.rand(shape, dtype=rd, device="cuda", generator=gen)
            npts = 1
            for m in n:
                npts *= m
            for cnt in counts:
                ph = torch.randn((cnt,) + shape, dtype=cd, device="cuda", generator=gen)
                o = torch.empty_like(ph)
                row = {"auto": pl.apply_kernel_for(cnt)}
                for kind in ("plane", "passes"):
                    gpe.set_apply_kernel(kind)
                    try:
                        for _ in range(3):
                            pl.apply_H_batched(ph, Vd, o)
                        torch.cuda.synchronize()
                        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
                        r = 5 if profile_run else reps
                        e0.record()
                        for _ in range(r):
                            pl.apply_H_batched(ph, Vd, o)
                        e1.record()
                        torch.cuda.synchronize()
                    finally:
                        gpe.set_apply_kernel("auto")
                    sec = e0.elapsed_time(e1) * 1e-3 / r
                    per = (5 if dim == 2 else 11) if kind == "plane" else (11 if dim == 2 else 17)
                    nbytes = ((per - 1) * cnt + 1) * sb * npts
                    row[kind] = {"us": sec * 1e6, "GB_s": nbytes / sec / 1e9, "bytes": nbytes}
                row["speedup_plane"] = row["passes"]["us"] / row["plane"]["us"]
                res[f"{'x'.join(map(str, n))}_{dt}_x{cnt}"] = row
                del ph, o
        return res

    def profile_more(iters):
        """Per-kernel profiles beyond the step's configuration, each launch timed by its own HIP events
        on the solver's stream: the 3-D 128^3 workload (one instance, FP32 fields and FP64 fields),
        and the 64-instance sweep's three grid groups (128^2, 256^2, 512^2; each group one batched
        launch set in FP32, as in the sweep's mixed phase; the largest group's working set is beyond
        the 256 MB MALL)."""
        import collections
        from gpe_inputs import batch_instances, workload_3d
        out = {}
        p3, V3, f3 = workload_3d(128)
        V3d, f3d = torch.from_numpy(V3).to("cuda"), torch.from_numpy(f3).to("cuda")
        for prec, tag in (("mixed", "fp32"), ("fp64", "fp64")):
            out[f"3d_128_{tag}"] = kernel_rows(gpe.pcg_profile_batched([p3], [V3d], [f3d], "f64", iters=iters,
                                                                       precision=prec))
        groups = collections.defaultdict(list)
        for bi in batch_instances(64):
            groups[bi.prob.n[0]].append(bi)
        for m in sorted(groups):
            items = groups[m]
            probs_ = [bi.prob for bi in items]
            Vs_ = [torch.from_numpy(bi.V).to("cuda") for bi in items]
            phis_ = [torch.from_numpy(bi.phi0).to("cuda") for bi in items]

            def prof(idx):
                return gpe.pcg_profile_batched([probs_[k] for k in idx], [Vs_[k] for k in idx],
                                               [phis_[k] for k in idx], "f64", iters=iters, precision="mixed",
                                               tol=1e-300)

            # every instance must stay active through the instrumented iterations: a start that ends
            # within them (its FP32 phase stops at a failed line search) is left out, and counted
            idx = list(range(len(items)))
            try:
                rows = prof(idx)
            except gpe.GpeError:
                keep = []
                for k in idx:
                    try:
                        prof([k])
                        keep.append(k)
                    except gpe.GpeError:
                        pass
                idx = keep
                try:
                    rows = prof(idx) if idx else []
                except gpe.GpeError as exc:
                    out[f"sweep_{m}x{m}_fp32"] = {"error": str(exc)}
                    continue
            out[f"sweep_{m}x{m}_fp32_x{len(idx)}"] = kernel_rows(rows)
            if len(idx) < len(items):
                out[f"sweep_{m}x{m}_left_out"] = {"instances": len(items) - len(idx),
                                                  "reason": "finished within the instrumented iterations"}
        for rows in out.values():
            if isinstance(rows, list):
                for r in rows:
                    r["frac"] = r["GB_s"] / HBM_PEAK_GBS
        return out

    if args.profile_more:
        profile_more(2)  # first launches load the kernels
        more = profile_more(args.profile_iters)
        a = torch.empty(512 << 20, dtype=torch.uint8, device="cuda").fill_(1)  # counter scale
        torch.empty_like(a).copy_(a)
        torch.cuda.synchronize()
        print(json.dumps({"profile_more": True, "copy_bytes": a.numel(), "kernels": more}), flush=True)
        return

    if args.profile_plane:
        rates = plane_rates(profile_run=True)
        a = torch.empty(512 << 20, dtype=torch.uint8, device="cuda").fill_(1)  # counter scale
        torch.empty_like(a).copy_(a)
        torch.cuda.synchronize()
        print(json.dumps({"profile_plane": True, "copy_bytes": a.numel(), "rates": rates}), flush=True)
        return

    if args.profile_only:
        for prec in ("mixed", "fp64"):  # first launches load the kernels: keep them out of the averages
            gpe.pcg_profile_batched(probs, Vs, starts0, "f64", iters=2, precision=prec)
        prof32, prof64 = profile("mixed"), profile("fp64")
        big = above_mall()
        # a plain copy of known size, to scale the HBM byte counters
        a = torch.empty(512 << 20, dtype=torch.uint8, device="cuda").fill_(1)
        b = torch.empty_like(a)
        b.copy_(a)
        torch.cuda.synchronize()
        print(json.dumps({"profile_only": True, "copy_bytes": a.numel(),
                          "kernels": {"fp32": kernel_rows(prof32), "fp64": kernel_rows(prof64)},
                          "above_mall": big}), flush=True)
        return

    def step(opts):
        phis = [x.clone() for x in starts0]
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        _, reps = gpe.pcg_solve_batched(probs, Vs, phis, "f64", **opts)
        torch.cuda.synchronize()
        return time.perf_counter() - t0, reps

    log(f"[bench] warmup {args.warmup} step(s)")
    for _ in range(args.warmup):
        step(mixed)

    # timed region: exactly K steps, each the batched mixed-precision solve of the eight starts
    log(f"[bench] timing {args.steps} mixed step(s) of {S} starts")
    t_mixed, reps_mixed = [], None
    for _ in range(args.steps):
        sec, reps_mixed = step(mixed)
        t_mixed.append(sec)
    log(f"[bench] mixed: {mean(t_mixed):.4f} s/step, iters {[r['iters'] for r in reps_mixed]}")
    t_fp64, reps_fp64 = [], None
    for _ in range(args.steps):
        sec, reps_fp64 = step(fp64)
        t_fp64.append(sec)
    log(f"[bench] fp64:  {mean(t_fp64):.4f} s/step, iters {[r['iters'] for r in reps_fp64]}")
    bad = [r["status"] for r in reps_mixed + reps_fp64 if r["status"] != 0]
    if bad:
        log(f"[bench] WARNING: non-converged statuses {bad}")

    # the step controls and CG coefficient the paper names as alternatives (Sections 5.1-5.2), one
    # batched mixed step each (outside the timed region): iterations and seconds beside the
    # heuristic's.  Fletcher-Reeves stalls on most of these starts, so its solves stop at 40 000
    # iterations (four times the heuristic's longest).
    step_rules = None
    if not args.no_step_rules:
        step_rules = {"heuristic_pr": {"s": mean(t_mixed), "iters": [r["iters"] for r in reps_mixed]}}
        for tag, extra in (("armijo_pr", {"line_search": "armijo"}), ("full_pr", {"line_search": "full"}),
                           ("wolfe_pr", {"line_search": "wolfe"}),
                           ("heuristic_fr", {"beta_rule": "fr", "max_iter": 40000})):
            sec, reps = step({**mixed, **extra})
            step_rules[tag] = {"s": sec, "iters": [r["iters"] for r in reps],
                               "converged": sum(r["status"] == 0 for r in reps),
                               "E_min": min(r["E"] for r in reps)}
            log(f"[bench] step rule {tag}: {sec:.4f} s, iters {step_rules[tag]['iters']}")

    # each start solved alone (one plan, one start at a time)
    single = None
    if not args.no_single:
        plan = gpe.Plan.from_problem(prob, "f64")
        single = {}
        for tag, opts in (("mixed", mixed), ("fp64", fp64)):
            secs, its = [], []
            for x in starts0:
                phi = x.clone()
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                r = plan.pcg_solve(V, phi, **opts)
                torch.cuda.synchronize()
                secs.append(time.perf_counter() - t0)
                its.append(r["iters"])
            single[tag] = {"mean_s_per_solve": mean(secs), "iters": its,
                           "pcg_iters_per_s": sum(its) / sum(secs)}
            log(f"[bench] single {tag}: {mean(secs):.4f} s/solve, iters {its}")

    # the same eight starts on nested grids 64^2 -> 512^2 (the paper's multigrid preparation of
    # initial data): each start generated on the coarsest grid, solved there to tol_coarse,
    # interpolated and solved again on each finer grid, the last to 1e-8
    nested = None
    if not args.no_nested:
        prob_c, _, starts_c_np = workload_2d_set(64)
        levels = 4
        lv_probs = [type(prob_c)(2, (64 << l, 64 << l), prob_c.L, prob_c.beta, prob_c.omega) for l in range(levels)]
        lv_V = [torch.from_numpy(harmonic_potential(p)).to("cuda") for p in lv_probs]
        starts_c = [torch.from_numpy(x).to("cuda") for x in starts_c_np]
        nested = {"levels": [64 << l for l in range(levels)], "tol_coarse": args.tol_coarse}
        for tag, opts in (("mixed", mixed), ("fp64", fp64)):
            secs = []
            for _ in range(max(1, args.steps)):
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                _, _, lrep = gpe.pcg_solve_nested([prob_c] * S, [[Vl] * S for Vl in lv_V], starts_c, "f64",
                                                  tol_coarse=args.tol_coarse, **opts)
                torch.cuda.synchronize()
                secs.append(time.perf_counter() - t0)
            nested[tag] = {"s_per_step": mean(secs), "iters_per_level": [[r["iters"] for r in lv] for lv in lrep],
                           "E": [r["E"] for r in lrep[-1]], "res_inf": max(r["res_inf"] for r in lrep[-1]),
                           "status": [r["status"] for r in lrep[-1]]}
            log(f"[bench] nested {tag}: {mean(secs):.4f} s/step, iterations per level (max) "
                f"{[max(r['iters'] for r in lv) for lv in lrep]}")

    # the 64-instance sweep (Omega ~ U[0, 0.95], beta ~ U{100, 500, 1000, 2000}, M ~ U{128, 256, 512},
    # boxes from the Thomas-Fermi radius, vortex-seed starts) as one batched solve to 1e-8
    sweep = None
    if not args.no_sweep:
        import collections
        from gpe_inputs import batch_instances
        inst = batch_instances(64)
        sw_probs = [bi.prob for bi in inst]
        sw_V = [torch.from_numpy(bi.V).to("cuda") for bi in inst]
        sweep = {"instances": len(inst), "grids": dict(collections.Counter(f"{bi.prob.n[0]}^2" for bi in inst))}
        for tag, opts in (("mixed", mixed), ("fp64", fp64)):
            phis = [torch.from_numpy(bi.phi0).to("cuda") for bi in inst]
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            _, sw_reps = gpe.pcg_solve_batched(sw_probs, sw_V, phis, "f64", **opts)
            torch.cuda.synchronize()
            sec = time.perf_counter() - t0
            by = collections.defaultdict(int)
            for bi, r in zip(inst, sw_reps):
                by[f"{bi.prob.n[0]}^2"] = max(by[f"{bi.prob.n[0]}^2"], r["iters"])
            sweep[tag] = {"s": sec, "max_iters_per_grid": dict(by), "all_converged": all(r["status"] == 0 for r in sw_reps),
                          "total_iters": sum(r["iters"] for r in sw_reps)}
            log(f"[bench] sweep of 64 {tag}: {sec:.3f} s, max iterations per grid {dict(by)}")

    # the other single-solve configurations of the workload set: 1-D 256 points (FP64 to 1e-10, and
    # beta = 0 whose exact energy is 1/2), 2-D 256^2 at Omega = 0.9 (FP64 and mixed to 1e-8), 3-D 128^3
    # at Omega = 0.8 (complex64 fields with FP64 scalars, then the FP64 refinement, to 1e-8)
    configs = None
    if not args.no_configs:
        from gpe_inputs import workload_1d, workload_2d, workload_3d
        configs = {}

        def timed_solve(p, Vn, phin, dtype, **opts):
            pl = gpe.Plan.from_problem(p, dtype)
            cd = torch.complex128 if dtype == "f64" else torch.complex64
            rd = torch.float64 if dtype == "f64" else torch.float32
            Vd = torch.from_numpy(Vn).to("cuda", rd)
            ph = torch.from_numpy(phin).to("cuda", cd)
            pl.pcg_solve(Vd, ph.clone(), **dict(opts, max_iter=50))  # warm the plan
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            r = pl.pcg_solve(Vd, ph, **opts)
            torch.cuda.synchronize()
            return {"s": time.perf_counter() - t0, "iters": r["iters"], "E": r["E"], "res_inf": r["res_inf"],
                    "status": r["status_name"]}

        p1, V1, f1 = workload_1d()
        configs["1d_256_fp64_tol1e-10"] = timed_solve(p1, V1, f1, "f64", tol=1e-10)
        p0 = type(p1)(1, (256,), (16.0,), 0.0, 0.0)
        configs["1d_256_beta0_fp64"] = timed_solve(p0, V1, f1, "f64", tol=1e-10)
        configs["1d_256_beta0_fp64"]["E_exact"] = 0.5
        p2, V2, f2 = workload_2d(256)
        configs["2d_256_fp64"] = timed_solve(p2, V2, f2, "f64", tol=1e-8, max_iter=200000)
        configs["2d_256_mixed"] = timed_solve(p2, V2, f2, "f64", tol=1e-8, max_iter=200000, precision="mixed")
        p3, V3, f3 = workload_3d(128)
        configs["3d_128_mixed"] = timed_solve(p3, V3, f3, "f64", tol=1e-8, max_iter=200000, precision="mixed")
        # the paper's fast-rotation example (harmonic + quartic trap, eta = 1000, Omega = 2, Thomas-Fermi
        # start) on its own grid, 640^2 points of [-20, 20]^2 (radix-5 transforms), and on 512^2
        from gpe_inputs import workload_quartic_2d
        for m in (640, 512):
            pq, Vq, fq = workload_quartic_2d(m, 2.0, 1000.0)
            for prec in ("fp64", "mixed"):
                configs[f"2d_{m}_quartic_omega2_{prec}"] = timed_solve(pq, Vq, fq, "f64", tol=1e-8, max_iter=200000,
                                                                      precision=prec)
        for k, v in configs.items():
            log(f"[bench] config {k}: {v['s']:.4f} s, {v['iters']} iterations, E = {v['E']:.10f}, {v['status']}")
        # the paper's fast-rotation series on its own grid: Omega = 1 ... 4.5 at eta = 1000, 640^2 points
        # of [-20, 20]^2, Thomas-Fermi start, FP64 PCG to 1e-8
        series = {}
        for om in (1.0, 1.5, 2.0, 2.5, 3.0, 3.5, 4.0, 4.5):
            pq, Vq, fq = workload_quartic_2d(640, om, 1000.0)
            series[f"{om:g}"] = timed_solve(pq, Vq, fq, "f64", tol=1e-8, max_iter=200000)
        configs["2d_640_quartic_omega_series_fp64"] = series
        log("[bench] fast-rotation series on 640^2 (Omega: s, iterations): " +
            ", ".join(f"{k}: {v['s']:.3f} s {v['iters']}" for k, v in series.items()))

    # the differentiation workload (2-D 256^2 on [-16, 16]^2, beta = 1000, Omega = 0.85, harmonic trap
    # with 9 Gaussian pins): loss = E(phi*) + h^2 sum (|phi*|^2 - rho_t)^2, rho_t from a solve at the
    # seeded target parameters; forward = the FP64 ground-state solve to 1e-11, backward = the implicit
    # adjoint solve and the parameter gradients (gamma_y, A, beta, Omega) through torch autograd
    diff = None
    if not args.no_diff:
        import numpy as np
        from gpe_inputs import differentiation_workload, mesh, target_parameters
        from paper_1611_02045_amd.autograd import Grid, energy as energy_fn, ground_state
        dprob, cent, _, dphi0 = differentiation_workload()
        dgrid = Grid(2, dprob.n, dprob.L)
        x, y = mesh(dprob)
        X = torch.from_numpy(np.broadcast_to(x, dprob.shape).copy()).to("cuda")
        Y = torch.from_numpy(np.broadcast_to(y, dprob.shape).copy()).to("cuda")
        Cc = torch.tensor(cent, device="cuda")
        f64 = dict(dtype=torch.float64, device="cuda")

        def pinned(gy, A):
            Vp = 0.5 * (X ** 2 + gy ** 2 * Y ** 2)
            for j in range(Cc.shape[0]):
                Vp = Vp + A * torch.exp(-((X - Cc[j, 0]) ** 2 + (Y - Cc[j, 1]) ** 2) / (2 * 0.5 ** 2))
            return Vp

        gy_t, A_t = target_parameters()
        phi_t = torch.from_numpy(dphi0).to("cuda")
        gpe.Plan.from_problem(dprob, "f64").pcg_solve(pinned(torch.tensor(gy_t, **f64), torch.tensor(A_t, **f64))
                                                      .contiguous(), phi_t, tol=1e-10, max_iter=200000)
        rho_t = (phi_t.abs() ** 2).detach()
        theta = [torch.tensor(v, requires_grad=True, **f64) for v in (1.05, 2.0, dprob.beta, dprob.omega)]
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        Vt = pinned(theta[0], theta[1])
        phis = ground_state(Vt, theta[2], theta[3], torch.from_numpy(dphi0).to("cuda"), dgrid)
        loss = energy_fn(phis, Vt, theta[2], theta[3], dgrid) + dgrid.cell * torch.sum((phis.abs() ** 2 - rho_t) ** 2)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        loss.backward()
        torch.cuda.synchronize()
        t2 = time.perf_counter()
        diff = {"workload": "2-D 256^2, beta=1000, Omega=0.85, 9 pins; d loss / d(gamma_y, A, beta, Omega)",
                "forward_s": t1 - t0, "backward_s": t2 - t1, "loss": float(loss.item()),
                "grad": [float(t.grad.item()) for t in theta]}
        log(f"[bench] differentiation: forward {t1 - t0:.3f} s, backward {t2 - t1:.3f} s, grad {diff['grad']}")

    # the paper's fast-rotation table on its grid with its stopping rule (opt-in: about a minute)
    table = None
    if args.paper_table:
        from gpe_inputs import workload_quartic_2d
        table = {}
        for eta in (1000.0, 5000.0, 10000.0):
            row = {}
            for om in (1.0, 1.5, 2.0, 2.5, 3.0, 3.5, 4.0, 4.5):
                pq, Vq, fq = workload_quartic_2d(640, om, eta)
                pl = gpe.Plan.from_problem(pq, "f64")
                Vd, ph = torch.from_numpy(Vq).to("cuda"), torch.from_numpy(fq.copy()).to("cuda")
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                r = pl.pcg_solve(Vd, ph, tol=0.0, tol_energy=1e-14, max_iter=100000)
                torch.cuda.synchronize()
                row[f"{om:g}"] = {"s": time.perf_counter() - t0, "iters": r["iters"], "E": r["E"],
                                  "res_inf": r["res_inf"], "status": r["status_name"]}
            table[f"{eta:g}"] = row
            log(f"[bench] paper table eta = {eta:g}: " + ", ".join(f"{k}: {v['s']:.2f} s" for k, v in row.items()))

    # H_phi applies/s (single field and a batch of 32 fields, FP64 and FP32)
    log("[bench] H applies")
    plan64 = gpe.Plan.from_problem(prob, "f64")
    plan32 = gpe.Plan.from_problem(prob, "f32")
    phi0 = starts0[0]
    V32, phi32 = V.float(), phi0.to(torch.complex64)
    ap64, _ = applies_per_s(torch, plan64, phi0, V, 400)
    ap32, _ = applies_per_s(torch, plan32, phi32, V32, 400)
    batch = 32
    bphi64 = phi0.unsqueeze(0).repeat(batch, 1, 1).contiguous()
    bphi32 = phi32.unsqueeze(0).repeat(batch, 1, 1).contiguous()
    apb64, tb64 = applies_per_s(torch, plan64, bphi64, V, 20, batched=True)
    apb32, tb32 = applies_per_s(torch, plan32, bphi32, V32, 20, batched=True)
    # the same on the paper's 640^2 grid (every line transform ends in a radix-5 stage)
    ap640 = None
    if not args.no_configs:
        from gpe_inputs import workload_quartic_2d
        pq, Vq, fq = workload_quartic_2d(640, 2.0, 1000.0)
        ap640 = {}
        for dt, cd, rd in (("f64", torch.complex128, torch.float64), ("f32", torch.complex64, torch.float32)):
            pl = gpe.Plan.from_problem(pq, dt)
            ap640[dt], _ = applies_per_s(torch, pl, torch.from_numpy(fq).to("cuda", cd),
                                         torch.from_numpy(Vq).to("cuda", rd), 400)
        log(f"[bench] H applies at 640^2: {ap640}")
    log("[bench] whole-plane H apply against the passes")
    planes = plane_rates()
    log("[bench] whole-plane: " + ", ".join(f"{k}: {v['plane']['us']:.1f} us vs {v['passes']['us']:.1f} us"
                                             for k, v in planes.items()))
    apg64 = apg32 = None
    try:
        apg64 = applies_per_s_graph(torch, plan64, phi0, V)
        apg32 = applies_per_s_graph(torch, plan32, phi32, V32)
    except RuntimeError as exc:  # reported, not fatal: the captured loop is an extra figure
        log(f"[bench] graph-replayed applies unavailable: {exc}")

    # per-kernel timings of the step's iteration (all eight starts), FP32 fields and FP64 fields
    log("[bench] kernel profile")
    prof32, prof64 = profile("mixed"), profile("fp64")
    # a batched mixed solve runs its FP32 phase until every start has left it, then the FP64 phase
    n32 = max(r["iters_fp32"] for r in reps_mixed)
    n64 = max(r["iters"] for r in reps_mixed) - n32
    weight = {"fp32": n32, "fp64": max(n64, 0)}
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
                "timing": f"HIP start/stop events recorded by each launch (kernel execution only), {S} instances",
                "cache": "the step's working set (8 FP32 instances, ~136 MiB) fits in the 256 MB MALL: "
                         "see roofline_above_mall for the same kernel with a DRAM-sized working set"}
    # a streaming kernel of known size as a second denominator: torch's elementwise kernel reading and
    # writing 1 GiB of FP32 (beyond the MALL)
    ca = torch.ones(1 << 28, dtype=torch.float32, device="cuda")
    cb = torch.empty_like(ca)
    for _ in range(3):
        torch.mul(ca, 1.0, out=cb)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(10):
        torch.mul(ca, 1.0, out=cb)
    e1.record()
    torch.cuda.synchronize()
    copy_gbs = 2 * ca.numel() * 4 / (e0.elapsed_time(e1) * 1e-3 / 10) / 1e9
    del ca, cb
    roofline["copy_GB_s"] = copy_gbs
    roofline["frac_of_copy"] = achieved / copy_gbs
    log("[bench] above-MALL profile")
    big = above_mall()
    log("[bench] 3-D and sweep-group profiles")
    try:
        more = profile_more(args.profile_iters)
    except Exception as exc:  # an extra figure: reported, never fatal to the bench line
        more = {"error": str(exc)}
    row = next(r for r in big["iteration_fp32_x24"] if r["name"] == name)
    roofline_big = {"bound": "hbm", "achieved": row["GB_s"], "peak": HBM_PEAK_GBS, "unit": "GB/s",
                    "frac": row["GB_s"] / HBM_PEAK_GBS, "traffic": measured_traffic(f"{name} (fp32 x24)"),
                    "kernel": f"{name} (fp32)", "instances": 3 * S, "bytes_per_launch": row["bytes"],
                    "avg_ms": row["avg_ms"], "working_set_MiB": 3 * S * (8 * 8 + 4) * 512 * 512 / 2 ** 20,
                    "iteration": big["iteration_fp32_x24"], "fp64_iteration_x8": kernel_rows(prof64),
                    "applies": {k: v for k, v in big.items() if k.startswith("apply")},
                    "copy_GB_s": copy_gbs, "frac_of_copy": row["GB_s"] / copy_gbs}

    # the same measurements as fractions of the HBM peak: an iteration of the step's configuration as the
    # sum of its passes' bytes over the sum of their kernel times, and the batched H applies
    def iteration_frac(rows):
        by = sum(r["bytes"] for r in rows)
        sec = sum(r["avg_ms"] for r in rows) * 1e-3
        return {"bytes": by, "us": sec * 1e6, "GB_s": by / sec / 1e9, "frac": by / sec / 1e9 / HBM_PEAK_GBS}
    hbm_fractions = {
        "pcg_iteration_fp32_x8": iteration_frac(kernel_rows(prof32)),
        "pcg_iteration_fp64_x8": iteration_frac(kernel_rows(prof64)),
        "pcg_iteration_fp32_x24_beyond_mall": iteration_frac(big["iteration_fp32_x24"]),
        "h_apply_fp32_x64_beyond_mall": big["apply_fp32_x64"]["GB_s"] / HBM_PEAK_GBS,
        "h_apply_fp64_x32_beyond_mall": big["apply_fp64_x32"]["GB_s"] / HBM_PEAK_GBS,
        "h_apply_fp32_x32": (10 * batch + 1) * 4 * 512 * 512 / tb32 / 1e9 / HBM_PEAK_GBS,
        "h_apply_fp64_x32": (10 * batch + 1) * 8 * 512 * 512 / tb64 / 1e9 / HBM_PEAK_GBS,
        "h_apply_whole_plane_128x128_fp32_x1024": planes["128x128_f32_x1024"]["plane"]["GB_s"] / HBM_PEAK_GBS,
    }

    it_fp64_single = single["fp64"]["iters"] if single else [r["iters"] for r in reps_fp64]
    cpu = None
    if not args.no_cpu:
        log(f"[bench] CPU oracle sample ({args.cpu_iters} iterations)")
        cpu = cpu_baseline(prob, V_np, starts_np[0], args.cpu_iters, int(sum(it_fp64_single)))
        log("[bench] CPU oracle sample on all cores")
        cpu["all_cores"] = cpu_all_cores(prob, V_np, starts_np, args.cpu_iters, it_fp64_single)

    it_mixed = [r["iters"] for r in reps_mixed]
    it_fp64 = [r["iters"] for r in reps_fp64]
    out = {
        "metric": METRIC,
        "value": mean(t_mixed),
        "unit": "s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": mean(t_mixed) * 1e3,
        "higher_is_better": False,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "mixed fp32/fp64 (fp32 fields, fp64 scalars, fp64 refinement)",
        "data": "synthetic (seeded vortex-seed starts, analytic trap)",
        "config": {"workload": f"2D 512^2 rotating GPE on [-16,16]^2, V=(x^2+y^2)/2, beta=1000, Omega=0.9, "
                               f"{S} seeded starts solved as one batched PCG (combined preconditioner, "
                               f"per-instance masks, two parts on two streams) until every start has "
                               f"||r||_inf <= 1e-8; value = seconds per step (the whole batch)",
                   "grid": [512, 512], "beta": 1000.0, "omega": 0.9, "tol": tol, "starts": S,
                   "seeds": list(SEEDS_2D_512_SET)},
        "time_to_tol_fp64_s": mean(t_fp64),
        "speedup_mixed_vs_fp64": mean(t_fp64) / mean(t_mixed),
        "iters_mixed": {"per_start": it_mixed, "fp32": [r["iters_fp32"] for r in reps_mixed]},
        "iters_fp64": it_fp64,
        "single_start": single,
        "step_rules": step_rules,
        "differentiation": diff,
        "paper_table_640": table,
        "nested_grids": nested,
        "sweep_64": sweep,
        "other_configs": configs,
        "pcg_iters_per_s_step": {"mixed": max(it_mixed) / mean(t_mixed), "fp64": max(it_fp64) / mean(t_fp64)},
        "h_applies_per_s": {"fp64": ap64, "fp32": ap32, "fp64_batch32": apb64, "fp32_batch32": apb32,
                            "fp64_graph1000": apg64, "fp32_graph1000": apg32, "at_640x640": ap640},
        "h_apply_whole_plane": planes,
        "h_apply_batch32_hbm_gbs": {  # (10 B + 1) s N bytes: phi twice, W twice, H phi once, the shared V once
            "fp64": (10 * batch + 1) * 8 * 512 * 512 / tb64 / 1e9, "fp32": (10 * batch + 1) * 4 * 512 * 512 / tb32 / 1e9},
        "final": {"E_mixed": [r["E"] for r in reps_mixed], "res_mixed": max(r["res_inf"] for r in reps_mixed),
                  "E_fp64": [r["E"] for r in reps_fp64], "res_fp64": max(r["res_inf"] for r in reps_fp64)},
        "kernels": {"fp32": kernel_rows(prof32), "fp64": kernel_rows(prof64)},
        "hbm_peak_fractions": hbm_fractions,
        "kernels_more": more,
        "roofline": roofline,
        "roofline_above_mall": roofline_big,
        "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
