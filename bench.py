#!/usr/bin/env python3
"""Throughput benchmark of the IRK stage solve on one MI355X.

Workload (default): 2-D nonlinear diffusion u_t = div((1+u^2) grad u) + f on
a periodic 512 x 512 grid (5-point stencil, manufactured forcing from
u* = sin(2 pi x) sin(2 pi y) cos t), 3-stage Gauss (order 6), dt = 5e-3,
the 50-step job t = 0 -> 0.25 starting from u*(0); float64 FGMRES with
float32 geometric-multigrid V-cycles (Chebyshev degree 3).  Inputs are
seeded/synthetic and resident in HBM before the timed region.

One "step" = one IRK step (the whole hot path: stage residual, eigenbasis
transform, FGMRES per eigen-block with V-cycle preconditioning, update).
The timed region runs --steps steps from t = 0 after --warmup untimed steps
(the state is reset to u*(0) after warm-up), bracketed by
torch.cuda.synchronize().

Printed: one JSON line with DOF*stages/s (value), steps/s, p50/p99 step
latency, the same workload with float64 V-cycles on the same GPU, a roofline
entry for the dominant kernel measured live with HIP events, and the CPU
oracle (full Newton + SuperLU) timed on a bounded sample.
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

METRIC = "IRK steps/sec & DOF·stages/s vs plain FP64 on same GPU; p50/p99 step latency"
HBM_PEAK_GBS = 8000.0


def run_job(torch, irk, inputs, n, s, dt, steps, warmup, prec_fp32, profile=False):
    op = irk.make_operator(irk.OP_NLDIFF_2D, n, forcing=irk.FORCING_MMS)
    solver = irk.Solver("gauss", s, op, irk.make_options(prec_fp32=prec_fp32))
    u0 = torch.tensor(inputs.nldiff_u0(n), dtype=torch.float64, device="cuda")
    a = u0.clone()
    b = torch.empty_like(a)
    t = 0.0
    for _ in range(warmup):
        solver.step(a, t, dt, out=b)
        a, b = b, a
        t += dt
    a.copy_(u0)
    t = 0.0
    if profile:
        irk.irk_profile_enable(solver.ctx, True)
    stream = torch.cuda.current_stream()
    lat = []
    stats = []
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        _, st = solver.step(a, t, dt, out=b)
        e1.record(stream)
        lat.append((e0, e1))
        stats.append(st)
        a, b = b, a
        t += dt
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    lat_ms = sorted(e0.elapsed_time(e1) for e0, e1 in lat)
    prof = irk.irk_profile_read(solver.ctx) if profile else None
    final = a.clone()
    solver.close()
    return wall, lat_ms, stats, prof, final


def pct(sorted_vals, q):
    if not sorted_vals:
        return None
    k = min(len(sorted_vals) - 1, max(0, int(round(q / 100.0 * (len(sorted_vals) - 1)))))
    return sorted_vals[k]


def cpu_baseline(n_sample, s, dt):
    """The oracle as it stands (full Newton, SuperLU) on one step of the same
    workload at a reduced grid, single-threaded."""
    try:
        from threadpoolctl import threadpool_limits
    except Exception:  # pragma: no cover
        threadpool_limits = None
    from oracle import newton as nw
    from oracle import problems as pb
    from oracle import tableau as tb
    from paper_2101_01776_amd import inputs
    A, b, c = tb.tableau("gauss", s)
    prob = pb.NonlinearDiffusion2D(n_sample, forcing="continuous")
    u0 = inputs.nldiff_u0(n_sample).ravel()
    ctx = threadpool_limits(limits=1) if threadpool_limits else None
    try:
        t0 = time.perf_counter()
        _, _, info = nw.irk_step(prob, A, b, c, u0, 0.0, dt)
        el = time.perf_counter() - t0
    finally:
        if ctx is not None:
            ctx.unregister() if hasattr(ctx, "unregister") else None
    dof = n_sample * n_sample
    return {"value": dof * s / el, "unit": "DOF*stages/s", "cores": 1, "kind": "oracle",
            "sample": f"one Gauss-{s} step (dt={dt}) of the same nonlinear-diffusion workload on a "
                      f"{n_sample}x{n_sample} grid: full Newton ({info.newton_its} iterations) with a "
                      f"SuperLU factorization each, single thread; {el:.2f} s for the step"}


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--n", type=int, default=512, help="grid side (default 512)")
    ap.add_argument("--stages", type=int, default=3)
    ap.add_argument("--dt", type=float, default=5e-3)
    ap.add_argument("--no-fp64", action="store_true", help="skip the float64-V-cycle comparison run")
    ap.add_argument("--no-profile", action="store_true", help="skip the per-kernel roofline pass")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-sample-n", type=int, default=128)
    args = ap.parse_args()

    if args.gpus != 1:
        print("bench.py: this build runs on one GPU only; multi-GPU runs are not supported "
              "(the request-level sharding design is described in DESIGN.md).", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2101_01776_amd import inputs, irk

    if not torch.cuda.is_available():
        print("bench.py: no GPU visible", file=sys.stderr)
        sys.exit(1)
    irk.lib()
    n, s, dt, K, W = args.n, args.stages, args.dt, args.steps, args.warmup
    dof = n * n

    wall, lat, stats, _, _ = run_job(torch, irk, inputs, n, s, dt, K, W, prec_fp32=1)
    value = dof * s * K / wall
    out = {
        "metric": METRIC,
        "value": value,
        "unit": "DOF*stages/s",
        "n_gpus": 1,
        "steps": K,
        "warmup": W,
        "ms_per_step": 1e3 * wall / K,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": f"nonlinear-diffusion-2d periodic {n}x{n}, Gauss s={s}, dt={dt}, "
                               f"{K} steps from t=0, manufactured forcing",
                   "grid": n, "stages": s, "dt": dt,
                   "precision": "float64 Newton/FGMRES/transform, float32 multigrid V-cycle",
                   "parallelism": "single GPU"},
        "steps_per_s": K / wall,
        "p50_ms": pct(lat, 50),
        "p99_ms": pct(lat, 99),
        "newton_its_per_step": sum(x["newton_its"] for x in stats) / K,
        "krylov_its_per_step": sum(x["krylov_its"] for x in stats) / K,
        "prec_applications_per_step": sum(x["prec_applications"] for x in stats) / K,
    }
    if not args.no_fp64:
        w64, lat64, st64, _, _ = run_job(torch, irk, inputs, n, s, dt, K, W, prec_fp32=0)
        out["fp64_vcycle"] = {"value": dof * s * K / w64, "ms_per_step": 1e3 * w64 / K,
                              "steps_per_s": K / w64, "p50_ms": pct(lat64, 50), "p99_ms": pct(lat64, 99),
                              "krylov_its_per_step": sum(x["krylov_its"] for x in st64) / K}
        out["mixed_speedup_vs_fp64"] = w64 / wall
    if not args.no_profile:
        _, _, _, prof, _ = run_job(torch, irk, inputs, n, s, dt, min(K, 10), 1, prec_fp32=1, profile=True)
        prof.sort(key=lambda r: -r["ms"])
        top = prof[0]
        achieved = top["bytes"] / (top["ms"] * 1e-3) / 1e9
        out["roofline"] = {"bound": "hbm", "kernel": top["name"], "achieved": achieved, "peak": HBM_PEAK_GBS,
                           "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS, "traffic": None,
                           "launches": top["launches"], "avg_us": 1e3 * top["ms"] / max(1, top["launches"]),
                           "avg_bytes": top["bytes"] / max(1, top["launches"])}
        tot = sum(r["ms"] for r in prof)
        out["kernel_share"] = [{"kernel": r["name"], "share": r["ms"] / tot, "launches": r["launches"],
                                "avg_us": 1e3 * r["ms"] / max(1, r["launches"]),
                                "GB/s": r["bytes"] / max(1e-12, r["ms"] * 1e-3) / 1e9} for r in prof[:8]]
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(args.cpu_sample_n, s, dt)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
