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


WORKLOADS = {
    # name: (problem, grid side, family, stages, dt, steps, nu)
    "nldiff512-gauss3": ("nldiff", 512, "gauss", 3, 5e-3, 50, 0.0),
    "vsf1024-radau3": ("vsf", 1024, "radau", 3, 2e-3, 20, 1e-3),
    "nldiff1024-gauss5": ("nldiff", 1024, "gauss", 5, 1e-2, 20, 0.0),
}


def describe(problem, n, family, s, dt, steps, nu):
    fam = "Gauss" if family == "gauss" else "Radau IIA"
    if problem == "vsf":
        return (f"vorticity-streamfunction 2-D DAE periodic {n}x{n}, nu={nu:g}, 32 seeded Gaussian vortices, "
                f"{fam} s={s}, dt={dt:g}, {steps} steps from t=0")
    return (f"nonlinear-diffusion-2d periodic {n}x{n}, {fam} s={s}, dt={dt:g}, {steps} steps from t=0, "
            f"manufactured forcing")


def make_problem(irk, inputs, problem, n, nu):
    if problem == "vsf":
        return irk.make_operator(irk.OP_VSF_2D, n, nu=nu), inputs.vsf_state0(n, 0, 32), 2 * n * n
    return irk.make_operator(irk.OP_NLDIFF_2D, n, forcing=irk.FORCING_MMS), inputs.nldiff_u0(n), n * n


BATCH_MG = 0      # shared V-cycle launches (irk_options.batch_mg), off by default
MG_OPTS = {}      # multigrid option overrides (--cheb-degree, --mg-coarsest)


def run_job(torch, irk, inputs, wl, steps, warmup, prec_fp32, profile=False):
    problem, n, family, s, dt, _, nu = wl
    op, u_init, _ = make_problem(irk, inputs, problem, n, nu)
    solver = irk.Solver(family, s, op, irk.make_options(prec_fp32=prec_fp32, batch_mg=BATCH_MG, **MG_OPTS))
    u0 = torch.tensor(u_init, dtype=torch.float64, device="cuda")
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
    prof = None
    if profile:
        prof = irk.irk_profile_read(solver.ctx)
        # the dominant group also timed back-to-back (no per-launch event
        # overhead), on the stream it ran on
        top = max(prof, key=lambda r: r["ms"])
        top["replay"] = irk.irk_profile_replay(solver.ctx, top["name"], 20)
    final = a.clone()
    solver.close()
    return wall, lat_ms, stats, prof, final


def ablation(torch, irk, inputs, wl, steps):
    """Preconditioner variants of the paper's solver study on the same job:
    gamma* = eta + beta^2/eta vs gamma = eta in the 2x2 Schur approximation
    (Table 4's comparison), and the Newton-like truncations (0) last stage,
    (1) lumped to the largest stage weight, (2) the row's stage weights,
    (3) plus the coupling of the rows of a pair; (1) and (3) in the real Schur
    basis (blocks by back-substitution, (3) with the stage-weighted coupling
    of the blocks); and the adaptive Krylov tolerance against the paper's
    fixed one; for the DAE also the reordered system and the streamfunction
    rows' Poisson block applied by a V-cycle instead of the spectral solve.
    Preconditioner applications are the paper's cost unit."""
    problem, n, family, s, dt, _, nu = wl
    op, u_init, dof = make_problem(irk, inputs, problem, n, nu)
    res = []
    # (gamma_mode, newton_like, krylov_adaptive, dae_reorder, transform, psi_solve)
    variants = [(0, 1, 1, 0, 0, 0), (0, 1, 0, 0, 0, 0), (1, 1, 1, 0, 0, 0), (0, 0, 1, 0, 0, 0),
                (0, 2, 1, 0, 0, 0), (0, 3, 1, 0, 0, 0)]
    if problem == "vsf":
        variants.append((0, 1, 1, 1, 0, 0))       # the reordered DAE system, eq (vsf-system-2)
        variants.append((0, 1, 1, 0, 0, 1))       # Poisson V-cycle for the streamfunction rows
    else:
        variants += [(0, 1, 1, 0, 1, 0), (0, 3, 1, 0, 1, 0)]   # real Schur basis, back-substitution
    for gm, nl, ka, ro, tr, ps in variants:
        solver = irk.Solver(family, s, op, irk.make_options(gamma_mode=gm, newton_like=nl, krylov_adaptive=ka,
                                                            dae_reorder=ro, transform=tr, psi_solve=ps))
        u = torch.tensor(u_init, dtype=torch.float64, device="cuda")
        b = torch.empty_like(u)
        t = 0.0
        stats = []
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            _, st = solver.step(u, t, dt, out=b)
            stats.append(st)
            u, b = b, u
            t += dt
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        solver.close()
        res.append({"gamma": "gamma*" if gm == 0 else "eta", "newton_like": nl,
                    "basis": "real Schur (back-substitution)" if tr else "eigenbasis (independent blocks)",
                    "krylov_tol": "adaptive" if ka else "fixed",
                    "dae_system": ("reordered (vsf-system-2)" if ro else "whole (vsf-system-1)") if problem == "vsf"
                    else None,
                    "psi_solve": ("V-cycle" if ps else "spectral") if problem == "vsf" else None,
                    "ms_per_step": 1e3 * wall / steps,
                    "vcycles_per_step": sum(x["vcycles"] for x in stats) / steps,
                    "newton_its_per_step": sum(x["newton_its"] for x in stats) / steps,
                    "krylov_its_per_step": sum(x["krylov_its"] for x in stats) / steps,
                    "krylov_its_per_block": [sum(x["krylov_its_block"][k] for x in stats) / steps
                                             for k in range(5)],
                    "prec_applications_per_step": sum(x["prec_applications"] for x in stats) / steps})
    return res


def sdirk_compare(torch, irk, inputs, wl, steps):
    """The paper's comparison on the same kernels: fully implicit Gauss /
    Radau IIA against SDIRK of equal order on the same job (same dt, same
    preconditioner: one V-cycle per real block or per diagonal of a 2x2
    block), with the error at the end of the job against a Gauss-3 run at
    dt/4 of the same semi-discrete system."""
    problem, n, _, _, dt, _, nu = wl
    op, u_init, dof = make_problem(irk, inputs, problem, n, nu)

    def job(family, s, dtt, nsteps):
        # both classes start every step the same way (zero or explicit; the
        # extrapolated start is a property of the fully implicit stages only)
        # and solve every block to the paper's fixed Krylov tolerance
        solver = irk.Solver(family, s, op, irk.make_options(start_extrapolate=0, krylov_adaptive=0))
        u = torch.tensor(u_init, dtype=torch.float64, device="cuda")
        b = torch.empty_like(u)
        t, stats = 0.0, []
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(nsteps):
            _, st = solver.step(u, t, dtt, out=b)
            stats.append(st)
            u, b = b, u
            t += dtt
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        solver.close()
        return u, wall, stats

    ref, _, _ = job("gauss", 3, dt / 4, 4 * steps)
    out = []
    for order, fam, s in ((2, "gauss", 1), (2, "sdirk", 2), (3, "radau", 2), (3, "sdirk", 3),
                          (4, "gauss", 2), (4, "sdirk", 5)):
        u, wall, stats = job(fam, s, dt, steps)
        err = float(torch.linalg.norm(u - ref) / torch.linalg.norm(ref))
        out.append({"order": order, "method": f"{fam}-{s}", "ms_per_step": 1e3 * wall / steps,
                    "newton_its_per_step": sum(x["newton_its"] for x in stats) / steps,
                    "prec_applications_per_step": sum(x["prec_applications"] for x in stats) / steps,
                    "rel_error_at_end": err})
    return {"dt": dt, "steps": steps, "reference": "gauss-3 at dt/4", "runs": out}


def measured_traffic(workload, kernel):
    """HBM bytes per launch of `kernel` in `workload` from the committed
    rocprofv3 counter runs (FETCH_SIZE and WRITE_SIZE averaged over the
    kernel's dispatches, each scaled by the same counter on a plain device
    copy of known size), or None when absent or taken on kernel sources other
    than the ones built here."""
    import hashlib
    path = os.path.join(ROOT, "profiles", "pmc_traffic.json")
    try:
        with open(path) as f:
            rec = json.load(f)
    except (OSError, ValueError):
        return None
    run = rec.get("workloads", {}).get(workload)
    if run is None:
        return None
    for src, want in run.get("sources_sha256", {}).items():
        try:
            with open(os.path.join(ROOT, src), "rb") as f:
                if hashlib.sha256(f.read()).hexdigest() != want:
                    return None
        except OSError:
            return None
    ent = run.get("kernels", {}).get(kernel)
    return None if ent is None else ent["hbm_bytes_per_launch"]


def copy_probe(torch, mib=256, reps=3):
    """A plain device copy of known size (read + write `mib` MiB each), for
    scaling the hardware byte counters."""
    x = torch.ones(mib << 17, dtype=torch.float64, device="cuda")
    y = torch.empty_like(x)
    for _ in range(reps):
        y.copy_(x)
    torch.cuda.synchronize()


def copy_bandwidth(torch, mib=512, reps=5):
    """Rate of a plain device-to-device copy (read + write of `mib` MiB),
    best of `reps`, between events on the current stream: the HBM rate a
    streaming kernel can reach on this GPU, as context for `frac`."""
    x = torch.ones(mib << 17, dtype=torch.float64, device="cuda")
    y = torch.empty_like(x)
    y.copy_(x)
    best = None
    for _ in range(reps):
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record()
        y.copy_(x)
        e1.record()
        e1.synchronize()
        ms = e0.elapsed_time(e1)
        best = ms if best is None else min(best, ms)
    del x, y
    return 2.0 * (mib << 20) / (best * 1e-3) / 1e9


def pct(sorted_vals, q):
    if not sorted_vals:
        return None
    k = min(len(sorted_vals) - 1, max(0, int(round(q / 100.0 * (len(sorted_vals) - 1)))))
    return sorted_vals[k]


def host_info():
    """CPU model, usable cores and the BLAS thread pools of this process
    (their current limits)."""
    model = None
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    try:
        usable = len(os.sched_getaffinity(0))
    except AttributeError:  # pragma: no cover
        usable = os.cpu_count()
    blas = None
    try:
        import numpy  # noqa: F401  (load the BLAS the oracle uses before listing the pools)
        import scipy.sparse.linalg  # noqa: F401
        from threadpoolctl import threadpool_info
        blas = [{"api": p.get("internal_api"), "threads": p.get("num_threads")} for p in threadpool_info()]
    except Exception:  # pragma: no cover
        pass
    return {"cpu_model": model, "nproc": os.cpu_count(), "usable_cores": usable, "blas_pools": blas,
            "omp_num_threads": os.environ.get("OMP_NUM_THREADS")}


def sample_problem(wl, n_sample):
    from paper_2101_01776_amd import inputs
    problem, _, family, s, dt, _, nu = wl
    if problem == "vsf":
        return inputs.vsf_state0(n_sample, 0, 32), 2 * n_sample * n_sample
    return inputs.nldiff_u0(n_sample), n_sample * n_sample


def cpu_baseline(wl, n_sample):
    """The oracle as it stands (full Newton, SuperLU) on the first step of the
    same workload at a reduced grid, single-threaded (SuperLU factorizes on
    one thread; the BLAS pools are limited to one as well)."""
    try:
        from threadpoolctl import threadpool_limits
    except Exception:  # pragma: no cover
        threadpool_limits = None
    from oracle import newton as nw
    from oracle import problems as pb
    from oracle import tableau as tb
    problem, _, family, s, dt, _, nu = wl
    A, b, c = tb.tableau(family, s)
    u0, dof = sample_problem(wl, n_sample)
    if problem == "vsf":
        prob = pb.VorticityStreamfunction2D(n_sample, nu=nu)
    else:
        prob = pb.NonlinearDiffusion2D(n_sample, forcing="continuous")
    ctx = threadpool_limits(limits=1) if threadpool_limits else None
    try:
        t0 = time.perf_counter()
        _, _, info = nw.irk_step(prob, A, b, c, u0.ravel(), 0.0, dt)
        el = time.perf_counter() - t0
        host = host_info()                 # the thread pools as limited for the oracle's run
    finally:
        if ctx is not None and hasattr(ctx, "unregister"):
            ctx.unregister()
    return {"value": dof * s / el, "unit": "DOF*stages/s", "cores": 1, "kind": "oracle",
            "sample": f"the first {family} s={s} step (dt={dt:g}, t=0) of the same workload on a "
                      f"{n_sample}x{n_sample} grid: full Newton ({info.newton_its} iterations) with a SuperLU "
                      f"factorization each, one thread; {el:.2f} s for the step",
            "s_per_step": el, "threads_used": 1, "host": host}


def gpu_same_size(torch, irk, wl, n_sample, reps=10):
    """The library on the oracle's sample: the same first step from t = 0
    repeated (each from the same input, so none is a continued step), mixed
    precision, inputs resident on the device."""
    from paper_2101_01776_amd import inputs  # noqa: F401
    problem, _, family, s, dt, _, nu = wl
    u0, dof = sample_problem(wl, n_sample)
    if problem == "vsf":
        op = irk.make_operator(irk.OP_VSF_2D, n_sample, nu=nu)
    else:
        op = irk.make_operator(irk.OP_NLDIFF_2D, n_sample, forcing=irk.FORCING_MMS)
    solver = irk.Solver(family, s, op, irk.make_options(prec_fp32=1))
    a = torch.tensor(u0, dtype=torch.float64, device="cuda")
    b = torch.empty_like(a)
    for _ in range(2):
        solver.step(a, 0.0, dt, out=b)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        solver.step(a, 0.0, dt, out=b)
    torch.cuda.synchronize()
    el = (time.perf_counter() - t0) / reps
    solver.close()
    return {"value": dof * s / el, "unit": "DOF*stages/s", "s_per_step": el,
            "sample": f"the same first step on {n_sample}x{n_sample}, {reps} repetitions"}


def serve_inputs(torch, inputs, count, seed):
    """Seeded serving stream (unit-rate arrivals; scaled by 1/lambda when
    replayed) with every request's initial field resident on the device."""
    reqs = inputs.serving_requests(count, 1.0, seed=seed)
    fields = [torch.tensor(inputs.nldiff_random_u0(r.n, r.seed), dtype=torch.float64, device="cuda")
              for r in reqs]
    return reqs, fields


def serve_run(torch, irk, reqs, fields, lam, prec_fp32, budget, slots, arena):
    """Replay the stream through the native serving loop.  lam=None: closed
    loop (everything submitted at t=0); otherwise open-loop Poisson arrivals
    at lam requests/s.  Returns wall time, per-request latencies (arrival to
    result, ms), per-step latencies (ms) and serving statistics."""
    ops = {n: irk.make_operator(irk.OP_NLDIFF_2D, n, forcing=irk.FORCING_MMS) for n in {r.n for r in reqs}}
    opt = irk.make_options(prec_fp32=prec_fp32, batch_mg=BATCH_MG)
    outs = [torch.empty_like(f) for f in fields]
    arrive = [0.0] * len(reqs) if lam is None else [r.arrival / lam for r in reqs]
    srv = irk.Server(budget, slots, arena=arena)
    torch.cuda.synchronize()
    ids, late = [], []
    k = 0
    t0 = time.perf_counter()
    t_note = 20.0
    while True:
        now = time.perf_counter() - t0
        if now > t_note:                     # progress note for long runs
            print(f"serve: {now:.0f} s, {k} of {len(reqs)} submitted", file=sys.stderr, flush=True)
            t_note += 20.0
        while k < len(reqs) and arrive[k] <= now:
            r = reqs[k]
            ids.append(srv.submit(r.family, r.s, ops[r.n], fields[k], r.dt, r.nsteps, opt=opt, out=outs[k]))
            late.append(time.perf_counter() - t0 - arrive[k])      # submit delay after arrival
            k += 1
        left = srv.progress()
        if left == 0 and k == len(reqs):
            break
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    lat, failed, steps = [], 0, 0
    for rid, d in zip(ids, late):
        info = srv.info(rid)
        failed += info["state"] != "done"
        steps += info["steps_done"]
        lat.append(1e3 * (info["t_done"] - info["t_submit"] + d))
    st = srv.stats()
    srv.close()
    return wall, sorted(lat), sorted(st["step_ms"]), {"failed": failed, "steps": steps,
                                                      "peak_running": st["peak_running"],
                                                      "peak_bytes": st["peak_bytes"]}


def serve_bench(torch, irk, inputs, count, budget_gb, slots, load, seed, fp64=True, sweep=()):
    """Continuous-batching serving workload: nonlinear-diffusion requests,
    grid side log-uniform in {128..1024}, Gauss or Radau IIA with s in
    {2,3,4}, dt log-uniform in [1e-3, 1e-2], 10 steps each.  First the
    closed-loop saturation throughput mu, then open-loop Poisson arrivals at
    lambda = load * mu; the same stream with float64 V-cycles beside it.
    sweep: further loads (fractions of mu) run open-loop with float32
    V-cycles only."""
    reqs, fields = serve_inputs(torch, inputs, count, seed)
    budget = int(budget_gb * (1 << 30)) & ~255
    arena = torch.empty(budget + 256, dtype=torch.uint8, device="cuda")     # the HBM budget, allocated once
    dofs = sum(r.n * r.n * r.s * r.nsteps for r in reqs)
    warm = min(len(reqs), 16)
    serve_run(torch, irk, reqs[:warm], fields[:warm], None, 1, budget, slots, arena)       # load kernels, pools
    out = {"requests": count, "seed": seed, "budget_gb": budget_gb, "max_slots": slots,
           "stream": "nonlinear-diffusion-2d requests, side log-uniform {128,256,512,1024}, "
                     "Gauss/Radau IIA s in {2,3,4}, dt log-uniform [1e-3,1e-2], 10 steps each, "
                     "manufactured forcing, seeded smooth initial fields"}
    for prec in ((1, 0) if fp64 else (1,)):
        key = "mixed" if prec else "fp64_vcycle"
        wall, lat, step_lat, st = serve_run(torch, irk, reqs, fields, None, prec, budget, slots, arena)
        mu = count / wall
        res = {"closed_loop": {"req_per_s": mu, "steps_per_s": st["steps"] / wall,
                               "dof_stages_per_s": dofs / wall, "wall_s": wall,
                               "step_p50_ms": pct(step_lat, 50), "step_p99_ms": pct(step_lat, 99),
                               "req_p50_ms": pct(lat, 50), "req_p99_ms": pct(lat, 99), **st}}
        if prec:
            lam = load * mu
            out["lambda_req_per_s"] = lam
        wall, lat, step_lat, st = serve_run(torch, irk, reqs, fields, lam, prec, budget, slots, arena)
        res["open_loop"] = {"lambda_req_per_s": lam, "req_per_s": count / wall, "steps_per_s": st["steps"] / wall,
                            "dof_stages_per_s": dofs / wall, "wall_s": wall,
                            "step_p50_ms": pct(step_lat, 50), "step_p99_ms": pct(step_lat, 99),
                            "req_p50_ms": pct(lat, 50), "req_p99_ms": pct(lat, 99), **st}
        if prec and sweep:
            res["open_loop_sweep"] = []
            for ld in sweep:
                print(f"serve: open loop at {ld:g} x mu", file=sys.stderr, flush=True)
                wall, lat, step_lat, st = serve_run(torch, irk, reqs, fields, ld * mu, prec, budget, slots, arena)
                res["open_loop_sweep"].append({
                    "load": ld, "lambda_req_per_s": ld * mu, "req_per_s": count / wall,
                    "steps_per_s": st["steps"] / wall, "step_p50_ms": pct(step_lat, 50),
                    "step_p99_ms": pct(step_lat, 99), "req_p50_ms": pct(lat, 50), "req_p99_ms": pct(lat, 99),
                    "failed": st["failed"], "peak_running": st["peak_running"]})
        out[key] = res
    return out


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=None, help="timed steps (default: the workload's job)")
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="vsf1024-radau3", choices=sorted(WORKLOADS),
                    help="vsf1024-radau3 (default; the largest single-GPU job by DOF*stages): "
                         "vorticity-streamfunction DAE 1024^2, Radau IIA-3, dt 2e-3, 20 steps; "
                         "nldiff512-gauss3: 2-D nonlinear diffusion 512^2, Gauss-3, dt 5e-3, "
                         "50 steps; nldiff1024-gauss5: nonlinear diffusion 1024^2, Gauss-5, "
                         "dt 1e-2, 20 steps")
    ap.add_argument("--n", type=int, default=None, help="override the grid side")
    ap.add_argument("--stages", type=int, default=None, help="override s")
    ap.add_argument("--dt", type=float, default=None, help="override dt")
    ap.add_argument("--no-fp64", action="store_true", help="skip the float64-V-cycle comparison run")
    ap.add_argument("--no-profile", action="store_true", help="skip the per-kernel roofline pass")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-sample-n", type=int, default=None,
                    help="grid side of the oracle sample (default 128; 32 for the DAE, 96 for Gauss-5)")
    ap.add_argument("--sdirk-compare", action="store_true",
                    help="also compare Gauss/Radau IIA with SDIRK of equal order on the workload")
    ap.add_argument("--ablation", action="store_true",
                    help="also compare gamma* vs eta, the Newton-like truncations (0)-(3), fixed vs "
                         "adaptive Krylov tolerance and (DAE) the reordered system on the workload")
    ap.add_argument("--cheb-degree", type=int, default=None, help="Chebyshev smoothing degree (default 3)")
    ap.add_argument("--mg-coarsest", type=int, default=None, help="coarsest multigrid side (default 16)")
    ap.add_argument("--batch-mg", action="store_true",
                    help="run the V-cycles of blocks/requests that wait together as shared launches")
    ap.add_argument("--copy-probe", action="store_true",
                    help="run a 256 MiB device copy first (counter calibration)")
    ap.add_argument("--serve", action="store_true",
                    help="run the serving workload instead (one JSON line of its own)")
    ap.add_argument("--requests", type=int, default=2000)
    ap.add_argument("--budget-gb", type=float, default=200.0)
    ap.add_argument("--slots", type=int, default=32)
    ap.add_argument("--load", type=float, default=0.8, help="open-loop lambda as a fraction of mu")
    ap.add_argument("--serve-seed", type=int, default=0)
    ap.add_argument("--serve-sweep", default="",
                    help="comma-separated further open-loop loads (fractions of mu), float32 V-cycles only")
    ap.add_argument("--serve-sample", type=int, default=0,
                    help="also run a serving sample of this many requests in the default bench")
    args = ap.parse_args()

    if args.gpus != 1:
        print("bench.py: one GPU only; runs on several GPUs are not supported (requests are independent "
              "and would shard over GPUs with one admission ledger per GPU, which is not built).", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2101_01776_amd import inputs, irk

    if not torch.cuda.is_available():
        print("bench.py: no GPU visible", file=sys.stderr)
        sys.exit(1)
    irk.lib()
    global BATCH_MG, MG_OPTS
    BATCH_MG = 1 if args.batch_mg else 0
    if args.cheb_degree:
        MG_OPTS["cheb_degree"] = args.cheb_degree
    if args.mg_coarsest:
        MG_OPTS["mg_coarsest"] = args.mg_coarsest
    if args.copy_probe:
        copy_probe(torch)
    if args.serve:
        t0 = time.perf_counter()
        sweep = tuple(float(x) for x in args.serve_sweep.split(",") if x.strip())
        sv = serve_bench(torch, irk, inputs, args.requests, args.budget_gb, args.slots, args.load,
                         args.serve_seed, fp64=not args.no_fp64, sweep=sweep)
        m = sv["mixed"]["open_loop"]
        out = {"metric": METRIC, "value": m["steps_per_s"], "unit": "IRK steps/s", "n_gpus": 1,
               "steps": m["steps"], "warmup": 16, "ms_per_step": 1e3 / m["steps_per_s"],
               "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64",
               "data": "synthetic",
               "config": {"workload": f"serving: {args.requests} nonlinear-diffusion step-solve requests, "
                                      f"open-loop Poisson arrivals at {args.load:g} x saturation",
                          "precision": "float64 Newton/FGMRES/transform, float32 multigrid V-cycle",
                          "parallelism": "single GPU"},
               "p50_ms": m["step_p50_ms"], "p99_ms": m["step_p99_ms"], "serving": sv,
               "bench_wall_s": time.perf_counter() - t0}
        print(json.dumps(out), flush=True)
        return
    problem, n, family, s, dt, K, nu = WORKLOADS[args.workload]
    n = args.n or n
    s = args.stages or s
    dt = args.dt or dt
    K = args.steps or K
    W = args.warmup
    wl = (problem, n, family, s, dt, K, nu)
    dof = n * n * (2 if problem == "vsf" else 1)
    dflt = WORKLOADS[args.workload]
    default_shape = (n, s, dt) == (dflt[1], dflt[3], dflt[4])

    wall, lat, stats, _, _ = run_job(torch, irk, inputs, wl, K, W, prec_fp32=1)
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
        "config": {"workload": describe(problem, n, family, s, dt, K, nu),
                   "grid": n, "family": family, "stages": s, "dt": dt, "dof_per_stage": dof,
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
        w64, lat64, st64, _, _ = run_job(torch, irk, inputs, wl, K, W, prec_fp32=0)
        out["fp64_vcycle"] = {"value": dof * s * K / w64, "ms_per_step": 1e3 * w64 / K,
                              "steps_per_s": K / w64, "p50_ms": pct(lat64, 50), "p99_ms": pct(lat64, 99),
                              "krylov_its_per_step": sum(x["krylov_its"] for x in st64) / K}
        out["mixed_speedup_vs_fp64"] = w64 / wall
    if not args.no_profile:
        kp = min(K, 10)
        wp, _, _, prof, _ = run_job(torch, irk, inputs, wl, kp, 1, prec_fp32=1, profile=True)
        prof.sort(key=lambda r: -r["ms"])
        top = prof[0]
        rep = top["replay"]
        achieved = rep["bytes"] / (rep["ms"] * 1e-3) / 1e9
        out["roofline"] = {"bound": "hbm", "kernel": top["name"], "achieved": achieved, "peak": HBM_PEAK_GBS,
                           "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS,
                           "traffic": measured_traffic(args.workload, top["name"]) if default_shape else None,
                           "avg_us": 1e3 * rep["ms"], "avg_bytes": rep["bytes"],
                           "timing": "back-to-back replays of the kernel's most recent launches of the profiled "
                                     "pass (20 rounds) between HIP events on its stream",
                           "in_run": {"launches": top["launches"],
                                      "avg_us_event_bracketed": 1e3 * top["ms"] / max(1, top["launches"]),
                                      "avg_bytes": top["bytes"] / max(1, top["launches"])}}
        cb = copy_bandwidth(torch)
        out["roofline"]["copy_reference"] = {"GB_per_s": cb, "frac_of_peak": cb / HBM_PEAK_GBS,
                                             "what": "512 MiB device-to-device copy (read + write), best of 5"}
        tot = sum(r["ms"] for r in prof)
        step_bytes = sum(r["bytes"] for r in prof) / kp
        out["step_traffic"] = {"algorithmic_MB_per_step": step_bytes / 1e6,
                               "GB_per_s_over_step": step_bytes / (wall / K) / 1e9,
                               "frac_of_peak": step_bytes / (wall / K) / 1e9 / HBM_PEAK_GBS,
                               "kernel_ms_per_step_summed_over_concurrent_lanes": tot / kp}
        out["kernel_share"] = [{"kernel": r["name"], "share": r["ms"] / tot, "launches": r["launches"],
                                "avg_us": 1e3 * r["ms"] / max(1, r["launches"]),
                                "GB/s": r["bytes"] / max(1e-12, r["ms"] * 1e-3) / 1e9} for r in prof[:8]]
    if args.ablation:
        out["ablation"] = ablation(torch, irk, inputs, wl, min(K, 20))
    if args.sdirk_compare:
        out["sdirk_compare"] = sdirk_compare(torch, irk, inputs, wl, K)
    if args.serve_sample > 0:
        out["serving"] = serve_bench(torch, irk, inputs, args.serve_sample, args.budget_gb, args.slots,
                                     args.load, args.serve_seed, fp64=not args.no_fp64)
    if not args.no_cpu_baseline:
        ns = args.cpu_sample_n or {"vsf1024-radau3": 32, "nldiff1024-gauss5": 96}.get(args.workload, 128)
        cb = cpu_baseline(wl, ns)
        g = gpu_same_size(torch, irk, wl, ns)
        cb["gpu_same_sample"] = g
        cb["gpu_over_oracle_same_sample"] = cb["s_per_step"] / g["s_per_step"]
        out["cpu_baseline"] = cb
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
