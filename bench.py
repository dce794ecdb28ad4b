#!/usr/bin/env python
"""Benchmark of the ABAC-preconditioned MINRES wave solver on one MI355X.

A step is one whole solve: right-hand side assembly from device-resident source
samples and initial data, then preconditioned MINRES to relative residual tol.
Prints ONE JSON line on stdout (progress goes to stderr).

    python bench.py [--steps K] [--warmup W] [--workload NAME] [--prec fp64|fp32]
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "solves/s at rel. residual 1e-8 (FP32-precond vs FP64); p50/p99 latency"
HBM_PEAK_GBS = 8000.0

WORKLOADS = {
    # name: nx, ny, nt, alpha, batch, source recipe
    "wave2d_255x255x256": dict(nx=255, ny=255, nt=256, alpha=1e-3, batch=1, source="manufactured2d"),
    # the same grid with an i.i.d. N(0,1) source (seed 2) and zero initial data: a
    # right-hand side without the manufactured solution's smoothness
    "wave2d_255x255x256_random": dict(nx=255, ny=255, nt=256, alpha=1e-3, batch=1, source="random", seed=2),
    "wave2d_511x511x512": dict(nx=511, ny=511, nt=512, alpha=1e-3, batch=1, source="gaussian_field"),
    "batch64_wave2d_127x127x128": dict(nx=127, ny=127, nt=128, alpha=1e-3, batch=64, source="jacobi"),
    "wave1d_63x64": dict(nx=63, ny=0, nt=64, alpha=1e-3, batch=1, source="manufactured1d"),
    # the same 1D problem as a batch (throughput of the launch-bound size): right-hand
    # side b draws its noise with seed 1 + b, so b = 0 is the single-solve workload
    "batch256_wave1d_63x64": dict(nx=63, ny=0, nt=64, alpha=1e-3, batch=256, source="manufactured1d"),
    "serving_mix": dict(nx=0, ny=0, nt=0, alpha=0.0, batch=1, source="serving"),
}
KERNEL_CLASSES = ["stencil", "dstx_fwd", "dsty", "time", "dstx_inv", "update", "form", "residual", "init", "rhs", "fin",
                  "gmres", "iter"]


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def make_inputs(w):
    import synth
    nx, ny, nt, B = w["nx"], w["ny"], w["nt"], w["batch"]
    srcs, p0s, p1s = [], [], []
    for b in range(B):
        if w["source"] == "manufactured2d":
            src, p0, p1, _ = synth.manufactured_2d(nx, ny, nt)
        elif w["source"] == "manufactured1d":
            src, p0, p1, _ = synth.manufactured_1d(nx, nt, noise_std=0.1, seed=1 + b)
        elif w["source"] == "random":
            src, p0, p1 = synth.random_source(nx, ny, nt, seed=w["seed"] + b)
        elif w["source"] == "gaussian_field":
            src, p0, p1 = synth.gaussian_field_source(nx, ny, nt, seed=3)
        elif w["source"] == "jacobi":
            src, p0, p1 = synth.jacobi_smoothed_source(nx, ny, nt, seed=4000 + b)
        else:
            raise ValueError(w["source"])
        srcs.append(src)
        p0s.append(p0)
        p1s.append(p1)
    return np.stack(srcs), np.stack(p0s), np.stack(p1s)


def algorithmic_bytes(w, prec, iters_total, solves, fused=False):
    """Algorithmic HBM bytes of every kernel class over `solves` right-hand-side solves
    that took `iters_total` MINRES iterations in total (summed over right-hand sides).

    Per right-hand side, with N unknowns, NS = nt*(nx+1)*max(ny,1) scratch values of
    s bytes (8 for FP64, 4 for FP32 transforms):
      stencil   16 N           (read z, write A z) per iteration
      dstx_fwd  32 N + s NS    (read A z, v_j, v_{j-1}; write q; write scratch) per
                8 N + s NS      iteration, plus the set-up pass (read b)
      dsty      2 s NS         (read + write scratch) per launch, 2 launches per apply
      time      2 s NS         (read + write scratch) per apply
      dstx_inv  s NS + 8 N     (read scratch, write p) per apply; <q, p> comes from the
                               time pass (the squared norm of its first factor's output)
      update    24 N           (read r, v; write r) per iteration while the Krylov basis
                               is resident (iterations 1..12), 72 N after it (also
                               read z, w1, w2, x; write w, x)
      form      8 (k+1) N      (read z_1..z_k, write u) once per solve of k <= 12
                               iterations (the convergence check)
      init      24 N           (read f; write v1 = r0, u) per solve
    With `fused` (small 1D plans: one launch per solve, one workgroup per right-hand side
    runs the set-up with its first preconditioner apply and every iteration) all of the
    above is the "iter" class.
    """
    nx, ny, nt = w["nx"], w["ny"], w["nt"]
    N = nt * nx * max(ny, 1)
    NS = nt * (nx + 1) * max(ny, 1)
    s = 8 if prec == "fp64" else 4
    applies = iters_total + solves
    if fused:
        per_iter = 16 * N + (32 * N + s * NS) + 2 * s * NS + (s * NS + 8 * N) + 24 * N
        setup = 24 * N + (8 * N + s * NS) + 2 * s * NS + (s * NS + 8 * N)
        return {"iter": per_iter * iters_total + 8 * N * (iters_total + solves) + setup * solves}
    return {
        "stencil": 16 * N * iters_total,
        "dstx_fwd": (32 * N + s * NS) * iters_total + (8 * N + s * NS) * solves,
        "dsty": 2 * (2 * s * NS) * applies if ny else 0,
        "time": 2 * s * NS * applies,
        "dstx_inv": (s * NS + 8 * N) * applies,
        "update": 24 * N * iters_total,
        "form": 8 * N * (iters_total + solves),
        "init": 24 * N * solves,
    }


def algorithmic_bytes_gmres(w, prec, steps_total, applies, solves):
    """Algorithmic HBM bytes of right-preconditioned GMRES with C_alpha^{-1}: `applies`
    applications of C^{-1} (one per Arnoldi step plus one per formed iterate), one T
    matvec per step (16 N), one explicit residual vector per formed iterate (read u
    and f, write f - T u: 24 N).  C^{-1} passes: x-DST 8 N + s NS, y-DST 2 x 2 s NS,
    time 2 s NS, inverse x-DST s NS + 8 N.  The Gram-Schmidt vector kernels are not
    modelled (their bytes grow with the column index)."""
    nx, ny, nt = w["nx"], w["ny"], w["nt"]
    N = nt * nx * max(ny, 1)
    NS = nt * (nx + 1) * max(ny, 1)
    s = 8 if prec == "fp64" else 4
    forms = applies - steps_total
    return {
        "stencil": 16 * N * steps_total,
        "dstx_fwd": (8 * N + s * NS) * applies,
        "dsty": 2 * (2 * s * NS) * applies if ny else 0,
        "time": 2 * s * NS * applies,
        "dstx_inv": (s * NS + 8 * N) * applies,
        "residual": 24 * N * forms,
        "init": 32 * N * solves,
    }


def pmc_traffic(kernel_class, workload, prec):
    """Per-launch HBM bytes from a committed rocprofv3 counter summary, if it was taken
    on the current kernel sources; else None."""
    path = os.path.join(ROOT, "profiles", f"pmc_{kernel_class}_{workload}_{prec}.json")
    if not os.path.exists(path):
        return None
    rec = json.load(open(path))
    if rec.get("source_sha") != source_sha():
        return None
    return rec.get("bytes_per_launch")


def source_sha():
    from paper_2306_03574_amd.profiling import source_sha as sha
    return sha()


COPY_PROBE_BYTES = 1 << 30


def copy_probe(nbytes=None, pattern="copy"):
    """A plain device copy of COPY_PROBE_BYTES (read and written once per dispatch):
    the calibration run for the HBM byte counters.  Prints its own bandwidth.  Another
    size (nbytes) gives the copy ceiling at that size.  pattern "half" instead reads the
    first 64 bytes of every 128-byte line of the buffer into a packed half-size buffer
    (a second access pattern for the counters: half-line reads at a 128-byte stride)."""
    import torch
    nbytes = nbytes or COPY_PROBE_BYTES
    a = torch.ones(nbytes // 8, dtype=torch.float64, device="cuda:0")
    if pattern == "half":
        src = a.view(-1, 16)[:, :8]
        moved = (nbytes // 2, nbytes // 2)
    else:
        src = a
        moved = (nbytes, nbytes)
    b = torch.empty(src.shape, dtype=src.dtype, device=src.device)
    b.copy_(src)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    n = 5
    for _ in range(n):
        b.copy_(src)
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / n
    print(json.dumps({"copy_bytes": nbytes, "pattern": pattern, "read_bytes": moved[0], "write_bytes": moved[1],
                      "GB/s": round((moved[0] + moved[1]) / dt / 1e9, 1)}), flush=True)


def run_gpu(w, prec, steps, warmup, tol, maxit, profile=True, solver="minres", restart=15):
    """Time `steps` whole solves (production path: graph-replayed iterations, no
    per-kernel events), then, if `profile`, repeat the same steps with every kernel
    bracketed by HIP events on the plan stream to get per-kernel durations."""
    import torch
    from paper_2306_03574_amd import Plan
    dev = torch.device("cuda:0")
    src, p0, p1 = make_inputs(w)
    d_src = torch.from_numpy(src).to(dev)
    d_p0 = torch.from_numpy(p0).to(dev)
    d_p1 = torch.from_numpy(p1).to(dev)
    del src
    plan = Plan(w["nx"], w["ny"], w["nt"], T=1.0, alpha=w["alpha"], prec=prec, batch=w["batch"], device=dev)
    f = plan.empty()
    u = plan.empty()
    def solve():
        if solver == "gmres":
            return plan.gmres(f, u, tol=tol, maxit=maxit, restart=restart)
        return plan.solve(f, u, tol=tol, maxit=maxit)

    for i in range(warmup):
        plan.build_rhs(d_src, d_p0, d_p1, f)
        solve()
    torch.cuda.synchronize()

    def timed(n):
        lat, iters_total, last = [], 0, None
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for i in range(n):
            ts = time.perf_counter()
            plan.build_rhs(d_src, d_p0, d_p1, f)
            last = solve()
            lat.append(time.perf_counter() - ts)
            iters_total += sum(last[1])
        torch.cuda.synchronize()
        return time.perf_counter() - t0, lat, iters_total, last

    elapsed, lat, iters_total, last = timed(steps)
    prof, prof_elapsed, prof_iters = {}, None, None
    if profile:
        plan.profile(True)
        plan.profile_reset()
        prof_elapsed, _, prof_iters, _ = timed(steps)
        for k in KERNEL_CLASSES:
            ms, n = plan.profile_read(k)
            prof[k] = {"ms": ms, "launches": n}
        plan.profile(False)
    _, iters, relres, status = last
    u_host = u.cpu().numpy()
    return dict(elapsed=elapsed, lat=lat, iters=iters, relres=relres, status=status, iters_total=iters_total,
                prof=prof, prof_elapsed=prof_elapsed, prof_iters=prof_iters, u=u_host, tiles=plan.tiles())


def cpu_model():
    """The host CPU's model name (from /proc/cpuinfo), or the platform string."""
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    import platform
    return platform.processor() or platform.machine()


def golden_oracle(workload):
    """The oracle's stored solve of a workload (tests/golden/c3_oracle.json for the
    511^2 x 512 grid; written by a script that calls only the oracle), or None."""
    if workload != "wave2d_511x511x512":
        return None
    path = os.path.join(ROOT, "tests", "golden", "c3_oracle.json")
    if not os.path.exists(path):
        return None
    with open(path) as fh:
        return json.load(fh)


def cpu_baseline(w, tol, maxit, solver="minres", restart=15, full_iters=None):
    """The oracle, as it stands, on the host: FP64, scipy.fft on every core.

    Where no count is stored for the workload the whole solve runs (first right-hand
    side only for batched workloads; below 3 s the median of three after a warm-up is
    reported).  Where the oracle's solve is stored (the 511^2 x 512 grid, several
    minutes on the host) the run is a bounded sample: right-hand side assembly, the set-up
    P^{-1} apply and `sample_iters` MINRES iterations are timed, operator calls
    separately, and the whole solve of `full_iters` iterations (the oracle's own count,
    stored for that workload) is extrapolated as
        t_rhs + (full_iters + 1) t_Pinv + full_iters (t_A + t_vec),
    t_vec the MINRES vector work per iteration."""
    from oracle.discretization import Grid, L_matrix
    from oracle import allatonce as aao, preconditioner as pc, minres as mr
    g = Grid(w["nx"], w["ny"], w["nt"], 1.0)
    src, p0, p1 = make_inputs(dict(w, batch=1))
    L = L_matrix(g)
    tA, tP = [], []

    def timed_op(fn, acc):
        def op(v):
            t1 = time.perf_counter()
            out = fn(v)
            acc.append(time.perf_counter() - t1)
            if g.N > 50_000_000:
                log(f"oracle operator call {len(tA) + len(tP)}: {acc[-1]:.1f} s")
            return out
        return op

    def one_solve(fixed=None):
        t1 = time.perf_counter()
        f = aao.build_rhs(g, src[0], p0[0], p1[0])
        t_rhs = time.perf_counter() - t1
        if solver == "gmres":
            from oracle import gmres as gm
            return t_rhs, f, gm.gmres(timed_op(lambda v: aao.apply_T(g, v, L), tA),
                                      timed_op(lambda y: pc.apply_C_inv(g, w["alpha"], y), tP), f,
                                      tol=tol, maxit=maxit, restart=restart)
        return t_rhs, f, mr.minres(timed_op(lambda v: aao.apply_A(g, v, L), tA),
                                   timed_op(lambda y: pc.apply_Pinv(g, w["alpha"], y), tP),
                                   aao.reverse_time(f), tol=tol, maxit=maxit, fixed_iters=fixed)

    sampled = full_iters is not None and solver == "minres"
    ncores = os.cpu_count()
    c0, t0 = time.process_time(), time.perf_counter()
    if sampled:
        k = 2
        t_rhs, f, res = one_solve(fixed=k)
        wall = time.perf_counter() - t0
        t_vec = max(0.0, (wall - t_rhs - sum(tA) - sum(tP)) / k)
        t_P = float(np.median(tP))
        t_A = float(np.median(tA))
        est = t_rhs + (full_iters + 1) * t_P + full_iters * (t_A + t_vec)
        threads = (time.process_time() - c0) / wall
        return dict(value=1.0 / est, unit="solves/s", cores=max(1, int(round(threads))), kind="oracle",
                    sample=(f"bounded sample of one FP64 oracle solve of the same workload: right-hand side, "
                            f"set-up P^-1 and {k} MINRES iterations timed ({wall:.1f} s wall), whole solve of "
                            f"{full_iters} iterations extrapolated to {est:.1f} s; {ncores} host cores visible, "
                            f"{cpu_model()}"),
                    iters=None, x=None,
                    per_operator={"apply_A_s": float(f"{t_A:.4g}"), "apply_Pinv_s": float(f"{t_P:.4g}"),
                                  "minres_vectors_per_iter_s": float(f"{t_vec:.4g}"),
                                  "rhs_s": float(f"{t_rhs:.4g}")})
    _, f, res = one_solve()
    wall = time.perf_counter() - t0
    cpu = time.process_time() - c0
    # a short solve (small workloads) is repeated: the first one was the warm-up, the
    # median of the next three is reported; a long one is timed once
    nrep = 1
    if wall < 3.0:
        walls = []
        c0, t0 = time.process_time(), time.perf_counter()
        for _ in range(3):
            t1 = time.perf_counter()
            one_solve()
            walls.append(time.perf_counter() - t1)
        threads = (time.process_time() - c0) / (time.perf_counter() - t0)
        wall, nrep = float(np.median(walls)), 3
        cpu = threads * wall
    # the oracle's operators on their own, median of 3 (the solve above was their warm-up)
    ops = {}
    if solver == "minres":
        y = aao.reverse_time(f)
        for name, fn in (("apply_A_s", lambda: aao.apply_A(g, y, L)),
                         ("apply_Pinv_s", lambda: pc.apply_Pinv(g, w["alpha"], y))):
            ts = []
            for _ in range(3):
                t1 = time.perf_counter()
                fn()
                ts.append(time.perf_counter() - t1)
            ops[name] = float(f"{np.median(ts):.4g}")
    return dict(value=1.0 / wall, unit="solves/s", cores=max(1, int(round(cpu / wall))), kind="oracle",
                sample=(f"one whole FP64 oracle solve of the same workload ({res.iters} iterations, "
                        + (f"median of 3 after a warm-up solve, {wall * 1e3:.2f} ms wall" if nrep == 3 else
                           f"{wall:.1f} s wall") + f", {ncores} host cores visible, {cpu_model()})"),
                iters=res.iters, x=res.x,
                per_operator=ops)


def run_serving(args):
    """Poisson arrivals of mixed solves through the native server (FP32 transforms,
    FP64 Krylov): completed solves/s and p50/p99 latency from arrival to result."""
    from paper_2306_03574_amd.serve import run_trace
    import synth
    budget = int(args.budget_gb * (1 << 30))
    prec = args.prec or "fp32"
    # warm every shape class once (plans, workspaces and graphs are cached by the server)
    classes = sorted({(nx, ny, nt, a) for (nx, ny) in synth.workloads.SERVING_SHAPES for nt in synth.workloads.SERVING_NT
                      for a in synth.workloads.SERVING_ALPHA})
    log(f"serving: rate {args.rate}/s, {args.requests} requests, budget {args.budget_gb} GB, max_active {args.max_active}")
    out = None
    trace = synth.serving_trace(args.rate, args.requests, seed=5)
    results, wall = run_trace(trace, budget, max_active=args.max_active, prec=prec, tol=args.tol, maxit=args.maxit,
                              progress=log, warm_classes=classes, group_max_unknowns=args.group_lane)
    lat = np.array([r["latency"] for r in results]) * 1e3
    ok = sum(1 for r in results if r["status"] == 0 and r["relres"] <= args.tol)
    per_class = {}
    for tr, r in zip(trace, results):
        k = f"{'2d' if tr['ny'] else '1d'}_{tr['nx']}_nt{tr['nt']}"
        per_class.setdefault(k, []).append(r["latency"] * 1e3)
    out = {
        "metric": METRIC, "value": round(len(results) / wall, 3), "unit": "solves/s", "n_gpus": 1,
        "steps": len(results), "warmup": len(classes), "ms_per_step": round(wall / len(results) * 1e3, 3),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64-krylov/f32-transforms"
        if prec == "fp32" else "f64", "data": "synthetic",
        "config": {"workload": "serving_mix", "rate_per_s": args.rate, "requests": len(results),
                   "budget_gb": args.budget_gb, "max_active": args.max_active, "tol": args.tol,
                   "precond_precision": prec, "group_lane_max_unknowns": args.group_lane},
        "p50_ms": round(float(np.percentile(lat, 50)), 2), "p99_ms": round(float(np.percentile(lat, 99)), 2),
        "converged": ok,
        "per_class_p50_p99_ms": {k: [round(float(np.percentile(v, 50)), 2), round(float(np.percentile(v, 99)), 2),
                                     len(v)] for k, v in sorted(per_class.items())},
        "mean_iters": round(float(np.mean([r["iters"] for r in results])), 2),
    }
    print(json.dumps(out), flush=True)


def run_group_compare(args):
    """Time per MINRES iteration of mixed-grid groups (abac_group_*): one launch per step
    (advance) against one persistent launch (run) at several grid sizes.  Sources are
    random, the tolerance unreachable, so every iteration does the full work."""
    import torch
    from paper_2306_03574_amd import Plan, Group
    import synth
    DEV = torch.device("cuda:0")
    prec = args.prec or "fp32"
    grids = [int(x) for x in args.group_blocks.split(",")]
    K = args.steps
    out = {"metric": "group iteration time", "unit": "us per iteration", "prec": prec, "iterations": K,
           "higher_is_better": False, "data": "synthetic", "mixes": {}}
    for name in args.group_compare.split(","):
        cases = synth.workloads.GROUP_MIXES[name]
        log(f"group mix {name} ({len(cases)} members) {prec}")
        plans, fs, us = [], [], []
        for i, (nx, ny, nt, a) in enumerate(cases):
            p = Plan(nx, ny, nt, alpha=a, prec=prec, batch=1, device=DEV)
            src, z0, z1 = synth.random_source(nx, ny, nt, seed=50 + i)
            fs.append(p.build_rhs(torch.from_numpy(src[None]).to(DEV), torch.from_numpy(z0[None]).to(DEV),
                                  torch.from_numpy(z1[None]).to(DEV)))
            us.append(p.empty())
            plans.append(p)
        res = {}
        for mode in ["advance"] + [f"run{b}" for b in grids]:
            for p, f, u in zip(plans, fs, us):
                p.begin(f, u, tol=1e-30, maxit=1 << 20)
            g = Group(device=DEV)
            g.set(plans)
            blocks = None if mode == "advance" else int(mode[3:])
            step = (lambda k: g.advance(k)) if blocks is None else (lambda k: g.run(k, blocks=blocks))
            step(args.warmup)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            step(K)
            torch.cuda.synchronize()
            res[mode] = round((time.perf_counter() - t0) / K * 1e6, 1)
            if blocks is not None and g.check():
                raise RuntimeError(f"persistent launch of mix {name} gave up at a barrier")
            for p in plans:
                p.finish()
            g.close()
            log(f"  {mode}: {res[mode]} us per iteration")
        out["mixes"][name] = {"members": [list(c) for c in cases], "us_per_iteration": res}
    print(json.dumps(out), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="wave2d_511x511x512", choices=sorted(WORKLOADS))
    ap.add_argument("--prec", default=None, choices=["fp64", "fp32"])
    ap.add_argument("--alpha", type=float, default=None, help="override the workload's alpha")
    ap.add_argument("--tol", type=float, default=1e-8)
    ap.add_argument("--maxit", type=int, default=500)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-compare", action="store_true", help="skip the other-precision comparison leg")
    ap.add_argument("--rate", type=float, default=50.0, help="serving: Poisson arrival rate (req/s)")
    ap.add_argument("--requests", type=int, default=200, help="serving: requests in the trace")
    ap.add_argument("--budget-gb", type=float, default=160.0, help="serving: HBM budget")
    ap.add_argument("--max-active", type=int, default=16, help="serving: concurrent solves")
    ap.add_argument("--group-lane", type=int, default=0,
                    help="serving: requests with at most this many unknowns advance together in one group "
                         "(one launch per MINRES step for all of them); 0 = off")
    ap.add_argument("--copy-probe", action="store_true", help="only run the HBM counter calibration copy")
    ap.add_argument("--copy-gib", type=float, default=None, help="copy probe: buffer size in GiB (default 1)")
    ap.add_argument("--copy-pattern", default="copy", choices=["copy", "half"],
                    help="copy probe: a plain copy, or half-line reads at a 128-byte stride")
    ap.add_argument("--solver", default="minres", choices=["minres", "gmres"],
                    help="minres: Y T u = Y f with the ABAC preconditioner (the method); gmres: T u = f "
                         "right-preconditioned by the block alpha-circulant C_alpha")
    ap.add_argument("--restart", type=int, default=15, help="gmres: restart length (<= 15)")
    ap.add_argument("--group-compare", default=None,
                    help="only time groups of these mixes (comma-separated, synth.workloads.GROUP_MIXES): one "
                         "launch per step against one persistent launch; --steps iterations timed")
    ap.add_argument("--group-blocks", default="0,64,128,256",
                    help="group compare: persistent grid sizes (0 = the library's default)")
    args = ap.parse_args()
    if args.copy_probe:
        copy_probe(int(args.copy_gib * (1 << 30)) // 128 * 128 if args.copy_gib else None, args.copy_pattern)
        return
    if args.group_compare:
        run_group_compare(args)
        return
    if args.gpus != 1:
        print("bench.py measures one GPU: the solver runs on a single GPU and sharding one solve over "
              "several GPUs is not implemented. Run with --gpus 1.", file=sys.stderr)
        sys.exit(2)
    if args.workload == "serving_mix":
        run_serving(args)
        return
    w = dict(WORKLOADS[args.workload])
    if args.alpha is not None:
        w["alpha"] = args.alpha
    prec = args.prec or ("fp32" if args.workload == "wave2d_511x511x512" else "fp64")
    other = "fp32" if prec == "fp64" else "fp64"
    log(f"workload {args.workload} prec {prec} steps {args.steps} warmup {args.warmup}")
    main_run = run_gpu(w, prec, args.steps, args.warmup, args.tol, args.maxit, solver=args.solver,
                       restart=args.restart)
    log(f"{prec}: {args.steps / main_run['elapsed']:.2f} solves/s iters {main_run['iters'][:4]} "
        f"relres {max(main_run['relres']):.2e}")
    B = w["batch"]
    solves = args.steps * B
    value = solves / main_run["elapsed"]
    lat_ms = np.array(main_run["lat"]) * 1e3

    # roofline of the dominant kernel class over the timed region
    prof = main_run["prof"]
    if args.solver == "gmres":
        abytes = algorithmic_bytes_gmres(w, prec, main_run["prof_iters"], prof["time"]["launches"],
                                         args.steps * B)
    else:
        abytes = algorithmic_bytes(w, prec, main_run["prof_iters"], args.steps * B,
                                   fused=main_run["tiles"].get("small", 0) > 0)
    dom = max((k for k in prof if prof[k]["launches"] > 0 and k in abytes), key=lambda k: prof[k]["ms"])
    launches = prof[dom]["launches"]
    avg_s = prof[dom]["ms"] / 1e3 / launches
    bytes_per_launch = abytes.get(dom, 0) / launches
    achieved = bytes_per_launch / avg_s / 1e9
    roofline = {"bound": "hbm", "kernel": dom, "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": pmc_traffic(dom, args.workload, prec),
                "avg_launch_us": round(avg_s * 1e6, 2), "algorithmic_bytes_per_launch": int(bytes_per_launch),
                "timing": "HIP events around every launch on the plan stream, over a second pass of the same "
                          f"{args.steps} solves ({args.steps / main_run['prof_elapsed']:.2f} solves/s with events on)"}
    # the preconditioner apply as a whole (MINRES, separate kernels): every transform pass's
    # time and algorithmic bytes, and the floor-based effective rate (16 N bytes per apply:
    # read r, write z)
    pinv = None
    pinv_classes = [k for k in ("dstx_fwd", "dsty", "time", "dstx_inv") if prof.get(k, {}).get("launches")]
    if args.solver == "minres" and pinv_classes and "iter" not in abytes:
        t_s = sum(prof[k]["ms"] for k in pinv_classes) / 1e3
        b_alg = sum(abytes.get(k, 0) for k in pinv_classes)
        N = w["nt"] * w["nx"] * max(w["ny"], 1)   # per right-hand side
        applied = main_run["prof_iters"] + args.steps * B   # applies over all right-hand sides
        pinv = {"ms_total": round(t_s * 1e3, 3), "rhs_applies": applied,
                "achieved_GBs": round(b_alg / t_s / 1e9, 1),
                "frac": round(b_alg / t_s / 1e9 / HBM_PEAK_GBS, 4),
                "effective_frac": round(16 * N * applied / t_s / 1e9 / HBM_PEAK_GBS, 4),
                "note": "all transform passes of the preconditioner (Lanczos step and <q, p> fused in), "
                        "algorithmic bytes over their summed event time; effective_frac counts only 16 "
                        "bytes per unknown (read r, write z)"}
    kernel_table = {k: {"ms": round(v["ms"], 3), "launches": v["launches"],
                        "GB/s": round(abytes[k] / (v["ms"] / 1e3) / 1e9, 1) if k in abytes and v["ms"] > 0 else None}
                    for k, v in prof.items() if v["launches"]}

    out = {
        "metric": METRIC, "value": round(value, 3), "unit": "solves/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": round(main_run["elapsed"] / args.steps * 1e3, 3),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f64" if prec == "fp64" else "f64-krylov/f32-transforms", "data": "synthetic",
        "config": {"workload": args.workload, "nx": w["nx"], "ny": w["ny"], "nt": w["nt"], "T": 1.0,
                   "alpha": w["alpha"], "batch": B, "tol": args.tol, "precond_precision": prec,
                   "source": w["source"], "solver": args.solver if args.solver == "minres" else
                   f"gmres({args.restart}) on T u = f, right preconditioner C_alpha"},
        "p50_ms": round(float(np.percentile(lat_ms, 50)), 3), "p99_ms": round(float(np.percentile(lat_ms, 99)), 3),
        "iters": main_run["iters"][:8], "relres_max": max(main_run["relres"]),
        "roofline": roofline, "kernels": kernel_table,
    }
    if pinv:
        out["preconditioner_apply"] = pinv
    if not args.no_compare:
        log(f"comparison leg: {other}")
        cmp_run = run_gpu(w, other, max(3, args.steps // 2), 1, args.tol, args.maxit, profile=False,
                          solver=args.solver, restart=args.restart)
        cmp_val = max(3, args.steps // 2) * B / cmp_run["elapsed"]
        diff = float(np.max(np.abs(cmp_run["u"] - main_run["u"])) / np.max(np.abs(main_run["u"])))
        out[f"{other}_precond"] = {"value": round(cmp_val, 3), "unit": "solves/s", "iters": cmp_run["iters"][:8],
                                   "relres_max": max(cmp_run["relres"]), "rel_diff_vs_" + prec: diff}
    gold = golden_oracle(args.workload)
    if gold is not None and (gold["alpha"] != w["alpha"] or gold["tol"] != args.tol or args.solver != "minres"):
        gold = None
    if gold is not None:
        # the stored oracle solve of this workload: its count, and the GPU iterate at the
        # stored entries against the oracle's
        idx = np.array(gold["index"])
        err = float(np.max(np.abs(main_run["u"][0].reshape(-1)[idx] - np.array(gold["x"]))) / gold["x_maxabs"])
        out["oracle_iters"] = gold["iters"]
        out["gpu_vs_oracle_rel_err_sampled"] = err
    if not args.no_cpu_baseline:
        log("cpu baseline: the oracle on the host")
        cb = cpu_baseline(w, args.tol, args.maxit, args.solver, args.restart,
                          full_iters=gold["iters"] if gold is not None else None)
        out["cpu_baseline"] = {k: cb[k] for k in ("value", "unit", "cores", "kind", "sample")}
        if cb["per_operator"]:
            out["cpu_baseline"]["per_operator_s"] = cb["per_operator"]
        out["cpu_baseline"]["value"] = round(cb["value"], 6)
        if cb["x"] is not None:
            out["gpu_vs_oracle_rel_err"] = float(np.max(np.abs(main_run["u"][0] - cb["x"])) / np.max(np.abs(cb["x"])))
            out["oracle_iters"] = cb["iters"]
    # FP32 transforms against the FP64 oracle's count (the +2 bar), per result
    if "oracle_iters" in out and args.solver == "minres":
        legs = {prec: main_run["iters"][0]}
        if f"{other}_precond" in out:
            legs[other] = out[f"{other}_precond"]["iters"][0]
        if "fp32" in legs:
            out["fp32_iters_vs_oracle"] = {"fp32": legs["fp32"], "oracle_fp64": out["oracle_iters"],
                                           "within_2": legs["fp32"] <= out["oracle_iters"] + 2}
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
