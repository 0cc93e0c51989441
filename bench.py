#!/usr/bin/env python3
"""Solves/s of the LS-AMG-DD solve phase on one MI355X.

Workload: 2D rotated anisotropic diffusion in least-squares form, N = 512
cells per side (261,121 unknowns, 524,286 rows of G), theta = pi/6,
eps = 1e-4, right-hand side uniform[-1,1] from seed 1; hierarchy of
Algorithm 1 with 4x4 lattice aggregates, one-layer overlap, threshold rule
with c_min = 2 on every level, coarsened until below 2000 unknowns.

One step = one whole solve: FP64 preconditioned CG to 1e-8 relative residual
from x0 = 0, one V-cycle per iteration (RAS, G^T(G x) residuals, P^T / P,
dense coarsest inverse, RAS-T).  The headline value is the mixed-precision
path (FP32 V-cycle, FP64 CG); the plain FP64 V-cycle is timed beside it.
Inputs are resident in HBM when the timed region starts; setup is excluded.

Printed: one JSON line with the headline numbers, the live roofline of the
dominant kernel (HIP events on the library's stream) and the CPU oracle
baseline (a bounded sample of the same solve on the host cores).
"""
import argparse
import json
import math
import os
import subprocess
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0          # MI355X HBM3E, published
METRIC = "solves/s to 1e-8 rel. residual (mixed vs FP64 V-cycle); p50/p99 latency"


def cpu_baseline_cmd(N: int, iters: int):
    code = f"""
import json, os, sys, time
sys.path.insert(0, {ROOT!r})
import numpy as np
import oracle as O
import problems as P
prob = P.config2({N})
t0 = time.time()
H = O.setup(prob.G, 2, prob.grid, O.Params(cmin=(2,)))
t_setup = time.time() - t0
b = P.rhs_uniform(prob.n, P.CONFIG_RHS_SEED[2])
t0 = time.time()
x, info = O.pcg(H, b, tol=0.0, fixed_iters={iters})
t = time.time() - t0
print(json.dumps(dict(t_setup=t_setup, t_sample=t, iters={iters})))
"""
    return [sys.executable, "-c", code]


def percentile(v, q):
    v = sorted(v)
    if not v:
        return float("nan")
    k = (len(v) - 1) * q
    lo, hi = math.floor(k), math.ceil(k)
    return v[lo] + (v[hi] - v[lo]) * (k - lo)


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--N", type=int, default=512)
    ap.add_argument("--cpu-iters", type=int, default=2,
                    help="PCG iterations of the oracle's timed sample")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU: this build has no multi-GPU path "
              "(the per-GPU shard would be a block of aggregates; see the "
              "design notes). Run with --gpus 1.", file=sys.stderr)
        sys.exit(2)

    # CPU oracle baseline runs in a child process on the host cores while the
    # GPU part runs (single-threaded BLAS: it uses one core)
    cpu_proc = None
    if not args.no_cpu_baseline:
        env = dict(os.environ, OMP_NUM_THREADS="1", OPENBLAS_NUM_THREADS="1",
                   MKL_NUM_THREADS="1")
        cpu_proc = subprocess.Popen(cpu_baseline_cmd(args.N, args.cpu_iters),
                                    stdout=subprocess.PIPE, stderr=subprocess.PIPE,
                                    text=True, env=env)

    import torch
    import problems as P
    from paper_2601_04112_amd import lsamg as L

    prob = P.config2(args.N)
    t0 = time.time()
    s = L.Solver(prob.G, 2, prob.grid, device=0, cmin=(2,))
    t_setup = time.time() - t0
    inf = s.info()
    b = torch.tensor(P.rhs_uniform(prob.n, P.CONFIG_RHS_SEED[2]), dtype=torch.float64,
                     device="cuda:0")
    x = torch.empty_like(b)
    stream = torch.cuda.current_stream()

    def timed(prec, steps, warmup, only=None):
        s.set_precision(prec)
        for _ in range(warmup):
            s.solve(b, tol=1e-8, out=x)
        if only is not None:
            s.profile(True, only)
        torch.cuda.synchronize()
        lat = []
        t_start = time.perf_counter()
        for _ in range(steps):
            t1 = time.perf_counter()
            _, st = s.solve(b, tol=1e-8, out=x)
            lat.append((time.perf_counter() - t1) * 1e3)
        torch.cuda.synchronize()
        elapsed = time.perf_counter() - t_start
        kp = s.profile_read() if only is not None else []
        if only is not None:
            s.profile(False)
        return dict(solves_per_s=steps / elapsed, ms_per_step=elapsed * 1e3 / steps,
                    p50_ms=percentile(lat, 0.5), p99_ms=percentile(lat, 0.99),
                    iters=st[0]["iters"], true_rel_res=st[0]["true_rel_res"],
                    converged=bool(st[0]["converged"])), kp

    # untimed pass over every kernel: find the dominant kernel of the mixed path
    s.set_precision(L.MIXED)
    s.solve(b, tol=1e-8, out=x)
    s.profile(True)
    s.solve(b, tol=1e-8, out=x)
    allk = sorted(s.profile_read(), key=lambda r: -r["ms"])
    s.profile(False)
    dominant = allk[0]["name"]
    ktotal = sum(r["ms"] for r in allk)

    mixed, kp = timed(L.MIXED, args.steps, args.warmup, only=dominant)
    fp64, _ = timed(L.FP64, args.steps, args.warmup)
    dom = next((r for r in kp if r["name"] == dominant), None)
    roofline = None
    if dom and dom["launches"] > 0 and dom["ms"] > 0:
        avg_s = dom["ms"] / dom["launches"] * 1e-3
        bytes_per_launch = dom["bytes"] / dom["launches"]
        achieved = bytes_per_launch / avg_s / 1e9
        roofline = dict(bound="hbm", achieved=round(achieved, 1), peak=HBM_PEAK_GBS,
                        unit="GB/s", frac=round(achieved / HBM_PEAK_GBS, 4),
                        traffic=None, kernel=dominant,
                        avg_launch_us=round(avg_s * 1e6, 3),
                        algorithmic_bytes_per_launch=int(bytes_per_launch),
                        launches=dom["launches"],
                        share_of_kernel_time=round(allk[0]["ms"] / ktotal, 3))

    cpu = None
    if cpu_proc is not None:
        out, err = cpu_proc.communicate(timeout=1800)
        if cpu_proc.returncode == 0:
            r = json.loads(out.strip().splitlines()[-1])
            # a solve = the initial V-cycle plus `iters` iterations each with one
            # A-apply and one V-cycle; the sample ran cpu_iters of them
            per_solve = r["t_sample"] * (fp64["iters"] + 1) / (r["iters"] + 1)
            cpu = dict(value=round(1.0 / per_solve, 6), unit="solves/s", cores=1,
                       kind="oracle",
                       sample=(f"{r['iters']} PCG iterations ({r['iters'] + 1} V-cycles) of "
                               f"the same solve, scaled to {fp64['iters']} iterations; "
                               f"oracle setup {r['t_setup']:.0f} s untimed; 1 thread"),
                       sample_seconds=round(r["t_sample"], 2))
        else:
            cpu = dict(value=None, unit="solves/s", cores=1, kind="oracle",
                       sample="failed: " + err.strip().splitlines()[-1][:200])

    smoother_entries = sum(l["smoother_entries"] for l in inf["levels"])
    line = {
        "metric": METRIC,
        "value": round(mixed["solves_per_s"], 3),
        "unit": "solves/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(mixed["ms_per_step"], 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32 V-cycle / f64 CG",
        "data": "synthetic",
        "config": {
            "workload": (f"aniso2d N={args.N} theta=pi/6 eps=1e-4 (n={prob.n}, "
                         f"m={prob.m}), rhs uniform[-1,1] seed 1, tol 1e-8, "
                         f"4x4 aggregates, c_min=2, coarsest<2000"),
            "levels": inf["nlevels"],
            "n_per_level": [l["n"] for l in inf["levels"]],
            "op_complexity": round(inf["op_complexity"], 3),
            "smoother_complexity": round(inf["smoother_complexity"], 3),
            "smoother_entries": smoother_entries,
            "setup_s": round(t_setup, 2),
            "parallelism": "single GPU",
        },
        "p50_ms": round(mixed["p50_ms"], 3),
        "p99_ms": round(mixed["p99_ms"], 3),
        "iters": mixed["iters"],
        "true_rel_res": mixed["true_rel_res"],
        "vcycles_per_s": round(mixed["solves_per_s"] * (mixed["iters"] + 1), 1),
        "fp64": {k: (round(v, 4) if isinstance(v, float) else v) for k, v in fp64.items()},
        "mixed_vs_fp64_speedup": round(mixed["solves_per_s"] / fp64["solves_per_s"], 3),
        "top_kernels": [dict(name=r["name"], ms_per_solve=round(r["ms"], 3),
                             launches=r["launches"],
                             gbs=round(r["bytes"] / (r["ms"] * 1e-3) / 1e9, 1))
                        for r in allk[:6]],
        "roofline": roofline,
        "cpu_baseline": cpu,
    }
    print(json.dumps(line))


if __name__ == "__main__":
    main()
