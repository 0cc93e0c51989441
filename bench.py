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


def cpu_baseline_cmd(N: int, reps: int):
    """The oracle's solve phase in its assembled form (one CSR smoother per
    level, its transpose for RAS-T, CSR A_l and P_l, the coarsest Cholesky
    factor), timed on the host cores.  The child builds the hierarchy while
    the GPU part runs, reports, then waits for a line on stdin before it
    times one warm-up solve and `reps` solves to 1e-8, so the timed region
    has the host to itself."""
    code = f"""
import json, os, platform, sys, time
sys.path.insert(0, {ROOT!r})
import numpy as np
import oracle as O
import problems as P
prob = P.config2({N})
t0 = time.time()
H = O.setup(prob.G, 2, prob.grid, O.Params(cmin=(2,), compress_rows=True))
t_setup = time.time() - t0
t0 = time.time()
AV = O.AssembledVcycle(H)
t_asm = time.time() - t0
b = P.rhs_uniform(prob.n, P.CONFIG_RHS_SEED[2])
print(json.dumps(dict(ready=True, t_setup=t_setup, t_assemble=t_asm)), flush=True)
sys.stdin.readline()
O.pcg(H, b, tol=1e-8, precond=AV)
times, iters = [], []
for _ in range({reps}):
    t = time.perf_counter()
    x, info = O.pcg(H, b, tol=1e-8, precond=AV)
    times.append(time.perf_counter() - t)
    iters.append(info["iters"])
try:
    from threadpoolctl import threadpool_info
    blas = [d for d in threadpool_info() if d.get("user_api") == "blas"]
    blas_threads = max(d.get("num_threads", 1) for d in blas) if blas else 1
    blas_name = blas[0].get("internal_api", "?") if blas else "?"
except Exception:
    blas_threads, blas_name = 1, "?"
model = "?"
try:
    for ln in open("/proc/cpuinfo"):
        if ln.startswith("model name"):
            model = ln.split(":", 1)[1].strip()
            break
except OSError:
    pass
print(json.dumps(dict(t_setup=t_setup, t_assemble=t_asm, times=times, iters=iters,
                      blas_threads=blas_threads, blas=blas_name, cpu_model=model,
                      cpu_count=os.cpu_count(), affinity=len(os.sched_getaffinity(0)),
                      true_rel_res=info["true_rel_res"])), flush=True)
"""
    return [sys.executable, "-c", code]


def source_hash(rel_path: str) -> str:
    """First 16 hex digits of the SHA-256 of a repository file."""
    import hashlib
    with open(os.path.join(ROOT, rel_path), "rb") as fh:
        return hashlib.sha256(fh.read()).hexdigest()[:16]


def measured_traffic(kernel: str):
    """HBM bytes per launch of `kernel` from the committed counter summary
    (profiles/*_traffic.md: FETCH_SIZE and WRITE_SIZE per dispatch, scaled by
    the counters' reading for a plain streaming kernel of known size), or
    None when no summary covers this kernel or the source file that defines
    it changed since the counters were taken."""
    import glob
    for f in sorted(glob.glob(os.path.join(ROOT, "profiles", "*_traffic.md"))):
        txt = open(f).read()
        if "```json" not in txt:
            continue
        rec = json.loads(txt.split("```json", 1)[1].split("```", 1)[0])
        if (rec.get("kernel") == kernel and rec.get("source_file")
                and rec.get("source_sha256") == source_hash(rec["source_file"])):
            return rec["traffic_bytes_per_launch"]
    return None


def method_bytes(inf, s: int):
    """Bytes the method itself moves per PCG iteration, from the hierarchy's
    sizes: per V-cycle level, both smoothers read the local-inverse rows
    (2 s sum|omega||Omega|), two fused A-applies read G_l (nnz (s+4) + 4 m)
    and two vectors each, P^T and P read P_l, plus about six vector passes;
    the coarsest level reads its dense inverse once; each iteration adds a
    fused FP64 A-apply and about ten FP64 vector passes.  Levels that the
    library applies as one dense operator (the dense tail) are counted by
    these, the method's own, steps.  s = bytes per V-cycle scalar."""
    lv = inf["levels"]
    per = []
    for l, L in enumerate(lv):
        if l == inf["nlevels"] - 1:
            per.append(s * L["n"] ** 2)
        else:
            per.append(2 * s * L["smoother_entries"]
                       + 2 * (L["g_nnz"] * (s + 4) + 4 * L["g_rows"] + 2 * s * L["n"])
                       + 2 * s * L["p_entries"] + 6 * s * L["n"])
    L0 = lv[0]
    cg = L0["g_nnz"] * 12 + 4 * L0["g_rows"] + 16 * L0["n"] + 80 * L0["n"]
    return sum(per) + cg, per, cg


def percentile(v, q):
    v = sorted(v)
    if not v:
        return float("nan")
    k = (len(v) - 1) * q
    lo, hi = math.floor(k), math.ceil(k)
    return v[lo] + (v[hi] - v[lo]) * (k - lo)


def run_serving(args):
    """Request stream: Poisson arrivals at each rate of args.qps, operators
    drawn from a seeded pool of args.pool distinct 2D problems (N in
    {64,...,1024}, theta ~ U[0, pi), log10 eps ~ U[-6, 0]), 1-8 right-hand
    sides each, FP32 V-cycle under FP64 CG to 1e-8.  Hierarchies stay
    resident (HBM budget args.budget_gb); a request for an operator whose
    solve is running joins it at the next PCG iteration boundary.  With
    several rates the same server (and its resident hierarchies) serves one
    stream per rate, one after another."""
    import numpy as np
    import problems as P
    from paper_2601_04112_amd import lsamg as L

    rng = np.random.default_rng(5)
    sizes = [64, 128, 256, 512, 1024]
    pool = []
    for k in range(args.pool):
        N = int(rng.choice(sizes))
        pool.append((N, float(rng.uniform(0, math.pi)), float(10 ** rng.uniform(-6, 0))))
    probs = {}
    srv = L.Server(hbm_budget=int(args.budget_gb * (1 << 30)), max_slots=args.slots)
    t_warm = 0.0
    warm = []
    if args.prewarm:
        # steady state: one request per pool operator first, so every hierarchy
        # is resident before the clock starts (their setup is reported apart);
        # it carries --prewarm-rhs columns, so the multi-right-hand-side
        # buffers of the widths the solves use are allocated and their
        # matrix-core shapes tuned before the clock starts too
        tw = time.perf_counter()
        for k in range(args.pool):
            probs[k] = P.aniso2d(*pool[k])
            bw = np.stack([P.rhs_uniform(probs[k].n, 7 + j) for j in range(args.prewarm_rhs)])
            srv.submit(k, probs[k].G, 2, probs[k].grid, bw,
                       tol=1e-8, precision=L.MIXED, req_id=10 ** 6 + k, cmin=(2,),
                       setup_device=args.setup)
        got = 0
        warm = []
        while got < args.pool:
            ds = srv.poll(wait_ms=1000)
            got += len(ds)
            for d in ds:
                k = d["id"] - 10 ** 6
                warm.append(dict(N=pool[k][0], setup_s=round(d["t_setup"], 1), status=d["status"]))
                print(f"[serve] prewarm {got}/{args.pool}: N={pool[k][0]} setup "
                      f"{d['t_setup']:.1f} s status {d['status']} {d['msg']}",
                      file=sys.stderr, flush=True)
        t_warm = time.perf_counter() - tw
    sweep = []
    next_id = 0
    for qps in [float(q) for q in str(args.qps).split(",")]:
        rq = np.random.default_rng(int(5 + 1000 * qps))
        reqs = []
        t = 0.0
        for i in range(args.requests):
            t += float(rq.exponential(1.0 / qps))
            reqs.append((t, int(rq.integers(args.pool)), int(rq.integers(1, 9)), 10000 + 8 * i))
        st0 = srv.stats()
        done = {}
        t0 = time.perf_counter()
        t_report = t0
        i = 0
        while len(done) < len(reqs):
            now = time.perf_counter() - t0
            while i < len(reqs) and reqs[i][0] <= now:
                _, k, nr, seed = reqs[i]
                if k not in probs:
                    probs[k] = P.aniso2d(*pool[k])
                p = probs[k]
                b = np.stack([P.rhs_uniform(p.n, seed + j) for j in range(nr)])
                srv.submit(k, p.G, 2, p.grid, b, tol=1e-8, precision=L.MIXED,
                           req_id=next_id + i, cmin=(2,), setup_device=args.setup)
                i += 1
            wait = 5 if i >= len(reqs) else max(0, int((reqs[i][0] - now) * 1e3))
            for d in srv.poll(wait_ms=min(wait, 20)):
                d.pop("x")
                done[d["id"]] = d
            if time.perf_counter() - t_report > 5.0:
                t_report = time.perf_counter()
                print(f"[serve] qps {qps:g} t={t_report - t0:.0f}s submitted {i}/{len(reqs)} "
                      f"done {len(done)}", file=sys.stderr, flush=True)
        makespan = time.perf_counter() - t0
        next_id += len(reqs)
        st = srv.stats()
        lat = [d["t_total"] * 1e3 for d in done.values()]
        hit_lat = [d["t_total"] * 1e3 for d in done.values() if d["cache_hit"]]
        solve_lat = [(d["t_queue"] + d["t_solve"]) * 1e3 for d in done.values()]
        nrhs_total = sum(r[2] for r in reqs)
        ok = sum(1 for d in done.values() if d["status"] == 0)
        status_counts = {}
        errors = {}
        for d in done.values():
            status_counts[str(d["status"])] = status_counts.get(str(d["status"]), 0) + 1
            if d["status"] != 0 and d["msg"]:
                errors[d["msg"]] = errors.get(d["msg"], 0) + 1
        sweep.append({
            "qps": qps, "value": round(nrhs_total / makespan, 2), "unit": "solves/s",
            "requests": len(reqs), "rhs_total": nrhs_total, "makespan_s": round(makespan, 2),
            "ok": ok, "status_counts": status_counts, "errors": errors,
            "p50_ms": round(percentile(lat, 0.5), 2), "p99_ms": round(percentile(lat, 0.99), 2),
            "p50_ms_hit": round(percentile(hit_lat, 0.5), 2) if hit_lat else None,
            "p99_ms_hit": round(percentile(hit_lat, 0.99), 2) if hit_lat else None,
            "p50_ms_excl_setup": round(percentile(solve_lat, 0.5), 2),
            "p99_ms_excl_setup": round(percentile(solve_lat, 0.99), 2),
            "joined_running_solve": sum(1 for d in done.values() if d["joined_at"] > 0),
            "max_true_rel_res": max(d["true_rel_res_max"] for d in done.values()),
            "max_batch_rhs": max(d["batch_rhs"] for d in done.values()),
            "misses": st["misses"] - st0["misses"], "evictions": st["evictions"] - st0["evictions"],
            "pcg_iterations": st["iterations"] - st0["iterations"],
            "setup_s_total": round(sum(d["t_setup"] for d in done.values()), 1)})
        print(f"[serve] qps {qps:g}: {sweep[-1]['value']} solves/s, p50 {sweep[-1]['p50_ms']} ms, "
              f"p99 {sweep[-1]['p99_ms']} ms", file=sys.stderr, flush=True)
    st = srv.stats()
    srv.close()
    head = sweep[0]
    line = {
        "metric": "serving: solves/s and p50/p99 latency, 1e-8 rel. residual",
        "value": head["value"], "unit": "solves/s", "qps": head["qps"],
        "p50_ms": head["p50_ms"], "p99_ms": head["p99_ms"], "sweep": sweep,
        "server": st, "pool": args.pool, "slots": args.slots,
        "prewarm_s": round(t_warm, 1) if args.prewarm else None,
        "prewarm": warm if args.prewarm else None,
        "dtype": "f32 V-cycle / f64 CG", "data": "synthetic",
        "config": {"workload": f"{args.requests} Poisson requests per rate over a pool of "
                               f"{args.pool} aniso2d operators, N in {sizes}, theta~U[0,pi), "
                               f"log10 eps~U[-6,0], 1-8 rhs"
                               + (f", hierarchies resident and tuned ({args.prewarm_rhs}-column "
                                  f"request each) before the clock starts"
                                  if args.prewarm else "")},
    }
    print(json.dumps(line))


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", choices=("aniso2d", "ls3d"), default="aniso2d",
                    help="aniso2d: 2D rotated anisotropy (default); ls3d: 3D "
                         "A = D1 + B^T D2^-1 B on a 128^3 grid")
    ap.add_argument("--N", type=int, default=0,
                    help="cells per side (default 512 for aniso2d, 128 for ls3d)")
    ap.add_argument("--cpu-reps", type=int, default=3,
                    help="timed oracle solves of the CPU baseline (after one warm-up)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--batch", type=int, default=64,
                    help="right-hand sides of the batched workload (0: skip)")
    ap.add_argument("--serve", action="store_true",
                    help="run the request-stream serving benchmark instead")
    ap.add_argument("--qps", default="50",
                    help="serving: request rate(s) per second, comma-separated for a sweep")
    ap.add_argument("--requests", type=int, default=1024)
    ap.add_argument("--pool", type=int, default=16)
    ap.add_argument("--slots", type=int, default=4)
    ap.add_argument("--budget-gb", type=float, default=160.0)
    ap.add_argument("--prewarm", action="store_true",
                    help="serving: make every pool operator resident before timing")
    ap.add_argument("--prewarm-rhs", type=int, default=64,
                    help="serving: right-hand sides of each operator's prewarm request")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MIB",
                    help="before the solves, negate a float32 buffer of this many MiB "
                         "into another (a plain streaming kernel of known bytes, the "
                         "reference for hardware byte counters)")
    ap.add_argument("--cmin", default="2",
                    help="aniso2d: minimum coarsening ratio per level (LS_{a,b,...} of "
                         "sec. 3.4), comma-separated, the last repeats")
    ap.add_argument("--batch-krylov", choices=("cg", "fcg", "block"), default="cg",
                    help="outer iteration of the batched legs: per-column CG, flexible "
                         "CG, or block CG over the batch")
    ap.add_argument("--omega-max", type=int, default=800,
                    help="aniso2d: coarse aggregates of at most this many unknowns")
    ap.add_argument("--cycle", choices=("v", "additive"), default="v",
                    help="aniso2d: the multiplicative V-cycle or the additive cycle of "
                         "sec. 3.1.1 (single right-hand sides only)")
    ap.add_argument("--setup", choices=("auto", "device", "host"), default="auto",
                    help="where the setup's dense local problems run (untimed): "
                         "batched on the GPU, on the host's cores, or (auto) on "
                         "the GPU from 100,000 unknowns on")
    ap.add_argument("--verbose-setup", action="store_true",
                    help="per-level setup lines on stderr (always on for ls3d)")
    ap.add_argument("--maxit", type=int, default=0,
                    help="PCG iteration cap (default 1000; 200 for ls3d)")
    args = ap.parse_args()
    if args.serve:
        if args.gpus != 1:
            sys.exit(2)
        run_serving(args)
        return
    three_d = args.workload == "ls3d"
    if args.N == 0:
        args.N = 128 if three_d else 512
    if args.maxit == 0:
        args.maxit = 200 if three_d else 1000
    if three_d:
        # the oracle's Python setup of a 2M-unknown hierarchy takes hours, and
        # the multi-right-hand-side section is defined on the 2D operator
        args.no_cpu_baseline = True
        args.batch = 0
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU: this build has no multi-GPU path "
              "(the per-GPU shard would be a block of aggregates; see the "
              "design notes). Run with --gpus 1.", file=sys.stderr)
        sys.exit(2)

    # CPU oracle baseline: its setup runs in a child process while the GPU
    # part runs; its timed solves run after the GPU part (BLAS on every core
    # the host gives it)
    cmin = tuple(int(c) for c in str(args.cmin).split(","))
    if cmin != (2,) or args.cycle != "v" or args.omega_max != 800:
        args.no_cpu_baseline = True         # the oracle baseline runs the default method
    if args.cycle != "v":
        args.batch = 0                      # the additive cycle solves columns one by one
    cpu_proc = None
    if not args.no_cpu_baseline:
        cpu_proc = subprocess.Popen(cpu_baseline_cmd(args.N, args.cpu_reps),
                                    stdin=subprocess.PIPE, stdout=subprocess.PIPE,
                                    stderr=subprocess.PIPE, text=True)

    import torch
    import problems as P
    from paper_2601_04112_amd import lsamg as L

    t0 = time.time()
    if three_d:
        prob = P.config3(args.N)
        print(f"ls3d N={args.N}: n={prob.n}, m={prob.m}, nnz={prob.G.nnz}; setup ...",
              file=sys.stderr, flush=True)
        s = L.Solver(prob.G, 3, prob.grid, device=0, block=3, cmin=(3, 4), verbose=True,
                     setup_device=args.setup)
        seed = P.CONFIG_RHS_SEED[3]
    else:
        prob = P.config2(args.N)
        s = L.Solver(prob.G, 2, prob.grid, device=0, cmin=cmin, cycle=args.cycle,
                     omega_max=args.omega_max, setup_device=args.setup,
                     verbose=args.verbose_setup)
        seed = P.CONFIG_RHS_SEED[2]
    t_setup = time.time() - t0
    print(f"setup {t_setup:.1f} s", file=sys.stderr, flush=True)
    inf = s.info()
    if args.copy_calibration > 0:
        src = torch.rand(args.copy_calibration << 18, device="cuda:0")
        dst = torch.empty_like(src)
        torch.neg(src, out=dst)
        torch.cuda.synchronize()
        del src, dst
    b = torch.tensor(P.rhs_uniform(prob.n, seed), dtype=torch.float64, device="cuda:0")
    x = torch.empty_like(b)
    stream = torch.cuda.current_stream()

    def timed(prec, steps, warmup, only=None):
        s.set_precision(prec)
        for _ in range(warmup):
            s.solve(b, tol=1e-8, out=x, maxit=args.maxit)
        if only is not None:
            s.profile(True, only, by_level=" @L" in only)
        torch.cuda.synchronize()
        lat = []
        t_start = time.perf_counter()
        for _ in range(steps):
            t1 = time.perf_counter()
            _, st = s.solve(b, tol=1e-8, out=x, maxit=args.maxit)
            lat.append((time.perf_counter() - t1) * 1e3)
        torch.cuda.synchronize()
        elapsed = time.perf_counter() - t_start
        kp = s.profile_read() if only is not None else []
        if only is not None:
            s.profile(False)
        return dict(solves_per_s=steps / elapsed, ms_per_step=elapsed * 1e3 / steps,
                    p50_ms=percentile(lat, 0.5), p99_ms=percentile(lat, 0.99),
                    iters=st[0]["iters"], true_rel_res=st[0]["true_rel_res"],
                    converged=bool(st[0]["converged"]),
                    ms_per_iteration=elapsed * 1e3 / steps / max(1, st[0]["iters"])), kp

    # untimed pass over every kernel and level: the dominant kernel of the
    # mixed path is the one operator (kernel at one level) with the most time;
    # each kernel's algorithmic bytes (the library's per-launch formula) over
    # its time
    s.set_precision(L.MIXED)
    s.solve(b, tol=1e-8, out=x, maxit=args.maxit)
    s.profile(True, by_level=True)
    s.solve(b, tol=1e-8, out=x, maxit=args.maxit)
    byl = sorted(s.profile_read(), key=lambda r: -r["ms"])
    s.profile(False)
    allk = byl
    dominant = byl[0]["name"]
    ktotal = sum(r["ms"] for r in byl)
    kernel_fracs = [dict(name=r["name"], us_per_launch=round(r["ms"] / r["launches"] * 1e3, 2),
                         gbs=round(r["bytes"] / (r["ms"] * 1e-3) / 1e9, 1),
                         frac=round(r["bytes"] / (r["ms"] * 1e-3) / 1e9 / HBM_PEAK_GBS, 3),
                         share=round(r["ms"] / ktotal, 3))
                    for r in byl[:16] if r["launches"] and r["ms"] > 0]

    # timed region: the dominant kernel's launches carry HIP events (so the
    # V-cycle is launched kernel by kernel); the same solve replaying its
    # V-cycle from a HIP graph is timed next, without events
    mixed, kp = timed(L.MIXED, args.steps, args.warmup, only=dominant)
    print(f"mixed {mixed['solves_per_s']:.2f} solves/s", file=sys.stderr, flush=True)
    mixed_graph, _ = timed(L.MIXED, args.steps, args.warmup)
    print(f"mixed (graph) {mixed_graph['solves_per_s']:.2f} solves/s", file=sys.stderr, flush=True)
    fp64, _ = timed(L.FP64, args.steps, args.warmup)
    print(f"fp64 {fp64['solves_per_s']:.2f} solves/s", file=sys.stderr, flush=True)

    # batched workload: the same operator with 64 right-hand sides (seeds
    # 100-163) solved together, one FP64 CG per column, with the FP32
    # V-cycle and again with the FP64 one
    def run_batched(prec, peak, steps):
        import numpy as np
        B = torch.tensor(np.stack([P.rhs_uniform(prob.n, 100 + j) for j in range(args.batch)]),
                         dtype=torch.float64, device="cuda:0")
        XB = torch.empty_like(B)
        s.set_precision(prec)
        s.set_option(L.OPT_KRYLOV, {"cg": L.KRYLOV_CG, "fcg": L.KRYLOV_FCG,
                                    "block": L.KRYLOV_BLOCK}[args.batch_krylov])
        s.solve(B, tol=1e-8, out=XB)     # first batched solve: autotunes the MFMA tiles
        s.profile(True, by_level=True)
        s.solve(B, tol=1e-8, out=XB)
        bkl = s.profile_read()
        s.profile(False)
        merged = {}
        for r in bkl:
            nm = r["name"].split(" @L")[0]
            m = merged.setdefault(nm, dict(name=nm, ms=0.0, launches=0, bytes=0.0))
            m["ms"] += r["ms"]
            m["launches"] += r["launches"]
            m["bytes"] += r["bytes"]
        bk = sorted(merged.values(), key=lambda r: -r["ms"])
        # matrix-core utilisation of the dense level's GEMM (2 n^2 NB flops)
        mfma = None
        lt = inf["tail_level"] if inf["tail_level"] >= 0 else inf["nlevels"] - 1
        nt = inf["levels"][lt]["n"]
        for r in bkl:
            if (r["name"].startswith("k_bmm<") or r["name"].startswith("k_dense_mm64")
                    or r["name"].startswith("k_bgemm<")) \
                    and r["name"].endswith(f"@L{lt}") and r["launches"]:
                us = r["ms"] / r["launches"] * 1e3
                tf = 2.0 * nt * nt * args.batch / (us * 1e-6) / 1e12
                mfma = dict(kernel=r["name"], n=nt, nrhs=args.batch, avg_launch_us=round(us, 2),
                            achieved=round(tf, 2), peak=peak, unit="TFLOP/s",
                            frac=round(tf / peak, 4))
        # matrix-core rate of the aggregate-block products on levels 1-2
        # (RAS, P^T, P, RAS-T as per-aggregate GEMMs of 64 columns)
        mfma_levels = []
        for r in bkl:
            nm = r["name"]
            if (r["flops"] > 0 and r["launches"] and (" @L1" in nm or " @L2" in nm)
                    and nm.split("<")[0] in ("k_bmm", "k_bmm_lds", "k_bmmd", "k_bmmd_lds", "k_bgemm")):
                us = r["ms"] / r["launches"] * 1e3
                tf = r["flops"] / (r["ms"] * 1e-3) / 1e12
                mfma_levels.append(dict(kernel=nm, avg_launch_us=round(us, 2),
                                        gflop_per_launch=round(r["flops"] / r["launches"] / 1e9, 3),
                                        achieved=round(tf, 2), peak=peak, unit="TFLOP/s",
                                        frac=round(tf / peak, 4),
                                        gbs=round(r["bytes"] / (r["ms"] * 1e-3) / 1e9, 1)))
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        for _ in range(steps):
            _, bst = s.solve(B, tol=1e-8, out=XB)
        torch.cuda.synchronize()
        el = time.perf_counter() - t1
        its = [r["iters"] for r in bst]
        s.set_option(L.OPT_KRYLOV, L.KRYLOV_CG)
        return dict(nrhs=args.batch, krylov=args.batch_krylov,
                    solves_per_s=round(args.batch * steps / el, 2),
                    ms_per_batch=round(el * 1e3 / steps, 3), steps=steps,
                    iters_min=min(its), iters_max=max(its),
                    all_converged=all(r["converged"] for r in bst),
                    max_true_rel_res=max(r["true_rel_res"] for r in bst),
                    mfma_dense=mfma, mfma_levels_1_2=mfma_levels,
                    top_kernels=[dict(name=r["name"], ms_per_batch=round(r["ms"], 3),
                                      launches=r["launches"],
                                      gbs=round(r["bytes"] / (r["ms"] * 1e-3) / 1e9, 1))
                                 for r in bk[:6]])

    batched = batched64 = None
    if args.batch > 0:
        batched = run_batched(L.MIXED, 157.3, max(2, args.steps // 4))
        print(f"batched mixed {batched['solves_per_s']:.2f} solves/s", file=sys.stderr,
              flush=True)
        batched64 = run_batched(L.FP64, 78.6, 2)
        print(f"batched fp64 {batched64['solves_per_s']:.2f} solves/s", file=sys.stderr,
              flush=True)
    dom = next((r for r in kp if r["name"] == dominant), None)
    # whole-solve roofline: the method's bytes per iteration over the time
    # per iteration of the timed solves
    solve_roof = {}
    for tag, res, sz in (("mixed", mixed, 4), ("fp64", fp64, 8)):
        if args.workload == "aniso2d" and args.cycle != "v":
            solve_roof[tag] = None          # the per-level formula is the V-cycle's
            continue
        mb, per, cg = method_bytes(inf, sz)
        gbs = mb / (res["ms_per_iteration"] * 1e-3) / 1e9
        solve_roof[tag] = dict(bytes_per_iteration=int(mb), per_level_bytes=[int(v) for v in per],
                               cg_bytes=int(cg), ms_per_iteration=round(res["ms_per_iteration"], 4),
                               achieved=round(gbs, 1), frac=round(gbs / HBM_PEAK_GBS, 4))
    roofline = None
    if dom and dom["launches"] > 0 and dom["ms"] > 0:
        avg_s = dom["ms"] / dom["launches"] * 1e-3
        bytes_per_launch = dom["bytes"] / dom["launches"]
        achieved = bytes_per_launch / avg_s / 1e9
        roofline = dict(bound="hbm", achieved=round(achieved, 1), peak=HBM_PEAK_GBS,
                        unit="GB/s", frac=round(achieved / HBM_PEAK_GBS, 4),
                        traffic=measured_traffic(dominant), kernel=dominant,
                        avg_launch_us=round(avg_s * 1e6, 3),
                        algorithmic_bytes_per_launch=int(bytes_per_launch),
                        launches=dom["launches"],
                        share_of_kernel_time=round(allk[0]["ms"] / ktotal, 3))
        if dominant.startswith("k_sym_gemv") and inf["tail_level"] >= 0:
            roofline["bytes_basis"] = (
                f"dense-equivalent: the kernel applies the V-cycle of levels "
                f">= {inf['tail_level']} as one packed symmetric matrix formed at "
                f"setup; its bytes are that matrix's, not the method's steps for "
                f"those levels (see solve)")
    if roofline is not None:
        roofline["solve"] = solve_roof
        roofline["kernels"] = kernel_fracs

    cpu = None
    if cpu_proc is not None:
        print("cpu baseline: waiting for the oracle setup ...", file=sys.stderr, flush=True)
        ready = cpu_proc.stdout.readline()
        if ready.strip():
            rd = json.loads(ready)
            print(f"cpu baseline: oracle setup {rd['t_setup']:.0f} s, assembly "
                  f"{rd['t_assemble']:.0f} s; timing {args.cpu_reps + 1} solves",
                  file=sys.stderr, flush=True)
        out, err = cpu_proc.communicate("go\n", timeout=1800)
        if cpu_proc.returncode == 0:
            r = json.loads(out.strip().splitlines()[-1])
            tot = sum(r["times"])
            cpu = dict(value=round(len(r["times"]) / tot, 6), unit="solves/s",
                       cores=r["blas_threads"], kind="oracle",
                       sample=(f"{len(r['times'])} whole solves to 1e-8 "
                               f"({'/'.join(str(i) for i in sorted(set(r['iters'])))} PCG "
                               f"iterations each) after one warm-up, the same workload; "
                               f"assembled form: each level's RAS smoother one CSR matrix, "
                               f"RAS-T its transpose, CSR A_l and P_l, coarsest Cholesky; "
                               f"scipy sparse products on one thread, dense solves on "
                               f"{r['blas_threads']} {r['blas']} BLAS threads; "
                               f"oracle setup (coarse rows of G compressed exactly) "
                               f"{r['t_setup']:.0f} s + assembly {r['t_assemble']:.0f} s "
                               f"untimed"),
                       sample_seconds=round(tot, 2),
                       p50_ms=round(percentile(r["times"], 0.5) * 1e3, 1),
                       cpu_model=r["cpu_model"], cpu_count=r["cpu_count"],
                       affinity=r["affinity"], true_rel_res=r["true_rel_res"])
        else:
            cpu = dict(value=None, unit="solves/s", cores=None, kind="oracle",
                       sample="failed: " + (err.strip().splitlines() or ["?"])[-1][:200])

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
            "workload": (f"ls3d N={args.N} A=D1+B^T D2^-1 B, K=Q diag(1,1e-3,1e-3) Q^T, "
                         f"lognormal coefficient (n={prob.n}, m={prob.m}), rhs "
                         f"uniform[-1,1] seed {seed}, tol 1e-8, 3x3x3 aggregates, "
                         f"c_min=3,4, coarsest<2000" if three_d else
                         f"aniso2d N={args.N} theta=pi/6 eps=1e-4 (n={prob.n}, "
                         f"m={prob.m}), rhs uniform[-1,1] seed {seed}, tol 1e-8, "
                         f"4x4 aggregates, c_min={args.cmin}, omega_max={args.omega_max}, "
                         f"{args.cycle}-cycle, coarsest<2000"),
            "levels": inf["nlevels"],
            "n_per_level": [l["n"] for l in inf["levels"]],
            "op_complexity": round(inf["op_complexity"], 3),
            "smoother_complexity": round(inf["smoother_complexity"], 3),
            "smoother_entries": smoother_entries,
            "setup_s": round(t_setup, 2),
            "setup": ("device" if args.setup == "device"
                      or (args.setup == "auto" and prob.n >= 100000) else "host"),
            "dense_tail_level": inf["tail_level"],
            "device_gb": round(inf["device_bytes"] / 1e9, 2),
            "parallelism": "single GPU",
        },
        "p50_ms": round(mixed["p50_ms"], 3),
        "p99_ms": round(mixed["p99_ms"], 3),
        "iters": mixed["iters"],
        "converged": mixed["converged"],
        "true_rel_res": mixed["true_rel_res"],
        "ms_per_iteration": round(mixed["ms_per_iteration"], 4),
        "vcycles_per_s": round(mixed["solves_per_s"] * (mixed["iters"] + 1), 1),
        "mixed_graph": {k: (round(v, 4) if isinstance(v, float) and k != "true_rel_res" else v)
                        for k, v in mixed_graph.items()},
        "fp64": {k: (round(v, 4) if isinstance(v, float) and k != "true_rel_res" else v)
                 for k, v in fp64.items()},
        "batched_mixed": batched,
        "batched_fp64": batched64,
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
