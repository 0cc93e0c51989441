"""Write ``config2_oracle.json``: the oracle's hierarchy summary and PCG run on
the rotated-anisotropic workload (N=512 cells per side, theta=pi/6,
eps=1e-4, right-hand side uniform[-1,1] from seed 1, c_min = 2 on every
level).

Calls only the ``oracle`` and ``problems`` packages.  The GPU tests use the
stored values to check the library at full size without re-running the
(several-minute) FP64 oracle setup: per-level integer setup (sizes, k
histograms, a hash of aggregates / Omega lists / counts), the iteration
count to 1e-8, and sampled entries of the oracle's iterate after exactly that
many iterations.

Usage: python tests/golden/make_config2_fixture.py [N]
"""
import hashlib
import json
import math
import os
import sys
import time

import numpy as np

sys.path.insert(0, os.path.join(os.path.dirname(__file__), "..", ".."))
import oracle as O          # noqa: E402
import problems as P        # noqa: E402


def level_hash(L) -> str:
    h = hashlib.sha256()
    h.update(np.asarray(L.agg, dtype=np.int64).tobytes())
    h.update(np.asarray(L.k, dtype=np.int64).tobytes())
    for Om in L.Omega:
        h.update(np.asarray(Om, dtype=np.int64).tobytes())
        h.update(b"|")
    return h.hexdigest()


def main(N: int = 512):
    prob = P.config2(N)
    t0 = time.time()
    H = O.setup(prob.G, 2, prob.grid, O.Params(cmin=(2,)))
    t_setup = time.time() - t0
    levels = []
    for L in H.levels:
        d = dict(n=int(L.n), coarsest=bool(L.coarsest))
        if not L.coarsest:
            d.update(nagg=int(L.n_agg), block=int(L.block),
                     n_color=int(L.n_color), n_mult=int(L.n_mult),
                     thresh=float(L.thresh), k_sum=int(L.k.sum()),
                     k_hist=np.bincount(L.k).tolist(),
                     smoother_entries=int(sum(len(w) * len(Om) for w, Om in
                                              zip(L.omega, L.Omega))),
                     hash=level_hash(L), hazards=len(L.hazards))
        levels.append(d)
    b = P.rhs_uniform(prob.n, P.CONFIG_RHS_SEED[2])
    t0 = time.time()
    x, info = O.pcg(H, b, tol=1e-8, maxit=500)
    t_pcg = time.time() - t0
    rng = np.random.default_rng(12345)
    idx = np.sort(rng.choice(prob.n, size=256, replace=False))
    out = dict(
        workload=f"aniso2d N={N} theta=pi/6 eps=1e-4 rhs seed 1, c_min=(2,)",
        n=int(prob.n), m=int(prob.m), levels=levels,
        iters=int(info["iters"]), true_rel_res=float(info["true_rel_res"]),
        rho=float(info["rho"]), x_norm=float(np.linalg.norm(x)),
        sample_idx=idx.tolist(), x_sample=x[idx].tolist(),
        oracle_setup_seconds=t_setup, oracle_pcg_seconds=t_pcg,
        stats=O.stats(H))
    path = os.path.join(os.path.dirname(__file__),
                        "config2_oracle.json" if N == 512 else f"aniso2d_N{N}_oracle.json")
    with open(path, "w") as f:
        json.dump(out, f, indent=1)
    print(path, out["iters"], out["true_rel_res"])


if __name__ == "__main__":
    main(int(sys.argv[1]) if len(sys.argv) > 1 else 512)
