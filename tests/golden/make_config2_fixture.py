"""Write the stored oracle run of the rotated-anisotropic workload (N=512
cells per side, theta=pi/6, eps=1e-4, right-hand side uniform[-1,1] from
seed 1, c_min = 2 on every level).

Calls only the ``oracle`` and ``problems`` packages.  The GPU tests use the
stored values to check the library at full size without re-running the
(several-minute) FP64 oracle setup:

* ``config2_oracle.json``: per-level integer setup (sizes, k histograms, a
  hash of aggregates / Omega lists / counts), the iteration count to 1e-8 and
  the complexity statistics;
* ``config2_oracle_x.npy``: the oracle's whole iterate after exactly that many
  PCG iterations (FP64, 261,121 entries);
* ``config2_oracle_batch.npz``: the 64 right-hand sides of seeds 100-163,
  each run for ``BATCH_ITERS`` PCG iterations by the oracle: every column's
  2-norm, and the entries at ``BATCH_SAMPLES`` fixed indices of every column.

The oracle hierarchy is built with exact row compression of the coarse
G_l (each group of rows touching the same parents replaced by its QR R
factor), as the library stores them; the integer setup is the same as the
plain form's.

Usage: python tests/golden/make_config2_fixture.py [N]
"""
import hashlib
import json
import math
import multiprocessing as mp
import os
import sys
import time

import numpy as np

sys.path.insert(0, os.path.join(os.path.dirname(__file__), "..", ".."))
import oracle as O          # noqa: E402
import problems as P        # noqa: E402

BATCH_SEEDS = list(range(100, 164))
BATCH_ITERS = 20
BATCH_SAMPLES = 4096

_H = None                   # the hierarchy, shared with forked workers


def level_hash(L) -> str:
    h = hashlib.sha256()
    h.update(np.asarray(L.agg, dtype=np.int64).tobytes())
    h.update(np.asarray(L.k, dtype=np.int64).tobytes())
    for Om in L.Omega:
        h.update(np.asarray(Om, dtype=np.int64).tobytes())
        h.update(b"|")
    return h.hexdigest()


def _batch_column(seed):
    n = _H.levels[0].n
    x, _ = O.pcg(_H, P.rhs_uniform(n, seed), fixed_iters=BATCH_ITERS)
    return x


def main(N: int = 512):
    global _H
    prob = P.config2(N)
    t0 = time.time()
    H = O.setup(prob.G, 2, prob.grid, O.Params(cmin=(2,), compress_rows=True))
    t_setup = time.time() - t0
    _H = H
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
    xk = x
    if info["restarts"]:            # the fixed-count iterate, without restarts
        xk, _ = O.pcg(H, b, fixed_iters=info["iters"])
    here = os.path.dirname(__file__)
    stem = "config2_oracle" if N == 512 else f"aniso2d_N{N}_oracle"
    np.save(os.path.join(here, stem + "_x.npy"), xk)
    t0 = time.time()
    with mp.get_context("fork").Pool(min(8, os.cpu_count() or 1)) as pool:
        cols = pool.map(_batch_column, BATCH_SEEDS)
    t_batch = time.time() - t0
    idx = np.sort(np.random.default_rng(12345).choice(prob.n, min(BATCH_SAMPLES, prob.n),
                                                      replace=False))
    Xb = np.stack(cols)
    np.savez(os.path.join(here, stem + "_batch.npz"),
             seeds=np.asarray(BATCH_SEEDS), iters=np.asarray(BATCH_ITERS),
             idx=idx, x_sample=Xb[:, idx], x_norm=np.linalg.norm(Xb, axis=1))
    out = dict(
        workload=f"aniso2d N={N} theta=pi/6 eps=1e-4 rhs seed 1, c_min=(2,)",
        n=int(prob.n), m=int(prob.m), levels=levels,
        iters=int(info["iters"]), restarts=int(info["restarts"]),
        true_rel_res=float(info["true_rel_res"]),
        rho=float(info["rho"]), x_norm=float(np.linalg.norm(xk)),
        oracle_setup_seconds=t_setup, oracle_pcg_seconds=t_pcg,
        oracle_batch_seconds=t_batch, stats=O.stats(H))
    path = os.path.join(here, stem + ".json")
    with open(path, "w") as f:
        json.dump(out, f, indent=1)
    print(path, out["iters"], out["true_rel_res"], f"setup {t_setup:.0f}s")


if __name__ == "__main__":
    main(int(sys.argv[1]) if len(sys.argv) > 1 else 512)
