"""The allocation-free entry point lsamg_apply_op_noalloc, through the C-ABI.

On the GPU: its result equals lsamg_apply_op's bit for bit (the same kernels
on the same data; only the staging addresses differ) for every operator and
both V-cycle precisions, on two calls in a row, the second on a smaller
problem (so the second call finds the first call's data in the staging
array), and it leaves the handle's device bytes unchanged.  On the CPU: an
operator whose staging would exceed the array is refused with LSAMG_EINVAL
before any device work (a host-only handle reaches that check and, for an
operator that fits, stops at LSAMG_ENODEV).
"""
import math

import numpy as np
import pytest
import scipy.sparse as sp

import problems as P
from paper_2601_04112_amd import lsamg as L

OPS = [L.OP_A, L.OP_RAS, L.OP_RAST, L.OP_VCYCLE]


def tall_factor(n_cols=1000, extra_rows=4_200_000, seed=3):
    """G with few columns and many rows: one identity row per column plus
    random difference rows (A = G^T G is SPD and its hierarchy is a single
    dense level), so 8 (2n + m) bytes exceed the 32 MiB staging array."""
    rng = np.random.default_rng(seed)
    i = rng.integers(0, n_cols, extra_rows)
    j = (i + 1 + rng.integers(0, n_cols - 1, extra_rows)) % n_cols
    rows = np.concatenate([np.arange(n_cols), np.repeat(n_cols + np.arange(extra_rows), 2)])
    cols = np.concatenate([np.arange(n_cols), np.stack([i, j], 1).ravel()])
    vals = np.concatenate([np.ones(n_cols), np.tile([1.0, -1.0], extra_rows)])
    return sp.csr_matrix((vals, (rows, cols)), shape=(n_cols + extra_rows, n_cols))


def test_noalloc_refuses_oversize_staging():
    G = tall_factor()
    s = L.Solver(G, 2, (40, 25), device=-1, max_coarse=2000)
    assert s.info()["nlevels"] == 1
    lib = L.load()
    dummy = L.C.c_void_p(256)           # never dereferenced: the checks come first
    rc = lib.lsamg_apply_op_noalloc(s._h, L.OP_A, dummy, dummy, None)
    assert rc == L.LSAMG_EINVAL
    assert "staging" in lib.lsamg_last_error().decode()
    rc = lib.lsamg_apply_op_noalloc(s._h, L.OP_VCYCLE, dummy, dummy, None)
    assert rc == L.LSAMG_ENODEV
    s.close()


@pytest.mark.gpu
def test_noalloc_equals_apply_op(gpu_device):
    import torch
    big = P.aniso2d(64, math.pi / 6, 1e-4)
    small = P.config1()
    sb = L.Solver(big.G, 2, big.grid, device=0, cmin=(2,), max_coarse=150, dense_tail=2000)
    ss = L.Solver(small.G, 2, small.grid, device=0, max_levels=2, max_coarse=0, block=4,
                  n_eig_fixed=4)
    try:
        for prec in (L.FP64, L.MIXED):
            for op in OPS:
                for s, p, seed in ((sb, big, 1), (ss, small, 2)):
                    print(f"[case] noalloc prec={prec} op={op} n={p.n}", flush=True)
                    s.set_precision(prec)
                    x = torch.tensor(np.random.default_rng(seed).standard_normal(p.n),
                                     dtype=torch.float64, device="cuda:0")
                    ref = s.apply(op, x)
                    bytes0 = L.load().lsamg_device_bytes(s._h)
                    out = torch.full_like(x, float("nan"))
                    s.apply_noalloc(op, x, out)
                    torch.cuda.synchronize()
                    assert L.load().lsamg_device_bytes(s._h) == bytes0
                    assert torch.equal(out, ref), (prec, op, p.n,
                                                   float((out - ref).abs().max()))
    finally:
        sb.close()
        ss.close()
