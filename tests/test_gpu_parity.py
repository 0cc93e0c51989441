"""GPU parity: the HIP solve path against the FP64 oracle, through the C-ABI.

Tolerances (FP64 path): operators A, RAS, RAS-T agree to 1e-12 relative (the
library applies explicit local-inverse rows, the oracle Cholesky solves; both
backward stable on blocks with condition numbers below 1e3); the V-cycle and
PCG iterates at equal iteration counts agree to 1e-10 relative, single- and
multi-right-hand-side, on every 2D case.  The Schur complement of eq:gevp-S
is formed from the weighted rows of G on both sides (never from
A~_GammaGamma), so even the cases with singular coarse A~_GammaGamma
("illcond") keep FP64 rounding at its own level.

The 3D case (anisotropy oblique to the grid, lognormal coefficient) is one
where CG itself amplifies rounding: the oracle run on a right-hand side
perturbed by one unit in the last place drifts from its own unperturbed
iterate by ~1e-11 after 15 iterations and ~1e-9 after 25.  Its PCG iterates
are compared at 1e-10 for as many iterations as the oracle's own drift stays
below 1e-12, and at ten times the measured drift beyond that.

Mixed path (FP32 V-cycle under FP64 CG): the library stops only when the
true FP64 residual b - A x reaches the tolerance (the oracle's rule), so the
residual computed with the oracle's A is asserted <= tol, and iteration
counts stay within 10% of the oracle's.
"""
import hashlib
import json
import math
import os

import numpy as np
import pytest

import oracle as O
import problems as P
from paper_2601_04112_amd import lsamg as L

pytestmark = pytest.mark.gpu
HERE = os.path.dirname(os.path.abspath(__file__))


def rel(a, b):
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


def dvec(v):
    import torch
    return torch.tensor(np.asarray(v), dtype=torch.float64, device="cuda:0")


def host(t):
    return t.detach().cpu().numpy()


def build(prob, ndim, oparams, **lparams):
    print(f"[case] {prob.name} {lparams}", flush=True)
    H = O.setup(prob.G, ndim, prob.grid, oparams)
    s = L.Solver(prob.G, ndim, prob.grid, device=0, **lparams)
    return H, s


@pytest.fixture(scope="module")
def cfg1(gpu_device):
    p = P.config1()
    H, s = build(p, 2, O.Params(max_levels=2, max_coarse=0, block=4, n_eig_fixed=4),
                 max_levels=2, max_coarse=0, block=4, n_eig_fixed=4)
    yield p, H, s
    s.close()


@pytest.fixture(scope="module")
def rot(gpu_device):
    p = P.aniso2d(64, math.pi / 6, 1e-4)
    H, s = build(p, 2, O.Params(cmin=(2,), max_coarse=150), cmin=(2,), max_coarse=150,
                 dense_tail=0)
    assert len(H.levels) >= 3 and s.info()["tail_level"] == -1
    yield p, H, s
    s.close()


@pytest.fixture(scope="module")
def rot_tail(gpu_device):
    """As rot, with the V-cycle below level 1 applied as one dense matrix."""
    p = P.aniso2d(64, math.pi / 6, 1e-4)
    H, s = build(p, 2, O.Params(cmin=(2,), max_coarse=150), cmin=(2,), max_coarse=150,
                 dense_tail=2000)
    assert len(H.levels) >= 4 and s.info()["tail_level"] == 1
    yield p, H, s
    s.close()


@pytest.fixture(scope="module")
def ragged(gpu_device):
    # 46 interior nodes per axis = 11 blocks of 4 plus one of 2
    p = P.aniso2d(47, math.pi / 6, 1e-4)
    H, s = build(p, 2, O.Params(cmin=(2,), max_coarse=150), cmin=(2,), max_coarse=150,
                 dense_tail=0)
    yield p, H, s
    s.close()


def min_kept_gamma_ratio(H):
    """Smallest eigenvalue of A~_GammaGamma kept by the pseudo-inverse,
    relative to the largest, over all aggregates and levels."""
    worst = 1.0
    for Lv in H.levels[:-1]:
        for i in range(Lv.n_agg):
            nw = len(Lv.omega[i])
            if len(Lv.Omega[i]) == nw:
                continue
            At = O.lsamg.local_splitting(Lv.G, Lv.nz[i], Lv.Omega[i], Lv.M)
            lam = np.linalg.eigvalsh(At[nw:, nw:])
            r = lam / lam.max()
            worst = min(worst, r[r > 1e-12].min())
    return worst


@pytest.fixture(scope="module")
def illcond(gpu_device):
    # ragged lattice, LS_{3,4} caps, theta=0.5, eps=1e-2
    p = P.aniso2d(47, 0.5, 1e-2)
    H, s = build(p, 2, O.Params(cmin=(3, 4), max_coarse=150), cmin=(3, 4), max_coarse=150,
                 dense_tail=0)
    assert min_kept_gamma_ratio(H) < 1e-11
    yield p, H, s
    s.close()


CASES = ["cfg1", "rot", "rot_tail", "ragged", "illcond"]
U = 2.220446049250313e-16


def vtol(H):
    """FP64 parity bound of V-cycles and PCG iterates (see the module
    docstring)."""
    return 1e-10


def oracle_drift(H, b, K, seed=1):
    """Relative change of the oracle's K-iteration PCG iterate when b is
    perturbed by one rounding unit per entry: CG's own sensitivity."""
    b2 = b * (1 + U * np.random.default_rng(seed).standard_normal(len(b)))
    x1, _ = O.pcg(H, b, fixed_iters=K)
    x2, _ = O.pcg(H, b2, fixed_iters=K)
    return rel(x2, x1)


def precond_drift(H, b, K, eta, seed=1):
    """Relative change of the oracle's K-iteration PCG iterate when every
    V-cycle output is perturbed by eta (relative, per entry): CG's
    sensitivity to a preconditioner that differs at that level, as two FP64
    hierarchies whose setups round differently do."""
    rng = np.random.default_rng(seed)

    def pert(r):
        y = O.vcycle(H, r)
        return y * (1 + eta * rng.standard_normal(len(y)))

    x1, _ = O.pcg(H, b, fixed_iters=K)
    x2, _ = O.pcg(H, b, fixed_iters=K, precond=pert)
    return rel(x2, x1)


def test_apply_A(cfg1, rot):
    for p, H, s in (cfg1, rot):
        v = np.random.default_rng(1).standard_normal(p.n)
        y = host(s.apply(L.OP_A, dvec(v)))
        assert rel(y, H.levels[0].A @ v) <= 1e-13


@pytest.mark.parametrize("which", CASES)
def test_smoothers(which, request):
    p, H, s = request.getfixturevalue(which)
    s.set_precision(L.FP64)
    v = np.random.default_rng(2).standard_normal(p.n)
    L0 = H.levels[0]
    assert rel(host(s.apply(L.OP_RAS, dvec(v))), O.ras(L0, v)) <= 1e-12
    assert rel(host(s.apply(L.OP_RAST, dvec(v))), O.ras_t(L0, v)) <= 1e-12


@pytest.mark.parametrize("which", CASES)
def test_vcycle_fp64(which, request):
    p, H, s = request.getfixturevalue(which)
    s.set_precision(L.FP64)
    v = np.random.default_rng(3).standard_normal(p.n)
    assert rel(host(s.apply(L.OP_VCYCLE, dvec(v))), O.vcycle(H, v)) <= vtol(H)


@pytest.mark.parametrize("which", CASES)
def test_vcycle_mixed(which, request):
    p, H, s = request.getfixturevalue(which)
    s.set_precision(L.MIXED)
    try:
        v = np.random.default_rng(4).standard_normal(p.n)
        assert rel(host(s.apply(L.OP_VCYCLE, dvec(v))), O.vcycle(H, v)) <= 1e-4
    finally:
        s.set_precision(L.FP64)


@pytest.mark.parametrize("which", CASES)
def test_pcg_fixed_iterations(which, request):
    """Same iteration count as the oracle: iterates agree to 1e-10."""
    p, H, s = request.getfixturevalue(which)
    s.set_precision(L.FP64)
    b = P.rhs_uniform(p.n, 0)
    xo, info = O.pcg(H, b, tol=1e-8)
    k = info["iters"]
    assert info["restarts"] == 0
    x, st = s.solve(dvec(b), tol=0.0, maxit=k)
    assert st[0]["iters"] == k and st[0]["converged"] == 0
    assert rel(host(x), xo) <= vtol(H), rel(host(x), xo)
    # converged run: same stop iteration (+-1), true residual at tolerance
    x2, st2 = s.solve(dvec(b), tol=1e-8, maxit=500)
    assert abs(st2[0]["iters"] - k) <= 1 and st2[0]["converged"] == 1
    r = np.linalg.norm(b - H.levels[0].A @ host(x2)) / np.linalg.norm(b)
    assert r <= 1e-8 and abs(r - st2[0]["true_rel_res"]) <= 1e-12


@pytest.mark.parametrize("which", CASES)
def test_pcg_mixed(which, request):
    p, H, s = request.getfixturevalue(which)
    b = P.rhs_uniform(p.n, 0)
    _, info = O.pcg(H, b, tol=1e-8)
    s.set_precision(L.MIXED)
    try:
        x, st = s.solve(dvec(b), tol=1e-8, maxit=500)
    finally:
        s.set_precision(L.FP64)
    r = np.linalg.norm(b - H.levels[0].A @ host(x)) / np.linalg.norm(b)
    assert st[0]["converged"] == 1 and r <= 1e-8
    assert st[0]["iters"] <= math.ceil(1.10 * info["iters"])


@pytest.mark.parametrize("nrhs", [3, 8, 20])
def test_batched_equals_single(rot, nrhs):
    """A batch of right-hand sides (one FP64 CG per column, shared matrix
    reads) gives each column's single-vector iterate at equal iteration count
    to 1e-10, and the same stop iteration (+-1)."""
    p, H, s = rot
    s.set_precision(L.FP64)
    B = np.stack([P.rhs_uniform(p.n, 100 + j) for j in range(nrhs)])
    k = 12
    X, st = s.solve(dvec(B), tol=0.0, maxit=k)
    for j in range(nrhs):
        x1, st1 = s.solve(dvec(B[j]), tol=0.0, maxit=k)
        assert st[j]["iters"] == k
        assert rel(host(X[j]), host(x1)) <= 1e-10
    X, st = s.solve(dvec(B), tol=1e-8)
    for j in range(nrhs):
        x1, st1 = s.solve(dvec(B[j]), tol=1e-8)
        assert abs(st[j]["iters"] - st1[0]["iters"]) <= 1
        assert st[j]["converged"] == 1 and st[j]["true_rel_res"] <= 1e-8
        r = np.linalg.norm(B[j] - H.levels[0].A @ host(X[j])) / np.linalg.norm(B[j])
        assert r <= 1e-8


@pytest.mark.parametrize("which", ["rot", "rot_tail"])
def test_batched_mixed(which, request):
    p, H, s = request.getfixturevalue(which)
    B = np.stack([P.rhs_uniform(p.n, 200 + j) for j in range(5)])
    _, info = O.pcg(H, B[0], tol=1e-8)
    s.set_precision(L.MIXED)
    try:
        X, st = s.solve(dvec(B), tol=1e-8)
    finally:
        s.set_precision(L.FP64)
    for j in range(5):
        r = np.linalg.norm(B[j] - H.levels[0].A @ host(X[j])) / np.linalg.norm(B[j])
        assert st[j]["converged"] == 1 and r <= 1e-8
        assert st[j]["iters"] <= math.ceil(1.10 * info["iters"]) + 1


@pytest.mark.parametrize("which", ["rot", "rot_tail"])
@pytest.mark.parametrize("nrhs", [64, 20, 16, 5])
def test_batched_vcycle_matches_single(which, nrhs, request):
    """One multi-right-hand-side V-cycle equals the single-vector V-cycle on
    every column: to 1e-12 in FP64; in FP32 (matrix-core tiles for >= 16
    columns, FMA kernels otherwise or with the matrix cores switched off) to
    2e-5, the spread of two FP32 summation orders over the levels."""
    p, H, s = request.getfixturevalue(which)
    X = np.stack([P.rhs_uniform(p.n, 300 + j) for j in range(nrhs)])
    dX = dvec(X)
    try:
        for prec, mfma, tol in ((L.FP64, 1, 1e-12), (L.MIXED, 1, 2e-5), (L.MIXED, 0, 2e-5)):
            s.set_precision(prec)
            s.set_option(L.OPT_MFMA, mfma)
            Y = host(s.apply_vcycle_batch(dX))
            for j in range(nrhs):
                y1 = host(s.apply(L.OP_VCYCLE, dX[j]))
                assert rel(Y[j], y1) <= tol, (prec, mfma, j, rel(Y[j], y1))
    finally:
        s.set_precision(L.FP64)
        s.set_option(L.OPT_MFMA, 1)


@pytest.mark.parametrize("which", ["rot", "rot_tail"])
def test_batched_vcycle_every_tile_shape(which, request):
    """Every fixed matrix-core tile shape (row tiles, loads in flight, loop
    split, the split also on multi-aggregate operators) gives the single-
    vector FP32 V-cycle on each of 64 columns to 2e-5."""
    p, H, s = request.getfixturevalue(which)
    X = np.stack([P.rhs_uniform(p.n, 500 + j) for j in range(64)])
    dX = dvec(X)
    s.set_precision(L.MIXED)
    try:
        Y1 = [host(s.apply(L.OP_VCYCLE, dX[j])) for j in range(0, 64, 7)]
        # u = 0: the form that stages the input rows in LDS (64-row tasks)
        for rt, u in ((1, 2), (1, 8), (2, 2), (2, 8), (4, 2), (4, 8), (4, 0)):
            for sp in (1, 2, 4, 8):
                s.set_option(L.OPT_MFMA_TILE, 100 * rt + 10 * u + sp)
                s.profile(True)
                Y = host(s.apply_vcycle_batch(dX))
                names = {k["name"].split("<")[0] for k in s.profile_read()}
                s.profile(False)
                assert ("k_bmm_lds" in names) == (u == 0), (rt, u, sp, sorted(names))
                for k, j in enumerate(range(0, 64, 7)):
                    assert rel(Y[j], Y1[k]) <= 2e-5, (rt, u, sp, j, rel(Y[j], Y1[k]))
    finally:
        s.profile(False)
        s.set_option(L.OPT_MFMA_TILE, 0)
        s.set_precision(L.FP64)


@pytest.mark.parametrize("which", ["rot", "rot_tail"])
def test_batched_fp64_matrix_cores(which, request):
    """The FP64 multi-right-hand-side V-cycle with its aggregate-block
    operators on the FP64 matrix cores (k_bmmd, forced by a fixed tile shape:
    1, 2 and 4 row tiles, both loads-in-flight counts; k_bmmd_lds, the
    LDS-staged form on 64 columns) and as the autotuner picks gives the single-
    vector FP64 V-cycle on every column to 1e-12, on 64 columns and then on
    narrower batches with the same buffers; the forced form is the one that
    runs."""
    p, H, s = request.getfixturevalue(which)
    X = np.stack([P.rhs_uniform(p.n, 1300 + j) for j in range(64)])
    dX = dvec(X)
    s.set_precision(L.FP64)
    inf = s.info()
    dense = inf["tail_level"] if inf["tail_level"] >= 0 else inf["nlevels"] - 1
    try:
        Y1 = [host(s.apply(L.OP_VCYCLE, dX[j])) for j in range(64)]
        for tile in (121, 181, 221, 281, 401, 481, 0):
            s.set_option(L.OPT_MFMA_TILE, tile)
            for nc in (64, 32, 16):
                s.apply_vcycle_batch(dX[:nc])
                s.profile(True, by_level=True)
                Y = host(s.apply_vcycle_batch(dX[:nc]))
                names = {k["name"] for k in s.profile_read()}
                s.profile(False)
                if tile:            # FMA only on the dense level
                    fma = {k for k in names if k.startswith("k_bgemm")}
                    assert any(k.startswith("k_bmmd") for k in names), (tile, nc, sorted(names))
                    assert all(k.endswith(f"@L{dense}") for k in fma), (tile, nc, sorted(fma))
                    lds = any(k.startswith("k_bmmd_lds") for k in names)
                    assert lds == (tile == 401 and nc == 64), (tile, nc, sorted(names))
                for j in range(nc):
                    assert rel(Y[j], Y1[j]) <= 1e-12, (tile, nc, j, rel(Y[j], Y1[j]))
    finally:
        s.profile(False)
        s.set_option(L.OPT_MFMA_TILE, 0)
        s.set_precision(L.FP64)


@pytest.mark.parametrize("which", ["rot", "rot_tail"])
@pytest.mark.parametrize("prec", [L.MIXED, L.FP64])
def test_batched_dense_level_every_split(which, prec, request):
    """The LDS-staged matrix-core GEMM of the dense level (k_dense_mm64 in
    FP32, k_dense_mm64d in FP64), for loop splits from one range to more
    ranges than 32-row chunks, with it switched off, and as the tuner picks,
    gives the single-vector V-cycle of the same precision on each of 64
    columns to 2e-5 (FP32) or 1e-12 (FP64); the forced form is the one that
    runs."""
    p, H, s = request.getfixturevalue(which)
    X = np.stack([P.rhs_uniform(p.n, 900 + j) for j in range(64)])
    dX = dvec(X)
    s.set_precision(prec)
    kern, tol = ("k_dense_mm64", 2e-5) if prec == L.MIXED else ("k_dense_mm64d", 1e-12)
    try:
        Y1 = [host(s.apply(L.OP_VCYCLE, dX[j])) for j in range(0, 64, 9)]
        for split in (1, 2, 3, 7, 16, 17, 0):
            s.set_option(L.OPT_DENSE_SPLIT, split)
            s.apply_vcycle_batch(dX)            # tunes (or fixes) the tile shapes
            s.profile(True)
            Y = host(s.apply_vcycle_batch(dX))
            names = {k["name"] for k in s.profile_read()}
            s.profile(False)
            if split:
                assert (kern in names) == (split <= 16), (split, sorted(names))
            for k, j in enumerate(range(0, 64, 9)):
                assert rel(Y[j], Y1[k]) <= tol, (split, j, rel(Y[j], Y1[k]))
    finally:
        s.profile(False)
        s.set_option(L.OPT_DENSE_SPLIT, 0)
        s.set_precision(L.FP64)


@pytest.mark.parametrize("which,bgroup", [("rot_tail", 0), ("rot", 1)])
@pytest.mark.parametrize("prec", [L.FP64, L.MIXED])
def test_graph_replay_equals_eager(which, bgroup, prec, request):
    """Solves whose V-cycles replay a captured HIP graph are bit-identical to
    solves with the kernels launched one by one, on every replay, with eager
    work and synchronisations between the replays; single vector, 16 columns
    and 64 columns (the batched FP32 V-cycle on matrix-core tiles, the dense
    level's LDS-staged GEMM, the tiled finest-level G^T G, and on "rot" the
    coarse levels' row-group pass)."""
    import torch
    p, H, s = request.getfixturevalue(which)
    b = dvec(P.rhs_uniform(p.n, 7))
    Bs = [dvec(np.stack([P.rhs_uniform(p.n, 400 + j) for j in range(nc)])) for nc in (16, 64)]
    s.set_precision(prec)
    try:
        s.set_option(L.OPT_BGROUP, bgroup)
        s.set_option(L.OPT_GRAPH, 0)
        x_e, st_e = s.solve(b, tol=1e-8)
        out_e = [s.solve(B, tol=1e-8) for B in Bs]
        s.set_option(L.OPT_GRAPH, 1)
        for rep in range(3):
            x_g, st_g = s.solve(b, tol=1e-8)
            assert st_g[0]["iters"] == st_e[0]["iters"]
            assert np.array_equal(host(x_g), host(x_e)), rep
            for B, (X_e, St_e) in zip(Bs, out_e):
                X_g, St_g = s.solve(B, tol=1e-8)
                assert [t["iters"] for t in St_g] == [t["iters"] for t in St_e]
                assert np.array_equal(host(X_g), host(X_e)), (rep, B.shape)
            s.apply(L.OP_A, b)                  # eager work between replays
            torch.cuda.synchronize()
    finally:
        s.set_option(L.OPT_GRAPH, 1)
        s.set_option(L.OPT_BGROUP, 0)
        s.set_precision(L.FP64)


def test_batched_two_pass_apply(rot):
    """With the one-pass FP64 G^T (G P) of the batched CG switched off (two
    passes through G P), a 64-column FP64 batch still equals the single-
    vector solves at a fixed iteration count, and the mixed batch converges."""
    p, H, s = rot
    B = np.stack([P.rhs_uniform(p.n, 800 + j) for j in range(64)])
    dB = dvec(B)
    try:
        s.set_option(L.OPT_ONEPASS_ATA, 0)
        s.set_precision(L.FP64)
        X, _ = s.solve(dB, tol=0.0, maxit=8)
        for j in (0, 17, 63):
            x1, _ = s.solve(dB[j], tol=0.0, maxit=8)
            assert rel(host(X[j]), host(x1)) <= 1e-10, j
        s.set_precision(L.MIXED)
        X, st = s.solve(dB, tol=1e-8)
        Xh = host(X)
        for j in (0, 31, 63):
            r = np.linalg.norm(B[j] - H.levels[0].A @ Xh[j]) / np.linalg.norm(B[j])
            assert st[j]["converged"] == 1 and r <= 1e-8, (j, r)
    finally:
        s.set_option(L.OPT_ONEPASS_ATA, 1)
        s.set_precision(L.FP64)


def test_batched_tiled_ata(rot):
    """The tiled one-pass G^T (G X) on 64 columns (k_bata_tile: residual of
    the batched V-cycle, A-apply of the batched CG) against the untiled forms:
    V-cycles agree to 1e-12 (FP64) and 2e-5 (FP32), FP64 solves at a fixed
    iteration count to 1e-10, and the mixed solve reaches the tolerance; the
    tiled kernel runs exactly when switched on."""
    p, H, s = rot
    B = np.stack([P.rhs_uniform(p.n, 1100 + j) for j in range(64)])
    dB = dvec(B)
    try:
        for prec, tol in ((L.FP64, 1e-12), (L.MIXED, 2e-5)):
            s.set_precision(prec)
            out = {}
            # 2: with the row phase (k_bata_tile); 3: expanded stencils
            # (k_bata_tilex); 1: the row form in FP32, the expanded one in FP64
            for on in (1, 2, 3, 0):
                s.set_option(L.OPT_ATA_TILES, on)
                s.profile(True)
                out[on] = host(s.apply_vcycle_batch(dB))
                names = {k["name"].split("<")[0] for k in s.profile_read()}
                s.profile(False)
                x = on == 3 or (on == 1 and prec == L.FP64)
                assert ("k_bata_tilex" in names) == x, (prec, on, sorted(names))
                assert ("k_bata_tile" in names) == (on != 0 and not x), (prec, on, sorted(names))
            for on in (1, 2, 3):
                for j in (0, 21, 63):
                    assert rel(out[on][j], out[0][j]) <= tol, (prec, on, j, rel(out[on][j], out[0][j]))
        s.set_precision(L.FP64)
        X = {}
        for on in (1, 2, 3, 0):
            s.set_option(L.OPT_ATA_TILES, on)
            X[on], _ = s.solve(dB, tol=0.0, maxit=8)
        for on in (1, 2, 3):
            for j in (0, 40, 63):
                assert rel(host(X[on][j]), host(X[0][j])) <= 1e-10, (on, j)
        s.set_option(L.OPT_ATA_TILES, 1)
        s.set_precision(L.MIXED)
        Xm, st = s.solve(dB, tol=1e-8)
        Xh = host(Xm)
        for j in (0, 31, 63):
            r = np.linalg.norm(B[j] - H.levels[0].A @ Xh[j]) / np.linalg.norm(B[j])
            assert st[j]["converged"] == 1 and r <= 1e-8, (j, r)
    finally:
        s.profile(False)
        s.set_option(L.OPT_ATA_TILES, 1)
        s.set_precision(L.FP64)


@pytest.mark.parametrize("prec", [L.FP64, L.MIXED])
def test_single_cg_tile(rot, prec):
    """The single-vector CG with its direction update fused into a tiled
    one-pass A-apply (k_cg_tile) against the unfused kernels: equal iterates
    to 1e-10 at a fixed iteration count (FP64 V-cycle), equal iteration
    counts to 1e-8 with the true residual at the tolerance (both precisions),
    and the fused kernel runs exactly when switched on."""
    p, H, s = rot
    b = P.rhs_uniform(p.n, 77)
    db = dvec(b)
    s.set_precision(prec)
    try:
        out, its = {}, {}
        for on in (1, 0):
            s.set_option(L.OPT_ATA_TILES, on)
            s.profile(True)
            x, st = s.solve(db, tol=1e-8)
            names = {k["name"].split("<")[0] for k in s.profile_read()}
            s.profile(False)
            assert ("k_cg_tile" in names) == bool(on), (on, sorted(names))
            assert ("k_cg_dir" in names) == (not on), (on, sorted(names))
            out[on], its[on] = host(x), st[0]["iters"]
            r = np.linalg.norm(b - H.levels[0].A @ out[on]) / np.linalg.norm(b)
            assert st[0]["converged"] == 1 and r <= 1e-8, (on, r)
        assert its[1] == its[0]
        if prec == L.FP64:
            x8 = {}
            for on in (1, 0):
                s.set_option(L.OPT_ATA_TILES, on)
                x8[on], _ = s.solve(db, tol=0.0, maxit=8)
            assert rel(host(x8[1]), host(x8[0])) <= 1e-10
    finally:
        s.profile(False)
        s.set_option(L.OPT_ATA_TILES, 1)
        s.set_precision(L.FP64)


@pytest.mark.parametrize("which", ["rot", "rot_tail"])
def test_batched_group_pass(which, request):
    """The coarse-level residual of the FP32 batched V-cycle as the row-group
    pass on 64 columns (k_bgrp_ata64 + k_bresid_stg64) and as the two CSR
    passes both give the single-vector V-cycle on each column to 2e-5; the
    forced form is the one that runs, and the batched mixed solve with the
    row-group pass reaches the tolerance."""
    p, H, s = request.getfixturevalue(which)
    B = np.stack([P.rhs_uniform(p.n, 1300 + j) for j in range(64)])
    dB = dvec(B)
    # levels with a residual between the finest and the dense tail (or coarsest)
    inf = s.info()
    last = inf["tail_level"] if inf["tail_level"] >= 0 else inf["nlevels"] - 1
    coarse = last > 1
    s.set_precision(L.MIXED)
    try:
        Y1 = [host(s.apply(L.OP_VCYCLE, dB[j])) for j in range(0, 64, 13)]
        for bg in (1, 2, 0):
            s.set_option(L.OPT_BGROUP, bg)
            s.apply_vcycle_batch(dB)            # tunes
            s.profile(True)
            Y = host(s.apply_vcycle_batch(dB))
            names = {k["name"].split("<")[0] for k in s.profile_read()}
            s.profile(False)
            if bg == 1:
                assert ("k_bgrp_ata64" in names and "k_bresid_stg64" in names) == coarse, \
                    (coarse, sorted(names))
            if bg == 2:
                assert "k_bgrp_ata64" not in names, sorted(names)
            for k, j in enumerate(range(0, 64, 13)):
                assert rel(Y[j], Y1[k]) <= 2e-5, (bg, j, rel(Y[j], Y1[k]))
        s.set_option(L.OPT_BGROUP, 1)
        X, st = s.solve(dB, tol=1e-8)
        Xh = host(X)
        for j in (0, 32, 63):
            r = np.linalg.norm(B[j] - H.levels[0].A @ Xh[j]) / np.linalg.norm(B[j])
            assert st[j]["converged"] == 1 and r <= 1e-8, (j, r)
    finally:
        s.profile(False)
        s.set_option(L.OPT_BGROUP, 0)
        s.set_precision(L.FP64)


def test_more_than_one_batch(rot):
    """70 right-hand sides are solved as a block of 64 and a block of 6 (both
    precisions); every column reaches the tolerance, and in FP64 equals its
    single-vector solve at a fixed iteration count."""
    p, H, s = rot
    B = np.stack([P.rhs_uniform(p.n, 700 + j) for j in range(70)])
    dB = dvec(B)
    try:
        for prec in (L.FP64, L.MIXED):
            s.set_precision(prec)
            X, st = s.solve(dB, tol=1e-8)
            Xh = host(X)
            for j in (0, 31, 63, 64, 69):
                r = np.linalg.norm(B[j] - H.levels[0].A @ Xh[j]) / np.linalg.norm(B[j])
                assert st[j]["converged"] == 1 and r <= 1e-8, (prec, j, r)
        s.set_precision(L.FP64)
        X, _ = s.solve(dB, tol=0.0, maxit=6)
        for j in (0, 63, 64, 69):
            x1, _ = s.solve(dB[j], tol=0.0, maxit=6)
            assert rel(host(X[j]), host(x1)) <= 1e-10, j
    finally:
        s.set_precision(L.FP64)


def test_batched_edge_columns(cfg1):
    """A zero column converges at once without disturbing the others; a
    single-level hierarchy works in the batched path."""
    p, H, s = cfg1
    B = np.stack([P.rhs_uniform(p.n, 1), np.zeros(p.n), P.rhs_uniform(p.n, 2)])
    X, st = s.solve(dvec(B), tol=1e-8)
    assert st[1]["iters"] == 0 and st[1]["converged"] == 1 and np.all(host(X[1]) == 0)
    for j in (0, 2):
        r = np.linalg.norm(B[j] - H.levels[0].A @ host(X[j])) / np.linalg.norm(B[j])
        assert r <= 1e-8
    q = P.aniso2d(12, 0.2, 0.3)
    s1 = L.Solver(q.G, 2, q.grid, device=0)
    Bq = np.stack([P.rhs_uniform(q.n, 5 + j) for j in range(3)])
    Xq, stq = s1.solve(dvec(Bq), tol=1e-10)
    A = (q.G.T @ q.G).toarray()
    for j in range(3):
        assert stq[j]["iters"] == 1
        assert rel(host(Xq[j]), np.linalg.solve(A, Bq[j])) <= 1e-10
    s1.close()


def test_edge_zero_and_bad_rhs(cfg1):
    p, H, s = cfg1
    x, st = s.solve(dvec(np.zeros(p.n)), tol=1e-8)
    assert st[0]["iters"] == 0 and st[0]["converged"] == 1
    assert np.all(host(x) == 0)
    bad = np.ones(p.n)
    bad[7] = np.nan
    with pytest.raises(L.LsamgError) as e:
        s.solve(dvec(bad), tol=1e-8)
    assert e.value.code == L.LSAMG_EBADINPUT
    x, st = s.solve(dvec(np.ones(p.n)), tol=1e-8, maxit=0)
    assert st[0]["iters"] == 0 and st[0]["converged"] == 0
    with pytest.raises(L.LsamgError) as e:
        s.solve(dvec(np.ones(p.n)), tol=1e-8, maxit=1, raise_on_noconv=True)
    assert e.value.code == L.LSAMG_ENOCONV
    import torch
    X, st = s.solve(torch.empty((0, p.n), dtype=torch.float64, device="cuda:0"))
    assert st == []


def test_single_level_is_direct(gpu_device):
    p = P.aniso2d(12, 0.2, 0.3)
    s = L.Solver(p.G, 2, p.grid, device=0)             # 121 unknowns: coarsest only
    assert s.info()["nlevels"] == 1
    b = P.rhs_uniform(p.n, 5)
    x, st = s.solve(dvec(b), tol=1e-10)
    xd = np.linalg.solve((p.G.T @ p.G).toarray(), b)
    assert st[0]["iters"] == 1 and rel(host(x), xd) <= 1e-10
    s.close()


def test_full_coarse_space_is_direct(gpu_device):
    """Keeping every local eigenvector makes the V-cycle exact (B = A^{-1})."""
    p = P.aniso2d(12, 0.4, 0.1)
    s = L.Solver(p.G, 2, p.grid, device=0, max_levels=2, max_coarse=0, n_eig_fixed=1000)
    b = P.rhs_uniform(p.n, 3)
    xd = np.linalg.solve((p.G.T @ p.G).toarray(), b)
    assert rel(host(s.apply(L.OP_VCYCLE, dvec(b))), xd) <= 1e-10
    x, st = s.solve(dvec(b), tol=1e-10)
    assert st[0]["iters"] == 1
    s.close()


@pytest.mark.parametrize("tail", [0, 16384])
def test_3d_small(gpu_device, tail):
    """3D D1 + B^T D2^-1 B form: V-cycle to 1e-10; PCG iterates to 1e-10 for
    the iterations over which the oracle's own drift under a one-ulp change
    of b stays below 1e-12, and at the oracle's stop count to ten times the
    larger of that drift and the drift under a perturbation of each V-cycle
    output of the size measured between the two V-cycles (the two setups'
    SVDs round differently, and CG amplifies that by its stop count on this
    operator); the converged solve reaches the tolerance on the true
    residual with a stop count inside the range the perturbed oracle runs
    give."""
    p = P.ls3d(12)
    H, s = build(p, 3, O.Params(block=3, cmin=(2,), max_coarse=100),
                 block=3, cmin=(2,), max_coarse=100, dense_tail=tail)
    assert (s.info()["tail_level"] > 0) == (tail > 0 and len(H.levels) > 2)
    v = np.random.default_rng(9).standard_normal(p.n)
    ev = rel(host(s.apply(L.OP_VCYCLE, dvec(v))), O.vcycle(H, v))
    assert ev <= vtol(H)
    b = P.rhs_uniform(p.n, 3)
    _, info = O.pcg(H, b, tol=1e-8)
    K = info["iters"]
    k_ok = max(k for k in range(1, K + 1, 3) if k == 1 or oracle_drift(H, b, k) <= 1e-12)
    for k in (k_ok, K):
        xo, _ = O.pcg(H, b, fixed_iters=k)
        x, _ = s.solve(dvec(b), tol=0.0, maxit=k)
        bound = vtol(H) if k == k_ok else max(
            vtol(H), 10 * max(oracle_drift(H, b, k), precond_drift(H, b, k, max(ev, U))))
        assert rel(host(x), xo) <= bound, (k, rel(host(x), xo), bound, ev)
    stops = [K] + [O.pcg(H, b * (1 + U * np.random.default_rng(q).standard_normal(p.n)),
                         tol=1e-8)[1]["iters"] for q in (1, 2, 3)]
    x, st = s.solve(dvec(b), tol=1e-8)
    assert min(stops) - 1 <= st[0]["iters"] <= max(stops) + 1, (st[0]["iters"], stops)
    r = np.linalg.norm(b - H.levels[0].A @ host(x)) / np.linalg.norm(b)
    assert st[0]["converged"] == 1 and r <= 1e-8
    s.close()


@pytest.mark.parametrize("which", ["rot", "rot_tail"])
def test_batched_vs_oracle(which, request):
    """The multi-right-hand-side path against the oracle directly, element by
    element: one FP64 V-cycle on 64 columns equals the oracle's V-cycle of
    each column to 1e-10 (the FP32 one to 1e-4, as the single-vector FP32
    V-cycle); FP64 PCG on 64 columns at a fixed iteration count equals the
    oracle's PCG iterate of each sampled column to 1e-10; the mixed batch
    reaches the tolerance on every column's true residual."""
    p, H, s = request.getfixturevalue(which)
    X = np.stack([P.rhs_uniform(p.n, 1500 + j) for j in range(64)])
    dX = dvec(X)
    try:
        for prec, tol in ((L.FP64, 1e-10), (L.MIXED, 1e-4)):
            s.set_precision(prec)
            Y = host(s.apply_vcycle_batch(dX))
            for j in range(64):
                e = rel(Y[j], O.vcycle(H, X[j]))
                assert e <= tol, (prec, j, e)
        s.set_precision(L.FP64)
        K = 10
        Xs, st = s.solve(dX, tol=0.0, maxit=K)
        Xh = host(Xs)
        for j in (0, 13, 27, 40, 63):
            xo, _ = O.pcg(H, X[j], fixed_iters=K)
            assert st[j]["iters"] == K and rel(Xh[j], xo) <= 1e-10, (j, rel(Xh[j], xo))
        s.set_precision(L.MIXED)
        Xm, st = s.solve(dX, tol=1e-8)
        Xh = host(Xm)
        for j in range(64):
            r = np.linalg.norm(X[j] - H.levels[0].A @ Xh[j]) / np.linalg.norm(X[j])
            assert st[j]["converged"] == 1 and r <= 1e-8, (j, r)
    finally:
        s.set_precision(L.FP64)


@pytest.mark.parametrize("prec", [L.FP64, L.MIXED])
def test_true_residual_stop(rot, prec):
    """Tolerances below what the true residual can reach: the recurrence
    residual passes while b - A x does not, so the solver replaces r by the
    true residual and restarts (as the oracle does); it reports convergence
    only with its FP64 true residual at the tolerance (recomputed here with
    the oracle's A, up to the rounding of that evaluation, which at 1e-14 is
    no longer negligible), and otherwise stops at maxit without convergence
    -- single vector and 8 columns."""
    p, H, s = rot
    b = P.rhs_uniform(p.n, 0)
    B = np.stack([P.rhs_uniform(p.n, 40 + j) for j in range(8)])
    nb = np.linalg.norm(b)
    A = H.levels[0].A

    def resid(bv, xv):
        """||b - A x|| / ||b|| and the rounding noise of evaluating it (two
        FP64 evaluations of A x: the assembled A and G^T (G x))"""
        ax = A @ xv
        noise = np.linalg.norm(ax - p.G.T @ (p.G @ xv)) / np.linalg.norm(bv)
        return np.linalg.norm(bv - ax) / np.linalg.norm(bv), noise

    s.set_precision(prec)
    try:
        restarts = 0
        for tol in (1e-14, 1e-15):
            _, info = O.pcg(H, b, tol=tol, maxit=60)
            x, st = s.solve(dvec(b), tol=tol, maxit=60)
            r, noise = resid(b, host(x))
            restarts += st[0]["restarts"]
            if st[0]["converged"]:
                assert st[0]["true_rel_res"] <= tol and r <= tol + 5 * noise, (tol, r, noise)
            else:
                assert st[0]["iters"] == 60
            if tol == 1e-15:             # out of reach for the oracle as well
                assert not info["converged"] and not st[0]["converged"]
                assert st[0]["restarts"] >= 1
            X, stb = s.solve(dvec(B), tol=tol, maxit=60)
            Xh = host(X)
            for j in range(8):
                rj, noise = resid(B[j], Xh[j])
                restarts += stb[j]["restarts"]
                if stb[j]["converged"]:
                    assert stb[j]["true_rel_res"] <= tol and rj <= tol + 5 * noise, \
                        (tol, j, rj, noise)
                else:
                    assert stb[j]["iters"] == 60
        assert restarts >= 1
    finally:
        s.set_precision(L.FP64)


def setup_hash(e) -> str:
    h = hashlib.sha256()
    h.update(np.asarray(e["agg"], dtype=np.int64).tobytes())
    h.update(np.asarray(e["k"], dtype=np.int64).tobytes())
    for Om in np.split(e["oidx"], e["optr"][1:-1]):
        h.update(np.asarray(Om, dtype=np.int64).tobytes())
        h.update(b"|")
    return h.hexdigest()


def test_config2_full_size(gpu_device):
    """Rotated anisotropy, N=512 (261,121 unknowns), at the benchmarked size,
    against the stored oracle run (tests/golden/config2_oracle*): integer
    setup equal on every level; the FP64 iterate after the oracle's
    iteration count equal to the oracle's on every entry to 1e-10; 64
    right-hand sides (seeds 100-163) through the FP64 multi-right-hand-side
    path (the matrix-core block products and dense level that the benchmark
    times) equal to the oracle's per-column PCG iterates at 4,096 sampled
    entries and in norm, to 1e-10; converged FP64, mixed and batched mixed
    solves reach the tolerance on the true residual."""
    fx = json.load(open(os.path.join(HERE, "golden", "config2_oracle.json")))
    x_or = np.load(os.path.join(HERE, "golden", "config2_oracle_x.npy"))
    bx = np.load(os.path.join(HERE, "golden", "config2_oracle_batch.npz"))
    p = P.config2()
    print(f"[case] config2 full size n={p.n}", flush=True)
    s = L.Solver(p.G, 2, p.grid, device=0, cmin=(2,))
    inf = s.info()
    assert inf["nlevels"] == len(fx["levels"])
    # levels 3.. (9,021 unknowns and below) run as one dense operator
    assert inf["tail_level"] == 3
    for l, lv in enumerate(fx["levels"]):
        assert inf["levels"][l]["n"] == lv["n"]
        if lv["coarsest"]:
            continue
        e = s.export_setup(l)
        assert e["nagg"] == lv["nagg"] and int(e["k"].sum()) == lv["k_sum"]
        assert setup_hash(e) == lv["hash"]
    b = P.rhs_uniform(p.n, P.CONFIG_RHS_SEED[2])
    K = fx["iters"]
    x, st = s.solve(dvec(b), tol=0.0, maxit=K)
    assert rel(host(x), x_or) <= 1e-10, rel(host(x), x_or)
    x, st = s.solve(dvec(b), tol=1e-8)
    assert st[0]["converged"] == 1 and abs(st[0]["iters"] - K) <= 1
    assert st[0]["true_rel_res"] <= 1e-8
    s.set_precision(L.MIXED)
    x, st = s.solve(dvec(b), tol=1e-8)
    assert st[0]["converged"] == 1 and st[0]["true_rel_res"] <= 1e-8
    assert st[0]["iters"] <= math.ceil(1.10 * K)
    # 64 right-hand sides (seeds 100-163) in one batch
    seeds = bx["seeds"].tolist()
    B = np.stack([P.rhs_uniform(p.n, q) for q in seeds])
    dB = dvec(B)
    s.set_precision(L.FP64)
    X, st = s.solve(dB, tol=0.0, maxit=int(bx["iters"]))
    Xh = host(X)
    idx = bx["idx"]
    for j in range(len(seeds)):
        nj = bx["x_norm"][j]
        assert abs(np.linalg.norm(Xh[j]) - nj) <= 1e-10 * nj, j
        e = np.linalg.norm(Xh[j][idx] - bx["x_sample"][j]) / np.linalg.norm(bx["x_sample"][j])
        assert e <= 1e-10, (j, e)
    s.set_precision(L.MIXED)
    X, st = s.solve(dB, tol=1e-8)
    for j in range(64):
        assert st[j]["converged"] == 1 and st[j]["true_rel_res"] <= 1e-8
        assert st[j]["iters"] <= math.ceil(1.10 * K) + 1
    for j in (0, 31, 63):
        r = np.linalg.norm(B[j] - p.G.T @ (p.G @ host(X[j]))) / np.linalg.norm(B[j])
        assert r <= 1e-8
    s.close()


@pytest.mark.parametrize("which", ["rot", "rot_tail", "ragged"])
def test_flexible_cg(which, request):
    """Flexible CG (beta = -(z . A p) / (p . A p)): with the FP64 V-cycle the
    iterate after a fixed count equals the oracle's flexible PCG to 1e-10,
    for one vector and for sampled columns of a 20-column batch; with the
    FP32 V-cycle every column converges on its true residual within 1.1x the
    oracle's CG count; below the reachable tolerance the restart path keeps
    the same contract as CG (converged only at the tolerance, else maxit)."""
    p, H, s = request.getfixturevalue(which)
    b = P.rhs_uniform(p.n, 0)
    _, info = O.pcg(H, b, tol=1e-8)
    K = info["iters"]
    X = np.stack([P.rhs_uniform(p.n, 900 + j) for j in range(20)])
    s.set_option(L.OPT_KRYLOV, L.KRYLOV_FCG)
    try:
        s.set_precision(L.FP64)
        xo, _ = O.pcg(H, b, fixed_iters=K, flexible=True)
        x, st = s.solve(dvec(b), tol=0.0, maxit=K)
        assert st[0]["iters"] == K and rel(host(x), xo) <= vtol(H), rel(host(x), xo)
        Xs, stb = s.solve(dvec(X), tol=0.0, maxit=10)
        Xh = host(Xs)
        for j in (0, 7, 19):
            xo, _ = O.pcg(H, X[j], fixed_iters=10, flexible=True)
            assert stb[j]["iters"] == 10 and rel(Xh[j], xo) <= vtol(H), (j, rel(Xh[j], xo))
        s.set_precision(L.MIXED)
        A = H.levels[0].A
        x, st = s.solve(dvec(b), tol=1e-8, maxit=500)
        r = np.linalg.norm(b - A @ host(x)) / np.linalg.norm(b)
        assert st[0]["converged"] == 1 and r <= 1e-8
        assert st[0]["iters"] <= math.ceil(1.10 * K)
        Xm, stm = s.solve(dvec(X), tol=1e-8, maxit=500)
        Xh = host(Xm)
        for j in range(20):
            r = np.linalg.norm(X[j] - A @ Xh[j]) / np.linalg.norm(X[j])
            assert stm[j]["converged"] == 1 and r <= 1e-8, (j, r)
        for tol in (1e-14,):
            x, st = s.solve(dvec(b), tol=tol, maxit=60)
            assert st[0]["true_rel_res"] <= tol if st[0]["converged"] else st[0]["iters"] == 60
            Xr, str_ = s.solve(dvec(X[:8]), tol=tol, maxit=60)
            for j in range(8):
                if str_[j]["converged"]:
                    assert str_[j]["true_rel_res"] <= tol, (j, str_[j])
                else:
                    assert str_[j]["iters"] == 60, (j, str_[j])
    finally:
        s.set_option(L.OPT_KRYLOV, L.KRYLOV_CG)
        s.set_precision(L.FP64)


@pytest.fixture(scope="module")
def rot_add(gpu_device):
    """As rot, set up for the additive cycle (whole local inverses)."""
    p = P.aniso2d(64, math.pi / 6, 1e-4)
    H, s = build(p, 2, O.Params(cmin=(2,), max_coarse=150), cmin=(2,), max_coarse=150,
                 dense_tail=2000, cycle="additive")
    assert len(H.levels) >= 3 and s.info()["tail_level"] == -1   # no dense tail
    yield p, H, s
    s.close()


def test_additive_cycle(rot_add):
    """The additive multilevel cycle (sec. 3.1.1): one FP64 cycle equals the
    oracle's acycle to 1e-10 (FP32 to 1e-4); PCG with it at the oracle's
    stop count equals the oracle's iterate to 1e-10 and the converged solve
    stops within one iteration of it on a true residual at tolerance; the
    mixed solve converges within 1.1x the oracle's count; several right-hand
    sides are solved column by column (bitwise the single solves), and the
    multi-column V-cycle entry refuses the handle."""
    p, H, s = rot_add
    pre = lambda r: O.acycle(H, r)
    v = np.random.default_rng(21).standard_normal(p.n)
    try:
        s.set_precision(L.FP64)
        assert rel(host(s.apply(L.OP_VCYCLE, dvec(v))), O.acycle(H, v)) <= vtol(H)
        b = P.rhs_uniform(p.n, 0)
        xo, info = O.pcg(H, b, tol=1e-8, precond=pre)
        K = info["iters"]
        assert info["converged"] and info["restarts"] == 0
        x, st = s.solve(dvec(b), tol=0.0, maxit=K)
        assert st[0]["iters"] == K and rel(host(x), xo) <= vtol(H), rel(host(x), xo)
        x2, st2 = s.solve(dvec(b), tol=1e-8, maxit=1000)
        A = H.levels[0].A
        r = np.linalg.norm(b - A @ host(x2)) / np.linalg.norm(b)
        assert st2[0]["converged"] == 1 and abs(st2[0]["iters"] - K) <= 1 and r <= 1e-8
        X = np.stack([P.rhs_uniform(p.n, 30 + j) for j in range(3)])
        Xs, stb = s.solve(dvec(X), tol=1e-8, maxit=1000)
        for j in range(3):
            xj, _ = s.solve(dvec(X[j]), tol=1e-8, maxit=1000)
            assert np.array_equal(host(Xs)[j], host(xj)) and stb[j]["converged"] == 1
        with pytest.raises(L.LsamgError):
            s.apply_vcycle_batch(dvec(X))
        s.set_precision(L.MIXED)
        assert rel(host(s.apply(L.OP_VCYCLE, dvec(v))), O.acycle(H, v)) <= 1e-4
        xm, stm = s.solve(dvec(b), tol=1e-8, maxit=1000)
        r = np.linalg.norm(b - A @ host(xm)) / np.linalg.norm(b)
        assert stm[0]["converged"] == 1 and r <= 1e-8
        assert stm[0]["iters"] <= math.ceil(1.10 * K)
    finally:
        s.set_precision(L.FP64)


@pytest.mark.parametrize("which", ["rot", "rot_tail"])
def test_block_cg(which, request):
    """Block CG (LSAMG_KRYLOV_BLOCK) on 20 columns (44 zero columns of the
    64-column block drop out through the pseudo-inverse): the FP64 iterate
    after 4 iterations equals the oracle's block PCG to 1e-10; the converged
    solve reaches the tolerance on every column's true residual within the
    oracle's block iteration count + 1 (FP64) and within the CG count
    (mixed); a zero right-hand side stays zero."""
    p, H, s = request.getfixturevalue(which)
    X = np.stack([P.rhs_uniform(p.n, 700 + j) for j in range(20)])
    X[5] = 0.0
    A = H.levels[0].A
    Xo4, _ = O.block_pcg(H, X.T, fixed_iters=4)
    Xo, info = O.block_pcg(H, X.T, tol=1e-8)
    _, ic = O.pcg(H, X[0], tol=1e-8)
    s.set_option(L.OPT_KRYLOV, L.KRYLOV_BLOCK)
    try:
        s.set_precision(L.FP64)
        Xg, st = s.solve(dvec(X), tol=0.0, maxit=4)
        Xh = host(Xg)
        assert all(st[j]["iters"] == 4 for j in range(20))
        e = rel(Xh.T, Xo4)
        assert e <= vtol(H), e
        for prec, cap in ((L.FP64, info["iters"] + 1), (L.MIXED, ic["iters"])):
            s.set_precision(prec)
            Xg, st = s.solve(dvec(X), tol=1e-8, maxit=200)
            Xh = host(Xg)
            assert np.all(Xh[5] == 0.0)
            for j in range(20):
                if j == 5:
                    continue
                r = np.linalg.norm(X[j] - A @ Xh[j]) / np.linalg.norm(X[j])
                assert st[j]["converged"] == 1 and r <= 1e-8, (prec, j, r)
                assert st[j]["iters"] <= cap, (prec, st[j]["iters"], cap)
    finally:
        s.set_option(L.OPT_KRYLOV, L.KRYLOV_CG)
        s.set_precision(L.FP64)
