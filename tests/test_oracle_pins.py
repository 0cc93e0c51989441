"""Pins of the FP64 oracle against what the paper and the mathematics fix.

Each test checks the oracle against something other than itself: an exact
identity stated in the paper (the SPSD splitting Lemma of sec. 3.1.1, the
partition of unity eq:PoU, RAS-T = RAS^T after eq:ras-t, A_{l+1} = P^T A P =
G_{l+1}^T G_{l+1} of sec. 3.1.3), a special case that reduces to a direct
solve, a brute-force QZ solution of the unreduced eigenproblem eq:gevp, the
additive two-level bound of sec. 3.1.1, or a closed-form count.
"""
import math

import numpy as np
import pytest
import scipy.linalg as sla
import scipy.sparse as sp

import oracle as O
import problems as P


@pytest.fixture(scope="module")
def cfg1():
    p = P.config1()
    H = O.setup(p.G, 2, p.grid, O.Params(max_levels=2, max_coarse=0, block=4,
                                          n_eig_fixed=4))
    return p, H


@pytest.fixture(scope="module")
def rot():
    """Small rotated-anisotropic multilevel hierarchy (>= 3 levels)."""
    p = P.aniso2d(24, math.pi / 6, 1e-4)
    H = O.setup(p.G, 2, p.grid, O.Params(cmin=(2,), max_coarse=60))
    assert len(H.levels) >= 3
    return p, H


def assemble_split(L):
    n = L.n
    S = np.zeros((n, n))
    for i in range(L.n_agg):
        At = O.lsamg.local_splitting(L.G, L.nz[i], L.Omega[i], L.M)
        S[np.ix_(L.Omega[i], L.Omega[i])] += At
    return S


# P1 -- the local splitting sums to A (Lemma, sec. 3.1.1)
def test_splitting_exact_config1(cfg1):
    p, H = cfg1
    L = H.levels[0]
    S = assemble_split(L)
    # entries of G are +-32 and weights 1 or 1/2: every sum is exact in FP64
    assert np.array_equal(S, L.A.toarray())


def test_splitting_rotated_all_levels(rot):
    p, H = rot
    for L in H.levels[:-1]:
        S = assemble_split(L)
        Ad = (L.G.T @ L.G).toarray()
        assert np.abs(S - Ad).max() <= 1e-13 * np.abs(Ad).max()


# P2 -- every A~_i is SPSD
def test_splitting_spsd(rot):
    p, H = rot
    for L in H.levels[:-1]:
        for i in range(L.n_agg):
            At = O.lsamg.local_splitting(L.G, L.nz[i], L.Omega[i], L.M)
            ev = np.linalg.eigvalsh(At)
            assert ev.min() >= -1e-13 * max(ev.max(), 1.0)


# P3 -- Boolean partition of unity (eq:PoU, eq:pou2)
def test_partition_of_unity(rot):
    p, H = rot
    for L in H.levels[:-1]:
        cnt = np.zeros(L.n, dtype=np.int64)
        for i in range(L.n_agg):
            cnt[L.omega[i]] += 1
            assert np.array_equal(L.Omega[i][:len(L.omega[i])], L.omega[i])
            assert np.intersect1d(L.gamma[i], L.omega[i]).size == 0
        assert np.all(cnt == 1)


# P4 -- theta = 0, eps = 1 is the 5-point Laplacian (sec. 4.1)
def test_five_point(cfg1):
    p, H = cfg1
    A = H.levels[0].A.toarray() * p.h ** 2
    assert np.array_equal(np.diag(A), np.full(p.n, 4.0))
    off = A - np.diag(np.diag(A))
    assert set(np.unique(off)) <= {-1.0, 0.0}
    assert np.all((off != 0).sum(axis=1) <= 4)


# P5 -- mu = 1/lambda lies in [0, 1]; mu = 0 where the constant is in the
# null space of A~_i (aggregates whose rows avoid the Dirichlet boundary)
def test_mu_range_and_constant_mode(rot):
    p, H = rot
    L = H.levels[0]
    G = L.G
    rowsum = np.abs(np.asarray(G.sum(axis=1)).ravel())
    scale = np.abs(G).max()
    n_interior = 0
    for i in range(L.n_agg):
        mu = L.mu[i]
        assert mu.min() >= -1e-12 and mu.max() <= 1 + 1e-12
        if np.all(rowsum[L.nz[i]] <= 1e-12 * scale):
            n_interior += 1
            assert mu[0] <= 1e-10
        else:
            assert mu[0] > 1e-10
    assert n_interior > 0


# brute force: the reduced problem eq:gevp-S has the finite nonzero
# eigenvalues of the full pencil eq:gevp, D A_i D u = lambda A~_i u (QZ)
def test_schur_reduction_matches_full_pencil(cfg1):
    p, H = cfg1
    L = H.levels[0]
    for i in (0, 9, 27, 63):
        Om, nw = L.Omega[i], len(L.omega[i])
        Ai = L.A[Om][:, Om].toarray()
        D = np.diag([1.0] * nw + [0.0] * (len(Om) - nw))
        At = O.lsamg.local_splitting(L.G, L.nz[i], Om, L.M)
        lam = sla.eigvals(D @ Ai @ D, At)
        lam = lam[np.isfinite(lam)]
        lam = np.sort(lam.real[(np.abs(lam) > 1e-8) & (np.abs(lam) < 1e8)])
        mu = L.mu[i]
        ref = np.sort(1.0 / mu[mu > 1e-8])
        assert lam.size == ref.size
        assert np.allclose(lam, ref, rtol=1e-8)


# closed-form counts of config 1: 64 aggregates of 16/12/9 nodes; k = 4 per
# aggregate except the two corner aggregates whose reflection symmetry makes
# the 4th and 5th eigenvalues equal, where the cut moves down to 3
def test_config1_counts(cfg1):
    p, H = cfg1
    L = H.levels[0]
    sizes = np.bincount([len(w) for w in L.omega])
    assert sizes[16] == 49 and sizes[12] == 14 and sizes[9] == 1
    assert L.n_agg == 64
    assert L.k.sum() == 254
    assert L.k[0] == 3 and L.k[63] == 3
    assert abs(L.mu[0][3] - L.mu[0][4]) < 1e-12


def test_axis_blocks_rule():
    ab = O.lsamg.axis_blocks
    assert ab(31, 4).max() + 1 == 8 and np.sum(ab(31, 4) == 7) == 3     # 7x4 + 3
    b = ab(127, 3)                                                    # 42x3 + 1
    assert b.max() + 1 == 42 and np.sum(b == 41) == 4
    assert ab(511, 4).max() + 1 == 128
    assert np.all(ab(3, 4) == 0)


# P6 -- P is block diagonal by aggregate, full column rank (eq:mg-p)
def test_interpolation_structure(cfg1):
    p, H = cfg1
    L = H.levels[0]
    Pd = L.P.toarray()
    off = np.concatenate([[0], np.cumsum(L.k)])
    for i in range(L.n_agg):
        cols = Pd[:, off[i]:off[i + 1]]
        rows = np.nonzero(np.any(cols != 0, axis=1))[0]
        assert np.all(np.isin(rows, L.omega[i]))
    assert np.linalg.matrix_rank(Pd) == Pd.shape[1]
    # A_ww-orthonormal columns
    for i in range(L.n_agg):
        w = L.omega[i]
        Z = L.Zhat[i]
        Aww = L.A[w][:, w].toarray()
        assert np.allclose(Z.T @ Aww @ Z, np.eye(Z.shape[1]), atol=1e-10)


# P7 -- A_{l+1} = P^T A_l P = G_{l+1}^T G_{l+1} and it is SPD (sec. 3.1.3)
def test_galerkin_least_squares(rot):
    p, H = rot
    for l in range(len(H.levels) - 1):
        L, N = H.levels[l], H.levels[l + 1]
        gal = (L.P.T @ L.A @ L.P).toarray()
        ls = (N.G.T @ N.G).toarray()
        assert np.abs(gal - ls).max() <= 1e-12 * np.abs(gal).max()
        np.linalg.cholesky(ls)


def dense_op(f, n):
    M = np.zeros((n, n))
    for j in range(n):
        e = np.zeros(n)
        e[j] = 1.0
        M[:, j] = f(e)
    return M


# P8 -- RAS-T is the transpose of RAS (after eq:ras-t); the V-cycle is symmetric
def test_rast_is_transpose(cfg1):
    p, H = cfg1
    L = H.levels[0]
    R = dense_op(lambda v: O.ras(L, v), L.n)
    RT = dense_op(lambda v: O.ras_t(L, v), L.n)
    assert np.abs(RT - R.T).max() <= 1e-13 * np.abs(R).max()


def test_vcycle_symmetric(rot):
    p, H = rot
    rng = np.random.default_rng(7)
    x, y = rng.standard_normal((2, p.n))
    a = x @ O.vcycle(H, y)
    b = y @ O.vcycle(H, x)
    assert abs(a - b) <= 1e-12 * max(abs(a), abs(b))


# two-grid error propagation: I - B A = (I - S^T A)(I - P A_c^{-1} P^T A)(I - S A)
def test_two_grid_error_propagation(cfg1):
    p, H = cfg1
    L = H.levels[0]
    n = L.n
    A = L.A.toarray()
    S = dense_op(lambda v: O.ras(L, v), n)
    Pd = L.P.toarray()
    Ac = Pd.T @ A @ Pd
    I = np.eye(n)
    E = (I - S.T @ A) @ (I - Pd @ np.linalg.solve(Ac, Pd.T @ A)) @ (I - S @ A)
    B = dense_op(lambda v: O.vcycle(H, v), n)
    assert np.abs((I - B @ A) - E).max() <= 1e-10


# P9 -- B is SPD (claim of sec. 3.1.1) and the V-cycle contracts: eig(BA) in (0, 1]
def test_preconditioner_spd(cfg1):
    p, H = cfg1
    B = dense_op(lambda v: O.vcycle(H, v), p.n)
    assert np.abs(B - B.T).max() <= 1e-12 * np.abs(B).max()
    ev = np.linalg.eigvalsh(0.5 * (B + B.T))
    assert ev.min() > 0
    A = H.levels[0].A.toarray()
    Lc = np.linalg.cholesky(A)
    evBA = np.linalg.eigvalsh(Lc.T @ B @ Lc)
    assert evBA.min() > 0 and evBA.max() <= 1 + 1e-10


# P10 -- PCG reaches the direct solution
def test_pcg_matches_direct(cfg1):
    p, H = cfg1
    b = P.rhs_uniform(p.n, 0)
    x, info = O.pcg(H, b, tol=1e-13)
    xd = sla.cho_solve(sla.cho_factor(H.levels[0].A.toarray()), b)
    assert np.linalg.norm(x - xd) <= 1e-10 * np.linalg.norm(xd)
    assert info["true_rel_res"] <= 1e-12


# P11 -- keeping every eigenvector makes P square and invertible: the coarse
# correction is exact, B = A^{-1} and PCG converges in one iteration
def test_full_coarse_space_is_direct():
    p = P.aniso2d(12, 0.4, 0.1)
    H = O.setup(p.G, 2, p.grid, O.Params(max_levels=2, max_coarse=0, block=4,
                                          n_eig_fixed=1000))
    assert H.levels[1].n == p.n
    b = P.rhs_uniform(p.n, 3)
    xd = np.linalg.solve(H.levels[0].A.toarray(), b)
    assert np.linalg.norm(O.vcycle(H, b) - xd) <= 1e-10 * np.linalg.norm(xd)
    x, info = O.pcg(H, b, tol=1e-10)
    assert info["iters"] == 1


# P12 -- one aggregate covering the domain: Gamma empty, M = 1, A~ = A,
# every mu = 1 and RAS = A^{-1}
def test_single_aggregate():
    p = P.aniso2d(10, 0.3, 0.05)
    H = O.setup(p.G, 2, p.grid, O.Params(max_levels=2, max_coarse=0, block=9,
                                          omega_max=10000, n_eig_fixed=3))
    L = H.levels[0]
    assert L.n_agg == 1 and L.gamma[0].size == 0 and np.all(L.M == 1)
    At = O.lsamg.local_splitting(L.G, L.nz[0], L.Omega[0], L.M)
    assert np.allclose(At, L.A.toarray(), rtol=0, atol=1e-12 * np.abs(At).max())
    assert np.allclose(L.mu[0], 1.0, atol=1e-10)
    b = P.rhs_uniform(p.n, 4)
    xd = np.linalg.solve(L.A.toarray(), b)
    assert np.linalg.norm(O.ras(L, b) - xd) <= 1e-11 * np.linalg.norm(xd)


# P13 -- additive two-level bound of sec. 3.1.1: lambda_max(M2^{-1} A) <= k_c + 1
# with M1^{-1} the additive Schwarz operator (eq:ras without the PoU)
def test_additive_two_level_upper_bound():
    p = P.aniso2d(16, math.pi / 6, 1e-2)
    H = O.setup(p.G, 2, p.grid, O.Params(max_levels=2, max_coarse=0, block=4,
                                          cmin=(2,)))
    L = H.levels[0]
    n = L.n
    A = L.A.toarray()
    AS = np.zeros((n, n))
    for i in range(L.n_agg):
        Om = L.Omega[i]
        AS[np.ix_(Om, Om)] += np.linalg.inv(A[np.ix_(Om, Om)])
    Pd = L.P.toarray()
    M2 = Pd @ np.linalg.solve(Pd.T @ A @ Pd, Pd.T) + AS
    ev = np.linalg.eigvals(M2 @ A).real
    assert ev.max() <= L.n_color + 1 + 1e-8
    assert ev.min() > 0
    # the oracle's additive cycle on two levels is this M_2 (exact coarse
    # solve), and its smoother this additive Schwarz sum
    v = P.rhs_uniform(n, 6)
    assert np.linalg.norm(O.additive_schwarz(L, v) - AS @ v) <= 1e-12 * np.linalg.norm(AS @ v)
    assert np.linalg.norm(O.acycle(H, v) - M2 @ v) <= 1e-11 * np.linalg.norm(M2 @ v)


def test_additive_cycle_multilevel(rot):
    """The multilevel additive cycle is the recursion B_l = M_{1,l}^{-1} +
    P_l B_{l+1} P_l^T with B_L = A_L^{-1}, written out here with dense
    matrices (inverted local blocks, explicit P_l) from the finest level
    down; it is symmetric and positive definite, its spectrum against A is
    bounded above by the two-level bound's k_c + 1 summed over the levels
    (each term is an A-bounded projection sum), and PCG with it reaches
    1e-8 on the true residual.  A dropped coarse term, a transposed P or the
    RAS partition of unity in the smoother fails one of these."""
    p, H = rot
    Bd = np.linalg.inv(H.levels[-1].A.toarray())
    bound = 1.0
    for L in reversed(H.levels[:-1]):
        A = L.A.toarray()
        AS = np.zeros_like(A)
        for i in range(L.n_agg):
            Om = L.Omega[i]
            AS[np.ix_(Om, Om)] += np.linalg.inv(A[np.ix_(Om, Om)])
        Pd = L.P.toarray()
        Bd = AS + Pd @ Bd @ Pd.T
        bound += L.n_color
    v = P.rhs_uniform(p.n, 7)
    y = O.acycle(H, v)
    assert np.linalg.norm(y - Bd @ v) <= 1e-11 * np.linalg.norm(Bd @ v)
    w = P.rhs_uniform(p.n, 8)
    assert abs(w @ O.acycle(H, v) - v @ O.acycle(H, w)) <= 1e-12 * np.linalg.norm(v) * np.linalg.norm(y) * 10
    A0 = H.levels[0].A.toarray()
    ev = np.linalg.eigvals(Bd @ A0).real
    assert ev.min() > 0 and ev.max() <= bound + 1e-8
    b = P.rhs_uniform(p.n, 9)
    x, info = O.pcg(H, b, tol=1e-8, precond=lambda r: O.acycle(H, r))
    assert info["converged"]
    assert np.linalg.norm(b - A0 @ x) <= 1e-8 * np.linalg.norm(b)


# P14 -- any basis of span(Zhat_i) gives the same preconditioner
def test_basis_invariance(rot):
    p, _ = rot
    rng = np.random.default_rng(11)

    def hook(level, i, Z):
        Q, _ = np.linalg.qr(rng.standard_normal((Z.shape[1], Z.shape[1])))
        return Z @ Q * 1.7

    prm = O.Params(cmin=(2,), max_coarse=60)
    H1 = O.setup(p.G, 2, p.grid, prm)
    H2 = O.setup(p.G, 2, p.grid, prm, basis_hook=hook)
    v = rng.standard_normal(p.n)
    a, b = O.vcycle(H1, v), O.vcycle(H2, v)
    assert np.linalg.norm(a - b) <= 1e-11 * np.linalg.norm(a)


def test_stats_fields(cfg1):
    p, H = cfg1
    s = O.stats(H)
    assert s["levels"] == 2 and s["n"] == [961, 254]
    assert s["op_complexity"] > 1 and s["smoother_complexity"] > 1


def test_assembled_vcycle(rot):
    """The assembled form of the solve phase (one CSR smoother per level, its
    transpose for RAS-T) is the same operator as the per-aggregate Cholesky
    form: the smoother matrix applies eq:ras column by column, its transpose
    eq:ras-t, it has sum_i |omega_i||Omega_i| entries, and the assembled
    V-cycle and PCG iterates equal the oracle's to 1e-13.  (Taking the
    Omega-columns of A_i^{-1} on omega instead of its omega-rows would give
    RAS-T in place of RAS and fail the first check.)"""
    p, H = rot
    AV = O.AssembledVcycle(H)
    L = H.levels[0]
    S = AV.S[0].toarray()
    R = dense_op(lambda v: O.ras(L, v), L.n)
    RT = dense_op(lambda v: O.ras_t(L, v), L.n)
    assert np.abs(S - R).max() <= 1e-13 * np.abs(R).max()
    assert np.abs(AV.ST[0].toarray() - RT).max() <= 1e-13 * np.abs(R).max()
    for l, Sl in enumerate(AV.S):
        Lv = H.levels[l]
        assert Sl.nnz == sum(len(w) * len(Om) for w, Om in zip(Lv.omega, Lv.Omega))
    v = np.random.default_rng(11).standard_normal(p.n)
    y = O.vcycle(H, v)
    assert np.linalg.norm(AV(v) - y) <= 1e-13 * np.linalg.norm(y)
    b = P.rhs_uniform(p.n, 0)
    x1, i1 = O.pcg(H, b, fixed_iters=8)
    x2, i2 = O.pcg(H, b, fixed_iters=8, precond=AV)
    assert np.linalg.norm(x2 - x1) <= 1e-13 * np.linalg.norm(x1)


def test_row_compression_is_exact():
    """Replacing each group of coarse rows of G_{l+1} = G_l P_l that touch the
    same parent aggregates by the R factor of their QR leaves the hierarchy
    unchanged: the same aggregates, Omega lists and counts on every level,
    eigenvalues to 1e-12, A_1 = P_0^T A_0 P_0 to 1e-13 (deeper A_l depend on
    the basis picked inside near-degenerate eigenvalue clusters, which
    rounding may turn), and the V-cycle, which depends only on the spans, to
    1e-12; the compressed factor has fewer rows."""
    p = P.aniso2d(40, math.pi / 6, 1e-4)
    prm = dict(cmin=(2,), max_coarse=60)
    H1 = O.setup(p.G, 2, p.grid, O.Params(**prm))
    H2 = O.setup(p.G, 2, p.grid, O.Params(compress_rows=True, **prm))
    assert len(H1.levels) == len(H2.levels) >= 3
    for l, (a, b) in enumerate(zip(H1.levels, H2.levels)):
        if l <= 1:
            assert abs(a.A - b.A).max() <= 1e-13 * abs(a.A).max()
        if l > 0:
            assert b.G.shape[0] < a.G.shape[0]
        if a.coarsest:
            continue
        assert np.array_equal(a.agg, b.agg) and np.array_equal(a.k, b.k)
        assert all(np.array_equal(x, y) for x, y in zip(a.Omega, b.Omega))
        for x, y in zip(a.mu, b.mu):
            assert np.abs(x - y).max() <= 1e-12
    v = np.random.default_rng(5).standard_normal(p.n)
    y1, y2 = O.vcycle(H1, v), O.vcycle(H2, v)
    assert np.linalg.norm(y1 - y2) <= 1e-12 * np.linalg.norm(y1)


def test_flexible_cg_equals_cg_with_symmetric_preconditioner(rot):
    """With the (symmetric, fixed) V-cycle, flexible CG's A-orthogonalised
    direction beta = -(z_{k+1}.q_k)/(p_k.q_k) equals the standard
    beta = rho_{k+1}/rho_k in exact arithmetic, so both give the same iterates
    (to 1e-10 after 12 iterations) and reach 1e-8 at the same count; a sign
    error in either beta would part them after the first iteration."""
    p, H = rot
    b = P.rhs_uniform(p.n, 3)
    x1, i1 = O.pcg(H, b, fixed_iters=12)
    x2, i2 = O.pcg(H, b, fixed_iters=12, flexible=True)
    assert np.linalg.norm(x2 - x1) <= 1e-10 * np.linalg.norm(x1)
    _, c1 = O.pcg(H, b, tol=1e-8)
    _, c2 = O.pcg(H, b, tol=1e-8, flexible=True)
    assert c1["converged"] and c2["converged"] and abs(c1["iters"] - c2["iters"]) <= 1


def test_block_pcg(rot):
    """Block PCG (O'Leary) pins: (1) on one column it is CG (same iterate
    after 12 iterations to 1e-10); (2) after k iterations every column's
    A-norm error is at most that of its own CG after k iterations, since its
    iterate minimises the error over the sum of all columns' Krylov spaces,
    which contains its own (strictly smaller on every column here); (3) a
    repeated right-hand side makes the block Gram matrix singular: the
    pseudo-inverse drops the dependent direction and both copies equal the
    solve without the repeat; (4) all columns converge on their true
    residuals within the CG count.  A sign error in D, directions not
    A-orthogonalised against the previous block (P = Z), or a plain inverse
    of the singular Gram matrix fails one of these.  (P^T R and Z^T R are
    equal here in exact arithmetic, since the previous block is orthogonal
    to the new residual, so either may form C.)"""
    p, H = rot
    A = H.levels[0].A.toarray()
    b = P.rhs_uniform(p.n, 11)
    x1, _ = O.pcg(H, b, fixed_iters=12)
    xb, _ = O.block_pcg(H, b[:, None], fixed_iters=12)
    assert np.linalg.norm(xb[:, 0] - x1) <= 1e-10 * np.linalg.norm(x1)
    B = np.stack([P.rhs_uniform(p.n, 20 + j) for j in range(6)], axis=1)
    xs = np.linalg.solve(A, B)
    k = 4
    Xb, _ = O.block_pcg(H, B, fixed_iters=k)
    for j in range(6):
        xc, _ = O.pcg(H, B[:, j], fixed_iters=k)
        eb, ec = Xb[:, j] - xs[:, j], xc - xs[:, j]
        assert eb @ A @ eb < (ec @ A @ ec) * (1 - 1e-6), j
    B2 = np.concatenate([B[:, :3], B[:, :1], B[:, 3:]], axis=1)
    X2, _ = O.block_pcg(H, B2, fixed_iters=6)
    X1, _ = O.block_pcg(H, B, fixed_iters=6)
    assert np.linalg.norm(X2[:, 0] - X2[:, 3]) <= 1e-12 * np.linalg.norm(X2[:, 0])
    keep = [0, 1, 2, 4, 5, 6]
    assert np.linalg.norm(X2[:, keep] - X1) <= 1e-9 * np.linalg.norm(X1)
    Xc, info = O.block_pcg(H, B, tol=1e-8)
    _, ic = O.pcg(H, B[:, 0], tol=1e-8)
    assert info["converged"] and info["true_rel_res"].max() <= 1e-8
    assert info["iters"] <= ic["iters"]
