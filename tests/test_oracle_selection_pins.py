"""Pins of the oracle's eigenvector selection (section 3.4), the pseudo-
inverse Schur complement of eq:gevp-S on coarse levels, the coarse-level
block rule and the complexity statistics.

Each value checked here is fixed by something other than the oracle: the
geometry of the lattice (closed-form colour and overlap counts), a
brute-force QZ solution of the unreduced pencil eq:gevp, the minimum-energy
characterisation of the Schur complement computed by least squares on the
weighted rows of G, or counts derived by hand.  Each docstring names a
plausible mistake that the test catches.
"""
import math

import numpy as np
import pytest
import scipy.linalg as sla
import scipy.sparse as sp

import oracle as O
import problems as P

ROT = dict(theta=math.pi / 6, eps=1e-4)


@pytest.fixture(scope="module")
def rot32():
    """Rotated anisotropy, N = 32 (31 x 31 interior nodes, 8 x 8 blocks),
    threshold rule with c_min = 2 (cap 8 on 16-node aggregates)."""
    p = P.aniso2d(32, ROT["theta"], ROT["eps"])
    H = O.setup(p.G, 2, p.grid, O.Params(cmin=(2,), max_coarse=60))
    return p, H


@pytest.fixture(scope="module")
def rot48():
    """N = 48: 12 x 12 level-0 blocks, so level 1 has 3 x 3 blocks."""
    p = P.aniso2d(48, ROT["theta"], ROT["eps"])
    H = O.setup(p.G, 2, p.grid, O.Params(cmin=(2,), max_coarse=60, max_levels=3))
    return p, H


def test_colour_and_overlap_counts_closed_form(rot48):
    """On the 4 x 4 block lattice the rows of a rotated-anisotropy cell touch
    the nodes (i,j), (i+1,j), (i,j+1), so A has the 7-point pattern
    (E, W, N, S, NW, SE).  One-layer overlap then puts a block's top-left
    corner node in four Omega_i (its own block, the left, upper and
    upper-left ones): n_mult = 4.  Two blocks are adjacent in
    A(Omega_i, Omega_j) exactly when they are lattice neighbours including
    diagonals (their halos share a node), so the aggregate graph is the
    king's graph, whose index-order greedy colouring uses 4 colours.  Hence
    thresh = (50 - 4) / (4 * 4) = 2.875 on level 0, and the same on level 1
    (4 x 4 blocks of parent aggregates, the same stencil between parents).

    Caught: colouring the graph of omega adjacency A(omega_i, omega_j) (a
    triangular lattice: 3 colours), counting row multiplicities M (max 3)
    instead of Omega covers, or a threshold formula with other precedence."""
    p, H = rot48
    for l in (0, 1):
        L = H.levels[l]
        assert L.n_agg >= 9, l
        assert (L.n_color, L.n_mult) == (4, 4), (l, L.n_color, L.n_mult)
        assert L.thresh == 46.0 / 16.0


def test_colour_and_overlap_counts_isotropic():
    """theta = 0, eps = 1: every row of G has two entries (x or y
    difference), A is the 5-point Laplacian; a block corner node lies in
    three Omega_i (own, left or right, up or down): n_mult = 3.  Diagonal
    blocks still share halo nodes, so the king's graph again gives 4
    colours and thresh = 46 / 12."""
    p = P.aniso2d(32, 0.0, 1.0)
    H = O.setup(p.G, 2, p.grid, O.Params(max_levels=2, max_coarse=0))
    L = H.levels[0]
    assert (L.n_color, L.n_mult) == (4, 3)
    assert L.thresh == 46.0 / 12.0


def qz_count_above(Ai, At, nw, thresh):
    """Number of eigenvalues lambda > thresh of the unreduced pencil
    D A_i D u = lambda A~_i u (eq:gevp), infinite ones included, from the
    QZ algorithm in homogeneous form (alpha, beta)."""
    D = np.diag([1.0] * nw + [0.0] * (Ai.shape[0] - nw))
    ab = sla.eigvals(D @ Ai @ D, At, homogeneous_eigvals=True)
    alpha, beta = ab[0], ab[1]
    big = np.abs(alpha) > 0
    infinite = big & (np.abs(beta) <= 1e-9 * np.abs(alpha))
    finite = ~infinite & (np.abs(beta) > 0)
    lam = (alpha[finite] / beta[finite]).real
    return int(infinite.sum()) + int(np.sum(lam > thresh))


def test_threshold_count_brute_force(rot32):
    """k = #{lambda > thresh} (capped at floor(|omega| / c_min)) of section
    3.4, counted from a QZ solve of the full pencil eq:gevp (no Schur
    complement, no reversed form, no pseudo-inverse) for every level-0
    aggregate.  On this workload the threshold, not the cap, decides k on
    most aggregates (k = 7 of a possible 8 on interior ones).

    Caught: keeping the smallest lambda instead of the largest, comparing
    mu with thresh instead of 1/thresh, rounding the cap up, or a wrong
    thresh (all change k on some aggregate)."""
    p, H = rot32
    L = H.levels[0]
    below_cap = 0
    for i in range(L.n_agg):
        Om, nw = L.Omega[i], len(L.omega[i])
        Ai = L.A[Om][:, Om].toarray()
        At = O.lsamg.local_splitting(L.G, L.nz[i], Om, L.M)
        cnt = qz_count_above(Ai, At, nw, L.thresh)
        cap = nw // 2
        assert L.k[i] == max(1, min(cnt, cap)), (i, L.k[i], cnt, cap)
        below_cap += cnt < cap
    assert below_cap >= L.n_agg // 2


def test_threshold_count_cap_binds():
    """With c_min = 3 the cap floor(16/3) = 5 binds on interior aggregates
    (7 eigenvalues above thresh), floor(12/3) = 4 and floor(9/3) = 3 on the
    ragged ones: k = min(#{lambda > thresh}, cap) from the QZ count again.

    Caught: rounding the cap up (6 on 16-node aggregates)."""
    p = P.aniso2d(32, ROT["theta"], ROT["eps"])
    H = O.setup(p.G, 2, p.grid, O.Params(cmin=(3,), max_coarse=60, max_levels=2))
    L = H.levels[0]
    capped = 0
    for i in range(L.n_agg):
        Om, nw = L.Omega[i], len(L.omega[i])
        Ai = L.A[Om][:, Om].toarray()
        At = O.lsamg.local_splitting(L.G, L.nz[i], Om, L.M)
        cnt = qz_count_above(Ai, At, nw, L.thresh)
        assert L.k[i] == max(1, min(cnt, nw // 3)), (i, L.k[i], cnt)
        capped += cnt > nw // 3
    assert capped >= L.n_agg // 2


@pytest.fixture(scope="module")
def coarse_singular():
    """Level 1 of an LS_{3,4} hierarchy, where A~_GammaGamma is rank
    deficient (whole parent blocks of coarse unknowns share structure)."""
    p = P.aniso2d(40, ROT["theta"], ROT["eps"])
    H = O.setup(p.G, 2, p.grid, O.Params(cmin=(3, 4), max_coarse=60, max_levels=3))
    return p, H


def test_schur_equals_eq_gevp_s_when_nonsingular(rot32):
    """On level 0 every A~_GammaGamma is nonsingular and the least-squares
    Schur complement used by the setup equals eq:gevp-S as printed,
    A~_ww - A~_wG A~_GG^{-1} A~_Gw, with a plain solve.

    Caught: a wrong weight (W instead of W^{1/2} on the rows), an
    off-by-one split between omega and Gamma, or projecting B_w onto the
    range of B_Gamma instead of its complement."""
    p, H = rot32
    L = H.levels[0]
    for i in range(0, L.n_agg, 5):
        nz, Om, nw = L.nz[i], L.Omega[i], len(L.omega[i])
        At = O.lsamg.local_splitting(L.G, nz, Om, L.M)
        ref = At[:nw, :nw] - At[:nw, nw:] @ np.linalg.solve(At[nw:, nw:], At[nw:, :nw])
        St = O.lsamg.schur_ls(O.lsamg.weighted_rows(L.G, nz, Om, L.M), nw, 1e-12)
        assert np.abs(St - ref).max() <= 1e-9 * np.abs(At).max(), i


def test_schur_is_minimum_energy_when_singular(coarse_singular):
    """With a rank-deficient A~_GammaGamma (level 1), the Schur complement is
    the minimum energy: u^T S~ u = min over v of [u; v]^T A~ [u; v].  The
    minimiser is computed here column by column with a pivoted-QR least-
    squares solver (LAPACK gelsy), never with an SVD or with A~_GammaGamma;
    a random v never gives less energy.

    Caught: a plain inverse (singular block), keeping the numerically null
    singular directions, swapped off-diagonal blocks, or a dropped weight."""
    p, H = coarse_singular
    L = H.levels[1]
    rng = np.random.default_rng(3)
    checked = 0
    for i in range(L.n_agg):
        nz, Om, nw = L.nz[i], L.Omega[i], len(L.omega[i])
        if len(Om) == nw:
            continue
        B = O.lsamg.weighted_rows(L.G, nz, Om, L.M)
        Bw, Bg = B[:, :nw], B[:, nw:]
        sv = np.linalg.svd(Bg, compute_uv=False)
        if not np.any(sv < 1e-13 * sv[0]):
            continue                                    # A~_GG nonsingular
        V = sla.lstsq(Bg, -Bw, cond=1e-12, lapack_driver="gelsy")[0]
        E = Bw + Bg @ V
        ref = E.T @ E
        St = O.lsamg.schur_ls(B, nw, 1e-12)
        scale = np.abs(B.T @ B).max()
        assert np.abs(St - ref).max() <= 1e-8 * scale, i
        At = B.T @ B
        for _ in range(3):
            u = rng.standard_normal(nw)
            v = rng.standard_normal(len(Om) - nw)
            x = np.concatenate([u, v])
            assert u @ St @ u <= x @ At @ x + 1e-10 * scale * (x @ x)
        checked += 1
    assert checked >= 4


def test_coarse_block_rule_closed_form():
    """Coarse-level aggregation on the lattice of parent aggregates: with 4
    eigenvectors kept per level-0 aggregate (8 x 8 parents for N = 32) and
    omega_max = 36, the block shrinks from 4 (64 unknowns) to 3, whose
    largest aggregate (3 x 3 parents) holds exactly 36; the 8 parents per
    axis split as 3 + 3 + 2 (a remainder of 2 >= 3/2 stays a block of its
    own), giving 9 aggregates of 36, 24, 24, 36, ... unknowns.

    Caught: a strict '< omega_max' test (gives block 2), counting parents
    instead of unknowns (keeps block 4), or merging the remainder."""
    p = P.aniso2d(32, ROT["theta"], 1e-2)
    H = O.setup(p.G, 2, p.grid, O.Params(n_eig_fixed=4, omega_max=36, max_coarse=20,
                                          max_levels=3))
    assert np.all(H.levels[0].k == 4)
    L1 = H.levels[1]
    assert L1.block == 3 and L1.n_agg == 9
    sizes = sorted(len(w) for w in L1.omega)
    assert sizes == sorted([36] * 4 + [24] * 4 + [16])


def test_stats_closed_form():
    """Operator and smoother complexity on the isotropic N = 32 two-level
    hierarchy, from the geometry alone: nnz(A_0) = 961 + 4 * 31 * 30 (5-point
    pattern); A_1 = P^T A P couples two aggregates exactly when A couples
    their nodes (the 4-neighbour block graph: diagonal blocks meet only at a
    corner, where the 5-point stencil has no entry), giving
    sum_a k_a^2 + sum_{a~b} k_a k_b entries; |Omega_i| = |omega_i| plus one
    side of halo for every block side that is not on the boundary.

    Caught: counting A_1's diagonal-block couplings, leaving out the
    coarsest level, or dividing by nnz(G) instead of nnz(A_0)."""
    p = P.config1()
    H = O.setup(p.G, 2, p.grid, O.Params(max_levels=2, max_coarse=0, block=4,
                                          n_eig_fixed=4))
    L0 = H.levels[0]
    nnz0 = 961 + 4 * 31 * 30
    k = L0.k.reshape(8, 8)              # aggregate id = bx + 8 by
    nnz1 = int((k ** 2).sum() + 2 * (k[:, 1:] * k[:, :-1]).sum()
               + 2 * (k[1:, :] * k[:-1, :]).sum())
    widths = [4] * 7 + [3]
    se = 0
    for by in range(8):
        for bx in range(8):
            a, b = widths[bx], widths[by]
            halo = b * ((bx > 0) + (bx < 7)) + a * ((by > 0) + (by < 7))
            se += a * b * (a * b + halo)
    s = O.stats(H)
    assert s["nnz_A"] == [nnz0, nnz1]
    assert s["op_complexity"] == (nnz0 + nnz1) / nnz0
    assert s["smoother_complexity"] == se / nnz0
