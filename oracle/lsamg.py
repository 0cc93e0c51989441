"""FP64 reference of LS-AMG-DD setup and solve (test infrastructure only).

Section references are to the paper (Southworth, Al Daas, Wimmer,
Threlfall, "Algebraic Multigrid with Overlapping Schwarz Smoothers and Local
Spectral Coarse Grids for Least Squares Problems").

Setup follows Algorithm 1 (section 3.2): per level, lattice aggregation,
one-layer overlap, Boolean partition of unity (eq:pou2), the multiplicity-
weighted SPSD splitting of the Lemma in section 3.1.1 (eq:local_splitting),
the reduced local generalized eigenproblem eq:gevp-S (section 3.1.2), the
eigenvector selection of section 3.4, the block-diagonal interpolation
eq:mg-p and the least-squares propagation ``G_{l+1} = G_l P_l`` of section
3.1.3.  Solve is preconditioned CG around a V-cycle with one RAS (eq:ras)
pre-smoothing and one RAS-T (eq:ras-t) post-smoothing per level and an exact
coarsest solve (sections 2.1, 3.1.1).

Readings taken where the paper is silent or ambiguous (each is also listed in
the design notes of the repository):

* aggregation: lattice blocks of ``b`` points per axis, a remainder narrower
  than ``b/2`` merged into the last block; coarse levels aggregate the
  lattice of parent aggregates, with ``b`` shrunk per level until the largest
  aggregate has at most ``omega_max`` unknowns;
* overlap: ``Gamma_i`` = the columns, outside ``omega_i``, of the rows of G
  that have a structural nonzero in ``omega_i``; coarse-level structure is
  symbolic (a row touches every coarse unknown of every parent aggregate it
  touched);
* eigenproblem: solved in the reversed, well-posed form
  ``S_omega u = mu A_omega_omega u`` with ``lambda = 1/mu`` (``mu = 0`` is
  ``lambda = infinity``); ``(A~_GammaGamma)^{-1}`` is the Moore-Penrose
  pseudo-inverse, i.e. the Schur complement is the minimum energy over
  ``u_Gamma``, computed as ``B_w^T (I - Q Q^T) B_w`` from the weighted rows
  ``B = W^{1/2} G_{nz,Omega}`` (Q: range of ``B_Gamma``, singular values at
  or below ``pinv_rtol`` = 1e-6 times the largest counted as zero: the
  eigenvalue cutoff 1e-12 of ``A~_GammaGamma = B_G^T B_G``, far enough above
  rounding that two FP64 codes make the same rank decision);
* selection: ``k = #{lambda > thresh}`` capped at ``floor(|omega|/c_min)``
  (or a fixed count), at least one, and never splitting a cluster of equal
  eigenvalues (the cut moves down to the cluster start, or up to its end if
  that would leave none); ``n_color`` is the greedy colouring (index order)
  of the aggregate graph ``A(Omega_i, Omega_j) != 0`` and ``n_multiplicity``
  the largest number of overlapping aggregates sharing an unknown;
* eigenvectors are ``A_omega_omega``-orthonormal, ascending ``mu``, sign
  such that the largest-magnitude entry (first on ties) is positive;
* PCG stops when the recurrence residual and the true residual both satisfy
  ``||r|| <= tol ||b||`` (2-norm, x0 = 0); a recurrence residual that passes
  while the true one does not is replaced by it and CG restarts.
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import Callable, Optional

import numpy as np
import scipy.linalg as sla
import scipy.sparse as sp


# --------------------------------------------------------------------------
# parameters
# --------------------------------------------------------------------------
@dataclass
class Params:
    """Inputs of Algorithm 1 (section 3.2) plus the readings' knobs."""
    max_levels: int = 10            # L_max
    max_coarse: int = 2000          # n_coarse
    block: int = 4                  # lattice block per axis on level 0
    omega_max: int = 800            # largest aggregate on coarse levels
    n_eig_fixed: int = 0            # > 0: fixed count per aggregate
    kappa: float = 50.0             # target condition number (section 3.4)
    cmin: tuple = (3, 4)            # per-level minimum coarsening ratio
    tie_rtol: float = 1e-8          # eigenvalue-cluster tolerance
    tie_atol: float = 1e-12
    pinv_rtol: float = 1e-6         # rank cutoff of W^{1/2} G_{nz, Gamma} (singular values)
    thresh_margin: float = 1e-10    # strict side of the threshold test
    stall_ratio: float = 0.9        # stop if n_{l+1} > stall_ratio * n_l
    aggregation: str = "lattice"    # "lattice" blocks or "standard" (sec. 3.3)
    compress_rows: bool = False     # coarse G_l: each group of rows touching the same
                                    # parent aggregates replaced by its QR R factor
    agg_passes: tuple = (1,)        # n_agg of Algorithm 1 per level (last repeats)

    def cmin_at(self, level: int) -> int:
        c = tuple(self.cmin)
        return int(c[min(level, len(c) - 1)])

    def passes_at(self, level: int) -> int:
        c = tuple(self.agg_passes)
        return int(c[min(level, len(c) - 1)])


# --------------------------------------------------------------------------
# per-level data
# --------------------------------------------------------------------------
@dataclass
class Level:
    G: sp.csr_matrix                 # m x n values of G_l
    S: sp.csr_matrix                 # m x n symbolic structure of G_l (0/1)
    A: sp.csr_matrix                 # n x n, A_l = G_l^T G_l
    coord: np.ndarray                # (n, ndim) lattice coordinate per unknown
    extent: tuple                    # lattice extent per axis
    coarsest: bool = False
    # aggregation and overlap (non-coarsest levels)
    block: int = 0
    agg: Optional[np.ndarray] = None          # aggregate id per unknown
    n_agg: int = 0
    agg_coord: Optional[np.ndarray] = None    # (n_agg, ndim) block coordinate
    agg_extent: tuple = ()
    omega: list = field(default_factory=list)
    gamma: list = field(default_factory=list)
    Omega: list = field(default_factory=list)
    nz: list = field(default_factory=list)
    M: Optional[np.ndarray] = None
    # spectral coarse space
    n_color: int = 0
    n_mult: int = 0
    thresh: float = 0.0
    mu: list = field(default_factory=list)
    k: Optional[np.ndarray] = None
    Zhat: list = field(default_factory=list)
    P: Optional[sp.csr_matrix] = None
    hazards: list = field(default_factory=list)
    # smoother: Cholesky factors of A_i = A(Omega_i, Omega_i)
    chol: list = field(default_factory=list)
    # coarsest: Cholesky factor of the dense A_L
    chol_coarse: object = None

    @property
    def n(self) -> int:
        return self.A.shape[0]


@dataclass
class Hierarchy:
    levels: list
    params: Params


# --------------------------------------------------------------------------
# aggregation (reading: lattice blocks, see module docstring)
# --------------------------------------------------------------------------
def axis_blocks(extent: int, b: int) -> np.ndarray:
    """Block id of every lattice index 0..extent-1 for block width ``b``.

    ``extent = q b + r``: ``q`` blocks of width ``b``; a remainder ``r`` with
    ``2r < b`` is merged into the last block, otherwise it forms a block of
    its own.  An extent below ``b`` is one block.
    """
    x = np.arange(extent)
    q, r = divmod(extent, b)
    if q == 0:
        return np.zeros(extent, dtype=np.int64)
    if r == 0 or 2 * r >= b:
        return x // b
    return np.minimum(x // b, q - 1)


def aggregate_lattice(coord: np.ndarray, extent: tuple, b: int):
    """Aggregate id (x-fastest over block coordinates) of every unknown."""
    ndim = len(extent)
    ids = []
    nblk = []
    for d in range(ndim):
        blk = axis_blocks(extent[d], b)
        ids.append(blk[coord[:, d]])
        nblk.append(int(blk.max()) + 1)
    agg = np.zeros(coord.shape[0], dtype=np.int64)
    stride = 1
    for d in range(ndim):
        agg += ids[d] * stride
        stride *= nblk[d]
    n_agg = stride
    agg_coord = np.zeros((n_agg, ndim), dtype=np.int64)
    rem = np.arange(n_agg)
    for d in range(ndim):
        agg_coord[:, d] = rem % nblk[d]
        rem //= nblk[d]
    return agg, n_agg, agg_coord, tuple(nblk)


def choose_block(coord, extent, b0: int, omega_max: int):
    """Largest block width ``b <= b0`` whose largest aggregate has at most
    ``omega_max`` unknowns (each lattice point carries its unknowns)."""
    for b in range(b0, 0, -1):
        agg, n_agg, agg_coord, nblk = aggregate_lattice(coord, extent, b)
        sizes = np.bincount(agg, minlength=n_agg)
        if sizes.max() <= omega_max or b == 1:
            return b, agg, n_agg, agg_coord, nblk


# --------------------------------------------------------------------------
# aggregation on matrix entries (section 3.3, Algorithm 1)
# --------------------------------------------------------------------------
def standard_aggregation(adj: sp.csr_matrix):
    """Aggregates of the graph ``adj`` (structural off-diagonal pattern of a
    matrix), by the greedy passes of standard aggregation (Vanek, Mandel,
    Brezina) taken directly on matrix entries, nodes visited in index order:

    1. a node whose neighbours are all unaggregated starts a new aggregate
       holding it and its neighbours;
    2. a node left over joins the aggregate (from pass 1) of its
       lowest-numbered neighbour that pass 1 aggregated.

    A node that pass 1 did not take had, when it was visited, a neighbour
    already in an aggregate, so pass 2 places every remaining node and the
    clean-up pass of the general method (for nodes whose strong connections
    were all dropped) has nothing to do; a node without neighbours starts its
    own aggregate in pass 1.  This is what the paper's extra assignment of
    unaggregated nodes to a neighbouring aggregate guarantees.  Aggregate
    ids are numbered in order of creation.  Returns ``(agg, n_agg)``.
    """
    adj = sp.csr_matrix(adj)
    n = adj.shape[0]
    ptr, col = adj.indptr, adj.indices
    agg = -np.ones(n, dtype=np.int64)
    n_agg = 0
    for i in range(n):
        nb = col[ptr[i]:ptr[i + 1]]
        nb = nb[nb != i]
        if agg[i] < 0 and np.all(agg[nb] < 0):
            agg[i] = n_agg
            agg[nb] = n_agg
            n_agg += 1
    first = agg.copy()
    for i in range(n):
        if agg[i] >= 0:
            continue
        nb = col[ptr[i]:ptr[i + 1]]
        nb = np.sort(nb[(nb != i)])
        done = nb[first[nb] >= 0]
        agg[i] = first[done[0]]
    return agg, n_agg


def aggregate_standard(A_pattern: sp.csr_matrix, passes: int):
    """``passes`` rounds of standard aggregation (section 3.3): the first on
    the graph of ``A``, each further one on the graph of the aggregates
    (``T^T A T`` with T the 0/1 aggregation matrix), composed, as the
    paper's ``T_1 T_2``.  Returns ``(agg, n_agg)``."""
    B = sp.csr_matrix(A_pattern, dtype=np.float64, copy=True)
    B.data[:] = 1.0
    n = B.shape[0]
    agg = np.arange(n, dtype=np.int64)
    n_agg = n
    for _ in range(max(1, passes)):
        a, na = standard_aggregation(B)
        agg = a[agg]
        n_agg = na
        T = sp.csr_matrix((np.ones(len(a)), (np.arange(len(a)), a)),
                          shape=(len(a), na))
        B = (T.T @ B @ T).tocsr()
        B.data[:] = 1.0
    return agg, n_agg


# --------------------------------------------------------------------------
# overlap, partition of unity, multiplicity (sections 2.2, 3.1.1)
# --------------------------------------------------------------------------
def overlap(S: sp.csr_matrix, agg: np.ndarray, n_agg: int):
    """nz_i, omega_i, Gamma_i, Omega_i = [omega_i, Gamma_i] and M(j).

    ``nz_i`` are the rows of G with a nonzero in ``omega_i`` (eq:permuted_G);
    ``Gamma_i`` the other columns those rows touch; ``M(j)`` the number of
    aggregates whose ``nz`` set holds row ``j`` (the Lemma of section 3.1.1).
    """
    n = S.shape[1]
    T = sp.csr_matrix((np.ones(n), (np.arange(n), agg)), shape=(n, n_agg))
    R = (S @ T).tocsc()                      # m x n_agg, entries = counts
    R.data[:] = 1.0
    M = np.asarray(R.sum(axis=1)).ravel().astype(np.int64)
    C = (S.T.tocsr() @ R).tocsc()            # unknown d in Omega_i
    omega, gamma, Omega, nz = [], [], [], []
    order = np.argsort(agg, kind="stable")
    starts = np.searchsorted(agg[order], np.arange(n_agg + 1))
    for i in range(n_agg):
        w = np.sort(order[starts[i]:starts[i + 1]])
        rows = np.sort(R.indices[R.indptr[i]:R.indptr[i + 1]])
        cover = np.sort(C.indices[C.indptr[i]:C.indptr[i + 1]])
        g = np.setdiff1d(cover, w, assume_unique=True)
        omega.append(w)
        gamma.append(g)
        Omega.append(np.concatenate([w, g]))
        nz.append(rows)
    return omega, gamma, Omega, nz, M, R.tocsr(), C.tocsr()


def coloring(C: sp.csr_matrix, S: sp.csr_matrix):
    """Greedy colouring (aggregates in index order, smallest free colour) of
    the graph ``i ~ j iff A(Omega_i, Omega_j) != 0`` (structural); and the
    largest number of overlapping aggregates that share one unknown."""
    Cb = C.copy()
    Cb.data[:] = 1.0
    # A(Omega_i, Omega_j) != 0 iff some row of G touches both Omega_i and
    # Omega_j: the pattern of C^T (S^T S) C, computed as (S C)^T (S C)
    SC = (S @ Cb).tocsr()
    SC.data[:] = 1.0
    adj = (SC.T @ SC).tocsr()
    n_agg = adj.shape[0]
    color = -np.ones(n_agg, dtype=np.int64)
    for i in range(n_agg):
        nb = adj.indices[adj.indptr[i]:adj.indptr[i + 1]]
        used = set(color[nb[nb != i]].tolist())
        c = 0
        while c in used:
            c += 1
        color[i] = c
    n_color = int(color.max()) + 1
    n_mult = int(np.asarray(Cb.sum(axis=1)).max())
    return n_color, n_mult


def threshold(kappa: float, n_color: int, n_mult: int) -> float:
    """Local eigenvalue threshold of section 3.4."""
    return max(0.1, (kappa - n_color) / (n_color * n_mult))


# --------------------------------------------------------------------------
# local splitting and eigenproblem (sections 3.1.1, 3.1.2)
# --------------------------------------------------------------------------
def local_splitting(G: sp.csr_matrix, nz: np.ndarray, Omega: np.ndarray,
                    M: np.ndarray) -> np.ndarray:
    """``A~_i = G_{nz,Omega}^T W(nz,nz) G_{nz,Omega}``, ``W = diag(1/M)``
    (eq:local_splitting)."""
    Gs = G[nz][:, Omega]
    W = sp.diags(1.0 / M[nz])
    return (Gs.T @ (W @ Gs)).toarray()


def schur_pinv(At: np.ndarray, nw: int, pinv_rtol: float) -> np.ndarray:
    """``S~_omega = A~_ww - A~_wG (A~_GG)^+ A~_Gw`` (eq:gevp-S), with the
    Moore-Penrose pseudo-inverse of the SPSD block ``A~_GG`` (eigenvalues at
    or below ``pinv_rtol`` times the largest dropped).  Kept as the plain
    definition for the tests; the setup uses ``schur_ls``."""
    Aww = At[:nw, :nw]
    if At.shape[0] == nw:
        return Aww.copy()
    AwG = At[:nw, nw:]
    AGG = At[nw:, nw:]
    lam, V = np.linalg.eigh(AGG)
    keep = lam > pinv_rtol * max(lam.max(), 0.0)
    Y = V[:, keep].T @ AwG.T
    return Aww - Y.T @ (Y / lam[keep][:, None])


def schur_ls(B: np.ndarray, nw: int, rank_rtol: float) -> np.ndarray:
    """The Schur complement of eq:gevp-S from the weighted rows
    ``B = W^{1/2} G_{nz, Omega}`` (``A~ = B^T B``) without forming A~.

    ``S~_omega = min_{u_Gamma} [u_w; u_G]^T A~ [u_w; u_G] = B_w^T (I - Q Q^T)
    B_w`` with Q an orthonormal basis of range(B_Gamma); on a singular
    ``A~_GammaGamma`` this is the Moore-Penrose (minimum-energy) reading.
    Q and the numerical rank come from the SVD of B_Gamma (singular values
    at or below ``rank_rtol`` times the largest count as zero), so the
    conditioning of B_Gamma enters once, not squared as in
    ``A~_GammaGamma``, and the truncated range does not depend on the basis
    of the columns (an orthogonal change of an aggregate's eigenvector basis
    on the finer level leaves it unchanged).

    The energy ``||B u||`` is unchanged when B is replaced by R from its QR
    factorisation ``B = Q_B R`` (Q_B has orthonormal columns), so the same
    formula is applied to R: at most |Omega_i| rows instead of every row of G
    that touches the aggregate (on coarse levels, where G_l keeps all the
    rows of G, tens of thousands).
    """
    if B.shape[0] > B.shape[1]:
        B = sla.qr(B, mode="r", check_finite=False)[0]
    Bw = B[:, :nw]
    if B.shape[1] == nw:
        return Bw.T @ Bw
    U, sv, _ = np.linalg.svd(B[:, nw:], full_matrices=False)
    r = int(np.sum(sv > rank_rtol * sv[0])) if sv.size and sv[0] > 0 else 0
    Q = U[:, :r]
    E = Bw - Q @ (Q.T @ Bw)
    return E.T @ E


def weighted_rows(G: sp.csr_matrix, nz: np.ndarray, Omega: np.ndarray,
                  M: np.ndarray) -> np.ndarray:
    """``W^{1/2} G_{nz, Omega}`` dense (section 3.1.1, ``W = diag(1/M)``)."""
    return (sp.diags(1.0 / np.sqrt(M[nz])) @ G[nz][:, Omega]).toarray()


def select_count(mu: np.ndarray, nw: int, p: Params, level: int,
                 thresh: float):
    """Number of eigenvectors kept for one aggregate (section 3.4).

    Returns ``(k, hazard)``; ``hazard`` flags an eigenvalue within 1e-8
    (relative) of the threshold, where two FP64 eigensolvers could decide
    differently.
    """
    hazard = False
    if p.n_eig_fixed > 0:
        k = min(p.n_eig_fixed, nw)
    else:
        cut = (1.0 / thresh) * (1.0 - p.thresh_margin)
        count = int(np.sum(mu < cut))
        hazard = bool(np.any(np.abs(mu - 1.0 / thresh) <= 1e-8 / thresh))
        k = min(count, nw // p.cmin_at(level))
    k = max(k, 1)

    def tie(j):        # mu[j] and mu[j-1] in one cluster
        return abs(mu[j] - mu[j - 1]) <= p.tie_rtol * abs(mu[j]) + p.tie_atol

    k0 = k
    while 0 < k < nw and tie(k):
        k -= 1
    if k == 0:
        k = k0
        while k < nw and tie(k):
            k += 1
    return k, hazard


def fix_signs(U: np.ndarray) -> np.ndarray:
    """Make the largest-magnitude entry of every column positive."""
    U = U.copy()
    for t in range(U.shape[1]):
        j = int(np.argmax(np.abs(U[:, t])))
        if U[j, t] < 0:
            U[:, t] = -U[:, t]
    return U


# --------------------------------------------------------------------------
# Algorithm 1
# --------------------------------------------------------------------------
def setup(G: sp.csr_matrix, ndim: int, grid: tuple, params: Params,
          basis_hook: Optional[Callable] = None) -> Hierarchy:
    """Build the hierarchy ``{A_l, G_l, P_l}`` (Algorithm 1).

    ``G`` is the m x n least-squares factor whose columns sit on an
    ``ndim``-dimensional lattice of extent ``grid`` (x fastest).
    ``basis_hook(level, i, Zhat) -> Zhat'`` may replace an aggregate's
    eigenvector block by another basis of its span (tests only).
    """
    p = params
    G = sp.csr_matrix(G, dtype=np.float64)
    G.eliminate_zeros()
    G.sort_indices()
    rows_used = np.diff(G.indptr) > 0
    G = G[rows_used]
    S = G.copy()
    S.data[:] = 1.0
    n = G.shape[1]
    ext = tuple(int(e) for e in grid)
    coord = np.zeros((n, ndim), dtype=np.int64)
    rem = np.arange(n)
    for d in range(ndim):
        coord[:, d] = rem % ext[d]
        rem //= ext[d]
    A = (G.T @ G).tocsr()
    levels = []
    lvl = Level(G=G, S=S, A=A, coord=coord, extent=ext)
    levels.append(lvl)
    l = 0
    while l < p.max_levels - 1 and lvl.n > p.max_coarse:
        _build_level(lvl, l, p, basis_hook)
        nxt = _next_level(lvl, p.compress_rows)
        levels.append(nxt)
        l += 1
        stalled = nxt.n > p.stall_ratio * lvl.n
        lvl = nxt
        if stalled:
            break
    lvl.coarsest = True
    lvl.chol_coarse = sla.cho_factor(lvl.A.toarray(), lower=True)
    return Hierarchy(levels=levels, params=p)


def _build_level(L: Level, l: int, p: Params, basis_hook):
    if p.aggregation == "standard":
        pat = (L.S.T @ L.S).tocsr()
        agg, n_agg = aggregate_standard(pat, p.passes_at(l))
        b, agg_coord, nblk = 0, np.zeros((n_agg, L.coord.shape[1]), dtype=np.int64), ()
    else:
        b, agg, n_agg, agg_coord, nblk = choose_block(L.coord, L.extent, p.block,
                                                      p.omega_max)
    L.block, L.agg, L.n_agg, L.agg_coord, L.agg_extent = (b, agg, n_agg,
                                                           agg_coord, nblk)
    (L.omega, L.gamma, L.Omega, L.nz, L.M, _R, C) = overlap(L.S, agg, n_agg)
    L._R = _R
    L.n_color, L.n_mult = coloring(C, L.S)
    L.thresh = threshold(p.kappa, L.n_color, L.n_mult)
    Ad = L.A
    ks = np.zeros(n_agg, dtype=np.int64)
    for i in range(n_agg):
        w, Om = L.omega[i], L.Omega[i]
        nw = len(w)
        # G_{nz,w}^T G_{nz,w} = A(w, w): rows outside nz vanish on w
        Aww = L.A[w][:, w].toarray()
        St = schur_ls(weighted_rows(L.G, L.nz[i], Om, L.M), nw, p.pinv_rtol)
        mu, U = sla.eigh(St, Aww)                        # U^T Aww U = I
        k, hazard = select_count(mu, nw, p, l, L.thresh)
        if hazard:
            L.hazards.append(i)
        Z = fix_signs(U[:, :k])
        if basis_hook is not None:
            Z = basis_hook(l, i, Z)
        L.mu.append(mu)
        L.Zhat.append(Z)
        ks[i] = k
        # smoother block A_i = A(Omega_i, Omega_i), factored once (sec. 3.1.1)
        Ai = Ad[Om][:, Om].toarray()
        L.chol.append(sla.cho_factor(Ai, lower=True))
    L.k = ks
    # eq:mg-p: coarse unknowns ordered by aggregate, then eigen index
    off = np.concatenate([[0], np.cumsum(ks)])
    rr, cc, vv = [], [], []
    for i in range(n_agg):
        Z = L.Zhat[i]
        w = L.omega[i]
        rr.append(np.repeat(w, Z.shape[1]))
        cc.append(np.tile(off[i] + np.arange(Z.shape[1]), len(w)))
        vv.append(Z.ravel())
    L.P = sp.csr_matrix((np.concatenate(vv), (np.concatenate(rr),
                                              np.concatenate(cc))),
                        shape=(L.n, int(off[-1])))


def _next_level(L: Level, compress_rows: bool = False) -> Level:
    """``G_{l+1} = G_l P_l``, ``A_{l+1} = P_l^T A_l P_l`` (section 3.1.3);
    coarse unknowns inherit their aggregate's lattice coordinate.

    With ``compress_rows`` the rows of ``G_{l+1}`` that touch the same set of
    parent aggregates (hence share one symbolic support, one multiplicity M
    and one set of overlapping aggregates on the next level) are replaced by
    the R factor of their QR factorisation: every sum of ``w g^T g`` over
    them, so ``A_{l+1}``, each local ``A~_i`` and every Omega_i, is unchanged
    in exact arithmetic, with at most |support| rows per group instead of the
    fine rows (a CPU-time saving only)."""
    nc = L.P.shape[1]
    parent = np.repeat(np.arange(L.n_agg), L.k)
    E = sp.csr_matrix((np.ones(nc), (parent, np.arange(nc))),
                      shape=(L.n_agg, nc))
    S = (L._R @ E).tocsr()
    S.data[:] = 1.0
    G = (L.G @ L.P).tocsr()
    A = (L.P.T @ L.A @ L.P).tocsr()
    if compress_rows:
        Rt = L._R.tocsr()
        groups = {}
        for j in range(Rt.shape[0]):
            key = tuple(np.sort(Rt.indices[Rt.indptr[j]:Rt.indptr[j + 1]]))
            groups.setdefault(key, []).append(j)
        rr, cc, vv, sr, sc = [], [], [], [], []
        row = 0
        for key in sorted(groups):
            idx = np.asarray(groups[key])
            supp = S.indices[S.indptr[idx[0]]:S.indptr[idx[0] + 1]]
            supp = np.sort(supp)
            blk = G[idx][:, supp].toarray()
            Rg = sla.qr(blk, mode="r", check_finite=False)[0]
            k = min(len(idx), len(supp))
            Rg = Rg[:k]
            ii, jj = np.nonzero(Rg)
            rr.append(row + ii)
            cc.append(supp[jj])
            vv.append(Rg[ii, jj])
            sr.append(np.repeat(row + np.arange(k), len(supp)))
            sc.append(np.tile(supp, k))
            row += k
        G = sp.csr_matrix((np.concatenate(vv), (np.concatenate(rr), np.concatenate(cc))),
                          shape=(row, nc))
        S = sp.csr_matrix((np.ones(sum(len(x) for x in sr)),
                           (np.concatenate(sr), np.concatenate(sc))), shape=(row, nc))
    return Level(G=G, S=S, A=A, coord=L.agg_coord[parent],
                 extent=L.agg_extent)


# --------------------------------------------------------------------------
# smoothers, V-cycle and PCG
# --------------------------------------------------------------------------
def apply_A(L: Level, x: np.ndarray) -> np.ndarray:
    return L.A @ x


def ras(L: Level, r: np.ndarray) -> np.ndarray:
    """``sum_i R_i^T D_i A_i^{-1} R_i r`` (eq:ras)."""
    out = np.zeros_like(r)
    for i in range(L.n_agg):
        Om = L.Omega[i]
        y = sla.cho_solve(L.chol[i], r[Om])
        y[len(L.omega[i]):] = 0.0                       # D_i after the solve
        out[Om] += y
    return out


def ras_t(L: Level, r: np.ndarray) -> np.ndarray:
    """``sum_i R_i^T A_i^{-1} D_i R_i r`` (eq:ras-t)."""
    out = np.zeros_like(r)
    for i in range(L.n_agg):
        Om = L.Omega[i]
        v = r[Om].copy()
        v[len(L.omega[i]):] = 0.0                       # D_i before the solve
        out[Om] += sla.cho_solve(L.chol[i], v)
    return out


def vcycle(H: Hierarchy, b: np.ndarray, level: int = 0) -> np.ndarray:
    """One V-cycle from x0 = 0: RAS pre-smoothing, coarse-grid correction
    (eq:cgc) with the next level's V-cycle, RAS-T post-smoothing."""
    L = H.levels[level]
    if L.coarsest:
        return sla.cho_solve(L.chol_coarse, b)
    x = ras(L, b)
    r = b - apply_A(L, x)
    e = vcycle(H, L.P.T @ r, level + 1)
    x = x + L.P @ e
    r = b - apply_A(L, x)
    return x + ras_t(L, r)


def block_pcg(H: Hierarchy, B: np.ndarray, tol: float = 1e-8, maxit: int = 500,
              fixed_iters: Optional[int] = None, precond: Optional[Callable] = None,
              pinv_rtol: float = 1e-12):
    """Block preconditioned CG (O'Leary 1980) on the columns of B (n x s),
    X0 = 0, in the form whose block of search directions is made
    A-orthogonal to the previous block explicitly:

        Q = A P,  G = P^T Q,  C = G^+ (P^T R),  X += P C,  R -= Q C,
        Z = M R,  D = -G^+ (Q^T Z),  P = Z + P D,

    starting from P = Z = M B.  G^+ is the pseudo-inverse of the symmetric
    s x s matrix G (eigenvalues at or below pinv_rtol times the largest count
    as zero), so directions that have become linearly dependent (columns
    that converged, or equal right-hand sides) drop out instead of breaking
    the iteration.  Every column's iterate minimises the A-norm of its error
    over the sum of all columns' Krylov spaces.  Stops when every nonzero
    column has ||r_j|| <= tol ||b_j|| and then its true residual too
    (otherwise R is replaced by B - A X and P by M R, as in ``pcg``); with
    ``fixed_iters`` runs exactly that many iterations.  Returns ``(X, info)``
    with the iteration count, restarts and per-column relative residuals."""
    apply_b = precond if precond is not None else (lambda v: vcycle(H, v))
    M = lambda V: np.stack([apply_b(V[:, j]) for j in range(V.shape[1])], axis=1)
    A0 = H.levels[0]
    X = np.zeros_like(B)
    R = B.copy()
    nb = np.linalg.norm(B, axis=0)
    live = nb > 0
    Z = M(R)
    Pd = Z.copy()
    its = restarts = 0
    limit = fixed_iters if fixed_iters is not None else maxit
    conv = not live.any()
    while its < limit and not conv:
        Q = apply_A(A0, Pd)
        G = Pd.T @ Q
        w, V = np.linalg.eigh(0.5 * (G + G.T))
        keep = w > pinv_rtol * max(w.max(), 0.0)
        Gp = (V[:, keep] / w[keep]) @ V[:, keep].T
        C = Gp @ (Pd.T @ R)
        X = X + Pd @ C
        R = R - Q @ C
        its += 1
        if fixed_iters is None:
            rn = np.linalg.norm(R, axis=0)
            if np.all(rn[live] <= tol * nb[live]):
                Rt = B - apply_A(A0, X)
                if np.all(np.linalg.norm(Rt, axis=0)[live] <= tol * nb[live]):
                    conv = True
                    break
                R = Rt
                restarts += 1
                Z = M(R)
                Pd = Z.copy()
                continue
        Z = M(R)
        Pd = Z - Pd @ (Gp @ (Q.T @ Z))
    nbs = np.where(live, nb, 1.0)
    true_res = np.linalg.norm(B - apply_A(A0, X), axis=0) / nbs
    return X, dict(iters=its, converged=bool(conv), restarts=restarts,
                   rel_res=np.linalg.norm(R, axis=0) / nbs, true_rel_res=true_res)


def additive_schwarz(L: Level, r: np.ndarray) -> np.ndarray:
    """``sum_i R_i^T A_i^{-1} R_i r``: eq:ras without the partition of unity,
    the smoother M_1^{-1} of the additive two-level method (sec. 3.1.1)."""
    out = np.zeros_like(r)
    for i in range(L.n_agg):
        Om = L.Omega[i]
        out[Om] += sla.cho_solve(L.chol[i], r[Om])
    return out


def acycle(H: Hierarchy, b: np.ndarray, level: int = 0) -> np.ndarray:
    """The additive method of sec. 3.1.1, ``(P (P^T A P)^{-1} P^T + M_1^{-1})
    b`` with M_1^{-1} the additive Schwarz smoother, made multilevel by
    applying the same form to the coarse operator P^T A P = G_{l+1}^T
    G_{l+1} instead of inverting it (exact at the coarsest level).  Every
    term is symmetric positive semi-definite, so the cycle is a symmetric
    preconditioner for CG."""
    L = H.levels[level]
    if L.coarsest:
        return sla.cho_solve(L.chol_coarse, b)
    return additive_schwarz(L, b) + L.P @ acycle(H, L.P.T @ b, level + 1)


def pcg(H: Hierarchy, b: np.ndarray, tol: float = 1e-8, maxit: int = 500,
        fixed_iters: Optional[int] = None,
        precond: Optional[Callable] = None, flexible: bool = False):
    """Preconditioned CG, x0 = 0, preconditioner = one V-cycle.

    Stops when ``||r_k||_2 <= tol ||b||_2`` for the recurrence residual and
    the true residual ``b - A x_k`` recomputed at that point; when only the
    recurrence residual passes, the true residual replaces it and CG restarts
    from ``x_k`` (direction ``p = z``), so a reported convergence always holds
    for ``b - A x``.  With ``fixed_iters`` it runs exactly that many
    iterations.  ``precond(r)`` replaces the V-cycle by another form of the
    same operator (``AssembledVcycle``).  With ``flexible`` the direction is
    made A-orthogonal to the previous one explicitly, ``beta = -(z_{k+1}^T
    q_k) / (p_k^T q_k)`` with ``q_k = A p_k`` (flexible CG with one stored
    direction, Notay 2000), which stays a CG method when the preconditioner
    varies or is slightly unsymmetric (a V-cycle in lower precision); with
    a fixed symmetric preconditioner it equals the standard ``beta`` in exact
    arithmetic.  Returns ``(x, info)`` with iteration count and residual
    history (``restarts`` counts the replacements).
    """
    apply_b = precond if precond is not None else (lambda v: vcycle(H, v))
    A0 = H.levels[0]
    x = np.zeros_like(b)
    r = b.copy()
    nb = np.linalg.norm(b)
    hist = [np.linalg.norm(r)]
    z = apply_b(r)
    pdir = z.copy()
    rho = r @ z
    its = 0
    restarts = 0
    limit = fixed_iters if fixed_iters is not None else maxit
    conv = nb == 0.0
    while its < limit and not conv:
        q = apply_A(A0, pdir)
        alpha = rho / (pdir @ q)
        x += alpha * pdir
        r -= alpha * q
        its += 1
        hist.append(np.linalg.norm(r))
        restart = False
        if fixed_iters is None and hist[-1] <= tol * nb:
            rt = b - apply_A(A0, x)
            if np.linalg.norm(rt) <= tol * nb:
                conv = True
                break
            r = rt
            hist[-1] = np.linalg.norm(r)
            restart = True
            restarts += 1
        z = apply_b(r)
        rho_new = r @ z
        if restart:
            pdir = z.copy()
        elif flexible:
            pdir = z - ((z @ q) / (pdir @ q)) * pdir
        else:
            pdir = z + (rho_new / rho) * pdir
        rho = rho_new
    true_res = np.linalg.norm(b - apply_A(A0, x)) / nb if nb > 0 else 0.0
    rhoavg = (hist[-1] / hist[0]) ** (1.0 / max(its, 1)) if nb > 0 else 0.0
    return x, dict(iters=its, hist=np.array(hist), true_rel_res=true_res,
                   converged=bool(conv), rho=rhoavg, restarts=restarts)


class AssembledVcycle:
    """The same V-cycle with each level's operators assembled once as sparse
    matrices, the plain form in which a CPU library would run the solve
    phase: the RAS smoother ``S_l = sum_i R_i^T D_i A_i^{-1} R_i`` (eq:ras) as
    one CSR matrix (its rows are the disjoint omega_i blocks of the local
    inverses, ``sum_i |omega_i||Omega_i|`` entries), RAS-T (eq:ras-t) as its
    transpose (``A_i^{-1}`` is symmetric and ``D_i`` diagonal), ``A_l`` and
    ``P_l`` as CSR, and the coarsest level's Cholesky factor.  Applying it is
    the V-cycle of ``vcycle`` with the local solves done through these
    matrices instead of per-aggregate Cholesky solves."""

    def __init__(self, H: Hierarchy):
        self.H = H
        self.S = []
        self.ST = []
        for L in H.levels:
            if L.coarsest:
                break
            rr, cc, vv = [], [], []
            for i in range(L.n_agg):
                w, Om = L.omega[i], L.Omega[i]
                Ainv = sla.cho_solve(L.chol[i], np.eye(len(Om)))
                rr.append(np.repeat(w, len(Om)))
                cc.append(np.tile(Om, len(w)))
                vv.append(Ainv[:len(w), :].ravel())
            S = sp.csr_matrix((np.concatenate(vv), (np.concatenate(rr), np.concatenate(cc))),
                              shape=(L.n, L.n))
            self.S.append(S)
            self.ST.append(S.T.tocsr())

    def apply(self, b: np.ndarray, level: int = 0) -> np.ndarray:
        L = self.H.levels[level]
        if L.coarsest:
            return sla.cho_solve(L.chol_coarse, b)
        x = self.S[level] @ b
        r = b - L.A @ x
        x = x + L.P @ self.apply(L.P.T @ r, level + 1)
        r = b - L.A @ x
        return x + self.ST[level] @ r

    __call__ = apply


def dense_preconditioner(H: Hierarchy) -> np.ndarray:
    """The V-cycle as a dense matrix (columns = V-cycle of unit vectors)."""
    n = H.levels[0].n
    B = np.zeros((n, n))
    for j in range(n):
        e = np.zeros(n)
        e[j] = 1.0
        B[:, j] = vcycle(H, e)
    return B


def stats(H: Hierarchy) -> dict:
    """Operator complexity sum nnz(A_l)/nnz(A_0), smoother complexity
    sum |omega_i||Omega_i| / nnz(A_0), and per-level sizes.  nnz counts the
    structural entries of ``A_l = G_l^T G_l`` (the pattern of ``S_l^T S_l``
    for the symbolic structure ``S_l`` of ``G_l``), not the entries that
    happen to cancel to zero."""
    nnzs = [int((L.S.T @ L.S).nnz) for L in H.levels]
    nnz0 = nnzs[0]
    oc = sum(nnzs) / nnz0
    sc = sum(sum(len(w) * len(O) for w, O in zip(L.omega, L.Omega))
             for L in H.levels if not L.coarsest) / nnz0
    return dict(levels=len(H.levels), n=[L.n for L in H.levels],
                nnz_A=nnzs,
                n_agg=[L.n_agg for L in H.levels if not L.coarsest],
                block=[L.block for L in H.levels if not L.coarsest],
                n_color=[L.n_color for L in H.levels if not L.coarsest],
                n_mult=[L.n_mult for L in H.levels if not L.coarsest],
                thresh=[L.thresh for L in H.levels if not L.coarsest],
                op_complexity=oc, smoother_complexity=sc)
