"""Finite-difference least-squares factors ``G`` and seeded right-hand sides.

Two problem families, both on the unit square / cube with ``N`` cells per
side, spacing ``h = 1/N`` and zero Dirichlet data (boundary nodes are
eliminated, so the unknowns are the interior nodes):

* ``aniso2d`` -- rotated anisotropic diffusion ``-div(K grad u) = f``
  (section 4.1).  Each cell contributes the two rows ``K^{1/2} grad+ u``
  where ``grad+`` is the forward-difference gradient of the cell's lower-left
  node, so that ``G^T G = -div- (K grad+)``.  ``K = R(theta) diag(1, eps)
  R(theta)^T`` and ``K^{1/2}`` is its symmetric square root.
* ``ls3d`` -- the ``A = D1 + B^T D2^{-1} B`` form of the introduction,
  written as ``G = [sqrt(D1); sqrt(D2^{-1}) B]`` with ``B`` the 3D
  forward-difference gradient and ``D2^{-1}`` a per-cell SPD tensor
  ``a_c K`` (``K`` a rotated diagonal tensor, ``a_c`` lognormal).

Unknowns are numbered x-fastest over the interior lattice:
``idx = (i-1) + (N-1)(j-1) [+ (N-1)^2 (k-1)]``.  Rows are numbered
cell-major (cells x-fastest), components consecutive.  Exact-zero entries
and rows with no entry left after eliminating boundary nodes are dropped.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np
import scipy.sparse as sp


@dataclass
class Problem:
    """A least-squares system: sparse ``G`` (m x n) plus its lattice layout."""
    name: str
    G: sp.csr_matrix
    ndim: int
    grid: tuple          # interior lattice extent per axis (x fastest)
    h: float
    meta: dict = field(default_factory=dict)

    @property
    def n(self) -> int:
        return self.G.shape[1]

    @property
    def m(self) -> int:
        return self.G.shape[0]


def _assemble(rows, cols, vals, m_full, n):
    """COO -> CSR, dropping entries on eliminated nodes, exact zeros and
    empty rows (in that order); column indices sorted within each row."""
    keep = (cols >= 0) & (vals != 0.0)
    rows, cols, vals = rows[keep], cols[keep], vals[keep]
    used = np.zeros(m_full, dtype=bool)
    used[rows] = True
    newid = np.cumsum(used) - 1
    m = int(used.sum())
    G = sp.csr_matrix((vals, (newid[rows], cols)), shape=(m, n))
    G.sum_duplicates()
    G.sort_indices()
    return G


def _node2d(i, j, N):
    inside = (i >= 1) & (i <= N - 1) & (j >= 1) & (j <= N - 1)
    return np.where(inside, (i - 1) + (N - 1) * (j - 1), -1)


def _node3d(i, j, k, N):
    inside = ((i >= 1) & (i <= N - 1) & (j >= 1) & (j <= N - 1)
              & (k >= 1) & (k <= N - 1))
    return np.where(inside, (i - 1) + (N - 1) * ((j - 1) + (N - 1) * (k - 1)),
                    -1)


def sqrt_tensor_2d(theta: float, eps: float) -> np.ndarray:
    """Symmetric square root of ``K = R(theta) diag(1, eps) R(theta)^T``."""
    c, s = math.cos(theta), math.sin(theta)
    R = np.array([[c, -s], [s, c]])
    return R @ np.diag([1.0, math.sqrt(eps)]) @ R.T


def aniso2d(N: int, theta: float, eps: float) -> Problem:
    """2D rotated anisotropic diffusion in least-squares form, N cells/side."""
    h = 1.0 / N
    Kh = sqrt_tensor_2d(theta, eps)
    ci, cj = np.meshgrid(np.arange(N), np.arange(N), indexing="xy")
    ci, cj = ci.ravel(), cj.ravel()          # cell index = ci + N*cj
    a = _node2d(ci, cj, N)
    b = _node2d(ci + 1, cj, N)
    c = _node2d(ci, cj + 1, N)
    ncell = N * N
    rows, cols, vals = [], [], []
    for q in range(2):
        r = 2 * np.arange(ncell) + q
        coef = (-(Kh[q, 0] + Kh[q, 1]) / h, Kh[q, 0] / h, Kh[q, 1] / h)
        for node, cf in zip((a, b, c), coef):
            rows.append(r)
            cols.append(node)
            vals.append(np.full(ncell, cf))
    n = (N - 1) ** 2
    G = _assemble(np.concatenate(rows), np.concatenate(cols),
                  np.concatenate(vals), 2 * ncell, n)
    return Problem(name=f"aniso2d_N{N}_theta{theta:.6g}_eps{eps:.3g}", G=G,
                   ndim=2, grid=(N - 1, N - 1), h=h,
                   meta=dict(N=N, theta=theta, eps=eps))


def rotation_from_seed(seed: int, rng: np.random.Generator | None = None):
    """Random 3x3 rotation: Q of the QR of a standard-normal matrix with
    ``diag(R) > 0`` and ``det(Q) = +1``."""
    rng = np.random.default_rng(seed) if rng is None else rng
    X = rng.standard_normal((3, 3))
    Q, R = np.linalg.qr(X)
    Q = Q * np.sign(np.diag(R))[None, :]
    if np.linalg.det(Q) < 0:
        Q[:, -1] *= -1.0
    return Q


def ls3d(N: int, eps_perp: float = 1e-3, d1: float = 1e-6,
         seed: int = 2, sigma: float = 1.0) -> Problem:
    """3D ``D1 + B^T D2^{-1} B`` with ``D2^{-1} = a_c Q diag(1,e,e) Q^T``.

    ``G = [sqrt(d1) I ; sqrt(a_c) K^{1/2} grad+]``: the ``n`` rows of
    ``sqrt(D1)`` come first, then three rows per cell.  The rotation ``Q``
    and the per-cell lognormal(0, sigma) coefficients (sigma = 1 in the
    workload) are drawn, in that order, from
    ``numpy.random.default_rng(seed)``; cells are x-fastest.
    """
    h = 1.0 / N
    rng = np.random.default_rng(seed)
    Q = rotation_from_seed(seed, rng)
    Kh = Q @ np.diag([1.0, math.sqrt(eps_perp), math.sqrt(eps_perp)]) @ Q.T
    ncell = N ** 3
    acoef = rng.lognormal(0.0, sigma, ncell)
    sa = np.sqrt(acoef)
    ci, cj, ck = np.meshgrid(np.arange(N), np.arange(N), np.arange(N),
                             indexing="ij")
    # x fastest: flatten with k slowest
    ci = ci.transpose(2, 1, 0).ravel()
    cj = cj.transpose(2, 1, 0).ravel()
    ck = ck.transpose(2, 1, 0).ravel()
    nodes = (_node3d(ci, cj, ck, N), _node3d(ci + 1, cj, ck, N),
             _node3d(ci, cj + 1, ck, N), _node3d(ci, cj, ck + 1, N))
    n = (N - 1) ** 3
    rows = [np.arange(n)]
    cols = [np.arange(n)]
    vals = [np.full(n, math.sqrt(d1))]
    for q in range(3):
        r = n + 3 * np.arange(ncell) + q
        coef = (-(Kh[q, 0] + Kh[q, 1] + Kh[q, 2]) / h, Kh[q, 0] / h,
                Kh[q, 1] / h, Kh[q, 2] / h)
        for node, cf in zip(nodes, coef):
            rows.append(r)
            cols.append(node)
            vals.append(cf * sa)
    G = _assemble(np.concatenate(rows), np.concatenate(cols),
                  np.concatenate(vals), n + 3 * ncell, n)
    return Problem(name=f"ls3d_N{N}", G=G, ndim=3, grid=(N - 1,) * 3, h=h,
                   meta=dict(N=N, eps_perp=eps_perp, d1=d1, seed=seed, Q=Q))


def rhs_uniform(n: int, seed: int) -> np.ndarray:
    """Right-hand side with entries uniform on [-1, 1) from ``seed``."""
    return np.random.default_rng(seed).uniform(-1.0, 1.0, n)


# The right-hand-side seeds of the named workloads.
CONFIG_RHS_SEED = {1: 0, 2: 1, 3: 3}


def config1() -> Problem:
    """Tiny isotropic 2D problem: N=32, theta=0, eps=1 (961 unknowns)."""
    return aniso2d(32, 0.0, 1.0)


def config2(N: int = 512) -> Problem:
    """Large rotated-anisotropic 2D problem: theta=pi/6, eps=1e-4."""
    return aniso2d(N, math.pi / 6, 1e-4)


def config3(N: int = 128) -> Problem:
    """3D ``D1 + B^T D2^{-1} B`` problem on a 128^3 grid."""
    return ls3d(N)
