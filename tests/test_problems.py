"""Generators: sizes and structure of the synthetic least-squares factors."""
import math

import numpy as np
import pytest

import problems as P


def count_rows_2d(N, both_components_dense):
    """Closed-form row count: 2 rows per cell minus rows left empty."""
    if both_components_dense:          # rows touch (i,j),(i+1,j),(i,j+1)
        return 2 * N * N - 2           # only cell (0,0) touches no interior node
    return 2 * N * N - 2 * N           # x-rows of cells j=0, y-rows of cells i=0


def test_config1_sizes():
    p = P.config1()
    assert p.n == 31 ** 2 == 961
    assert p.m == count_rows_2d(32, False) == 1984
    assert p.G.nnz == 3844
    A = (p.G.T @ p.G).tocsr()
    assert A.nnz == 5 * 961 - 4 * 31          # 5-point stencil with boundary


def test_config2_sizes():
    p = P.aniso2d(64, math.pi / 6, 1e-4)
    assert p.n == 63 ** 2
    assert p.m == count_rows_2d(64, True)
    # every row has at most 3 entries: nodes (i,j), (i+1,j), (i,j+1)
    assert np.diff(p.G.indptr).max() == 3


def test_five_point_stencil_golden():
    """theta=0, eps=1 gives the 5-point Laplacian (section 4.1)."""
    import os
    here = os.path.dirname(__file__)
    rows = [l.split() for l in open(os.path.join(here, "golden", "five_point_stencil.txt"))
            if l.strip() and not l.startswith("#")]
    st = np.array(rows, dtype=float)
    N = 8
    p = P.aniso2d(N, 0.0, 1.0)
    A = (p.G.T @ p.G).toarray() * p.h ** 2
    ni = N - 1
    i, j = 3, 4                      # interior node (1-based coordinates)
    c = (i - 1) + ni * (j - 1)
    got = np.zeros((3, 3))
    for dy in (1, 0, -1):
        for dx in (-1, 0, 1):
            got[1 - dy, dx + 1] = A[c, (i - 1 + dx) + ni * (j - 1 + dy)]
    assert np.array_equal(got, st)


def test_rotated_tensor():
    """G^T G equals the discretisation of -div(K grad u) with K = R diag(1,eps) R^T:
    the cell-wise quadratic form of K^{1/2} equals the one of K."""
    th, eps = 0.7, 1e-3
    Kh = P.grids.sqrt_tensor_2d(th, eps)
    c, s = math.cos(th), math.sin(th)
    R = np.array([[c, -s], [s, c]])
    K = R @ np.diag([1, eps]) @ R.T
    assert np.allclose(Kh @ Kh, K, atol=1e-15)
    assert np.allclose(Kh, Kh.T)


def test_ls3d_structure():
    p = P.ls3d(6)
    n = 5 ** 3
    assert p.n == n
    # first n rows are sqrt(D1) = 1e-3 I
    top = p.G[:n].toarray()
    assert np.allclose(top, 1e-3 * np.eye(n))
    Q = p.meta["Q"]
    assert np.allclose(Q.T @ Q, np.eye(3), atol=1e-14)
    assert np.linalg.det(Q) > 0
    # 3 rows per cell; a cell whose 4 nodes are all on the boundary (two or
    # more of its coordinates zero: 3N - 2 cells) has none
    N = 6
    assert (p.m - n) == 3 * (N ** 3 - (3 * N - 2))
    A = (p.G.T @ p.G).toarray()
    assert np.all(np.linalg.eigvalsh(A) > 0)


def test_rhs_seeded():
    a = P.rhs_uniform(100, 1)
    b = P.rhs_uniform(100, 1)
    assert np.array_equal(a, b)
    assert a.min() >= -1 and a.max() < 1
