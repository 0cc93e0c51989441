"""Pins of the oracle's aggregation on matrix entries (section 3.3 and the
aggregation step of Algorithm 1): hand-derived aggregates of small graphs,
the partition invariants every aggregation must satisfy, and multi-pass
composition (the paper's T_1 T_2)."""
import math

import numpy as np
import scipy.sparse as sp

import oracle as O
import problems as P

SA = O.lsamg.standard_aggregation
AS = O.lsamg.aggregate_standard


def path(n):
    e = np.ones(n - 1)
    return sp.diags([e, e], [-1, 1], shape=(n, n), format="csr")


def grid5(nx, ny):
    """5-point pattern, node x + nx*y."""
    I = sp.identity
    Tx, Ty = path(nx), path(ny)
    return (sp.kron(I(ny), Tx) + sp.kron(Ty, I(nx))).tocsr()


def groups(agg):
    out = {}
    for i, a in enumerate(agg):
        out.setdefault(int(a), []).append(i)
    return [out[k] for k in sorted(out)]


def test_path_graphs():
    """Path 0-1-...-(n-1): node 0 takes {0,1}; node 2 sees the aggregated 1
    and waits; node 3 takes {2,3,4}; and so on every three nodes.  n = 6:
    node 5 (neighbour 4 aggregated) joins {2,3,4} in pass 2.  n = 7: node 6
    sees only the free node 5, so pass 1 creates {5,6}.

    Caught: pass 2 joining the highest-numbered aggregated neighbour, or
    pass 1 checking only the node itself (not its neighbours)."""
    assert groups(SA(path(8))[0]) == [[0, 1], [2, 3, 4], [5, 6, 7]]
    assert groups(SA(path(6))[0]) == [[0, 1], [2, 3, 4, 5]]
    assert groups(SA(path(7))[0]) == [[0, 1], [2, 3, 4], [5, 6]]


def test_grid_3x3():
    """5-point 3 x 3 grid (row-major).  Pass 1: node 0 takes {0,1,3}; nodes
    2 and 4 touch node 1, which is taken; node 5 takes {2,4,5,8}; nodes 6, 7
    touch taken nodes.  Pass 2: node 6's lowest aggregated neighbour is 3
    (aggregate 0), node 7's is 4 (aggregate 1)."""
    agg, na = SA(grid5(3, 3))
    assert na == 2
    assert groups(agg) == [[0, 1, 3, 6], [2, 4, 5, 7, 8]]


def test_special_graphs():
    """Complete graph: one aggregate.  Star with the centre last: the first
    leaf takes {leaf, centre}, every other leaf joins it in pass 2.  An
    isolated node forms its own aggregate (the paper's extra step for
    unaggregated nodes is then never needed)."""
    n = 6
    K = sp.csr_matrix(np.ones((n, n)) - np.eye(n))
    assert groups(SA(K)[0]) == [list(range(n))]
    S = sp.lil_matrix((n, n))
    for i in range(n - 1):
        S[i, n - 1] = S[n - 1, i] = 1
    assert groups(SA(S.tocsr())[0]) == [list(range(n))]
    Z = sp.csr_matrix((3, 3))
    assert groups(SA(Z)[0]) == [[0], [1], [2]]


def test_pass2_places_every_leftover_node():
    """Two triangles {0,1,2} and {3,4,5} joined by the edge 2-3: pass 1
    takes {0,1,2} at node 0; node 3 touches the taken node 2 and waits; node
    4's neighbours 3, 5 are free, so pass 1 takes {3,4,5}.  Adding the edge
    1-4 makes node 4 wait too; node 5's neighbours 3, 4 are free: {3,4,5}
    again.  With the edge 1-5 as well, nodes 3, 4, 5 all wait and pass 2
    sends each to the aggregate of its lowest aggregated neighbour: 0."""
    edges = [(0, 1), (0, 2), (1, 2), (2, 3), (3, 4), (3, 5), (4, 5)]
    A = sp.lil_matrix((6, 6))
    for a, b in edges:
        A[a, b] = A[b, a] = 1
    assert groups(SA(A.tocsr())[0]) == [[0, 1, 2], [3, 4, 5]]
    A[1, 4] = A[4, 1] = 1
    assert groups(SA(A.tocsr())[0]) == [[0, 1, 2], [3, 4, 5]]
    A[1, 5] = A[5, 1] = 1
    assert groups(SA(A.tocsr())[0]) == [[0, 1, 2, 3, 4, 5]]


def test_two_passes_compose():
    """Two passes on the 8-node path: the first gives {0,1},{2,3,4},{5,6,7},
    whose graph is a 3-node path; the second aggregates that path into one
    aggregate, so T_1 T_2 maps every node to aggregate 0."""
    agg, na = AS(path(8), 2)
    assert na == 1 and np.all(agg == 0)
    agg1, na1 = AS(path(8), 1)
    assert na1 == 3


def test_partition_invariants_on_workload():
    """On a rotated-anisotropy grid (7-point pattern): every unknown lies in
    exactly one aggregate, every pass-1 aggregate contains its root's whole
    neighbourhood, every aggregate is connected in the matrix graph, and a
    second pass only merges whole first-pass aggregates."""
    p = P.aniso2d(20, math.pi / 6, 1e-3)
    S = p.G.copy()
    S.data[:] = 1
    pat = (S.T @ S).tocsr()
    agg, na = AS(pat, 1)
    assert agg.min() == 0 and agg.max() == na - 1 and len(agg) == p.n
    adj = pat.tolil()
    for a in range(na):
        mem = set(np.nonzero(agg == a)[0].tolist())
        seen = {min(mem)}
        todo = [min(mem)]
        while todo:
            u = todo.pop()
            for v in adj.rows[u]:
                if v in mem and v not in seen:
                    seen.add(v)
                    todo.append(v)
        assert seen == mem, a
    agg2, na2 = AS(pat, 2)
    for a in range(na):
        assert len(set(agg2[agg == a].tolist())) == 1
    assert na2 < na


def test_setup_with_standard_aggregation():
    """Algorithm 1 with aggregation on matrix entries: the hierarchy keeps
    the Lemma (local splittings sum to A) on every level, P has disjoint
    column supports, and PCG reaches the tolerance on the true residual."""
    p = P.aniso2d(24, math.pi / 6, 1e-4)
    H = O.setup(p.G, 2, p.grid, O.Params(cmin=(3, 4), max_coarse=80,
                                          aggregation="standard", agg_passes=(2, 1)))
    assert len(H.levels) >= 3
    for L in H.levels[:-1]:
        Ssum = np.zeros((L.n, L.n))
        for i in range(L.n_agg):
            At = O.lsamg.local_splitting(L.G, L.nz[i], L.Omega[i], L.M)
            Ssum[np.ix_(L.Omega[i], L.Omega[i])] += At
        Ad = (L.G.T @ L.G).toarray()
        assert np.abs(Ssum - Ad).max() <= 1e-12 * np.abs(Ad).max()
        cnt = np.zeros(L.n, dtype=int)
        for w in L.omega:
            cnt[w] += 1
        assert np.all(cnt == 1)
    b = P.rhs_uniform(p.n, 2)
    x, info = O.pcg(H, b, tol=1e-8)
    assert info["converged"] and info["true_rel_res"] <= 1e-8
