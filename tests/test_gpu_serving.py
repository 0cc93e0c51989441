"""Continuous-batching server (lsamg_server_*) on the GPU, through the C-ABI.

A result must be the same alone and in a mix of concurrent requests, within
the solve tolerance: both solutions reach ||b - A x|| <= tol ||b|| (checked
here in FP64 with A = G^T G) and differ by at most what two such solutions
can differ by.  Admission against the device budget, eviction, a failing
setup, an oversize hierarchy and setups on the device are covered as well.
"""
import math

import numpy as np
import pytest

import problems as P
from paper_2601_04112_amd import lsamg as L

pytestmark = pytest.mark.gpu

OPS = [(48, 0.3, 1e-2), (40, 1.1, 1e-4), (56, math.pi / 6, 1e-3), (32, 0.0, 1.0)]


def op(k):
    N, th, eps = OPS[k]
    return P.aniso2d(N, th, eps)


def drain(srv, count, timeout_ms=120000):
    out = {}
    waited = 0
    while len(out) < count and waited < timeout_ms:
        for d in srv.poll(wait_ms=200):
            out[d["id"]] = d
        waited += 200
    assert len(out) == count, f"only {len(out)} of {count} requests completed"
    return out


def check(prob, b, x, tol):
    A_b = np.atleast_2d(b)
    X = np.atleast_2d(x)
    for j in range(A_b.shape[0]):
        r = A_b[j] - prob.G.T @ (prob.G @ X[j])
        assert np.linalg.norm(r) <= tol * np.linalg.norm(A_b[j])


def test_alone_equals_in_mix(gpu_device):
    probs = [op(k) for k in range(len(OPS))]
    rng = np.random.default_rng(5)
    b0 = np.stack([P.rhs_uniform(probs[0].n, 900 + j) for j in range(3)])
    # alone
    srv = L.Server(hbm_budget=8 << 30, max_slots=4)
    rid = srv.submit(0, probs[0].G, 2, probs[0].grid, b0, tol=1e-8, cmin=(2,), max_coarse=200)
    alone = drain(srv, 1)[rid]
    srv.close()
    assert alone["status"] == 0 and alone["cache_hit"] == 0
    check(probs[0], b0, alone["x"], 1e-8)
    # in a mix: 24 requests over 4 operators, submitted at once
    srv = L.Server(hbm_budget=8 << 30, max_slots=4)
    ids = {}
    for i in range(24):
        k = int(rng.integers(len(OPS)))
        nr = int(rng.integers(1, 5))
        b = np.stack([P.rhs_uniform(probs[k].n, 1000 + 10 * i + j) for j in range(nr)])
        ids[srv.submit(k, probs[k].G, 2, probs[k].grid, b, tol=1e-8, cmin=(2,),
                       max_coarse=200)] = (k, b)
        if i == 11:
            mid = srv.submit(0, probs[0].G, 2, probs[0].grid, b0, tol=1e-8, cmin=(2,),
                             max_coarse=200)
    res = drain(srv, 25)
    st = srv.stats()
    srv.close()
    for rid_, (k, b) in ids.items():
        assert res[rid_]["status"] == 0
        check(probs[k], b, res[rid_]["x"], 1e-8)
    mix = res[mid]
    assert mix["status"] == 0
    check(probs[0], b0, mix["x"], 1e-8)
    for j in range(3):
        d = np.linalg.norm(mix["x"][j] - alone["x"][j]) / np.linalg.norm(alone["x"][j])
        assert d <= 1e-6
    # one setup per operator; later requests either joined a running batch or hit
    assert st["misses"] == len(OPS) and st["completed"] == 25
    assert max(r["batch_rhs"] for r in res.values()) > 4     # requests were merged


def test_join_running_solve(gpu_device):
    """Requests for an operator whose solve is running enter it at the next
    PCG iteration boundary and finish on their own while it goes on: a
    two-column request that cannot converge (tol 1e-15) runs its 300
    iterations while three requests submitted after it started join it,
    converge to 1e-8 and are reported first; each equals its solve alone to
    within what two solutions at that tolerance can differ by
    (2 tol cond(A) relative)."""
    import time
    p = op(0)
    A = (p.G.T @ p.G).toarray()
    ev = np.linalg.eigvalsh(A)
    bound = 2 * 1e-8 * ev[-1] / ev[0]
    long_b = np.stack([P.rhs_uniform(p.n, 50 + j) for j in range(2)])
    joiners = [np.stack([P.rhs_uniform(p.n, 60 + 4 * i + j) for j in range(1 + i)])
               for i in range(3)]
    alone = []
    for b in joiners:
        srv = L.Server(hbm_budget=8 << 30, max_slots=1)
        rid = srv.submit(0, p.G, 2, p.grid, b, tol=1e-8, cmin=(2,), max_coarse=200)
        alone.append(drain(srv, 1)[rid])
        srv.close()
    srv = L.Server(hbm_budget=8 << 30, max_slots=2)
    r_long = srv.submit(0, p.G, 2, p.grid, long_b, tol=1e-15, maxit=300, cmin=(2,),
                        max_coarse=200)
    t0 = time.time()
    while srv.stats()["iterations"] < 5:   # until the long solve is iterating
        assert time.time() - t0 < 60
        time.sleep(0.002)
    ids = [srv.submit(0, p.G, 2, p.grid, b, tol=1e-8, cmin=(2,), max_coarse=200)
           for b in joiners]
    order = []
    res = {}
    t0 = time.time()
    while len(res) < 4 and time.time() - t0 < 120:
        for d in srv.poll(wait_ms=200):
            res[d["id"]] = d
            order.append(d["id"])
    st = srv.stats()
    srv.close()
    assert len(res) == 4
    assert res[r_long]["status"] == L.LSAMG_ENOCONV and res[r_long]["iters_max"] == 300
    assert order[-1] == r_long           # the joiners finished while it ran
    for rid, b, a in zip(ids, joiners, alone):
        d = res[rid]
        assert d["status"] == 0 and d["joined_at"] > 0 and d["cache_hit"] == 1
        check(p, b, d["x"], 1e-8)
        for j in range(b.shape[0]):
            e = np.linalg.norm(d["x"][j] - a["x"][j]) / np.linalg.norm(a["x"][j])
            assert e <= bound, (rid, j, e, bound)
    assert st["joins"] >= 3 and st["misses"] == 1


def _start_long(srv, p, nr=2):
    """a request that cannot converge (tol 1e-15) and keeps its solve running
    for 200 iterations; returns its id once that solve is iterating"""
    import time
    b = np.stack([P.rhs_uniform(p.n, 70 + j) for j in range(nr)])
    rid = srv.submit(0, p.G, 2, p.grid, b, tol=1e-15, maxit=200, cmin=(2,), max_coarse=200)
    t0 = time.time()
    while srv.stats()["iterations"] < 5:
        assert time.time() - t0 < 60
        time.sleep(0.002)
    return rid


def test_admission_first_come_first_served(gpu_device):
    """Requests enter a running solve in arrival order: with 6 of its 8
    columns free, a 5-column request joins, a 4-column one then waits for
    columns, and a 1-column request behind it (which would fit the last free
    column at once) must not overtake it."""
    p = op(0)
    srv = L.Server(hbm_budget=8 << 30, max_slots=1)
    r_long = _start_long(srv, p)
    bs = [np.stack([P.rhs_uniform(p.n, 80 + 10 * i + j) for j in range(nr)])
          for i, nr in enumerate((5, 4, 1))]
    ids = [srv.submit(0, p.G, 2, p.grid, b, tol=1e-8, cmin=(2,), max_coarse=200) for b in bs]
    res = drain(srv, 4)
    srv.close()
    assert res[r_long]["status"] == L.LSAMG_ENOCONV
    for rid, b in zip(ids, bs):
        assert res[rid]["status"] == 0
        check(p, b, res[rid]["x"], 1e-8)
    a, b4, c1 = (res[r] for r in ids)
    assert a["joined_at"] > 0 and b4["joined_at"] > a["joined_at"]
    assert c1["joined_at"] >= b4["joined_at"], (b4["joined_at"], c1["joined_at"])


def test_waiting_batch_widens_the_next_solve(gpu_device):
    """When the columns waiting for an operator fill a whole batch of the
    running width, that solve takes no more requests: of three 4-column
    requests arriving at an 8-column solve with 6 free columns, the first
    joins it, and the other two start together in the next solve (joined at
    its first iteration) instead of trickling into the narrow one."""
    p = op(0)
    srv = L.Server(hbm_budget=8 << 30, max_slots=1)
    r_long = _start_long(srv, p)
    bs = [np.stack([P.rhs_uniform(p.n, 120 + 10 * i + j) for j in range(4)]) for i in range(3)]
    ids = [srv.submit(0, p.G, 2, p.grid, b, tol=1e-8, cmin=(2,), max_coarse=200) for b in bs]
    res = drain(srv, 4)
    srv.close()
    assert res[r_long]["status"] == L.LSAMG_ENOCONV and res[r_long]["iters_max"] == 200
    for rid, b in zip(ids, bs):
        assert res[rid]["status"] == 0 and res[rid]["cache_hit"] == 1
        check(p, b, res[rid]["x"], 1e-8)
    assert res[ids[0]]["joined_at"] > 0
    assert res[ids[1]]["joined_at"] == 0 and res[ids[2]]["joined_at"] == 0
    assert res[ids[1]]["batch_rhs"] == 8 and res[ids[2]]["batch_rhs"] == 8


def test_budget_admission_and_eviction(gpu_device):
    probs = [op(k) for k in range(3)]
    # size the budget for about one hierarchy
    s = L.Solver(probs[2].G, 2, probs[2].grid, device=0, cmin=(2,), max_coarse=200)
    one = s.info()["device_bytes"]
    s.close()
    srv = L.Server(hbm_budget=int(one * 1.5), max_slots=2)
    ids = {}
    for i in range(9):
        k = i % 3
        b = P.rhs_uniform(probs[k].n, 300 + i)
        ids[srv.submit(k, probs[k].G, 2, probs[k].grid, b, tol=1e-8, cmin=(2,),
                       max_coarse=200, precision=L.FP64)] = (k, b)
    res = drain(srv, 9)
    st = srv.stats()
    srv.close()
    for rid, (k, b) in ids.items():
        assert res[rid]["status"] == 0
        check(probs[k], b, res[rid]["x"], 1e-8)
    assert st["evictions"] >= 1
    # every solve's own device memory was admitted before it ran
    assert st["peak_bytes"] <= int(one * 1.5) and st["reserve_misses"] == 0


def test_failed_setup_is_isolated(gpu_device):
    good = op(3)
    bad = P.aniso2d(32, 0.0, 1.0)
    Gb = bad.G.tolil()
    Gb[:, 7] = 0.0                       # an unknown no row touches: A singular
    import scipy.sparse as sp
    Gb = sp.csr_matrix(Gb)
    srv = L.Server(hbm_budget=4 << 30, max_slots=2)
    r_bad = srv.submit(9, Gb, 2, bad.grid, np.ones(bad.n), tol=1e-8, max_coarse=100)
    r_bad2 = srv.submit(9, Gb, 2, bad.grid, np.ones(bad.n), tol=1e-8, max_coarse=100)
    b = P.rhs_uniform(good.n, 4)
    r_ok = srv.submit(3, good.G, 2, good.grid, b, tol=1e-8, max_coarse=100)
    res = drain(srv, 3)
    srv.close()
    assert res[r_bad]["status"] == L.LSAMG_ENOTSPD
    assert res[r_bad2]["status"] == L.LSAMG_ENOTSPD
    assert res[r_ok]["status"] == 0
    check(good, b, res[r_ok]["x"], 1e-8)


def test_hierarchy_larger_than_budget(gpu_device):
    p = op(0)
    srv = L.Server(hbm_budget=1 << 20, max_slots=1)
    rid = srv.submit(0, p.G, 2, p.grid, np.ones(p.n), tol=1e-8, cmin=(2,), max_coarse=200)
    res = drain(srv, 1)
    srv.close()
    assert res[rid]["status"] == L.LSAMG_ENOMEM


def test_device_setup_in_server(gpu_device):
    """Requests asking for the setup on the device: the server runs it on its
    device with 24 GiB of the budget held meanwhile; the solutions reach the
    tolerance and equal those of a host setup within it; a singular operator
    fails alone (its device Cholesky reports it); a budget below the setup's
    transient need fails the request with LSAMG_ENOMEM."""
    probs = [op(0), op(1)]
    bad = P.aniso2d(32, 0.0, 1.0)
    Gb = bad.G.tolil()
    Gb[:, 7] = 0.0
    import scipy.sparse as sp
    Gb = sp.csr_matrix(Gb)
    srv = L.Server(hbm_budget=40 << 30, max_slots=2)
    ids = {}
    for i in range(6):
        k = i % 2
        b = np.stack([P.rhs_uniform(probs[k].n, 500 + 4 * i + j) for j in range(2)])
        ids[srv.submit(k, probs[k].G, 2, probs[k].grid, b, tol=1e-8, cmin=(2,),
                       max_coarse=200, setup_device=True)] = (k, b)
    r_bad = srv.submit(9, Gb, 2, bad.grid, np.ones(bad.n), tol=1e-8, max_coarse=100,
                       setup_device=True)
    res = drain(srv, 7)
    st = srv.stats()
    srv.close()
    assert res[r_bad]["status"] == L.LSAMG_ENOTSPD
    for rid, (k, b) in ids.items():
        assert res[rid]["status"] == 0, res[rid]["msg"]
        check(probs[k], b, res[rid]["x"], 1e-8)
    assert st["peak_bytes"] <= 40 << 30
    # the same requests with a host setup: solutions within the tolerance
    srv = L.Server(hbm_budget=8 << 30, max_slots=2)
    host_ids = {}
    for rid, (k, b) in ids.items():
        host_ids[srv.submit(k, probs[k].G, 2, probs[k].grid, b, tol=1e-8, cmin=(2,),
                            max_coarse=200)] = rid
    hres = drain(srv, len(ids))
    srv.close()
    for hid, rid in host_ids.items():
        xd, xh = np.atleast_2d(res[rid]["x"]), np.atleast_2d(hres[hid]["x"])
        for j in range(xd.shape[0]):
            assert np.linalg.norm(xd[j] - xh[j]) <= 1e-6 * np.linalg.norm(xh[j])
    # a budget below the setup's transient need: a request that asks for the
    # device fails, one in the automatic mode (an operator of over 100,000
    # unknowns, which would go to the device) is set up on the host
    big = P.aniso2d(320, 0.4, 1e-3)
    srv = L.Server(hbm_budget=8 << 30, max_slots=1)
    rid = srv.submit(0, probs[0].G, 2, probs[0].grid, np.ones(probs[0].n), tol=1e-8, cmin=(2,),
                     max_coarse=200, setup_device=True)
    bb = P.rhs_uniform(big.n, 77)
    rid2 = srv.submit(1, big.G, 2, big.grid, bb, tol=1e-8, cmin=(2,), setup_device="auto")
    r = drain(srv, 2)
    srv.close()
    assert r[rid]["status"] == L.LSAMG_ENOMEM
    assert big.n >= 100000 and r[rid2]["status"] == 0, r[rid2]["msg"]
    check(big, bb, r[rid2]["x"], 1e-8)
