"""Continuous batching on the GPU: requests of several shapes served
together return what each returns alone (bitwise: per-item masks, fixed-order
reductions and size-independent kernel choices), match the FP64 oracle to
the mixed-path bar, respect the memory budget and complete out of order."""
import time

import numpy as np
import pytest

import hom_inputs as hi

gpu = pytest.mark.gpu


@pytest.fixture(scope="module")
def hom():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1311_0089_amd as h
    h.lib()
    return h


def drain(server, tickets, timeout=120.0):
    out = {}
    t0 = time.time()
    while len(out) < len(tickets):
        assert time.time() - t0 < timeout, "server did not finish"
        for key, (t, L, d) in tickets.items():
            if key in out:
                continue
            r = server.poll(t, L, d)
            if r is not None:
                out[key] = r
        time.sleep(0.002)
    return out


def make_requests(hom, n=8):
    reqs = []
    shapes = [((31, 31), 0), ((15, 15, 15), 0), ((63, 63), 1), ((15, 31, 15), 2), ((31, 31), 0)]
    for i in range(n):
        N, kind = shapes[i % len(shapes)]
        d = len(N)
        A = hi.random_spd_field(N, kind, seed=300 + i, contrast=10.0 ** (1 + (i % 3)))
        L = 1 + i % d
        reqs.append((hom.Cell(A, N, kind=kind, prec=hom.MIXED, check_every=8), A, N, kind, L))
    return reqs


@gpu
def test_served_equals_alone_and_oracle(hom, oracle):
    reqs = make_requests(hom, 8)
    alone = []
    for cell, A, N, kind, L in reqs:
        alone.append(cell.solve(np.eye(len(N))[:L], tol=1e-8)["W"])
    srv = hom.Server(hbm_budget_bytes=8 << 30, prec=hom.MIXED, check_every=8)
    tickets = {}
    for rep in range(2):
        for i, (cell, A, N, kind, L) in enumerate(reqs):
            tickets[(rep, i)] = (srv.submit(cell, np.eye(len(N))[:L], tol=1e-8), L, len(N))
    res = drain(srv, tickets)
    srv.close()
    for (rep, i), r in res.items():
        assert r["status"] == 0
        np.testing.assert_array_equal(r["W"], alone[i])
    # accuracy against the oracle for the first two shapes
    for i in (0, 1):
        cell, A, N, kind, L = reqs[i]
        oc = oracle.Cell(A, N, kind=kind)
        _, W, _, _ = oc.solve(np.eye(len(N))[:L], tol=1e-12)
        assert np.abs(res[(0, i)]["W"] - W).max() / np.abs(W).max() < 1e-6


@gpu
def test_out_of_order_completion(hom):
    """Small requests submitted after a large one are admitted into their own
    class at once and finish first; results equal the solves alone."""
    big = hom.Cell(hi.bernoulli_majority((127, 127, 127), 0.4, 3, 1000.0, 1.0, seed=1),
                   (127, 127, 127), prec=hom.MIXED)
    small = [hom.Cell(hi.random_spd_field((15, 15), 0, seed=10 + i, contrast=10.0), (15, 15),
                      prec=hom.MIXED) for i in range(4)]
    ref_big = big.solve(np.eye(3), tol=1e-7)["W"]
    ref_small = [c.solve(np.eye(2)[:1], tol=1e-7)["W"] for c in small]
    srv = hom.Server(hbm_budget_bytes=4 << 30, prec=hom.MIXED)
    tickets = {"big": (srv.submit(big, np.eye(3), tol=1e-7), 3, 3)}
    for i, c in enumerate(small):
        tickets[i] = (srv.submit(c, np.eye(2)[:1], tol=1e-7), 1, 2)
    res = drain(srv, tickets)
    srv.close()
    np.testing.assert_array_equal(res["big"]["W"], ref_big)
    for i in range(4):
        np.testing.assert_array_equal(res[i]["W"], ref_small[i])
    assert max(res[i]["times"][2] for i in range(4)) < res["big"]["times"][2]


@gpu
def test_admission_waits_for_memory(hom):
    """With a budget of one slot of the class, a second request waits until
    the first has retired and frees its slot; a request larger than the whole
    budget is rejected at submit."""
    cells = [hom.Cell(hi.random_spd_field((63, 63, 63), 0, seed=20 + i, contrast=30.0),
                      (63, 63, 63), prec=hom.MIXED) for i in range(2)]
    refs = [c.solve(np.eye(3)[:1], tol=1e-7)["W"] for c in cells]
    srv = hom.Server(hbm_budget_bytes=200 << 20, prec=hom.MIXED)
    tickets = {i: (srv.submit(c, np.eye(3)[:1], tol=1e-7), 1, 3) for i, c in enumerate(cells)}
    res = drain(srv, tickets)
    for i in range(2):
        np.testing.assert_array_equal(res[i]["W"], refs[i])
    first, second = sorted(res.values(), key=lambda r: r["times"][1])
    assert second["times"][1] >= first["times"][2] - 1e-6
    huge = hom.Cell(hi.random_spd_field((127, 127, 127), 0, seed=2, contrast=10.0),
                    (127, 127, 127), prec=hom.MIXED)
    with pytest.raises(hom.HomError) as ei:
        srv.submit(huge, np.eye(3), tol=1e-6)
    assert ei.value.code == -3
    srv.close()
