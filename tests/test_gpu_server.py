"""GPU tests of the served form (tc_server_*): continuous batching with
HBM-budget admission and a device graph cache.

The bar is exactness: every request's count (and support array, in U order)
is the same integer result alone as in the mix, and equals the plain
tc_preprocess + tc_count / tc_edge_support path (itself parity-tested against
the oracle); sampled requests are also checked against the oracle directly.
"""
import time

import numpy as np
import pytest

import graphgen
import oracle

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

GiB = 1 << 30


@pytest.fixture(scope="module")
def tc():
    if not torch.cuda.is_available():
        pytest.fail("no GPU visible")
    import paper_1907_09575_amd as tc
    torch.cuda.set_device(0)
    return tc


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.int32)).to("cuda")


def plain(tc, op, s, d, n):
    """The single-request path: tc_preprocess + tc_count / tc_edge_support."""
    g = tc.tc_preprocess(dev(s), dev(d), n)
    if op == "count":
        c = int(tc.tc_count(g).item())
        sup = None
    else:
        mode = tc.TC_SUPPORT_FULL if op in ("support", "support_full") else tc.TC_SUPPORT_ORIENTED
        cnt = torch.empty(1, dtype=torch.int64, device="cuda")
        sup_t, _ = tc.tc_edge_support(g, mode, count=cnt)
        torch.cuda.synchronize()
        c, sup = int(cnt.item()), sup_t.cpu().numpy()
    g.free()
    return c, sup


@pytest.fixture(scope="module")
def trace():
    # a small version of the serving mix: lognormal sizes, ER/RMAT, count and
    # support, 30% re-queries of earlier graphs
    reqs = graphgen.serving_trace(90, rate_per_s=3000.0, seed=11, median_log2n=11.0, sigma=1.0,
                                  nmax=1 << 15, max_rmat_scale=15)
    graphs = {}
    for r in reqs:
        if r.spec.seed not in graphs:
            graphs[r.spec.seed] = r.spec.generate()
    print("trace: %d requests, %d graphs" % (len(reqs), len(graphs)), flush=True)
    return reqs, graphs


def run_trace(tc, srv, reqs, graphs, paced=True):
    t0 = time.perf_counter()
    tickets = []
    for r in reqs:
        if paced:
            dt = r.arrival_s - (time.perf_counter() - t0)
            if dt > 0:
                time.sleep(dt)
        s, d = graphs[r.spec.seed]
        tickets.append(srv.submit(r.op, s, d, r.spec.n, key=r.spec.seed))
    return [srv.poll(t) for t in tickets]


def test_server_mix_equals_alone(tc, trace):
    reqs, graphs = trace
    with tc.Server(64 * GiB, max_slots=32) as srv:
        mixed = run_trace(tc, srv, reqs, graphs)
        st = srv.stats()
    print(st, flush=True)
    assert st["done"] == len(reqs) and st["failed"] == 0
    assert st["max_tick_requests"] > 1, "no two requests ever shared a tick"
    assert st["cache_hits"] > 0
    # alone: the same requests one at a time through a server with one slot
    with tc.Server(64 * GiB, max_slots=1) as srv1:
        for r, mres in zip(reqs, mixed):
            s, d = graphs[r.spec.seed]
            a = srv1.poll(srv1.submit(r.op, s, d, r.spec.n))
            assert a["status"] == 0 and mres["status"] == 0
            assert a["count"] == mres["count"], r
            assert a["m"] == mres["m"]
            if r.op != "count":
                assert np.array_equal(a["support"], mres["support"]), r
    # and the plain single-graph path
    for r, mres in list(zip(reqs, mixed))[::3]:
        s, d = graphs[r.spec.seed]
        c, sup = plain(tc, r.op, s, d, r.spec.n)
        assert c == mres["count"], r
        if sup is not None:
            assert np.array_equal(sup, mres["support"]), r


def test_server_against_oracle(tc, trace):
    reqs, graphs = trace
    sample = reqs[:12]
    with tc.Server(16 * GiB, max_slots=8) as srv:
        res = run_trace(tc, srv, sample, graphs, paced=False)
    for r, x in zip(sample, res):
        s, d = graphs[r.spec.seed]
        U = oracle.preprocess(s, d, r.spec.n)
        if r.op == "count":
            assert x["count"] == oracle.count(U)
        else:
            T, sref = oracle.support(U, oracle.MODE_FULL)
            assert x["count"] == T
            assert np.array_equal(x["support"], sref)


def test_server_cache_hits_without_edges(tc):
    s, d = graphgen.rmat(12, seed=77)
    n = 1 << 12
    with tc.Server(8 * GiB, max_slots=4) as srv:
        a = srv.poll(srv.submit("count", s, d, n, key=12345))
        assert not a["cache_hit"]
        b = srv.poll(srv.submit("count", None, None, n, key=12345))
        assert b["cache_hit"] and b["count"] == a["count"]
        sup = np.empty(len(s), np.int32)
        c = srv.poll(srv.submit("support", None, None, n, key=12345, support_out=sup))
        assert c["cache_hit"] and c["count"] == a["count"]
        T, sref = oracle.support(oracle.preprocess(s, d, n), oracle.MODE_FULL)
        assert np.array_equal(c["support"], sref)
        # an unknown key without its edge list fails cleanly (m_raw > 0, no edges)
        e = srv.poll(srv.submit("support", None, None, n, key=999, support_out=np.empty(10, np.int32)))
        assert e["status"] == 1
        # m_raw == 0 is an edgeless graph, not a missing one
        z = srv.poll(srv.submit("count", None, None, n, key=998))
        assert z["status"] == 0 and z["count"] == 0 and z["m"] == 0
        st = srv.stats()
        assert st["cache_hits"] == 2 and st["cached_graphs"] == 2


def test_server_budget_admission_and_eviction(tc):
    graphs = [graphgen.rmat(13, seed=200 + i) for i in range(6)]
    n = 1 << 13
    want = [plain(tc, "count", s, d, n)[0] for s, d in graphs]
    # room for about two graphs at a time: requests wait for memory, cached
    # graphs are evicted, every result is still exact
    one = 56 * len(graphs[0][0]) + 40 * n + (1 << 20)
    with tc.Server(int(2.5 * one), max_slots=16) as srv:
        tickets = [srv.submit("count", s, d, n, key=i + 1) for i, (s, d) in enumerate(graphs)]
        res = [srv.poll(t) for t in tickets]
        again = [srv.poll(srv.submit("count", s, d, n, key=i + 1)) for i, (s, d) in enumerate(graphs)]
        st = srv.stats()
    assert [r["count"] for r in res] == want
    assert [r["count"] for r in again] == want
    assert st["peak_reserved_bytes"] <= st["budget_bytes"]
    assert st["evicted"] > 0
    # a request that can never fit fails with TC_ENOMEM instead of waiting
    with tc.Server(1 << 20, max_slots=4) as srv:
        s, d = graphs[0]
        r = srv.poll(srv.submit("count", s, d, n))
        assert r["status"] == 2


def test_server_cancel_and_shutdown(tc):
    graphs = [graphgen.er(3000, 40000, seed=300 + i) for i in range(24)]
    with tc.Server(8 * GiB, max_slots=1) as srv:
        tickets = [srv.submit("count", s, d, 3000) for s, d in graphs]
        cancelled = [srv.cancel(t) for t in tickets[12:]]
        res = [srv.poll(t) for t in tickets]
    for i, r in enumerate(res):
        if i >= 12 and cancelled[i - 12] and r["status"] == 6:
            continue
        assert r["status"] == 0
        assert r["count"] == plain(tc, "count", *graphs[i], 3000)[0]
    # destroying a server with queued requests returns promptly
    srv = tc.Server(8 * GiB, max_slots=1)
    for s, d in graphs[:8]:
        srv.submit("count", s, d, 3000)
    srv.close()


def test_server_one_and_two_ticks_in_flight_agree(tc, trace):
    reqs, graphs = trace
    res = {}
    for ticks in (1, 2):
        with tc.Server(64 * GiB, max_slots=32, options={"ticks": ticks}) as srv:
            res[ticks] = run_trace(tc, srv, reqs, graphs, paced=False)
            st = srv.stats()
        print(ticks, st, flush=True)
        assert st["tick_slots"] == ticks and st["done"] == len(reqs) and st["failed"] == 0
    for r, a, b in zip(reqs, res[1], res[2]):
        assert a["status"] == 0 and b["status"] == 0
        assert a["count"] == b["count"] and a["m"] == b["m"], r
        if r.op != "count":
            assert np.array_equal(a["support"], b["support"]), r


def test_server_rejects_bad_requests(tc):
    with tc.Server(GiB, max_slots=2) as srv:
        with pytest.raises(tc.TCError):
            srv.submit(7, np.zeros(2, np.int32), np.ones(2, np.int32), 4)
        with pytest.raises(tc.TCError):
            srv.submit("count", np.zeros(2, np.int32), np.ones(2, np.int32), 0)
        r = srv.poll(srv.submit("count", np.array([0, 5], np.int32), np.array([1, 2], np.int32), 4))
        assert r["status"] == 1  # id outside [0, n): the preprocessing rejects it
    with pytest.raises(tc.TCError):
        tc.Server(0, max_slots=2)
    with pytest.raises(tc.TCError):
        tc.Server(GiB, max_slots=2, options={"prep_threads": 99})
    with pytest.raises(tc.TCError):
        tc.Server(GiB, max_slots=2, options={"ticks": 3})
