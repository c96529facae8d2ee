"""Stream ordering of the library's frees (GPU).

tc_graph_free and tc_batch_free return without draining the device: the
memory of a graph goes back to the library's cache reusable only after the
work of every stream that used the graph, and a plan's free waits for its
own launches. Here a graph built on one stream is counted repeatedly on a
second stream, freed at once, and its memory is immediately taken again by
preprocessing on the first stream; the counts on the second stream must
still be the oracle's T. The count's side stream (its light classes run
beside the heavy ones) is also captured into HIP graphs with it. Threads
that preprocess, count and free at once, each on its own stream, take one
another's freed blocks from the cache (a reuse on another stream waits for
that stream's work): their counts must all be the oracle's."""
import numpy as np
import pytest

import graphgen
import oracle

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def tc():
    if not torch.cuda.is_available():
        pytest.fail("no GPU visible")
    import paper_1907_09575_amd as tc
    torch.cuda.set_device(0)
    return tc


def test_free_waits_for_the_streams_that_used_the_graph(tc):
    n = 1 << 17
    s, d = graphgen.rmat(17, seed=9)
    T = oracle.count(oracle.preprocess(s, d, n))
    src = torch.from_numpy(s).cuda()
    dst = torch.from_numpy(d).cuda()
    torch.cuda.synchronize()
    sa, sb = torch.cuda.Stream(), torch.cuda.Stream()
    g = tc.tc_preprocess(src, dst, n, stream=sa)
    outs = []
    for rep in range(4):
        print("free ordering round %d" % rep, flush=True)
        out = torch.full((8,), -1, dtype=torch.int64, device="cuda")
        torch.cuda.synchronize()
        for i in range(8):
            tc.tc_count(g, out[i:i + 1], stream=sb)
        g.free()  # no host wait: sb's counts may still run
        g = tc.tc_preprocess(src, dst, n, stream=sa)  # takes cached blocks again
        outs.append(out)
    sb.synchronize()
    sa.synchronize()
    for out in outs:
        assert out.cpu().tolist() == [T] * 8
    c = tc.tc_count(g, stream=sa)
    sa.synchronize()  # (the count runs on sa; .item() reads on the current stream)
    assert int(c.item()) == T
    g.free()


def test_threads_preprocessing_on_their_own_streams(tc):
    import threading
    scales = [10 + k % 4 for k in range(12)]
    lists = [graphgen.rmat(sc, seed=20 + k) for k, sc in enumerate(scales)]
    want = [oracle.count(oracle.preprocess(s, d, 1 << sc)) for (s, d), sc in zip(lists, scales)]
    dev = [(torch.from_numpy(s).cuda(), torch.from_numpy(d).cuda(), 1 << sc) for (s, d), sc in zip(lists, scales)]
    torch.cuda.synchronize()
    nthreads, reps = 4, 3
    got = [[] for _ in range(nthreads)]
    errors = []

    def worker(k):
        try:
            st = torch.cuda.Stream()
            order = [(k + j) % len(dev) for j in range(len(dev))]
            for _ in range(reps):
                for i in order:
                    s, d, n = dev[i]
                    g = tc.tc_preprocess(s, d, n, stream=st)
                    c = tc.tc_count(g, stream=st)
                    g.free()  # no host wait: another thread may take its blocks
                    st.synchronize()
                    got[k].append((i, int(c.item())))
        except Exception as e:  # reported by the main thread
            errors.append(e)

    print("%d threads x %d graphs x %d rounds" % (nthreads, len(dev), reps), flush=True)
    threads = [threading.Thread(target=worker, args=(k,)) for k in range(nthreads)]
    for th in threads:
        th.start()
    for th in threads:
        th.join()
    assert not errors, errors
    for k in range(nthreads):
        assert len(got[k]) == reps * len(dev)
        for i, c in got[k]:
            assert c == want[i], (k, i, c, want[i])


def test_plan_free_waits_for_its_launches(tc):
    lists = [graphgen.rmat(12, seed=k) for k in range(6)]
    want = [oracle.count(oracle.preprocess(s, d, 1 << 12)) for s, d in lists]
    graphs = [tc.tc_preprocess(torch.from_numpy(s).cuda(), torch.from_numpy(d).cuda(), 1 << 12) for s, d in lists]
    sb = torch.cuda.Stream()
    torch.cuda.synchronize()
    outs = []
    for rep in range(3):
        plan = tc.tc_batch_create(graphs)
        out = torch.full((len(graphs),), -1, dtype=torch.int64, device="cuda")
        torch.cuda.synchronize()
        for _ in range(4):
            tc.tc_batch_count(plan, out, stream=sb)
        plan.free()
        outs.append(out)
    sb.synchronize()
    for out in outs:
        assert out.cpu().tolist() == want


def test_count_and_support_captured_in_a_graph(tc):
    # tc_count and tc_edge_support run their light classes on a side stream
    # forked from the caller's: captured into a HIP graph, both branches are
    # recorded, and every replay (with eager work between replays) gives the
    # eager results
    s, d = graphgen.rmat(18, seed=4)
    n = 1 << 18
    G = tc.tc_preprocess(torch.from_numpy(s).cuda(), torch.from_numpy(d).cuda(), n)
    assert G.info()["probes"] >= 1 << 24  # large enough to fork
    T = int(tc.tc_count(G).item())
    m = G.info()["m"]
    full_eager, _ = tc.tc_edge_support(G, tc.TC_SUPPORT_FULL)
    full_eager = full_eager[:m].clone()
    torch.cuda.synchronize()
    out = torch.zeros(1, dtype=torch.int64, device="cuda")
    sup = torch.zeros(m, dtype=torch.int32, device="cuda")
    st = torch.cuda.Stream()
    with torch.cuda.stream(st):  # warm-up on the stream before capturing (creates its side stream)
        tc.tc_count(G, out, stream=st)
    st.synchronize()
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph, stream=st):
        tc.tc_count(G, out, stream=st)
        tc.tc_edge_support(G, tc.TC_SUPPORT_FULL, sup, stream=st)
    for r in range(4):
        out.fill_(-1)
        sup.fill_(-1)
        graph.replay()
        torch.cuda.synchronize()
        assert int(out.item()) == T, "replay %d" % r
        assert torch.equal(sup, full_eager), "replay %d" % r
        assert int(tc.tc_count(G).item()) == T  # eager work between replays
    del graph
    torch.cuda.synchronize()
