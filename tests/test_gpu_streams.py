"""Stream ordering of the library's frees (GPU).

tc_graph_free and tc_batch_free return without draining the device: the
memory of a graph goes back to the library's cache reusable only after the
work of every stream that used the graph, and a plan's free waits for its
own launches. Here a graph built on one stream is counted repeatedly on a
second stream, freed at once, and its memory is immediately taken again by
preprocessing on the first stream; the counts on the second stream must
still be the oracle's T."""
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
    assert int(tc.tc_count(g, stream=sa).item()) == T
    g.free()


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
