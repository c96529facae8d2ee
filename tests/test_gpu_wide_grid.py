"""Launch shapes at 2^26 vertices: kernels that give one wave to each vertex,
row or work-group item must keep a dispatch below 2^32 work-items (a wave per
row of a 2^26-vertex graph is exactly 2^32). A complete graph K6 on six ids
spread over [0, 2^26) reaches every such launch cheaply: the work-set
rebuilds (tc_graph_retune and the ablation variants), per-vertex counts and
clustering, the k-truss peel, and a q = 1 block (one rank holding every
row). Expected values are closed forms of K6: C(6, 3) = 20 triangles,
C(5, 2) = 10 through each of its vertices and 0 elsewhere, every edge of
trussness 6."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

N = 1 << 26
IDS = [0, 1, 1 << 25, N - 3, N - 2, N - 1]


@pytest.fixture(scope="module")
def tc():
    if not torch.cuda.is_available():
        pytest.fail("no GPU visible")
    import paper_1907_09575_amd as tc
    torch.cuda.set_device(0)
    return tc


@pytest.fixture(scope="module")
def g(tc):
    pairs = [(u, v) for i, u in enumerate(IDS) for v in IDS[i + 1:]]
    s = torch.tensor([p[0] for p in pairs], dtype=torch.int32, device="cuda")
    d = torch.tensor([p[1] for p in pairs], dtype=torch.int32, device="cuda")
    G = tc.tc_preprocess(s, d, N)
    yield G
    G.free()


def test_count_retune_and_variants(tc, g):
    print("K6 in n = 2^26: count, retune, variants", flush=True)
    assert int(tc.tc_count(g).item()) == 20
    info = tc.tc_graph_info(g)
    assert info["m"] == 15
    for params in ({"wave_chunk": 1024, "heavy_min": 1024}, {"min_groups": 0}):
        h = tc.tc_graph_retune(g, params)
        assert int(tc.tc_count(h).item()) == 20, params
        h.free()
    for flags in (tc.TC_VARIANT_IJK, tc.TC_VARIANT_NO_DCSR, tc.TC_VARIANT_MUL_HASH):
        v = tc.tc_graph_variant(g, flags)
        assert int(tc.tc_count(v).item()) == 20, flags
        v.free()


def test_vertex_counts_clustering_truss(tc, g):
    print("K6 in n = 2^26: vertex counts, clustering, truss", flush=True)
    t = tc.tc_vertex_triangles(g).cpu().numpy()
    want = np.zeros(N, dtype=np.int64)
    want[IDS] = 10
    assert np.array_equal(t, want)
    cc, _, _ = tc.tc_clustering(g)
    cc = cc.cpu().numpy()
    assert np.all(cc[IDS] == 1.0) and np.count_nonzero(cc) == len(IDS)
    tau, kmax = tc.tc_truss(g)
    assert kmax == 6 and np.all(tau.cpu().numpy() == 6)


def test_block_q1(tc, g):
    print("K6 in n = 2^26: block q = 1", flush=True)
    ps = torch.empty(1, dtype=torch.int64, device="cuda")
    cnt, _ = tc.tc_block_count(g, 1, 0, 0, per_shift=ps)
    assert int(cnt.item()) == 20 and ps.cpu().tolist() == [20]
    st = tc.tc_block_stats(g, 1, 0, 0).cpu().tolist()
    info = tc.tc_graph_info(g)
    assert st[0] == info["tasks"] and st[1] == info["probes"]
    assert st[2] == info["probes"] and st[3] == info["tasks"]
