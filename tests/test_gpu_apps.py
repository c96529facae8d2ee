"""GPU parity of the uses of the counts the paper's introduction names
(Section 1): per-vertex triangle counts, local clustering coefficients and
transitivity, and trussness (the k-truss decomposition), through the C ABI,
against the CPU oracle. Counts and trussness are integers (equality); the
clustering coefficients are single correctly rounded divisions of exact
integers on both sides, so they are compared for equality too."""
import numpy as np
import pytest

import graphgen
import oracle
import smallgraphs as sg

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def tc():
    if not torch.cuda.is_available():
        pytest.fail("no GPU visible")
    import paper_1907_09575_amd as tc
    torch.cuda.set_device(0)
    return tc


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.int32)).to("cuda")


def graphs():
    out = [("K12", sg.complete(12)), ("wheel30", sg.wheel(30)), ("friendship9", sg.friendship(9)),
           ("cliques7_11", sg.cliques_sharing_vertex(7, 11)), ("clique_pend", sg.clique_with_pendants(9, 6)),
           ("tripartite", sg.complete_tripartite(3, 5, 7)[0]), ("tree", sg.random_tree(300, 4)),
           ("star", sg.star(40)), ("messy", sg.messy(*sg.random_graph(150, 0.12, 5), seed=2))]
    s, d = graphgen.er(4096, 32768, seed=1)
    out.append(("er4096", (s, d, 4096)))
    for scale, seed in ((10, 3), (12, 5)):
        s, d = graphgen.rmat(scale, seed=seed)
        out.append(("rmat%d" % scale, (s, d, 1 << scale)))
    return out


@pytest.mark.parametrize("name,g", graphs(), ids=[x[0] for x in graphs()])
def test_vertex_counts_and_clustering(tc, name, g):
    s, d, n = g
    print("case %s n=%d m_raw=%d" % (name, n, len(s)), flush=True)
    U = oracle.preprocess(s, d, n)
    cc_ref, tr_ref, t_ref, W = oracle.clustering(U)
    G = tc.tc_preprocess(dev(s), dev(d), n)
    t = tc.tc_vertex_triangles(G)
    tri = torch.empty(n, dtype=torch.int64, device="cuda")
    sums = torch.empty(2, dtype=torch.int64, device="cuda")
    cc, _, _ = tc.tc_clustering(G, tri=tri, sums=sums)
    torch.cuda.synchronize()
    assert np.array_equal(t.cpu().numpy(), t_ref)
    assert np.array_equal(tri.cpu().numpy(), t_ref)
    assert np.array_equal(cc.cpu().numpy(), cc_ref)
    assert sums.cpu().tolist() == [int(t_ref.sum()), W]
    assert tc.tc_transitivity(G) == tr_ref
    G.free()


@pytest.mark.parametrize("name,g", graphs(), ids=[x[0] for x in graphs()])
def test_truss(tc, name, g):
    s, d, n = g
    print("case %s n=%d m_raw=%d" % (name, n, len(s)), flush=True)
    U = oracle.preprocess(s, d, n)
    kmax_ref, tau_ref = oracle.truss(U)
    G = tc.tc_preprocess(dev(s), dev(d), n)
    tau, kmax = tc.tc_truss(G)
    torch.cuda.synchronize()
    assert kmax == kmax_ref
    assert np.array_equal(tau.cpu().numpy(), tau_ref)
    G.free()


def test_truss_rmat13_and_repeat(tc):
    # a larger graph, twice on one handle (the handle is not changed)
    s, d = graphgen.rmat(13, seed=7)
    n = 1 << 13
    U = oracle.preprocess(s, d, n)
    kmax_ref, tau_ref = oracle.truss(U)
    G = tc.tc_preprocess(dev(s), dev(d), n)
    for _ in range(2):
        tau, kmax = tc.tc_truss(G)
        torch.cuda.synchronize()
        assert kmax == kmax_ref
        assert np.array_equal(tau.cpu().numpy(), tau_ref)
    assert int(tc.tc_count(G).item()) == oracle.count(U)


def test_apps_empty_graph(tc):
    G = tc.tc_preprocess(dev(np.zeros(0)), dev(np.zeros(0)), 5)
    t = tc.tc_vertex_triangles(G)
    cc, _, _ = tc.tc_clustering(G)
    torch.cuda.synchronize()
    assert not t.cpu().numpy().any() and not cc.cpu().numpy().any()
    assert tc.tc_transitivity(G) == 0.0
    tau, kmax = tc.tc_truss(G)
    assert kmax == 0 and tau.numel() == 0
    with pytest.raises(tc.TCError):
        tc._check(tc._lib.tc_clustering(G.handle, None, None, None, None), "tc_clustering")
