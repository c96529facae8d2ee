"""GPU parity of the ablation variants of Section 7.3 (tc_graph_variant) and
of the per-rank work of Section 7.2 (tc_block_stats), through the C ABI
against the CPU oracle.

Every variant counts the same T (Eq. 2) with a different amount of work:
- <i,j,k> (hash U_i, look up all of U_j): probes = sum of |U_j| over the
  nonzeros (i, j) (the oracle's probes_ijk);
- no doubly sparse traversal: intersections with an empty hashed list are
  kept, so probes = W+ (sum_a C(|U_a|, 2));
- multiplicative hashing: the default work, other table addressing.
"""
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


def cases():
    out = [("K40", sg.complete(40)), ("wheel100", sg.wheel(100)), ("tripartite", sg.complete_tripartite(4, 6, 9)[0]),
           ("messy", sg.messy(*sg.random_graph(200, 0.1, 3), seed=1)), ("star", sg.star(30))]
    s, d = graphgen.er(4096, 32768, seed=2)
    out.append(("er4096", (s, d, 4096)))
    for scale, seed in ((12, 1), (16, 2)):
        s, d = graphgen.rmat(scale, seed=seed)
        out.append(("rmat%d" % scale, (s, d, 1 << scale)))
    return out


@pytest.mark.parametrize("name,g", cases(), ids=[c[0] for c in cases()])
def test_variants_count_T_with_their_work(tc, name, g):
    s, d, n = g
    U = oracle.preprocess(s, d, n)
    T = oracle.count(U)
    w = oracle.wedges(U)
    deg = np.diff(U.row_ptr)
    ijk_tasks = int((deg[U.col] > 0).sum())
    all_tasks = int(np.maximum(deg - 1, 0).sum())
    G = tc.tc_preprocess(dev(s), dev(d), n)
    for flags in range(1, 8):
        print("case %s flags %d" % (name, flags), flush=True)
        V = tc.tc_graph_variant(G, flags)
        info = V.info()
        ijk, nodcsr = bool(flags & tc.TC_VARIANT_IJK), bool(flags & tc.TC_VARIANT_NO_DCSR)
        if ijk:
            assert info["probes"] == w["probes_ijk"] and info["tasks"] == ijk_tasks
        elif nodcsr:
            assert info["probes"] == w["wedges_plus"] and info["tasks"] == all_tasks
        else:
            assert info["probes"] == w["probes"] and info["tasks"] == w["tasks"]
        c = tc.tc_count(V)
        torch.cuda.synchronize()
        assert int(c.item()) == T, flags
        tc.tc_graph_class_stats(V)
        V.free()
    G.free()


def test_variant_refusals(tc):
    s, d, n = sg.complete(10)
    G = tc.tc_preprocess(dev(s), dev(d), n)
    V = tc.tc_graph_variant(G, tc.TC_VARIANT_IJK)
    with pytest.raises(tc.TCError):
        tc.tc_graph_variant(V, tc.TC_VARIANT_MUL_HASH)
    with pytest.raises(tc.TCError):
        tc.tc_edge_support(V, tc.TC_SUPPORT_FULL)
    with pytest.raises(tc.TCError):
        tc.tc_block_count(V, 2, 0, 0)
    with pytest.raises(tc.TCError):
        tc.tc_truss(V)
    with pytest.raises(tc.TCError):
        tc.tc_batch_create([V])
    with pytest.raises(tc.TCError):
        tc.tc_graph_variant(G, 8)
    assert int(tc.tc_count(V).item()) == 120
    V.free()
    G.free()


def _check_rank(tc, G, U, q, x, y):
    want = oracle.block_work(U, q, x, y)
    got = tc.tc_block_stats(G, q, x, y).cpu().numpy()
    assert got[0] == want["tasks"] and got[1] == want["probes"], (q, x, y)
    assert np.array_equal(got[2:2 + q], want["shift_probes"]), (q, x, y)
    assert np.array_equal(got[2 + q:], want["shift_tasks"]), (q, x, y)


@pytest.mark.parametrize("q", [1, 2, 3, 5, 13])
def test_block_stats_every_rank_small(tc, q):
    s, d = graphgen.rmat(10, seed=17)
    n = 1 << 10
    U = oracle.preprocess(s, d, n)
    G = tc.tc_preprocess(dev(s), dev(d), n)
    for x in range(q):
        for y in range(q):
            _check_rank(tc, G, U, q, x, y)


def test_block_stats_rmat16_and_20(tc):
    for scale, q, ranks in ((16, 13, [(0, 0), (5, 11), (12, 12)]), (20, 4, [(1, 3)])):
        print("block stats rmat%d q=%d" % (scale, q), flush=True)
        s, d = graphgen.rmat(scale, seed=scale)
        n = 1 << scale
        U = oracle.preprocess(s, d, n)
        G = tc.tc_preprocess(dev(s), dev(d), n)
        for x, y in ranks:
            _check_rank(tc, G, U, q, x, y)
        G.free()
