"""GPU checks of the row-bucket thresholds and the autotuners.

The thresholds only change how a graph's work is cut into packs and items:
under any of them tc_count must give the oracle's T (Eq. 2) and tc_edge_support
the same per-edge values (Eq. 1), and the class statistics must still cover
every probe exactly once. The autotuners store their best setting in the
tuning table, which later tc_preprocess calls and batch plans pick up; every
entry a test stores is removed again.
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


def support(tc, g, mode):
    sup, _ = tc.tc_edge_support(g, mode)
    return sup[: g.info()["m"]].cpu().numpy()


def cases():
    out = [("K300", sg.complete(300)), ("wheel500", sg.wheel(500)),
           ("tripartite", sg.complete_tripartite(20, 30, 45)[0]),
           ("messy", sg.messy(*sg.random_graph(300, 0.08, 3), seed=4))]
    s, d = graphgen.er(4096, 65536, seed=5)
    out.append(("er4096", (s, d, 4096)))
    s, d = graphgen.rmat(16, seed=3)
    out.append(("rmat16", (s, d, 1 << 16)))
    return out


PARAMS = [
    {"heavy_min": 0},                                    # no packs at all
    {"heavy_min": 1 << 24, "pack_target": 1 << 24},      # every row of a small table packed
    {"wave_chunk": 1024, "pack_target": 1024, "pack_slots": 1024},   # finest cuts
    {"pack_slots": 16384, "wave_chunk": 4096, "heavy_min": 8192},
    {"wave_chunk": 32767, "min_groups": 0},              # largest items, no class-size rule
    {"min_groups": 1 << 22},                             # every item class at the smallest items
]


@pytest.mark.parametrize("name,g", cases(), ids=[c[0] for c in cases()])
def test_retuned_counts_and_support(tc, name, g):
    s, d, n = g
    U = oracle.preprocess(s, d, n)
    T = oracle.count(U)
    G = tc.tc_preprocess(dev(s), dev(d), n)
    info = G.info()
    full0 = support(tc, G, tc.TC_SUPPORT_FULL)
    ori0 = support(tc, G, tc.TC_SUPPORT_ORIENTED)
    assert full0.sum() == 3 * T and ori0.sum() == T
    for p in PARAMS:
        print("case %s params %s" % (name, p), flush=True)
        H = tc.tc_graph_retune(G, p)
        wp = tc.tc_graph_work_params(H)
        for k, v in p.items():
            assert wp[k] == v
        assert int(tc.tc_count(H).item()) == T
        assert np.array_equal(support(tc, H, tc.TC_SUPPORT_FULL), full0)
        assert np.array_equal(support(tc, H, tc.TC_SUPPORT_ORIENTED), ori0)
        hi = H.info()
        assert (hi["m"], hi["probes"], hi["tasks"]) == (info["m"], info["probes"], info["tasks"])
        st = tc.tc_graph_class_stats(H)
        assert sum(c["probes"] for c in st.values()) == info["probes"]
        assert sum(c["tasks"] for c in st.values()) == info["tasks"]
        packed = st["pack_small"]["rows"] + st["pack_large"]["rows"]
        if p.get("heavy_min") == 0:
            assert packed == 0
        H.free()
    torch.cuda.synchronize()


def test_retune_invalid(tc):
    s, d, n = sg.complete(20)
    G = tc.tc_preprocess(dev(s), dev(d), n)
    for bad in ['{"wave_chunk": 512}', '{"wave_chunk": 32768}', '{"pack_slots": 100000}', '{"heavy_min": -1}',
                '{"min_groups": 4194305}',
                '{"pack_target": 10}', '{"nope": 1}', 'not json']:
        with pytest.raises(tc.TCError) as e:
            tc.tc_graph_retune(G, bad)
        assert e.value.status == 1, bad
    V = tc.tc_graph_variant(G, tc.TC_VARIANT_IJK)
    with pytest.raises(tc.TCError):
        tc.tc_graph_retune(V, {"heavy_min": 0})


def test_tuning_key_names_the_device(tc):
    key = tc.tc_tuning_key("graph", 1 << 20)
    arch, cus, tail = key.split("/")
    assert arch.startswith("gfx") and cus.endswith("cu") and tail == "graph_e20"
    assert tc.tc_tuning_key("batch", (1 << 21) - 1).endswith("/batch_e20")


def test_graph_autotune_feeds_preprocess(tc):
    s, d = graphgen.rmat(16, seed=7)
    n = 1 << 16
    T = oracle.count(oracle.preprocess(s, d, n))
    G = tc.tc_preprocess(dev(s), dev(d), n)
    res = tc.tc_graph_autotune(G)
    key = res["key"]
    try:
        best = res["best"]
        assert tc.tc_tuning_get(key) == best
        assert len(res["candidates"]) >= 8 and all(c["ms"] > 0 for c in res["candidates"])
        assert best["ms"] == min(c["ms"] for c in res["candidates"])
        # a graph of the same size preprocessed now is cut by the tuned thresholds
        G2 = tc.tc_preprocess(dev(s), dev(d), n)
        wp = tc.tc_graph_work_params(G2)
        assert all(wp[k] == best[k] for k in ("heavy_min", "pack_target", "pack_slots", "wave_chunk", "min_groups"))
        assert int(tc.tc_count(G2).item()) == T
    finally:
        tc.tc_tuning_set(key, None)
    G3 = tc.tc_preprocess(dev(s), dev(d), n)
    assert tc.tc_graph_work_params(G3) == {"heavy_min": 32768, "pack_target": 65536, "pack_slots": 4096,
                                           "wave_chunk": 32767, "min_groups": 16384}
