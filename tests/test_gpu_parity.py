"""GPU parity: the HIP path (through the C ABI) against the CPU oracle, bit-exact.

Every value compared here is an integer (counts, CSR arrays, per-edge support,
work counts), so the bar is equality.
"""
from math import comb

import numpy as np
import pytest

import graphgen
import grid_tasks
import oracle
import sampled_support
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


def gpu_graph(tc, src, dst, n):
    print("case n=%d m_raw=%d" % (n, len(src)), flush=True)
    return tc.tc_preprocess(dev(src), dev(dst), n)


def gpu_count(tc, g):
    c = tc.tc_count(g)
    torch.cuda.synchronize()
    return int(c.item())


def gpu_support(tc, g, mode):
    cnt = torch.empty(1, dtype=torch.int64, device="cuda")
    s, _ = tc.tc_edge_support(g, mode, count=cnt)
    torch.cuda.synchronize()
    return int(cnt.item()), s.cpu().numpy()


def check_full(tc, src, dst, n, support=True):
    U = oracle.preprocess(src, dst, n)
    g = gpu_graph(tc, src, dst, n)
    rp, col, perm = tc.tc_graph_export(g)
    torch.cuda.synchronize()
    assert np.array_equal(perm.cpu().numpy(), U.rank)
    assert np.array_equal(rp.cpu().numpy(), U.row_ptr)
    assert np.array_equal(col.cpu().numpy(), U.col)
    info = g.info()
    w = oracle.wedges(U)
    assert info["m"] == U.m
    assert info["wedges_plus"] == w["wedges_plus"]
    assert info["probes"] == w["probes"]
    assert info["tasks"] == w["tasks"]
    T = oracle.count(U)
    assert gpu_count(tc, g) == T
    if support:
        for mode in (oracle.MODE_FULL, oracle.MODE_ORIENTED):
            Tr, s_ref = oracle.support(U, mode)
            Tg, s = gpu_support(tc, g, mode)
            assert Tg == Tr == T
            assert np.array_equal(s, s_ref), "support mode %d differs" % mode
    return g, T


@pytest.mark.parametrize("name,make,expected", sg.CLOSED_FORMS, ids=[c[0] for c in sg.CLOSED_FORMS])
def test_closed_forms(tc, name, make, expected):
    s, d, n = make()
    g, T = check_full(tc, s, d, n)
    assert T == expected


def test_support_closed_forms(tc):
    m = 37
    s, d, n = sg.wheel(m)
    g = gpu_graph(tc, s, d, n)
    _, sup = gpu_support(tc, g, tc.TC_SUPPORT_FULL)
    rp, col, perm = tc.tc_graph_export(g)
    inv = np.empty(n, np.int64)
    inv[perm.cpu().numpy()] = np.arange(n)
    rp = rp.cpu().numpy()
    col = col.cpu().numpy()
    for a in range(n):
        for p in range(rp[a], rp[a + 1]):
            spoke = 0 in (inv[a], inv[col[p]])
            assert sup[p] == (2 if spoke else 1)
    s, d, n = sg.complete(50)
    g = gpu_graph(tc, s, d, n)
    _, sup = gpu_support(tc, g, tc.TC_SUPPORT_FULL)
    assert set(sup.tolist()) == {48}


@pytest.mark.parametrize("seed", range(5))
def test_random_small(tc, seed):
    s, d, n = sg.random_graph(60 + 20 * seed, 0.15, 200 + seed)
    check_full(tc, *sg.messy(s, d, n, seed=seed))


def test_er_config(tc):
    # Erdos-Renyi G(n=4096, m=32768), seed 1
    n = 4096
    s, d = graphgen.er(n, 32768, seed=1)
    check_full(tc, s, d, n)


@pytest.mark.parametrize("scale,seed", [(8, 1), (12, 2), (14, 3), (16, 4)])
def test_rmat_small(tc, scale, seed):
    s, d = graphgen.rmat(scale, seed=seed)
    check_full(tc, s, d, 1 << scale)


def test_rmat_non_power_of_two(tc):
    n = 50000
    s, d = graphgen.rmat(graphgen.scale_for(n), n=n, m=16 * n, seed=8)
    check_full(tc, s, d, n)


def test_rmat_scale20(tc):
    s, d = graphgen.rmat(20, seed=1)
    check_full(tc, s, d, 1 << 20)


def test_rmat_scale24_full_config(tc):
    # the benchmark's graph and launch configuration (RMAT scale 24, edge
    # factor 16, seed 1): the exported CSR and rank map equal the oracle's
    # entry by entry, the total equals the oracle's Eq. 2, the oriented
    # support summed over sampled row ranges equals the oracle's row counts,
    # and full support sums to 3T and equals |Adj(a) & Adj(b)| on sampled
    # edges (uniform ones and the longest rows, whose tables are the largest)
    n = 1 << 24
    s, d = graphgen.rmat(24, seed=1, threads=16)
    g = gpu_graph(tc, s, d, n)
    T = gpu_count(tc, g)
    print("gpu T=%d; oracle preprocessing ..." % T, flush=True)
    U = oracle.preprocess(s, d, n)
    del s, d
    rp, col, perm = tc.tc_graph_export(g)
    torch.cuda.synchronize()
    assert np.array_equal(perm.cpu().numpy(), U.rank)
    rp = rp.cpu().numpy()
    assert np.array_equal(rp, U.row_ptr)
    assert np.array_equal(col.cpu().numpy(), U.col)
    del col
    print("CSR equal; oracle count ...", flush=True)
    assert T == oracle.count(U, threads=16)
    Tg, sup = gpu_support(tc, g, tc.TC_SUPPORT_ORIENTED)
    assert Tg == T
    rng = np.random.default_rng(24)
    for lo in list(rng.integers(0, n - 2048, 24)) + [0, n - 2048]:
        hi = int(lo) + 2048
        want = oracle.count_rows(U, int(lo), hi, threads=16)
        assert int(sup[rp[lo]:rp[hi]].sum(dtype=np.int64)) == want, (lo, hi)
    del sup
    print("oriented support equal; full support ...", flush=True)
    Tf, full = gpu_support(tc, g, tc.TC_SUPPORT_FULL)
    assert Tf == T
    assert int(full.sum(dtype=np.int64)) == 3 * T
    pos = sampled_support.sample_positions(U.row_ptr, seed=24)
    want = sampled_support.sampled_full_support(U.row_ptr, U.col, pos)
    assert np.array_equal(full[pos].astype(np.int64), want)
    del full
    # one rank's block of the 13 x 13 grid at its real shape (Section 5.1):
    # rank (0, 0) and the rank with the most tasks, count and per-shift
    # counts (Eq. 5) against the oracle's
    q = 13
    xm, ym = grid_tasks.max_task_rank(U.row_ptr, U.col, q)
    ps = torch.empty(q, dtype=torch.int64, device="cuda")
    for x, y in ((0, 0), (xm, ym)):
        print("block (%d, %d) of %d x %d" % (x, y, q, q), flush=True)
        cnt, _ = tc.tc_block_count(g, q, x, y, per_shift=ps)
        torch.cuda.synchronize()
        b, shifts = oracle.block_count_one(U, q, x, y)
        assert int(cnt.item()) == b
        assert np.array_equal(ps.cpu().numpy(), shifts)


def test_more_than_2_pow_30_edges(tc):
    # 533,000 disjoint copies of K_64 and one K_300, under a random
    # relabelling: 1,074,572,850 edges (past 2^30, where probes switch to
    # 64-bit addresses; the K_300 rows are heavy enough for the item kernels).
    # Closed forms: T = W+ = probes = copies * C(64, 3) + C(300, 3); a row of
    # out-degree d holds d - 1 tasks, so tasks = copies * C(63, 2) + C(299, 2);
    # edges of a K_k lie in k - 2 triangles
    k, copies, big = 64, 533000, 300
    iu = np.triu_indices(k, 1)
    ib = np.triu_indices(big, 1)
    base = np.arange(copies, dtype=np.int32) * k
    n = k * copies + big
    rng = np.random.default_rng(30)
    relabel = rng.permutation(n).astype(np.int32)
    s = relabel[np.concatenate([(base[:, None] + iu[0].astype(np.int32)[None, :]).ravel(),
                                ib[0].astype(np.int32) + k * copies])]
    d = relabel[np.concatenate([(base[:, None] + iu[1].astype(np.int32)[None, :]).ravel(),
                                ib[1].astype(np.int32) + k * copies])]
    del relabel, base
    m = copies * comb(k, 2) + comb(big, 2)
    T = copies * comb(k, 3) + comb(big, 3)
    assert m > (1 << 30) and len(s) == m
    print("case K64 x %d + K300: m = %d" % (copies, m), flush=True)
    g = tc.tc_preprocess(torch.from_numpy(s).cuda(), torch.from_numpy(d).cuda(), n)
    del s, d
    info = g.info()
    assert info["m"] == m
    assert info["wedges_plus"] == info["probes"] == T
    assert info["tasks"] == copies * comb(k - 1, 2) + comb(big - 1, 2)
    cls = tc.tc_graph_class_stats(g)
    assert sum(v["rows"] for c, v in cls.items() if c.startswith("wg_")) > 0
    assert gpu_count(tc, g) == T
    cnt = torch.empty(1, dtype=torch.int64, device="cuda")
    for mode in (tc.TC_SUPPORT_FULL, tc.TC_SUPPORT_ORIENTED):
        sup, _ = tc.tc_edge_support(g, mode, count=cnt)
        torch.cuda.synchronize()
        assert int(cnt.item()) == T
        total = int(sup.sum(dtype=torch.int64).item())
        if mode == tc.TC_SUPPORT_FULL:
            assert int(sup.min().item()) == k - 2 and int(sup.max().item()) == big - 2
            assert int((sup == big - 2).sum().item()) == comb(big, 2)
            assert total == 3 * T
        else:
            assert total == T
        del sup
    g.free()
    torch.cuda.empty_cache()


def test_edge_cases(tc):
    # empty edge list
    g = gpu_graph(tc, np.zeros(0, np.int32), np.zeros(0, np.int32), 10)
    assert gpu_count(tc, g) == 0
    assert g.info()["m"] == 0
    # one vertex
    g = gpu_graph(tc, np.zeros(0, np.int32), np.zeros(0, np.int32), 1)
    assert gpu_count(tc, g) == 0
    # only self loops and duplicates of one edge
    s = np.array([3, 3, 4, 1, 2, 1], np.int32)
    d = np.array([3, 3, 4, 2, 1, 2], np.int32)
    g = gpu_graph(tc, s, d, 5)
    assert g.info()["m"] == 1 and gpu_count(tc, g) == 0
    # a triangle given 40 times in every orientation
    tri = np.array([[0, 1], [1, 2], [2, 0], [1, 0], [2, 1], [0, 2]] * 40, np.int32)
    g = gpu_graph(tc, tri[:, 0], tri[:, 1], 3)
    assert gpu_count(tc, g) == 1
    _, sup = gpu_support(tc, g, tc.TC_SUPPORT_FULL)
    assert sup.tolist() == [1, 1, 1]


def test_invalid_ids_rejected(tc):
    for s, d, n in [([0, 5], [1, 2], 5), ([-1], [0], 3), ([0], [2 ** 31 - 1], 4)]:
        with pytest.raises(tc.TCError) as e:
            tc.tc_preprocess(dev(s), dev(d), n)
        assert e.value.status == 1


def test_repeatable_and_concurrent_streams(tc):
    s, d = graphgen.rmat(15, seed=21)
    g = gpu_graph(tc, s, d, 1 << 15)
    T = gpu_count(tc, g)
    streams = [torch.cuda.Stream() for _ in range(3)]
    outs = []
    for st in streams:
        with torch.cuda.stream(st):
            outs.append(tc.tc_count(g, stream=st))
    torch.cuda.synchronize()
    assert all(int(o.item()) == T for o in outs)
    for _ in range(3):
        assert gpu_count(tc, g) == T


def test_hbm_fallback_rows(tc):
    # K_n with n - 1 > 8192 out-neighbours on the first rows: their tables do
    # not fit LDS and take the binary-search path; T = C(n, 3) exactly.
    n = 8300
    iu = np.triu_indices(n, 1)
    g = gpu_graph(tc, iu[0].astype(np.int32), iu[1].astype(np.int32), n)
    assert g.info()["max_out_degree"] == n - 1
    assert gpu_count(tc, g) == comb(n, 3)
    T, sup = gpu_support(tc, g, tc.TC_SUPPORT_ORIENTED)
    assert T == comb(n, 3)
    # oriented c(a, b) in K_n with ranks = ids: n - 1 - b for every a < b
    rp, col, _ = tc.tc_graph_export(g)
    col = col.cpu().numpy()
    assert np.array_equal(sup, (n - 1 - col).astype(np.int32))


# ------------------------------------------------ one rank's block (Eq. 5) --

def gpu_block(tc, g, q, x, y):
    ps = torch.full((q,), -1, dtype=torch.int64, device="cuda")
    c, _ = tc.tc_block_count(g, q, x, y, per_shift=ps)
    torch.cuda.synchronize()
    return int(c.item()), ps.cpu().numpy()


def check_blocks(tc, g, U, q):
    B, S = oracle.block_counts(U, q)
    for x in range(q):
        for y in range(q):
            b, s = gpu_block(tc, g, q, x, y)
            assert b == B[x, y], "block (%d, %d) of q=%d" % (x, y, q)
            assert np.array_equal(s, S[x, y]), "shifts of block (%d, %d) of q=%d" % (x, y, q)
    return B


@pytest.mark.parametrize("q", [1, 2, 3, 13])
def test_block_small_graphs(tc, q):
    cases = [sg.complete(12), sg.wheel(30), sg.messy(*sg.random_graph(70, 0.2, 31), seed=3),
             (*graphgen.rmat(10, seed=5), 1 << 10), sg.complete(5)]
    for s, d, n in cases:
        U = oracle.preprocess(s, d, n)
        g = gpu_graph(tc, s, d, n)
        B = check_blocks(tc, g, U, q)
        assert int(B.sum()) == oracle.count(U)


def test_block_rmat16_q13(tc):
    s, d = graphgen.rmat(16, seed=6)
    U = oracle.preprocess(s, d, 1 << 16)
    g = gpu_graph(tc, s, d, 1 << 16)
    check_blocks(tc, g, U, 13)


def test_block_rmat20_q13(tc):
    # sampled ranks against the oracle one by one; the whole grid sums to T
    s, d = graphgen.rmat(20, seed=1)
    U = oracle.preprocess(s, d, 1 << 20)
    g = gpu_graph(tc, s, d, 1 << 20)
    for x, y in [(0, 0), (3, 9), (12, 12), (7, 1)]:
        b1, s1 = oracle.block_count_one(U, 13, x, y)
        b, sh = gpu_block(tc, g, 13, x, y)
        assert b == b1 and np.array_equal(sh, s1), (x, y)
    total = 0
    for x in range(13):
        for y in range(13):
            b, sh = gpu_block(tc, g, 13, x, y)
            assert int(sh.sum()) == b
            total += b
    assert total == gpu_count(tc, g) == oracle.count(U)


def test_block_hbm_fallback_rows(tc):
    # K_n, ranks = ids: rank (x, y) counts i < j < k with i % q == y,
    # j % q == x and shift z taking k % q == (x + y + z) % q; the first hashed
    # rows have more than 4096 entries and take the binary-search path
    n, q = 8300, 2
    iu = np.triu_indices(n, 1)
    g = gpu_graph(tc, iu[0].astype(np.int32), iu[1].astype(np.int32), n)
    v = np.arange(n)
    for x in range(q):
        for y in range(q):
            b, sh = gpu_block(tc, g, q, x, y)
            exp = np.zeros(q, np.int64)
            for z in range(q):
                c = (x + y + z) % q
                below = np.cumsum(v % q == y) - (v % q == y)       # i < j with i % q == y
                above = np.cumsum((v % q == c)[::-1])[::-1] - (v % q == c)  # k > j with k % q == c
                jm = v % q == x
                exp[z] = int((below[jm] * above[jm]).sum())
            assert np.array_equal(sh, exp), (x, y)
            assert b == int(exp.sum())


def test_block_tiny_grid_larger_than_graph(tc):
    # q > n: most ranks own no rows at all
    s, d, n = sg.complete(5)
    U = oracle.preprocess(s, d, n)
    g = gpu_graph(tc, s, d, n)
    check_blocks(tc, g, U, 13)
    b, sh = gpu_block(tc, g, 64, 63, 63)
    assert b == 0 and not sh.any()


def test_sort_wide_lookback_words(tc, monkeypatch):
    # sorts of 2^31 keys or more publish their look-back state in 64-bit
    # words; the environment switch forces that path at small sizes, where
    # the whole preprocessing (five sorts) and the count must still match
    monkeypatch.setenv("TC_SORT_WIDE_WORDS", "1")
    s, d = graphgen.rmat(16, seed=21)
    check_full(tc, s, d, 1 << 16, support=False)
    s, d, n = sg.random_graph(300, 0.05, 77)
    check_full(tc, *sg.messy(s, d, n, seed=3), support=False)


def test_largest_vertex_id_space(tc):
    # n = 2^31 - 1, the largest vertex count the ABI takes: 62-bit sort keys
    # (8 radix passes), 64 KiB digit histograms and n-sized rank, row and
    # work arrays. K6 + a wheel + a friendship graph (with duplicates and
    # self loops) are placed on ids spread over [0, n), the largest id
    # included; the oracle runs on the same graph with its ids compacted in
    # order, which keeps the degree order and therefore U's order, W+ and
    # both support arrays
    n = 2 ** 31 - 1
    s, d, k = sg.disjoint_union(sg.disjoint_union(sg.complete(6), sg.wheel(8)), sg.friendship(3))
    s, d, k = sg.messy(s, d, k, seed=9)
    rng = np.random.default_rng(5)
    ids = np.concatenate([[0], np.sort(rng.choice(n - 2, size=k - 2, replace=False) + 1), [n - 1]])
    ids = ids.astype(np.int64)
    assert len(ids) == k and np.all(np.diff(ids) > 0)
    U = oracle.preprocess(s, d, k)
    T = oracle.count(U)
    assert T == comb(6, 3) + 8 + 3
    g = gpu_graph(tc, ids[s].astype(np.int32), ids[d].astype(np.int32), n)
    info = g.info()
    w = oracle.wedges(U)
    assert info["n"] == n and info["m"] == U.m
    assert (info["wedges_plus"], info["probes"], info["tasks"]) == (w["wedges_plus"], w["probes"], w["tasks"])
    assert gpu_count(tc, g) == T
    for mode in (oracle.MODE_FULL, oracle.MODE_ORIENTED):
        Tr, s_ref = oracle.support(U, mode)
        Tg, sup = gpu_support(tc, g, mode)
        assert Tg == Tr == T
        assert np.array_equal(sup, s_ref), "support mode %d differs" % mode
    g.free()


def test_raw_edge_list_past_2_pow_31(tc):
    # m_raw = 2^31 + 12345 raw pairs (a sort of 2^31 keys or more publishes
    # its look-back state in 64-bit words): seeded random pairs over 40
    # vertices are K40 with self loops and ~1.3 million duplicates of every
    # pair, so T = C(40, 3), m = 780 and every edge has full support 38
    m_raw = 2 ** 31 + 12345
    gen = torch.Generator(device="cuda")
    gen.manual_seed(31)
    src = torch.randint(0, 40, (m_raw,), dtype=torch.int32, device="cuda", generator=gen)
    dst = torch.randint(0, 40, (m_raw,), dtype=torch.int32, device="cuda", generator=gen)
    print("case n=40 m_raw=%d" % m_raw, flush=True)
    g = tc.tc_preprocess(src, dst, 40)
    del src, dst
    info = g.info()
    assert info["m_raw"] == m_raw and info["m"] == comb(40, 2)
    assert gpu_count(tc, g) == comb(40, 3)
    Tg, sup = gpu_support(tc, g, tc.TC_SUPPORT_FULL)
    assert Tg == comb(40, 3) and np.all(sup == 38)
    g.free()
    torch.cuda.empty_cache()
