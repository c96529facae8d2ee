"""Pins for the CPU oracle (no GPU): closed forms, brute force, trace(A^3)/6,
invariants and the paper's decomposition identities (Eq. 2, Eq. 5)."""
import importlib.util
import os
from math import comb

import numpy as np
import pytest

import graphgen
import oracle
import smallgraphs as sg


def _tri_count(g):
    s, d, n = g
    return oracle.count(oracle.preprocess(s, d, n))


# ---------------------------------------------------------------- count ----

@pytest.mark.parametrize("name,make,expected", sg.CLOSED_FORMS, ids=[c[0] for c in sg.CLOSED_FORMS])
def test_closed_forms(name, make, expected):
    assert _tri_count(make()) == expected


@pytest.mark.parametrize("seed", range(6))
def test_brute_force_random(seed):
    n = 30 + 7 * seed
    g = sg.random_graph(n, 0.25, seed)
    assert _tri_count(g) == oracle.brute_count(*g)


@pytest.mark.parametrize("n,p,seed", [(200, 0.05, 1), (600, 0.02, 2), (1500, 0.01, 3)])
def test_trace_a_cubed(n, p, seed):
    s, d, _ = sg.random_graph(n, p, seed)
    A = np.zeros((n, n), np.int64)
    A[s, d] = 1
    A[d, s] = 1
    t = int(np.trace(A @ A @ A)) // 6
    assert _tri_count((s, d, n)) == t


def test_trace_rmat_small():
    s, d = graphgen.rmat(10, seed=5)
    n = 1 << 10
    A = np.zeros((n, n), np.int64)
    keep = s != d
    A[s[keep], d[keep]] = 1
    A[d[keep], s[keep]] = 1
    assert _tri_count((s, d, n)) == int(np.trace(A @ A @ A)) // 6


@pytest.mark.parametrize("seed", range(3))
def test_invariance_relabel_duplicates_loops(seed):
    g = sg.random_graph(80, 0.12, 10 + seed)
    t = _tri_count(g)
    assert _tri_count(sg.relabel(*g, seed=seed)) == t
    assert _tri_count(sg.messy(*g, seed=seed)) == t


def test_disjoint_union_additive():
    g1 = sg.complete(12)
    g2 = sg.wheel(30)
    g3 = sg.random_graph(50, 0.2, 4)
    u = sg.disjoint_union(sg.disjoint_union(g1, g2), g3)
    assert _tri_count(u) == _tri_count(g1) + _tri_count(g2) + _tri_count(g3)


def test_empty_and_degenerate():
    empty = (np.zeros(0, np.int32), np.zeros(0, np.int32), 5)
    assert _tri_count(empty) == 0
    loops = (np.arange(6, dtype=np.int32), np.arange(6, dtype=np.int32), 6)
    assert _tri_count(loops) == 0
    one = (np.array([0], np.int32), np.array([1], np.int32), 2)
    assert _tri_count(one) == 0
    assert _tri_count((np.zeros(0, np.int32), np.zeros(0, np.int32), 1)) == 0


def test_out_of_range_rejected():
    with pytest.raises(ValueError):
        oracle.preprocess(np.array([0, 5], np.int32), np.array([1, 2], np.int32), 5)
    with pytest.raises(ValueError):
        oracle.preprocess(np.array([-1], np.int32), np.array([1], np.int32), 5)


def test_er_expected_count():
    # G(n, m) with n = 4096, m = 32768: E[T] ~ C(n,3) p^3 with p = m / C(n,2).
    n, m = 4096, 32768
    p = m / comb(n, 2)
    expected = comb(n, 3) * p ** 3
    ts = [_tri_count((*graphgen.er(n, m, seed), n)) for seed in range(1, 9)]
    assert abs(np.mean(ts) - expected) < 0.1 * expected


# ---------------------------------------------------- preprocessing -------

@pytest.mark.parametrize("seed", range(3))
def test_preprocess_structure(seed):
    s, d = graphgen.rmat(11, seed=20 + seed)
    n = 1 << 11
    U = oracle.preprocess(s, d, n)
    E = oracle.brute_edge_set(s, d)
    assert U.m == len(E)
    # degrees of the simple graph
    deg = np.zeros(n, np.int64)
    for e in E:
        for v in e:
            deg[v] += 1
    assert np.array_equal(U.deg, deg)
    # rank is a bijection, degree non-decreasing along rank, ties by id
    assert np.array_equal(np.sort(U.rank), np.arange(n))
    inv = np.empty(n, np.int64)
    inv[U.rank] = np.arange(n)
    key = deg[inv] * (n + 1) + inv
    assert np.all(np.diff(key) > 0)
    # rows strictly ascending, every col above its row, and U holds exactly E
    got = set()
    for a in range(n):
        row = U.col[U.row_ptr[a]:U.row_ptr[a + 1]]
        assert np.all(np.diff(row) > 0)
        assert np.all(row > a)
        for b in row:
            got.add(frozenset((int(inv[a]), int(inv[b]))))
    assert got == E


def test_preprocess_idempotent_on_simple_input():
    s, d = graphgen.rmat(10, seed=3)
    U1 = oracle.preprocess(s, d, 1 << 10)
    U2 = oracle.preprocess(U1.lo, U1.hi, 1 << 10)
    assert np.array_equal(U1.row_ptr, U2.row_ptr)
    assert np.array_equal(U1.col, U2.col)
    assert np.array_equal(U1.rank, U2.rank)


# ----------------------------------------------------------- support ------

def _support_by_pair(U, mode):
    T, s = oracle.support(U, mode)
    inv = np.empty(U.n, np.int64)
    inv[U.rank] = np.arange(U.n)
    out = {}
    for a in range(U.n):
        for p in range(U.row_ptr[a], U.row_ptr[a + 1]):
            out[frozenset((int(inv[a]), int(inv[U.col[p]])))] = int(s[p])
    return T, out


def test_support_complete():
    g = sg.complete(15)
    T, sup = _support_by_pair(oracle.preprocess(*g), oracle.MODE_FULL)
    assert T == comb(15, 3)
    assert set(sup.values()) == {13}


def test_support_wheel_and_friendship():
    m = 11
    T, sup = _support_by_pair(oracle.preprocess(*sg.wheel(m)), oracle.MODE_FULL)
    assert T == m
    for e, v in sup.items():
        assert v == (2 if 0 in e else 1)
    T, sup = _support_by_pair(oracle.preprocess(*sg.friendship(9)), oracle.MODE_FULL)
    assert T == 9 and set(sup.values()) == {1}


def test_support_tripartite():
    (s, d, n), parts = sg.complete_tripartite(3, 4, 6)
    sizes = [len(p) for p in parts]
    where = {v: i for i, p in enumerate(parts) for v in p}
    T, sup = _support_by_pair(oracle.preprocess(s, d, n), oracle.MODE_FULL)
    assert T == 72
    for e, v in sup.items():
        u, w = tuple(e)
        assert v == sizes[3 - where[u] - where[w]]


@pytest.mark.parametrize("seed", range(4))
def test_support_brute(seed):
    g = sg.random_graph(40, 0.3, 100 + seed)
    U = oracle.preprocess(*g)
    T, sup = _support_by_pair(U, oracle.MODE_FULL)
    assert sup == oracle.brute_edge_support(*g)
    Tf, sf = oracle.support(U, oracle.MODE_FULL)
    To, so = oracle.support(U, oracle.MODE_ORIENTED)
    assert Tf == To == oracle.count(U)
    assert int(sf.sum()) == 3 * Tf
    assert int(so.sum()) == To


def test_oriented_support_definition():
    # c(a, b) = |U_a & U_b| (Eq. 1) by Python sets on the oracle's own U
    s, d = graphgen.rmat(9, seed=9)
    U = oracle.preprocess(s, d, 1 << 9)
    _, so = oracle.support(U, oracle.MODE_ORIENTED)
    rows = [set(U.col[U.row_ptr[a]:U.row_ptr[a + 1]].tolist()) for a in range(U.n)]
    for a in range(U.n):
        for p in range(U.row_ptr[a], U.row_ptr[a + 1]):
            assert so[p] == len(rows[a] & rows[U.col[p]])


# ------------------------------------------------------------- wedges -----

def test_wedges_brute():
    s, d = graphgen.rmat(9, seed=11)
    U = oracle.preprocess(s, d, 1 << 9)
    w = oracle.wedges(U)
    wp = probes = tasks = pijk = 0
    for a in range(U.n):
        row = U.col[U.row_ptr[a]:U.row_ptr[a + 1]].tolist()
        for i, b in enumerate(row):
            db = int(U.row_ptr[b + 1] - U.row_ptr[b])
            pijk += db
            for k in row[i + 1:]:
                wp += 1
                if db:
                    probes += 1
            if db and i + 1 < len(row):
                tasks += 1
    assert w == {"wedges_plus": wp, "probes": probes, "probes_ijk": pijk, "tasks": tasks}


# -------------------------------------------------------------- blocks ----

def _brute_blocks(U, q):
    B = np.zeros((q, q), np.int64)
    S = np.zeros((q, q, q), np.int64)
    rows = [set(U.col[U.row_ptr[a]:U.row_ptr[a + 1]].tolist()) for a in range(U.n)]
    for a in range(U.n):
        for b in rows[a]:
            for k in rows[a] & rows[b]:
                x, y = b % q, a % q
                B[x, y] += 1
                S[x, y, (k - x - y) % q] += 1
    return B, S


@pytest.mark.parametrize("q", [1, 2, 3, 13])
def test_block_counts(q):
    s, d = graphgen.rmat(9, seed=12)
    U = oracle.preprocess(s, d, 1 << 9)
    B, S = oracle.block_counts(U, q)
    T = oracle.count(U)
    assert int(B.sum()) == T
    assert np.array_equal(S.sum(axis=2), B)
    Bb, Sb = _brute_blocks(U, q)
    assert np.array_equal(B, Bb)
    assert np.array_equal(S, Sb)
    if q == 1:
        assert B[0, 0] == T
    for x in range(q):
        for y in range(q):
            b1, s1 = oracle.block_count_one(U, q, x, y)
            assert b1 == Bb[x, y]
            assert np.array_equal(s1, Sb[x, y])


# ----------------------------------------------------------- pair common --

def test_pair_common_matches_support():
    s, d = graphgen.rmat(10, seed=13)
    U = oracle.preprocess(s, d, 1 << 10)
    adj = oracle.adjacency(U.lo, U.hi, U.n)
    _, sup = _support_by_pair(U, oracle.MODE_FULL)
    for e, v in list(sup.items())[:500]:
        u, w = tuple(e)
        assert adj.common(u, w) == v


# ------------------------------------------------------------ generator ---

def test_generator_deterministic_and_thread_independent():
    s1, d1 = graphgen.rmat(12, seed=4, threads=1)
    s2, d2 = graphgen.rmat(12, seed=4, threads=4)
    assert np.array_equal(s1, s2) and np.array_equal(d1, d2)
    s3, _ = graphgen.rmat(12, seed=5)
    assert not np.array_equal(s1, s3)
    assert s1.min() >= 0 and s1.max() < 4096


def test_generator_non_power_of_two():
    s, d = graphgen.rmat(graphgen.scale_for(3000), n=3000, m=30000, seed=2)
    assert s.max() < 3000 and d.max() < 3000 and s.min() >= 0


def test_er_simple():
    s, d = graphgen.er(500, 4000, seed=3)
    assert np.all(s != d)
    keys = np.minimum(s, d).astype(np.int64) * 500 + np.maximum(s, d)
    assert len(np.unique(keys)) == 4000


# -------------------------------------------- sampled full support helper --

def test_sampled_full_support_helper():
    # the large-graph spot check of full support equals the oracle's full
    # support on every edge of a small graph and on the sampled ones of a
    # larger graph
    import sampled_support as ss
    for scale, seed in ((10, 3), (14, 7)):
        s, d = graphgen.rmat(scale, seed=seed)
        U = oracle.preprocess(s, d, 1 << scale)
        _, full = oracle.support(U, oracle.MODE_FULL)
        pos = np.arange(U.m) if scale == 10 else ss.sample_positions(U.row_ptr, seed=scale)
        assert np.array_equal(ss.sampled_full_support(U.row_ptr, U.col, pos), full[pos].astype(np.int64))


# ------------------------------------------------------- row-range sums ---

def test_count_rows_partition_sums_to_total():
    # Eq. 2's sum split at random row boundaries adds up to the whole sum
    s, d = graphgen.rmat(12, seed=31)
    U = oracle.preprocess(s, d, 1 << 12)
    T = oracle.count(U)
    rng = np.random.default_rng(31)
    cuts = np.unique(np.concatenate([[0, U.n], rng.integers(0, U.n, 17)]))
    parts = [oracle.count_rows(U, int(a), int(b)) for a, b in zip(cuts[:-1], cuts[1:])]
    assert sum(parts) == T
    assert oracle.count_rows(U, 0, U.n, threads=1) == T


def test_count_rows_single_row_is_eq1_by_sets():
    # one row a: sum over b in U_a of |U_a & U_b| (Eq. 1), by Python sets
    s, d = graphgen.rmat(10, seed=32)
    U = oracle.preprocess(s, d, 1 << 10)
    rows = [set(U.col[U.row_ptr[a]:U.row_ptr[a + 1]].tolist()) for a in range(U.n)]
    for a in range(U.n):
        want = sum(len(rows[a] & rows[b]) for b in rows[a])
        assert oracle.count_rows(U, a, a + 1, threads=1) == want, a


def test_count_rows_empty_and_closed_form():
    n = 30
    U = oracle.preprocess(*sg.complete(n))
    # K_n: every degree is n - 1, so rank = id and U_a = {a + 1, ..., n - 1};
    # row a closes C(n - 1 - a, 2) triangles (its lowest vertex is a)
    for a in range(n):
        assert oracle.count_rows(U, a, a + 1) == comb(n - 1 - a, 2)
        assert oracle.count_rows(U, a, a) == 0
    assert oracle.count_rows(U, 7, 3) == 0


def test_count_rows_equals_oriented_support_row_sums():
    s, d = graphgen.rmat(11, seed=33)
    U = oracle.preprocess(s, d, 1 << 11)
    _, so = oracle.support(U, oracle.MODE_ORIENTED)
    for lo, hi in [(0, 1), (0, 100), (517, 1203), (2000, 2048), (1500, 1501)]:
        assert oracle.count_rows(U, lo, hi) == int(so[U.row_ptr[lo]:U.row_ptr[hi]].sum())


# ---------------------------------------------------------- registry ------

def test_every_oracle_function_is_pinned():
    # every public oracle function names the tests that pin it, and they exist
    import inspect
    import sys
    public = {name for name, f in inspect.getmembers(oracle, inspect.isfunction)
              if not name.startswith("_") and f.__module__ == "oracle"}
    public -= {"build", "max_threads"}
    assert public <= set(oracle.PINS), sorted(public - set(oracle.PINS))
    here = os.path.dirname(os.path.abspath(__file__))
    known = {}
    for fn in ("test_oracle.py", "test_oracle_apps.py", "test_oracle_properties.py"):
        mod = os.path.splitext(fn)[0]
        if mod not in sys.modules:
            spec = importlib.util.spec_from_file_location(mod, os.path.join(here, fn))
            m = importlib.util.module_from_spec(spec)
            spec.loader.exec_module(m)
        else:
            m = sys.modules[mod]
        known.update({k: fn for k in dir(m) if k.startswith("test_")})
    for name, tests in oracle.PINS.items():
        assert tests, name
        for t in tests:
            assert t in known, (name, t)


# ---------------------------------------------- the brute-force layer -----

@pytest.mark.parametrize("name,make,expected", [c for c in sg.CLOSED_FORMS if c[0] not in ("K40", "wheel100")],
                         ids=[c[0] for c in sg.CLOSED_FORMS if c[0] not in ("K40", "wheel100")])
def test_closed_forms_brute(name, make, expected):
    # the pure-Python triple count agrees with the textbook values too
    assert oracle.brute_count(*make()) == expected


def test_support_brute_closed_forms():
    sup = oracle.brute_edge_support(*sg.complete(9))
    assert len(sup) == comb(9, 2) and set(sup.values()) == {7}
    sup = oracle.brute_edge_support(*sg.wheel(8))
    assert all(v == (2 if 0 in e else 1) for e, v in sup.items())
    sup = oracle.brute_edge_support(*sg.complete_bipartite(3, 4))
    assert set(sup.values()) == {0}
