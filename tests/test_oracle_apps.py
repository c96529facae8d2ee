"""Pins for the oracle's per-vertex counts, clustering coefficients,
trussness and per-rank work (no GPU): closed forms, the diagonal of A^3,
brute force over edge subsets, and identities with the whole-graph counts."""
from itertools import combinations
from math import comb

import numpy as np
import pytest

import graphgen
import oracle
import smallgraphs as sg


def _U(g):
    return oracle.preprocess(*g)


def _edges_orig(U):
    """U's entries as (u, v) original-id pairs with u < v, in U order."""
    inv = np.empty(U.n, np.int64)
    inv[U.rank] = np.arange(U.n)
    out = []
    for a in range(U.n):
        for p in range(U.row_ptr[a], U.row_ptr[a + 1]):
            u, v = int(inv[a]), int(inv[U.col[p]])
            out.append((min(u, v), max(u, v)))
    return out


# --------------------------------------------------- per-vertex triangles ---

def test_vertex_triangles_closed_forms():
    n = 12
    assert set(oracle.vertex_triangles(_U(sg.complete(n))).tolist()) == {comb(n - 1, 2)}
    m = 9
    # wheel: the hub is in all m triangles, a rim vertex in the two on its
    # rim edges (hub, v, v - 1) and (hub, v, v + 1)
    t = oracle.vertex_triangles(_U(sg.wheel(m)))
    assert t[0] == m and set(t[1:].tolist()) == {2}
    k = 7
    t = oracle.vertex_triangles(_U(sg.friendship(k)))
    assert t[0] == k and set(t[1:].tolist()) == {1}
    (s, d, nn), parts = sg.complete_tripartite(2, 3, 5)
    t = oracle.vertex_triangles(oracle.preprocess(s, d, nn))
    sizes = [len(p) for p in parts]
    for i, p in enumerate(parts):
        other = [sizes[j] for j in range(3) if j != i]
        assert set(t[p].tolist()) == {other[0] * other[1]}
    for g in (sg.complete_bipartite(5, 7), sg.star(20), sg.random_tree(50, 1), sg.cycle(9)):
        assert not oracle.vertex_triangles(_U(g)).any()


@pytest.mark.parametrize("n,p,seed", [(60, 0.2, 1), (300, 0.05, 2)])
def test_vertex_triangles_diagonal_of_a_cubed(n, p, seed):
    # t(v) = (A^3)[v, v] / 2: closed walks of length 3 from v, two per triangle
    s, d, _ = sg.random_graph(n, p, seed)
    A = np.zeros((n, n), np.int64)
    A[s, d] = 1
    A[d, s] = 1
    diag = np.diag(A @ A @ A) // 2
    U = oracle.preprocess(s, d, n)
    t = oracle.vertex_triangles(U)
    assert np.array_equal(t, diag)
    assert int(t.sum()) == 3 * oracle.count(U)


def test_vertex_triangles_rmat_sum_and_relabel():
    s, d = graphgen.rmat(11, seed=41)
    n = 1 << 11
    U = oracle.preprocess(s, d, n)
    t = oracle.vertex_triangles(U)
    assert int(t.sum()) == 3 * oracle.count(U)
    perm = np.random.default_rng(3).permutation(n).astype(np.int32)
    t2 = oracle.vertex_triangles(oracle.preprocess(perm[s], perm[d], n))
    assert np.array_equal(t2[perm], t)


# ---------------------------------------------------------- clustering -----

def test_clustering_closed_forms():
    cc, tr, _, _ = oracle.clustering(_U(sg.complete(9)))
    assert np.all(cc == 1.0) and tr == 1.0
    cc, tr, _, W = oracle.clustering(_U(sg.complete_bipartite(4, 6)))
    assert not cc.any() and tr == 0.0 and W == 4 * comb(6, 2) + 6 * comb(4, 2)
    m = 10
    cc, tr, t, W = oracle.clustering(_U(sg.wheel(m)))
    # hub: m triangles among C(m, 2) neighbour pairs; rim vertex: 2 of its
    # C(3, 2) neighbour pairs are adjacent (its two rim neighbours are not)
    assert cc[0] == m / comb(m, 2) and np.all(cc[1:] == 2 / 3)
    assert W == comb(m, 2) + m * comb(3, 2)
    assert tr == 3 * m / W
    # isolated vertices and degree-1 vertices have coefficient 0
    cc, tr, _, _ = oracle.clustering(_U(sg.star(5)))
    assert not cc.any() and tr == 0.0
    cc, tr, _, W = oracle.clustering(oracle.preprocess(np.zeros(0, np.int32), np.zeros(0, np.int32), 4))
    assert not cc.any() and tr == 0.0 and W == 0


def test_transitivity_matches_counts():
    s, d = graphgen.rmat(10, seed=42)
    U = oracle.preprocess(s, d, 1 << 10)
    _, tr, t, W = oracle.clustering(U)
    deg = np.bincount(np.concatenate([U.lo, U.hi]), minlength=U.n).astype(np.int64)
    assert W == int((deg * (deg - 1) // 2).sum())
    assert tr == 3 * oracle.count(U) / W


# ----------------------------------------------------------- trussness -----

def _truss_by_pair(g):
    U = _U(g)
    kmax, tau = oracle.truss(U)
    return kmax, dict(zip(_edges_orig(U), tau.tolist()))


def test_truss_closed_forms():
    for n in (3, 4, 7, 12):
        kmax, t = _truss_by_pair(sg.complete(n))
        assert kmax == n and set(t.values()) == {n}
    kmax, t = _truss_by_pair(sg.cliques_sharing_vertex(6, 9))
    assert kmax == 9
    for (u, v), k in t.items():
        assert k == (6 if max(u, v) < 6 else 9)
    kmax, t = _truss_by_pair(sg.clique_with_pendants(8, 5))
    for (u, v), k in t.items():
        assert k == (8 if max(u, v) < 8 else 2)
    for g, want in ((sg.wheel(12), 3), (sg.friendship(6), 3), (sg.cycle(3), 3), (sg.cycle(8), 2),
                    (sg.random_tree(40, 2), 2), (sg.grid(5, 6), 2), (sg.complete_bipartite(4, 5), 2)):
        kmax, t = _truss_by_pair(g)
        assert set(t.values()) == {want} and kmax == want
    kmax, tau = oracle.truss(oracle.preprocess(np.zeros(0, np.int32), np.zeros(0, np.int32), 3))
    assert kmax == 0 and len(tau) == 0


def _brute_truss(edges, n):
    """Trussness by the definition over all edge subsets: the k-truss is the
    union of all subsets in which every edge lies in >= k - 2 triangles of
    the subset (a union of such subsets is one, so the union is the largest)."""
    m = len(edges)
    best = {e: 2 for e in edges}
    valid_by_k = {}
    for mask in range(1, 1 << m):
        H = [edges[i] for i in range(m) if mask >> i & 1]
        Hs = set(H)
        adj = {}
        for u, v in H:
            adj.setdefault(u, set()).add(v)
            adj.setdefault(v, set()).add(u)
        low = min(len(adj[u] & adj[v]) for u, v in H)
        # H is valid for every k <= low + 2
        for e in Hs:
            if low + 2 > best[e]:
                best[e] = low + 2
    return best


@pytest.mark.parametrize("seed", range(8))
def test_truss_brute_force_over_subsets(seed):
    rng = np.random.default_rng(seed)
    n = 7
    pairs = [p for p in combinations(range(n), 2) if rng.random() < 0.55][:13]
    s = np.array([p[0] for p in pairs], np.int32)
    d = np.array([p[1] for p in pairs], np.int32)
    kmax, t = _truss_by_pair((s, d, n))
    want = _brute_truss(pairs, n)
    assert t == want
    assert kmax == (max(want.values()) if want else 0)


def test_truss_invariants_rmat():
    s, d = graphgen.rmat(11, seed=43)
    n = 1 << 11
    U = oracle.preprocess(s, d, n)
    kmax, tau = oracle.truss(U)
    _, sup = oracle.support(U, oracle.MODE_FULL)
    assert np.all(tau >= 2) and np.all(tau <= sup + 2) and tau.max() == kmax
    edges = _edges_orig(U)
    # each level {tau >= k} is a subgraph whose every edge lies in >= k - 2
    # of its triangles
    for k in range(3, kmax + 1):
        H = [e for e, t in zip(edges, tau) if t >= k]
        adj = {}
        for u, v in H:
            adj.setdefault(u, set()).add(v)
            adj.setdefault(v, set()).add(u)
        assert all(len(adj[u] & adj[v]) >= k - 2 for u, v in H), k
    # relabelling the vertices does not change any edge's trussness
    perm = np.random.default_rng(5).permutation(n).astype(np.int32)
    U2 = oracle.preprocess(perm[s], perm[d], n)
    _, tau2 = oracle.truss(U2)
    t1 = {(int(perm[u]), int(perm[v])): t for (u, v), t in zip(edges, tau.tolist())}
    t1 = {(min(k), max(k)): t for k, t in t1.items()}
    assert dict(zip(_edges_orig(U2), tau2.tolist())) == t1


# ------------------------------------------------------------ rank work ----

@pytest.mark.parametrize("q", [1, 2, 3, 5])
def test_block_work_sums_over_ranks(q):
    s, d = graphgen.rmat(10, seed=44)
    U = oracle.preprocess(s, d, 1 << 10)
    w = oracle.wedges(U)
    tasks = probes = 0
    for x in range(q):
        for y in range(q):
            bw = oracle.block_work(U, q, x, y)
            _, hits = oracle.block_count_one(U, q, x, y)
            tasks += bw["tasks"]
            probes += bw["probes"]
            assert int(bw["shift_probes"].sum()) == bw["probes"]
            # a hit is a probe of its shift, and a shift with a hit intersects
            assert np.all(bw["shift_probes"] >= hits)
            assert np.all(bw["shift_tasks"] <= bw["tasks"])
            assert np.all(bw["shift_tasks"][hits > 0] >= 1)
            if q == 1:
                assert bw["shift_tasks"][0] == bw["tasks"]
    assert tasks == w["tasks"] and probes == w["probes"]


def test_block_work_by_sets():
    # per-shift intersections from Python sets: task (i, j) of rank (x, y)
    # meets shift z when both its probe list (U_i after j) and U_j hold an
    # entry of the class (x + y + z) mod q; and shift z's tasks with a hit
    # are at most that many
    s, d = graphgen.rmat(9, seed=45)
    U = oracle.preprocess(s, d, 1 << 9)
    q = 3
    rows = [U.col[U.row_ptr[a]:U.row_ptr[a + 1]].tolist() for a in range(U.n)]
    for x in range(q):
        for y in range(q):
            st = np.zeros(q, np.int64)
            hit_tasks = np.zeros(q, np.int64)
            for i in range(y, U.n, q):
                for pos, j in enumerate(rows[i]):
                    tail = rows[i][pos + 1:]
                    if j % q != x or not tail or not rows[j]:
                        continue
                    cls_p = {(k - x - y) % q for k in tail}
                    cls_h = {(k - x - y) % q for k in rows[j]}
                    for z in cls_p & cls_h:
                        st[z] += 1
                    for z in {(k - x - y) % q for k in set(tail) & set(rows[j])}:
                        hit_tasks[z] += 1
            bw = oracle.block_work(U, q, x, y)
            assert np.array_equal(bw["shift_tasks"], st)
            assert np.all(hit_tasks <= st)
