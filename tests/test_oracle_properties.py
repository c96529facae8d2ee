"""Property tests of the CPU oracle on random small graphs (hypothesis).

Each generated case is a raw edge list over n <= 24 vertices with duplicates,
both orientations and self loops, as the preprocessing of Sections 2 and 6.1
must accept. The oracle is checked against the plain definitions and
invariants rather than against itself:
- T equals the number of vertex triples whose three pairs are edges;
- T is invariant under relabelling, added duplicates and self loops, and is
  additive over disjoint unions;
- full support of every edge is its number of triangles (brute force), and
  sums to 3T;
- oriented support of U's edge (a, b) is Eq. 1, the number of k > b adjacent
  to both (rank space), and sums to T;
- the q x q blocks of Section 5.1 sum to T, their shifts (Eq. 5) to each
  block, and one rank computed alone equals its entry of the grid;
- per-vertex triangle counts equal the number of triangles through each
  vertex (brute force over triples);
- trussness of every edge equals its definition over all edge subsets
  (graphs of at most 11 edges).
"""
import numpy as np
import pytest
from hypothesis import HealthCheck, given, settings
from hypothesis import strategies as st

import oracle

SETTINGS = settings(max_examples=60, deadline=None, derandomize=True, database=None,
                    suppress_health_check=[HealthCheck.too_slow])


@st.composite
def raw_graphs(draw, max_n=24, max_pairs=140):
    n = draw(st.integers(min_value=1, max_value=max_n))
    pairs = draw(st.lists(st.tuples(st.integers(0, n - 1), st.integers(0, n - 1)), max_size=max_pairs))
    src = np.array([p[0] for p in pairs], dtype=np.int32)
    dst = np.array([p[1] for p in pairs], dtype=np.int32)
    return src, dst, n


def original_edges(U):
    """U's entries as original-id edges, in U order."""
    inv = np.empty(U.n, np.int64)
    inv[U.rank] = np.arange(U.n)
    out = []
    for a in range(U.n):
        for p in range(U.row_ptr[a], U.row_ptr[a + 1]):
            out.append(frozenset((int(inv[a]), int(inv[U.col[p]]))))
    return out


@SETTINGS
@given(raw_graphs())
def test_count_is_the_triple_definition(g):
    src, dst, n = g
    U = oracle.preprocess(src, dst, n)
    assert oracle.count(U) == oracle.brute_count(src, dst, n)
    assert U.m == len(oracle.brute_edge_set(src, dst))


@SETTINGS
@given(raw_graphs(), st.randoms(use_true_random=False))
def test_relabel_duplicate_and_loop_invariance(g, rnd):
    src, dst, n = g
    T = oracle.count(oracle.preprocess(src, dst, n))
    perm = list(range(n))
    rnd.shuffle(perm)
    perm = np.array(perm, dtype=np.int32)
    assert oracle.count(oracle.preprocess(perm[src], perm[dst], n)) == T
    # every pair again, reversed, plus a loop on each vertex
    loops = np.arange(n, dtype=np.int32)
    src2 = np.concatenate([src, dst, loops])
    dst2 = np.concatenate([dst, src, loops])
    assert oracle.count(oracle.preprocess(src2, dst2, n)) == T


@SETTINGS
@given(raw_graphs(max_n=16, max_pairs=80), raw_graphs(max_n=16, max_pairs=80))
def test_disjoint_union_is_additive(g1, g2):
    s1, d1, n1 = g1
    s2, d2, n2 = g2
    T1 = oracle.count(oracle.preprocess(s1, d1, n1))
    T2 = oracle.count(oracle.preprocess(s2, d2, n2))
    src = np.concatenate([s1, s2 + n1]).astype(np.int32)
    dst = np.concatenate([d1, d2 + n1]).astype(np.int32)
    assert oracle.count(oracle.preprocess(src, dst, n1 + n2)) == T1 + T2


@SETTINGS
@given(raw_graphs())
def test_full_support_is_triangles_per_edge(g):
    src, dst, n = g
    U = oracle.preprocess(src, dst, n)
    T, s = oracle.support(U, oracle.MODE_FULL)
    ref = oracle.brute_edge_support(src, dst, n)
    edges = original_edges(U)
    assert [int(v) for v in s] == [ref[e] for e in edges]
    assert int(s.sum()) == 3 * T


@SETTINGS
@given(raw_graphs())
def test_oriented_support_is_eq1(g):
    src, dst, n = g
    U = oracle.preprocess(src, dst, n)
    T, s = oracle.support(U, oracle.MODE_ORIENTED)
    # adjacency in rank space from the simple edge set
    adj = [set() for _ in range(n)]
    for e in oracle.brute_edge_set(src, dst):
        u, v = (int(U.rank[x]) for x in e)
        adj[u].add(v)
        adj[v].add(u)
    expect = []
    for a in range(n):
        for p in range(U.row_ptr[a], U.row_ptr[a + 1]):
            b = int(U.col[p])
            assert b > a  # upper triangular in rank order
            expect.append(sum(1 for k in adj[a] & adj[b] if k > b))
    assert [int(v) for v in s] == expect
    assert int(s.sum()) == T == oracle.brute_count(src, dst, n)


@SETTINGS
@given(raw_graphs(), st.sampled_from([1, 2, 3, 5]), st.data())
def test_blocks_and_shifts_decompose_T(g, q, data):
    src, dst, n = g
    U = oracle.preprocess(src, dst, n)
    T = oracle.count(U)
    B, S = oracle.block_counts(U, q)
    assert int(B.sum()) == T
    assert np.array_equal(S.sum(axis=2), B)
    x = data.draw(st.integers(0, q - 1))
    y = data.draw(st.integers(0, q - 1))
    b, s = oracle.block_count_one(U, q, x, y)
    assert b == int(B[x, y])
    assert np.array_equal(s, S[x, y])


@SETTINGS
@given(raw_graphs(max_n=18, max_pairs=90))
def test_vertex_triangles_are_triangles_through_each_vertex(g):
    src, dst, n = g
    E = oracle.brute_edge_set(src, dst)
    t = np.zeros(n, np.int64)
    for i in range(n):
        for j in range(i + 1, n):
            for k in range(j + 1, n):
                if {frozenset((i, j)), frozenset((i, k)), frozenset((j, k))} <= E:
                    t[[i, j, k]] += 1
    assert np.array_equal(oracle.vertex_triangles(oracle.preprocess(src, dst, n)), t)


@settings(max_examples=40, deadline=None, derandomize=True, database=None,
          suppress_health_check=[HealthCheck.too_slow])
@given(raw_graphs(max_n=7, max_pairs=14))
def test_truss_is_the_subset_definition(g):
    src, dst, n = g
    E = sorted(tuple(sorted(e)) for e in oracle.brute_edge_set(src, dst))
    if len(E) > 11:
        E = E[:11]
        src = np.array([e[0] for e in E], np.int32)
        dst = np.array([e[1] for e in E], np.int32)
    want = {e: 2 for e in E}
    for mask in range(1, 1 << len(E)):
        H = [E[i] for i in range(len(E)) if mask >> i & 1]
        adj = {}
        for u, v in H:
            adj.setdefault(u, set()).add(v)
            adj.setdefault(v, set()).add(u)
        low = min(len(adj[u] & adj[v]) for u, v in H)
        for e in H:
            want[e] = max(want[e], low + 2)
    U = oracle.preprocess(src, dst, n)
    _, tau = oracle.truss(U)
    edges = [tuple(sorted(e)) for e in original_edges(U)]
    assert dict(zip(edges, tau.tolist())) == want


if __name__ == "__main__":
    pytest.main([__file__, "-q"])
