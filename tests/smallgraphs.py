"""Small named graphs with known triangle counts and per-edge supports.

Each constructor returns (src, dst, n) as int32 numpy arrays plus n. The
closed forms live beside them so the CPU oracle and the GPU path are checked
against the same textbook values.
"""
from __future__ import annotations

import itertools
from math import comb

import numpy as np


def _arr(pairs, n):
    if not pairs:
        return np.zeros(0, np.int32), np.zeros(0, np.int32), n
    p = np.asarray(pairs, dtype=np.int32)
    return p[:, 0].copy(), p[:, 1].copy(), n


def complete(n):
    """K_n: C(n, 3) triangles; every edge lies in n - 2 of them."""
    return _arr(list(itertools.combinations(range(n), 2)), n)


def cycle(n):
    """C_n: 1 triangle for n = 3, else 0."""
    return _arr([(i, (i + 1) % n) for i in range(n)], n)


def wheel(m):
    """Hub 0 joined to a rim cycle 1..m (m >= 4): m triangles; rim edges have
    support 1, spokes support 2."""
    rim = [(1 + i, 1 + (i + 1) % m) for i in range(m)]
    spokes = [(0, 1 + i) for i in range(m)]
    return _arr(rim + spokes, m + 1)


def friendship(k):
    """F_k: k triangles sharing vertex 0; every edge has support 1."""
    pairs = []
    for i in range(k):
        a, b = 1 + 2 * i, 2 + 2 * i
        pairs += [(0, a), (0, b), (a, b)]
    return _arr(pairs, 2 * k + 1)


def complete_tripartite(a, b, c):
    """K_{a,b,c}: a*b*c triangles; an edge between two parts has support equal
    to the size of the third part."""
    parts = [list(range(0, a)), list(range(a, a + b)), list(range(a + b, a + b + c))]
    pairs = []
    for p, q in ((0, 1), (0, 2), (1, 2)):
        pairs += [(u, v) for u in parts[p] for v in parts[q]]
    return _arr(pairs, a + b + c), parts


def complete_bipartite(a, b):
    """K_{a,b}: bipartite, 0 triangles."""
    return _arr([(u, a + v) for u in range(a) for v in range(b)], a + b)


def star(n):
    """Star with n leaves: 0 triangles."""
    return _arr([(0, i) for i in range(1, n + 1)], n + 1)


def random_tree(n, seed=0):
    """Random recursive tree: 0 triangles."""
    rng = np.random.default_rng(seed)
    return _arr([(i, int(rng.integers(0, i))) for i in range(1, n)], n)


def grid(r, c):
    """r x c grid graph: bipartite, 0 triangles."""
    pairs = []
    for i in range(r):
        for j in range(c):
            v = i * c + j
            if j + 1 < c:
                pairs.append((v, v + 1))
            if i + 1 < r:
                pairs.append((v, v + c))
    return _arr(pairs, r * c)


def random_graph(n, p, seed):
    """G(n, p) by coin flips (numpy), for brute-force comparisons."""
    rng = np.random.default_rng(seed)
    pairs = [(i, j) for i in range(n) for j in range(i + 1, n) if rng.random() < p]
    return _arr(pairs, n)


def messy(src, dst, n, seed=0, dup=0.5, loops=5):
    """The same graph with random orientation, duplicates and self loops added."""
    rng = np.random.default_rng(seed)
    m = len(src)
    flip = rng.random(m) < 0.5
    s = np.where(flip, dst, src)
    d = np.where(flip, src, dst)
    k = int(dup * m)
    idx = rng.integers(0, max(m, 1), size=k) if m else np.zeros(0, np.int64)
    s2 = np.concatenate([s, d[idx], rng.integers(0, n, size=loops)]).astype(np.int32)
    d2 = np.concatenate([d, s[idx], np.zeros(loops, np.int64)]).astype(np.int32)
    d2[len(s) + k:] = s2[len(s) + k:]
    perm = rng.permutation(len(s2))
    return s2[perm].copy(), d2[perm].copy(), n


def relabel(src, dst, n, seed=0):
    rng = np.random.default_rng(seed)
    p = rng.permutation(n).astype(np.int32)
    return p[src], p[dst], n


def disjoint_union(g1, g2):
    s1, d1, n1 = g1
    s2, d2, n2 = g2
    return (np.concatenate([s1, s2 + n1]).astype(np.int32),
            np.concatenate([d1, d2 + n1]).astype(np.int32), n1 + n2)


CLOSED_FORMS = [
    ("K3", lambda: complete(3), 1),
    ("K4", lambda: complete(4), 4),
    ("K10", lambda: complete(10), comb(10, 3)),
    ("K40", lambda: complete(40), comb(40, 3)),
    ("C3", lambda: cycle(3), 1),
    ("C4", lambda: cycle(4), 0),
    ("C17", lambda: cycle(17), 0),
    ("wheel4", lambda: wheel(4), 4),
    ("wheel9", lambda: wheel(9), 9),
    ("wheel100", lambda: wheel(100), 100),
    ("friendship1", lambda: friendship(1), 1),
    ("friendship25", lambda: friendship(25), 25),
    ("K2,3,4", lambda: complete_tripartite(2, 3, 4)[0], 24),
    ("K5,6,7", lambda: complete_tripartite(5, 6, 7)[0], 210),
    ("K7,9", lambda: complete_bipartite(7, 9), 0),
    ("star50", lambda: star(50), 0),
    ("tree200", lambda: random_tree(200, 3), 0),
    ("grid9x11", lambda: grid(9, 11), 0),
]


def cliques_sharing_vertex(p, q):
    """K_p and K_q with one common vertex (0): trussness p inside the first
    clique, q inside the second."""
    a = list(range(p))
    b = [0] + list(range(p, p + q - 1))
    pairs = list(itertools.combinations(a, 2)) + list(itertools.combinations(b, 2))
    return _arr(pairs, p + q - 1)


def clique_with_pendants(p, k):
    """K_p plus k pendant vertices hung on vertex 0: trussness p on the
    clique's edges, 2 on the pendant edges."""
    pairs = list(itertools.combinations(range(p), 2)) + [(0, p + i) for i in range(k)]
    return _arr(pairs, p + k)
