/*
 * oracle.c - plain, slow, obviously correct CPU reference for exact triangle
 * counting as defined by Tom and Karypis, "A 2D Parallel Triangle Counting
 * Algorithm for Distributed-Memory Architectures" (ICPP 2019).
 *
 * TEST INFRASTRUCTURE ONLY. Nothing in the library's product path may link,
 * load or call this file; only the tests, the package smoke check and the
 * benchmark's CPU-baseline leg use it. It shares no code with the GPU path:
 * the only common module is the seeded input generator.
 *
 * Every function follows the paper's definitions in the paper's order, using
 * qsort (a library sort) as its only primitive:
 *
 *   oc_simple_edges   Section 2 (simple undirected graph) and Section 6.1 (inputs
 *                     converted to undirected simple graphs): the set of
 *                     unordered pairs {u, v}, u != v.
 *   oc_degree_order   Section 3.1 / Section 5.3 ("Reorder vertices based on
 *                     non-decreasing degree"): rank = position after sorting by
 *                     degree; ties broken by original id (the paper leaves the
 *                     tie order open; any total order gives the same count).
 *   oc_build_upper    Section 5.3 (the split into upper and lower triangular
 *                     parts): each edge goes to the row of its lower-ranked
 *                     endpoint, rows sorted ascending (Section 5.2's pruning of
 *                     needless intersections relies on sorted rows).
 *   oc_count          Eq. 1 and Eq. 2: c(i,j) = |Adj>(i) & Adj>(j)| for every
 *                     nonzero (i,j) of U, T = sum c(i,j). The intersection uses
 *                     the list-based method of Section 3.1 (a joint traversal of
 *                     two sorted lists), deliberately unlike the GPU path's
 *                     map-based one.
 *   oc_support        per-edge values: ORIENTED = c(i,j) of Eq. 1 (sums to T);
 *                     FULL = number of triangles containing the edge (sums to
 *                     3T), obtained by crediting every triangle i<j<k found by
 *                     Eq. 1 to (i,j), (i,k) and (j,k).
 *   oc_wedges         work counts: W+ = sum_a C(|U_a|, 2), the probes of the
 *                     <j,i,k> map-based scheme of Section 3.1, and the probes left
 *                     after skipping intersections whose hashed list is empty;
 *                     plus the probes of the <i,j,k> scheme for comparison.
 *   oc_block_counts   Section 5.1, Eq. 4 and Eq. 5 under the C[L] task
 *                     convention: for a q x q cyclic grid, block (x, y) owns the
 *                     tasks (i, j) with j % q == x and i % q == y; shift z of
 *                     Eq. 5 contributes the triangles whose closing vertex k has
 *                     k % q == (x + y + z) % q.
 *   oc_block_count_one  the same for one rank (x, y) only.
 *   oc_count_rows     Eq. 2's sum restricted to the rows a of U in [a_lo, a_hi).
 *   oc_block_work     the work of one rank (x, y) of the same decomposition:
 *                     its tasks and probes under the <j,i,k> rule, the probes
 *                     whose closing vertex falls in each shift's residue class,
 *                     and per shift the intersections a rank would perform
 *                     (both the probe list and the hashed list hold an entry
 *                     of that residue class).
 *   oc_pair_common    |Adj(u) & Adj(v)| for one pair by joint traversal of the
 *                     two full sorted adjacency lists (the definition of a
 *                     triangle in Section 2), for spot checks on large graphs.
 *   oc_vertex_triangles  per-vertex triangle counts t(v) (Section 1 names local
 *                     clustering coefficients as a use of triangle counts):
 *                     each triangle a<b<k found by Eq. 1 adds one to each of
 *                     its three vertices.
 *   oc_truss          trussness of every edge (Section 1 names the k-truss as
 *                     a use of per-edge triangle counts): the k-truss is the
 *                     largest subgraph whose every edge lies in at least k - 2
 *                     of its triangles; computed level by level from that
 *                     definition, recounting every edge's triangles inside the
 *                     remaining subgraph after each round of deletions.
 *
 * Integer widths: counts are int64 (Table "datasets" has counts near 5e11);
 * per-edge values int32.
 *
 * Errors: functions that allocate return a negative value (-2) when malloc
 * fails; the Python layer turns it into MemoryError.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#ifdef _OPENMP
#include <omp.h>
#endif

static int cmp_u64(const void* x, const void* y) {
  uint64_t a = *(const uint64_t*)x, b = *(const uint64_t*)y;
  return (a > b) - (a < b);
}

/* ---------------------------------------------------------------------------
 * Simple undirected graph (Section 2; Section 6.1).
 * Input: m_raw directed pairs with ids in [0, n). Output: the distinct
 * unordered pairs {u, v}, u != v, written as (lo, hi) with lo < hi, sorted by
 * (lo, hi). Returns the number of pairs, or -1 if an id is out of range.
 * ------------------------------------------------------------------------- */
int64_t oc_simple_edges(const int32_t* src, const int32_t* dst, int64_t m_raw, int64_t n,
                        int32_t* out_lo, int32_t* out_hi) {
  uint64_t* key = (uint64_t*)malloc((size_t)(m_raw > 0 ? m_raw : 1) * sizeof(uint64_t));
  if (!key) return -2;
  int64_t m = 0;
  for (int64_t e = 0; e < m_raw; ++e) {
    int64_t u = src[e], v = dst[e];
    if (u < 0 || u >= n || v < 0 || v >= n) {
      free(key);
      return -1;
    }
    if (u == v) continue; /* no self loops in a simple graph */
    uint64_t lo = (uint64_t)(u < v ? u : v), hi = (uint64_t)(u < v ? v : u);
    key[m++] = (lo << 32) | hi;
  }
  qsort(key, (size_t)m, sizeof(uint64_t), cmp_u64);
  int64_t k = 0;
  for (int64_t e = 0; e < m; ++e) {
    if (e > 0 && key[e] == key[e - 1]) continue; /* a set: drop repeats */
    out_lo[k] = (int32_t)(key[e] >> 32);
    out_hi[k] = (int32_t)(key[e] & 0xFFFFFFFFu);
    ++k;
  }
  free(key);
  return k;
}

/* ---------------------------------------------------------------------------
 * Degree order (Section 3.1; Section 5.3).
 * deg[v] = |Adj(v)| in the simple graph. rank[v] = position of v after
 * sorting all vertices by (deg, v) ascending.
 * ------------------------------------------------------------------------- */
int oc_degree_order(const int32_t* lo, const int32_t* hi, int64_t m, int64_t n, int32_t* deg,
                    int32_t* rank) {
  uint64_t* key = (uint64_t*)malloc((size_t)(n > 0 ? n : 1) * sizeof(uint64_t));
  if (!key) return -2;
  for (int64_t v = 0; v < n; ++v) deg[v] = 0;
  for (int64_t e = 0; e < m; ++e) {
    deg[lo[e]]++;
    deg[hi[e]]++;
  }
  for (int64_t v = 0; v < n; ++v) key[v] = ((uint64_t)(uint32_t)deg[v] << 32) | (uint64_t)v;
  qsort(key, (size_t)n, sizeof(uint64_t), cmp_u64);
  for (int64_t r = 0; r < n; ++r) rank[key[r] & 0xFFFFFFFFu] = (int32_t)r;
  free(key);
  return 0;
}

/* ---------------------------------------------------------------------------
 * Upper triangular CSR U in rank space (Section 5.3).
 * Row a holds Adj>(a) = {rank(w) : {v, w} in E, rank(v) = a, rank(w) > a},
 * sorted ascending. row_ptr has n + 1 entries.
 * ------------------------------------------------------------------------- */
int oc_build_upper(const int32_t* lo, const int32_t* hi, int64_t m, int64_t n, const int32_t* rank,
                   int64_t* row_ptr, int32_t* col) {
  uint64_t* key = (uint64_t*)malloc((size_t)(m > 0 ? m : 1) * sizeof(uint64_t));
  if (!key) return -2;
  for (int64_t e = 0; e < m; ++e) {
    uint64_t ru = (uint64_t)rank[lo[e]], rv = (uint64_t)rank[hi[e]];
    uint64_t a = ru < rv ? ru : rv, b = ru < rv ? rv : ru;
    key[e] = (a << 32) | b;
  }
  qsort(key, (size_t)m, sizeof(uint64_t), cmp_u64);
  for (int64_t a = 0; a <= n; ++a) row_ptr[a] = 0;
  for (int64_t e = 0; e < m; ++e) row_ptr[(key[e] >> 32) + 1]++;
  for (int64_t a = 0; a < n; ++a) row_ptr[a + 1] += row_ptr[a];
  for (int64_t e = 0; e < m; ++e) col[e] = (int32_t)(key[e] & 0xFFFFFFFFu);
  free(key);
  return 0;
}

/* |U_a & U_b| restricted to k > b, by joint traversal of the two sorted lists
 * (list-based intersection, Section 3.1). Since every entry of U_b exceeds b,
 * the restriction k > b of Eq. 1 holds automatically. */
static int64_t merge_common(const int32_t* x, int64_t nx, const int32_t* y, int64_t ny) {
  int64_t i = 0, j = 0, c = 0;
  while (i < nx && j < ny) {
    if (x[i] < y[j]) ++i;
    else if (x[i] > y[j]) ++j;
    else { ++c; ++i; ++j; }
  }
  return c;
}

/* ---------------------------------------------------------------------------
 * Eq. 1 and Eq. 2: T = sum over nonzeros (a, b) of U of |U_a & U_b|.
 * ------------------------------------------------------------------------- */
int64_t oc_count(const int64_t* row_ptr, const int32_t* col, int64_t n, int nthreads) {
  int64_t total = 0;
  if (nthreads < 1) nthreads = 1;
#pragma omp parallel for schedule(dynamic, 256) reduction(+ : total) num_threads(nthreads)
  for (int64_t a = 0; a < n; ++a) {
    for (int64_t p = row_ptr[a]; p < row_ptr[a + 1]; ++p) {
      int64_t b = col[p];
      total += merge_common(col + row_ptr[a], row_ptr[a + 1] - row_ptr[a], col + row_ptr[b],
                            row_ptr[b + 1] - row_ptr[b]);
    }
  }
  return total;
}

/* Eq. 2's sum restricted to the rows a in [a_lo, a_hi): the triangles whose
 * lowest-ranked vertex lies in that range (a bounded sample of the sum, used
 * to time the oracle and to check per-row sums of oriented support). */
int64_t oc_count_rows(const int64_t* row_ptr, const int32_t* col, int64_t a_lo, int64_t a_hi,
                      int nthreads) {
  int64_t total = 0;
  if (nthreads < 1) nthreads = 1;
#pragma omp parallel for schedule(dynamic, 256) reduction(+ : total) num_threads(nthreads)
  for (int64_t a = a_lo; a < a_hi; ++a) {
    for (int64_t p = row_ptr[a]; p < row_ptr[a + 1]; ++p) {
      int64_t b = col[p];
      total += merge_common(col + row_ptr[a], row_ptr[a + 1] - row_ptr[a], col + row_ptr[b],
                            row_ptr[b + 1] - row_ptr[b]);
    }
  }
  return total;
}

/* ---------------------------------------------------------------------------
 * Per-edge values, indexed by U position (row-major, rows sorted).
 * mode 1 (ORIENTED): s[p] = c(a, b) of Eq. 1 for the nonzero p = (a, b).
 * mode 0 (FULL): s[p] = number of triangles containing the edge p.
 * Returns T.
 * ------------------------------------------------------------------------- */
int64_t oc_support(const int64_t* row_ptr, const int32_t* col, int64_t n, int mode, int32_t* s) {
  int64_t m = row_ptr[n];
  for (int64_t p = 0; p < m; ++p) s[p] = 0;
  int64_t total = 0;
  for (int64_t a = 0; a < n; ++a) {
    for (int64_t p = row_ptr[a]; p < row_ptr[a + 1]; ++p) {
      int64_t b = col[p];
      /* joint traversal of U_a and U_b, remembering positions of common k */
      int64_t i = row_ptr[a], ie = row_ptr[a + 1], j = row_ptr[b], je = row_ptr[b + 1];
      while (i < ie && j < je) {
        if (col[i] < col[j]) ++i;
        else if (col[i] > col[j]) ++j;
        else {
          /* triangle a < b < k with edges p=(a,b), i=(a,k), j=(b,k) */
          ++total;
          s[p]++;
          if (mode == 0) {
            s[i]++;
            s[j]++;
          }
          ++i;
          ++j;
        }
      }
    }
  }
  return total;
}

/* ---------------------------------------------------------------------------
 * Work counts.
 * out[0] = W+ = sum_a C(|U_a|, 2): probes of the <j,i,k> scheme when, for each
 *          nonzero (a, b), the entries of U_a after b are looked up in U_b.
 * out[1] = the same sum restricted to nonzeros (a, b) with U_b non-empty
 *          (an intersection with an empty list needs no probe).
 * out[2] = sum over nonzeros (a, b) of |U_b|: the probes of the <i,j,k> scheme
 *          when U_a is hashed and all of U_b is looked up.
 * out[3] = number of nonzeros (a, b) with at least one probe in out[1]'s rule
 *          (the tasks).
 * ------------------------------------------------------------------------- */
void oc_wedges(const int64_t* row_ptr, const int32_t* col, int64_t n, int64_t* out) {
  int64_t w = 0, wk = 0, pijk = 0, tasks = 0;
  for (int64_t a = 0; a < n; ++a) {
    int64_t d = row_ptr[a + 1] - row_ptr[a];
    w += d * (d - 1) / 2;
    for (int64_t p = row_ptr[a]; p < row_ptr[a + 1]; ++p) {
      int64_t b = col[p];
      int64_t db = row_ptr[b + 1] - row_ptr[b];
      int64_t after = row_ptr[a + 1] - p - 1;
      pijk += db;
      if (db > 0 && after > 0) {
        wk += after;
        tasks += 1;
      }
    }
  }
  out[0] = w;
  out[1] = wk;
  out[2] = pijk;
  out[3] = tasks;
}

/* ---------------------------------------------------------------------------
 * 2D cyclic decomposition (Section 5.1, Eq. 4, Eq. 5), C[L] convention.
 * Rank (x, y) of a q x q grid owns the tasks (i, j) of U with j % q == x and
 * i % q == y. B[x*q + y] = triangles i<j<k counted by those tasks;
 * per_shift[(x*q + y)*q + z] = the part whose closing k satisfies
 * k % q == (x + y + z) % q. Each entry of B is the sum of its q shifts.
 * ------------------------------------------------------------------------- */
void oc_block_counts(const int64_t* row_ptr, const int32_t* col, int64_t n, int64_t q, int64_t* B,
                     int64_t* per_shift) {
  for (int64_t c = 0; c < q * q; ++c) B[c] = 0;
  for (int64_t c = 0; c < q * q * q; ++c) per_shift[c] = 0;
  for (int64_t i = 0; i < n; ++i) {
    for (int64_t p = row_ptr[i]; p < row_ptr[i + 1]; ++p) {
      int64_t j = col[p];
      int64_t x = j % q, y = i % q;
      int64_t a = row_ptr[i], ae = row_ptr[i + 1], b = row_ptr[j], be = row_ptr[j + 1];
      while (a < ae && b < be) {
        if (col[a] < col[b]) ++a;
        else if (col[a] > col[b]) ++b;
        else {
          int64_t k = col[a];
          int64_t z = ((k % q) - x - y) % q;
          if (z < 0) z += q;
          B[x * q + y]++;
          per_shift[(x * q + y) * q + z]++;
          ++a;
          ++b;
        }
      }
    }
  }
}

/* One rank's share of the same decomposition: rank (x, y) alone, for graphs
 * where all q * q blocks would take too long. Visits only the rows i with
 * i % q == y and their entries j with j % q == x; per_shift[z] as above.
 * Returns B[x][y]. */
int64_t oc_block_count_one(const int64_t* row_ptr, const int32_t* col, int64_t n, int64_t q, int64_t x,
                           int64_t y, int64_t* per_shift) {
  int64_t total = 0;
  for (int64_t z = 0; z < q; ++z) per_shift[z] = 0;
  for (int64_t i = y; i < n; i += q) {
    for (int64_t p = row_ptr[i]; p < row_ptr[i + 1]; ++p) {
      int64_t j = col[p];
      if (j % q != x) continue;
      int64_t a = row_ptr[i], ae = row_ptr[i + 1], b = row_ptr[j], be = row_ptr[j + 1];
      while (a < ae && b < be) {
        if (col[a] < col[b]) ++a;
        else if (col[a] > col[b]) ++b;
        else {
          int64_t z = ((col[a] % q) - x - y) % q;
          if (z < 0) z += q;
          per_shift[z]++;
          total++;
          ++a;
          ++b;
        }
      }
    }
  }
  return total;
}

/* ---------------------------------------------------------------------------
 * |Adj(u) & Adj(v)| for one pair, from the full symmetric adjacency
 * (adj_ptr, adj) with sorted lists: the number of triangles on edge {u, v}.
 * ------------------------------------------------------------------------- */
int64_t oc_pair_common(const int64_t* adj_ptr, const int32_t* adj, int64_t u, int64_t v) {
  return merge_common(adj + adj_ptr[u], adj_ptr[u + 1] - adj_ptr[u], adj + adj_ptr[v],
                      adj_ptr[v + 1] - adj_ptr[v]);
}

/* Full symmetric adjacency of the simple graph, lists sorted (for
 * oc_pair_common). adj has 2m entries, adj_ptr n + 1. */
int oc_build_adjacency(const int32_t* lo, const int32_t* hi, int64_t m, int64_t n, int64_t* adj_ptr,
                       int32_t* adj) {
  uint64_t* key = (uint64_t*)malloc((size_t)(2 * m > 0 ? 2 * m : 1) * sizeof(uint64_t));
  if (!key) return -2;
  for (int64_t e = 0; e < m; ++e) {
    key[2 * e] = ((uint64_t)(uint32_t)lo[e] << 32) | (uint32_t)hi[e];
    key[2 * e + 1] = ((uint64_t)(uint32_t)hi[e] << 32) | (uint32_t)lo[e];
  }
  qsort(key, (size_t)(2 * m), sizeof(uint64_t), cmp_u64);
  for (int64_t v = 0; v <= n; ++v) adj_ptr[v] = 0;
  for (int64_t e = 0; e < 2 * m; ++e) adj_ptr[(key[e] >> 32) + 1]++;
  for (int64_t v = 0; v < n; ++v) adj_ptr[v + 1] += adj_ptr[v];
  for (int64_t e = 0; e < 2 * m; ++e) adj[e] = (int32_t)(key[e] & 0xFFFFFFFFu);
  free(key);
  return 0;
}

/* ---------------------------------------------------------------------------
 * Work of one rank (x, y) of the q x q cyclic decomposition (Section 5.1,
 * C[L] convention; Section 7.2 reports its per-shift balance and how the
 * number of intersections grows with the number of ranks).
 * The rank's tasks are the nonzeros (i, j) of U with j % q == x, i % q == y
 * whose row i has entries after j and whose row j is not empty (the <j,i,k>
 * rule of Section 3.1 with empty hashed lists skipped); each such task probes
 * the entries k of U_i after j.
 * out[0]        tasks
 * out[1]        probes
 * out[2 + z]    probes whose k has k % q == (x + y + z) % q (shift z of Eq. 5)
 * out[2 + q + z] tasks that shift z would intersect: both the task's probe
 *               list and U_j hold an entry of that residue class.
 * Returns 0, or -2 if malloc fails.
 * ------------------------------------------------------------------------- */
int oc_block_work(const int64_t* row_ptr, const int32_t* col, int64_t n, int64_t q, int64_t x, int64_t y,
                  int64_t* out) {
  char* in_probe = (char*)malloc((size_t)q);
  char* in_hash = (char*)malloc((size_t)q);
  if (!in_probe || !in_hash) {
    free(in_probe);
    free(in_hash);
    return -2;
  }
  for (int64_t c = 0; c < 2 + 2 * q; ++c) out[c] = 0;
  for (int64_t i = y; i < n; i += q) {
    for (int64_t p = row_ptr[i]; p < row_ptr[i + 1]; ++p) {
      int64_t j = col[p];
      if (j % q != x) continue;
      int64_t after = row_ptr[i + 1] - p - 1;
      int64_t dj = row_ptr[j + 1] - row_ptr[j];
      if (after <= 0 || dj <= 0) continue;
      out[0] += 1;
      out[1] += after;
      memset(in_probe, 0, (size_t)q);
      memset(in_hash, 0, (size_t)q);
      for (int64_t a = p + 1; a < row_ptr[i + 1]; ++a) {
        int64_t z = ((col[a] % q) - x - y) % q;
        if (z < 0) z += q;
        out[2 + z] += 1;
        in_probe[z] = 1;
      }
      for (int64_t b = row_ptr[j]; b < row_ptr[j + 1]; ++b) {
        int64_t z = ((col[b] % q) - x - y) % q;
        if (z < 0) z += q;
        in_hash[z] = 1;
      }
      for (int64_t z = 0; z < q; ++z) out[2 + q + z] += in_probe[z] && in_hash[z];
    }
  }
  free(in_probe);
  free(in_hash);
  return 0;
}

/* ---------------------------------------------------------------------------
 * Per-vertex triangle counts in rank space: t[v] = number of triangles that
 * contain v. Every triangle a < b < k is found once, by Eq. 1's intersection
 * for the nonzero (a, b), and adds one to t[a], t[b] and t[k].
 * Returns T.
 * ------------------------------------------------------------------------- */
int64_t oc_vertex_triangles(const int64_t* row_ptr, const int32_t* col, int64_t n, int64_t* t) {
  int64_t total = 0;
  for (int64_t v = 0; v < n; ++v) t[v] = 0;
  for (int64_t a = 0; a < n; ++a) {
    for (int64_t p = row_ptr[a]; p < row_ptr[a + 1]; ++p) {
      int64_t b = col[p];
      int64_t i = row_ptr[a], ie = row_ptr[a + 1], j = row_ptr[b], je = row_ptr[b + 1];
      while (i < ie && j < je) {
        if (col[i] < col[j]) ++i;
        else if (col[i] > col[j]) ++j;
        else {
          t[a]++;
          t[b]++;
          t[col[i]]++;
          ++total;
          ++i;
          ++j;
        }
      }
    }
  }
  return total;
}

/* ---------------------------------------------------------------------------
 * Trussness of every edge, indexed by U position. The k-truss (k >= 2) is the
 * largest subgraph in which every edge lies in at least k - 2 triangles of
 * that subgraph; the trussness of an edge is the largest k whose k-truss
 * holds it (every edge is in the 2-truss).
 * Level by level from the definition: H starts as the whole graph (the
 * 2-truss). For k = 3, 4, ...: count every edge's triangles inside H, delete
 * from H every edge with fewer than k - 2 of them (their trussness is k - 1),
 * and count again, until a round deletes nothing; H is then the k-truss.
 * (Deleting only lowers the counts of other edges, and an edge of any
 * subgraph that meets the k-truss condition keeps at least k - 2 triangles in
 * every H containing that subgraph, so no such edge is ever deleted.)
 * Triangles inside H are found by the joint traversal of Eq. 1 over the
 * entries of U still in H. Returns the largest trussness (0 for a graph
 * without edges), or -2 if malloc fails.
 * ------------------------------------------------------------------------- */
int64_t oc_truss(const int64_t* row_ptr, const int32_t* col, int64_t n, int32_t* tau) {
  const int64_t m = row_ptr[n];
  char* alive = (char*)malloc((size_t)(m > 0 ? m : 1));
  int64_t* sup = (int64_t*)malloc((size_t)(m > 0 ? m : 1) * sizeof(int64_t));
  if (!alive || !sup) {
    free(alive);
    free(sup);
    return -2;
  }
  for (int64_t p = 0; p < m; ++p) {
    alive[p] = 1;
    tau[p] = 0;
  }
  int64_t left = m, kmax = 0;
  for (int64_t k = 3; left > 0; ++k) {
    for (;;) {
      /* triangles of every edge of H */
      for (int64_t p = 0; p < m; ++p) sup[p] = 0;
      for (int64_t a = 0; a < n; ++a) {
        for (int64_t p = row_ptr[a]; p < row_ptr[a + 1]; ++p) {
          if (!alive[p]) continue;
          int64_t b = col[p];
          int64_t i = row_ptr[a], ie = row_ptr[a + 1], j = row_ptr[b], je = row_ptr[b + 1];
          while (i < ie && j < je) {
            if (col[i] < col[j]) ++i;
            else if (col[i] > col[j]) ++j;
            else {
              if (alive[i] && alive[j]) { /* edges (a, k) and (b, k) also in H */
                sup[p]++;
                sup[i]++;
                sup[j]++;
              }
              ++i;
              ++j;
            }
          }
        }
      }
      int64_t deleted = 0;
      for (int64_t p = 0; p < m; ++p) {
        if (alive[p] && sup[p] < k - 2) {
          alive[p] = 0;
          tau[p] = (int32_t)(k - 1);
          ++deleted;
        }
      }
      left -= deleted;
      if (deleted) kmax = k - 1;
      if (deleted == 0 || left == 0) break;
    }
  }
  free(alive);
  free(sup);
  return kmax;
}

int oc_max_threads(void) {
#ifdef _OPENMP
  return omp_get_max_threads();
#else
  return 1;
#endif
}
