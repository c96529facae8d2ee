/* Driver for the sanitizer test: runs the C oracle (oracle/oracle.c) and the
 * C generators (graphgen/graphgen.c) on small seeded graphs and edge cases,
 * built with AddressSanitizer and UndefinedBehaviorSanitizer, and checks the
 * results against each other and against closed forms (K12: C(12, 3) = 220
 * triangles, trussness 12 on every edge). Exit status 0 when every check
 * holds; a sanitizer report aborts the run. Test infrastructure only. */
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>

int64_t oc_simple_edges(const int32_t* src, const int32_t* dst, int64_t m_raw, int64_t n, int32_t* out_lo,
                        int32_t* out_hi);
int oc_degree_order(const int32_t* lo, const int32_t* hi, int64_t m, int64_t n, int32_t* deg, int32_t* rank);
int oc_build_upper(const int32_t* lo, const int32_t* hi, int64_t m, int64_t n, const int32_t* rank,
                   int64_t* row_ptr, int32_t* col);
int64_t oc_count(const int64_t* row_ptr, const int32_t* col, int64_t n, int nthreads);
int64_t oc_count_rows(const int64_t* row_ptr, const int32_t* col, int64_t a_lo, int64_t a_hi, int nthreads);
int64_t oc_support(const int64_t* row_ptr, const int32_t* col, int64_t n, int mode, int32_t* s);
void oc_wedges(const int64_t* row_ptr, const int32_t* col, int64_t n, int64_t* out);
void oc_block_counts(const int64_t* row_ptr, const int32_t* col, int64_t n, int64_t q, int64_t* B,
                     int64_t* per_shift);
int64_t oc_block_count_one(const int64_t* row_ptr, const int32_t* col, int64_t n, int64_t q, int64_t x,
                           int64_t y, int64_t* per_shift);
int64_t oc_pair_common(const int64_t* adj_ptr, const int32_t* adj, int64_t u, int64_t v);
int oc_build_adjacency(const int32_t* lo, const int32_t* hi, int64_t m, int64_t n, int64_t* adj_ptr,
                       int32_t* adj);
int oc_block_work(const int64_t* row_ptr, const int32_t* col, int64_t n, int64_t q, int64_t x, int64_t y,
                  int64_t* out);
int64_t oc_vertex_triangles(const int64_t* row_ptr, const int32_t* col, int64_t n, int64_t* t);
int64_t oc_truss(const int64_t* row_ptr, const int32_t* col, int64_t n, int32_t* tau);
int gg_rmat(int scale, int64_t n, int64_t m, uint64_t seed, double a, double b, double c, int permute,
            int32_t* src, int32_t* dst, int nthreads);
int gg_er(int64_t n, int64_t m, uint64_t seed, int32_t* src, int32_t* dst);

static int failures = 0;
#define CHECK(cond, ...)                      \
  do {                                        \
    if (!(cond)) {                            \
      fprintf(stderr, "FAIL %s:%d: ", __FILE__, __LINE__); \
      fprintf(stderr, __VA_ARGS__);           \
      fprintf(stderr, "\n");                  \
      ++failures;                             \
    }                                         \
  } while (0)

static void* xmalloc(size_t b) {
  void* p = malloc(b ? b : 1);
  if (!p) {
    fprintf(stderr, "out of host memory\n");
    exit(2);
  }
  return p;
}

/* The whole oracle on one raw pair list; returns T (or -1 if the ids are
 * rejected). want_T < 0: no closed form to compare with. */
static int64_t run(const char* name, const int32_t* src, const int32_t* dst, int64_t m_raw, int64_t n,
                   int64_t want_T, int32_t want_truss) {
  int32_t* lo = xmalloc(sizeof(int32_t) * (size_t)m_raw);
  int32_t* hi = xmalloc(sizeof(int32_t) * (size_t)m_raw);
  const int64_t m = oc_simple_edges(src, dst, m_raw, n, lo, hi);
  if (m < 0) {
    free(lo);
    free(hi);
    return -1;
  }
  int32_t* deg = xmalloc(sizeof(int32_t) * (size_t)n);
  int32_t* rank = xmalloc(sizeof(int32_t) * (size_t)n);
  int64_t* row_ptr = xmalloc(sizeof(int64_t) * (size_t)(n + 1));
  int32_t* col = xmalloc(sizeof(int32_t) * (size_t)m);
  CHECK(oc_degree_order(lo, hi, m, n, deg, rank) == 0, "%s: degree order", name);
  CHECK(oc_build_upper(lo, hi, m, n, rank, row_ptr, col) == 0, "%s: upper", name);
  CHECK(row_ptr[n] == m, "%s: row_ptr[n] %lld != m %lld", name, (long long)row_ptr[n], (long long)m);

  const int64_t T = oc_count(row_ptr, col, n, 1);
  CHECK(oc_count(row_ptr, col, n, 2) == T, "%s: count with 2 threads", name);
  CHECK(oc_count_rows(row_ptr, col, 0, n / 2, 1) + oc_count_rows(row_ptr, col, n / 2, n, 2) == T,
        "%s: row-range sums", name);
  if (want_T >= 0) CHECK(T == want_T, "%s: T %lld, want %lld", name, (long long)T, (long long)want_T);

  int32_t* s = xmalloc(sizeof(int32_t) * (size_t)m);
  int64_t sum = 0;
  CHECK(oc_support(row_ptr, col, n, 0, s) == T, "%s: FULL support T", name);
  for (int64_t p = 0; p < m; ++p) sum += s[p];
  CHECK(sum == 3 * T, "%s: FULL support sums to %lld, want 3T", name, (long long)sum);
  sum = 0;
  CHECK(oc_support(row_ptr, col, n, 1, s) == T, "%s: ORIENTED support T", name);
  for (int64_t p = 0; p < m; ++p) sum += s[p];
  CHECK(sum == T, "%s: ORIENTED support sums to %lld, want T", name, (long long)sum);

  int64_t* t = xmalloc(sizeof(int64_t) * (size_t)n);
  CHECK(oc_vertex_triangles(row_ptr, col, n, t) == T, "%s: vertex triangles T", name);
  sum = 0;
  for (int64_t v = 0; v < n; ++v) sum += t[v];
  CHECK(sum == 3 * T, "%s: vertex triangles sum to %lld, want 3T", name, (long long)sum);

  int64_t w[4];
  oc_wedges(row_ptr, col, n, w);
  CHECK(w[0] >= T, "%s: wedges below T", name);

  const int64_t q = 3;
  int64_t B[9], shifts[27], one[3], work[2 + 2 * 3];
  oc_block_counts(row_ptr, col, n, q, B, shifts);
  sum = 0;
  for (int c = 0; c < 9; ++c) {
    int64_t bs = 0;
    for (int z = 0; z < 3; ++z) bs += shifts[c * 3 + z];
    CHECK(bs == B[c], "%s: block %d shifts", name, c);
    sum += B[c];
  }
  CHECK(sum == T, "%s: blocks sum to %lld, want T", name, (long long)sum);
  CHECK(oc_block_count_one(row_ptr, col, n, q, 1, 2, one) == B[1 * 3 + 2], "%s: one block", name);
  CHECK(oc_block_work(row_ptr, col, n, q, 1, 2, work) == 0, "%s: block work", name);

  int64_t* adj_ptr = xmalloc(sizeof(int64_t) * (size_t)(n + 1));
  int32_t* adj = xmalloc(sizeof(int32_t) * (size_t)(2 * m));
  CHECK(oc_build_adjacency(lo, hi, m, n, adj_ptr, adj) == 0, "%s: adjacency", name);
  sum = 0;
  for (int64_t e = 0; e < m; ++e) sum += oc_pair_common(adj_ptr, adj, lo[e], hi[e]);
  CHECK(sum == 3 * T, "%s: common neighbours of the edges sum to %lld, want 3T", name, (long long)sum);

  int32_t* tau = xmalloc(sizeof(int32_t) * (size_t)m);
  const int64_t kmax = oc_truss(row_ptr, col, n, tau);
  CHECK(kmax >= 0 && (m == 0 || kmax >= 2), "%s: truss %lld", name, (long long)kmax);
  if (want_truss > 0) {
    CHECK(kmax == want_truss, "%s: kmax %lld, want %d", name, (long long)kmax, want_truss);
    for (int64_t p = 0; p < m; ++p) CHECK(tau[p] == want_truss, "%s: tau[%lld]", name, (long long)p);
  }
  printf("%s: n %lld, m_raw %lld, m %lld, T %lld, kmax %lld\n", name, (long long)n, (long long)m_raw,
         (long long)m, (long long)T, (long long)kmax);
  free(lo), free(hi), free(deg), free(rank), free(row_ptr), free(col), free(s), free(t), free(adj_ptr),
      free(adj), free(tau);
  return T;
}

int main(void) {
  /* K12, every pair in both orientations, plus self loops */
  {
    int32_t src[12 * 12], dst[12 * 12];
    int64_t k = 0;
    for (int u = 0; u < 12; ++u)
      for (int v = 0; v < 12; ++v) src[k] = u, dst[k] = v, ++k;
    run("K12", src, dst, k, 12, 220, 12);
  }
  /* RMAT scale 11 (edge factor 16) and ER */
  {
    const int64_t n = 2048, m = 16 * 2048;
    int32_t* src = xmalloc(sizeof(int32_t) * (size_t)m);
    int32_t* dst = xmalloc(sizeof(int32_t) * (size_t)m);
    CHECK(gg_rmat(11, n, m, 5, 0.57, 0.19, 0.19, 1, src, dst, 2) == 0, "gg_rmat");
    run("rmat11", src, dst, m, n, -1, 0);
    CHECK(gg_er(700, 5000, 3, src, dst) == 0, "gg_er");
    run("er700", src, dst, 5000, 700, -1, 0);
    free(src);
    free(dst);
  }
  /* edge cases: no pairs, only self loops, an id out of range */
  {
    int32_t src[4] = {0, 1, 2, 3}, dst[4] = {0, 1, 2, 3};
    CHECK(run("empty", src, dst, 0, 5, 0, 0) == 0, "empty graph");
    CHECK(run("loops", src, dst, 4, 5, 0, 0) == 0, "self loops only");
    int32_t bad_dst[4] = {1, 2, 3, 9};
    CHECK(run("bad_id", src, bad_dst, 4, 5, -1, 0) == -1, "id outside [0, n) accepted");
  }
  if (failures) {
    fprintf(stderr, "%d checks failed\n", failures);
    return 1;
  }
  printf("all checks passed\n");
  return 0;
}
