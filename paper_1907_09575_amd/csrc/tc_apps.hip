// tc_apps.hip - the uses of exact triangle counts that the paper's
// introduction (Section 1) names, built on the per-edge support of Eq. 1's
// intersections: per-vertex triangle counts, local clustering coefficients
// and transitivity, and the k-truss decomposition.
//
// Both need every vertex's full neighbourhood, not only U: the lower part
// L_v = {a : v in U_a} (U's column lists) is built by a stable radix sort of
// U's entries by column, each keeping the U position of its edge. In rank
// space every entry of L_v is below v and every entry of U_v above it, so
// N(v) in ascending order is L_v followed by U_v, with no merge.
//
// Per-vertex counts: every triangle through v has two edges at v, so
// t(v) = (sum of the full support of v's edges) / 2.
//
// k-truss: the k-truss is the largest subgraph whose every edge lies in at
// least k - 2 of its triangles; an edge's trussness is the largest k whose
// k-truss holds it. Peeling, level by level: starting from the full support,
// every round removes the alive edges whose current support is below k - 2
// (trussness k - 1) and takes the triangles they close out of the support of
// their other two edges; when a round removes nothing, k rises to the next
// level that removes something. A triangle that loses several edges in one
// round is taken out once, by its removed edge of smallest id; a triangle
// with an edge removed in an earlier round is already gone.
#include <algorithm>

#include "tc_prims.h"

namespace tc {

namespace {

constexpr int kAT = 256;
inline unsigned grid_threads(int64_t n) { return (unsigned)std::max<int64_t>(1, div_up(n, kAT)); }
inline unsigned grid_waves(int64_t n) { return wave_grid(n); }  // (one wave per item, grid-stride)

// ---- lower adjacency ---------------------------------------------------------

struct Lower {
  DevBuf ptr;   // int64 [n + 1]: L_v = [ptr[v], ptr[v + 1])
  DevBuf nbr;   // int32 [m]: a of every entry, ascending within a column
  DevBuf eid;   // int32 [m]: U position of the edge (a, v)
  DevBuf erow;  // uint32 [m]: row of every U entry
};

__global__ void k_lower_keys(const int32_t* __restrict__ col, const uint32_t* __restrict__ erow, int64_t m,
                             uint32_t* __restrict__ key, uint64_t* __restrict__ val) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= m) return;
  key[i] = (uint32_t)col[i];
  val[i] = (uint64_t)erow[i] | ((uint64_t)i << 32);
}

__global__ void k_lower_split(const uint64_t* __restrict__ val, int64_t m, int32_t* __restrict__ nbr,
                              int32_t* __restrict__ eid) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= m) return;
  const uint64_t v = val[i];
  nbr[i] = (int32_t)(uint32_t)v;
  eid[i] = (int32_t)(v >> 32);
}

__global__ void k_fill_i64v(int64_t* p, int64_t n, int64_t v) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = v;
}

void build_lower(Lower& L, const Graph& g, hipStream_t st) {
  const int64_t n = g.n, m = g.m;
  L.ptr.alloc(sizeof(int64_t) * (size_t)(n + 1));
  L.nbr.alloc(sizeof(int32_t) * (size_t)std::max<int64_t>(m, 1));
  L.eid.alloc(sizeof(int32_t) * (size_t)std::max<int64_t>(m, 1));
  L.erow.alloc(sizeof(uint32_t) * (size_t)std::max<int64_t>(m, 1));
  if (m == 0) {
    TC_LAUNCH("fill_i64", k_fill_i64v, dim3(grid_threads(n + 1)), dim3(kAT), 0, st, L.ptr.as<int64_t>(), n + 1,
              (int64_t)0);
    return;
  }
  TC_LAUNCH("entry_rows", k_entry_rows, dim3(grid_waves(n)), dim3(kAT), 0, st, g.row_ptr, n,
            L.erow.as<uint32_t>());
  DevBuf ka(sizeof(uint32_t) * (size_t)m), kb(sizeof(uint32_t) * (size_t)m);
  DevBuf va(sizeof(uint64_t) * (size_t)m), vb(sizeof(uint64_t) * (size_t)m);
  TC_LAUNCH("lower_keys", k_lower_keys, dim3(grid_threads(m)), dim3(kAT), 0, st, g.col, L.erow.as<uint32_t>(), m,
            ka.as<uint32_t>(), va.as<uint64_t>());
  // stable by column: within a column the rows keep U's ascending order
  const bool alt = radix_sort<uint32_t, uint64_t>(ka.as<uint32_t>(), kb.as<uint32_t>(), va.as<uint64_t>(),
                                                  vb.as<uint64_t>(), m, 0, g.sbits, st, "lower");
  const uint32_t* keys = alt ? kb.as<uint32_t>() : ka.as<uint32_t>();
  const uint64_t* vals = alt ? vb.as<uint64_t>() : va.as<uint64_t>();
  TC_LAUNCH("bounds", (k_bounds<uint32_t>), dim3(grid_threads(n + 1)), dim3(kAT), 0, st, keys, m, 0, n,
            L.ptr.as<int64_t>());
  TC_LAUNCH("lower_split", k_lower_split, dim3(grid_threads(m)), dim3(kAT), 0, st, vals, m, L.nbr.as<int32_t>(),
            L.eid.as<int32_t>());
  TC_HIP(hipGetLastError());
}

// ---- per-vertex counts and clustering ------------------------------------------

// t(v) in rank space: half the full support summed over v's edges (one wave
// per vertex: U_v is read contiguously, L_v gathers support by edge id).
__global__ __launch_bounds__(256) void k_vertex_tri(const int64_t* __restrict__ row_ptr,
                                                    const int64_t* __restrict__ lptr,
                                                    const int32_t* __restrict__ leid,
                                                    const int32_t* __restrict__ sup, int64_t n,
                                                    int64_t* __restrict__ t_rank) {
  const int lane = lane_id();
  const int64_t stride = (int64_t)gridDim.x * (blockDim.x / 64);
  for (int64_t v = (int64_t)blockIdx.x * (blockDim.x / 64) + (threadIdx.x >> 6); v < n; v += stride) {
    uint64_t s = 0;
    for (int64_t p = row_ptr[v] + lane; p < row_ptr[v + 1]; p += 64) s += (uint32_t)sup[p];
    for (int64_t i = lptr[v] + lane; i < lptr[v + 1]; i += 64) s += (uint32_t)sup[leid[i]];
    s = wave_sum(s);
    if (lane == 0) t_rank[v] = (int64_t)(s / 2);
  }
}

// Per original vertex u (rank r = perm[u]): t, the local clustering
// coefficient t / C(d, 2) (0 if d < 2; one correctly rounded division of two
// exact integers) and the sums of t (= 3T) and of C(d, 2) over all vertices.
__global__ __launch_bounds__(256) void k_vertex_out(const int32_t* __restrict__ perm, int64_t n,
                                                    const int64_t* __restrict__ t_rank,
                                                    const int64_t* __restrict__ row_ptr,
                                                    const int64_t* __restrict__ lptr, int64_t* __restrict__ t_orig,
                                                    double* __restrict__ cc, unsigned long long* __restrict__ sums) {
  __shared__ unsigned long long s_t[4], s_w[4];
  const int64_t u = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  uint64_t t = 0, pairs = 0;
  if (u < n) {
    const int64_t r = perm[u];
    t = (uint64_t)t_rank[r];
    const uint64_t d = (uint64_t)((row_ptr[r + 1] - row_ptr[r]) + (lptr[r + 1] - lptr[r]));
    pairs = d * (d - (d > 0)) / 2;
    if (t_orig) t_orig[u] = (int64_t)t;
    if (cc) cc[u] = pairs ? (double)t / (double)pairs : 0.0;
  }
  if (!sums) return;
  const unsigned long long wt = wave_sum((unsigned long long)t), ww = wave_sum((unsigned long long)pairs);
  if (lane_id() == 0) {
    s_t[threadIdx.x >> 6] = wt;
    s_w[threadIdx.x >> 6] = ww;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    const unsigned long long a = s_t[0] + s_t[1] + s_t[2] + s_t[3], b = s_w[0] + s_w[1] + s_w[2] + s_w[3];
    if (a) atomicAdd(&sums[0], a);
    if (b) atomicAdd(&sums[1], b);
  }
}

__global__ void k_zero_u64x2(unsigned long long* p) {
  if (threadIdx.x < 2) p[threadIdx.x] = 0;
}

void vertex_counts(const Graph& g, int64_t* d_tri, double* d_cc, int64_t* d_sums, hipStream_t st) {
  require_plain(g, "per-vertex triangle counts");
  TempStream temps(st);
  const int64_t n = g.n;
  auto* sums = reinterpret_cast<unsigned long long*>(d_sums);
  if (sums) TC_LAUNCH("zero_sums", k_zero_u64x2, dim3(1), dim3(64), 0, st, sums);
  DevBuf sup(sizeof(int32_t) * (size_t)std::max<int64_t>(g.m, 1));
  launch_count(graph_view(g), MODE_SUPPORT_FULL, nullptr, sup.as<int32_t>(), nullptr, st);
  Lower L;
  build_lower(L, g, st);
  DevBuf t_rank(sizeof(int64_t) * (size_t)n);
  TC_LAUNCH("vertex_tri", k_vertex_tri, dim3(grid_waves(n)), dim3(kAT), 0, st, g.row_ptr, L.ptr.as<int64_t>(),
            L.eid.as<int32_t>(), sup.as<int32_t>(), n, t_rank.as<int64_t>());
  TC_LAUNCH("vertex_out", k_vertex_out, dim3(grid_threads(n)), dim3(kAT), 0, st, g.perm, n, t_rank.as<int64_t>(),
            g.row_ptr, L.ptr.as<int64_t>(), d_tri, d_cc, sums);
  TC_HIP(hipGetLastError());
  note_use(g, st);
  check_sorts(st);
}

// ---- k-truss ---------------------------------------------------------------------

constexpr int32_t kAlive = 0x7FFFFFFF;  // state of an edge not yet removed (else: its round)

// Alive edges whose support is below lim (the round's removals).
struct FrontierPred {
  const int32_t* state;
  const int32_t* sup;
  int32_t lim;
  int32_t* out;
  struct Item {};
  __device__ bool operator()(int64_t i, Item&) const { return state[i] == kAlive && sup[i] < lim; }
  __device__ void emit(int64_t i, const Item&, uint32_t pos) const { out[pos] = (int32_t)i; }
};

__global__ void k_fill_i32(int32_t* p, int64_t n, int32_t v) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = v;
}

// Smallest support among alive edges (for the next level with removals).
__global__ __launch_bounds__(256) void k_min_alive(const int32_t* __restrict__ state, const int32_t* __restrict__ sup,
                                                   int64_t m, int* __restrict__ out) {
  int v = kAlive;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < m; i += (int64_t)gridDim.x * blockDim.x)
    if (state[i] == kAlive) v = min(v, sup[i]);
#pragma unroll
  for (int d = 32; d >= 1; d >>= 1) v = min(v, __shfl_xor(v, d, 64));
  if (lane_id() == 0 && v != kAlive) atomicMin(out, v);
}

__global__ void k_truss_mark(const int32_t* __restrict__ F, int64_t nF, int32_t round, int32_t tau_val,
                             int32_t* __restrict__ state, int32_t* __restrict__ tau) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= nF) return;
  const int32_t e = F[i];
  state[e] = round;
  tau[e] = tau_val;
}

// N(v) = L_v followed by U_v (ascending), with the U position of each edge.
struct FullAdj {
  const int64_t* row_ptr;
  const int32_t* col;
  const int64_t* lptr;
  const int32_t* lnbr;
  const int32_t* leid;
};

// First position in the sorted list a[0, len) holding w, or -1.
__device__ __forceinline__ int64_t find_sorted(const int32_t* __restrict__ a, int64_t len, int32_t w) {
  int64_t lo = 0, hi = len;
  while (lo < hi) {
    const int64_t mid = (lo + hi) >> 1;
    if (a[mid] < w) lo = mid + 1;
    else hi = mid;
  }
  return (lo < len && a[lo] == w) ? lo : -1;
}

// One wave per removed edge e = (a, b) of this round: the lanes walk the
// neighbourhood of the endpoint of smaller degree and look every w up in the
// other's (binary search in its L or U part); each triangle (e, e1, e2) still
// whole before this round, and whose removed edge of smallest id is e, takes
// one from the support of each of e1, e2 still alive.
__device__ void truss_peel_one(const FullAdj& A, const uint32_t* __restrict__ erow,
                               const int32_t* __restrict__ F, int64_t f, int32_t round,
                               const int32_t* __restrict__ state, int32_t* __restrict__ sup) {
  const int lane = lane_id();
  const int32_t e = F[f];
  const int32_t a = (int32_t)erow[e], b = A.col[e];
  const int64_t la = A.lptr[a + 1] - A.lptr[a], ua = A.row_ptr[a + 1] - A.row_ptr[a];
  const int64_t lb = A.lptr[b + 1] - A.lptr[b], ub = A.row_ptr[b + 1] - A.row_ptr[b];
  const bool a_small = la + ua <= lb + ub;
  const int32_t x = a_small ? a : b, y = a_small ? b : a;
  const int64_t lx = a_small ? la : lb, dx = a_small ? la + ua : lb + ub;
  const int64_t ly = a_small ? lb : la, uy = a_small ? ub : ua;
  for (int64_t i = lane; i < dx; i += 64) {
    const bool in_l = i < lx;
    const int32_t w = in_l ? A.lnbr[A.lptr[x] + i] : A.col[A.row_ptr[x] + (i - lx)];
    if (w == y) continue;
    int32_t e2;
    if (w < y) {
      const int64_t j = find_sorted(A.lnbr + A.lptr[y], ly, w);
      if (j < 0) continue;
      e2 = A.leid[A.lptr[y] + j];
    } else {
      const int64_t j = find_sorted(A.col + A.row_ptr[y], uy, w);
      if (j < 0) continue;
      e2 = (int32_t)(A.row_ptr[y] + j);
    }
    const int32_t e1 = in_l ? A.leid[A.lptr[x] + i] : (int32_t)(A.row_ptr[x] + (i - lx));
    const int32_t s1 = state[e1], s2 = state[e2];
    if (s1 < round || s2 < round) continue;  // an edge went in an earlier round
    int32_t owner = e;
    if (s1 == round && e1 < owner) owner = e1;
    if (s2 == round && e2 < owner) owner = e2;
    if (owner != e) continue;
    if (s1 == kAlive) atomicSub(&sup[e1], 1);
    if (s2 == kAlive) atomicSub(&sup[e2], 1);
  }
}

__global__ __launch_bounds__(256) void k_truss_peel(FullAdj A, const uint32_t* __restrict__ erow,
                                                    const int32_t* __restrict__ F, int64_t nF, int32_t round,
                                                    const int32_t* __restrict__ state, int32_t* __restrict__ sup) {
  const int64_t stride = (int64_t)gridDim.x * (blockDim.x / 64);
  for (int64_t f = (int64_t)blockIdx.x * (blockDim.x / 64) + (threadIdx.x >> 6); f < nF; f += stride)
    truss_peel_one(A, erow, F, f, round, state, sup);
}

template <class T>
T read_scalar(const T* d, hipStream_t st) {
  T h{};
  TC_HIP(hipMemcpyAsync(&h, d, sizeof(T), hipMemcpyDeviceToHost, st));
  TC_HIP(hipStreamSynchronize(st));
  return h;
}

int32_t truss(const Graph& g, int32_t* d_tau, hipStream_t st) {
  require_plain(g, "tc_truss");
  TempStream temps(st);
  const int64_t m = g.m;
  if (m == 0) return 0;
  TC_REQUIRE(m < ((int64_t)1 << 31), TC_EOVERFLOW, "tc_truss: 2^31 or more edges");
  DevBuf sup(sizeof(int32_t) * (size_t)m), state(sizeof(int32_t) * (size_t)m), F(sizeof(int32_t) * (size_t)m);
  DevBuf dmin(sizeof(int));
  launch_count(graph_view(g), MODE_SUPPORT_FULL, nullptr, sup.as<int32_t>(), nullptr, st);
  Lower L;
  build_lower(L, g, st);
  TC_LAUNCH("truss_fill", k_fill_i32, dim3(grid_threads(m)), dim3(kAT), 0, st, state.as<int32_t>(), m, kAlive);
  TC_LAUNCH("truss_fill", k_fill_i32, dim3(grid_threads(m)), dim3(kAT), 0, st, d_tau, m, 0);
  check_sorts(st);
  const FullAdj A{g.row_ptr, g.col, L.ptr.as<int64_t>(), L.nbr.as<int32_t>(), L.eid.as<int32_t>()};
  int64_t alive = m;
  int64_t k = 3;
  int32_t round = 0, kmax = 0;
  while (alive > 0) {
    FrontierPred fp{state.as<int32_t>(), sup.as<int32_t>(), (int32_t)(k - 2), F.as<int32_t>()};
    const int64_t nF = compact("truss_frontier", m, fp, [](int64_t, FrontierPred&) {}, st);
    if (nF == 0) {
      // no alive edge is below k - 2: the next level that removes one
      const int big = kAlive;
      TC_HIP(hipMemcpyAsync(dmin.p, &big, sizeof(int), hipMemcpyHostToDevice, st));
      TC_LAUNCH("truss_min", k_min_alive, dim3((unsigned)std::min<int64_t>(1024, grid_threads(m))), dim3(kAT), 0,
                st, state.as<int32_t>(), sup.as<int32_t>(), m, dmin.as<int>());
      const int mn = read_scalar(dmin.as<int>(), st);
      TC_REQUIRE(mn != kAlive && (int64_t)mn + 3 > k, TC_EDEVICE, "tc_truss: no level removes an edge");
      k = (int64_t)mn + 3;
      continue;
    }
    TC_REQUIRE(round < kAlive - 1, TC_EOVERFLOW, "tc_truss: too many rounds");
    TC_LAUNCH("truss_mark", k_truss_mark, dim3(grid_threads(nF)), dim3(kAT), 0, st, F.as<int32_t>(), nF, round,
              (int32_t)(k - 1), state.as<int32_t>(), d_tau);
    TC_LAUNCH("truss_peel", k_truss_peel, dim3(grid_waves(nF)), dim3(kAT), 0, st, A, L.erow.as<uint32_t>(),
              F.as<int32_t>(), nF, round, state.as<int32_t>(), sup.as<int32_t>());
    TC_HIP(hipGetLastError());
    kmax = (int32_t)(k - 1);
    alive -= nF;
    ++round;
  }
  TC_HIP(hipStreamSynchronize(st));
  note_use(g, st);
  return kmax;
}

template <class F>
tc_status guarded(const char* where, F&& f) {
  try {
    f();
    set_last_error("");
    return TC_OK;
  } catch (const Error& e) {
    set_last_error(e.what());
    return e.status;
  } catch (const std::bad_alloc&) {
    set_last_error(std::string(where) + ": host allocation failed");
    return TC_ENOMEM;
  } catch (const std::exception& e) {
    set_last_error(e.what());
    return TC_EDEVICE;
  }
}

}  // namespace

}  // namespace tc

extern "C" {

tc_status tc_vertex_triangles(const tc_graph* gh, int64_t* d_tri, void* stream) {
  return tc::guarded("tc_vertex_triangles", [&] {
    TC_REQUIRE(gh != nullptr && d_tri != nullptr, TC_EINVAL, "tc_vertex_triangles: null argument");
    tc::vertex_counts(*tc::G(gh), d_tri, nullptr, nullptr, static_cast<hipStream_t>(stream));
  });
}

tc_status tc_clustering(const tc_graph* gh, double* d_cc, int64_t* d_tri, int64_t* d_sums, void* stream) {
  return tc::guarded("tc_clustering", [&] {
    TC_REQUIRE(gh != nullptr, TC_EINVAL, "tc_clustering: null graph");
    TC_REQUIRE(d_cc || d_tri || d_sums, TC_EINVAL, "tc_clustering: no output array");
    tc::vertex_counts(*tc::G(gh), d_tri, d_cc, d_sums, static_cast<hipStream_t>(stream));
  });
}

tc_status tc_transitivity(const tc_graph* gh, double* out, void* stream) {
  return tc::guarded("tc_transitivity", [&] {
    TC_REQUIRE(gh != nullptr && out != nullptr, TC_EINVAL, "tc_transitivity: null argument");
    hipStream_t st = static_cast<hipStream_t>(stream);
    tc::TempStream temps(st);
    tc::DevBuf sums(2 * sizeof(int64_t));
    tc::vertex_counts(*tc::G(gh), nullptr, nullptr, sums.as<int64_t>(), st);
    int64_t h[2] = {0, 0};
    TC_HIP(hipMemcpyAsync(h, sums.p, sizeof(h), hipMemcpyDeviceToHost, st));
    TC_HIP(hipStreamSynchronize(st));
    *out = h[1] ? (double)h[0] / (double)h[1] : 0.0;
  });
}

tc_status tc_truss(const tc_graph* gh, int32_t* d_tau, int32_t* kmax, void* stream) {
  return tc::guarded("tc_truss", [&] {
    TC_REQUIRE(gh != nullptr, TC_EINVAL, "tc_truss: null graph");
    const tc::Graph& g = *tc::G(gh);
    TC_REQUIRE(d_tau != nullptr || g.m == 0, TC_EINVAL, "tc_truss: null trussness array");
    const int32_t k = tc::truss(g, d_tau, static_cast<hipStream_t>(stream));
    if (kmax) *kmax = k;
  });
}

}  // extern "C"
