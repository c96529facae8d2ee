// tc_block.hip - one rank's share of the 2D cyclic decomposition (Section 5.1,
// Eq. 4 and Eq. 5) at its real shape.
//
// For a q x q grid, rank (x, y) owns the tasks (i, j) of U with j % q == x and
// i % q == y. It hashes the rows j == x (mod q) and probes the rows
// i == y (mod q); both are gathered into rank-local CSRs indexed by the
// transformed index v / q (Section 5.1), entries keeping their global ids so
// that the closing vertex k of a hit names its shift: under the cyclic
// distribution the pair of blocks multiplied in shift z holds exactly the k
// with k % q == (x + y + z) % q (Eq. 5). All q shifts of the rank run in one
// pass of the count kernels (the union of their lookups is exactly the rank's
// lookups), and every hit is credited to its shift's counter.
//
// Tasks are built like the whole graph's: the entry of b = j in local probe
// row a = i starts a task when b % q == x, U_a has entries after it and U_b is
// not empty; tasks are grouped by local hashed row b / q and split into the
// same work classes.
#include "tc_prims.h"

namespace tc {

namespace {

constexpr int kBT = 256;
inline unsigned blocks_for(int64_t n) { return (unsigned)std::max<int64_t>(1, div_up(n, kBT)); }

template <class T>
T read_dev(const T* d, hipStream_t st) {
  T h{};
  TC_HIP(hipMemcpyAsync(&h, d, sizeof(T), hipMemcpyDeviceToHost, st));
  TC_HIP(hipStreamSynchronize(st));
  return h;
}

// Rows v == r (mod q) of [0, n): count and local index v / q.
inline int64_t residue_rows(int64_t n, int64_t q, int64_t r) { return r < n ? (n - 1 - r) / q + 1 : 0; }

// |U_v| of every local row lv (v = lv * q + r).
__global__ void k_local_deg(const int64_t* __restrict__ row_ptr, int64_t nloc, int32_t q, int32_t r,
                            uint32_t* __restrict__ deg) {
  const int64_t lv = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (lv >= nloc) return;
  const int64_t v = lv * q + r;
  deg[lv] = (uint32_t)(row_ptr[v + 1] - row_ptr[v]);
}

// Copy of the local rows, one wave per row (coalesced runs).
__global__ __launch_bounds__(256) void k_gather_rows(const int64_t* __restrict__ row_ptr,
                                                     const int32_t* __restrict__ col, int64_t nloc,
                                                     int32_t q, int32_t r,
                                                     const int64_t* __restrict__ lrow_ptr,
                                                     int32_t* __restrict__ lcol) {
  const int64_t lv = (int64_t)blockIdx.x * (blockDim.x / 64) + (threadIdx.x >> 6);
  if (lv >= nloc) return;
  const int64_t v = lv * q + r;
  const int64_t s = row_ptr[v], d = row_ptr[v + 1] - s, o = lrow_ptr[lv];
  for (int64_t i = threadIdx.x & 63; i < d; i += 64) lcol[o + i] = col[s + i];
}

// Entry p of local probe row a (= erow[p]) holding b starts a task iff
// b % q == x, the row has entries after p, and U_b is not empty; the task's
// key is the local hashed row b / q and its value the probe range
// [p + 1, end of row a).
struct BlockTaskPred {
  const int32_t* pcol;
  const uint32_t* erow;
  const int64_t* prow_ptr;
  const int64_t* hrow_ptr;
  int64_t nh;
  int32_t q, x;
  uint32_t* tkey;
  uint64_t* tval;
  struct Item {
    uint32_t lb, end;
  };
  __device__ bool operator()(int64_t p, Item& it) const {
    const int32_t b = pcol[p];
    if (b % q != x) return false;
    const int64_t lb = b / q;
    it.lb = (uint32_t)lb;
    it.end = (uint32_t)prow_ptr[erow[p] + 1];
    return lb < nh && (int64_t)it.end - p - 1 > 0 && hrow_ptr[lb + 1] > hrow_ptr[lb];
  }
  __device__ void emit(int64_t p, const Item& it, uint32_t pos) const {
    tkey[pos] = it.lb;
    tval[pos] = (uint64_t)(p + 1) | ((uint64_t)it.end << 32);
  }
};

// Local CSR of the rows v == r (mod q).
struct LocalRows {
  int64_t nloc = 0, nnz = 0;
  DevBuf row_ptr;  // int64 [nloc + 1]
  DevBuf col;      // int32 [nnz], global ids
};

void gather_local(LocalRows& L, const Graph& g, int32_t q, int32_t r, hipStream_t st) {
  L.nloc = residue_rows(g.n, q, r);
  L.row_ptr.alloc(sizeof(int64_t) * (size_t)(L.nloc + 1));
  int64_t* lp = L.row_ptr.as<int64_t>();
  if (L.nloc == 0) {
    TC_HIP(hipMemsetAsync(lp, 0, sizeof(int64_t), st));
    return;
  }
  DevBuf deg(sizeof(uint32_t) * (size_t)L.nloc);
  TC_LAUNCH("block_deg", k_local_deg, dim3(blocks_for(L.nloc)), dim3(kBT), 0, st, g.row_ptr, L.nloc, q, r,
            deg.as<uint32_t>());
  device_excl_scan<uint32_t, uint64_t>(deg.as<uint32_t>(), reinterpret_cast<uint64_t*>(lp), L.nloc,
                                       reinterpret_cast<uint64_t*>(lp) + L.nloc, st);
  TC_HIP(hipGetLastError());
  L.nnz = read_dev(lp + L.nloc, st);
  L.col.alloc(sizeof(int32_t) * (size_t)std::max<int64_t>(L.nnz, 1));
  if (L.nnz > 0)
    TC_LAUNCH("block_gather", k_gather_rows, dim3((unsigned)div_up(L.nloc, kBT / 64)), dim3(kBT), 0, st,
              g.row_ptr, g.col, L.nloc, q, r, lp, L.col.as<int32_t>());
  TC_HIP(hipGetLastError());
}

}  // namespace

void block_count(const Graph& g, int32_t q, int32_t x, int32_t y, int64_t* d_count, int64_t* d_per_shift,
                 hipStream_t st) {
  TempStream temps(st);
  Owned own;
  own.st = st;
  LocalRows H, P;
  gather_local(H, g, q, x, st);  // hash side: rows j == x
  gather_local(P, g, q, y, st);  // probe side: rows i == y
  TC_REQUIRE(P.nnz <= kMaxEdges, TC_EOVERFLOW, "tc_block_count: probe side exceeds 2^30 entries");

  int64_t T = 0;
  TaskLists tl;
  if (P.nnz > 0 && H.nnz > 0) {
    DevBuf erow(sizeof(uint32_t) * (size_t)P.nnz);
    TC_LAUNCH("block_entry_rows", k_entry_rows, dim3((unsigned)div_up(P.nloc, kBT / 64)), dim3(kBT), 0,
              st, P.row_ptr.as<int64_t>(), P.nloc, erow.as<uint32_t>());
    DevBuf tk, tv;
    BlockTaskPred bp{P.col.as<int32_t>(), erow.as<uint32_t>(), P.row_ptr.as<int64_t>(), H.row_ptr.as<int64_t>(),
                     H.nloc, q, x, nullptr, nullptr};
    T = compact("block_tasks", P.nnz, bp, [&](int64_t total, BlockTaskPred& pr) {
      tk.alloc(sizeof(uint32_t) * (size_t)total);
      tv.alloc(sizeof(uint64_t) * (size_t)total);
      pr.tkey = tk.as<uint32_t>();
      pr.tval = tv.as<uint64_t>();
    }, st);
    if (T > 0) {
      const int bits = std::max(1, ceil_log2_u64((uint64_t)H.nloc));
      sort_tasks(tl, tk, tv, T, H.nloc, bits, st, "block_tasks");
    }
  }
  WorkSet w;
  build_work(w, own, H.nloc, H.row_ptr.as<int64_t>(), T, tl.row.as<uint32_t>(), tl.ptr.as<int64_t>(),
             tl.val.as<uint64_t>(), tl.prefix.as<uint64_t>(), st);
  CountView v{H.row_ptr.as<int64_t>(), H.col.as<int32_t>(), P.col.as<int32_t>(), P.nnz, &w, q,
              (x + y) % q};
  launch_count(v, MODE_BLOCK, d_count, nullptr, d_per_shift, st);
  check_task_sorts(st);
}

}  // namespace tc

extern "C" tc_status tc_block_count(const tc_graph* gh, int32_t q, int32_t x, int32_t y, int64_t* d_count,
                                    int64_t* d_per_shift, void* stream) {
  try {
    TC_REQUIRE(gh != nullptr, TC_EINVAL, "tc_block_count: null graph");
    TC_REQUIRE(q >= 1 && q <= 64, TC_EINVAL, "tc_block_count: q must be in [1, 64]");
    TC_REQUIRE(x >= 0 && x < q && y >= 0 && y < q, TC_EINVAL, "tc_block_count: (x, y) outside the grid");
    TC_REQUIRE(d_count != nullptr || d_per_shift != nullptr, TC_EINVAL,
               "tc_block_count: no output array");
    tc::block_count(*tc::G(gh), q, x, y, d_count, d_per_shift, static_cast<hipStream_t>(stream));
    tc::set_last_error("");
    return TC_OK;
  } catch (const tc::Error& e) {
    tc::set_last_error(e.what());
    return e.status;
  } catch (const std::bad_alloc&) {
    tc::set_last_error("tc_block_count: host allocation failed");
    return TC_ENOMEM;
  } catch (const std::exception& e) {
    tc::set_last_error(e.what());
    return TC_EDEVICE;
  }
}
