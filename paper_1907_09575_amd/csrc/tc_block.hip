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

// Copy of the local rows, four per wave: rows of at most 64 entries are
// copied by 16 lanes each (rows here hold ~16 entries on average, so a wave
// per row would leave most lanes idle), longer rows then one after another
// by the whole wave. With erow, it also writes each entry's local row.
__device__ __forceinline__ int64_t shfl_i64(int64_t v, int src) {
  const int lo = __shfl((int)(uint32_t)v, src, 64), hi = __shfl((int)(uint32_t)((uint64_t)v >> 32), src, 64);
  return (int64_t)(((uint64_t)(uint32_t)hi << 32) | (uint32_t)lo);
}

__global__ __launch_bounds__(256) void k_gather_rows(const int64_t* __restrict__ row_ptr,
                                                     const int32_t* __restrict__ col, int64_t nloc,
                                                     int32_t q, int32_t r,
                                                     const int64_t* __restrict__ lrow_ptr,
                                                     int32_t* __restrict__ lcol, uint32_t* __restrict__ erow) {
  const int lane = lane_id(), grp = lane >> 4, sub = lane & 15;
  const int64_t stride = (int64_t)gridDim.x * (blockDim.x / 64) * 4;  // (grid-stride over groups of 4 rows)
  for (int64_t lv0 = ((int64_t)blockIdx.x * (blockDim.x / 64) + (threadIdx.x >> 6)) * 4; lv0 < nloc;
       lv0 += stride) {
    const int64_t lv = lv0 + grp;
    int64_t s0 = 0, len = 0, o = 0;
    if (lv < nloc) {
      const int64_t v = lv * q + r;
      s0 = row_ptr[v];
      len = row_ptr[v + 1] - s0;
      o = lrow_ptr[lv];
    }
    if (len <= 64) {
      for (int64_t i = sub; i < len; i += 16) {
        lcol[o + i] = col[s0 + i];
        if (erow) erow[o + i] = (uint32_t)lv;
      }
    }
    // long rows (lane 16 g stands for group g), by the whole wave
    uint64_t longs = __ballot(len > 64 && sub == 0);
    while (longs) {
      const int src = __ffsll((long long)longs) - 1;
      longs &= longs - 1;
      const int64_t ls = shfl_i64(s0, src), ll = shfl_i64(len, src), lo = shfl_i64(o, src);
      const uint32_t lrow = (uint32_t)(lv0 + (src >> 4));
      for (int64_t i = lane; i < ll; i += 64) {
        lcol[lo + i] = col[ls + i];
        if (erow) erow[lo + i] = lrow;
      }
    }
  }
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

// Row pointers of the local rows of residue r (their total at [nloc]).
void local_ptrs(LocalRows& L, const Graph& g, int32_t q, int32_t r, hipStream_t st) {
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
}

// Columns of the local rows (L.nnz known), with each entry's local row in
// erow if given (erow->alloc'd here).
void local_gather(LocalRows& L, const Graph& g, int32_t q, int32_t r, DevBuf* erow, hipStream_t st) {
  L.col.alloc(sizeof(int32_t) * (size_t)std::max<int64_t>(L.nnz, 1));
  if (erow) erow->alloc(sizeof(uint32_t) * (size_t)std::max<int64_t>(L.nnz, 1));
  if (L.nnz > 0)
    TC_LAUNCH("block_gather", k_gather_rows, dim3(wave_grid(div_up(L.nloc, 4))), dim3(kBT), 0, st,
              g.row_ptr, g.col, L.nloc, q, r, L.row_ptr.as<int64_t>(), L.col.as<int32_t>(),
              erow ? erow->as<uint32_t>() : nullptr);
  TC_HIP(hipGetLastError());
}

// The rank's hashed rows H (residue x) and probe rows P (residue y), with
// one host synchronisation for both sizes; erow_p: P's entry rows.
void gather_pair(LocalRows& H, LocalRows& P, const Graph& g, int32_t q, int32_t x, int32_t y, DevBuf* erow_p,
                 hipStream_t st) {
  local_ptrs(H, g, q, x, st);
  local_ptrs(P, g, q, y, st);
  int64_t h[2] = {0, 0};
  TC_HIP(hipMemcpyAsync(&h[0], H.row_ptr.as<int64_t>() + H.nloc, sizeof(int64_t), hipMemcpyDeviceToHost, st));
  TC_HIP(hipMemcpyAsync(&h[1], P.row_ptr.as<int64_t>() + P.nloc, sizeof(int64_t), hipMemcpyDeviceToHost, st));
  TC_HIP(hipStreamSynchronize(st));
  H.nnz = h[0];
  P.nnz = h[1];
  local_gather(H, g, q, x, nullptr, st);
  local_gather(P, g, q, y, erow_p, st);
}

}  // namespace

void block_count(const Graph& g, int32_t q, int32_t x, int32_t y, int64_t* d_count, int64_t* d_per_shift,
                 hipStream_t st) {
  TempStream temps(st);
  Owned own;
  own.st = st;
  LocalRows H, P;  // hash side: rows j == x; probe side: rows i == y
  DevBuf erow;      // local row of each probe-side entry
  gather_pair(H, P, g, q, x, y, &erow, st);
  TC_REQUIRE(P.nnz <= kMaxBufferEdges, TC_EOVERFLOW, "tc_block_count: a rank's probe side of 2^30 entries or more");

  int64_t T = 0;
  TaskLists tl;
  if (P.nnz > 0 && H.nnz > 0) {
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
             tl.val.as<uint64_t>(), tl.prefix.as<uint64_t>(), WorkParams(), st);
  CountView v{H.row_ptr.as<int64_t>(), H.col.as<int32_t>(), P.col.as<int32_t>(), P.nnz, &w, q,
              (x + y) % q};
  launch_count(v, MODE_BLOCK, d_count, nullptr, d_per_shift, st);
  note_use(g, st);
  check_task_sorts(st);
}

namespace {

// Shift classes present in every local hashed row: bit z of mask[lb] is set
// when U_b (b = lb * q + x) holds an entry k with (k - x - y) mod q == z
// (one wave per row).
__global__ __launch_bounds__(256) void k_row_shift_mask(const int64_t* __restrict__ hrow_ptr,
                                                        const int32_t* __restrict__ hcol, int64_t nloc,
                                                        int32_t q, int32_t xy, uint64_t* __restrict__ mask) {
  const int64_t stride = (int64_t)gridDim.x * (blockDim.x / 64);
  for (int64_t lb = (int64_t)blockIdx.x * (blockDim.x / 64) + (threadIdx.x >> 6); lb < nloc; lb += stride) {
    uint64_t mk = 0;
    for (int64_t i = hrow_ptr[lb] + lane_id(); i < hrow_ptr[lb + 1]; i += 64) {
      int z = (int)((uint32_t)hcol[i] % (uint32_t)q) - xy;
      if (z < 0) z += q;
      mk |= 1ull << z;
    }
#pragma unroll
    for (int d = 32; d >= 1; d >>= 1) mk |= (uint64_t)__shfl_xor((unsigned long long)mk, d, 64);
    if (lane_id() == 0) mask[lb] = mk;
  }
}

// Work of the rank's tasks (tkey = local hashed row, tval = first probe | end
// << 32 in the local probe CSR), one wave per task, tasks strided over the
// grid: out[0] tasks, out[1] probes, out[2 + z] probes of shift z, out[2 + q
// + z] tasks whose probe list and hashed list both hold shift z's class.
__global__ __launch_bounds__(256) void k_block_work(const uint32_t* __restrict__ tkey,
                                                    const uint64_t* __restrict__ tval, int64_t T,
                                                    const int32_t* __restrict__ pcol,
                                                    const uint64_t* __restrict__ hmask, int32_t q, int32_t xy,
                                                    unsigned long long* __restrict__ out) {
  __shared__ unsigned int s_probe[64], s_task[64];
  __shared__ unsigned long long s_tot[2];
  if (threadIdx.x < 64) {
    s_probe[threadIdx.x] = 0;
    s_task[threadIdx.x] = 0;
  }
  if (threadIdx.x < 2) s_tot[threadIdx.x] = 0;
  __syncthreads();
  const int lane = lane_id();
  const int64_t waves = (int64_t)gridDim.x * (blockDim.x / 64);
  uint64_t tasks = 0, probes = 0;
  for (int64_t t = (int64_t)blockIdx.x * (blockDim.x / 64) + (threadIdx.x >> 6); t < T; t += waves) {
    const uint64_t v = tval[t];
    const uint32_t first = (uint32_t)v, end = (uint32_t)(v >> 32);
    uint64_t pm = 0;
    for (uint32_t i = first + (uint32_t)lane; i < end; i += 64) {
      int z = (int)((uint32_t)pcol[i] % (uint32_t)q) - xy;
      if (z < 0) z += q;
      pm |= 1ull << z;
      atomicAdd(&s_probe[z], 1u);
    }
#pragma unroll
    for (int d = 32; d >= 1; d >>= 1) pm |= (uint64_t)__shfl_xor((unsigned long long)pm, d, 64);
    const uint64_t both = pm & hmask[tkey[t]];
    if (lane < q && ((both >> lane) & 1ull)) atomicAdd(&s_task[lane], 1u);
    tasks += 1;
    probes += end - first;
  }
  if (lane == 0 && tasks) {
    atomicAdd(&s_tot[0], (unsigned long long)tasks);
    atomicAdd(&s_tot[1], (unsigned long long)probes);
  }
  __syncthreads();
  if (threadIdx.x < 2 && s_tot[threadIdx.x]) atomicAdd(&out[threadIdx.x], s_tot[threadIdx.x]);
  if ((int)threadIdx.x < q) {
    if (s_probe[threadIdx.x]) atomicAdd(&out[2 + threadIdx.x], (unsigned long long)s_probe[threadIdx.x]);
    if (s_task[threadIdx.x]) atomicAdd(&out[2 + q + threadIdx.x], (unsigned long long)s_task[threadIdx.x]);
  }
}

__global__ void k_zero_n(unsigned long long* p, int n) {
  if ((int)threadIdx.x < n) p[threadIdx.x] = 0;
}

}  // namespace

void block_stats(const Graph& g, int32_t q, int32_t x, int32_t y, int64_t* d_out, hipStream_t st) {
  TempStream temps(st);
  auto* out = reinterpret_cast<unsigned long long*>(d_out);
  TC_LAUNCH("zero_stats", k_zero_n, dim3(1), dim3(192), 0, st, out, 2 + 2 * q);
  LocalRows H, P;
  DevBuf erow;
  gather_pair(H, P, g, q, x, y, &erow, st);
  note_use(g, st);  // (later kernels read only the local copies)
  if (P.nnz == 0 || H.nnz == 0) return;
  DevBuf tk, tv;
  BlockTaskPred bp{P.col.as<int32_t>(), erow.as<uint32_t>(), P.row_ptr.as<int64_t>(), H.row_ptr.as<int64_t>(),
                   H.nloc, q, x, nullptr, nullptr};
  const int64_t T = compact("block_stats_tasks", P.nnz, bp, [&](int64_t total, BlockTaskPred& pr) {
    tk.alloc(sizeof(uint32_t) * (size_t)total);
    tv.alloc(sizeof(uint64_t) * (size_t)total);
    pr.tkey = tk.as<uint32_t>();
    pr.tval = tv.as<uint64_t>();
  }, st);
  if (T == 0) return;
  DevBuf hmask(sizeof(uint64_t) * (size_t)H.nloc);
  const int32_t xy = (x + y) % q;
  TC_LAUNCH("block_row_mask", k_row_shift_mask, dim3(wave_grid(H.nloc)), dim3(kBT), 0, st,
            H.row_ptr.as<int64_t>(), H.col.as<int32_t>(), H.nloc, q, xy, hmask.as<uint64_t>());
  const unsigned grid = (unsigned)std::min<int64_t>(4096, div_up(T, kBT / 64));
  TC_LAUNCH("block_work", k_block_work, dim3(grid), dim3(kBT), 0, st, tk.as<uint32_t>(), tv.as<uint64_t>(), T,
            P.col.as<int32_t>(), hmask.as<uint64_t>(), q, xy, out);
  TC_HIP(hipGetLastError());
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
    tc::require_plain(*tc::G(gh), "tc_block_count");
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

extern "C" tc_status tc_block_stats(const tc_graph* gh, int32_t q, int32_t x, int32_t y, int64_t* d_out,
                                    void* stream) {
  try {
    TC_REQUIRE(gh != nullptr && d_out != nullptr, TC_EINVAL, "tc_block_stats: null argument");
    TC_REQUIRE(q >= 1 && q <= 64, TC_EINVAL, "tc_block_stats: q must be in [1, 64]");
    TC_REQUIRE(x >= 0 && x < q && y >= 0 && y < q, TC_EINVAL, "tc_block_stats: (x, y) outside the grid");
    tc::require_plain(*tc::G(gh), "tc_block_stats");
    tc::block_stats(*tc::G(gh), q, x, y, d_out, static_cast<hipStream_t>(stream));
    tc::set_last_error("");
    return TC_OK;
  } catch (const tc::Error& e) {
    tc::set_last_error(e.what());
    return e.status;
  } catch (const std::bad_alloc&) {
    tc::set_last_error("tc_block_stats: host allocation failed");
    return TC_ENOMEM;
  } catch (const std::exception& e) {
    tc::set_last_error(e.what());
    return TC_EDEVICE;
  }
}
