// tc_count.hip - the map-based intersection of Section 3.1 (<j,i,k> order) and
// its reductions: exact triangle count (Eq. 2) and per-edge support (Eq. 1).
//
// Work unit. For a hashed row b, a task is a nonzero (a, b) of U (a in L_b,
// the column of b); it probes the entries of U_a after b - all of them exceed
// b, which is Eq. 1's k > j bound - against a hash of U_b. A hit is a
// triangle a < b < k. The probes of all tasks of one b form one contiguous
// range of the global probe index space (tasks grouped by b, prefix-summed by
// preprocessing).
//
// Hash table (Section 5.2, "Modifying the hashing routine"): U_b in LDS,
// 2^l >= 2 |U_b| slots, slot = k & (2^l - 1) (the direct bitwise AND), linear
// probing on collision. The build records the longest displacement D; a
// lookup stops at a match, an empty slot or after D + 1 slots, so a
// collision-free table (D = 0) costs one LDS read per probe and exactness
// never depends on the absence of collisions.
//
// Probe loop (one wave, flattened over tasks). A wave walks a range of
// probes in batches of 64, lane l taking probe base + l, so every col[] read
// is a coalesced run; kU batches form a super-batch whose loads and lookups
// are all in flight together. A window of 64 consecutive tasks sits one per
// lane (end of the task relative to the wave's position, and the col index its
// probes start from). The task of a probe is the number of window tasks that
// end at or before it: one ballot counts those ending before the super-batch,
// and the tasks ending inside it set bits of a small per-wave LDS bitmap whose
// masked popcounts give each lane its task; the task's col base is then
// fetched from its lane with one bpermute.
//
// Launch classes (decided in preprocessing from |U_b| and the row's probes):
//   packs  - light rows b are packed (about 2K probes per pack); one wave per
//            pack builds each row's table in its private LDS slice in turn.
//   heavy  - a row's probes are cut into per-wave ranges (8K probes); the 4
//            waves of a work-group share one table of that row.
//   global - a row whose table would not fit LDS (|U_b| > 8192): lookups are
//            binary searches in the sorted U_b in HBM.
// Reductions: per-lane 32-bit hit counters, wave reduction by xor shuffles,
// one 64-bit atomic per work-group into the caller's counter (order-free and
// exact).
#include "tc_prims.h"

namespace tc {

namespace {

struct Args {
  const int64_t* __restrict__ row_ptr;
  const int32_t* __restrict__ col;
  const uint32_t* __restrict__ tstart;
  const uint64_t* __restrict__ tprefix;
  const int64_t* __restrict__ tptr;
  int64_t T;
  uint32_t m;  // entries of col (probe positions are checked against it)
  unsigned long long* count;
  int32_t* support;
};

constexpr int kU = 8;                   // 64-probe batches per super-batch
constexpr int kBmWords = 2 * kU;        // per-wave task-end bitmap (64 * kU bits)
constexpr int kMarkInts = kWaves * kBmWords;

__device__ __forceinline__ uint64_t lanemask_le() { return (2ull << lane_id()) - 1ull; }

// Lookup by binary search in the sorted row col[rs, rs + d); returns the
// position of k or -1.
__device__ __forceinline__ int64_t hbm_find(const int32_t* __restrict__ col, int64_t rs, int64_t d,
                                            int32_t k) {
  int64_t lo = rs, hi = rs + d;
  while (lo < hi) {
    int64_t mid = (lo + hi) >> 1;
    int32_t v = col[mid];
    if (v < k) lo = mid + 1;
    else hi = mid;
  }
  return (lo < rs + d && col[lo] == k) ? lo : -1;
}

// Insert U_b = col[rs, rs + d) into a cleared table of S slots; threads
// tid, tid + nt, ... share the work. Returns this thread's longest
// displacement. VALS: also store the U position of every key.
template <bool VALS>
__device__ int build_table(int32_t* tab, int32_t* val, uint32_t mask, const int32_t* __restrict__ col,
                           int64_t rs, int64_t d, int tid, int nt) {
  // keys are fetched kB at a time so that their loads overlap, then inserted
  constexpr int kB = 8;
  int md = 0;
  for (int64_t i0 = tid; i0 < d; i0 += (int64_t)kB * nt) {
    int32_t key[kB];
#pragma unroll
    for (int j = 0; j < kB; ++j) {
      const int64_t i = i0 + (int64_t)j * nt;
      key[j] = i < d ? col[rs + i] : -1;
    }
#pragma unroll
    for (int j = 0; j < kB; ++j) {
      if (key[j] < 0) continue;
      uint32_t h = (uint32_t)key[j] & mask;
      int disp = 0;
      while (atomicCAS(&tab[h], -1, key[j]) != -1) {
        h = (h + 1) & mask;
        ++disp;
      }
      if (VALS) val[h] = (int32_t)(rs + i0 + (int64_t)j * nt);
      md = disp > md ? disp : md;
    }
  }
  return md;
}

// What to do with every probe k (at col position `pos`, task of lane whose
// first probe is at `ts`): count mode adds the hit; support modes also credit
// the triangle's edges.
struct TableRef {
  const int32_t* tab;
  const int32_t* val;
  uint32_t mask;
  int D;
  // global fallback
  int64_t rs, d;
};

template <int MODE, bool GLOBAL>
struct Prober {
  static constexpr bool kNeedTs = MODE != MODE_COUNT;
  // A hit: k = col[pos] was found in U_b at `where` (an LDS slot, or for the
  // HBM fallback the position in col). ts is the first probe position of the
  // task, so ts - 1 is the U entry of the task's own edge (a, b).
  __device__ __forceinline__ static void credit(const Args& A, const TableRef& t, int where,
                                                uint32_t pos, uint32_t ts, uint32_t& hits) {
    ++hits;
    // indices are checked against m so that no credit can leave the array
    if (MODE == MODE_SUPPORT_FULL) {
      const uint32_t other = (uint32_t)(GLOBAL ? where : t.val[where]);
      if (ts - 1u < A.m) atomicAdd(&A.support[ts - 1u], 1);  // edge (a, b)
      atomicAdd(&A.support[pos], 1);                          // edge (a, k): probed entry of U_a
      if (other < A.m) atomicAdd(&A.support[other], 1);       // edge (b, k): k's entry in U_b
    } else if (MODE == MODE_SUPPORT_ORIENTED) {
      if (ts - 1u < A.m) atomicAdd(&A.support[ts - 1u], 1);  // c(a, b) of Eq. 1
    }
  }
};

__device__ __forceinline__ void wave_sync_lds() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// One wave processes the probes [q, q + len) of the tasks of one hashed row;
// task t contains probe q.
//
// The range is walked window by window: a window is the next 64 tasks (one per
// lane) and covers their probes exactly. Inside a window the probes go in
// super-batches of 64 * U (lane l takes probes sb + 64 u + l, u < U), so each
// lane has U independent col[] loads and U table lookups in flight. The task
// of a probe r is c0 + (number of task ends in (sb, r]): c0 by one ballot, the
// ends inside the super-batch as bits of a per-wave LDS bitmap `bm`
// (U * 64 bits), read back word-wise and counted with masked popcounts.
template <int MODE, bool GLOBAL, int U>
__device__ void wave_probe(const Args& A, const TableRef& tr, uint32_t t, uint64_t q, uint32_t len,
                           uint32_t* bm, uint32_t& hits) {
  using P = Prober<MODE, GLOBAL>;
  constexpr uint32_t SB = 64u * U;
  const int lane = lane_id();
  const int64_t T = A.T;
  const uint64_t le = lanemask_le();
  uint32_t done = 0;
  while (done < len) {
    const uint32_t rem = len - done;
    const int64_t tj = (int64_t)t + lane;
    const int64_t tjs = tj < T ? tj : T;
    const int64_t tje = tj + 1 < T ? tj + 1 : T;
    const uint64_t Ps = A.tprefix[tjs];
    const uint64_t Pe = A.tprefix[tje];
    // end of the lane's task relative to q, clamped to the remaining range
    const uint64_t e64 = Pe - q;
    const uint32_t e = e64 > (uint64_t)rem ? rem : (uint32_t)e64;
    // col index of relative probe 0 for the lane's task (mod 2^32)
    const uint32_t tsj = A.tstart[tj < T ? tj : T - 1];
    const uint32_t cbase = tsj - (uint32_t)(Ps - q);
    const uint32_t lim = (uint32_t)__shfl((int)e, 63, 64);  // probes of this window
    if (lim == 0) break;  // unreachable when every task has a probe; guards progress
    for (uint32_t sb = 0; sb < lim; sb += SB) {
      const uint32_t c0 = (uint32_t)__popcll(__ballot(e <= sb));
      const bool inner = e > sb && e < sb + SB;
      uint32_t jl[U];
      if (__ballot(inner) == 0) {
#pragma unroll
        for (int u = 0; u < U; ++u) jl[u] = c0;
      } else {
        if (inner) atomicOr(&bm[(e - sb) >> 5], 1u << ((e - sb) & 31));
        wave_sync_lds();
        uint32_t pre = c0;
#pragma unroll
        for (int u = 0; u < U; ++u) {
          const uint64_t M = (uint64_t)bm[2 * u] | ((uint64_t)bm[2 * u + 1] << 32);
          const uint32_t j = pre + (uint32_t)__popcll(M & le);
          jl[u] = j < 63 ? j : 63;  // only lanes past the window (r >= lim) can exceed 63
          pre += (uint32_t)__popcll(M);
        }
        wave_sync_lds();
        if (lane < (int)(SB / 32)) bm[lane] = 0;
        wave_sync_lds();
      }
      uint32_t pos[U];
      bool ok[U];
      int32_t k[U];
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const uint32_t r = sb + 64u * u + (uint32_t)lane;
        pos[u] = (uint32_t)__shfl((int)cbase, (int)jl[u], 64) + r;
        ok[u] = r < lim && pos[u] < A.m;
      }
#pragma unroll
      for (int u = 0; u < U; ++u) k[u] = ok[u] ? A.col[pos[u]] : -1;
      // task start of every probe (support modes), read across lanes while all
      // lanes are active: a bpermute must not run under a divergent mask
      uint32_t ts[U];
#pragma unroll
      for (int u = 0; u < U; ++u)
        ts[u] = P::kNeedTs ? (uint32_t)__shfl((int)tsj, (int)jl[u], 64) : 0u;
      if constexpr (!GLOBAL) {
        // first slot of every lookup at once, then the (rare) probe chains
        int32_t v[U];
        uint32_t h[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
          h[u] = (uint32_t)k[u] & tr.mask;
          v[u] = tr.tab[h[u]];
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
          if (!ok[u]) continue;
          int slot = -1;
          if (v[u] == k[u]) {
            slot = (int)h[u];
          } else if (v[u] >= 0 && tr.D > 0) {
            uint32_t hh = h[u];
            for (int i = 1; i <= tr.D; ++i) {
              hh = (hh + 1) & tr.mask;
              const int32_t w = tr.tab[hh];
              if (w == k[u]) {
                slot = (int)hh;
                break;
              }
              if (w < 0) break;
            }
          }
          if (slot >= 0) P::credit(A, tr, slot, pos[u], ts[u], hits);
        }
      } else {
#pragma unroll
        for (int u = 0; u < U; ++u) {
          const int64_t where = ok[u] ? hbm_find(A.col, tr.rs, tr.d, k[u]) : -1;
          if (where >= 0) P::credit(A, tr, (int)where, pos[u], ts[u], hits);
        }
      }
    }
    t += (uint32_t)__popcll(__ballot(e <= lim));
    q += lim;
    done += lim;
  }
}


__device__ __forceinline__ void block_flush(uint32_t hits, unsigned long long* count) {
  __shared__ unsigned long long s_sum[kWaves];
  unsigned long long h = wave_sum((unsigned long long)hits);
  if (lane_id() == 0) s_sum[threadIdx.x >> 6] = h;
  __syncthreads();
  if (threadIdx.x == 0 && count) {
    unsigned long long tot = 0;
#pragma unroll
    for (int w = 0; w < kWaves; ++w) tot += s_sum[w];
    if (tot) atomicAdd(count, tot);
  }
}

// Packs of light rows: each wave owns a table slice of 2^log2Smax slots.
template <int MODE>
__global__ __launch_bounds__(256) void k_count_packs(Args A, const int32_t* __restrict__ rows,
                                                     const uint32_t* __restrict__ pack_ptr,
                                                     int64_t n_packs, int log2Smax) {
  extern __shared__ int32_t smem[];
  constexpr bool VALS = MODE == MODE_SUPPORT_FULL;
  const int lane = lane_id(), wave = threadIdx.x >> 6;
  uint32_t* bm = reinterpret_cast<uint32_t*>(smem) + wave * kBmWords;
  const uint32_t Smax = 1u << log2Smax;
  int32_t* tab = smem + kMarkInts + (size_t)wave * Smax * (VALS ? 2 : 1);
  int32_t* val = tab + Smax;
  if (lane < kBmWords) bm[lane] = 0;
  uint32_t hits = 0;
  const int64_t p = (int64_t)blockIdx.x * kWaves + wave;
  if (p < n_packs) {
    const uint32_t r0 = pack_ptr[p], r1 = pack_ptr[p + 1];
    for (uint32_t r = r0; r < r1; ++r) {
      const int32_t b = rows[r];
      const int64_t rs = A.row_ptr[b], d = A.row_ptr[b + 1] - rs;
      int l = 6;
      while ((1ll << l) < 2 * d) ++l;
      const uint32_t S = 1u << l, mask = S - 1;
      for (uint32_t i = lane; i < S; i += 64) tab[i] = -1;
      wave_sync_lds();
      int md = build_table<VALS>(tab, val, mask, A.col, rs, d, lane, 64);
      md = wave_max(md);
      wave_sync_lds();
      const int64_t tl = A.tptr[b], th = A.tptr[b + 1];
      const uint64_t q0 = A.tprefix[tl], q1 = A.tprefix[th];
      TableRef tr{tab, val, mask, md, rs, d};
      wave_probe<MODE, false, kU>(A, tr, (uint32_t)tl, q0, (uint32_t)(q1 - q0), bm, hits);
      wave_sync_lds();
    }
  }
  block_flush(hits, A.count);
}

// Heavy rows: work-group = kWaves consecutive items of the same row b.
template <int MODE, bool GLOBAL>
__global__ __launch_bounds__(256) void k_count_items(Args A, const CountItem* __restrict__ items) {
  extern __shared__ int32_t smem[];
  __shared__ int s_D;
  constexpr bool VALS = MODE == MODE_SUPPORT_FULL;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  uint32_t* bm = reinterpret_cast<uint32_t*>(smem) + wave * kBmWords;
  const CountItem* grp = items + (int64_t)blockIdx.x * kWaves;
  const int32_t b = grp[0].b;
  const int64_t rs = A.row_ptr[b], d = A.row_ptr[b + 1] - rs;
  if (lane < kBmWords) bm[lane] = 0;
  uint32_t hits = 0;
  TableRef tr{nullptr, nullptr, 0, 0, rs, d};
  if (!GLOBAL) {
    const uint32_t S = 1u << grp[0].log2S, mask = S - 1;
    int32_t* tab = smem + kMarkInts;
    int32_t* val = tab + S;
    for (uint32_t i = tid; i < S; i += 256) tab[i] = -1;
    if (tid == 0) s_D = 0;
    __syncthreads();
    int md = build_table<VALS>(tab, val, mask, A.col, rs, d, tid, 256);
    md = wave_max(md);
    if (lane == 0) atomicMax(&s_D, md);
    __syncthreads();
    tr.tab = tab;
    tr.val = val;
    tr.mask = mask;
    tr.D = s_D;
  }
  const CountItem it = grp[wave];
  wave_sync_lds();
  if (it.len) wave_probe<MODE, GLOBAL, kU>(A, tr, it.t0, it.q0, it.len, bm, hits);
  block_flush(hits, A.count);
}

__global__ void k_zero_i64(int64_t* p) { *p = 0; }

__global__ void k_zero_i32(int32_t* p, int64_t n) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = 0;
}

// launch names seen by the phase timer: "<mode>:<class>"
const char* const kLaunchNames[3][NUM_CLASSES] = {
    {"count:pack_small", "count:pack_large", "count:wg_small", "count:wg_large", "count:wg_huge",
     "count:global"},
    {"support_full:pack_small", "support_full:pack_large", "support_full:wg_small",
     "support_full:wg_large", "support_full:wg_huge", "support_full:global"},
    {"support_oriented:pack_small", "support_oriented:pack_large", "support_oriented:wg_small",
     "support_oriented:wg_large", "support_oriented:wg_huge", "support_oriented:global"}};

template <int MODE>
void launch_mode(const Graph& g, const Args& A, hipStream_t st) {
  constexpr bool VALS = MODE == MODE_SUPPORT_FULL;
  const size_t mark_bytes = sizeof(int32_t) * kMarkInts;
  for (int c = CLS_PACK_SMALL; c <= CLS_PACK_LARGE; ++c) {
    if (g.n_packs[c] == 0) continue;
    const int l = g.pack_log2S[c];
    const size_t lds = mark_bytes + sizeof(int32_t) * (size_t)kWaves * ((size_t)1 << l) * (VALS ? 2 : 1);
    const unsigned grid = (unsigned)div_up(g.n_packs[c], kWaves);
    if (lds > 65536)
      TC_HIP(hipFuncSetAttribute((const void*)k_count_packs<MODE>,
                                 hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
    TC_LAUNCH(kLaunchNames[MODE][c], k_count_packs<MODE>, dim3(grid), dim3(256), lds, st, A, g.pack_rows[c],
                       g.pack_ptr[c], g.n_packs[c], l);
  }
  for (int c = CLS_WG_SMALL; c <= CLS_GLOBAL; ++c) {
    if (g.n_items[c] == 0) continue;
    const unsigned grid = (unsigned)(g.n_items[c] / kWaves);
    if (c == CLS_GLOBAL) {
      TC_LAUNCH(kLaunchNames[MODE][c], (k_count_items<MODE, true>), dim3(grid), dim3(256), mark_bytes, st, A,
                         g.items[c]);
    } else {
      const size_t lds = mark_bytes + sizeof(int32_t) * ((size_t)1 << g.cls_log2S[c]) * (VALS ? 2 : 1);
      if (lds > 65536)
        TC_HIP(hipFuncSetAttribute((const void*)k_count_items<MODE, false>,
                                   hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
      TC_LAUNCH(kLaunchNames[MODE][c], (k_count_items<MODE, false>), dim3(grid), dim3(256), lds, st, A, g.items[c]);
    }
  }
  TC_HIP(hipGetLastError());
}

}  // namespace

void launch_count(const Graph& g, CountMode mode, int64_t* d_count, int32_t* d_support,
                  hipStream_t st) {
  if (d_count) TC_LAUNCH("zero_i64", k_zero_i64, dim3(1), dim3(1), 0, st, d_count);
  if (mode != MODE_COUNT && g.m > 0)
    TC_LAUNCH("zero_i32", k_zero_i32, dim3((unsigned)div_up(g.m, 256)), dim3(256), 0, st, d_support, g.m);
  TC_HIP(hipGetLastError());
  if (g.n_tasks == 0) return;
  Args A{g.row_ptr, g.col, g.tstart, g.tprefix, g.tptr, g.n_tasks, (uint32_t)g.m,
         reinterpret_cast<unsigned long long*>(d_count), d_support};
  switch (mode) {
    case MODE_COUNT: launch_mode<MODE_COUNT>(g, A, st); break;
    case MODE_SUPPORT_FULL: launch_mode<MODE_SUPPORT_FULL>(g, A, st); break;
    case MODE_SUPPORT_ORIENTED: launch_mode<MODE_SUPPORT_ORIENTED>(g, A, st); break;
  }
}

}  // namespace tc
