// tc_preprocess.hip - device preprocessing (Section 5.3 of the paper, on one GPU).
//
// Pipeline, all on the caller's stream:
//   1. canonical keys: each pair {u, v}, u != v, becomes min(u,v) * 2^s + max(u,v)
//      (s = ceil(log2 n)); self loops and invalid ids become a sentinel.
//   2. stable LSD radix sort of the 2s-bit keys: the distinct keys (those
//      that differ from their predecessor and are not the sentinel) are the
//      simple undirected graph of Section 2 / Section 6.1; they are selected
//      from the sorted keys by each later reader, never copied out.
//   3. degrees counted in LDS per vertex range: lower endpoints from the
//      sorted keys, upper endpoints from a radix partition of them by their
//      top bits; rank = position in the order (degree, id)
//      (a stable radix sort of degree * 2^s + id on the degree bits): the
//      non-decreasing degree relabelling of Section 5.3.
//   4. orientation by rank (Section 5.3: the global position stands in for the
//      degree), radix sort of rank keys -> U in CSR with sorted rows
//      (Section 5.2 requires sorted rows).
//   5. tasks (Section 3.1, <j,i,k>): every nonzero (a, b) of U whose row a has
//      entries after b and whose row b is non-empty probes U_a's entries after b
//      against a hash of U_b. Tasks are grouped by b (the transpose L = U^T of
//      Section 3.1), stably, so within one b the rows a ascend.
//   6. work classes and items for the count kernels (see tc_count.hip): rows b
//      are split by table size and work; the tasks are reordered class-major
//      (and their probe counts prefix-summed) so that each class, and each pack
//      of consecutive light rows, owns one contiguous task range; light rows
//      are packed, heavy rows are cut into per-wave probe ranges.
#include <algorithm>
#include <memory>
#include <mutex>
#include <set>

#include "tc_prims.h"

namespace tc {

namespace {

constexpr int kT = 256;
inline unsigned grid_for(int64_t n) { return (unsigned)std::max<int64_t>(1, div_up(n, kT)); }

// Elementwise gathers take 2 * kEw elements per thread, issued together
// (more bytes in flight per wave).
constexpr int kEw = 4;
// Grid of a key producer that also counts digits (grid-stride loop; one LDS
// histogram flush per work-group).
constexpr unsigned kProducerBlocks = 2048;

// The dedup sort's source: raw pair i as its canonical key (lo << s | hi),
// or the sentinel for a self loop or an id outside [0, n) (the digit
// counting kernel reports the latter).
struct CanonSrc {
  const int32_t* src;
  const int32_t* dst;
  int64_t n;
  int s;
  uint64_t sent;
  __device__ uint64_t key(int64_t i, bool& bad) const {
    const int64_t u = src[i], v = dst[i];
    bad = (u < 0) | (u >= n) | (v < 0) | (v >= n);
    const uint64_t lo = (uint64_t)(u < v ? u : v), hi = (uint64_t)(u < v ? v : u);
    return (bad | (u == v)) ? sent : ((lo << s) | hi);
  }
  __device__ bool operator()(int64_t i, uint64_t& k, char&) const {
    bool bad;
    k = key(i, bad);
    return true;
  }
};

// Digit counts of the canonical keys for every pass of the dedup sort, and
// the id check, in one read of the raw pairs (grid-stride, kDigitBatch pairs
// in flight per thread; one LDS histogram flush per work-group).
__global__ __launch_bounds__(256) void k_canon_digits(CanonSrc cs, int64_t m, int key_bits,
                                                      uint32_t* __restrict__ ghist, int* __restrict__ err) {
  extern __shared__ uint32_t h_dyn[];
  DigitCounter dc;
  dc.init(h_dyn, 0, key_bits);
  bool bad_any = false;
  const int64_t stride = (int64_t)gridDim.x * 256 * kDigitBatch;
  for (int64_t base = (int64_t)blockIdx.x * 256 * kDigitBatch + threadIdx.x; base < m; base += stride) {
    uint64_t k[kDigitBatch];
#pragma unroll
    for (int j = 0; j < kDigitBatch; ++j) {
      const int64_t i = base + (int64_t)j * 256;
      bool bad;
      k[j] = cs.key(i < m ? i : m - 1, bad);  // (no branch around the loads)
      bad_any |= bad;
    }
#pragma unroll
    for (int j = 0; j < kDigitBatch; ++j) {
      if (base + (int64_t)j * 256 >= m) break;
      dc.add(k[j]);
    }
  }
  if (bad_any) atomicOr(err, 1);
  dc.flush(ghist);
}

// Distinct keys of the sorted canonical keys S (duplicates adjacent, the
// sentinel for dropped self loops last): position i holds one iff S[i] is
// not the sentinel and differs from S[i - 1]. The distinct keys are never
// written out. k_distinct_mark finds them by comparing neighbours and marks
// every other key with bit 63 (keys take at most 62 bits: s <= 31); later
// readers (the degree count, its partition and the orientation) then select
// a key by its own word alone (DistinctSel) and mask the mark off where
// they use an unselected key's bits.
constexpr uint64_t kDupMark = 1ull << 63;

struct DistinctSel {
  const uint64_t* S;
  uint64_t sent;
  __device__ bool operator()(int64_t i, uint64_t& k) const {
    k = S[i];
    return ((k & kDupMark) == 0) & (k != sent);
  }
};

// The degree partition's source: the upper endpoint of each distinct key.
struct DistinctHiSrc {
  DistinctSel d;
  int s;
  __device__ bool operator()(int64_t i, uint32_t& hi, char&) const {
    uint64_t k;
    const bool ok = d(i, k);
    hi = (uint32_t)(k & ((1ull << s) - 1));
    return ok;
  }
};

// Distinct keys of S marked (see above) and counted, with the digit counts
// of their upper endpoints for the degree partition's passes (bits
// [bit_lo, s)), in one read of S. A neighbour may have marked S[i - 1]
// already: keys are compared with the mark masked off.
__global__ __launch_bounds__(256) void k_distinct_mark(uint64_t* __restrict__ S, uint64_t sent, int64_t m_raw,
                                                       int bit_lo, int s, uint32_t* __restrict__ ghist,
                                                       unsigned long long* __restrict__ total) {
  extern __shared__ uint32_t h_dyn[];
  __shared__ uint32_t s_c;
  if (threadIdx.x == 0) s_c = 0;
  DigitCounter dc;
  dc.init(h_dyn, bit_lo, s);  // (ends with a barrier)
  uint32_t c = 0;
  const uint64_t mask = (1ull << s) - 1;
  const int64_t stride = (int64_t)gridDim.x * 256 * kDigitBatch;
  for (int64_t base = (int64_t)blockIdx.x * 256 * kDigitBatch + threadIdx.x; base < m_raw; base += stride) {
    uint64_t k[kDigitBatch], prev[kDigitBatch];
#pragma unroll
    for (int j = 0; j < kDigitBatch; ++j) {
      const int64_t i = base + (int64_t)j * 256;
      const int64_t ic = i < m_raw ? i : m_raw - 1;
      k[j] = S[ic];
      prev[j] = S[ic > 0 ? ic - 1 : 0];
    }
#pragma unroll
    for (int j = 0; j < kDigitBatch; ++j) {
      const int64_t i = base + (int64_t)j * 256;
      if (i < m_raw && k[j] != sent) {
        if (i == 0 || (prev[j] & ~kDupMark) != k[j]) {
          dc.add((uint32_t)(k[j] & mask));
          ++c;
        } else {
          S[i] = k[j] | kDupMark;
        }
      }
    }
  }
  if (c) atomicAdd(&s_c, c);
  dc.flush(ghist);  // (starts with a barrier: s_c is complete)
  if (threadIdx.x == 0 && s_c) atomicAdd(total, (unsigned long long)s_c);
}

// Entry i of U (row a, column b) starts a task iff U_a has entries after i
// and U_b is not empty (one bit per row); the task's key is b and its value
// the probe range [i + 1, row end of a).
struct TaskPred {
  const uint64_t* okey;
  int s;
  const int64_t* row_ptr;
  const uint64_t* nonempty;
  uint32_t* tkey;
  uint64_t* tval;
  struct Item {
    uint32_t b, end;
  };
  __device__ bool operator()(int64_t i, Item& it) const {
    const uint64_t k = okey[i];
    const int64_t a = (int64_t)(k >> s);
    it.b = (uint32_t)(k & ((1ull << s) - 1));
    it.end = (uint32_t)row_ptr[a + 1];
    // (no short circuit: the loads of several entries can then be in flight)
    return ((int64_t)it.end - i - 1 > 0) & (bool)((nonempty[it.b >> 6] >> (it.b & 63)) & 1ull);
  }
  __device__ void emit(int64_t i, const Item& it, uint32_t pos) const {
    tkey[pos] = it.b;
    tval[pos] = (uint64_t)(i + 1) | ((uint64_t)it.end << 32);
  }
};

// The task sort's source: entry i of U gives the task (key b, value first
// probe | end << 32) when TaskPred selects it.
struct TaskSrc {
  TaskPred p;
  __device__ bool operator()(int64_t i, uint32_t& b, uint64_t& v) const {
    TaskPred::Item it;
    const bool ok = p(i, it);
    b = it.b;
    v = (uint64_t)(i + 1) | ((uint64_t)it.end << 32);
    return ok;
  }
};

// Tasks of U counted, with the digit counts of their keys for every pass of
// the task sort, in one read of U (grid-stride, kDigitBatch entries in
// flight per thread; one LDS histogram flush and one count per work-group).
__global__ __launch_bounds__(256) void k_task_digits(TaskSrc src, int64_t m, int key_bits,
                                                     uint32_t* __restrict__ ghist, uint32_t* __restrict__ total) {
  extern __shared__ uint32_t h_dyn[];
  __shared__ uint32_t s_c;
  if (threadIdx.x == 0) s_c = 0;
  DigitCounter dc;
  dc.init(h_dyn, 0, key_bits);  // (ends with a barrier)
  uint32_t c = 0;
  const int64_t stride = (int64_t)gridDim.x * 256 * kDigitBatch;
  for (int64_t base = (int64_t)blockIdx.x * 256 * kDigitBatch + threadIdx.x; base < m; base += stride) {
    uint32_t b[kDigitBatch];
    bool ok[kDigitBatch];
#pragma unroll
    for (int j = 0; j < kDigitBatch; ++j) {
      const int64_t i = base + (int64_t)j * 256;
      uint64_t v;
      ok[j] = src(i < m ? i : m - 1, b[j], v) & (i < m);  // (no branch around the loads)
    }
#pragma unroll
    for (int j = 0; j < kDigitBatch; ++j) {
      if (ok[j]) {
        dc.add(b[j]);
        ++c;
      }
    }
  }
  if (c) atomicAdd(&s_c, c);
  dc.flush(ghist);  // (starts with a barrier: s_c is complete)
  if (threadIdx.x == 0 && s_c) atomicAdd(total, s_c);
}

// Bit r of the bitmap: row r of a CSR is not empty.
__global__ __launch_bounds__(256) void k_nonempty_bits(const int64_t* __restrict__ row_ptr, int64_t n,
                                                       uint64_t* __restrict__ bits) {
  const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const uint64_t b = __ballot(r < n && row_ptr[r + 1] > row_ptr[r]);
  if (lane_id() == 0 && r < n) bits[r >> 6] = b;
}

__global__ void k_fill_u32(uint32_t* p, int64_t n, uint32_t v) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = v;
}

__global__ void k_fill_i64(int64_t* p, int64_t n, int64_t v) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = v;
}

// deg(v) = (edges whose lower endpoint is v) + (edges whose upper endpoint is
// v). The upper endpoints arrive partitioned by their top bits (bucket = v >>
// hshift; bucket j at [start(j), start(j + 1)), start(j) = bs32[j] or bs64[j]
// for j < nbs, m beyond). Each work-group counts one range [v0, v1) of at
// most kDegBins vertices of one bucket in LDS: the upper endpoints from that
// bucket's entries, the lower endpoints from the distinct keys of S in
// [v0 << s, v1 << s) (S is sorted by lower endpoint; the range is found by
// binary search), with kDegBatch loads in flight per thread before they are
// counted. It writes the rank keys deg(v) << s | v of its vertices.
constexpr int kDegBins = 32768;   // LDS counters of one work-group (128 KiB)
constexpr int kDegThreads = 1024;
constexpr int kDegBatch = 8;

// First position of the sorted S[0, n) whose key (duplicate mark masked
// off) is >= x.
__device__ int64_t lower_bound_u64(const uint64_t* __restrict__ S, int64_t n, uint64_t x) {
  int64_t lo = 0, hi = n;
  while (lo < hi) {
    const int64_t mid = (lo + hi) >> 1;
    if ((S[mid] & ~kDupMark) < x) lo = mid + 1;
    else hi = mid;
  }
  return lo;
}

__global__ __launch_bounds__(kDegThreads) void k_degree_hist(const uint32_t* __restrict__ hi,
                                                             const uint32_t* __restrict__ bs32,
                                                             const int64_t* __restrict__ bs64, int64_t nbs, int64_t m,
                                                             int hshift, int sub, DistinctSel d, int64_t m_raw,
                                                             int64_t n, int s, uint64_t* __restrict__ rk) {
  extern __shared__ uint32_t h_deg[];
  __shared__ int64_t s_r[2];
  const uint32_t bucket = blockIdx.x / (uint32_t)sub, part = blockIdx.x % (uint32_t)sub;
  const int64_t v0 = ((int64_t)bucket << hshift) + (int64_t)part * kDegBins;
  const int64_t span_end = (int64_t)(bucket + 1) << hshift;
  const int64_t v1 = std::min(std::min(v0 + kDegBins, span_end), n);
  if (v0 >= v1) return;  // (uniform per work-group)
  const int nv = (int)(v1 - v0);
  for (int j = threadIdx.x; j < nv; j += blockDim.x) h_deg[j] = 0;
  if (threadIdx.x < 2) s_r[threadIdx.x] = lower_bound_u64(d.S, m_raw, (uint64_t)(threadIdx.x ? v1 : v0) << s);
  __syncthreads();
  // upper endpoints
  auto start = [&](int64_t j) -> int64_t { return j >= nbs ? m : bs64 ? bs64[j] : (int64_t)bs32[j]; };
  const int64_t e0 = start(bucket), e1 = start((int64_t)bucket + 1);
  for (int64_t base = e0 + threadIdx.x; base < e1; base += (int64_t)blockDim.x * kDegBatch) {
    uint32_t v[kDegBatch];
#pragma unroll
    for (int b = 0; b < kDegBatch; ++b) {
      const int64_t i = base + (int64_t)b * blockDim.x;
      v[b] = i < e1 ? hi[i] : 0xFFFFFFFFu;
    }
#pragma unroll
    for (int b = 0; b < kDegBatch; ++b) {
      const int64_t x = (int64_t)v[b];  // (the fill value is past every range)
      if (x >= v0 && x < v1) atomicAdd(&h_deg[x - v0], 1u);
    }
  }
  // lower endpoints: the distinct keys among S[r0, r1) all have lo in [v0, v1).
  // A wave's 64 consecutive positions hold runs of equal lo (S is sorted):
  // the first lane of each run adds the run's distinct keys with one atomic
  // (one atomic per lane would serialise on a high-degree vertex's counter).
  const int64_t r0 = s_r[0], r1 = s_r[1];
  const int lane = threadIdx.x & 63;
  const uint64_t below = (1ull << lane) - 1ull;  // lanes before this one
  // (wb, a wave's first position, is uniform across the wave: every lane
  // takes part in the ballots; lanes past r1 read S[r1 - 1] and select nothing)
  for (int64_t wb = r0 + (int64_t)(threadIdx.x - lane) * kDegBatch; wb < r1;
       wb += (int64_t)blockDim.x * kDegBatch) {
    uint64_t k[kDegBatch];
    bool ok[kDegBatch];
#pragma unroll
    for (int b = 0; b < kDegBatch; ++b) {
      const int64_t i = wb + (int64_t)b * 64 + lane;
      ok[b] = d(i < r1 ? i : r1 - 1, k[b]) & (i < r1);
    }
#pragma unroll
    for (int b = 0; b < kDegBatch; ++b) {
      const uint32_t lo = (uint32_t)((k[b] & ~kDupMark) >> s);
      const uint32_t prev = (uint32_t)__shfl_up((int)lo, 1);
      const uint64_t heads = __ballot(lane == 0 || prev != lo);
      const uint64_t oks = __ballot(ok[b]);
      if ((heads >> lane) & 1ull) {
        const uint64_t after = heads & ~below & ~(1ull << lane);  // later heads
        const uint64_t run = (after ? (after & (~after + 1ull)) - 1ull : ~0ull) & ~below;
        const uint32_t c = (uint32_t)__popcll(oks & run);
        if (c) atomicAdd(&h_deg[(int64_t)lo - v0], c);
      }
    }
  }
  __syncthreads();
  for (int j = threadIdx.x; j < nv; j += blockDim.x) {
    const int64_t v = v0 + j;
    rk[v] = ((uint64_t)h_deg[j] << s) | (uint64_t)v;
  }
}

__global__ void k_rank_keys(const uint32_t* __restrict__ deg, int64_t n, int s,
                            uint64_t* __restrict__ rk) {
  int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (v < n) rk[v] = ((uint64_t)deg[v] << s) | (uint64_t)v;
}

__global__ void k_perm(const uint64_t* __restrict__ rk, int64_t n, int s, int32_t* __restrict__ perm) {
  int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (r < n) perm[rk[r] & ((1ull << s) - 1)] = (int32_t)r;
}

// Orientation in two steps, so that no rank is read at random from the
// whole rank map. (1) One radix pass partitions the distinct edges by the
// top 8 bits of their upper endpoint (the last digit pass of the degree
// count's partition, whose scanned digit starts it reuses); its source reads
// S in order, so the lower endpoints' ranks are read in nondecreasing vertex
// order: element = rank(lo) << 32 | hi. (2) k_orient_hi reads the ranks of
// the upper endpoints bucket by bucket (a bucket spans 2^(s-8) vertices: a
// 256 KiB slice of the rank map at s = 24, 1 MiB at s = 26, which stays in
// L2) and writes the oriented key in place.
struct LoRankSrc {
  DistinctSel d;
  const int32_t* perm;
  int s;
  __device__ bool operator()(int64_t i, uint64_t& k, char&) const {
    uint64_t e;
    const bool ok = d(i, e);
    // (an unselected position may hold the sentinel, whose lower endpoint
    // 2^s - 1 can lie past the rank map: read vertex 0 for it instead)
    k = ((uint64_t)(uint32_t)perm[ok ? e >> s : 0] << 32) | (e & ((1ull << s) - 1));
    return ok;
  }
};

// XCD-aware grid-stride sweep: work-groups are dealt to the 8 XCDs in turn,
// so work-group b sweeps the chunks of the b % 8-th eighth of [0, chunks)
// and each XCD's L2 holds the rank slices of its own eighth only. The grid
// is a multiple of 8.
__global__ __launch_bounds__(256) void k_orient_hi(uint64_t* __restrict__ pk, int64_t m, int s,
                                                   const int32_t* __restrict__ perm, uint32_t* __restrict__ hist) {
  extern __shared__ uint32_t h_dyn[];
  constexpr int kI = 2 * kEw;  // gathers: more in flight
  constexpr int64_t kChunk = (int64_t)kT * kI;
  DigitCounter dc;
  dc.init(h_dyn, 0, 2 * s);
  const uint64_t mask = (1ull << s) - 1;
  const int64_t chunks = (m + kChunk - 1) / kChunk;
  const int64_t per_xcd = (chunks + 7) / 8;
  const int64_t c0 = (int64_t)(blockIdx.x & 7) * per_xcd;
  const int64_t c1 = c0 + per_xcd < chunks ? c0 + per_xcd : chunks;
  for (int64_t c = c0 + (blockIdx.x >> 3); c < c1; c += gridDim.x >> 3) {
    const int64_t i0 = c * kChunk + threadIdx.x;
    uint64_t e[kI];
#pragma unroll
    for (int j = 0; j < kI; ++j) {
      const int64_t i = i0 + (int64_t)j * kT;
      e[j] = pk[i < m ? i : m - 1];
    }
    uint32_t rv[kI];
#pragma unroll
    for (int j = 0; j < kI; ++j) rv[j] = (uint32_t)perm[e[j] & mask];
#pragma unroll
    for (int j = 0; j < kI; ++j) {
      const int64_t i = i0 + (int64_t)j * kT;
      if (i < m) {
        const uint64_t a = e[j] >> 32, b = rv[j];
        const uint64_t k = a < b ? ((a << s) | b) : ((b << s) | a);
        pk[i] = k;
        dc.add(k);
      }
    }
  }
  dc.flush(hist);
}

// Column of a sorted orient key, written by the orient sort's last pass.
struct ColEpi {
  int32_t* col;
  int s;
  __device__ void operator()(uint64_t pos, uint64_t key) const {
    col[pos] = (int32_t)(key & ((1ull << s) - 1));
  }
};

__global__ void k_col(const uint64_t* __restrict__ okey, int64_t m, int s, int32_t* __restrict__ col) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < m) col[i] = (int32_t)(okey[i] & ((1ull << s) - 1));
}

// W+ = sum_a C(d+(a), 2) and max d+(a).
// Grids of the reducing kernels below: a few blocks per CU, each looping
// over its rows, so that the per-block global atomics stay few.
constexpr unsigned kReduceBlocks = 1024;
inline unsigned grid_reduce(int64_t n) { return (unsigned)std::min<int64_t>(kReduceBlocks, grid_for(n)); }

__global__ __launch_bounds__(256) void k_row_stats(const int64_t* __restrict__ row_ptr, int64_t n,
                                                   unsigned long long* __restrict__ wplus,
                                                   unsigned int* __restrict__ maxd) {
  __shared__ uint64_t s_w[4];
  __shared__ uint32_t s_m[4];
  uint64_t w = 0;
  uint32_t md = 0;
  for (int64_t a = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; a < n; a += (int64_t)gridDim.x * blockDim.x) {
    const uint64_t d = (uint64_t)(row_ptr[a + 1] - row_ptr[a]);
    w += d * (d - (d > 0)) / 2;
    md = max(md, (uint32_t)d);
  }
  w = wave_sum(w);
  md = wave_max(md);
  if (lane_id() == 0) {
    s_w[threadIdx.x >> 6] = w;
    s_m[threadIdx.x >> 6] = md;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    uint64_t tw = s_w[0] + s_w[1] + s_w[2] + s_w[3];
    uint32_t tm = max(max(s_m[0], s_m[1]), max(s_m[2], s_m[3]));
    if (tw) atomicAdd(wplus, (unsigned long long)tw);
    atomicMax(maxd, tm);
  }
}

// Class of every hashed row b (-1 = no work) and the class's largest table
// (maxima reduced per wave before one atomic per wave and class).
__global__ __launch_bounds__(256) void k_classify(const int64_t* __restrict__ tptr,
                                                  const uint64_t* __restrict__ tprefix,
                                                  const int64_t* __restrict__ row_ptr, int64_t n, bool all_rows,
                                                  uint64_t heavy_min, int8_t* __restrict__ cls,
                                                  int* __restrict__ cls_log2S,
                                                  unsigned long long* __restrict__ cls_probes) {
  __shared__ int s_max[NUM_CLASSES];
  __shared__ unsigned long long s_w[NUM_CLASSES];
  if (threadIdx.x < NUM_CLASSES) {
    s_max[threadIdx.x] = 0;
    s_w[threadIdx.x] = 0;
  }
  __syncthreads();
  int lmax[NUM_CLASSES];
  unsigned long long lw[NUM_CLASSES];
#pragma unroll
  for (int k = 0; k < NUM_CLASSES; ++k) {
    lmax[k] = 0;
    lw[k] = 0;
  }
  for (int64_t b = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; b < n; b += (int64_t)gridDim.x * blockDim.x) {
    int c = -1, l = 0;
    const uint64_t W = tprefix[tptr[b + 1]] - tprefix[tptr[b]];
    if (W > 0) {
      l = table_log2(row_ptr[b + 1] - row_ptr[b]);
      if (l > kMaxLog2S) c = CLS_GLOBAL;
      else if (l > 13) c = CLS_WG_GIANT;
      else if (l > 12) c = CLS_WG_HUGE;
      else if (W < heavy_min && l <= 10) c = l <= 8 ? CLS_PACK_SMALL : CLS_PACK_LARGE;
      else c = l <= 10 ? CLS_WG_SMALL : CLS_WG_LARGE;
    } else if (all_rows) {
      // no doubly sparse traversal: a row without work is still visited (a
      // pack member whose table stays empty: it has no task to look up)
      c = CLS_PACK_SMALL;
      l = table_log2(0);
    }
    cls[b] = (int8_t)c;
#pragma unroll
    for (int k = 0; k < NUM_CLASSES; ++k) {
      lmax[k] = c == k && l > lmax[k] ? l : lmax[k];
      lw[k] += c == k ? W : 0;
    }
  }
#pragma unroll
  for (int k = 0; k < NUM_CLASSES; ++k) {
    const int mk = wave_max(lmax[k]);
    const unsigned long long wk = wave_sum(lw[k]);
    if (lane_id() == 0 && mk > 0) atomicMax(&s_max[k], mk);
    if (lane_id() == 0 && wk > 0) atomicAdd(&s_w[k], wk);
  }
  __syncthreads();
  if (threadIdx.x < NUM_CLASSES && s_max[threadIdx.x] > 0) atomicMax(&cls_log2S[threadIdx.x], s_max[threadIdx.x]);
  if (threadIdx.x < NUM_CLASSES && s_w[threadIdx.x] > 0) atomicAdd(&cls_probes[threadIdx.x], s_w[threadIdx.x]);
}

// Per-class sums (rows, table keys, tasks, probes): LDS accumulation per
// block, one partial row per block, then a column reduction.
constexpr int kStatCols = NUM_CLASSES * 4;

__global__ __launch_bounds__(256) void k_class_stats(const int8_t* __restrict__ cls, int64_t n,
                                                     const uint32_t* __restrict__ tbeg,
                                                     const uint32_t* __restrict__ tend,
                                                     const uint64_t* __restrict__ tprefix,
                                                     const int64_t* __restrict__ row_ptr,
                                                     unsigned long long* __restrict__ partial) {
  __shared__ unsigned long long acc[kStatCols];
  if (threadIdx.x < kStatCols) acc[threadIdx.x] = 0;
  __syncthreads();
  for (int64_t b = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; b < n; b += (int64_t)gridDim.x * blockDim.x) {
    const int c = cls[b];
    if (c >= 0) {
      atomicAdd(&acc[c * 4 + 0], 1ull);
      atomicAdd(&acc[c * 4 + 1], (unsigned long long)(row_ptr[b + 1] - row_ptr[b]));
      atomicAdd(&acc[c * 4 + 2], (unsigned long long)(tend[b] - tbeg[b]));
      atomicAdd(&acc[c * 4 + 3], (unsigned long long)(tprefix[tend[b]] - tprefix[tbeg[b]]));
    }
  }
  __syncthreads();
  if (threadIdx.x < kStatCols) partial[(int64_t)blockIdx.x * kStatCols + threadIdx.x] = acc[threadIdx.x];
}

__global__ __launch_bounds__(256) void k_reduce_cols(const unsigned long long* __restrict__ partial,
                                                     int64_t rows, int cols,
                                                     unsigned long long* __restrict__ out) {
  __shared__ unsigned long long s_w[4];
  const int c = blockIdx.x;
  unsigned long long v = 0;
  for (int64_t r = threadIdx.x; r < rows; r += blockDim.x) v += partial[r * cols + c];
  v = wave_sum(v);
  if (lane_id() == 0) s_w[threadIdx.x >> 6] = v;
  __syncthreads();
  if (threadIdx.x == 0) out[c] = s_w[0] + s_w[1] + s_w[2] + s_w[3];
}

// Wave items of a heavy row with W probes: a multiple of the class's waves
// per work-group (each group of `waves` consecutive items shares one table).
__device__ __forceinline__ uint32_t wg_parts(uint64_t W, int waves, uint32_t chunk) {
  // (chunk >= kWaveChunkMin: per > 0)
  const uint64_t per = (uint64_t)waves * chunk;
  return (uint32_t)(waves * ((W + per - 1) / per));
}

// Rows with work (class >= 0): key = class, value = row (compacted in row
// order, then stably sorted by class: the class-major row order).
struct WorkRowPred {
  const int8_t* cls;
  uint32_t* key;
  uint32_t* row;
  struct Item {
    int8_t c;
  };
  __device__ bool operator()(int64_t b, Item& it) const {
    it.c = cls[b];
    return it.c >= 0;
  }
  __device__ void emit(int64_t b, const Item& it, uint32_t pos) const {
    key[pos] = (uint32_t)it.c;
    row[pos] = (uint32_t)b;
  }
};

// Per class-major row i (row b = crow[i]): its number of tasks, its probes
// W_b, and its wave items (item classes only).
struct CmTasks {
  const uint32_t* crow;
  const int64_t* tptr;
  __device__ uint32_t operator()(int64_t i) const {
    const uint32_t b = crow[i];
    return (uint32_t)(tptr[b + 1] - tptr[b]);
  }
};
struct CmProbes {
  const uint32_t* crow;
  const int64_t* tptr;
  const uint64_t* tprefix;
  __device__ uint64_t operator()(int64_t i) const {
    const uint32_t b = crow[i];
    return tprefix[tptr[b + 1]] - tprefix[tptr[b]];
  }
};
struct CmItems {
  const uint32_t* crow;
  const int8_t* cls;
  const int64_t* tptr;
  const uint64_t* tprefix;
  uint32_t chunk[NUM_CLASSES];
  __device__ uint32_t operator()(int64_t i) const {
    const uint32_t b = crow[i];
    const int c = cls[b];
    if (c == CLS_PACK_SMALL || c == CLS_PACK_LARGE) return 0;
    return wg_parts(tprefix[tptr[b + 1]] - tprefix[tptr[b]], class_waves(c), chunk[c]);
  }
};

// Task range of every row with work in the class-major task order, and the
// row's class-major position.
__global__ void k_cm_place(const uint32_t* __restrict__ crow, int64_t R, const uint32_t* __restrict__ tsc,
                           uint32_t* __restrict__ tbeg, uint32_t* __restrict__ tend,
                           uint32_t* __restrict__ cm_pos) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= R) return;
  const uint32_t b = crow[i];
  tbeg[b] = tsc[i];
  tend[b] = tsc[i + 1];
  cm_pos[b] = (uint32_t)i;
}

// Task t (hashed-row order) to its class-major slot: first probe and the
// class-major exclusive prefix (the row's base plus the prefix within the
// row, which keeps its order).
__global__ void k_task_permute(int64_t T, const uint32_t* __restrict__ tb_row,
                               const int64_t* __restrict__ tb_ptr, const uint64_t* __restrict__ tb_val,
                               const uint64_t* __restrict__ tb_prefix, const uint32_t* __restrict__ tbeg,
                               const uint32_t* __restrict__ cm_pos, const uint64_t* __restrict__ wsc,
                               uint32_t* __restrict__ tstart, uint64_t* __restrict__ tprefix) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= T) return;
  const uint32_t b = tb_row[t];
  const int64_t p0 = tb_ptr[b];
  const int64_t nt = (int64_t)tbeg[b] + (t - p0);
  tstart[nt] = (uint32_t)tb_val[t];
  tprefix[nt] = wsc[cm_pos[b]] + (tb_prefix[t] - tb_prefix[p0]);
}

// Values of a device array at NUM_CLASSES + 1 positions (class boundaries).
template <class T>
__global__ void k_gather_at(const T* __restrict__ a, const int64_t* __restrict__ at, int k, T* __restrict__ out) {
  if ((int)threadIdx.x < k) out[threadIdx.x] = a[at[threadIdx.x]];
}

__global__ void k_rows_work(const int32_t* __restrict__ rows, int64_t nr,
                            const uint32_t* __restrict__ tbeg, const uint32_t* __restrict__ tend,
                            const uint64_t* __restrict__ tprefix, const int64_t* __restrict__ row_ptr,
                            uint64_t* __restrict__ w, uint32_t* __restrict__ slots) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= nr) return;
  int64_t b = rows[i];
  w[i] = tprefix[tend[b]] - tprefix[tbeg[b]];
  // a row without tasks (visited only without the doubly sparse traversal)
  // needs no table
  slots[i] = 1u << pack_table_log2(tend[b] > tbeg[b] ? row_ptr[b + 1] - row_ptr[b] : 0);
}

// A pack starts at row i when the running probe total, the running table
// slots or the row index enters a new multiple of its budget; so a pack holds
// at most kPackRows rows, at most `slots` slots plus one row's table, and at
// most `target` probes plus one row's.
__global__ void k_pack_flags(const uint64_t* __restrict__ pw, const uint32_t* __restrict__ ps,
                             int64_t nr, uint64_t target, uint32_t slots, uint32_t* __restrict__ flags) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= nr) return;
  flags[i] = (i == 0 || pw[i] / target != pw[i - 1] / target || ps[i] / slots != ps[i - 1] / slots ||
              i / kPackRows != (i - 1) / kPackRows)
                 ? 1u
                 : 0u;
}

// Records of the pack rows (one thread per row) and of the packs (one thread
// per pack: probe range and each wave share's first task, by binary search in
// the pack's task prefixes).
__global__ void k_pack_recs(const int32_t* __restrict__ rows, int64_t nr, const int64_t* __restrict__ row_ptr,
                            const uint32_t* __restrict__ tbeg, const uint32_t* __restrict__ tend,
                            PackRow* __restrict__ recs) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= nr) return;
  const int32_t b = rows[i];
  PackRow r;
  r.rs = (uint32_t)row_ptr[b];
  r.tb = tbeg[b];
  r.te = tend[b];
  r.d = r.te > r.tb ? (uint32_t)(row_ptr[b + 1] - row_ptr[b]) : 0u;
  recs[i] = r;
}

__global__ void k_pack_info(const uint32_t* __restrict__ pack_ptr, int64_t np, const PackRow* __restrict__ recs,
                            const uint64_t* __restrict__ tprefix, PackInfo* __restrict__ info) {
  const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= np) return;
  PackInfo pi;
  pi.r0 = pack_ptr[p];
  pi.r1 = pack_ptr[p + 1];
  const uint32_t t_lo = recs[pi.r0].tb, t_hi = recs[pi.r1 - 1].te;
  pi.q0 = tprefix[t_lo];
  pi.q1 = tprefix[t_hi];
  const uint64_t W = pi.q1 - pi.q0;
  for (int w = 0; w < kWaves; ++w) {
    const uint64_t wq0 = pi.q0 + W * (uint64_t)w / kWaves;
    // last task t in [t_lo, t_hi) with tprefix[t] <= wq0 (t_lo when the pack
    // has no task: the share is then empty and never probed)
    uint32_t lo = t_lo, hi = t_hi > t_lo ? t_hi : t_lo + 1;
    while (hi - lo > 1) {
      const uint32_t mid = lo + (hi - lo) / 2;
      if (tprefix[mid] <= wq0) lo = mid;
      else hi = mid;
    }
    pi.wt[w] = lo;
  }
  info[p] = pi;
}

// Launch order of a class's packs: heaviest first (longest-processing-time
// order), so that the launch does not end on a few long packs. Classes of
// fewer than kPackLptMin packs keep pack order (their launch is short; the
// sort would cost more than it saves, and batch plans order units themselves).
// Key = the complement of the pack's weight (its probes plus 64 per row), so
// that an ascending sort puts the heaviest first.
constexpr int64_t kPackLptMin = 2048;
__global__ void k_pack_keys(const PackInfo* __restrict__ info, int64_t np, uint32_t* __restrict__ key,
                            uint32_t* __restrict__ idx) {
  const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= np) return;
  const uint64_t w = info[p].q1 - info[p].q0 + 64ull * (info[p].r1 - info[p].r0);
  key[p] = 0xFFFFFFFFu - (uint32_t)(w < 0xFFFFFFFFull ? w : 0xFFFFFFFFull);
  idx[p] = (uint32_t)p;
}

__global__ void k_pack_gather(const PackInfo* __restrict__ in, const uint32_t* __restrict__ idx, int64_t np,
                              PackInfo* __restrict__ out) {
  const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (p < np) out[p] = in[idx[p]];
}

__global__ void k_pack_emit(const uint32_t* __restrict__ flags, const uint32_t* __restrict__ pos,
                            int64_t nr, uint32_t* __restrict__ pack_ptr, int64_t np) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < nr && flags[i]) pack_ptr[pos[i]] = (uint32_t)i;
  if (i == 0) pack_ptr[np] = (uint32_t)nr;
}

// One thread per wave item of a work-group class: find its row b (upper bound
// in the per-row item offsets), cut the row's probe range evenly and find the
// task holding the first probe.
// Wave items of the nr class-major rows crow[0..nr) of one class: offs
// (nr + 1 entries, absolute) is the exclusive prefix of their item counts;
// item j (0 <= j < total) is part idx of the row whose range holds offs[0] + j.
__global__ void k_emit_items(const uint32_t* __restrict__ offs, const uint32_t* __restrict__ crow, int64_t nr,
                             int64_t total, const uint32_t* __restrict__ tbeg,
                             const uint32_t* __restrict__ tend, const uint64_t* __restrict__ tprefix,
                             const int64_t* __restrict__ row_ptr, CountItem* __restrict__ items) {
  const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= total) return;
  const int64_t target = (int64_t)offs[0] + j;
  // largest r with offs[r] <= target (every row has at least one item)
  int64_t lo = 0, hi = nr;  // invariant offs[lo] <= target < offs[hi]
  while (hi - lo > 1) {
    const int64_t mid = (lo + hi) >> 1;
    if ((int64_t)offs[mid] <= target) lo = mid;
    else hi = mid;
  }
  const int64_t b = crow[lo];
  const uint64_t parts = offs[lo + 1] - offs[lo];
  const uint64_t idx = (uint64_t)(target - (int64_t)offs[lo]);
  const int64_t t_lo = tbeg[b], t_hi = tend[b];
  const uint64_t P0 = tprefix[t_lo];
  const uint64_t W = tprefix[t_hi] - P0;
  const uint64_t per = W / parts, extra = W % parts;
  const uint64_t q0 = P0 + per * idx + (idx < extra ? idx : extra);
  const uint64_t q1 = q0 + per + (idx < extra ? 1 : 0);
  // task t in [t_lo, t_hi) with tprefix[t] <= q0 < tprefix[t+1]
  int64_t a = t_lo, z = t_hi;  // tprefix[a] <= q0 < tprefix[z] (if q0 < end)
  while (z - a > 1) {
    int64_t mid = (a + z) >> 1;
    if (tprefix[mid] <= q0) a = mid;
    else z = mid;
  }
  CountItem it;
  it.b = (int32_t)b;
  it.t0 = (uint32_t)a;
  it.q0 = q0;
  it.len = (uint32_t)(q1 - q0);
  it.log2S = (uint32_t)table_log2(row_ptr[b + 1] - row_ptr[b]);
  items[j] = it;
}

}  // namespace

struct GraphImpl : Graph {
  Owned owned;
};

void destroy_graph_idle(Graph* g) {
  GraphImpl* gi = static_cast<GraphImpl*>(g);
  gi->owned.release(true);
  delete gi;
}

void destroy_graph(Graph* g) {
  // work on the graph may still be queued on the streams that used it: the
  // memory goes back to the cache, reusable once that work is done
  GraphImpl* gi = static_cast<GraphImpl*>(g);
  gi->uses.release_after_uses(gi->owned);
  delete gi;
}

Graph* build_graph(const int32_t* d_src, const int32_t* d_dst, int64_t m_raw, int64_t n,
                   hipStream_t st) {
  std::unique_ptr<GraphImpl> g(new GraphImpl());
  g->owned.st = st;
  TC_HIP(hipGetDevice(&g->device));
  TempStream temps(st);  // temporaries are stream-ordered on st
  g->n = n;
  g->m_raw = m_raw;
  const int s = std::max(1, ceil_log2_u64((uint64_t)n));
  g->sbits = s;
  const uint64_t sent = (2 * s >= 64) ? ~0ull : ((1ull << (2 * s)) - 1);

  // Everything below that starts at zero, in one buffer cleared by one
  // memset: 64 bytes of scalars (id error (int) at 0, distinct count m
  // (u64) at 8, W+ (u64) at 16, largest d+ (u32) at 24, task count (u32) at
  // 28: two host reads of 16 bytes), then the digit counts of the degree
  // partition (2 x 256), of the canonical keys, of the oriented keys and of
  // the tasks (kSortPassesMax x 256 each).
  constexpr size_t kHistWords = 256 * kSortPassesMax;
  DevBuf zs(64 + sizeof(uint32_t) * (256 * 2 + 3 * kHistWords));
  TC_HIP(hipMemsetAsync(zs.p, 0, zs.bytes, st));
  char* const zb = zs.as<char>();
  int* d_err = reinterpret_cast<int*>(zb);
  unsigned long long* d_m = reinterpret_cast<unsigned long long*>(zb + 8);
  unsigned long long* d_wplus = reinterpret_cast<unsigned long long*>(zb + 16);
  unsigned int* d_maxd = reinterpret_cast<unsigned int*>(zb + 24);
  uint32_t* d_T = reinterpret_cast<uint32_t*>(zb + 28);
  uint32_t* const dh = reinterpret_cast<uint32_t*>(zb + 64);
  uint32_t* const ch = dh + 256 * 2;
  uint32_t* const ohist = ch + kHistWords;
  uint32_t* const th = ohist + kHistWords;

  // ---- 1-2: simple graph -------------------------------------------------
  // The canonical keys are sorted (duplicates adjacent, self loops as the
  // sentinel, which sorts last) into S; the distinct keys are never written
  // out: the degree count, its partition and the orientation select them
  // from S (DistinctSel). The other sort buffer later holds the oriented
  // keys, and S's buffer is the orient sort's ping-pong partner.
  int64_t m = 0;
  DevBuf ka(sizeof(uint64_t) * (size_t)std::max<int64_t>(m_raw, 1));
  DevBuf kb(sizeof(uint64_t) * (size_t)std::max<int64_t>(m_raw, 1));
  bool salt = false;  // S is in kb
  // degree partition: one radix pass (8 bits) up to s = 24 (a bucket then
  // spans at most 2 LDS ranges, each reading the bucket's entries), two
  // beyond; dh: its digit counts, which the sort scans into digit starts
  // (the bucket starts of the degree count; the last pass's are reused by
  // the orientation's partition)
  const int hshift = s <= 8 ? 0 : s <= 24 ? s - 8 : s - 16;
  const int hpasses = digit_passes(hshift, s);
  {
    // canonical keys are built by the first pass of the dedup sort from the
    // raw pairs (7168-pair tiles: the largest whose registers allow two
    // waves per SIMD); one read of the pairs before it counts their digits
    // and checks the ids
    const CanonSrc csrc{d_src, d_dst, n, s, sent};
    if (m_raw > 0) {
      TC_LAUNCH("canon_digits", k_canon_digits,
                dim3((unsigned)std::min<int64_t>(kProducerBlocks, div_up(m_raw, kT * kDigitBatch))), dim3(kT),
                digit_lds_bytes(0, 2 * s), st, csrc, m_raw, 2 * s, ch, d_err);
      TC_HIP(hipGetLastError());
      salt = radix_sort_from<uint64_t, NoVal, CanonSrc, 28>(csrc, m_raw, ka.as<uint64_t>(), kb.as<uint64_t>(),
                                                            nullptr, nullptr, m_raw, 0, 2 * s, ch,
                                                            st, "dedup");
      // duplicates marked, distinct keys counted, with their upper
      // endpoints' partition digits
      TC_LAUNCH("distinct_mark", k_distinct_mark,
                dim3((unsigned)std::min<int64_t>(kProducerBlocks, div_up(m_raw, kT * kDigitBatch))), dim3(kT),
                digit_lds_bytes(hshift, s), st, salt ? kb.as<uint64_t>() : ka.as<uint64_t>(), sent, m_raw, hshift,
                s, dh, d_m);
      TC_HIP(hipGetLastError());
    }
    // the id check and the distinct count: one host sync for both
    struct {
      int err;
      int pad;
      unsigned long long m;
    } h;
    static_assert(sizeof(h) == 16, "scalar layout");
    TC_HIP(hipMemcpyAsync(&h, zb, sizeof(h), hipMemcpyDeviceToHost, st));
    TC_HIP(hipStreamSynchronize(st));
    const unsigned long long h_m = h.m;
    TC_REQUIRE(h.err == 0, TC_EINVAL, "tc_preprocess: vertex id outside [0, n)");
    TC_REQUIRE(h_m < (unsigned long long)kMaxEdges, TC_EOVERFLOW, "tc_preprocess: 2^32 - 256 or more edges");
    m = (int64_t)h_m;
  }
  g->m = m;
  DevBuf& sbuf = salt ? kb : ka;     // S
  DevBuf& obuf = salt ? ka : kb;     // free: the oriented keys go here
  const DistinctSel dsel{sbuf.as<uint64_t>(), sent};

  // ---- 3: degree order ---------------------------------------------------
  g->perm = g->owned.alloc<int32_t>(n);
  const uint32_t* hi_starts = dh + 256 * (hpasses - 1);  // valid once m > 0
  {
    DevBuf ra(sizeof(uint64_t) * (size_t)n), rb(sizeof(uint64_t) * (size_t)n);
    if (m > 0) {
      // upper endpoints partitioned by their top bits (read from S through
      // the distinct keys) and counted per bucket in LDS with the lower
      // endpoints (k_degree_hist, which writes the rank keys)
      DevBuf hb(sizeof(uint32_t) * (size_t)m), hb2(hpasses > 1 ? sizeof(uint32_t) * (size_t)m : 0);
      const bool halt = radix_sort_from<uint32_t, NoVal>(DistinctHiSrc{dsel, s}, m_raw, hb.as<uint32_t>(),
                                                         hb2.as<uint32_t>(), nullptr, nullptr, m, hshift, s,
                                                         dh, st, "degree");
      const uint32_t* hsorted = halt ? hb2.as<uint32_t>() : hb.as<uint32_t>();
      const int64_t span = (int64_t)1 << hshift;  // vertices per bucket
      const int sub = (int)div_up(span, kDegBins);
      const int64_t nbuckets = div_up(n, span);
      const int64_t groups = nbuckets * sub;
      const size_t lds = sizeof(uint32_t) * kDegBins;
      {
        // (the attribute is set once per device)
        static std::mutex mu;
        static std::set<int> done;
        std::lock_guard<std::mutex> lk(mu);
        if (!done.count(g->device)) {
          TC_HIP(hipFuncSetAttribute((const void*)k_degree_hist, hipFuncAttributeMaxDynamicSharedMemorySize,
                                     (int)lds));
          done.insert(g->device);
        }
      }
      // bucket starts: with one digit pass, its digit starts as the sort
      // scanned them (256 exclusive starts); else found by binary search
      DevBuf bp;
      const uint32_t* bs32 = dh;
      int64_t nbs = 256;
      if (hpasses != 1) {
        bp.alloc(sizeof(int64_t) * (size_t)(nbuckets + 1));
        TC_LAUNCH("bounds", (k_bounds<uint32_t>), dim3(grid_for(nbuckets + 1)), dim3(kT), 0, st, hsorted, m,
                  hshift, nbuckets, bp.as<int64_t>());
        bs32 = nullptr;
        nbs = nbuckets + 1;
      }
      TC_LAUNCH("degree_hist", k_degree_hist, dim3((unsigned)groups), dim3(kDegThreads), lds, st, hsorted, bs32,
                bs32 ? nullptr : bp.as<int64_t>(), nbs, m, hshift, sub, dsel, m_raw, n, s, ra.as<uint64_t>());
      TC_HIP(hipGetLastError());
    } else {
      DevBuf deg(sizeof(uint32_t) * (size_t)n);
      TC_LAUNCH("fill_u32", k_fill_u32, dim3(grid_for(n)), dim3(kT), 0, st, deg.as<uint32_t>(), n, 0u);
      TC_LAUNCH("rank_keys", k_rank_keys, dim3(grid_for(n)), dim3(kT), 0, st, deg.as<uint32_t>(), n, s,
                ra.as<uint64_t>());
      TC_HIP(hipGetLastError());
    }
    bool alt = radix_sort<uint64_t, NoVal>(ra.as<uint64_t>(), rb.as<uint64_t>(), nullptr, nullptr, n,
                                           s, 2 * s, st, "rank");
    TC_LAUNCH("perm", k_perm, dim3(grid_for(n)), dim3(kT), 0, st,
                       alt ? rb.as<uint64_t>() : ra.as<uint64_t>(), n, s, g->perm);
    TC_HIP(hipGetLastError());
  }

  // ---- 4: orient, U in CSR -------------------------------------------------
  g->row_ptr = g->owned.alloc<int64_t>(n + 1);
  g->col = g->owned.alloc<int32_t>(m);
  const uint64_t* okey = obuf.as<uint64_t>();
  {
    if (m > 0) {
      // partition by the top 8 bits of hi (one pass from S into the free
      // buffer), then the oriented keys in place
      // (28 edges per thread, as the canonicalising pass: a source that
      // loads twice per element needs the registers)
      const bool palt = radix_sort_from<uint64_t, NoVal, LoRankSrc, 28>(
          LoRankSrc{dsel, g->perm, s}, m_raw, obuf.as<uint64_t>(), nullptr, nullptr, nullptr, m,
          s > 8 ? s - 8 : 0, s, const_cast<uint32_t*>(hi_starts), st, "orient_part", NoEpi{}, true);
      TC_REQUIRE(!palt, TC_EDEVICE, "tc_preprocess: the orientation partition is one pass");
      const int64_t og = std::min<int64_t>(kProducerBlocks, div_up(m, kT * 2 * kEw));
      TC_LAUNCH("orient", k_orient_hi, dim3((unsigned)(div_up(og, 8) * 8)), dim3(kT), digit_lds_bytes(0, 2 * s),
                st, obuf.as<uint64_t>(), m, s, g->perm, ohist);
      TC_HIP(hipGetLastError());
      // S's buffer is the ping-pong partner (S is not read after the
      // partition); the last pass also writes each key's column: U's col
      bool alt = radix_sort<uint64_t, NoVal, ColEpi>(obuf.as<uint64_t>(), sbuf.as<uint64_t>(), nullptr, nullptr,
                                                     m, 0, 2 * s, st, "orient", ColEpi{g->col, s},
                                                     ohist);
      if (alt) okey = sbuf.as<uint64_t>();
      TC_LAUNCH("bounds", (k_bounds<uint64_t>), dim3(grid_for(n + 1)), dim3(kT), 0, st, okey, m, s, n,
                         g->row_ptr);
      if (m == 1)  // no sort pass ran
        TC_LAUNCH("col", k_col, dim3(grid_for(m)), dim3(kT), 0, st, okey, m, s, g->col);
    } else {
      TC_LAUNCH("fill_i64", k_fill_i64, dim3(grid_for(n + 1)), dim3(kT), 0, st, g->row_ptr, n + 1,
                         (int64_t)0);
    }
    TC_LAUNCH("row_stats", k_row_stats, dim3(grid_reduce(n)), dim3(kT), 0, st, g->row_ptr, n, d_wplus,
              d_maxd);
    TC_HIP(hipGetLastError());
  }
  // the buffer that does not hold the oriented keys is free now
  (okey == sbuf.as<uint64_t>() ? obuf : sbuf).release();
  // (W+ and the largest d+ are read back with the task count below: one
  // host sync)

  // ---- 5: tasks grouped by hashed row b -----------------------------------
  // one read of U counts the tasks and their key digits; the first pass of
  // the task sort reads U again and builds the tasks it ranks (no task list
  // is written in U order)
  TaskLists tl;
  {
    DevBuf ne;
    TaskSrc src{};
    if (m > 0) {
      ne.alloc(sizeof(uint64_t) * (size_t)div_up(n, 64));
      TC_LAUNCH("nonempty_bits", k_nonempty_bits, dim3(grid_for(n)), dim3(kT), 0, st, g->row_ptr, n,
                ne.as<uint64_t>());
      src.p = TaskPred{okey, s, g->row_ptr, ne.as<uint64_t>(), nullptr, nullptr};
      TC_LAUNCH("task_digits", k_task_digits,
                dim3((unsigned)std::min<int64_t>(kProducerBlocks, div_up(m, kT * kDigitBatch))), dim3(kT),
                digit_lds_bytes(0, s), st, src, m, s, th, d_T);
      TC_HIP(hipGetLastError());
    }
    struct {
      unsigned long long wplus;
      unsigned int maxd;
      uint32_t T;
    } h;
    static_assert(sizeof(h) == 16, "scalar layout");
    TC_HIP(hipMemcpyAsync(&h, zb + 16, sizeof(h), hipMemcpyDeviceToHost, st));
    TC_HIP(hipStreamSynchronize(st));  // the task count, W+ and the largest d+
    const int64_t T = h.T;
    tl.T = T;
    tl.ptr.alloc(sizeof(int64_t) * (size_t)(n + 1));
    if (T > 0) {
      tl.row.alloc(sizeof(uint32_t) * (size_t)T);
      tl.val.alloc(sizeof(uint64_t) * (size_t)T);
      DevBuf tk(sizeof(uint32_t) * (size_t)T), tv(sizeof(uint64_t) * (size_t)T);
      const bool alt = radix_sort_from<uint32_t, uint64_t>(src, m, tl.row.as<uint32_t>(), tk.as<uint32_t>(),
                                                           tl.val.as<uint64_t>(), tv.as<uint64_t>(), T, 0, s,
                                                           th, st, "tasks");
      if (alt) {
        tl.row.swap(tk);
        tl.val.swap(tv);
      }
    }
    finish_tasks(tl, n, st);
    g->wedges_plus = (int64_t)h.wplus;
    g->max_dplus = (int64_t)h.maxd;
  }
  ka.release();
  kb.release();

  // ---- 6: work classes ------------------------------------------------------
  build_work(g->w, g->owned, n, g->row_ptr, tl.T, tl.row.as<uint32_t>(), tl.ptr.as<int64_t>(),
             tl.val.as<uint64_t>(), tl.prefix.as<uint64_t>(), default_work_params(m), st);
  check_sorts(st);
  g->arena_bytes = g->owned.bytes;
  note_use(*g, st);
  return g.release();
}

void check_task_sorts(hipStream_t st) { check_sorts(st); }

namespace {

// Tasks of a variant work set, one test per nonzero p = (a, b) of U (a from
// erow). <j,i,k> (the default): hashed row b, probes = U_a's entries after b,
// skipped when there are none, and also when U_b is empty unless keep_empty.
// <i,j,k>: hashed row a, probes = all of U_b (skipped when U_b is empty: such
// a task has nothing to look up).
struct VariantTaskPred {
  const int64_t* row_ptr;
  const int32_t* col;
  const uint32_t* erow;
  bool ijk, keep_empty;
  uint32_t* tkey;
  uint64_t* tval;
  struct Item {
    uint32_t key;
    uint64_t val;
  };
  __device__ bool operator()(int64_t p, Item& it) const {
    const uint32_t a = erow[p];
    const int32_t b = col[p];
    const int64_t bs = row_ptr[b], be = row_ptr[b + 1];
    if (ijk) {
      it.key = a;
      it.val = (uint64_t)bs | ((uint64_t)be << 32);
      return be > bs;
    }
    const int64_t end = row_ptr[a + 1];
    it.key = (uint32_t)b;
    it.val = (uint64_t)(p + 1) | ((uint64_t)end << 32);
    return end - p - 1 > 0 && (keep_empty || be > bs);
  }
  __device__ void emit(int64_t, const Item& it, uint32_t pos) const {
    tkey[pos] = it.key;
    tval[pos] = it.val;
  }
};

}  // namespace

Graph* build_variant(const Graph& base, int flags, const WorkParams& wp, hipStream_t st) {
  std::unique_ptr<GraphImpl> g(new GraphImpl());
  g->owned.st = st;
  TC_HIP(hipGetDevice(&g->device));
  TC_REQUIRE(g->device == base.device, TC_EINVAL, "tc_graph_variant: graph built on another device");
  TempStream temps(st);
  g->n = base.n;
  g->m_raw = base.m_raw;
  g->m = base.m;
  g->wedges_plus = base.wedges_plus;
  g->max_dplus = base.max_dplus;
  g->sbits = base.sbits;
  g->row_ptr = base.row_ptr;  // U is shared, not owned
  g->col = base.col;
  g->perm = base.perm;
  g->variant = flags;
  g->hash = (flags & TC_VARIANT_MUL_HASH) ? 1 : 0;
  g->base = &base;
  const bool ijk = (flags & TC_VARIANT_IJK) != 0, no_dcsr = (flags & TC_VARIANT_NO_DCSR) != 0;
  const int64_t n = g->n, m = g->m;
  TaskLists tl;
  if (m > 0) {
    DevBuf erow(sizeof(uint32_t) * (size_t)m);
    TC_LAUNCH("entry_rows", k_entry_rows, dim3(wave_grid(n)), dim3(kT), 0, st, g->row_ptr, n,
              erow.as<uint32_t>());
    DevBuf tk, tv;
    VariantTaskPred vp{g->row_ptr, g->col, erow.as<uint32_t>(), ijk, no_dcsr, nullptr, nullptr};
    const int64_t T = compact("variant_tasks", m, vp, [&](int64_t total, VariantTaskPred& pr) {
      tk.alloc(sizeof(uint32_t) * (size_t)total);
      tv.alloc(sizeof(uint64_t) * (size_t)total);
      pr.tkey = tk.as<uint32_t>();
      pr.tval = tv.as<uint64_t>();
    }, st);
    if (T > 0) sort_tasks(tl, tk, tv, T, n, g->sbits, st, "variant_tasks");
  }
  build_work(g->w, g->owned, n, g->row_ptr, tl.T, tl.row.as<uint32_t>(), tl.ptr.as<int64_t>(),
             tl.val.as<uint64_t>(), tl.prefix.as<uint64_t>(), wp, st, no_dcsr);
  check_sorts(st);
  g->arena_bytes = g->owned.bytes;
  note_use(*g, st);  // (and the base, whose U the build read)
  return g.release();
}

// Probes of a task from its (first probe | end << 32) value.
struct TaskLenLoad {
  const uint64_t* val;
  __device__ uint64_t operator()(int64_t t) const {
    const uint64_t v = val[t];
    return (uint64_t)((uint32_t)(v >> 32) - (uint32_t)v);
  }
};

// Probe prefixes and row pointers of the tasks in tl.row / tl.val (tl.T of
// them, sorted by row; tl.ptr allocated with nrows + 1 entries).
void finish_tasks(TaskLists& tl, int64_t nrows, hipStream_t st) {
  const int64_t T = tl.T;
  if (T == 0) {
    TC_LAUNCH("fill_i64", k_fill_i64, dim3(grid_for(nrows + 1)), dim3(kT), 0, st, tl.ptr.as<int64_t>(),
              nrows + 1, (int64_t)0);
    return;
  }
  tl.prefix.alloc(sizeof(uint64_t) * (size_t)(T + 1));
  device_excl_scan_f<uint64_t>(TaskLenLoad{tl.val.as<uint64_t>()}, tl.prefix.as<uint64_t>(), T,
                               tl.prefix.as<uint64_t>() + T, st);
  TC_LAUNCH("bounds", (k_bounds<uint32_t>), dim3(grid_for(nrows + 1)), dim3(kT), 0, st,
            tl.row.as<uint32_t>(), T, 0, nrows, tl.ptr.as<int64_t>());
  TC_HIP(hipGetLastError());
}

void sort_tasks(TaskLists& tl, DevBuf& tk, DevBuf& tv, int64_t T, int64_t nrows, int key_bits,
                hipStream_t st, const char* name) {
  tl.T = T;
  tl.ptr.alloc(sizeof(int64_t) * (size_t)(nrows + 1));
  if (T > 0) {
    tl.row.alloc(sizeof(uint32_t) * (size_t)T);
    tl.val.alloc(sizeof(uint64_t) * (size_t)T);
    const bool alt = radix_sort<uint32_t, uint64_t>(tk.as<uint32_t>(), tl.row.as<uint32_t>(),
                                                    tv.as<uint64_t>(), tl.val.as<uint64_t>(), T, 0, key_bits, st,
                                                    name);
    if (!alt) {  // sorted data ended in the input buffers: take them over
      tl.row.swap(tk);
      tl.val.swap(tv);
    }
  }
  finish_tasks(tl, nrows, st);
}

void build_work(WorkSet& w, Owned& own, int64_t n, const int64_t* hrow_ptr, int64_t T,
                const uint32_t* tb_row, const int64_t* tb_ptr, const uint64_t* tb_val,
                const uint64_t* tb_prefix, const WorkParams& wp, hipStream_t st, bool all_rows) {
  w.nrows = n;
  w.wp = wp;
  w.n_tasks = T;
  w.tbeg = own.alloc<uint32_t>(n);
  w.tend = own.alloc<uint32_t>(n);
  w.tstart = own.alloc<uint32_t>(T);
  w.tprefix = own.alloc<uint64_t>(T + 1);
  DevBuf dscal(64);
  uint32_t* d_tot32 = dscal.as<uint32_t>();
  uint64_t* d_tot64 = reinterpret_cast<uint64_t*>(dscal.as<char>() + 32);
  // rows without tasks keep the empty range [0, 0)
  TC_LAUNCH("fill_u32", k_fill_u32, dim3(grid_for(n)), dim3(kT), 0, st, w.tbeg, n, 0u);
  TC_LAUNCH("fill_u32", k_fill_u32, dim3(grid_for(n)), dim3(kT), 0, st, w.tend, n, 0u);
  if (T == 0) {
    TC_HIP(hipMemsetAsync(w.tprefix, 0, sizeof(uint64_t), st));
    w.probes = 0;
    return;
  }
  // the probe total is read back with the row count below (one host sync)
  uint64_t h_probes = 0;
  TC_HIP(hipMemcpyAsync(&h_probes, tb_prefix + T, sizeof(h_probes), hipMemcpyDeviceToHost, st));
  DevBuf cls(sizeof(int8_t) * (size_t)n);
  // per class: probes (64-bit counters first: 8-byte aligned for their
  // atomics), then the largest table (log2 slots)
  DevBuf clsl(sizeof(unsigned long long) * NUM_CLASSES + sizeof(int) * NUM_CLASSES);
  TC_HIP(hipMemsetAsync(clsl.p, 0, clsl.bytes, st));
  unsigned long long* d_cw = clsl.as<unsigned long long>();
  int* d_cl = reinterpret_cast<int*>(clsl.as<char>() + sizeof(unsigned long long) * NUM_CLASSES);
  TC_LAUNCH("classify", k_classify, dim3(grid_reduce(n)), dim3(kT), 0, st, tb_ptr, tb_prefix, hrow_ptr, n,
            all_rows, wp.heavy_min, cls.as<int8_t>(), d_cl, d_cw);
  TC_HIP(hipGetLastError());
  struct {
    unsigned long long cw[NUM_CLASSES];
    int cl[NUM_CLASSES];
  } hc;
  static_assert(sizeof(hc.cw) + sizeof(hc.cl) == sizeof(unsigned long long) * NUM_CLASSES + sizeof(int) * NUM_CLASSES,
                "class scalars layout");
  TC_HIP(hipMemcpyAsync(&hc, clsl.p, sizeof(hc.cw) + sizeof(hc.cl), hipMemcpyDeviceToHost, st));
  const unsigned long long* h_cw = hc.cw;
  const int* h_cl = hc.cl;

  // class-major row order: the rows of class 0 (ascending b), then class 1,
  // ...; each row keeps its tasks in b order, so every class - and every pack
  // of consecutive rows of a class - owns one contiguous task range
  DevBuf ckey, crow_in;
  WorkRowPred rowp{cls.as<int8_t>(), nullptr, nullptr};
  const int64_t R = compact("work_rows", n, rowp, [&](int64_t total, WorkRowPred& p) {
    ckey.alloc(sizeof(uint32_t) * (size_t)total);
    crow_in.alloc(sizeof(uint32_t) * (size_t)total);
    p.key = ckey.as<uint32_t>();
    p.row = crow_in.as<uint32_t>();
  }, st);
  w.probes = (int64_t)h_probes;
  TC_REQUIRE(R > 0, TC_EDEVICE, "build_work: tasks but no row with work");
  uint32_t* crow = reinterpret_cast<uint32_t*>(own.alloc<int32_t>(R));  // pack classes keep their rows
  {
    DevBuf ckey2(sizeof(uint32_t) * (size_t)R);
    const bool alt = radix_sort<uint32_t, uint32_t>(ckey.as<uint32_t>(), ckey2.as<uint32_t>(),
                                                    crow_in.as<uint32_t>(), crow, R, 0, 3, st, "classes");
    if (!alt) TC_HIP(hipMemcpyAsync(crow, crow_in.p, sizeof(uint32_t) * (size_t)R, hipMemcpyDeviceToDevice, st));
    const uint32_t* skey = alt ? ckey2.as<uint32_t>() : ckey.as<uint32_t>();
    DevBuf cptr(sizeof(int64_t) * (NUM_CLASSES + 1));
    TC_LAUNCH("bounds", (k_bounds<uint32_t>), dim3(1), dim3(kT), 0, st, skey, R, 0, (int64_t)NUM_CLASSES,
              cptr.as<int64_t>());
    // per class-major row: exclusive prefixes of tasks, probes and items
    DevBuf tsc(sizeof(uint32_t) * (size_t)(R + 1)), wsc(sizeof(uint64_t) * (size_t)(R + 1));
    DevBuf usc(sizeof(uint32_t) * (size_t)(R + 1));
    device_excl_scan_f<uint32_t>(CmTasks{crow, tb_ptr}, tsc.as<uint32_t>(), R, tsc.as<uint32_t>() + R, st);
    device_excl_scan_f<uint64_t>(CmProbes{crow, tb_ptr, tb_prefix}, wsc.as<uint64_t>(), R,
                                 wsc.as<uint64_t>() + R, st);
    // probes per wave item of each item class: wp.wave_chunk, smaller for a
    // class that would otherwise get fewer than wp.min_groups work-groups,
    // provided it has the probes to fill them with items of kWaveChunkMin (a
    // class too small for that stays at wp.wave_chunk: few, large units suit
    // a batch of many small graphs). h_cw is valid: compact synchronised st.
    CmItems cmi{crow, cls.as<int8_t>(), tb_ptr, tb_prefix, {}};
    for (int c = 0; c < NUM_CLASSES; ++c) {
      const uint64_t per_group = wp.min_groups ? h_cw[c] / ((uint64_t)wp.min_groups * class_waves(c)) : ~0ull;
      cmi.chunk[c] = per_group < kWaveChunkMin ? wp.wave_chunk
                                                : (uint32_t)std::min<uint64_t>(wp.wave_chunk, per_group);
      w.cls_chunk[c] = cmi.chunk[c];
    }
    device_excl_scan_f<uint32_t>(cmi, usc.as<uint32_t>(), R,
                                 usc.as<uint32_t>() + R, st);
    DevBuf cm_pos(sizeof(uint32_t) * (size_t)n);
    TC_LAUNCH("cm_place", k_cm_place, dim3(grid_for(R)), dim3(kT), 0, st, crow, R, tsc.as<uint32_t>(), w.tbeg,
              w.tend, cm_pos.as<uint32_t>());
    TC_LAUNCH("task_permute", k_task_permute, dim3(grid_for(T)), dim3(kT), 0, st, T, tb_row, tb_ptr, tb_val,
              tb_prefix, w.tbeg, cm_pos.as<uint32_t>(), wsc.as<uint64_t>(), w.tstart, w.tprefix);
    TC_HIP(hipMemcpyAsync(w.tprefix + T, tb_prefix + T, sizeof(uint64_t), hipMemcpyDeviceToDevice, st));
    // class boundaries and the item offsets there
    DevBuf ub(sizeof(uint32_t) * (NUM_CLASSES + 1));
    TC_LAUNCH("gather_at", (k_gather_at<uint32_t>), dim3(1), dim3(64), 0, st, usc.as<uint32_t>(),
              cptr.as<int64_t>(), NUM_CLASSES + 1, ub.as<uint32_t>());
    int64_t h_cp[NUM_CLASSES + 1];
    uint32_t h_ub[NUM_CLASSES + 1], h_tt = 0;
    TC_HIP(hipMemcpyAsync(h_cp, cptr.p, sizeof(h_cp), hipMemcpyDeviceToHost, st));
    TC_HIP(hipMemcpyAsync(h_ub, ub.p, sizeof(h_ub), hipMemcpyDeviceToHost, st));
    TC_HIP(hipMemcpyAsync(&h_tt, tsc.as<uint32_t>() + R, sizeof(uint32_t), hipMemcpyDeviceToHost, st));
    TC_HIP(hipStreamSynchronize(st));
    TC_REQUIRE((int64_t)h_tt == T && h_cp[NUM_CLASSES] == R, TC_EDEVICE,
               "build_work: class-major task order lost tasks");
    TC_HIP(hipGetLastError());

    // packs of the two pack classes: flags for both, one host sync for both
    // pack counts, then the pack pointers
    DevBuf pf[2], pp[2];
    DevBuf ptot(sizeof(uint32_t) * 2);
    for (int c = CLS_PACK_SMALL; c <= CLS_PACK_LARGE; ++c) {
      const int64_t r0 = h_cp[c], total = h_cp[c + 1] - h_cp[c];
      if (total == 0) continue;
      int32_t* rows = reinterpret_cast<int32_t*>(crow + r0);
      DevBuf wk(sizeof(uint64_t) * (size_t)total), pw(sizeof(uint64_t) * (size_t)total);
      DevBuf sl(sizeof(uint32_t) * (size_t)total), psl(sizeof(uint32_t) * (size_t)total);
      TC_LAUNCH("rows_work", k_rows_work, dim3(grid_for(total)), dim3(kT), 0, st, rows, total, w.tbeg,
                w.tend, w.tprefix, hrow_ptr, wk.as<uint64_t>(), sl.as<uint32_t>());
      device_excl_scan<uint64_t, uint64_t>(wk.as<uint64_t>(), pw.as<uint64_t>(), total, d_tot64, st);
      device_excl_scan<uint32_t, uint32_t>(sl.as<uint32_t>(), psl.as<uint32_t>(), total, d_tot32, st);
      pf[c].alloc(sizeof(uint32_t) * (size_t)total);
      pp[c].alloc(sizeof(uint32_t) * (size_t)total);
      TC_LAUNCH("pack_flags", k_pack_flags, dim3(grid_for(total)), dim3(kT), 0, st, pw.as<uint64_t>(),
                psl.as<uint32_t>(), total, wp.pack_target, wp.pack_slots, pf[c].as<uint32_t>());
      device_excl_scan<uint32_t, uint32_t>(pf[c].as<uint32_t>(), pp[c].as<uint32_t>(), total,
                                           ptot.as<uint32_t>() + c, st);
    }
    uint32_t h_np[2] = {0, 0};
    if (h_cp[CLS_PACK_LARGE + 1] > h_cp[CLS_PACK_SMALL]) {
      TC_HIP(hipMemcpyAsync(h_np, ptot.p, sizeof(h_np), hipMemcpyDeviceToHost, st));
      TC_HIP(hipStreamSynchronize(st));
    }
    for (int c = 0; c < NUM_CLASSES; ++c) {
      w.cls_log2S[c] = h_cl[c];
      const int64_t r0 = h_cp[c], nr = h_cp[c + 1] - h_cp[c];
      if (nr == 0) continue;
      if (c == CLS_PACK_SMALL || c == CLS_PACK_LARGE) {
        const int64_t np = h_np[c];
        uint32_t* pack_ptr = own.alloc<uint32_t>(np + 1);
        TC_LAUNCH("pack_emit", k_pack_emit, dim3(grid_for(nr)), dim3(kT), 0, st, pf[c].as<uint32_t>(),
                  pp[c].as<uint32_t>(), nr, pack_ptr, np);
        TC_HIP(hipGetLastError());
        w.pack_rows[c] = reinterpret_cast<int32_t*>(crow + r0);
        w.pack_ptr[c] = pack_ptr;
        w.pack_recs[c] = own.alloc<PackRow>(nr);
        w.pack_info[c] = own.alloc<PackInfo>(np);
        TC_LAUNCH("pack_recs", k_pack_recs, dim3(grid_for(nr)), dim3(kT), 0, st, w.pack_rows[c], nr, hrow_ptr,
                  w.tbeg, w.tend, w.pack_recs[c]);
        if (np < kPackLptMin) {
          // few packs (a launch of one or two rounds): pack order
          TC_LAUNCH("pack_info", k_pack_info, dim3(grid_for(np)), dim3(kT), 0, st, pack_ptr, np, w.pack_recs[c],
                    w.tprefix, w.pack_info[c]);
        } else {
          // the class's packs in launch order: heaviest first
          DevBuf raw(sizeof(PackInfo) * (size_t)np);
          DevBuf key(sizeof(uint32_t) * (size_t)np), key2(sizeof(uint32_t) * (size_t)np);
          DevBuf idx(sizeof(uint32_t) * (size_t)np), idx2(sizeof(uint32_t) * (size_t)np);
          TC_LAUNCH("pack_info", k_pack_info, dim3(grid_for(np)), dim3(kT), 0, st, pack_ptr, np, w.pack_recs[c],
                    w.tprefix, raw.as<PackInfo>());
          TC_LAUNCH("pack_keys", k_pack_keys, dim3(grid_for(np)), dim3(kT), 0, st, raw.as<PackInfo>(), np,
                    key.as<uint32_t>(), idx.as<uint32_t>());
          const bool alt = radix_sort<uint32_t, uint32_t>(key.as<uint32_t>(), key2.as<uint32_t>(), idx.as<uint32_t>(),
                                                          idx2.as<uint32_t>(), np, 0, 32, st, "pack_lpt");
          TC_LAUNCH("pack_gather", k_pack_gather, dim3(grid_for(np)), dim3(kT), 0, st, raw.as<PackInfo>(),
                    alt ? idx2.as<uint32_t>() : idx.as<uint32_t>(), np, w.pack_info[c]);
        }
        TC_HIP(hipGetLastError());
        w.n_pack_rows[c] = nr;
        w.n_packs[c] = np;
        w.pack_log2S[c] = h_cl[c];
      } else {
        const int64_t total = (int64_t)h_ub[c + 1] - (int64_t)h_ub[c];
        if (total == 0) continue;
        CountItem* items = own.alloc<CountItem>(total);
        TC_LAUNCH("emit_items", k_emit_items, dim3(grid_for(total)), dim3(kT), 0, st, usc.as<uint32_t>() + r0,
                  crow + r0, nr, total, w.tbeg, w.tend, w.tprefix, hrow_ptr, items);
        TC_HIP(hipGetLastError());
        w.items[c] = items;
        w.n_items[c] = total;
      }
    }
  }
  {
    const int64_t nb = (int64_t)grid_reduce(n);
    DevBuf part(sizeof(unsigned long long) * (size_t)nb * kStatCols);
    DevBuf sums(sizeof(unsigned long long) * kStatCols);
    TC_LAUNCH("class_stats", k_class_stats, dim3((unsigned)nb), dim3(kT), 0, st, cls.as<int8_t>(), n,
              w.tbeg, w.tend, w.tprefix, hrow_ptr, part.as<unsigned long long>());
    TC_LAUNCH("reduce_cols", k_reduce_cols, dim3(kStatCols), dim3(kT), 0, st,
              part.as<unsigned long long>(), nb, kStatCols, sums.as<unsigned long long>());
    TC_HIP(hipGetLastError());
    // (valid once st is synchronised: both callers check their sorts next)
    TC_HIP(hipMemcpyAsync(&w.cls_stats[0][0], sums.p, sizeof(w.cls_stats), hipMemcpyDeviceToHost, st));
  }
}

}  // namespace tc

extern "C" tc_status tc_graph_variant(const tc_graph* gh, int32_t flags, void* stream, tc_graph** out) {
  try {
    TC_REQUIRE(out != nullptr, TC_EINVAL, "tc_graph_variant: out is NULL");
    *out = nullptr;
    TC_REQUIRE(gh != nullptr, TC_EINVAL, "tc_graph_variant: null graph");
    TC_REQUIRE((flags & ~(TC_VARIANT_IJK | TC_VARIANT_NO_DCSR | TC_VARIANT_MUL_HASH)) == 0, TC_EINVAL,
               "tc_graph_variant: unknown flags");
    const tc::Graph& base = *tc::G(gh);
    tc::require_plain(base, "tc_graph_variant");
    tc::Graph* g = tc::build_variant(base, flags, base.w.wp, static_cast<hipStream_t>(stream));
    *out = reinterpret_cast<tc_graph*>(g);
    tc::set_last_error("");
    return TC_OK;
  } catch (const tc::Error& e) {
    tc::set_last_error(e.what());
    return e.status;
  } catch (const std::bad_alloc&) {
    tc::set_last_error("tc_graph_variant: host allocation failed");
    return TC_ENOMEM;
  } catch (const std::exception& e) {
    tc::set_last_error(e.what());
    return TC_EDEVICE;
  }
}

extern "C" tc_status tc_preprocess(const int32_t* d_src, const int32_t* d_dst, int64_t m_raw,
                                   int32_t n, void* stream, tc_graph** out) {
  try {
    TC_REQUIRE(out != nullptr, TC_EINVAL, "tc_preprocess: out is NULL");
    *out = nullptr;
    TC_REQUIRE(n >= 1, TC_EINVAL, "tc_preprocess: n must be >= 1");
    TC_REQUIRE(m_raw >= 0, TC_EINVAL, "tc_preprocess: m_raw must be >= 0");
    TC_REQUIRE(m_raw == 0 || (d_src != nullptr && d_dst != nullptr), TC_EINVAL,
               "tc_preprocess: null edge arrays");
    TC_REQUIRE(m_raw < (int64_t)0xFFFFFFFFLL, TC_EOVERFLOW, "tc_preprocess: m_raw >= 2^32 - 1");
    tc::Graph* g = tc::build_graph(d_src, d_dst, m_raw, n, static_cast<hipStream_t>(stream));
    *out = reinterpret_cast<tc_graph*>(g);
    tc::set_last_error("");
    return TC_OK;
  } catch (const tc::Error& e) {
    tc::set_last_error(e.what());
    return e.status;
  } catch (const std::bad_alloc&) {
    tc::set_last_error("tc_preprocess: host allocation failed");
    return TC_ENOMEM;
  } catch (const std::exception& e) {
    tc::set_last_error(e.what());
    return TC_EDEVICE;
  }
}
