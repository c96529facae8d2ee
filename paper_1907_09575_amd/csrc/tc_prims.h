// tc_prims.h - device primitives for preprocessing: block/wave scans, an
// exclusive scan over device arrays (reduce-then-scan, no inter-block waits)
// and a stable LSD radix sort (8-bit digits) with wave-ballot ranking.
//
// All kernels use 256-thread work-groups (4 wave64 waves).
#pragma once

#include <string>
#include <type_traits>
#include <vector>

#include "tc_internal.h"

namespace tc {

constexpr int kPrimThreads = 256;

__device__ __forceinline__ int lane_id() { return (int)__lane_id(); }

template <class T>
__device__ __forceinline__ T wave_incl_scan(T v) {
  const int lane = lane_id();
#pragma unroll
  for (int d = 1; d < 64; d <<= 1) {
    T t = __shfl_up(v, d, 64);
    if (lane >= d) v += t;
  }
  return v;
}

template <class T>
__device__ __forceinline__ T wave_sum(T v) {
#pragma unroll
  for (int d = 32; d >= 1; d >>= 1) v += __shfl_xor(v, d, 64);
  return v;
}

template <class T>
__device__ __forceinline__ T wave_max(T v) {
#pragma unroll
  for (int d = 32; d >= 1; d >>= 1) {
    T o = __shfl_xor(v, d, 64);
    v = o > v ? o : v;
  }
  return v;
}

// Exclusive scan across a 256-thread block; s_wave needs 4 entries. Also
// returns the block total. Contains two barriers: call from all threads.
template <class T>
__device__ __forceinline__ T block_excl_scan(T v, T* s_wave, T& total) {
  const int lane = lane_id(), wave = threadIdx.x >> 6;
  T inc = wave_incl_scan(v);
  if (lane == 63) s_wave[wave] = inc;
  __syncthreads();
  T woff = 0, tot = 0;
#pragma unroll
  for (int w = 0; w < 4; ++w) {
    T x = s_wave[w];
    if (w < wave) woff += x;
    tot += x;
  }
  __syncthreads();
  total = tot;
  return woff + inc - v;
}

// ---------------------------------------------------------------------------
// Exclusive scan of a device array: out[i] = sum_{j<i} in[j]; optionally
// *total = sum of all. Three kernels: tile reduce, scan of tile sums (one
// block), tile scan with carry-in.
// ---------------------------------------------------------------------------
constexpr int kScanItems = 8;
constexpr int kScanTile = kPrimThreads * kScanItems;

template <class Tin, class Tout>
__global__ __launch_bounds__(256) void k_scan_reduce(const Tin* __restrict__ in, int64_t n,
                                                     Tout* __restrict__ partial) {
  __shared__ Tout s_w[4];
  const int64_t base = (int64_t)blockIdx.x * kScanTile;
  Tout acc = 0;
#pragma unroll
  for (int i = 0; i < kScanItems; ++i) {
    int64_t idx = base + (int64_t)i * kPrimThreads + threadIdx.x;
    if (idx < n) acc += (Tout)in[idx];
  }
  acc = wave_sum(acc);
  if (lane_id() == 0) s_w[threadIdx.x >> 6] = acc;
  __syncthreads();
  if (threadIdx.x == 0) partial[blockIdx.x] = s_w[0] + s_w[1] + s_w[2] + s_w[3];
}

template <class T>
__global__ __launch_bounds__(256) void k_scan_partials(T* __restrict__ partial, int64_t nb,
                                                       T* __restrict__ total) {
  __shared__ T s_w[4];
  T carry = 0;
  for (int64_t base = 0; base < nb; base += kScanTile) {
    T v[kScanItems];
    T local = 0;
#pragma unroll
    for (int i = 0; i < kScanItems; ++i) {
      int64_t idx = base + (int64_t)threadIdx.x * kScanItems + i;
      v[i] = idx < nb ? partial[idx] : T(0);
      local += v[i];
    }
    T tot;
    T ex = block_excl_scan(local, s_w, tot) + carry;
#pragma unroll
    for (int i = 0; i < kScanItems; ++i) {
      int64_t idx = base + (int64_t)threadIdx.x * kScanItems + i;
      if (idx < nb) partial[idx] = ex;
      ex += v[i];
    }
    carry += tot;
  }
  if (total && threadIdx.x == 0) *total = carry;
}

template <class Tin, class Tout>
__global__ __launch_bounds__(256) void k_scan_final(const Tin* __restrict__ in, int64_t n,
                                                    const Tout* __restrict__ partial,
                                                    Tout* __restrict__ out) {
  __shared__ Tout s_w[4];
  const int64_t base = (int64_t)blockIdx.x * kScanTile;
  Tout v[kScanItems];
  Tout local = 0;
#pragma unroll
  for (int i = 0; i < kScanItems; ++i) {
    int64_t idx = base + (int64_t)threadIdx.x * kScanItems + i;
    v[i] = idx < n ? (Tout)in[idx] : Tout(0);
    local += v[i];
  }
  Tout tot;
  Tout ex = block_excl_scan(local, s_w, tot) + partial[blockIdx.x];
#pragma unroll
  for (int i = 0; i < kScanItems; ++i) {
    int64_t idx = base + (int64_t)threadIdx.x * kScanItems + i;
    if (idx < n) out[idx] = ex;
    ex += v[i];
  }
}

// Stream that preprocessing temporaries are ordered on (set by TempStream).
// While one is set, DevBuf allocates with hipMallocAsync and frees with
// hipFreeAsync on it, from the device's default memory pool (which keeps
// freed blocks for reuse), so freeing a temporary needs no synchronisation.
struct TempCtx {
  bool active = false;
  hipStream_t st = nullptr;
};
TempCtx& temp_ctx();

struct TempStream {
  TempCtx prev;
  explicit TempStream(hipStream_t st);
  ~TempStream() { temp_ctx() = prev; }
};

// Device buffer owned by one scope.
struct DevBuf {
  void* p = nullptr;
  size_t bytes = 0;
  hipStream_t st = nullptr;
  bool async = false;
  DevBuf() = default;
  explicit DevBuf(size_t b) { alloc(b); }
  void alloc(size_t b) {
    release();
    bytes = b;
    if (!b) return;
    st = temp_ctx().st;
    async = temp_ctx().active;
    if (async) TC_HIP(hipMallocAsync(&p, b, st));
    else TC_HIP(hipMalloc(&p, b));
  }
  void release() {
    if (p) (void)(async ? hipFreeAsync(p, st) : hipFree(p));
    p = nullptr;
    bytes = 0;
  }
  ~DevBuf() { release(); }
  DevBuf(const DevBuf&) = delete;
  DevBuf& operator=(const DevBuf&) = delete;
  template <class T>
  T* as() const {
    return static_cast<T*>(p);
  }
};

// Stable C string for a launch name built at run time.
const char* intern_name(const std::string& s);

inline int64_t div_up(int64_t a, int64_t b) { return (a + b - 1) / b; }

// Exclusive scan of n elements; out may alias in. If total != nullptr, the
// grand total is written there (device pointer).
template <class Tin, class Tout>
void device_excl_scan(const Tin* in, Tout* out, int64_t n, Tout* total, hipStream_t st) {
  if (n <= 0) {
    if (total) TC_HIP(hipMemsetAsync(total, 0, sizeof(Tout), st));
    return;
  }
  int64_t nb = div_up(n, kScanTile);
  DevBuf part(sizeof(Tout) * (size_t)nb);
  TC_LAUNCH("scan_reduce", (k_scan_reduce<Tin, Tout>), dim3((unsigned)nb), dim3(256), 0, st, in, n,
                     part.as<Tout>());
  TC_LAUNCH("scan_partials", (k_scan_partials<Tout>), dim3(1), dim3(256), 0, st, part.as<Tout>(), nb, total);
  TC_LAUNCH("scan_final", (k_scan_final<Tin, Tout>), dim3((unsigned)nb), dim3(256), 0, st, in, n,
                     part.as<Tout>(), out);
  TC_HIP(hipGetLastError());
}

// ---------------------------------------------------------------------------
// Stable LSD radix sort, 8-bit digits.
// Per pass: (1) per-tile digit histograms, stored digit-major
// hist[d * nblocks + tile]; (2) exclusive scan of hist gives every (digit,
// tile) its global output offset; (3) each tile ranks its keys stably with
// 8 wave ballots per key (peers = lanes with the same digit), stages them in
// LDS in digit order and writes each digit's run contiguously.
// ---------------------------------------------------------------------------
struct NoVal {};

constexpr int kSortItems = 8;
constexpr int kSortTile = kPrimThreads * kSortItems;

template <class K>
__global__ __launch_bounds__(256) void k_rs_hist(const K* __restrict__ kin, int64_t n, int shift,
                                                 uint32_t dmask, uint32_t* __restrict__ hist,
                                                 int64_t nblocks) {
  __shared__ uint32_t h[4][256];
  const int tid = threadIdx.x, wave = tid >> 6;
#pragma unroll
  for (int w = 0; w < 4; ++w) h[w][tid] = 0;
  __syncthreads();
  const int64_t base = (int64_t)blockIdx.x * kSortTile;
#pragma unroll
  for (int i = 0; i < kSortItems; ++i) {
    int64_t idx = base + (int64_t)i * kPrimThreads + tid;
    if (idx < n) {
      uint32_t d = (uint32_t)(kin[idx] >> shift) & dmask;
      atomicAdd(&h[wave][d], 1u);
    }
  }
  __syncthreads();
  hist[(int64_t)tid * nblocks + blockIdx.x] = h[0][tid] + h[1][tid] + h[2][tid] + h[3][tid];
}

template <class K, class V>
__global__ __launch_bounds__(256) void k_rs_scatter(const K* __restrict__ kin, K* __restrict__ kout,
                                                    const V* __restrict__ vin, V* __restrict__ vout,
                                                    int64_t n, int shift, uint32_t dmask,
                                                    const uint32_t* __restrict__ hist,
                                                    const uint32_t* __restrict__ offs,
                                                    int64_t nblocks) {
  constexpr bool HV = !std::is_same<V, NoVal>::value;
  using VS = typename std::conditional<HV, V, char>::type;
  __shared__ K s_k[kSortTile];
  __shared__ VS s_v[HV ? kSortTile : 1];
  __shared__ uint32_t s_goff[256], s_tstart[256], s_run[256];
  __shared__ uint32_t s_wc[2][4][256];
  __shared__ uint32_t s_tmp[4];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int64_t blk = blockIdx.x;
  const int64_t base = blk * kSortTile;

  uint32_t cnt = hist[(int64_t)tid * nblocks + blk];
  s_goff[tid] = offs[(int64_t)tid * nblocks + blk];
  uint32_t tot;
  s_tstart[tid] = block_excl_scan(cnt, s_tmp, tot);
  s_run[tid] = 0;
#pragma unroll
  for (int w = 0; w < 4; ++w) {
    s_wc[0][w][tid] = 0;
    s_wc[1][w][tid] = 0;
  }
  __syncthreads();

  const uint64_t lt_mask = (1ull << lane) - 1ull;
  for (int i = 0; i < kSortItems; ++i) {
    const int64_t idx = base + (int64_t)i * kPrimThreads + tid;
    const bool valid = idx < n;
    K k = valid ? kin[idx] : K(0);
    VS v{};
    if constexpr (HV) {
      if (valid) v = vin[idx];
    }
    const uint32_t d = (uint32_t)(k >> shift) & dmask;
    uint64_t peers = __ballot(valid);
#pragma unroll
    for (int bb = 0; bb < 8; ++bb) {
      const bool bit = (d >> bb) & 1u;
      const uint64_t m = __ballot(bit);
      peers &= bit ? m : ~m;
    }
    const uint32_t wr = (uint32_t)__popcll(peers & lt_mask);
    const int buf = i & 1;
    if (valid && wr == 0) s_wc[buf][wave][d] = (uint32_t)__popcll(peers);
    __syncthreads();
    {
      uint32_t c = s_run[tid];
#pragma unroll
      for (int w = 0; w < 4; ++w) {
        uint32_t t = s_wc[buf][w][tid];
        s_wc[buf][w][tid] = c;
        c += t;
      }
      s_run[tid] = c;
#pragma unroll
      for (int w = 0; w < 4; ++w) s_wc[buf ^ 1][w][tid] = 0;
    }
    __syncthreads();
    if (valid) {
      const uint32_t lp = s_tstart[d] + s_wc[buf][wave][d] + wr;
      s_k[lp] = k;
      if constexpr (HV) s_v[lp] = v;
    }
  }
  __syncthreads();
  const int64_t rem = n - base;
  const int tile_n = rem < kSortTile ? (int)rem : kSortTile;
#pragma unroll
  for (int i = 0; i < kSortItems; ++i) {
    const int lp = i * kPrimThreads + tid;
    if (lp < tile_n) {
      const K k = s_k[lp];
      const uint32_t d = (uint32_t)(k >> shift) & dmask;
      const uint64_t gp = (uint64_t)s_goff[d] + (uint64_t)(lp - (int)s_tstart[d]);
      kout[gp] = k;
      if constexpr (HV) vout[gp] = s_v[lp];
    }
  }
}

// Sorts keys[0..n) by bits [bit_lo, bit_hi) (stable), carrying vals if V is
// not NoVal. keys/vals and keys_alt/vals_alt are ping-pong buffers of n
// elements; returns true if the sorted data ended in the *_alt buffers.
template <class K, class V>
bool radix_sort(K* keys, K* keys_alt, V* vals, V* vals_alt, int64_t n, int bit_lo, int bit_hi,
                hipStream_t st, const char* name) {
  const char* n_hist = intern_name(std::string("rs_hist:") + name);
  const char* n_scat = intern_name(std::string("rs_scatter:") + name);
  if (n <= 1 || bit_hi <= bit_lo) return false;
  TC_REQUIRE(n < (int64_t)0xFFFFFFFFLL, TC_EOVERFLOW, "radix_sort: more than 2^32-1 keys");
  const int64_t nb = div_up(n, kSortTile);
  DevBuf hist(sizeof(uint32_t) * 256 * (size_t)nb), offs(sizeof(uint32_t) * 256 * (size_t)nb);
  const int64_t hn = 256 * nb;
  const int64_t pnb = div_up(hn, kScanTile);
  DevBuf part(sizeof(uint32_t) * (size_t)pnb);
  K* ka = keys;
  K* kb = keys_alt;
  V* va = vals;
  V* vb = vals_alt;
  bool alt = false;
  for (int shift = bit_lo; shift < bit_hi; shift += 8) {
    const int bits = bit_hi - shift < 8 ? bit_hi - shift : 8;
    const uint32_t dmask = (1u << bits) - 1u;
    TC_LAUNCH(n_hist, (k_rs_hist<K>), dim3((unsigned)nb), dim3(256), 0, st, ka, n, shift, dmask,
                       hist.as<uint32_t>(), nb);
    TC_LAUNCH("scan_reduce", (k_scan_reduce<uint32_t, uint32_t>), dim3((unsigned)pnb), dim3(256), 0, st,
                       hist.as<uint32_t>(), hn, part.as<uint32_t>());
    TC_LAUNCH("scan_partials", (k_scan_partials<uint32_t>), dim3(1), dim3(256), 0, st, part.as<uint32_t>(),
                       pnb, (uint32_t*)nullptr);
    TC_LAUNCH("scan_final", (k_scan_final<uint32_t, uint32_t>), dim3((unsigned)pnb), dim3(256), 0, st,
                       hist.as<uint32_t>(), hn, part.as<uint32_t>(), offs.as<uint32_t>());
    TC_LAUNCH(n_scat, (k_rs_scatter<K, V>), dim3((unsigned)nb), dim3(256), 0, st, ka, kb, va, vb, n,
                       shift, dmask, hist.as<uint32_t>(), offs.as<uint32_t>(), nb);
    TC_HIP(hipGetLastError());
    std::swap(ka, kb);
    std::swap(va, vb);
    alt = !alt;
  }
  return alt;
}

// Tasks in hashed-row order (the input of build_work).
struct TaskLists {
  int64_t T = 0;
  DevBuf row;     // uint32 [T]: hashed row of each task
  DevBuf start;   // uint32 [T]: first probe (probe-side index)
  DevBuf len;     // uint32 [T]: probes
  DevBuf prefix;  // uint64 [T + 1]: exclusive prefix of len, total at [T]
  DevBuf ptr;     // int64 [nrows + 1]: tasks of row b are [ptr[b], ptr[b + 1])
};

// Sort T emitted tasks (keys = hashed row in [0, 2^key_bits), values =
// first probe | end << 32) stably by row and fill `tl`. tk / tv are consumed
// as sort buffers.
void sort_tasks(TaskLists& tl, uint32_t* tk, uint64_t* tv, int64_t T, int64_t nrows, int key_bits,
                hipStream_t st, const char* name);

}  // namespace tc
