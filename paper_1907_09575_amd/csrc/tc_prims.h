// tc_prims.h - device primitives for preprocessing: block/wave scans, an
// exclusive scan over device arrays (reduce-then-scan, no inter-block waits)
// and a stable LSD radix sort (8-bit digits) with wave-ballot ranking.
//
// All kernels use 256-thread work-groups (4 wave64 waves).
#pragma once

#include <string>
#include <type_traits>
#include <utility>
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
// block), tile scan with carry-in; one (k_scan_small) for at most
// kScanSmallTiles tiles.
// ---------------------------------------------------------------------------
constexpr int kScanItems = 8;
constexpr int kScanTile = kPrimThreads * kScanItems;

// Element i of the scanned sequence as L::operator()(i) (an array read or a
// value computed from other arrays).
template <class Tin, class Tout>
struct ArrayLoad {
  const Tin* in;
  __device__ Tout operator()(int64_t i) const { return (Tout)in[i]; }
};

template <class L, class Tout>
__global__ __launch_bounds__(256) void k_scan_reduce(L load, int64_t n, Tout* __restrict__ partial) {
  __shared__ Tout s_w[4];
  const int64_t base = (int64_t)blockIdx.x * kScanTile;
  Tout acc = 0;
#pragma unroll
  for (int i = 0; i < kScanItems; ++i) {
    int64_t idx = base + (int64_t)i * kPrimThreads + threadIdx.x;
    if (idx < n) acc += load(idx);
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

// Tile scan with carry-in. Element j of the tile is item j / 256 of thread
// j % 256 (striped: every load and store of a wave is one contiguous run);
// each item row is scanned within its wave by shuffles, and one LDS exchange
// of the 8 x 4 wave totals gives every element its offset.
template <class L, class Tout>
__global__ __launch_bounds__(256) void k_scan_final(L load, int64_t n, const Tout* __restrict__ partial,
                                                    Tout* __restrict__ out) {
  __shared__ Tout s_w[kScanItems][4];
  const int lane = lane_id(), wave = threadIdx.x >> 6;
  const int64_t base = (int64_t)blockIdx.x * kScanTile;
  Tout v[kScanItems];
#pragma unroll
  for (int i = 0; i < kScanItems; ++i) {
    const int64_t idx = base + (int64_t)i * kPrimThreads + threadIdx.x;
    v[i] = idx < n ? load(idx) : Tout(0);
  }
  Tout inc[kScanItems];
#pragma unroll
  for (int i = 0; i < kScanItems; ++i) {
    inc[i] = wave_incl_scan(v[i]);
    if (lane == 63) s_w[i][wave] = inc[i];
  }
  __syncthreads();
  Tout off = partial[blockIdx.x];
#pragma unroll
  for (int i = 0; i < kScanItems; ++i) {
    Tout before = 0, row = 0;
#pragma unroll
    for (int w = 0; w < 4; ++w) {
      const Tout x = s_w[i][w];
      if (w < wave) before += x;
      row += x;
    }
    const int64_t idx = base + (int64_t)i * kPrimThreads + threadIdx.x;
    if (idx < n) out[idx] = off + before + inc[i] - v[i];
    off += row;
  }
}

// Exclusive scan of at most kScanSmallTiles tiles by one work-group: the
// tiles of k_scan_final in order, each with the running total of the ones
// before it as its carry-in; writes the grand total too. One launch instead
// of three for the short arrays (tile counts, per-class rows, the vertices
// of a small graph) that most scans of a small graph's preprocessing cover.
constexpr int kScanSmallTiles = 4;

template <class L, class Tout>
__global__ __launch_bounds__(256) void k_scan_small(L load, int64_t n, Tout* __restrict__ out,
                                                    Tout* __restrict__ total) {
  __shared__ Tout s_w[kScanItems][4];
  const int lane = lane_id(), wave = threadIdx.x >> 6;
  Tout off = 0;  // the same in every thread
  for (int64_t base = 0; base < n; base += kScanTile) {
    Tout v[kScanItems], inc[kScanItems];
#pragma unroll
    for (int i = 0; i < kScanItems; ++i) {
      const int64_t idx = base + (int64_t)i * kPrimThreads + threadIdx.x;
      v[i] = idx < n ? load(idx) : Tout(0);
    }
#pragma unroll
    for (int i = 0; i < kScanItems; ++i) {
      inc[i] = wave_incl_scan(v[i]);
      if (lane == 63) s_w[i][wave] = inc[i];
    }
    __syncthreads();
#pragma unroll
    for (int i = 0; i < kScanItems; ++i) {
      Tout before = 0, row = 0;
#pragma unroll
      for (int w = 0; w < 4; ++w) {
        const Tout x = s_w[i][w];
        if (w < wave) before += x;
        row += x;
      }
      const int64_t idx = base + (int64_t)i * kPrimThreads + threadIdx.x;
      if (idx < n) out[idx] = off + before + inc[i] - v[i];
      off += row;
    }
    __syncthreads();  // s_w is written again by the next tile
  }
  if (total && threadIdx.x == 0) *total = off;
}

// Stream that preprocessing temporaries are ordered on (set by TempStream).
// DevBuf allocates from the caching allocator on it and returns blocks to
// the cache with an event recorded on it, so freeing a temporary needs no
// synchronisation and the block is reused only after the work queued so far.
// Each TempStream also owns a device word that the radix sorts of its scope
// set when a look-back wait gives up (check_sorts reads it): a failure is
// reported to the call whose sort failed, never to a concurrent one.
struct TempCtx {
  bool active = false;
  hipStream_t st = nullptr;
  int* fail = nullptr;
};
TempCtx& temp_ctx();

struct TempStream {
  TempCtx prev;
  void* fail_word = nullptr;
  explicit TempStream(hipStream_t st);
  ~TempStream();
  TempStream(const TempStream&) = delete;
  TempStream& operator=(const TempStream&) = delete;
};

// Device buffer owned by one scope.
struct DevBuf {
  void* p = nullptr;
  size_t bytes = 0;
  hipStream_t st = nullptr;
  DevBuf() = default;
  explicit DevBuf(size_t b) { alloc(b); }
  void alloc(size_t b) {
    release();
    bytes = b;
    if (!b) return;
    st = temp_ctx().st;
    p = cache_alloc(b, st);
  }
  void release() {
    if (p) cache_free(p, st, false);
    p = nullptr;
    bytes = 0;
  }
  ~DevBuf() { release(); }
  void swap(DevBuf& o) {
    std::swap(p, o.p);
    std::swap(bytes, o.bytes);
    std::swap(st, o.st);
  }
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

// Exclusive scan of the n elements load(0..n-1) into out; if total !=
// nullptr, the grand total is written there (device pointer). out may alias
// what load reads only if element i depends on position i alone.
template <class Tout, class L>
void device_excl_scan_f(L load, Tout* out, int64_t n, Tout* total, hipStream_t st) {
  if (n <= 0) {
    if (total) TC_HIP(hipMemsetAsync(total, 0, sizeof(Tout), st));
    return;
  }
  int64_t nb = div_up(n, kScanTile);
  if (nb <= kScanSmallTiles) {
    TC_LAUNCH("scan_small", (k_scan_small<L, Tout>), dim3(1), dim3(256), 0, st, load, n, out, total);
    TC_HIP(hipGetLastError());
    return;
  }
  DevBuf part(sizeof(Tout) * (size_t)nb);
  TC_LAUNCH("scan_reduce", (k_scan_reduce<L, Tout>), dim3((unsigned)nb), dim3(256), 0, st, load, n,
            part.as<Tout>());
  TC_LAUNCH("scan_partials", (k_scan_partials<Tout>), dim3(1), dim3(256), 0, st, part.as<Tout>(), nb, total);
  TC_LAUNCH("scan_final", (k_scan_final<L, Tout>), dim3((unsigned)nb), dim3(256), 0, st, load, n,
            part.as<Tout>(), out);
  TC_HIP(hipGetLastError());
}

// Exclusive scan of n array elements; out may alias in.
template <class Tin, class Tout>
void device_excl_scan(const Tin* in, Tout* out, int64_t n, Tout* total, hipStream_t st) {
  device_excl_scan_f<Tout>(ArrayLoad<Tin, Tout>{in}, out, n, total, st);
}

// ---------------------------------------------------------------------------
// Stable stream compaction in two reads of the input and no per-element
// flag or position arrays: k_compact_count counts the selected elements of
// each tile (4096 elements: each wave a contiguous quarter, 16 rows of 64),
// an exclusive scan of the tile counts gives every tile's output base, and
// k_compact_emit evaluates the predicate again and hands each selected
// element its output position (tile base + earlier waves + running count +
// ballot rank), so the output keeps the input order.
//
// P is a functor with
//   __device__ bool operator()(int64_t i, Item& it) const  (select i; fill it)
//   __device__ void emit(int64_t i, const Item& it, uint32_t pos) const
// and a nested type Item (data the emit needs, loaded with the predicate).
// ---------------------------------------------------------------------------
constexpr int kCompactRows = 16;
constexpr int kCompactTile = 256 * kCompactRows;

template <class P>
__global__ __launch_bounds__(256) void k_compact_count(int64_t m, P pred, uint32_t* __restrict__ tile_cnt) {
  __shared__ uint32_t s_w[4];
  const int lane = lane_id(), wave = threadIdx.x >> 6;
  const int64_t wbase = (int64_t)blockIdx.x * kCompactTile + (int64_t)wave * (64 * kCompactRows);
  uint32_t c = 0;
#pragma unroll
  for (int j = 0; j < kCompactRows; ++j) {
    const int64_t i = wbase + 64 * j + lane;
    typename P::Item it;
    const bool sel = i < m && pred(i, it);
    c += (uint32_t)__popcll(__ballot(sel));
  }
  if (lane == 0) s_w[wave] = c;
  __syncthreads();
  if (threadIdx.x == 0) tile_cnt[blockIdx.x] = s_w[0] + s_w[1] + s_w[2] + s_w[3];
}

template <class P>
__global__ __launch_bounds__(256) void k_compact_emit(int64_t m, P pred, const uint32_t* __restrict__ tile_off) {
  __shared__ uint32_t s_w[4];
  const int lane = lane_id(), wave = threadIdx.x >> 6;
  const int64_t wbase = (int64_t)blockIdx.x * kCompactTile + (int64_t)wave * (64 * kCompactRows);
  const uint64_t lt_mask = (1ull << lane) - 1ull;
  typename P::Item it[kCompactRows];
  uint64_t bal[kCompactRows];
  uint32_t c = 0;
#pragma unroll
  for (int j = 0; j < kCompactRows; ++j) {
    const int64_t i = wbase + 64 * j + lane;
    const bool sel = i < m && pred(i, it[j]);
    bal[j] = __ballot(sel);
    c += (uint32_t)__popcll(bal[j]);
  }
  if (lane == 0) s_w[wave] = c;
  __syncthreads();
  uint32_t base = tile_off[blockIdx.x];
  for (int w = 0; w < wave; ++w) base += s_w[w];
#pragma unroll
  for (int j = 0; j < kCompactRows; ++j) {
    if ((bal[j] >> lane) & 1ull) pred.emit(wbase + 64 * j + lane, it[j], base + (uint32_t)__popcll(bal[j] & lt_mask));
    base += (uint32_t)__popcll(bal[j]);
  }
}

// Compacts [0, m) under predicate `pred` (see above) and returns the number
// of selected elements. `prepare(total, pred)` runs on the host between the
// count and the emit (to allocate the output and point pred at it); nothing
// is emitted when total is 0. Synchronises st once. m < 2^32.
template <class P, class F>
int64_t compact(const char* name, int64_t m, P pred, F&& prepare, hipStream_t st) {
  if (m <= 0) return 0;
  const int64_t tiles = div_up(m, kCompactTile);
  DevBuf cnt(sizeof(uint32_t) * (size_t)tiles), off(sizeof(uint32_t) * (size_t)tiles);
  DevBuf tot(sizeof(uint32_t));
  const char* n_count = intern_name(std::string("compact_count:") + name);
  const char* n_emit = intern_name(std::string("compact_emit:") + name);
  TC_LAUNCH(n_count, (k_compact_count<P>), dim3((unsigned)tiles), dim3(256), 0, st, m, pred,
            cnt.as<uint32_t>());
  device_excl_scan<uint32_t, uint32_t>(cnt.as<uint32_t>(), off.as<uint32_t>(), tiles, tot.as<uint32_t>(), st);
  uint32_t total = 0;
  TC_HIP(hipMemcpyAsync(&total, tot.p, sizeof(uint32_t), hipMemcpyDeviceToHost, st));
  TC_HIP(hipStreamSynchronize(st));
  if (total == 0) return 0;
  prepare((int64_t)total, pred);
  TC_LAUNCH(n_emit, (k_compact_emit<P>), dim3((unsigned)tiles), dim3(256), 0, st, m, pred,
            off.as<uint32_t>());
  TC_HIP(hipGetLastError());
  return (int64_t)total;
}

// ---------------------------------------------------------------------------
// Stable LSD radix sort, 8-bit digits, one kernel per digit.
// (1) One read of the keys counts the digits of every pass; an exclusive scan
//     of each pass's 256 counts gives the start of every digit's bucket.
// (2) Per pass, work-groups take tiles in ticket order (an atomic counter, so
//     a tile only ever waits for tiles that are already running), load the
//     tile into registers and rank its keys stably by digit with wave ballots
//     (peers = lanes with the same digit; counts carried across the tile's
//     rows in LDS). Each digit's thread then publishes the tile's count, the
//     tile is put in digit order in LDS (giving the predecessors time to
//     publish), each digit's thread walks back over earlier tiles' published
//     words until it meets an inclusive prefix (decoupled look-back) and
//     publishes its own, and the tile writes each digit's run contiguously.
//     A published word is 0 (nothing yet), an aggregate (count + 1) or an
//     inclusive prefix (value with the top bit set), in one 32-bit atomic
//     when the sort holds fewer than 2^31 keys, else one 64-bit atomic. The
//     wait is bounded: past the spin budget the kernel records a failure
//     (sort_failed) and goes on, so every wave always finishes.
// The first pass may read its elements through a source functor instead of
// the key and value arrays (radix_sort_from): it selects some of n_in input
// positions and builds their keys and values, and the pass ranks and writes
// only the selected ones, in input order within each digit.
// ---------------------------------------------------------------------------
struct NoVal {};

// Source of a pass that reads the key and value arrays.
struct NoSrc {};

// Epilogue of a sort's last pass: called with every key and its final
// position as it is written (NoEpi: nothing).
struct NoEpi {
  template <class K>
  __device__ void operator()(uint64_t, K) const {}
};

constexpr int kSortPassesMax = 8;
// Look-back words of all passes of a sort up to this size are cleared by
// one memset (see radix_sort_cfg).
constexpr size_t kLbClearOnceBytes = (size_t)4 << 20;
constexpr uint32_t kLbSpinMax = 1u << 16;
constexpr int kLbWin = 4;  // predecessors read per look-back step

template <class W>
__host__ __device__ constexpr W lb_top() {
  return (W)1 << (8 * sizeof(W) - 1);
}


template <class K>
__device__ __forceinline__ uint32_t rs_digit(K k, int shift, uint32_t dmask) {
  return (uint32_t)(k >> shift) & dmask;
}

// Lanes of a wave holding the same value d (8-bit): a mask of them.
__device__ __forceinline__ uint64_t rs_peers(uint32_t d, bool valid) {
  uint64_t peers = __ballot(valid);
#pragma unroll
  for (int bb = 0; bb < 8; ++bb) {
    const bool bit = (d >> bb) & 1u;
    const uint64_t m = __ballot(bit);
    peers &= bit ? m : ~m;
  }
  return peers;
}

// Digit counts of every pass in one read of the keys. Each thread loads 16
// keys before counting them (memory parallelism), and the work-group keeps 8
// copies of each histogram, lane l counting into copy l % 8, so that the many
// equal digits of skewed keys (the high bits of power-law vertex ids) do not
// serialise on one LDS word. Dynamic LDS: passes * 256 * 8 words.
constexpr int kDigitCopies = 8;
constexpr int kDigitBatch = 16;

template <class K>
__global__ __launch_bounds__(256) void k_rs_digits(const K* __restrict__ kin, int64_t n, int bit_lo,
                                                   int bit_hi, uint32_t* __restrict__ ghist) {
  extern __shared__ uint32_t h_dyn[];  // [pass][digit][copy]
  const int tid = threadIdx.x;
  const int passes = (bit_hi - bit_lo + 7) / 8;
  for (int x = tid; x < passes * 256 * kDigitCopies; x += 256) h_dyn[x] = 0;
  __syncthreads();
  const int cp = tid & (kDigitCopies - 1);
  const int64_t stride = (int64_t)gridDim.x * 256 * kDigitBatch;
  for (int64_t base = (int64_t)blockIdx.x * 256 * kDigitBatch + tid; base < n; base += stride) {
    K k[kDigitBatch];
#pragma unroll
    for (int b = 0; b < kDigitBatch; ++b) {
      const int64_t i = base + (int64_t)b * 256;
      k[b] = i < n ? kin[i] : K(0);
    }
#pragma unroll
    for (int b = 0; b < kDigitBatch; ++b) {
      if (base + (int64_t)b * 256 >= n) break;
      for (int p = 0; p < passes; ++p) {
        const int shift = bit_lo + 8 * p;
        const int bits = bit_hi - shift < 8 ? bit_hi - shift : 8;
        atomicAdd(&h_dyn[(p * 256 + rs_digit(k[b], shift, (1u << bits) - 1u)) * kDigitCopies + cp], 1u);
      }
    }
  }
  __syncthreads();
  for (int p = 0; p < passes; ++p) {
    uint32_t t = 0;
#pragma unroll
    for (int c = 0; c < kDigitCopies; ++c) t += h_dyn[(p * 256 + tid) * kDigitCopies + c];
    if (t) atomicAdd(&ghist[p * 256 + tid], t);
  }
}

// Digit counts taken by the kernel that produces a sort's keys, so that the
// sort needs no read of its own: every work-group counts the keys it writes
// into LDS (layout and copies as in k_rs_digits; dynamic LDS of
// digit_lds_bytes) and adds its counts to a [passes][256] global histogram
// once, at the end. Pass the histogram to radix_sort (zeroed before the
// producer runs).
__host__ __device__ constexpr int digit_passes(int bit_lo, int bit_hi) { return (bit_hi - bit_lo + 7) / 8; }
inline size_t digit_lds_bytes(int bit_lo, int bit_hi) {
  return sizeof(uint32_t) * 256 * kDigitCopies * (size_t)digit_passes(bit_lo, bit_hi);
}

struct DigitCounter {
  uint32_t* h;  // LDS
  int bit_lo, bit_hi, passes, cp;
  __device__ void init(uint32_t* lds, int lo, int hi) {
    h = lds;
    bit_lo = lo;
    bit_hi = hi;
    passes = digit_passes(lo, hi);
    cp = threadIdx.x & (kDigitCopies - 1);
    for (int x = threadIdx.x; x < passes * 256 * kDigitCopies; x += blockDim.x) h[x] = 0;
    __syncthreads();
  }
  template <class K>
  __device__ void add(K k) const {
    for (int p = 0; p < passes; ++p) {
      const int shift = bit_lo + 8 * p;
      const int bits = bit_hi - shift < 8 ? bit_hi - shift : 8;
      atomicAdd(&h[(p * 256 + rs_digit(k, shift, (1u << bits) - 1u)) * kDigitCopies + cp], 1u);
    }
  }
  // all threads, after the block's last add
  __device__ void flush(uint32_t* __restrict__ ghist) const {
    __syncthreads();
    for (int x = threadIdx.x; x < passes * 256; x += blockDim.x) {
      uint32_t t = 0;
#pragma unroll
      for (int c = 0; c < kDigitCopies; ++c) t += h[x * kDigitCopies + c];
      if (t) atomicAdd(&ghist[x], t);
    }
  }
};

// In-place exclusive scan of each pass's 256 digit counts (one work-group).
static __global__ __launch_bounds__(256) void k_rs_buckets(uint32_t* __restrict__ ghist, int passes) {
  __shared__ uint32_t s_w[4];
  for (int p = 0; p < passes; ++p) {
    uint32_t tot;
    const uint32_t v = ghist[p * 256 + threadIdx.x];
    const uint32_t e = block_excl_scan(v, s_w, tot);
    ghist[p * 256 + threadIdx.x] = e;
    __syncthreads();
  }
}

template <class K, class V, int KPT, class W, int WIN, class Epi, class Src = NoSrc>
__global__ __launch_bounds__(256) void k_rs_onesweep(const K* __restrict__ kin, K* __restrict__ kout,
                                                     const V* __restrict__ vin, V* __restrict__ vout,
                                                     int64_t n, int shift, uint32_t dmask,
                                                     const uint32_t* __restrict__ bucket,
                                                     W* __restrict__ status,
                                                     uint32_t* __restrict__ ticket, int* __restrict__ fail,
                                                     Epi epi, Src src = Src{}) {
  constexpr int TILE = 256 * KPT;
  constexpr int WCH = 64 * KPT;  // keys of the tile each wave ranks (a contiguous quarter)
  constexpr bool HV = !std::is_same<V, NoVal>::value;
  constexpr W TOP = lb_top<W>();
  using VS = typename std::conditional<HV, V, char>::type;
  __shared__ K s_k[TILE];
  __shared__ VS s_v[HV ? TILE : 1];
  __shared__ uint32_t s_cnt[4][256];  // per wave and digit: count, then the wave's offset
  __shared__ uint32_t s_goff[256], s_tstart[256];
  __shared__ uint32_t s_tmp[4];
  __shared__ uint32_t s_tile;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  if (tid == 0) s_tile = atomicAdd(ticket, 1u);
#pragma unroll
  for (int w = 0; w < 4; ++w) s_cnt[w][tid] = 0;
  __syncthreads();
  const uint32_t tile = s_tile;
  const int64_t wbase = (int64_t)tile * TILE + (int64_t)wave * WCH;

  // the wave's quarter in registers: item i of lane l is input position
  // wbase + 64 i + l; with a source, bit i of vmask says whether the item is
  // a key of the sort (without one, the positions below n are)
  constexpr bool FROM_SRC = !std::is_same<Src, NoSrc>::value;
  K k[KPT];
  VS v[KPT];
  static_assert(KPT <= 32, "one mask bit per item");
  uint32_t vmask = 0;
#pragma unroll
  for (int i = 0; i < KPT; ++i) {
    const int64_t idx = wbase + 64 * i + lane;
    if constexpr (!FROM_SRC) {
      k[i] = idx < n ? kin[idx] : K(0);
      if constexpr (HV) v[i] = idx < n ? vin[idx] : V{};
    } else {
      // evaluated at a position in bounds (n >= 1) without a branch, so that
      // the loads of all items are issued together
      const bool ok = src(idx < n ? idx : n - 1, k[i], v[i]);
      vmask |= (uint32_t)(ok & (idx < n)) << i;
    }
  }
  auto is_key = [&](int i) -> bool {
    if constexpr (FROM_SRC) return (vmask >> i) & 1u;
    else return wbase + 64 * i + lane < n;
  };
  // stable rank within the wave's quarter; the wave's own LDS counters carry
  // the counts from item to item (a wave's LDS accesses complete in order)
  uint32_t rank[KPT];
  const uint64_t lt_mask = (1ull << lane) - 1ull;
  uint32_t* cnt_w = s_cnt[wave];
#pragma unroll
  for (int i = 0; i < KPT; ++i) {
    const bool valid = is_key(i);
    const uint32_t d = rs_digit(k[i], shift, dmask);
    const uint64_t peers = rs_peers(d, valid);
    const uint32_t before = cnt_w[d];
    rank[i] = before + (uint32_t)__popcll(peers & lt_mask);
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    if (valid && (peers & lt_mask) == 0) cnt_w[d] = before + (uint32_t)__popcll(peers);
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
  }
  __syncthreads();
  // digit `tid`: offsets of the waves within the tile's run, the tile's count
  uint32_t cnt = 0;
#pragma unroll
  for (int w = 0; w < 4; ++w) {
    const uint32_t c = s_cnt[w][tid];
    s_cnt[w][tid] = cnt;
    cnt += c;
  }
  // publish the tile's count; put the tile in digit order in LDS (while the
  // predecessors publish theirs); then look back for the earlier tiles'
  // total and publish the inclusive prefix
  W* my = status + (uint64_t)tile * 256 + tid;
  __hip_atomic_store(my, tile == 0 ? (TOP | (W)cnt) : (W)cnt + 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  uint32_t tot;
  s_tstart[tid] = block_excl_scan(cnt, s_tmp, tot);
  __syncthreads();
#pragma unroll
  for (int i = 0; i < KPT; ++i) {
    if (is_key(i)) {
      const uint32_t d = rs_digit(k[i], shift, dmask);
      const uint32_t lp = s_tstart[d] + s_cnt[wave][d] + rank[i];
      s_k[lp] = k[i];
      if constexpr (HV) s_v[lp] = v[i];
    }
  }
  if (tile == 0) {
    s_goff[tid] = bucket[tid];
  } else {
    // walk back WIN predecessors per step (their words are read together):
    // add counts from the nearest one until an inclusive prefix; stop at a
    // tile that has published nothing yet and read again from there
    uint64_t excl = 0;
    uint32_t spins = 0;
    int64_t j = (int64_t)tile - 1;
    while (j >= 0) {
      W w[WIN];
#pragma unroll
      for (int q = 0; q < WIN; ++q)
        w[q] = j - q >= 0 ? __hip_atomic_load(status + (uint64_t)(j - q) * 256 + tid, __ATOMIC_RELAXED,
                                              __HIP_MEMORY_SCOPE_AGENT)
                          : TOP;  // before tile 0: an inclusive prefix of 0
      int q = 0;
      bool done = false;
      for (; q < WIN; ++q) {
        if (w[q] == 0) break;
        if (w[q] & TOP) {
          excl += w[q] & ~TOP;
          done = true;
          break;
        }
        excl += w[q] - 1;
      }
      if (done) break;
      j -= q;
      if (q < WIN) {  // tile j has not published yet
        if (++spins > kLbSpinMax) {  // never expected: give up rather than hang
          atomicExch(fail, 1);
          break;
        }
        __builtin_amdgcn_s_sleep(1);
      }
    }
    __hip_atomic_store(my, TOP | (W)(excl + cnt), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    s_goff[tid] = bucket[tid] + (uint32_t)excl;
  }
  __syncthreads();
  // keys of the tile
  int tile_n;
  if constexpr (FROM_SRC) {
    tile_n = (int)tot;
  } else {
    const int64_t rem = n - (int64_t)tile * TILE;
    tile_n = rem < TILE ? (int)rem : TILE;
  }
#pragma unroll
  for (int i = 0; i < KPT; ++i) {
    const int lp = i * 256 + tid;
    if (lp < tile_n) {
      const K kk = s_k[lp];
      const uint32_t d = rs_digit(kk, shift, dmask);
      const uint64_t gp = (uint64_t)s_goff[d] + (uint64_t)(lp - (int)s_tstart[d]);
      kout[gp] = kk;
      if constexpr (HV) vout[gp] = s_v[lp];
      epi(gp, kk);
    }
  }
}

// Default keys per thread of a sort tile for key type K and value type V:
// tiles of 6144 4-byte, 8192 8-byte and 6144 12-byte elements (48-72 KiB of
// LDS), the fastest measured that keep the registers of a tile without
// spills (larger tiles halve the look-back words per key, but past these
// sizes a wave runs out of registers).
template <class K, class V>
constexpr int rs_default_kpt() {
  constexpr int e = (int)sizeof(K) + (std::is_same<V, NoVal>::value ? 0 : (int)sizeof(V));
  return e <= 4 ? 24 : e <= 8 ? 32 : e <= 12 ? 24 : 16;
}

// Sorts keys[0..n) by bits [bit_lo, bit_hi) (stable), carrying vals if V is
// not NoVal, with KPT keys per thread per tile and look-back words of type W
// (uint32_t needs n < 2^31). keys/vals and keys_alt/vals_alt are ping-pong
// buffers of n elements; returns true if the sorted data ended in the *_alt
// buffers. The last pass calls epi(final position, key) for every key (no
// pass runs, and epi is not called, when n <= 1). hist: the keys' digit
// counts ([passes][256], from a DigitCounter in the producing kernel; it is
// scanned in place; hist_scanned: it already holds each pass's exclusive
// digit starts, as a sort leaves them), or nullptr to count them here.
//
// With a source (src != nullptr), the n keys are those that *src selects
// from the input positions [0, n_in): the first pass reads them through
// *src and writes them to keys/vals, later passes ping-pong as above, and
// hist is required. Src is a functor
//   __device__ bool operator()(int64_t i, K& key, V& val) const
// (false: position i holds no key), evaluated once per position; it should
// not branch around its loads (compute the selection with & rather than &&),
// so that a tile's loads are issued together.
template <class K, class V, int KPT, class W, int WIN = kLbWin, class Epi = NoEpi, class Src = NoSrc,
          int KPT_SRC = KPT>
bool radix_sort_cfg(K* keys, K* keys_alt, V* vals, V* vals_alt, int64_t n, int bit_lo, int bit_hi,
                    hipStream_t st, const char* name, Epi epi = Epi{}, uint32_t* hist = nullptr,
                    const Src* src = nullptr, int64_t n_in = 0, bool hist_scanned = false) {
  constexpr int TILE = 256 * KPT;
  const char* n_digits = intern_name(std::string("rs_digits:") + name);
  const char* n_pass = intern_name(std::string("rs_pass:") + name);
  if (src) {
    if (n <= 0) return false;
    TC_REQUIRE(hist != nullptr && bit_hi > bit_lo && n <= n_in, TC_EINVAL, "radix_sort: bad source sort");
  } else if (n <= 1 || bit_hi <= bit_lo) {
    return false;
  }
  TC_REQUIRE(n < (int64_t)0xFFFFFFFFLL && n_in < (int64_t)0xFFFFFFFFLL, TC_EOVERFLOW,
             "radix_sort: more than 2^32-1 keys");
  TC_REQUIRE(sizeof(W) == 8 || n < ((int64_t)1 << 31), TC_EINVAL, "radix_sort: 32-bit look-back words");
  TC_REQUIRE(bit_hi - bit_lo <= 8 * kSortPassesMax, TC_EINVAL, "radix_sort: key range too wide");
  const int passes = (bit_hi - bit_lo + 7) / 8;
  const int64_t ntiles = div_up(n, TILE);
  const int64_t ntiles_in = src ? div_up(n_in, 256 * KPT_SRC) : ntiles;  // (the source pass: KPT_SRC per thread)
  int* fail = temp_ctx().fail;
  TC_REQUIRE(fail != nullptr, TC_EDEVICE, "radix_sort: called outside a TempStream scope");
  // per pass: ticket counter (padded to 256 bytes) + tiles * 256 look-back
  // words. Up to kLbClearOnceBytes for all passes, each pass has a region of
  // its own and one memset clears them all (with the digit counts when the
  // sort counts them itself); else the passes share one region, cleared
  // before each pass.
  const int64_t pad = 256 / (int64_t)sizeof(W);
  const int64_t pass_words = pad + std::max(ntiles, ntiles_in) * 256;
  const size_t region = sizeof(W) * (size_t)pass_words;
  const bool clear_once = (size_t)passes * region <= kLbClearOnceBytes;
  const size_t hist_bytes = hist ? 0 : sizeof(uint32_t) * 256 * kSortPassesMax;
  DevBuf work(hist_bytes + (clear_once ? (size_t)passes : 1) * region);
  char* lb0 = work.as<char>() + hist_bytes;
  if (clear_once) TC_HIP(hipMemsetAsync(work.p, 0, work.bytes, st));
  uint32_t* gh = hist;
  if (!gh) {
    gh = work.as<uint32_t>();
    if (!clear_once) TC_HIP(hipMemsetAsync(gh, 0, sizeof(uint32_t) * 256 * (size_t)passes, st));
    const unsigned dgrid = (unsigned)std::min<int64_t>(2048, div_up(n, 256 * 16));
    TC_LAUNCH(n_digits, (k_rs_digits<K>), dim3(dgrid), dim3(256), digit_lds_bytes(bit_lo, bit_hi), st, keys,
              n, bit_lo, bit_hi, gh);
  }
  if (!hist_scanned) TC_LAUNCH("rs_buckets", k_rs_buckets, dim3(1), dim3(256), 0, st, gh, passes);
  K* ka = keys;
  K* kb = keys_alt;
  V* va = vals;
  V* vb = vals_alt;
  bool alt = false;
  for (int p = 0; p < passes; ++p) {
    const int shift = bit_lo + 8 * p;
    const int bits = bit_hi - shift < 8 ? bit_hi - shift : 8;
    const uint32_t dmask = (1u << bits) - 1u;
    const bool last = p + 1 == passes;
    if (!clear_once) TC_HIP(hipMemsetAsync(lb0, 0, region, st));
    W* words = reinterpret_cast<W*>(lb0 + (clear_once ? (size_t)p * region : 0));
    uint32_t* ticket = reinterpret_cast<uint32_t*>(words);
    if (p == 0 && src) {  // from the source into keys/vals
      if (last)
        TC_LAUNCH(n_pass, (k_rs_onesweep<K, V, KPT_SRC, W, WIN, Epi, Src>), dim3((unsigned)ntiles_in), dim3(256), 0,
                  st, nullptr, ka, nullptr, va, n_in, shift, dmask, gh, words + pad, ticket, fail, epi, *src);
      else
        TC_LAUNCH(n_pass, (k_rs_onesweep<K, V, KPT_SRC, W, WIN, NoEpi, Src>), dim3((unsigned)ntiles_in), dim3(256),
                  0, st, nullptr, ka, nullptr, va, n_in, shift, dmask, gh, words + pad, ticket, fail, NoEpi{},
                  *src);
      TC_HIP(hipGetLastError());
      continue;
    }
    if (!last)
      TC_LAUNCH(n_pass, (k_rs_onesweep<K, V, KPT, W, WIN, NoEpi>), dim3((unsigned)ntiles), dim3(256), 0, st, ka,
                kb, va, vb, n, shift, dmask, gh + 256 * p, words + pad, ticket, fail, NoEpi{});
    else
      TC_LAUNCH(n_pass, (k_rs_onesweep<K, V, KPT, W, WIN, Epi>), dim3((unsigned)ntiles), dim3(256), 0, st, ka,
                kb, va, vb, n, shift, dmask, gh + 256 * p, words + pad, ticket, fail, epi);
    TC_HIP(hipGetLastError());
    std::swap(ka, kb);
    std::swap(va, vb);
    alt = !alt;
  }
  return alt;
}

// True when the environment variable TC_SORT_WIDE_WORDS is set to a non-zero
// value: sorts then use 64-bit look-back words at every size (the path that
// sorts of 2^31 keys or more take), so that tests reach it at small sizes.
bool sort_wide_words_forced();

template <class K, class V, class Epi = NoEpi>
bool radix_sort(K* keys, K* keys_alt, V* vals, V* vals_alt, int64_t n, int bit_lo, int bit_hi,
                hipStream_t st, const char* name, Epi epi = Epi{}, uint32_t* hist = nullptr) {
  constexpr int KPT = rs_default_kpt<K, V>();
  if (n < ((int64_t)1 << 31) && !sort_wide_words_forced())
    return radix_sort_cfg<K, V, KPT, uint32_t, kLbWin, Epi>(keys, keys_alt, vals, vals_alt, n, bit_lo, bit_hi,
                                                            st, name, epi, hist);
  return radix_sort_cfg<K, V, KPT, uint64_t, kLbWin, Epi>(keys, keys_alt, vals, vals_alt, n, bit_lo, bit_hi, st,
                                                          name, epi, hist);
}

// Stable sort of the n keys (and values) that src selects from the input
// positions [0, n_in) (the source form of radix_sort_cfg): they end in
// keys/vals if this returns false, else in keys_alt/vals_alt, each buffer
// holding n elements. hist: their digit counts ([passes][256]), taken by the
// kernel that counted the selected positions (a DigitCounter).
// KPT_SRC: items per thread of the source pass (a source that loads more
// than the key and value may need smaller tiles to keep its registers).
template <class K, class V, class Src, int KPT_SRC = rs_default_kpt<K, V>(), class Epi = NoEpi>
bool radix_sort_from(const Src& src, int64_t n_in, K* keys, K* keys_alt, V* vals, V* vals_alt, int64_t n,
                     int bit_lo, int bit_hi, uint32_t* hist, hipStream_t st, const char* name,
                     Epi epi = Epi{}, bool hist_scanned = false) {
  constexpr int KPT = rs_default_kpt<K, V>();
  if (n < ((int64_t)1 << 31) && !sort_wide_words_forced())
    return radix_sort_cfg<K, V, KPT, uint32_t, kLbWin, Epi, Src, KPT_SRC>(keys, keys_alt, vals, vals_alt, n,
                                                                          bit_lo, bit_hi, st, name, epi, hist,
                                                                          &src, n_in, hist_scanned);
  return radix_sort_cfg<K, V, KPT, uint64_t, kLbWin, Epi, Src, KPT_SRC>(keys, keys_alt, vals, vals_alt, n,
                                                                        bit_lo, bit_hi, st, name, epi, hist,
                                                                        &src, n_in, hist_scanned);
}

// Throws TC_EDEVICE if a sort of the current TempStream scope gave up waiting
// in its look-back (and clears the word). Synchronises st.
static inline void check_sorts(hipStream_t st) {
  int* fail = temp_ctx().fail;
  TC_REQUIRE(fail != nullptr, TC_EDEVICE, "check_sorts: called outside a TempStream scope");
  int h = 0;
  TC_HIP(hipMemcpyAsync(&h, fail, sizeof(int), hipMemcpyDeviceToHost, st));
  TC_HIP(hipStreamSynchronize(st));
  if (h) {
    TC_HIP(hipMemsetAsync(fail, 0, sizeof(int), st));
    TC_HIP(hipStreamSynchronize(st));
    throw Error(TC_EDEVICE, "radix sort: a look-back wait exceeded its bound");
  }
}

// Row pointers from keys sorted by row (row = key >> s): row_ptr[r] = first i
// with row(i) >= r (binary search per row), so row_ptr[n] = m.
template <class K>
__global__ void k_bounds(const K* __restrict__ keys, int64_t m, int s, int64_t n,
                         int64_t* __restrict__ row_ptr) {
  int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (r > n) return;
  int64_t lo = 0, hi = m;
  while (lo < hi) {
    int64_t mid = (lo + hi) >> 1;
    if ((int64_t)(keys[mid] >> s) < r) lo = mid + 1;
    else hi = mid;
  }
  row_ptr[r] = lo;
}

// Work-groups of a 256-thread launch that gives one wave to each of `items`
// items: at most kWaveGridMax, the kernel striding over the rest (one
// dispatch holds fewer than 2^32 work-items: a wave per row of a 2^26-vertex
// graph would be exactly 2^32).
constexpr int64_t kWaveGridMax = (int64_t)1 << 20;
inline unsigned wave_grid(int64_t items) {
  return (unsigned)std::max<int64_t>(1, std::min<int64_t>(kWaveGridMax, div_up(items, 4)));
}

// Row of every entry of a CSR: erow[i] = r for row_ptr[r] <= i < row_ptr[r + 1]
// (one wave per row, coalesced writes; grid: wave_grid(nrows) x 256).
static __global__ __launch_bounds__(256) void k_entry_rows(const int64_t* __restrict__ row_ptr, int64_t nrows,
                                                           uint32_t* __restrict__ erow) {
  const int64_t stride = (int64_t)gridDim.x * (blockDim.x / 64);
  for (int64_t r = (int64_t)blockIdx.x * (blockDim.x / 64) + (threadIdx.x >> 6); r < nrows; r += stride) {
    const int64_t s = row_ptr[r], e = row_ptr[r + 1];
    for (int64_t i = s + (threadIdx.x & 63); i < e; i += 64) erow[i] = (uint32_t)r;
  }
}

// Tasks in hashed-row order (the input of build_work).
struct TaskLists {
  int64_t T = 0;
  DevBuf row;     // uint32 [T]: hashed row of each task
  DevBuf val;     // uint64 [T]: first probe | (end of the probe range) << 32
  DevBuf prefix;  // uint64 [T + 1]: exclusive prefix of the probe counts, total at [T]
  DevBuf ptr;     // int64 [nrows + 1]: tasks of row b are [ptr[b], ptr[b + 1])
};

// Sort T emitted tasks (tk = hashed row in [0, 2^key_bits), tv = first
// probe | end << 32) stably by row and fill `tl`. tk / tv are consumed as
// sort buffers (tl may take them over).
void sort_tasks(TaskLists& tl, DevBuf& tk, DevBuf& tv, int64_t T, int64_t nrows, int key_bits,
                hipStream_t st, const char* name);
// Probe prefixes (tl.prefix) and row pointers (tl.ptr, allocated by the
// caller with nrows + 1 entries) of the tl.T tasks in tl.row / tl.val,
// sorted by row; the tail of sort_tasks.
void finish_tasks(TaskLists& tl, int64_t nrows, hipStream_t st);
// check_sorts for the task sorts of sort_tasks (synchronises st).
void check_task_sorts(hipStream_t st);

}  // namespace tc
