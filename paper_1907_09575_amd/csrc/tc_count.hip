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
// Hash table (Section 5.2's change to the hashing routine): U_b in LDS in
// buckets of four 32-bit slots, bucket = k & (buckets - 1) (the direct bitwise
// AND of the paper), at least 4 |U_b| slots (2 |U_b| for rows of more than
// 2048 keys). A key goes to the first free slot of its bucket or, if the
// bucket is full, of the next ones; slots fill left to right, so a lookup
// reads one bucket with a single 16-byte LDS read and stops there unless the
// bucket is full. The build records the longest bucket displacement D, which
// bounds every lookup; exactness never depends on the absence of collisions.
//
// Probe loop (one wave, flattened over tasks). A wave walks a range of
// probes in batches of 64, lane l taking probe base + l, so every col[] read
// is a coalesced run; kU batches form a super-batch whose loads and lookups
// are all in flight together. A window of 64 consecutive tasks sits one per
// lane (end of the task relative to the wave's position, and the col index its
// probes start from); the next window is prefetched while the current one is
// probed. The task of a probe r is c0 (tasks ended at or before the
// super-batch start, one ballot) plus the number of task ends inside the
// super-batch that lie at or before r: ends set bits of a per-wave LDS bitmap,
// whose words are read back as wave-uniform masks and counted per lane with
// mbcnt. The task's col base then comes from its lane by one bpermute.
// Probe reads are raw buffer loads with a 32-bit byte offset; a lane past the
// range gets an offset beyond the buffer and reads 0, which is never a key of
// U_b (every key exceeds b >= 0), so it needs no branch.
//
// Launch classes (decided in preprocessing from |U_b| and the row's probes):
//   packs  - light rows b are packed (up to 256 rows per work-group); the
//            work-group builds all their tables in LDS, then its waves probe
//            the pack's task range, each task looking up its own row's table.
//   heavy  - a row's probes are cut into per-wave ranges (16K probes); the 4
//            waves of a work-group share one table of that row. One launch per
//            table size class (wg_small / wg_large / wg_huge / wg_giant), each
//            compiled for the occupancy its LDS allows.
//   global - a row whose table would not fit LDS (|U_b| > 8192): lookups are
//            binary searches in the sorted U_b in HBM.
// Reductions: per-lane 32-bit hit counters, wave reduction by xor shuffles,
// one 64-bit atomic per work-group into the caller's counter (order-free and
// exact).
#include "tc_prims.h"

namespace tc {

namespace {

using Args = CountArgs;

constexpr int kU = 8;                   // 64-probe batches per super-batch
constexpr int kBmWords = 2 * kU;        // per-wave task-end bitmap (64 * kU bits)
constexpr int kMarkInts = kWaves * kBmWords;          // packs
constexpr int kItemMarkInts = kWavesBig * kBmWords;   // item work-groups (up to 8 waves)

constexpr int32_t kEmpty = -1;
// FULL support, single-row LDS tables: a slot's value word is the key's index
// in its row (< 2^13: such rows have at most 8192 keys) plus its hits in this
// work-group times 2^13 (at most one per task, and a work-group holds at most
// 8 wave items of at most 32767 probes: < 2^18, so the word stays below 2^31).
constexpr int kValBits = 13;
static_assert((1 << kValBits) >= (1 << kMaxLog2S) / 2, "row index of an LDS table below the hit count");
static_assert((uint64_t)kWavesBig * kWaveChunkMax < (1ull << (31 - kValBits)),
              "hits of one slot in one work-group keep the value word below 2^31");
constexpr uint32_t kOffNone = 0xFFFFFFF0u;  // byte offset past any col buffer

__device__ __forceinline__ void wave_sync_lds() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

__device__ __forceinline__ __amdgpu_buffer_rsrc_t col_rsrc(const int32_t* col, uint32_t m) {
  // raw buffer over col[0, m): stride 0, num_records = bytes; reads at or past
  // the end return 0
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<int32_t*>(col), (short)0, (int)(m * 4u),
                                           0x00020000);
}

__device__ __forceinline__ int32_t col_load(__amdgpu_buffer_rsrc_t r, uint32_t byte_off) {
  return __builtin_amdgcn_raw_buffer_load_b32(r, byte_off, 0, 0);
}

// Code variants of the count kernels (template argument VAR):
//   VAR_BASE  - the direct AND of Section 5.2; probes read by raw buffer loads
//               with 32-bit byte offsets (probe sides of fewer than 2^30
//               entries);
//   VAR_MUL   - the ablation of the direct AND (tc_graph_variant): a
//               multiplicative hash for every table;
//   VAR_WIDE  - probe sides of 2^30 entries or more: probes read with 64-bit
//               addresses (positions stay 32-bit), masked for lanes past the
//               range.
enum CountVariant : int { VAR_BASE = 0, VAR_MUL = 1, VAR_WIDE = 2 };

// Bucket of key k in a table of bmask + 1 buckets: the direct bitwise AND of
// Section 5.2 (the key's low bits), or, MH (the ablation of that choice,
// tc_graph_variant), a multiplicative hash: the top log2(buckets) bits of
// k times 2^32 / golden ratio.
template <bool MH>
__device__ __forceinline__ uint32_t bucket_of(int32_t k, uint32_t bmask) {
  if constexpr (!MH) {
    return (uint32_t)k & bmask;
  } else {
    const uint32_t B = (uint32_t)__popc(bmask);
    return (uint32_t)(((uint64_t)((uint32_t)k * 0x9E3779B1u) << B) >> 32);
  }
}

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

// Insert U_b = col[rs, rs + d) into a cleared bucketed table of (bmask + 1)
// buckets; threads tid, tid + nt, ... share the work. Returns this thread's
// longest bucket displacement. VALS: also store every key's index in the row
// (its U position is rs + index), with a zero hit count above it.
template <bool VALS, bool MH>
__device__ int build_table(int32_t* tab, int32_t* val, uint32_t bmask, const int32_t* __restrict__ col,
                           int64_t rs, int64_t d, int tid, int nt) {
  constexpr int kB = 8;  // keys fetched at once so that their loads overlap
  int md = 0;
  for (int64_t i0 = tid; i0 < d; i0 += (int64_t)kB * nt) {
    int32_t key[kB];
#pragma unroll
    for (int j = 0; j < kB; ++j) {
      const int64_t i = i0 + (int64_t)j * nt;
      key[j] = i < d ? col[rs + i] : kEmpty;
    }
#pragma unroll
    for (int j = 0; j < kB; ++j) {
      if (key[j] == kEmpty) continue;
      uint32_t bk = bucket_of<MH>(key[j], bmask);
      int disp = 0;
      int slot = -1;
      while (true) {
#pragma unroll
        for (int s = 0; s < kBucket; ++s) {
          if (slot < 0 && atomicCAS(&tab[bk * kBucket + s], kEmpty, key[j]) == kEmpty)
            slot = (int)(bk * kBucket + s);
        }
        if (slot >= 0) break;
        bk = (bk + 1) & bmask;
        ++disp;
      }
      if (VALS) val[slot] = (int32_t)(i0 + (int64_t)j * nt);
      md = disp > md ? disp : md;
    }
  }
  return md;
}

// FULL support in packs: a pack of fewer than 2^17 probes keeps its (b, k)
// credits in LDS, the slot's value word holding the key's index in the pack's
// key list (kPackValBits, below 2^15 since a pack has at most kPackSlotsMax
// plus 1024 slots) plus its hits shifted by kPackValBits (at most the pack's
// probes, so the word stays below 2^32); larger packs hold U positions and
// credit (b, k) per hit.
constexpr int kPackValBits = 15;
static_assert(kPackSlotsMax + 1024 <= (1u << kPackValBits), "a pack's key index fits its field");
constexpr uint64_t kPackLdsHitsMax = (uint64_t)1 << (32 - kPackValBits);

struct TableRef {
  const int32_t* tab;  // (bmask + 1) * kBucket slots (a pack: all its rows' tables)
  int32_t* val;        // FULL support: single-row tables hold row index | hits <<
                       // kValBits, packs key index | hits << kPackValBits (both
                       // summed in LDS) or, in packs of 2^17 probes or more, U
                       // positions
  uint32_t bmask;
  int D;
  int64_t rs, d;  // the row itself (HBM fallback)
  // packs: row i of the pack owns tasks [row_t0[i], row_t0[i + 1]) and the
  // table at bucket (desc & 0xFFFF) with (desc >> 16) + 1 buckets
  const uint32_t* row_t0;
  const uint32_t* row_desc;
  int nrows;
  int lds_hits;  // packs, FULL: the (b, k) credits are counted in LDS
};

enum TableKind : int { TK_SINGLE = 0, TK_MULTI = 1, TK_GLOBAL = 2 };

// A hit: k = col[pos] was found in U_b at `where` (an LDS slot, or for the HBM
// fallback its position in col); ts is the first probe position of the task,
// so ts - 1 is the U entry of the task's own edge (a, b).
// Per-shift triangle counters of one work-group (MODE_BLOCK).
__device__ unsigned int* shift_counters() {
  __shared__ unsigned int s_shift[64];
  return s_shift;
}

// The per-hit credits other than the task's own edge (a, b), which goes
// through the wave's per-task counters (wave_probe). BLOCK: the shift
// counter of k; FULL: the probed entry (a, k) of U_a and k's entry (b, k) of
// U_b.
template <int MODE, int KIND>
__device__ __forceinline__ void credit(const Args& A, const TableRef& t, int where, uint32_t pos, int32_t k) {
  // indices are checked against m so that no credit can leave the array
  if (MODE == MODE_BLOCK) {
    // shift z of Eq. 5 closes the triangle with k = x + y + z (mod q)
    int z = (int)((uint32_t)k % (uint32_t)A.q) - A.xy;
    if (z < 0) z += A.q;
    atomicAdd(&shift_counters()[z], 1u);
  } else if (MODE == MODE_SUPPORT_FULL) {
    if (pos < A.m) atomicAdd(&A.support[pos], 1);  // edge (a, k): probed entry of U_a
    // edge (b, k): k's entry in U_b. A single-row table counts it in the
    // slot's LDS word (added to the array once per work-group, after the
    // probe loop of items_body).
    if (KIND == TK_SINGLE) {
      atomicAdd(&t.val[where], 1 << kValBits);
    } else if (KIND == TK_MULTI && t.lds_hits) {
      atomicAdd(reinterpret_cast<unsigned int*>(&t.val[where]), 1u << kPackValBits);
    } else {
      const uint32_t other = (uint32_t)(KIND == TK_GLOBAL ? where : t.val[where]);
      if (other < A.m) atomicAdd(&A.support[other], 1);
    }
  }
}

// Support modes credit every hit to its task's own edge (a, b) through the
// task window: lane j owns window task j and keeps its hits in a register.
// The lanes of one task are a contiguous run of each 64-probe batch, so after
// a batch's lookups lane j adds the hits of its run - the batch's hit ballot
// masked to the lanes [lo, hi) its task covers; when the window moves on (or
// the wave's range ends) it adds them to the task's edge with one global
// atomic. A task cut between waves gets one atomic from each.
__device__ __forceinline__ uint64_t lane_range_mask(int lo, int hi) {
  lo = lo < 0 ? 0 : (lo > 64 ? 64 : lo);
  hi = hi < 0 ? 0 : (hi > 64 ? 64 : hi);
  if (hi <= lo) return 0;
  const uint64_t below_hi = hi >= 64 ? ~0ull : ((1ull << hi) - 1ull);
  return below_hi & ~((1ull << lo) - 1ull);
}

// Count mode needs only whether the bucket holds k: an OR of four compares
// (no slot index, no branch).
__device__ __forceinline__ bool bucket_has(const int4& v, int32_t k) {
  return (v.x == k) | (v.y == k) | (v.z == k) | (v.w == k);
}

__device__ __forceinline__ int match_slot(const int4& v, int32_t k) {
  return v.x == k ? 0 : v.y == k ? 1 : v.z == k ? 2 : v.w == k ? 3 : -1;
}

// The first window of a wave's probe range [q, q + len) (task t holds probe
// q): each lane's task end, relative to q and clamped to len, and first-probe
// position, and the window's own start. Loaded before the table is built, so
// that these loads overlap the build.
struct Window {
  uint32_t Pe, tsj, P0;
};

__device__ __forceinline__ Window window_first(const Args& A, uint32_t t, uint64_t q, uint32_t len) {
  const int lane = lane_id();
  const int64_t T = A.T;
  const int64_t tj = (int64_t)t + lane;
  const uint64_t p = A.tprefix[tj + 1 < T ? tj + 1 : T] - q;
  Window w;
  w.Pe = p > (uint64_t)len ? len : (uint32_t)p;
  w.tsj = A.tstart[tj < T ? tj : T - 1];
  w.P0 = (uint32_t)(A.tprefix[t] - q);  // may wrap (a task starting before q)
  return w;
}

// One wave processes the probes [q, q + len) of the tasks of one hashed row;
// task t contains probe q; w0 = window_first(A, t, q, len).
template <int MODE, int KIND, int VAR>
__device__ void wave_probe(const Args& A, const TableRef& tr, uint32_t t, uint64_t q, uint32_t len,
                           uint32_t* bm, uint32_t& hits, const Window& w0) {
  // the range is the wave's own (uniform across its lanes): scalar registers
  // (readfirstlane returns int: widen through uint32_t, never sign-extend)
  t = (uint32_t)__builtin_amdgcn_readfirstlane((int)t);
  len = (uint32_t)__builtin_amdgcn_readfirstlane((int)len);
  q = ((uint64_t)(uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)(q >> 32)) << 32) |
      (uint64_t)(uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)q);
  constexpr bool GLOBAL = KIND == TK_GLOBAL;
  constexpr bool MULTI = KIND == TK_MULTI;
  constexpr bool MH = VAR == VAR_MUL, WIDE = VAR == VAR_WIDE;
  constexpr bool kTaskHits = MODE == MODE_SUPPORT_FULL || MODE == MODE_SUPPORT_ORIENTED;
  constexpr uint32_t SB = 64u * kU;
  const int lane = lane_id();
  const int64_t T = A.T;
  const __amdgpu_buffer_rsrc_t rsrc = col_rsrc(A.col, A.m);
  const int4* tab4 = reinterpret_cast<const int4*>(tr.tab);

  // window of tasks t .. t + 63, one per lane: end prefix and col start (the
  // start prefix of a task is the end prefix of the previous one). Prefixes
  // are kept relative to the range start q0 in 32 bits: ends are clamped to
  // len (a task ending past the range is cut there; the start of a task that
  // begins past the range is never used), and a start before q0 wraps.
  const uint64_t q0 = q;
  auto fetch = [&](int64_t tj, uint32_t& Pe, uint32_t& ts) {
    const uint64_t p = A.tprefix[tj + 1 < T ? tj + 1 : T] - q0;
    Pe = p > (uint64_t)len ? len : (uint32_t)p;
    ts = A.tstart[tj < T ? tj : T - 1];
  };
  uint32_t Pe = w0.Pe;
  uint32_t tsj = w0.tsj;
  uint32_t P0 = (uint32_t)__builtin_amdgcn_readfirstlane((int)w0.P0);  // start of the window's first task

  uint32_t done = 0;
  uint32_t tcnt = 0;  // support modes: hits of this lane's window task
  while (done < len) {
    const uint32_t rem = len - done;
    // end of the lane's task relative to the current position, within the range
    const uint32_t e = Pe - done;
    // start of the lane's task relative to the current position (wraps below
    // it for lane 0 when the range begins inside its task), so cbase = col
    // index of relative probe 0
    const uint32_t e_prev = (uint32_t)__shfl_up((int)e, 1, 64);
    const uint32_t s_rel = lane == 0 ? P0 - done : e_prev;
    const uint32_t cbase = tsj - s_rel;
    // probes of this window (wave-uniform: kept in a scalar register)
    const uint32_t lim = (uint32_t)__builtin_amdgcn_readfirstlane(__shfl((int)e, 63, 64));
    if (lim == 0) break;  // unreachable when every task has a probe; guards progress
    // packs: the table of the lane's task (last row whose first task <= it)
    uint32_t tdesc = 0;
    if constexpr (MULTI) {
      const uint32_t tj = t + (uint32_t)lane;
      int lo = 0, hi = tr.nrows;  // row_t0[lo] <= tj (lanes past the pack clamp to the last row)
      while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (tr.row_t0[mid] <= tj) lo = mid;
        else hi = mid;
      }
      tdesc = tr.row_desc[lo];
    }
    const bool more = lim < rem;
    uint32_t nPe = 0;
    uint32_t ntsj = 0;
    if (more) fetch((int64_t)t + 64 + lane, nPe, ntsj);  // next window, in flight meanwhile

    for (uint32_t sb = 0; sb < lim; sb += SB) {
      const uint32_t c0 = (uint32_t)__popcll(__ballot(e <= sb));
      const bool inner = e > sb && e <= sb + SB;
      uint32_t jl[kU];
      if (__ballot(inner) == 0) {
#pragma unroll
        for (int u = 0; u < kU; ++u) jl[u] = c0;
      } else {
        // bit p set <=> some task ends right after probe sb + p
        if (inner) atomicOr(&bm[(e - sb - 1) >> 5], 1u << ((e - sb - 1) & 31));
        wave_sync_lds();
        uint32_t pre = c0;
#pragma unroll
        for (int u = 0; u < kU; ++u) {
          const uint32_t lo = __builtin_amdgcn_readfirstlane(bm[2 * u]);
          const uint32_t hi = __builtin_amdgcn_readfirstlane(bm[2 * u + 1]);
          jl[u] = __builtin_amdgcn_mbcnt_hi(hi, __builtin_amdgcn_mbcnt_lo(lo, pre));
          pre += (uint32_t)__builtin_popcount(lo) + (uint32_t)__builtin_popcount(hi);
        }
        wave_sync_lds();
        if (lane < (int)(SB / 32)) bm[lane] = 0;
        wave_sync_lds();
      }
      uint32_t pos[kU], bbase[kU], bmask[kU];
      int32_t k[kU];
      bool ok[kU];
      uint32_t fmask = 0;  // support modes: bit u = this lane's probe of batch u hit
#pragma unroll
      for (int u = 0; u < kU; ++u) {
        // ds_bpermute uses lane index bits only, so lanes past the window
        // (jl >= 64, never used) wrap harmlessly
        const uint32_t r = sb + 64u * u + (uint32_t)lane;
        pos[u] = (uint32_t)__builtin_amdgcn_ds_bpermute((int)(jl[u] << 2), (int)cbase) + r;
        ok[u] = r < lim;
        if constexpr (MULTI) {
          const uint32_t dsc = (uint32_t)__builtin_amdgcn_ds_bpermute((int)(jl[u] << 2), (int)tdesc);
          bbase[u] = dsc & 0xFFFFu;
          bmask[u] = dsc >> 16;
        } else {
          bbase[u] = 0;
          bmask[u] = tr.bmask;
        }
      }
#pragma unroll
      for (int u = 0; u < kU; ++u) {
        if constexpr (WIDE) k[u] = ok[u] ? A.col[(uint64_t)pos[u]] : 0;
        else k[u] = col_load(rsrc, ok[u] ? pos[u] * 4u : kOffNone);
      }

      if constexpr (!GLOBAL) {
        // buckets are read in groups of kG so that the 16-byte results of one
        // group fit the register budget of 8 waves per SIMD
        constexpr int kG = 2;
        uint32_t bk[kU];
        bool unres[kU];
        bool any_unres = false;
#pragma unroll
        for (int g0 = 0; g0 < kU; g0 += kG) {
          int4 v[kG];
#pragma unroll
          for (int u = g0; u < g0 + kG; ++u) {
            bk[u] = bbase[u] + bucket_of<MH>(k[u], bmask[u]);
            v[u - g0] = tab4[bk[u]];
          }
#pragma unroll
          for (int u = g0; u < g0 + kG; ++u) {
            bool found;
            if constexpr (MODE == MODE_COUNT || MODE == MODE_SUPPORT_ORIENTED) {
              found = bucket_has(v[u - g0], k[u]);
            } else {
              const int j = match_slot(v[u - g0], k[u]);
              found = j >= 0;
              if (found) credit<MODE, KIND>(A, tr, (int)(bk[u] * kBucket + j), pos[u], k[u]);
            }
            hits += found ? 1u : 0u;
            if (kTaskHits) fmask |= (found ? 1u : 0u) << u;
            unres[u] = ok[u] & !found & (v[u - g0].w != kEmpty);
            any_unres |= unres[u];
          }
        }
        // full first bucket: continue into the next ones (bounded by D)
        if (tr.D > 0 && __ballot(any_unres)) {
#pragma unroll
          for (int u = 0; u < kU; ++u) {
            uint32_t b2 = bk[u] - bbase[u];
            for (int i = 1; i <= tr.D && unres[u]; ++i) {
              b2 = (b2 + 1) & bmask[u];
              const int4 w = tab4[bbase[u] + b2];
              bool found;
              if constexpr (MODE == MODE_COUNT || MODE == MODE_SUPPORT_ORIENTED) {
                found = bucket_has(w, k[u]);
              } else {
                const int j = match_slot(w, k[u]);
                found = j >= 0;
                if (found) credit<MODE, KIND>(A, tr, (int)((bbase[u] + b2) * kBucket + j), pos[u], k[u]);
              }
              hits += found ? 1u : 0u;
              if (kTaskHits) fmask |= (found ? 1u : 0u) << u;
              unres[u] = !found & (w.w != kEmpty);
            }
          }
        }
      } else {
#pragma unroll
        for (int u = 0; u < kU; ++u) {
          const int64_t where = ok[u] ? hbm_find(A.hcol, tr.rs, tr.d, k[u]) : -1;
          if (where >= 0) {
            ++hits;
            if (MODE != MODE_COUNT) credit<MODE, TK_GLOBAL>(A, tr, (int)where, pos[u], k[u]);
            if (kTaskHits) fmask |= 1u << u;
          }
        }
      }
      if constexpr (kTaskHits) {
        // this lane's task covers the relative probes [s_rel, e) (s_rel may
        // be below 0 for lane 0); add the hits of batch u that fall there
        const int ts0 = (int)s_rel, te0 = (int)e;
#pragma unroll
        for (int u = 0; u < kU; ++u) {
          const uint64_t hm = __ballot((fmask >> u) & 1u);
          if (hm) {
            const int base = (int)(sb + 64u * (uint32_t)u);
            tcnt += (uint32_t)__popcll(hm & lane_range_mask(ts0 - base, te0 - base));
          }
        }
      }
    }
    if (kTaskHits && tcnt) {  // the window task's own edge
      if (tsj - 1u < A.m) atomicAdd(&A.support[tsj - 1u], (int)tcnt);
      tcnt = 0;
    }
    if (more) {
      t += 64;  // a window that is not the last covers exactly its 64 tasks
      P0 = done + lim;
      Pe = nPe;
      tsj = ntsj;
    }
    done += lim;
  }
}

// Work-group total of the hits (returned to thread 0, which also adds it to
// A.count when that is set).
template <int MODE>
__device__ __forceinline__ unsigned long long block_flush(uint32_t hits, const Args& A) {
  __shared__ unsigned long long s_sum[kWavesBig];
  unsigned long long h = wave_sum((unsigned long long)hits);
  if (lane_id() == 0) s_sum[threadIdx.x >> 6] = h;
  __syncthreads();
  unsigned long long tot = 0;
  if (threadIdx.x == 0) {
    const int nw = (int)(blockDim.x >> 6);
    for (int w = 0; w < nw; ++w) tot += s_sum[w];
    if (A.count && tot) atomicAdd(A.count, tot);
  }
  if (MODE == MODE_BLOCK && A.per_shift && (int)threadIdx.x < A.q) {
    const unsigned int c = shift_counters()[threadIdx.x];
    if (c) atomicAdd(&A.per_shift[threadIdx.x], (unsigned long long)c);
  }
  return tot;
}

// Clear the work-group's shift counters (MODE_BLOCK); a barrier follows in
// every kernel before any credit.
template <int MODE>
__device__ __forceinline__ void block_init() {
  if (MODE == MODE_BLOCK && threadIdx.x < 64) shift_counters()[threadIdx.x] = 0;
}

// Packs of light rows (one work-group each): up to kPackRows rows, one per
// thread for its metadata; all their tables are built together in LDS (keys
// flattened over the work-group), then the pack's probe range - the tasks of
// its rows are contiguous - is split over the 4 waves and probed flattened,
// each task looking up its own row's table.
constexpr int kPackMetaWords = 3 * kPackRows + 1;  // row_t0, row_desc, key prefix (+ end)

template <int MODE, int VAR>
__device__ __forceinline__ unsigned long long pack_body(const Args& A, const PackRow* __restrict__ recs,
                                          const PackInfo* __restrict__ info, uint32_t pack,
                                          uint32_t pack_slots, int32_t* smem) {
  __shared__ int s_D;
  __shared__ uint32_t s_w[4], s_w2[4];
  constexpr bool VALS = MODE == MODE_SUPPORT_FULL;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  uint32_t* bm = reinterpret_cast<uint32_t*>(smem) + wave * kBmWords;
  uint32_t* row_t0 = reinterpret_cast<uint32_t*>(smem) + kMarkInts;
  uint32_t* row_desc = row_t0 + kPackRows;
  uint32_t* row_k0 = row_desc + kPackRows;  // kPackRows + 1 entries
  int32_t* tab = smem + kMarkInts + kPackMetaWords + 3;  // + 3 keeps 16-byte alignment
  int32_t* val = tab + pack_slots;
  if (lane < kBmWords) bm[lane] = 0;
  block_init<MODE>();

  const PackInfo& pi = info[pack];
  const uint32_t r0 = pi.r0, r1 = pi.r1;
  const int nr = (int)(r1 - r0);  // 1 .. kPackRows
  // this wave's quarter of the pack's probes, its first task, and its first
  // window (in flight while the tables are built)
  const uint64_t q0 = pi.q0, W = pi.q1 - pi.q0;
  const uint64_t wq0 = q0 + W * (uint64_t)wave / kWaves, wq1 = q0 + W * (uint64_t)(wave + 1) / kWaves;
  const uint32_t wt = (uint32_t)__builtin_amdgcn_readfirstlane((int)pi.wt[wave]);
  const uint32_t wlen = (uint32_t)(wq1 - wq0);
  const Window w0 = window_first(A, wt, wq0, wlen);
  const bool lds_hits = VALS && W < kPackLdsHitsMax;  // (uniform: the pack's probes)
  uint32_t d = 0, S = 0, rs = 0;
  if (tid < nr) {
    const PackRow pr = recs[r0 + tid];
    rs = pr.rs;
    // a row without tasks (a pack member only without the doubly sparse
    // traversal, tc_graph_variant) has d = 0: no table
    d = pr.d;
    S = 1u << pack_table_log2(d);
    row_t0[tid] = pr.tb;
  }
  uint32_t S_tot, K_tot;
  const uint32_t off = block_excl_scan(S, s_w, S_tot);
  const uint32_t k0 = block_excl_scan(d, s_w2, K_tot);
  if (tid < nr) {
    row_desc[tid] = (off / kBucket) | ((S / kBucket - 1) << 16);
    row_k0[tid] = k0;
  }
  if (tid == 0) {
    row_k0[nr] = K_tot;
    s_D = 0;
  }
  for (uint32_t i = tid; i < S_tot; i += 256) tab[i] = kEmpty;
  __syncthreads();

  // build: key x of the pack belongs to the last row i with row_k0[i] <= x;
  // this thread also remembers its own row's start (rows are few per thread)
  __shared__ uint32_t s_rs[kPackRows];
  if (tid < nr) s_rs[tid] = rs;
  __syncthreads();
  int md = 0;
  for (uint32_t x = tid; x < K_tot; x += 256) {
    int lo = 0, hi = nr;
    while (hi - lo > 1) {
      const int mid = (lo + hi) >> 1;
      if (row_k0[mid] <= x) lo = mid;
      else hi = mid;
    }
    const uint32_t p = s_rs[lo] + (x - row_k0[lo]);
    const int32_t key = A.hcol[p];
    const uint32_t dsc = row_desc[lo];
    const uint32_t base = dsc & 0xFFFFu, bmask = dsc >> 16;
    uint32_t bk = bucket_of<VAR == VAR_MUL>(key, bmask);
    int disp = 0, slot = -1;
    while (true) {
#pragma unroll
      for (int s2 = 0; s2 < kBucket; ++s2) {
        if (slot < 0 && atomicCAS(&tab[(base + bk) * kBucket + s2], kEmpty, key) == kEmpty)
          slot = (int)((base + bk) * kBucket + s2);
      }
      if (slot >= 0) break;
      bk = (bk + 1) & bmask;
      ++disp;
    }
    if (VALS) val[slot] = lds_hits ? (int32_t)x : (int32_t)p;  // key index, or U position
    md = disp > md ? disp : md;
  }
  // (a plain LDS max per lane: a wave reduction here would share its lane
  // addresses with the final one and keep them live across the probe loop)
  if (md) atomicMax(&s_D, md);
  __syncthreads();

  TableRef tr{tab, val, 0, s_D, 0, 0, row_t0, row_desc, nr, lds_hits ? 1 : 0};
  uint32_t hits = 0;
  if (wlen > 0) wave_probe<MODE, TK_MULTI, VAR>(A, tr, wt, wq0, wlen, bm, hits, w0);
  if constexpr (VALS) {
    if (lds_hits) {
      // the (b, k) credits of the pack: one atomic per slot that was hit, at
      // the U position of its key (row found from the key index)
      __syncthreads();
      for (uint32_t i = tid; i < S_tot; i += 256) {
        if (tab[i] == kEmpty) continue;
        const uint32_t w = (uint32_t)val[i];
        const uint32_t c = w >> kPackValBits;
        if (c == 0) continue;
        const uint32_t x = w & ((1u << kPackValBits) - 1u);
        int lo = 0, hi = nr;
        while (hi - lo > 1) {
          const int mid = (lo + hi) >> 1;
          if (row_k0[mid] <= x) lo = mid;
          else hi = mid;
        }
        const uint32_t p = s_rs[lo] + (x - row_k0[lo]);
        if (p < A.m) atomicAdd(&A.support[p], (int)c);
      }
    }
  }
  return block_flush<MODE>(hits, A);
}

// Register budgets (waves per SIMD) of the pack kernel and of the persistent
// batch kernel in count mode (their LDS use would allow about 6 work-groups per
// CU; 5 with spill-free registers runs faster).
constexpr int kOccPacks = 5, kOccBatch = 5;

template <int MODE, int VAR>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(
    MODE == MODE_COUNT || MODE == MODE_SUPPORT_ORIENTED ? kOccPacks : 4)))
void k_count_packs(Args A, const PackRow* __restrict__ recs, const PackInfo* __restrict__ info,
                   uint32_t pack_slots) {
  extern __shared__ int4 smem4[];  // 16-byte aligned: tables are read as int4 buckets
  pack_body<MODE, VAR>(A, recs, info, blockIdx.x, pack_slots, reinterpret_cast<int32_t*>(smem4));
}

// Heavy rows: work-group = kWaves consecutive items of the same row b.
template <int MODE, bool GLOBAL, int VAR>
__device__ __forceinline__ unsigned long long items_body(const Args& A, const CountItem* __restrict__ grp,
                                                         int32_t* smem) {
  __shared__ int s_D;
  constexpr bool VALS = MODE == MODE_SUPPORT_FULL;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  uint32_t* bm = reinterpret_cast<uint32_t*>(smem) + wave * kBmWords;
  const int32_t b = grp[0].b;
  const int64_t rs = A.row_ptr[b], d = A.row_ptr[b + 1] - rs;
  // this wave's item and its first window (in flight while the table is built)
  const CountItem it = grp[wave];
  const Window w0 = window_first(A, it.t0, it.q0, it.len);
  if (lane < kBmWords) bm[lane] = 0;
  block_init<MODE>();
  uint32_t hits = 0;
  TableRef tr{nullptr, nullptr, 0, 0, rs, d, nullptr, nullptr, 0};
  if (GLOBAL) {
    __syncthreads();  // shift counters cleared before any credit
  } else {
    const uint32_t S = 1u << grp[0].log2S;
    int32_t* tab = smem + kItemMarkInts;
    int32_t* val = tab + S;
    for (uint32_t i = tid; i < S; i += blockDim.x) tab[i] = kEmpty;
    if (tid == 0) s_D = 0;
    __syncthreads();
    const uint32_t bmask = S / kBucket - 1;
    int md = build_table<VALS, VAR == VAR_MUL>(tab, val, bmask, A.hcol, rs, d, tid, (int)blockDim.x);
    if (md) atomicMax(&s_D, md);  // per lane: see pack_body
    __syncthreads();
    tr.tab = tab;
    tr.val = val;
    tr.bmask = bmask;
    tr.D = s_D;
  }
  wave_sync_lds();
  if (it.len) wave_probe<MODE, GLOBAL ? TK_GLOBAL : TK_SINGLE, VAR>(A, tr, it.t0, it.q0, it.len, bm, hits, w0);
  if constexpr (VALS && !GLOBAL) {
    // the (b, k) credits of the work-group: one atomic per slot that was hit
    __syncthreads();
    const uint32_t S = 1u << grp[0].log2S;
    for (uint32_t i = threadIdx.x; i < S; i += blockDim.x) {
      if (tr.tab[i] == kEmpty) continue;
      const uint32_t w = (uint32_t)tr.val[i];
      const uint32_t c = w >> kValBits;
      const int64_t p = rs + (int64_t)(w & ((1u << kValBits) - 1u));
      if (c && p < (int64_t)A.m) atomicAdd(&A.support[p], (int)c);
    }
  }
  return block_flush<MODE>(hits, A);
}

// OCC: waves per SIMD the kernel's registers are budgeted for. A class whose
// tables limit a CU to fewer work-groups gets the registers that would
// otherwise go unused (fewer spills in the probe loop).
template <int MODE, bool GLOBAL, int OCC, int WAVES, int VAR>
__global__ __launch_bounds__(64 * WAVES) __attribute__((amdgpu_waves_per_eu(OCC)))
void k_count_items(Args A, const CountItem* __restrict__ items) {
  extern __shared__ int4 smem4[];  // 16-byte aligned: tables are read as int4 buckets
  items_body<MODE, GLOBAL, VAR>(A, items + (int64_t)blockIdx.x * WAVES, reinterpret_cast<int32_t*>(smem4));
}

// Count mode per class (chosen by timing at RMAT scale 24): wg_small and
// wg_large tables (<= 4 / 16 KiB) would allow 8 or more work-groups per CU,
// but 7 waves per SIMD with spill-free registers run faster; wg_huge tables
// (32 KiB) allow 4-5 work-groups per CU and wg_giant tables (64 KiB) 2.
// Support modes hold more state per probe and run at 4.
constexpr int kOccSmall = 7, kOccLarge = 7, kOccHuge = 5, kOccGiant = 4, kOccSupport = 5;

template <int MODE, bool GLOBAL, int VAR>
const void* items_kernel(int cls) {
  static_assert(class_waves(CLS_WG_HUGE) == kWavesBig && class_waves(CLS_WG_GIANT) == kWavesBig &&
                    class_waves(CLS_WG_LARGE) == kWaves && class_waves(CLS_GLOBAL) == kWaves,
                "work-group shapes of the item classes");
  // oriented support adds only the per-task counters to the count: same budgets;
  // wide probe addresses take more registers: the support budget
  constexpr bool kCountLike = (MODE == MODE_COUNT || MODE == MODE_SUPPORT_ORIENTED) && VAR != VAR_WIDE;
  if constexpr (GLOBAL) {  // no table: LDS does not limit
    return (const void*)k_count_items<MODE, GLOBAL, kCountLike ? kOccSmall : kOccSupport, kWaves, VAR>;
  } else if constexpr (!kCountLike) {
    if (class_waves(cls) == kWavesBig) return (const void*)k_count_items<MODE, GLOBAL, kOccSupport, kWavesBig, VAR>;
    return (const void*)k_count_items<MODE, GLOBAL, kOccSupport, kWaves, VAR>;
  } else {
    switch (cls) {
      case CLS_WG_LARGE: return (const void*)k_count_items<MODE, GLOBAL, kOccLarge, kWaves, VAR>;
      case CLS_WG_HUGE: return (const void*)k_count_items<MODE, GLOBAL, kOccHuge, kWavesBig, VAR>;
      case CLS_WG_GIANT: return (const void*)k_count_items<MODE, GLOBAL, kOccGiant, kWavesBig, VAR>;
      default: return (const void*)k_count_items<MODE, GLOBAL, kOccSmall, kWaves, VAR>;
    }
  }
}

__global__ void k_zero_i64(int64_t* p) { *p = 0; }

__global__ void k_zero_i32(int32_t* p, int64_t n) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = 0;
}

// launch names seen by the phase timer: "<mode>:<class>"
const char* const kLaunchNames[4][NUM_CLASSES] = {
    {"count:pack_small", "count:pack_large", "count:wg_small", "count:wg_large", "count:wg_huge",
     "count:wg_giant", "count:global"},
    {"support_full:pack_small", "support_full:pack_large", "support_full:wg_small",
     "support_full:wg_large", "support_full:wg_huge", "support_full:wg_giant", "support_full:global"},
    {"support_oriented:pack_small", "support_oriented:pack_large", "support_oriented:wg_small",
     "support_oriented:wg_large", "support_oriented:wg_huge", "support_oriented:wg_giant",
     "support_oriented:global"},
    {"block:pack_small", "block:pack_large", "block:wg_small", "block:wg_large", "block:wg_huge",
     "block:wg_giant", "block:global"}};

// Work-groups per launch of one class: a dispatch holds fewer than 2^32
// work-items (a class of more groups, e.g. small wave items on a very large
// graph, is launched in pieces; each group finds its data by its index).
constexpr int64_t kClassLaunchMax = (int64_t)1 << 22;

template <int MODE, int VAR>
void launch_items_class(const WorkSet& w, const Args& A, int c, size_t mark_bytes, hipStream_t st) {
  if (w.n_items[c] == 0) return;
  const int64_t groups = w.n_items[c] / class_waves(c);
  const bool global = c == CLS_GLOBAL;
  const void* f = global ? items_kernel<MODE, true, VAR>(c) : items_kernel<MODE, false, VAR>(c);
  const size_t lds = global ? mark_bytes : items_lds_bytes(w.cls_log2S[c], MODE);
  if (lds > 65536) TC_HIP(hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
  LaunchScope ls(kLaunchNames[MODE][c], st);
  for (int64_t g0 = 0; g0 < groups; g0 += kClassLaunchMax) {
    const unsigned grid = (unsigned)std::min<int64_t>(kClassLaunchMax, groups - g0);
    const CountItem* items = w.items[c] + g0 * class_waves(c);
    void* kargs[] = {const_cast<Args*>(&A), &items};
    TC_HIP(hipLaunchKernel(f, dim3(grid), dim3(64 * class_waves(c)), kargs, lds, st));
  }
}

// The light classes (packs, wg_small: small tables, few probes per row) run
// on a side stream beside the heavy ones, so that their launches - short,
// and ending on a few long work-groups that nothing else overlaps - fill the
// GPU while the heavy classes stream. One side stream per (device, caller
// stream), with a fork and a join event; never destroyed; default priority.
// At most kSideStreams of them exist: calls on further caller streams run
// every class on the caller's stream.
struct SideStream {
  hipStream_t aux = nullptr;
  hipEvent_t fork = nullptr, join = nullptr;
};

constexpr size_t kSideStreams = 64;

SideStream* side_stream(hipStream_t st) {
  static std::mutex mu;
  static std::map<std::pair<int, hipStream_t>, SideStream> streams;
  int dev = 0;
  TC_HIP(hipGetDevice(&dev));
  std::lock_guard<std::mutex> lk(mu);
  auto it = streams.find({dev, st});
  if (it == streams.end()) {
    if (streams.size() >= kSideStreams) return nullptr;
    SideStream s;
    TC_HIP(hipStreamCreateWithFlags(&s.aux, hipStreamNonBlocking));
    TC_HIP(hipEventCreateWithFlags(&s.fork, hipEventDisableTiming));
    TC_HIP(hipEventCreateWithFlags(&s.join, hipEventDisableTiming));
    it = streams.emplace(std::make_pair(dev, st), s).first;
  }
  return &it->second;
}

// Probes below which a graph's classes all run on the caller's stream (the
// fork and join would cost more than they save).
constexpr int64_t kSideMinProbes = (int64_t)1 << 24;

template <int MODE, int VAR>
void launch_mode(const WorkSet& w, const Args& A, hipStream_t st) {
  constexpr bool VALS = MODE == MODE_SUPPORT_FULL;
  const size_t mark_bytes = items_lds_bytes(-1, MODE);
  // the light classes go to the side stream when both sides have work
  bool light = false, heavy = false;
  for (int c = 0; c < NUM_CLASSES; ++c) {
    const bool any = c <= CLS_PACK_LARGE ? w.n_packs[c] > 0 : w.n_items[c] > 0;
    (c <= CLS_WG_SMALL ? light : heavy) |= any;
  }
  // (one rank's block keeps its classes on the caller's stream: its launches
  // are small, and its per-class times stay separable)
  SideStream* side =
      MODE != MODE_BLOCK && light && heavy && w.probes >= kSideMinProbes ? side_stream(st) : nullptr;
  if (side) {
    TC_HIP(hipEventRecord(side->fork, st));
    TC_HIP(hipStreamWaitEvent(side->aux, side->fork, 0));
  }
  // heavy classes first (on st), then the light ones (on the side stream)
  for (int c = CLS_WG_LARGE; c <= CLS_GLOBAL; ++c) launch_items_class<MODE, VAR>(w, A, c, mark_bytes, st);
  const hipStream_t ls = side ? side->aux : st;
  for (int c = CLS_PACK_SMALL; c <= CLS_PACK_LARGE; ++c) {
    if (w.n_packs[c] == 0) continue;
    // a pack's tables take at most wp.pack_slots plus one row's table
    const uint32_t slots = w.wp.pack_slots + (1u << w.pack_log2S[c]);
    const size_t lds = pack_lds_bytes(slots, MODE);
    if (lds > 65536)
      TC_HIP(hipFuncSetAttribute((const void*)k_count_packs<MODE, VAR>,
                                 hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
    for (int64_t p0 = 0; p0 < w.n_packs[c]; p0 += kClassLaunchMax)  // (pieces: see kClassLaunchMax)
      TC_LAUNCH(kLaunchNames[MODE][c], (k_count_packs<MODE, VAR>),
                dim3((unsigned)std::min<int64_t>(kClassLaunchMax, w.n_packs[c] - p0)), dim3(256), lds, ls, A,
                w.pack_recs[c], w.pack_info[c] + p0, slots);
  }
  launch_items_class<MODE, VAR>(w, A, CLS_WG_SMALL, mark_bytes, ls);
  if (side) {
    TC_HIP(hipEventRecord(side->join, side->aux));
    TC_HIP(hipStreamWaitEvent(st, side->join, 0));
  }
  TC_HIP(hipGetLastError());
}

__global__ void k_zero_u64(unsigned long long* p, int64_t n) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = 0;
}

// Batched count: clears the per-graph counters and the unit queue (a kernel,
// not a memset, so that the pair can be captured in a HIP graph).
__global__ void k_batch_clear(unsigned long long* counts, int64_t n, unsigned int* queue) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) counts[i] = 0;
  if (i == 0) *queue = 0;
}

// Persistent work-groups pull units from one queue until it is empty (every
// work-group reaches the exit once the counter passes the last chunk); the
// units were ordered when the plan was made (largest first by default). One
// atomic takes `chunk` consecutive units (a tuning choice: fewer atomics on
// the one counter against coarser balance). Each unit runs the same body as
// its class's own kernel with its graph's arguments.
template <int MODE>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(MODE == MODE_COUNT ? kOccBatch : 4)))
void k_count_batch(const Args* __restrict__ gargs, const BatchUnit* __restrict__ units, uint32_t n_units,
                   uint32_t chunk, unsigned int* __restrict__ queue, unsigned long long* __restrict__ counts) {
  extern __shared__ int4 smem4[];
  int32_t* smem = reinterpret_cast<int32_t*>(smem4);
  __shared__ uint32_t s_chunk;
  const uint32_t n_chunks = (n_units + chunk - 1) / chunk;
  for (;;) {
    __syncthreads();  // the previous chunk is done with s_chunk
    if (threadIdx.x == 0) s_chunk = atomicAdd(queue, 1u);
    __syncthreads();
    const uint32_t ci = __builtin_amdgcn_readfirstlane(s_chunk);  // uniform: unit loads go scalar
    if (ci >= n_chunks) break;
    const uint32_t u_end = ci * chunk + chunk < n_units ? ci * chunk + chunk : n_units;
    for (uint32_t u = ci * chunk; u < u_end; ++u) {
      __syncthreads();  // the previous unit is done with LDS
      const BatchUnit bu = units[u];
      Args A = gargs[bu.graph];
      A.count = counts + bu.graph;
      if (bu.kind == BK_PACK) {
        pack_body<MODE, VAR_BASE>(A, static_cast<const PackRow*>(bu.p0), static_cast<const PackInfo*>(bu.p1),
                                  bu.index, bu.slots, smem);
      } else if (bu.kind == BK_ITEMS) {
        items_body<MODE, false, VAR_BASE>(A, static_cast<const CountItem*>(bu.p0), smem);
      } else {
        items_body<MODE, true, VAR_BASE>(A, static_cast<const CountItem*>(bu.p0), smem);
      }
    }
  }
}

template <int MODE>
void launch_batch_mode(const Args* d_args, const BatchUnit* d_units, int64_t n_units, uint32_t chunk,
                       unsigned int* d_queue, unsigned long long* counts, unsigned grid, size_t lds,
                       hipStream_t st, bool timed) {
  static const char* const kNames[3] = {"count:batch", "support_full:batch", "support_oriented:batch"};
  if (n_units == 0) return;
  if (timed)
    TC_LAUNCH(kNames[MODE], k_count_batch<MODE>, dim3(grid), dim3(256), lds, st, d_args, d_units,
              (uint32_t)n_units, chunk, d_queue, counts);
  else
    hipLaunchKernelGGL(k_count_batch<MODE>, dim3(grid), dim3(256), lds, st, d_args, d_units,
                       (uint32_t)n_units, chunk, d_queue, counts);
}

}  // namespace

size_t pack_lds_bytes(uint32_t slots, int mode) {
  const size_t vals = mode == MODE_SUPPORT_FULL ? 2 : 1;
  return sizeof(int32_t) * ((size_t)kMarkInts + kPackMetaWords + 3 + (size_t)slots * vals);
}

size_t items_lds_bytes(int log2S, int mode) {
  const size_t vals = mode == MODE_SUPPORT_FULL ? 2 : 1;
  return sizeof(int32_t) * ((size_t)kItemMarkInts + (log2S < 0 ? 0 : ((size_t)1 << log2S) * vals));
}

void launch_batch(CountMode mode, const CountArgs* d_args, const BatchUnit* d_units, int64_t n_units,
                  uint32_t chunk, int64_t n_out, unsigned int* d_queue, int64_t* d_counts, unsigned grid,
                  size_t lds, hipStream_t st, bool timed) {
  TC_REQUIRE(chunk >= 1, TC_EINVAL, "launch_batch: chunk must be >= 1");
  TC_REQUIRE(mode == MODE_COUNT || mode == MODE_SUPPORT_FULL || mode == MODE_SUPPORT_ORIENTED, TC_EINVAL,
             "launch_batch: unsupported mode");
  auto* counts = reinterpret_cast<unsigned long long*>(d_counts);
  const unsigned cg = (unsigned)std::max<int64_t>(1, div_up(n_out, 256));
  if (timed) TC_LAUNCH("batch_clear", k_batch_clear, dim3(cg), dim3(256), 0, st, counts, n_out, d_queue);
  else hipLaunchKernelGGL(k_batch_clear, dim3(cg), dim3(256), 0, st, counts, n_out, d_queue);
  switch (mode) {
    case MODE_COUNT:
      launch_batch_mode<MODE_COUNT>(d_args, d_units, n_units, chunk, d_queue, counts, grid, lds, st, timed);
      break;
    case MODE_SUPPORT_FULL:
      launch_batch_mode<MODE_SUPPORT_FULL>(d_args, d_units, n_units, chunk, d_queue, counts, grid, lds, st, timed);
      break;
    default:
      launch_batch_mode<MODE_SUPPORT_ORIENTED>(d_args, d_units, n_units, chunk, d_queue, counts, grid, lds, st,
                                               timed);
      break;
  }
  TC_HIP(hipGetLastError());
}

void launch_count(const CountView& v, CountMode mode, int64_t* d_count, int32_t* d_support,
                  int64_t* d_per_shift, hipStream_t st) {
  const WorkSet& w = *v.w;
  if (d_count) TC_LAUNCH("zero_i64", k_zero_i64, dim3(1), dim3(1), 0, st, d_count);
  if ((mode == MODE_SUPPORT_FULL || mode == MODE_SUPPORT_ORIENTED) && v.pm > 0)
    TC_LAUNCH("zero_i32", k_zero_i32, dim3((unsigned)div_up(v.pm, 256)), dim3(256), 0, st, d_support,
              v.pm);
  if (mode == MODE_BLOCK && d_per_shift)
    TC_LAUNCH("zero_u64", k_zero_u64, dim3(1), dim3(64), 0, st,
              reinterpret_cast<unsigned long long*>(d_per_shift), (int64_t)v.q);
  TC_HIP(hipGetLastError());
  if (w.n_tasks == 0) return;
  TC_REQUIRE(v.pm < kMaxEdges, TC_EOVERFLOW, "launch_count: probe side of 2^32 - 256 entries or more");
  const bool wide = v.pm > kMaxBufferEdges;
  TC_REQUIRE(!wide || mode != MODE_BLOCK, TC_EOVERFLOW, "launch_count: a rank's probe side of 2^30 entries or more");
  Args A{v.hrow_ptr, v.hcol, v.pcol, w.tstart, w.tprefix, w.tbeg, w.tend, w.n_tasks, (uint32_t)v.pm,
         reinterpret_cast<unsigned long long*>(d_count), d_support,
         reinterpret_cast<unsigned long long*>(d_per_shift), v.q, v.xy};
  TC_REQUIRE(v.hash == 0 || mode == MODE_COUNT, TC_EINVAL, "launch_count: multiplicative hashing counts only");
  TC_REQUIRE(!(wide && v.hash), TC_EOVERFLOW, "launch_count: multiplicative hashing below 2^30 edges only");
  switch (mode) {
    case MODE_COUNT:
      if (v.hash) launch_mode<MODE_COUNT, VAR_MUL>(w, A, st);
      else if (wide) launch_mode<MODE_COUNT, VAR_WIDE>(w, A, st);
      else launch_mode<MODE_COUNT, VAR_BASE>(w, A, st);
      break;
    case MODE_SUPPORT_FULL:
      if (wide) launch_mode<MODE_SUPPORT_FULL, VAR_WIDE>(w, A, st);
      else launch_mode<MODE_SUPPORT_FULL, VAR_BASE>(w, A, st);
      break;
    case MODE_SUPPORT_ORIENTED:
      if (wide) launch_mode<MODE_SUPPORT_ORIENTED, VAR_WIDE>(w, A, st);
      else launch_mode<MODE_SUPPORT_ORIENTED, VAR_BASE>(w, A, st);
      break;
    case MODE_BLOCK: launch_mode<MODE_BLOCK, VAR_BASE>(w, A, st); break;
  }
}

void batch_kernel_lds(CountMode mode, size_t lds) {
  if (lds <= 65536) return;
  const void* f = mode == MODE_COUNT          ? (const void*)k_count_batch<MODE_COUNT>
                  : mode == MODE_SUPPORT_FULL ? (const void*)k_count_batch<MODE_SUPPORT_FULL>
                                              : (const void*)k_count_batch<MODE_SUPPORT_ORIENTED>;
  TC_HIP(hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
}

void zero_i32(int32_t* p, int64_t n, hipStream_t st, bool timed) {
  if (n <= 0) return;
  if (timed) TC_LAUNCH("zero_i32", k_zero_i32, dim3((unsigned)div_up(n, 256)), dim3(256), 0, st, p, n);
  else hipLaunchKernelGGL(k_zero_i32, dim3((unsigned)div_up(n, 256)), dim3(256), 0, st, p, n);
}

}  // namespace tc
