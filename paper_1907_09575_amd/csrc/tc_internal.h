// tc_internal.h - shared host/device declarations of libtc (not installed).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <cstdio>
#include <map>
#include <mutex>
#include <stdexcept>
#include <string>
#include <vector>

#include "../../include/tc.h"

namespace tc {

// ---- errors ------------------------------------------------------------------
// Internal code throws tc::Error; every extern "C" entry point catches it and
// converts it to a tc_status (no exception crosses the ABI).
struct Error : std::runtime_error {
  tc_status status;
  Error(tc_status s, const std::string& msg) : std::runtime_error(msg), status(s) {}
};

void set_last_error(const std::string& msg);

#define TC_HIP(expr)                                                                       \
  do {                                                                                     \
    hipError_t _e = (expr);                                                                \
    if (_e != hipSuccess) {                                                                \
      throw ::tc::Error(_e == hipErrorOutOfMemory ? TC_ENOMEM : TC_EDEVICE,                \
                        std::string(#expr) + ": " + hipGetErrorString(_e) + " (" __FILE__ \
                        ":" + std::to_string(__LINE__) + ")");                             \
    }                                                                                      \
  } while (0)

#define TC_REQUIRE(cond, status, msg)                       \
  do {                                                      \
    if (!(cond)) throw ::tc::Error((status), (msg));        \
  } while (0)

// ---- launches -----------------------------------------------------------------
// Every kernel launch goes through TC_LAUNCH so that an attached phase timer
// (tc_timer_attach) can bracket it with events.
struct LaunchScope {
  int slot = -1;
  void* timer = nullptr;
  hipStream_t st = nullptr;
  LaunchScope(const char* name, hipStream_t s);
  ~LaunchScope();
};

#define TC_LAUNCH(name, kern, grid, block, lds, st, ...)          \
  do {                                                           \
    ::tc::LaunchScope _tc_ls((name), (st));                      \
    hipLaunchKernelGGL(kern, grid, block, lds, st, __VA_ARGS__); \
  } while (0)

// ---- work items --------------------------------------------------------------
// One wave's share of the probes of one hashed row b: the probes with global
// index [q0, q0 + len) of the task list, where task t0 contains probe q0.
// Items of one launch class are grouped per work-group (WAVES items, same b).
struct alignas(8) CountItem {
  int32_t b;       // hashed row (rank)
  uint32_t t0;     // task containing q0
  uint64_t q0;     // first global probe index
  uint32_t len;    // number of probes
  uint32_t log2S;  // hash table size (slots) = 1 << log2S
};
static_assert(sizeof(CountItem) == 24, "CountItem layout");

// Launch classes of the count kernels (see tc_count.hip).
enum ItemClass : int {
  CLS_PACK_SMALL = 0,  // packs of light rows b (one work-group each), table <= 256 slots
  CLS_PACK_LARGE = 1,  // packs of light rows b, table <= 1024 slots
  CLS_WG_SMALL = 2,    // heavy rows, 4 waves share one table <= 1024 slots
  CLS_WG_LARGE = 3,    // heavy rows, table <= 4096 slots
  CLS_WG_HUGE = 4,     // table <= 8192 slots
  CLS_WG_GIANT = 5,    // table of 16384 slots (rows of 4097 .. 8192 keys)
  CLS_GLOBAL = 6,      // table would not fit LDS: binary search in U_b in HBM
  NUM_CLASSES = 7
};

constexpr int kWaves = 4;               // waves per work-group of packs, small item classes, batch units
constexpr int kWavesBig = 8;            // waves per work-group of wg_huge / wg_giant items
constexpr int kMaxLog2S = 14;           // largest LDS table: 16384 slots (64 KiB keys + 64 KiB values)
// Default row-bucket thresholds of a work decomposition (WorkParams below).
constexpr uint32_t kWaveChunk = 32767;  // target probes per wave item of a heavy row
constexpr uint64_t kHeavyMin = 32768;   // rows with fewer probes than this are packed
constexpr uint64_t kPackTarget = 65536; // target probes per pack of light rows (one work-group)
constexpr uint32_t kPackSlots = 4096;   // target table slots per pack (LDS: + one row's table)
constexpr uint32_t kMinGroups = 16384;  // work-groups an item class gets at least (chunks shrink)
// Their limits: a wave item's probes, times the waves sharing a table, must
// stay below the hit field of a table's value word (2^18); a pack's table
// offset is 16 bits of buckets.
constexpr uint32_t kWaveChunkMin = 1024, kWaveChunkMax = 32767;
constexpr uint64_t kHeavyMinMax = (uint64_t)1 << 24;
constexpr uint64_t kPackTargetMin = 1024, kPackTargetMax = (uint64_t)1 << 24;
constexpr uint32_t kPackSlotsMin = 1024, kPackSlotsMax = 16384;
constexpr uint32_t kMinGroupsMax = 1u << 22;
constexpr int kPackRows = 256;          // rows per pack at most (one per thread)
constexpr int kBucket = 4;              // slots per hash bucket (one 16-byte LDS read)
// U positions are 32-bit, and an elementwise launch over U's entries (rounded
// up to 256 threads) must stay below 2^32 work-items: fewer than kMaxEdges.
constexpr int64_t kMaxEdges = (1ll << 32) - 256;
constexpr int64_t kMaxBufferEdges = (1ll << 30) - 64;  // below: probe reads by 32-bit byte offsets

// Waves sharing one table in a work-group of item class c: the classes whose
// tables allow only a few work-groups per CU get twice the waves per table.
__host__ __device__ constexpr int class_waves(int c) {
  return (c == CLS_WG_HUGE || c == CLS_WG_GIANT) ? kWavesBig : kWaves;
}

// Slots of the LDS hash table of a row with d keys: a power of two >= 4 d
// (load factor <= 1/4, so almost every lookup ends in its first bucket) for
// rows of up to 2048 keys (tables of up to 8192 slots, 32 KiB), >= 2 d above
// (load <= 1/2: an absent key needs a second bucket read about once in seven,
// but such rows take half the LDS, so twice as many work-groups fit a CU and
// rows of up to 8192 keys stay in LDS); at least 64.
__host__ __device__ inline int table_log2(int64_t d) {
  const int64_t want = d <= 2048 ? 4 * d : 2 * d;
  int l = 6;
  while ((1ll << l) < want) ++l;
  return l;
}

// Packs of light rows give each row its own table, >= 4 d slots, at least 16.
__host__ __device__ inline int pack_table_log2(int64_t d) {
  int l = 4;
  while ((1ll << l) < 4 * d) ++l;
  return l;
}

// ---- device memory (tc_alloc.cpp) ------------------------------------------
// Caching allocator: blocks are kept per device after they are freed and
// reused (on another stream only after an event recorded at the free).
// cache_free: `st` is the stream of the block's last use; idle = no work on
// the block can be pending (no event needed).
void* cache_alloc(size_t bytes, hipStream_t st);
void cache_free(void* p, hipStream_t st, bool idle);
void cache_release_all();
// Call before destroying a stream that blocks were freed on: synchronises it
// and makes its cached blocks idle, so that no cached event refers to it.
void cache_retire_stream(hipStream_t st);

// Allocations owned by a graph or a temporary work set (freed together).
// `st` is the stream they are used on; release(idle) returns them to the
// cache (idle: the caller knows no work on them is pending).
struct Owned {
  std::vector<void*> ptrs;
  size_t bytes = 0;
  hipStream_t st = nullptr;
  template <class T>
  T* alloc(int64_t count) {
    const size_t b = sizeof(T) * (size_t)(count > 0 ? count : 1);
    void* p = cache_alloc(b, st);
    ptrs.push_back(p);
    bytes += b;
    return static_cast<T*>(p);
  }
  void release(bool idle = false) {
    for (void* p : ptrs) cache_free(p, st, idle);
    ptrs.clear();
    bytes = 0;
  }
  ~Owned() { release(); }
};

// Tasks of a set of hashed rows and the work units of the count kernels.
// Hashed rows are 0 .. nrows - 1 (ranks for a graph, rank-local rows for one
// rank's block); a task's probes are entries of the probe-side CSR.
// A row of a pack class, in pack order: all a pack work-group needs of it in
// one 16-byte load.
struct alignas(16) PackRow {
  uint32_t rs;      // start of U_b in col
  uint32_t d;       // |U_b|, 0 for a row without tasks (it needs no table)
  uint32_t tb, te;  // its tasks [tb, te) (class-major order)
};
// A pack: its rows [r0, r1) of the class, its probes [q0, q1) and, for each
// of its kWaves equal shares of them, the task holding the share's first
// probe (computed once when the work is built, instead of searched for by
// every launch).
struct alignas(16) PackInfo {
  uint64_t q0, q1;
  uint32_t r0, r1;
  uint32_t wt[kWaves];
};
static_assert(sizeof(PackRow) == 16 && sizeof(PackInfo) == 48, "pack record layout");

// Row-bucket thresholds: which rows are packed and how the work is cut.
struct WorkParams {
  uint64_t heavy_min = kHeavyMin;     // rows with fewer probes (and tables <= 2^10) go to packs
  uint64_t pack_target = kPackTarget; // probes per pack (plus one row's)
  uint32_t pack_slots = kPackSlots;   // table slots per pack (plus one row's table)
  uint32_t wave_chunk = kWaveChunk;   // probes per wave item of a heavy row (at most)
  uint32_t min_groups = kMinGroups;   // an item class with fewer work-groups gets smaller chunks
  bool operator==(const WorkParams& o) const {
    return heavy_min == o.heavy_min && pack_target == o.pack_target && pack_slots == o.pack_slots &&
           wave_chunk == o.wave_chunk && min_groups == o.min_groups;
  }
  bool operator!=(const WorkParams& o) const { return !(*this == o); }
};

struct WorkSet {
  int64_t nrows = 0, n_tasks = 0, probes = 0;
  WorkParams wp;  // the thresholds this decomposition was built with
  uint32_t* tbeg = nullptr;     // nrows, tasks of hashed row b: [tbeg[b], tend[b]) (class-major order)
  uint32_t* tend = nullptr;     // nrows
  uint32_t* tstart = nullptr;   // n_tasks, probe-side index of the task's first probe
  uint64_t* tprefix = nullptr;  // n_tasks + 1, exclusive prefix of task lengths

  // pack classes: pack p covers pack_rows[c][pack_ptr[c][p] .. pack_ptr[c][p+1])
  int32_t* pack_rows[2] = {nullptr, nullptr};   // light rows b of the class, ascending
  uint32_t* pack_ptr[2] = {nullptr, nullptr};
  PackRow* pack_recs[2] = {nullptr, nullptr};   // the rows' records, same order
  PackInfo* pack_info[2] = {nullptr, nullptr};  // one per pack, heaviest first (launch order)
  int64_t n_pack_rows[2] = {0, 0};
  int64_t n_packs[2] = {0, 0};
  int32_t pack_log2S[2] = {0, 0};               // largest row table of the class (log2 slots)

  // work-group classes: n_items[c] items (a multiple of kWaves)
  CountItem* items[NUM_CLASSES] = {};
  int64_t n_items[NUM_CLASSES] = {};
  int32_t cls_log2S[NUM_CLASSES] = {};
  uint32_t cls_chunk[NUM_CLASSES] = {};  // probes per wave item of each item class

  // per class: rows, table keys, tasks, probes (host copy)
  int64_t cls_stats[NUM_CLASSES][4] = {};
};

// Streams that have used an object's device memory, each with an event
// recorded after its latest use there: freeing the memory waits for those
// events (on a library stream), not for the whole device, and does not need
// the streams to be alive. A use inside a stream capture cannot be recorded
// that way; it makes the free synchronise the device.
struct UseLog {
  std::mutex mu;
  std::vector<std::pair<hipStream_t, hipEvent_t>> uses;
  bool captured = false;
  ~UseLog();
  void note(hipStream_t st);
  // Blocks the host until every recorded use is done.
  void wait_host();
  // Returns `owned` memory to the cache, reusable once every recorded use is
  // done (the host does not wait).
  void release_after_uses(Owned& owned);
};

// Device-resident graph: U in CSR (rank space) and its work set.
// A variant (tc_graph_variant) shares U with the graph it was made from and
// has a work set of its own: variant holds its TC_VARIANT_* flags and hash
// the table addressing (0: the direct AND, 1: multiplicative hashing).
struct Graph {
  int device = 0;
  int64_t n = 0, m_raw = 0, m = 0;
  int64_t wedges_plus = 0, max_dplus = 0;
  int sbits = 1;  // ceil(log2(n)), >= 1
  size_t arena_bytes = 0;
  int variant = 0;
  int hash = 0;
  mutable UseLog uses;         // streams that ran work on the graph (tc_graph_free)
  const Graph* base = nullptr;  // a variant: the graph whose U it reads

  int64_t* row_ptr = nullptr;  // n + 1, U rows
  int32_t* col = nullptr;      // m, rows sorted ascending
  int32_t* perm = nullptr;     // n, perm[original id] = rank
  WorkSet w;
};

extern const char* const kClassNames[NUM_CLASSES];

// Build a graph from a device edge list on `st` (tc_preprocess without the
// argument checks; synchronises st) and free one.
Graph* build_graph(const int32_t* d_src, const int32_t* d_dst, int64_t m_raw, int64_t n, hipStream_t st);
// destroy_graph returns the graph's memory once the work of every stream that
// used it (its UseLog) is done; destroy_graph_idle is for callers that know
// no such work is pending.
void destroy_graph(Graph* g);
void destroy_graph_idle(Graph* g);
// A variant of `base` (TC_VARIANT_* flags) sharing its U (tc_graph_variant);
// with flags 0 a plain graph whose work is cut by other thresholds
// (tc_graph_retune).
Graph* build_variant(const Graph& base, int flags, const WorkParams& wp, hipStream_t st);

inline const Graph* G(const tc_graph* g) { return reinterpret_cast<const Graph*>(g); }

// Record that work reading g (and a variant's base) was enqueued on st; call
// after enqueuing it.
inline void note_use(const Graph& g, hipStream_t st) {
  g.uses.note(st);
  if (g.base) g.base->uses.note(st);
}

// ---- launchers implemented in tc_count.hip ---------------------------------
enum CountMode : int {
  MODE_COUNT = 0,
  MODE_SUPPORT_FULL = 1,
  MODE_SUPPORT_ORIENTED = 2,
  MODE_BLOCK = 3  // count plus per-shift split of one rank's block (Eq. 5)
};

// What the count kernels read: the hash side (rows b, their sorted entries),
// the probe side (entries probed by tasks) and the work set.
struct CountView {
  const int64_t* hrow_ptr;
  const int32_t* hcol;
  const int32_t* pcol;
  int64_t pm;  // entries of pcol
  const WorkSet* w;
  int32_t q = 1, xy = 0;  // MODE_BLOCK: grid size and (x + y) % q
  int hash = 0;           // 1: multiplicative hashing (MODE_COUNT only)
};

void launch_count(const CountView& v, CountMode mode, int64_t* d_count, int32_t* d_support,
                  int64_t* d_per_shift, hipStream_t stream);

// Kernel arguments of the count kernels (one hashed side, one probe side and
// the task arrays of a work set).
struct CountArgs {
  const int64_t* __restrict__ row_ptr;  // hash side: rows b
  const int32_t* __restrict__ hcol;     // hash side: sorted entries of each row b
  const int32_t* __restrict__ col;      // probe side (the tasks' probes; U itself for a graph)
  const uint32_t* __restrict__ tstart;
  const uint64_t* __restrict__ tprefix;
  const uint32_t* __restrict__ tbeg;
  const uint32_t* __restrict__ tend;
  int64_t T;
  uint32_t m;  // entries of col
  unsigned long long* count;
  int32_t* support;
  unsigned long long* per_shift;  // MODE_BLOCK: q counters
  int32_t q, xy;                  // MODE_BLOCK: grid size, (x + y) % q
};

// ---- batched persistent count (tc_count.hip kernel, tc_batch.cpp plan) -------
// One unit of the persistent launch: a pack of light rows, a work-group of
// kWaves items sharing an LDS table, or such a group whose row is looked up
// in HBM.
enum BatchKind : int32_t { BK_PACK = 0, BK_ITEMS = 1, BK_ITEMS_HBM = 2 };

struct alignas(16) BatchUnit {
  const void* p0;      // pack: PackRow records of the class; items: the group's first item
  const void* p1;      // pack: PackInfo records of the class
  uint32_t index;      // pack: pack number
  uint32_t slots;      // pack: table slots reserved for the pack
  int32_t graph;       // entry of the plan's graph list (and of the output)
  int32_t kind;        // BatchKind
};
static_assert(sizeof(BatchUnit) == 32, "BatchUnit layout");

// Launch the persistent count in `mode` (count or a support mode) over n_units
// units (queue: device counter, counts: int64 per graph entry; both cleared
// by the same call's first kernel; support arrays are the entries' CountArgs
// and must be cleared by the caller). timed: through TC_LAUNCH (not inside a
// capture).
void launch_batch(CountMode mode, const CountArgs* d_args, const BatchUnit* d_units, int64_t n_units,
                  uint32_t chunk, int64_t n_out, unsigned int* d_queue, int64_t* d_counts, unsigned grid,
                  size_t lds, hipStream_t st, bool timed);
// Allow the persistent kernel of `mode` `lds` bytes of dynamic LDS (call
// outside any capture).
void batch_kernel_lds(CountMode mode, size_t lds);
// Batch plans (tc_batch.hip): one persistent launch over many graphs in one
// mode; support modes write each entry's own support array (cleared by every
// launch of the plan). tuning_json as tc_batch_create's. Synchronises st.
struct BatchPlan;
struct PlanEntry {
  const Graph* g;
  int32_t* support;  // device int32[g->m] for support modes, else null
};
BatchPlan* make_plan(const PlanEntry* entries, int64_t num, CountMode mode, const char* tuning_json,
                     hipStream_t st);
// Launch the plan on st (its own HIP graph, or recorded into the caller's
// capture); per-entry counts go to d_counts[num].
void plan_count(BatchPlan& P, int64_t* d_counts, hipStream_t st);
int64_t plan_units(const BatchPlan& P);
// free_plan waits for the device to drain; free_plan_idle is for callers that
// know no launch of the plan is pending.
void free_plan(BatchPlan* P);
void free_plan_idle(BatchPlan* P);

// Clear an int32 device array by a kernel (timed: through TC_LAUNCH).
void zero_i32(int32_t* p, int64_t n, hipStream_t st, bool timed);

// Dynamic LDS bytes of a pack work-group with `slots` table slots, and of an
// item work-group with a 2^log2S-slot table (log2S < 0: no table, HBM
// lookups), in CountMode `mode` (full support tables also hold U positions).
size_t pack_lds_bytes(uint32_t slots, int mode);
size_t items_lds_bytes(int log2S, int mode);

inline CountView graph_view(const Graph& g) {
  return CountView{g.row_ptr, g.col, g.col, g.m, &g.w, 1, 0, g.hash};
}

// Entry points that rely on the <j,i,k> task layout of a graph's own work
// set (support, blocks, batches, the uses of support) refuse variants.
inline void require_plain(const Graph& g, const char* where) {
  if (g.variant != 0)
    throw Error(TC_EINVAL, std::string(where) + ": not defined for a variant graph (tc_graph_variant); "
                                                "use the graph it was made from");
}

// ---- work-set construction (tc_preprocess.hip) --------------------------------
// From T tasks in hashed-row order (tb_row = row of each task, tb_ptr = row
// bounds, tb_val = first probe | end << 32 of each task, tb_prefix = the
// exclusive prefix of their probe counts with the total at [T]): classes,
// class-major order, packs and items. hrow_ptr gives |U_b| of every hashed row.
// all_rows: every hashed row gets a work unit, also rows without tasks (the
// ablation of the doubly sparse traversal; they go to pack_small).
void build_work(WorkSet& w, Owned& own, int64_t nrows, const int64_t* hrow_ptr, int64_t T,
                const uint32_t* tb_row, const int64_t* tb_ptr, const uint64_t* tb_val,
                const uint64_t* tb_prefix, const WorkParams& wp, hipStream_t st, bool all_rows = false);

// ---- tuning table (tc_tuning.cpp) ----------------------------------------------
// Tuned settings by key "<arch>/<CUs>cu/<kind>_e<k>" (kind "graph" for one
// graph of about 2^k edges, "batch" for a batch of about 2^k edges in total),
// each a flat JSON object. Filled by tc_tuning_load, the TC_TUNING_FILE
// environment variable (read once, at the first lookup) and the autotuners.
std::string tuning_key(const char* kind, int64_t edges);
// The entry for `key`, or "" if there is none.
std::string tuning_lookup(const std::string& key);
void tuning_store(const std::string& key, const std::string& json);
// Parses the threshold keys of a flat JSON object into wp (other keys are
// left to the caller: `rest` receives them); TC_EINVAL on bad values.
std::map<std::string, std::string> parse_flat_json(const char* js);
bool parse_work_key(const std::string& k, const std::string& v, WorkParams& wp);
std::string work_params_json(const WorkParams& wp);
// The thresholds for one graph of m edges: the tuning table's entry for its
// size, else the defaults.
WorkParams default_work_params(int64_t m);


inline int ceil_log2_u64(uint64_t x) {
  int r = 0;
  while ((1ULL << r) < x) ++r;
  return r;
}

}  // namespace tc
