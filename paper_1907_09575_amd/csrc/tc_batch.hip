// tc_batch.hip - batched counting of many preprocessed graphs in one
// persistent launch, its plan (work units of every graph in one device queue),
// HIP-graph capture of the launch, and the schedule autotuner.
//
// The units are exactly the work units the single-graph launches run (packs
// of light rows, work-groups of items of heavy rows), so every per-graph count
// is the same integer as tc_count's. The plan orders them largest first
// (longest-processing-time order) so that the persistent work-groups finish
// together; the tuner picks the schedule on the actual batch:
//   blocks_per_cu - resident work-groups per compute unit (grid size);
//   lds_cap_log2  - largest table kept in LDS: item rows above it (the
//                   heaviest row bucket) are looked up in HBM instead, which
//                   shrinks the kernel's LDS and raises occupancy;
//   order         - "lpt" (largest unit first) or "input" (graph order);
//   graph         - 1: launch through a captured HIP graph, 0: plain launches.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cctype>
#include <cstring>
#include <map>
#include <memory>
#include <mutex>
#include <string>

#include "tc_prims.h"

namespace tc {

namespace {

struct Tuning {
  int blocks_per_cu = 0;  // 0: as many as LDS allows, at most kMaxBlocksPerCU
  int lds_cap_log2 = kMaxLog2S;
  bool lpt = true;
  bool graph = true;
  int chunk = 1;  // units per queue atomic (0: about 16 atomics per work-group)
  bool has_wp = false;  // row-bucket thresholds named: graphs cut otherwise get a retuned copy
  WorkParams wp;
};

constexpr int kMaxBlocksPerCU = 8;
constexpr size_t kLdsPerCU = 160 * 1024;

int to_int(const std::string& k, const std::string& v) {
  char* end = nullptr;
  long x = std::strtol(v.c_str(), &end, 10);
  TC_REQUIRE(end && *end == '\0' && !v.empty(), TC_EINVAL, "tuning json: " + k + " must be an integer");
  return (int)x;
}

Tuning parse_tuning(const char* js) {
  Tuning t;
  if (!js || !*js) return t;
  for (const auto& kv : parse_flat_json(js)) {
    const std::string& k = kv.first;
    const std::string& v = kv.second;
    if (k == "blocks_per_cu") {
      t.blocks_per_cu = to_int(k, v);
      TC_REQUIRE(t.blocks_per_cu >= 0 && t.blocks_per_cu <= 64, TC_EINVAL,
                 "tuning json: blocks_per_cu outside [0, 64]");
    } else if (k == "lds_cap_log2") {
      t.lds_cap_log2 = to_int(k, v);
      TC_REQUIRE(t.lds_cap_log2 >= 6 && t.lds_cap_log2 <= kMaxLog2S, TC_EINVAL,
                 "tuning json: lds_cap_log2 outside [6, 14]");
    } else if (k == "order") {
      TC_REQUIRE(v == "lpt" || v == "input", TC_EINVAL, "tuning json: order must be \"lpt\" or \"input\"");
      t.lpt = v == "lpt";
    } else if (k == "graph") {
      t.graph = to_int(k, v) != 0;
    } else if (k == "chunk") {
      t.chunk = to_int(k, v);
      TC_REQUIRE(t.chunk >= 0 && t.chunk <= 4096, TC_EINVAL, "tuning json: chunk outside [0, 4096]");
    } else if (k == "waves_per_block") {
      TC_REQUIRE(to_int(k, v) == kWaves, TC_EINVAL, "tuning json: waves_per_block must be 4");
    } else if (parse_work_key(k, v, t.wp)) {
      t.has_wp = true;
    } else if (k == "ms" || k == "units" || k == "hbm_units" || k == "grid" || k == "lds_bytes" ||
               k == "retuned") {
      // descriptive keys of the tuner's own output, accepted so that it can be passed back
    } else {
      throw Error(TC_EINVAL, "tuning json: unknown key \"" + k + "\"");
    }
  }
  return t;
}

constexpr int kItemClasses = NUM_CLASSES - CLS_WG_SMALL;  // wg_small .. global

// Per graph entry of the plan: where its units come from (device copy).
struct BatchSrc {
  const PackRow* pack_recs[2];
  const PackInfo* pack_info[2];
  const CountItem* items[kItemClasses];  // classes wg_small .. global
  const uint32_t* tbeg;
  const uint32_t* tend;
  const uint64_t* tprefix;
  const int64_t* row_ptr;
  uint32_t n_packs[2];
  uint32_t pack_slots[2];
  uint32_t n_groups[kItemClasses];
  int32_t kind[kItemClasses];  // BatchKind of each item class under the plan's LDS cap
  uint64_t unit_off;
};

// One work-group per graph entry: emit its units and their weights (probes
// plus per-row overheads; the LPT key is the complement of the weight; key
// and idx may be null when no order is wanted).
__global__ __launch_bounds__(256) void k_batch_units(const BatchSrc* __restrict__ src, BatchUnit* __restrict__ units,
                                                     uint32_t* __restrict__ key, uint32_t* __restrict__ idx) {
  const BatchSrc& s = src[blockIdx.x];
  const uint32_t np0 = s.n_packs[0], np1 = s.n_packs[1];
  uint32_t total = np0 + np1;
  for (int c = 0; c < kItemClasses; ++c) total += s.n_groups[c];
  for (uint32_t j = threadIdx.x; j < total; j += blockDim.x) {
    BatchUnit u;
    uint64_t wgt = 0;
    u.graph = (int32_t)blockIdx.x;
    if (j < np0 + np1) {
      const int c = j < np0 ? 0 : 1;
      const uint32_t p = j < np0 ? j : j - np0;
      const PackInfo& pi = s.pack_info[c][p];
      wgt = pi.q1 - pi.q0 + 64ull * (pi.r1 - pi.r0);
      u.p0 = s.pack_recs[c];
      u.p1 = s.pack_info[c];
      u.index = p;
      u.slots = s.pack_slots[c];
      u.kind = BK_PACK;
    } else {
      uint32_t r = j - np0 - np1;
      int c = 0;
      while (r >= s.n_groups[c]) r -= s.n_groups[c++];
      const CountItem* g = s.items[c] + (uint64_t)r * kWaves;
      for (int w = 0; w < kWaves; ++w) wgt += g[w].len;
      const int32_t b = g[0].b;
      wgt += (uint64_t)(s.row_ptr[b + 1] - s.row_ptr[b]);
      u.p0 = g;
      u.p1 = nullptr;
      u.index = r;
      u.slots = 0;
      u.kind = s.kind[c];
    }
    const uint64_t o = s.unit_off + j;
    units[o] = u;
    if (key) {  // LPT order wanted: weights for the sort
      key[o] = 0xFFFFFFFFu - (uint32_t)(wgt < 0xFFFFFFFFull ? wgt : 0xFFFFFFFFull);
      idx[o] = (uint32_t)o;
    }
  }
}

__global__ void k_gather_units(const BatchUnit* __restrict__ in, const uint32_t* __restrict__ order, int64_t n,
                               BatchUnit* __restrict__ out) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) out[i] = in[order[i]];
}

}  // namespace

struct BatchPlan {
  int device = 0;
  CountMode mode = MODE_COUNT;
  std::vector<std::pair<int32_t*, int64_t>> support;  // arrays cleared before each launch
  int64_t n_graphs = 0, n_units = 0, hbm_units = 0;
  int bpc = 0;  // resident work-groups per compute unit the grid was sized for
  uint32_t chunk = 1;  // units per queue atomic
  unsigned grid = 0;
  size_t lds = 0;
  int cus = 0;
  Tuning tun;
  Owned own;
  CountArgs* d_args = nullptr;
  BatchUnit* d_units = nullptr;
  unsigned int* d_queue = nullptr;
  hipStream_t cap_stream = nullptr;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  int64_t* exec_counts = nullptr;
  UseLog uses;  // streams the plan was launched on
  std::vector<Graph*> twins;  // retuned copies of graphs cut by other thresholds

  void drop_graph() {
    if (exec) (void)hipGraphExecDestroy(exec);
    if (graph) (void)hipGraphDestroy(graph);
    exec = nullptr;
    graph = nullptr;
    exec_counts = nullptr;
  }
  ~BatchPlan() {
    drop_graph();
    if (cap_stream) {
      cache_retire_stream(cap_stream);
      (void)hipStreamDestroy(cap_stream);
    }
    for (Graph* h : twins) destroy_graph(h);
  }
};

namespace {

// Host side of a plan: every entry's kernel arguments and unit sources, the
// dynamic LDS the persistent kernel needs, the number of units and how many
// of them look their rows up in HBM. Support arrays of support modes are
// recorded in `support` when it is not null.
struct PlanHost {
  std::vector<CountArgs> args;
  std::vector<BatchSrc> srcs;
  size_t lds = 0;
  uint64_t units = 0;
  int64_t hbm_units = 0;
};

void plan_host(PlanHost& H, const PlanEntry* entries, int64_t num, CountMode mode, const Tuning& t,
               int device, std::vector<std::pair<int32_t*, int64_t>>* support) {
  H.args.assign((size_t)std::max<int64_t>(num, 1), CountArgs{});
  H.srcs.assign((size_t)std::max<int64_t>(num, 1), BatchSrc{});
  size_t lds = 0;
  uint64_t off = 0;
  int64_t hbm_units = 0;
  for (int64_t i = 0; i < num; ++i) {
    TC_REQUIRE(entries[i].g != nullptr, TC_EINVAL, "batch plan: null graph handle");
    const Graph& g = *entries[i].g;
    TC_REQUIRE(g.device == device, TC_EINVAL, "batch plan: graph built on another device");
    require_plain(g, "batch plan");
    TC_REQUIRE(g.m <= kMaxBufferEdges, TC_EOVERFLOW,
               "batch plan: a graph of 2^30 edges or more (count it with tc_count)");
    const WorkSet& w = g.w;
    CountArgs& A = H.args[(size_t)i];
    std::memset(&A, 0, sizeof(A));
    A.row_ptr = g.row_ptr;
    A.hcol = g.col;
    A.col = g.col;
    A.tstart = w.tstart;
    A.tprefix = w.tprefix;
    A.tbeg = w.tbeg;
    A.tend = w.tend;
    A.T = w.n_tasks;
    A.m = (uint32_t)g.m;
    A.q = 1;
    if (mode != MODE_COUNT) {
      TC_REQUIRE(entries[i].support != nullptr || g.m == 0, TC_EINVAL, "batch plan: null support array");
      A.support = entries[i].support;
      if (g.m > 0 && support) support->emplace_back(entries[i].support, g.m);
    }
    BatchSrc& s = H.srcs[(size_t)i];
    std::memset(&s, 0, sizeof(s));
    s.tbeg = w.tbeg;
    s.tend = w.tend;
    s.tprefix = w.tprefix;
    s.row_ptr = g.row_ptr;
    s.unit_off = off;
    if (w.n_tasks == 0) continue;  // no units: the count stays 0
    for (int c = 0; c < 2; ++c) {
      s.pack_recs[c] = w.pack_recs[c];
      s.pack_info[c] = w.pack_info[c];
      s.n_packs[c] = (uint32_t)w.n_packs[c];
      if (w.n_packs[c] == 0) continue;
      s.pack_slots[c] = w.wp.pack_slots + (1u << w.pack_log2S[c]);
      lds = std::max(lds, pack_lds_bytes(s.pack_slots[c], mode));
      off += (uint64_t)w.n_packs[c];
    }
    for (int c = 0; c < kItemClasses; ++c) {
      const int cls = CLS_WG_SMALL + c;
      s.items[c] = w.items[cls];
      s.n_groups[c] = (uint32_t)(w.n_items[cls] / kWaves);
      if (s.n_groups[c] == 0) continue;
      const bool hbm = cls == CLS_GLOBAL || w.cls_log2S[cls] > t.lds_cap_log2;
      s.kind[c] = hbm ? BK_ITEMS_HBM : BK_ITEMS;
      lds = std::max(lds, items_lds_bytes(hbm ? -1 : w.cls_log2S[cls], mode));
      if (hbm) hbm_units += s.n_groups[c];
      off += s.n_groups[c];
    }
  }
  H.lds = std::max(lds, items_lds_bytes(-1, mode));
  H.units = off;
  H.hbm_units = hbm_units;
}

// Resident work-groups per CU and the persistent grid of a schedule.
void plan_grid(const Tuning& t, size_t lds, int64_t n_units, int cus, int& bpc, unsigned& grid,
               uint32_t& chunk) {
  bpc = t.blocks_per_cu;
  if (bpc == 0) bpc = (int)std::max<size_t>(1, std::min<size_t>(kMaxBlocksPerCU, kLdsPerCU / lds));
  grid = (unsigned)std::max<int64_t>(1, std::min<int64_t>(n_units, (int64_t)bpc * cus));
  chunk = t.chunk > 0 ? (uint32_t)t.chunk
                      : (uint32_t)std::max<int64_t>(1, std::min<int64_t>(64, n_units / ((int64_t)grid * 16)));
}

}  // namespace

BatchPlan* make_plan(const PlanEntry* entries, int64_t num, CountMode mode, const char* tuning_json,
                     hipStream_t st) {
  TC_REQUIRE(mode == MODE_COUNT || mode == MODE_SUPPORT_FULL || mode == MODE_SUPPORT_ORIENTED, TC_EINVAL,
             "batch plan: unsupported mode");
  TC_REQUIRE(num >= 0 && num < (1ll << 31), TC_EINVAL, "batch plan: bad number of graphs");
  std::unique_ptr<BatchPlan> P(new BatchPlan());
  P->own.st = st;
  std::string looked;
  if (!tuning_json || !*tuning_json) {
    // no schedule given: the tuning table's for batches of this size, if any
    int64_t edges = 0;
    for (int64_t i = 0; i < num; ++i) edges += entries[i].g ? entries[i].g->m : 0;
    looked = tuning_lookup(tuning_key("batch", edges));
    if (!looked.empty()) tuning_json = looked.c_str();
  }
  P->tun = parse_tuning(tuning_json);
  P->mode = mode;
  TC_HIP(hipGetDevice(&P->device));
  TC_HIP(hipDeviceGetAttribute(&P->cus, hipDeviceAttributeMultiprocessorCount, P->device));
  P->n_graphs = num;
  const Tuning& t = P->tun;
  std::vector<PlanEntry> ents(entries, entries + num);
  if (t.has_wp) {
    // graphs whose work is cut by other thresholds are counted through a
    // retuned copy (sharing their U), one per distinct graph
    std::map<const Graph*, Graph*> twin;
    for (PlanEntry& e : ents) {
      if (!e.g || e.g->w.wp == t.wp) continue;
      require_plain(*e.g, "batch plan");
      auto it = twin.find(e.g);
      if (it == twin.end()) {
        P->twins.push_back(build_variant(*e.g, 0, t.wp, st));
        it = twin.emplace(e.g, P->twins.back()).first;
      }
      e.g = it->second;
    }
  }
  PlanHost H;
  plan_host(H, ents.data(), num, mode, t, P->device, &P->support);
  std::vector<CountArgs>& args = H.args;
  std::vector<BatchSrc>& srcs = H.srcs;
  const uint64_t off = H.units;
  TC_REQUIRE(off < 0xFFFFFFF0ull, TC_EOVERFLOW, "tc_batch_create: more than 2^32 work units");
  P->n_units = (int64_t)off;
  P->hbm_units = H.hbm_units;
  P->lds = H.lds;
  plan_grid(t, P->lds, P->n_units, P->cus, P->bpc, P->grid, P->chunk);
  batch_kernel_lds(mode, P->lds);

  P->d_args = P->own.alloc<CountArgs>(std::max<int64_t>(num, 1));
  P->d_units = P->own.alloc<BatchUnit>(std::max<int64_t>(P->n_units, 1));
  P->d_queue = P->own.alloc<unsigned int>(1);
  TC_HIP(hipMemcpyAsync(P->d_args, args.data(), sizeof(CountArgs) * (size_t)num, hipMemcpyHostToDevice, st));
  if (P->n_units > 0) {
    TempStream temps(st);
    DevBuf dsrc(sizeof(BatchSrc) * (size_t)num);
    TC_HIP(hipMemcpyAsync(dsrc.p, srcs.data(), sizeof(BatchSrc) * (size_t)num, hipMemcpyHostToDevice, st));
    const int64_t n = P->n_units;
    if (!t.lpt) {
      // graph order: the units go straight to the plan (no sort, no sync)
      TC_LAUNCH("batch_units", k_batch_units, dim3((unsigned)num), dim3(256), 0, st, dsrc.as<BatchSrc>(),
                P->d_units, (uint32_t*)nullptr, (uint32_t*)nullptr);
      TC_HIP(hipGetLastError());
    } else {
      DevBuf raw(sizeof(BatchUnit) * (size_t)n);
      DevBuf key(sizeof(uint32_t) * (size_t)n), key2(sizeof(uint32_t) * (size_t)n);
      DevBuf idx(sizeof(uint32_t) * (size_t)n), idx2(sizeof(uint32_t) * (size_t)n);
      TC_LAUNCH("batch_units", k_batch_units, dim3((unsigned)num), dim3(256), 0, st, dsrc.as<BatchSrc>(),
                raw.as<BatchUnit>(), key.as<uint32_t>(), idx.as<uint32_t>());
      TC_HIP(hipGetLastError());
      const bool alt = radix_sort<uint32_t, uint32_t>(key.as<uint32_t>(), key2.as<uint32_t>(), idx.as<uint32_t>(),
                                                      idx2.as<uint32_t>(), n, 0, 32, st, "batch_lpt");
      const uint32_t* order = alt ? idx2.as<uint32_t>() : idx.as<uint32_t>();
      TC_LAUNCH("batch_gather", k_gather_units, dim3((unsigned)div_up(n, 256)), dim3(256), 0, st,
                raw.as<BatchUnit>(), order, n, P->d_units);
      TC_HIP(hipGetLastError());
      check_sorts(st);  // (synchronises st)
    }
  }
  return P.release();
}

namespace {

void plan_launch(BatchPlan& P, int64_t* d_counts, hipStream_t st, bool timed) {
  for (const auto& z : P.support) zero_i32(z.first, z.second, st, timed);
  launch_batch(P.mode, P.d_args, P.d_units, P.n_units, P.chunk, P.n_graphs, P.d_queue, d_counts, P.grid, P.lds, st,
               timed);
}

}  // namespace

void free_plan_idle(BatchPlan* P) {
  if (!P) return;
  P->own.release(true);
  delete P;
}

void free_plan(BatchPlan* P) {
  if (!P) return;
  // launches of the plan may still be queued on the streams it was launched
  // on: wait for them (not for the whole device). The graphs' memory stays
  // valid until then, as the plan's contract requires.
  P->uses.wait_host();
  free_plan_idle(P);
}

int64_t plan_units(const BatchPlan& P) { return P.n_units; }

void plan_count(BatchPlan& P, int64_t* d_counts, hipStream_t st) {
  hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
  TC_HIP(hipStreamIsCapturing(st, &cs));
  if (cs != hipStreamCaptureStatusNone) {
    // the caller is capturing: record the launches into its graph
    plan_launch(P, d_counts, st, false);
    P.uses.note(st);  // (marks the plan as captured: its free waits for the device)
    return;
  }
  if (!P.tun.graph) {
    plan_launch(P, d_counts, st, true);
    P.uses.note(st);
    return;
  }
  if (!P.exec || P.exec_counts != d_counts) {
    P.drop_graph();
    if (!P.cap_stream) TC_HIP(hipStreamCreateWithFlags(&P.cap_stream, hipStreamNonBlocking));
    TC_HIP(hipStreamBeginCapture(P.cap_stream, hipStreamCaptureModeThreadLocal));
    try {
      plan_launch(P, d_counts, P.cap_stream, false);
    } catch (...) {
      hipGraph_t g = nullptr;
      (void)hipStreamEndCapture(P.cap_stream, &g);
      if (g) (void)hipGraphDestroy(g);
      throw;
    }
    TC_HIP(hipStreamEndCapture(P.cap_stream, &P.graph));
    TC_HIP(hipGraphInstantiate(&P.exec, P.graph, nullptr, nullptr, 0));
    P.exec_counts = d_counts;
  }
  {
    LaunchScope ls("batch:graph", st);
    TC_HIP(hipGraphLaunch(P.exec, st));
  }
  P.uses.note(st);
}

namespace {

std::string plan_json(const BatchPlan& P, double ms) {
  char buf[512];
  std::snprintf(buf, sizeof(buf),
                "{\"blocks_per_cu\": %d, \"lds_cap_log2\": %d, \"order\": \"%s\", \"graph\": %d, "
                "\"chunk\": %d, ",
                P.bpc, P.tun.lds_cap_log2, P.tun.lpt ? "lpt" : "input", P.tun.graph ? 1 : 0, P.tun.chunk);
  std::string s = buf;
  if (P.tun.has_wp) s += work_params_json(P.tun.wp) + ", \"retuned\": " + std::to_string(P.twins.size()) + ", ";
  std::snprintf(buf, sizeof(buf),
                "\"units\": %lld, \"hbm_units\": %lld, \"grid\": %u, \"lds_bytes\": %zu, \"ms\": %.4f}",
                (long long)P.n_units, (long long)P.hbm_units, P.grid, P.lds, ms);
  return s + buf;
}

template <class F>
tc_status guard(const char* where, F&& f) {
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

void copy_out(const std::string& s, char* out, size_t cap) {
  TC_REQUIRE(out != nullptr && cap > s.size(), TC_EINVAL, "output buffer too small for the JSON text");
  std::memcpy(out, s.c_str(), s.size() + 1);
}

}  // namespace

// ---- counting without allocation -------------------------------------------
// tc_count_batched_noalloc keeps everything a batch plan would allocate -
// the queue counter, every graph's kernel arguments and unit sources, and the
// units themselves - in one fixed device array. Every GPU the library runs
// on holds its own copy of it until the process ends; host code must use the
// address hipGetSymbolAddress returns for the current device, never the
// array's name (which in host code is only a stand-in for the symbol).
namespace {

constexpr size_t kScratchBytes = 64ull << 20;  // 64 MiB: about 2 million units
constexpr int kScratchDevices = 64;
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

std::mutex g_scratch_mu;
void* g_scratch_ptr[kScratchDevices] = {};

// Address of this device's scratch array (looked up once per device, with
// that device current).
unsigned char* scratch_on(int device) {
  TC_REQUIRE(device >= 0 && device < kScratchDevices, TC_EINVAL, "tc_count_batched_noalloc: device id too large");
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch_ptr[device]) {
    void* p = nullptr;
    TC_HIP(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
    TC_REQUIRE(p != nullptr, TC_EDEVICE, "tc_count_batched_noalloc: no address for the scratch array");
    g_scratch_ptr[device] = p;
  }
  return static_cast<unsigned char*>(g_scratch_ptr[device]);
}

size_t align256(size_t b) { return (b + 255) & ~(size_t)255; }

// Layout of one call in the scratch array: queue counter, kernel arguments,
// unit sources, units (in graph order).
struct ScratchLayout {
  size_t args = 0, srcs = 0, units = 0, total = 0;
  ScratchLayout(int64_t num, int64_t n_units) {
    args = 256;
    srcs = args + align256(sizeof(CountArgs) * (size_t)std::max<int64_t>(num, 1));
    units = srcs + align256(sizeof(BatchSrc) * (size_t)std::max<int64_t>(num, 1));
    total = units + sizeof(BatchUnit) * (size_t)std::max<int64_t>(n_units, 1);
  }
};

void count_batched_noalloc(const PlanEntry* entries, int64_t num, int64_t* d_counts, hipStream_t st) {
  int device = 0;
  TC_HIP(hipGetDevice(&device));
  int cus = 0;
  TC_HIP(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, device));
  unsigned char* base = scratch_on(device);
  Tuning t;  // the default schedule, graph order (no sort: sorting needs temporaries)
  t.lpt = false;
  PlanHost H;
  plan_host(H, entries, num, MODE_COUNT, t, device, nullptr);
  TC_REQUIRE(H.units < 0xFFFFFFF0ull, TC_EOVERFLOW, "tc_count_batched_noalloc: more than 2^32 work units");
  const ScratchLayout L(num, (int64_t)H.units);
  if (L.total > kScratchBytes)
    throw Error(TC_EOVERFLOW, "tc_count_batched_noalloc: the batch needs " + std::to_string(L.total) +
                                  " bytes of scratch (" + std::to_string(H.units) + " work units), more than its " +
                                  std::to_string(kScratchBytes) + "-byte array; use tc_count_batched");
  int bpc = 0;
  unsigned grid = 0;
  uint32_t chunk = 1;
  plan_grid(t, H.lds, (int64_t)H.units, cus, bpc, grid, chunk);
  batch_kernel_lds(MODE_COUNT, H.lds);
  auto* d_queue = reinterpret_cast<unsigned int*>(base);
  auto* d_args = reinterpret_cast<CountArgs*>(base + L.args);
  auto* d_srcs = reinterpret_cast<BatchSrc*>(base + L.srcs);
  auto* d_units = reinterpret_cast<BatchUnit*>(base + L.units);
  TC_HIP(hipMemcpyAsync(d_args, H.args.data(), sizeof(CountArgs) * (size_t)num, hipMemcpyHostToDevice, st));
  TC_HIP(hipMemcpyAsync(d_srcs, H.srcs.data(), sizeof(BatchSrc) * (size_t)num, hipMemcpyHostToDevice, st));
  if (H.units > 0) {
    TC_LAUNCH("batch_units", k_batch_units, dim3((unsigned)num), dim3(256), 0, st, d_srcs, d_units,
              (uint32_t*)nullptr, (uint32_t*)nullptr);
    TC_HIP(hipGetLastError());
  }
  // clears the counts and the queue counter (a kernel), then the persistent launch
  launch_batch(MODE_COUNT, d_args, d_units, (int64_t)H.units, chunk, num, d_queue, d_counts, grid, H.lds, st, true);
  // the host copies above read H's vectors: they must be done before H goes
  TC_HIP(hipStreamSynchronize(st));
}

}  // namespace

}  // namespace tc

struct tc_batch {
  tc::BatchPlan* p;
};

extern "C" {

tc_status tc_batch_create(const tc_graph* const* graphs, int32_t num_graphs, const char* tuning_json,
                          void* stream, tc_batch** out) {
  return tc::guard("tc_batch_create", [&] {
    TC_REQUIRE(out != nullptr, TC_EINVAL, "tc_batch_create: out is NULL");
    *out = nullptr;
    TC_REQUIRE(num_graphs >= 0, TC_EINVAL, "tc_batch_create: num_graphs < 0");
    TC_REQUIRE(num_graphs == 0 || graphs != nullptr, TC_EINVAL, "tc_batch_create: null graph list");
    std::vector<tc::PlanEntry> e((size_t)num_graphs);
    for (int32_t i = 0; i < num_graphs; ++i) e[(size_t)i] = tc::PlanEntry{tc::G(graphs[i]), nullptr};
    std::unique_ptr<tc::BatchPlan> p(tc::make_plan(e.data(), num_graphs, tc::MODE_COUNT, tuning_json,
                                                   static_cast<hipStream_t>(stream)));
    *out = new tc_batch{p.release()};
  });
}

tc_status tc_batch_count(tc_batch* plan, int64_t* d_counts, void* stream) {
  return tc::guard("tc_batch_count", [&] {
    TC_REQUIRE(plan != nullptr && plan->p != nullptr, TC_EINVAL, "tc_batch_count: null plan");
    TC_REQUIRE(d_counts != nullptr || plan->p->n_graphs == 0, TC_EINVAL, "tc_batch_count: null counts");
    if (plan->p->n_graphs == 0) return;
    tc::plan_count(*plan->p, d_counts, static_cast<hipStream_t>(stream));
  });
}

void tc_batch_free(tc_batch* plan) {
  if (!plan) return;
  tc::free_plan(plan->p);
  delete plan;
}

tc_status tc_batch_describe(const tc_batch* plan, char* out, size_t cap) {
  return tc::guard("tc_batch_describe", [&] {
    TC_REQUIRE(plan != nullptr && plan->p != nullptr, TC_EINVAL, "tc_batch_describe: null plan");
    tc::copy_out(tc::plan_json(*plan->p, 0.0), out, cap);
  });
}

tc_status tc_count_batched(const tc_graph* const* graphs, int32_t num_graphs, int64_t* d_counts,
                           const char* tuning_json, void* stream) {
  tc_batch* plan = nullptr;
  tc_status s = tc_batch_create(graphs, num_graphs, tuning_json, stream, &plan);
  if (s != TC_OK) return s;
  s = tc_batch_count(plan, d_counts, stream);
  if (s == TC_OK) {
    hipError_t e = hipStreamSynchronize(static_cast<hipStream_t>(stream));
    if (e != hipSuccess) {
      tc::set_last_error(std::string("tc_count_batched: ") + hipGetErrorString(e));
      s = TC_EDEVICE;
    }
  }
  tc_batch_free(plan);
  return s;
}

tc_status tc_count_batched_noalloc(const tc_graph* const* graphs, int32_t num_graphs, int64_t* d_counts,
                                   void* stream) {
  return tc::guard("tc_count_batched_noalloc", [&] {
    TC_REQUIRE(num_graphs >= 0, TC_EINVAL, "tc_count_batched_noalloc: num_graphs < 0");
    TC_REQUIRE(num_graphs == 0 || graphs != nullptr, TC_EINVAL, "tc_count_batched_noalloc: null graph list");
    TC_REQUIRE(num_graphs == 0 || d_counts != nullptr, TC_EINVAL, "tc_count_batched_noalloc: null counts");
    if (num_graphs == 0) return;
    std::vector<tc::PlanEntry> e((size_t)num_graphs);
    for (int32_t i = 0; i < num_graphs; ++i) e[(size_t)i] = tc::PlanEntry{tc::G(graphs[i]), nullptr};
    tc::count_batched_noalloc(e.data(), num_graphs, d_counts, static_cast<hipStream_t>(stream));
  });
}

tc_status tc_batch_autotune(const tc_graph* const* graphs, int32_t num_graphs, void* stream, char* out_json,
                            size_t cap) {
  return tc::guard("tc_batch_autotune", [&] {
    TC_REQUIRE(num_graphs > 0 && graphs != nullptr, TC_EINVAL, "tc_batch_autotune: no graphs");
    hipStream_t st = static_cast<hipStream_t>(stream);
    int max_log2 = 0;
    int64_t edges = 0;
    for (int32_t i = 0; i < num_graphs; ++i) {
      TC_REQUIRE(graphs[i] != nullptr, TC_EINVAL, "tc_batch_autotune: null graph handle");
      tc::require_plain(*tc::G(graphs[i]), "tc_batch_autotune");
      const tc::WorkSet& w = tc::G(graphs[i])->w;
      edges += tc::G(graphs[i])->m;
      for (int c = tc::CLS_WG_SMALL; c <= tc::CLS_WG_GIANT; ++c)
        if (w.n_items[c]) max_log2 = std::max(max_log2, w.cls_log2S[c]);
    }
    std::vector<tc::PlanEntry> own_ents((size_t)num_graphs);
    for (int32_t i = 0; i < num_graphs; ++i) own_ents[(size_t)i] = tc::PlanEntry{tc::G(graphs[i]), nullptr};
    int64_t* d_counts = nullptr;
    TC_HIP(hipMalloc(&d_counts, sizeof(int64_t) * (size_t)num_graphs));
    std::unique_ptr<int64_t, void (*)(int64_t*)> hold(d_counts, [](int64_t* p) { (void)hipFree(p); });
    hipEvent_t e0, e1;
    TC_HIP(hipEventCreate(&e0));
    TC_HIP(hipEventCreate(&e1));
    struct EvHold {
      hipEvent_t a, b;
      ~EvHold() {
        (void)hipEventDestroy(a);
        (void)hipEventDestroy(b);
      }
    } eh{e0, e1};
    std::string best, all = "[";
    std::string best_sched;  // schedule keys of the best candidate (no thresholds)
    tc::WorkParams best_wp = tc::G(graphs[0])->w.wp;
    bool best_has_wp = false;
    double best_ms = 1e30;
    // A plan with thresholds other than the graphs' own builds a retuned copy
    // of every graph when it is created (about one work-set build per graph):
    // such a candidate must beat the best by this factor to be kept.
    constexpr double kRetuneGain = 0.98;
    // times one candidate (best of 3 after a warm-up) and keeps the best
    // (full = false: a sample of the graphs, timed for comparison only)
    auto run = [&](const std::vector<tc::PlanEntry>& ents, const std::string& sched, const tc::WorkParams* wp,
                   size_t retuned, bool full = true) {
      std::unique_ptr<tc::BatchPlan> P(
          tc::make_plan(ents.data(), (int64_t)ents.size(), tc::MODE_COUNT, sched.c_str(), st));
      if (wp) {  // describe the thresholds the entries were retuned with
        P->tun.has_wp = true;
        P->tun.wp = *wp;
      }
      tc::plan_count(*P, d_counts, st);  // warm-up (and graph capture)
      double ms = 1e30;
      for (int r = 0; r < 3; ++r) {
        TC_HIP(hipEventRecord(e0, st));
        tc::plan_count(*P, d_counts, st);
        TC_HIP(hipEventRecord(e1, st));
        TC_HIP(hipEventSynchronize(e1));
        float f = 0;
        TC_HIP(hipEventElapsedTime(&f, e0, e1));
        ms = std::min(ms, (double)f);
      }
      std::string j = tc::plan_json(*P, ms);
      if (wp) {
        const std::string k = "\"retuned\": 0";
        const size_t at = j.find(k);
        if (at != std::string::npos) j.replace(at, k.size(), "\"retuned\": " + std::to_string(retuned));
      }
      j.insert(j.size() - 1, ", \"graphs\": " + std::to_string(ents.size()));
      all += (all.size() > 1 ? ", " : "") + j;
      if (!full) return ms;
      if (ms < (wp && !best_has_wp ? best_ms * kRetuneGain : best_ms)) {
        best_ms = ms;
        best = j;
        best_sched = sched;
        if (wp) best_wp = *wp;
        best_has_wp = wp != nullptr;
      }
      return ms;
    };
    // 1: schedules on the graphs' own work: LDS caps that change the plan x
    // unit orders x grid sizes
    std::vector<int> caps = {tc::kMaxLog2S};
    for (int c : {12, 10})
      if (c < max_log2) caps.push_back(c);
    for (int cap_log2 : caps)
      for (int lpt = 1; lpt >= 0; --lpt)
        for (int bpc : {2, 4, 6, 8}) {
          char js[160];
          std::snprintf(js, sizeof(js), "{\"blocks_per_cu\": %d, \"lds_cap_log2\": %d, \"order\": \"%s\"}", bpc,
                        cap_log2, lpt ? "lpt" : "input");
          run(own_ents, js, nullptr, 0);
        }
    // 2: units per queue atomic, on the best schedule
    const std::string sched1 = best_sched;
    for (int chunk : {0, 4}) {
      std::string js = sched1;
      js.insert(js.size() - 1, ", \"chunk\": " + std::to_string(chunk));
      run(own_ents, js, nullptr, 0);
    }
    // 3: row-bucket thresholds, one at a time from the graphs' own. Each
    // candidate counts retuned copies of the graphs (a work-set build per
    // graph), so they are compared on a sample of at most kSample graphs
    // (every stride-th); thresholds that win there are then timed on the
    // whole batch.
    constexpr int64_t kSample = 512;
    const std::string sched2 = best_sched;
    const int64_t stride = (num_graphs + kSample - 1) / kSample;
    const bool sampled = stride > 1;
    std::vector<tc::PlanEntry> sample;
    for (int64_t i = 0; i < num_graphs; i += stride) sample.push_back(own_ents[(size_t)i]);
    auto retuned_entries = [&](const std::vector<tc::PlanEntry>& from, const tc::WorkParams& wp,
                               std::vector<std::unique_ptr<tc::Graph, void (*)(tc::Graph*)>>& held) {
      std::map<const tc::Graph*, tc::Graph*> twin;
      std::vector<tc::PlanEntry> ents = from;
      for (tc::PlanEntry& e : ents) {
        if (e.g->w.wp == wp) continue;
        auto it = twin.find(e.g);
        if (it == twin.end()) {
          held.emplace_back(tc::build_variant(*e.g, 0, wp, st), tc::destroy_graph);
          it = twin.emplace(e.g, held.back().get()).first;
        }
        e.g = it->second;
      }
      return ents;
    };
    const uint64_t heavy[] = {8192, 131072};
    const uint64_t target[] = {32768, 262144};
    const uint32_t slots[] = {2048, 8192};
    const uint32_t chunk[] = {8192, 16384};
    const uint32_t groups[] = {0, 65536};
    const tc::WorkParams own = best_wp;
    tc::WorkParams cur = own;
    double cur_ms = sampled ? run(sample, sched2, nullptr, 0, false) : best_ms;
    for (int param = 0; param < 5; ++param) {
      const tc::WorkParams start = cur;
      for (int c = 0; c < 2; ++c) {
        tc::WorkParams wp = start;
        if (param == 0) wp.heavy_min = heavy[c];
        if (param == 1) wp.pack_target = target[c];
        if (param == 2) wp.pack_slots = slots[c];
        if (param == 3) wp.wave_chunk = chunk[c];
        if (param == 4) wp.min_groups = groups[c];
        if (wp == start) continue;
        std::vector<std::unique_ptr<tc::Graph, void (*)(tc::Graph*)>> held;
        const std::vector<tc::PlanEntry> ents = retuned_entries(sampled ? sample : own_ents, wp, held);
        const double ms = run(ents, sched2, &wp, held.size(), !sampled);
        // (the first thresholds other than the graphs' own must win clearly)
        if (ms < (cur == own ? cur_ms * kRetuneGain : cur_ms)) {
          cur = wp;  // the next parameter starts from it
          cur_ms = ms;
        }
        TC_HIP(hipStreamSynchronize(st));  // the plan is gone; the copies go next
      }
    }
    if (sampled && cur != own) {
      std::vector<std::unique_ptr<tc::Graph, void (*)(tc::Graph*)>> held;
      run(retuned_entries(own_ents, cur, held), sched2, &cur, held.size());
      TC_HIP(hipStreamSynchronize(st));
    }
    // the best candidate's re-usable keys (schedule and thresholds) go into
    // the tuning table for batches of this size
    std::string entry = best_sched;
    if (best_has_wp) entry.insert(entry.size() - 1, ", " + tc::work_params_json(best_wp));
    char msb[48];
    std::snprintf(msb, sizeof(msb), ", \"ms\": %.4f", best_ms);
    entry.insert(entry.size() - 1, msb);
    const std::string key = tc::tuning_key("batch", edges);
    tc::tuning_store(key, entry);
    all += "]";
    const std::string res =
        "{\"key\": \"" + key + "\", \"best\": " + entry + ", \"plan\": " + best + ", \"candidates\": " + all + "}";
    tc::copy_out(res, out_json, cap);
  });
}

}  // extern "C"
