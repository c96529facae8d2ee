// tc_server.cpp - the served form: a request loop with continuous batching.
//
// Threads: one scheduler and a pool of preprocessing workers, each worker with
// its own stream. The scheduler
//   1. admits pending requests in arrival order while the in-flight ones stay
//      within max_slots and the reserved device bytes (estimates for requests
//      being preprocessed, resident cached graphs, support arrays) fit the
//      budget, evicting unused cached graphs (least recently used) for room;
//   2. hands graphs that are not resident to the workers (upload + the same
//      preprocessing as tc_preprocess), several at once;
//   3. when a tick slot is free (at most `ticks` ticks in flight, 1 by
//      default), starts a tick over every request whose graph is ready: one
//      batch plan and one persistent launch per operation on the tick
//      stream, then copies the counts to the slot's pinned host memory;
//   4. when a tick's event has completed, publishes its results (support
//      arrays copied to the caller's host buffers) and releases memory.
// Preprocessing of newly arrived requests overlaps the running ticks on the
// device; they join the next tick. With two slots, a tick of at least two
// requests is planned and launched while the previous one runs (both on the
// tick stream, so the device runs them one after the other without waiting
// for the host); on the benchmark's serving mix this measured no gain (open
// loop at 0.8 x capacity: 1529 against 1591 graphs/s), hence one by default.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <list>
#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <thread>
#include <vector>

#include "tc_internal.h"

namespace tc {
namespace {

using Clock = std::chrono::steady_clock;

struct CacheEntry;

struct Req {
  int64_t ticket = 0;
  tc_request r{};
  tc_result res{};
  std::string err;
  enum State { PENDING, PREP, READY, RUNNING, DONE } state = PENDING;
  size_t support_bytes = 0;  // reserved for the device support array
  size_t plan_bytes = 0;     // reserved for its share of a tick's batch plan
  CacheEntry* ce = nullptr;
  int32_t* d_support = nullptr;
  tc_status copy_status = TC_OK;  // support copy to the caller's buffer
  std::string copy_err;
};

struct CacheEntry {
  uint64_t key = 0;  // 0: private to one request (freed after it)
  Graph* g = nullptr;
  size_t est = 0;     // reservation while building
  size_t bytes = 0;   // resident bytes once built
  int refs = 0;       // admitted requests using it
  uint64_t last_use = 0;
  bool building = true;
  tc_status status = TC_OK;
  std::string err;
  // build input (host)
  const int32_t* src = nullptr;
  const int32_t* dst = nullptr;
  int64_t m_raw = 0;
  int32_t n = 0;
};

// Device bytes reserved while a graph is preprocessed: the uploaded edge list,
// the sort keys and flags of deduplication, the edge set, and the resident
// graph (CSR, rank map, tasks and work units).
size_t prep_estimate(int64_t m_raw, int64_t n) {
  return (size_t)(56 * m_raw + 40 * n) + ((size_t)1 << 20);
}

// Device bytes of a graph's share of a tick's batch plan: its kernel
// arguments and unit sources, and its work units (the plan's units and, while
// it is made, their first copy and sort keys).
size_t plan_estimate(const Graph& g) {
  int64_t units = g.w.n_packs[0] + g.w.n_packs[1];
  for (int c = CLS_WG_SMALL; c < NUM_CLASSES; ++c) units += g.w.n_items[c] / kWaves;
  return (size_t)512 + (size_t)units * (2 * sizeof(BatchUnit) + 4 * sizeof(uint32_t));
}

// Preprocessing workers by default: half the host's threads, 1 .. 8 (each
// worker spends much of its time waiting for its stream).
int default_prep_threads() {
  const unsigned hc = std::thread::hardware_concurrency();
  return (int)std::max(1u, std::min(8u, hc / 2));
}

struct Server {
  int device = 0;
  int64_t budget = 0;
  int max_slots = 1;
  int ticks_max = 1;  // ticks in flight (option "ticks": 1 or 2)
  int prep_threads = default_prep_threads();
  std::string tuning;  // batch schedule of every tick

  std::mutex mu;
  std::condition_variable cv_sched;  // work for the scheduler
  std::condition_variable cv_done;   // a request finished
  std::condition_variable cv_prep;   // work for the workers
  bool stop = false;

  int64_t next_ticket = 1;
  std::map<int64_t, std::unique_ptr<Req>> reqs;
  std::deque<Req*> pending;
  std::vector<Req*> active;  // admitted, not done
  std::deque<CacheEntry*> prep_jobs;
  std::list<std::unique_ptr<CacheEntry>> cache;  // every entry (building, resident)
  size_t reserved = 0, peak_reserved = 0;
  uint64_t use_clock = 0;
  std::vector<Graph*> graveyard;  // graphs to free outside the lock

  // statistics
  int64_t n_submitted = 0, n_done = 0, n_failed = 0, n_canceled = 0, n_hits = 0, n_evicted = 0;
  int64_t n_ticks = 0, tick_requests = 0, tick_units = 0, max_tick_requests = 0;

  Clock::time_point t0 = Clock::now();
  std::thread sched;
  std::vector<std::thread> workers;

  double now() const { return std::chrono::duration<double>(Clock::now() - t0).count(); }

  void reserve(size_t b) {
    reserved += b;
    peak_reserved = std::max(peak_reserved, reserved);
  }
  void unreserve(size_t b) { reserved -= std::min(reserved, b); }

  CacheEntry* find(uint64_t key) {
    if (key == 0) return nullptr;
    for (auto& e : cache)
      if (e->key == key && e->status == TC_OK) return e.get();
    return nullptr;
  }

  // Evict unused resident graphs (LRU) until `need` more bytes fit.
  bool make_room(size_t need, std::vector<Graph*>& to_free) {
    while (reserved + need > (size_t)budget) {
      CacheEntry* victim = nullptr;
      for (auto& e : cache)
        if (!e->building && e->refs == 0 && (!victim || e->last_use < victim->last_use)) victim = e.get();
      if (!victim) return false;
      unreserve(victim->bytes);
      to_free.push_back(victim->g);
      ++n_evicted;
      cache.remove_if([&](const std::unique_ptr<CacheEntry>& e) { return e.get() == victim; });
    }
    return true;
  }

  void finish(Req* q, tc_status st, const std::string& err) {
    q->res.status = st;
    q->err = err;
    q->res.t_done = now();
    q->state = Req::DONE;
    ++n_done;
    if (st != TC_OK) ++n_failed;
    cv_done.notify_all();
  }

  void release(Req* q) {
    unreserve(q->support_bytes + q->plan_bytes);
    q->support_bytes = 0;
    q->plan_bytes = 0;
    if (q->ce) {
      CacheEntry* e = q->ce;
      q->ce = nullptr;
      if (--e->refs == 0 && (e->key == 0 || e->status != TC_OK) && !e->building) {
        unreserve(e->bytes);
        if (e->g) graveyard.push_back(e->g);
        cache.remove_if([&](const std::unique_ptr<CacheEntry>& x) { return x.get() == e; });
      }
    }
    active.erase(std::remove(active.begin(), active.end(), q), active.end());
  }

  void admit_locked(std::vector<Graph*>& to_free) {
    while (!pending.empty() && (int)active.size() < max_slots) {
      Req* q = pending.front();
      CacheEntry* e = find(q->r.graph_key);
      const int64_t sup_entries = e && !e->building ? e->g->m : q->r.m_raw;
      const size_t sup = q->r.op == TC_REQ_COUNT ? 0 : (size_t)4 * (size_t)sup_entries;
      const size_t need = sup + (e ? 0 : prep_estimate(q->r.m_raw, q->r.n));
      if (!e && q->r.m_raw > 0 && (!q->r.src || !q->r.dst)) {
        pending.pop_front();
        finish(q, TC_EINVAL, "tc_server: graph_key not resident and no edge list given");
        continue;
      }
      if (reserved + need > (size_t)budget && !make_room(need, to_free)) {
        if (active.empty() && need > (size_t)budget) {
          pending.pop_front();
          finish(q, TC_ENOMEM, "tc_server: request footprint exceeds the HBM budget");
          continue;
        }
        break;  // wait for memory (arrival order is kept)
      }
      pending.pop_front();
      q->res.t_admit = now();
      q->support_bytes = sup;
      reserve(sup);
      if (e) {
        ++n_hits;
        q->res.cache_hit = 1;
        q->ce = e;
        e->refs++;
        e->last_use = ++use_clock;
        q->state = e->building ? Req::PREP : Req::READY;
        if (!e->building) q->res.t_ready = q->res.t_admit;
      } else {
        auto ne = std::make_unique<CacheEntry>();
        ne->key = q->r.graph_key;
        ne->est = prep_estimate(q->r.m_raw, q->r.n);
        ne->src = q->r.src;
        ne->dst = q->r.dst;
        ne->m_raw = q->r.m_raw;
        ne->n = q->r.n;
        ne->refs = 1;
        ne->last_use = ++use_clock;
        reserve(ne->est);
        q->ce = ne.get();
        q->state = Req::PREP;
        prep_jobs.push_back(ne.get());
        cache.push_back(std::move(ne));
        cv_prep.notify_one();
      }
      active.push_back(q);
    }
  }

  void worker_main() {
    (void)hipSetDevice(device);
    hipStream_t st = nullptr;
    if (hipStreamCreateWithFlags(&st, hipStreamNonBlocking) != hipSuccess) st = nullptr;
    for (;;) {
      CacheEntry* e = nullptr;
      {
        std::unique_lock<std::mutex> lk(mu);
        cv_prep.wait(lk, [&] { return stop || !prep_jobs.empty(); });
        if (prep_jobs.empty()) break;  // stopping
        e = prep_jobs.front();
        prep_jobs.pop_front();
      }
      Graph* g = nullptr;
      tc_status status = TC_OK;
      std::string err;
      int32_t* d_edges = nullptr;
      try {
        TC_REQUIRE(st != nullptr, TC_EDEVICE, "tc_server: worker stream");
        const size_t bytes = sizeof(int32_t) * (size_t)std::max<int64_t>(e->m_raw, 1);
        d_edges = static_cast<int32_t*>(cache_alloc(2 * bytes, st));
        if (e->m_raw > 0) {
          TC_HIP(hipMemcpyAsync(d_edges, e->src, bytes, hipMemcpyHostToDevice, st));
          TC_HIP(hipMemcpyAsync(d_edges + e->m_raw, e->dst, bytes, hipMemcpyHostToDevice, st));
        }
        g = build_graph(d_edges, d_edges + e->m_raw, e->m_raw, e->n, st);
      } catch (const Error& x) {
        status = x.status;
        err = x.what();
      } catch (const std::bad_alloc&) {
        status = TC_ENOMEM;
        err = "tc_server: host allocation failed";
      } catch (const std::exception& x) {
        status = TC_EDEVICE;
        err = x.what();
      }
      if (d_edges) {
        (void)hipStreamSynchronize(st);
        cache_free(d_edges, st, true);
      }
      std::lock_guard<std::mutex> lk(mu);
      e->building = false;
      unreserve(e->est);
      e->status = status;
      e->err = err;
      if (g) {
        e->g = g;
        e->bytes = g->arena_bytes;
        reserve(e->bytes);
      }
      const double t = now();
      for (Req* q : active) {
        if (q->ce != e || q->state != Req::PREP) continue;
        q->res.t_ready = t;
        if (status == TC_OK) {
          q->state = Req::READY;
        } else {
          finish(q, status, err);
        }
      }
      // failed requests release their entry (and with it the failed build)
      std::vector<Req*> failed;
      for (Req* q : active)
        if (q->state == Req::DONE) failed.push_back(q);
      for (Req* q : failed) release(q);
      cv_sched.notify_all();
    }
    if (st) {
      cache_retire_stream(st);
      (void)hipStreamDestroy(st);
    }
  }

  // Tick slots (ticks in flight at most), and the ready requests a tick
  // started beside a running one takes at least.
  static constexpr int kTickSlots = 2;
  static constexpr int kSecondTickMin = 2;

  // One tick: plans and launches over the ready requests, then (after the
  // event) results. Runs on the scheduler thread without holding the lock
  // except to read and publish request state.
  struct Tick {
    std::vector<Req*> reqs[3];
    BatchPlan* plans[3] = {nullptr, nullptr, nullptr};
    hipEvent_t ev = nullptr;
    bool running = false;
    int64_t* d_counts = nullptr;  // this slot's 3 * max_slots counts
    int64_t* h_counts = nullptr;  // (pinned)
  };

  hipStream_t tick_stream = nullptr;
  int64_t* d_counts = nullptr;   // kTickSlots * 3 * max_slots
  int64_t* h_counts = nullptr;   // pinned, kTickSlots * 3 * max_slots

  void start_tick(Tick& tk) {
    std::vector<Req*> ready;
    {
      // every ready request whose share of the tick's plans still fits the
      // budget (at least one, so that a tick always makes progress); the
      // others wait for the next tick
      std::lock_guard<std::mutex> lk(mu);
      for (Req* q : active) {
        if (q->state != Req::READY) continue;
        const size_t pb = plan_estimate(*q->ce->g);
        if (!ready.empty() && reserved + pb > (size_t)budget) continue;
        q->state = Req::RUNNING;
        q->plan_bytes = pb;
        reserve(pb);
        ready.push_back(q);
      }
    }
    if (ready.empty()) return;
    for (Req* q : ready) tk.reqs[q->r.op].push_back(q);
    int64_t units = 0;
    tc_status status = TC_OK;
    std::string err;
    try {
      for (int op = 0; op < 3; ++op) {
        auto& v = tk.reqs[op];
        if (v.empty()) continue;
        std::vector<PlanEntry> ents;
        for (Req* q : v) {
          int32_t* sup = nullptr;
          if (op != TC_REQ_COUNT && q->ce->g->m > 0) {
            q->d_support = static_cast<int32_t*>(cache_alloc(sizeof(int32_t) * (size_t)q->ce->g->m, tick_stream));
            sup = q->d_support;
          }
          ents.push_back(PlanEntry{q->ce->g, sup});
        }
        const CountMode mode = op == TC_REQ_COUNT         ? MODE_COUNT
                               : op == TC_REQ_SUPPORT_FULL ? MODE_SUPPORT_FULL
                                                           : MODE_SUPPORT_ORIENTED;
        tk.plans[op] = make_plan(ents.data(), (int64_t)ents.size(), mode, tuning.c_str(), tick_stream);
        plan_count(*tk.plans[op], tk.d_counts + (size_t)op * max_slots, tick_stream);
        units += plan_units(*tk.plans[op]);
      }
      TC_HIP(hipMemcpyAsync(tk.h_counts, tk.d_counts, sizeof(int64_t) * 3 * (size_t)max_slots,
                            hipMemcpyDeviceToHost, tick_stream));
      TC_HIP(hipEventRecord(tk.ev, tick_stream));
      tk.running = true;
    } catch (const Error& x) {
      status = x.status;
      err = x.what();
    } catch (const std::exception& x) {
      status = TC_EDEVICE;
      err = x.what();
    }
    std::lock_guard<std::mutex> lk(mu);
    ++n_ticks;
    tick_units += units;
    tick_requests += (int64_t)ready.size();
    max_tick_requests = std::max<int64_t>(max_tick_requests, (int64_t)ready.size());
    if (status != TC_OK) {
      (void)hipStreamSynchronize(tick_stream);
      end_tick_locked(tk, status, err);
    }
  }

  // Support arrays of a finished tick to the callers' host buffers. Runs on
  // the scheduler thread without the server lock: the tick's requests are
  // the scheduler's alone until it publishes them, and their graphs stay
  // resident while they hold a reference.
  void copy_tick_support(Tick& tk) {
    for (int op = 1; op < 3; ++op) {
      for (Req* q : tk.reqs[op]) {
        const int64_t m = q->ce->g->m;
        q->copy_status = TC_OK;
        if (m > q->r.m_raw) {
          q->copy_status = TC_EINVAL;
          q->copy_err = "tc_server: support_out (m_raw entries) is smaller than the graph's m";
        } else if (m > 0) {
          hipError_t he = hipMemcpy(q->r.support_out, q->d_support, sizeof(int32_t) * (size_t)m,
                                    hipMemcpyDeviceToHost);
          if (he != hipSuccess) {
            q->copy_status = TC_EDEVICE;
            q->copy_err = std::string("tc_server: support copy: ") + hipGetErrorString(he);
          }
        }
      }
    }
  }

  void end_tick_locked(Tick& tk, tc_status status, const std::string& err) {
    for (int op = 0; op < 3; ++op) {
      for (size_t i = 0; i < tk.reqs[op].size(); ++i) {
        Req* q = tk.reqs[op][i];
        tc_status s = status;
        std::string e = err;
        if (s == TC_OK) {
          q->res.count = tk.h_counts[(size_t)op * max_slots + i];
          q->res.m = q->ce->g->m;
          if (q->copy_status != TC_OK) {  // (copy_tick_support, before the lock)
            s = q->copy_status;
            e = q->copy_err;
          }
        }
        if (q->d_support) cache_free(q->d_support, tick_stream, status == TC_OK);
        q->d_support = nullptr;
        if (q->ce) q->ce->last_use = ++use_clock;
        finish(q, s, e);
        release(q);
      }
      tk.reqs[op].clear();
      if (tk.plans[op]) free_plan_idle(tk.plans[op]);
      tk.plans[op] = nullptr;
    }
    tk.running = false;
  }

  void sched_main() {
    (void)hipSetDevice(device);
    Tick tks[kTickSlots];
    for (int t = 0; t < kTickSlots; ++t) {
      if (hipEventCreateWithFlags(&tks[t].ev, hipEventDisableTiming) != hipSuccess) tks[t].ev = nullptr;
      tks[t].d_counts = d_counts + (size_t)t * 3 * max_slots;
      tks[t].h_counts = h_counts + (size_t)t * 3 * max_slots;
    }
    for (;;) {
      std::vector<Graph*> to_free;
      bool exit_now = false, any_running = false;
      int n_ready = 0;
      for (int t = 0; t < ticks_max; ++t) any_running |= tks[t].running;
      {
        std::unique_lock<std::mutex> lk(mu);
        admit_locked(to_free);
        to_free.insert(to_free.end(), graveyard.begin(), graveyard.end());
        graveyard.clear();
        for (Req* q : active) n_ready += q->state == Req::READY;
        exit_now = stop && active.empty() && prep_jobs.empty() && !any_running;
        if (!exit_now && n_ready == 0 && !any_running && to_free.empty())
          cv_sched.wait_for(lk, std::chrono::milliseconds(2));
      }
      for (Graph* g : to_free) destroy_graph_idle(g);  // no request and no tick uses them
      if (exit_now) break;
      // finished ticks first (in slot order; the tick stream ran them in order)
      bool progressed = false;
      for (int t = 0; t < ticks_max; ++t) {
        Tick& tk = tks[t];
        if (!tk.running) continue;
        hipError_t q = hipEventQuery(tk.ev);
        if (q == hipSuccess) {
          copy_tick_support(tk);  // (blocking copies, outside the lock)
          std::lock_guard<std::mutex> lk(mu);
          end_tick_locked(tk, TC_OK, "");
          progressed = true;
        } else if (q != hipErrorNotReady) {
          std::lock_guard<std::mutex> lk(mu);
          end_tick_locked(tk, TC_EDEVICE, std::string("tc_server: tick: ") + hipGetErrorString(q));
          progressed = true;
        }
      }
      // a tick when requests are ready and a slot is free; beside a running
      // tick only for at least kSecondTickMin ready requests (a lone request
      // waits to share the next tick, which keeps ticks batched)
      int running = 0;
      for (int t = 0; t < ticks_max; ++t) running += tks[t].running;
      if (n_ready > 0 && (running == 0 || n_ready >= kSecondTickMin)) {
        for (int t = 0; t < ticks_max; ++t) {
          if (tks[t].running) continue;
          start_tick(tks[t]);
          progressed = true;
          break;
        }
      }
      if (!progressed && any_running) std::this_thread::sleep_for(std::chrono::microseconds(50));
    }
    for (int t = 0; t < kTickSlots; ++t)
      if (tks[t].ev) (void)hipEventDestroy(tks[t].ev);
  }
};

}  // namespace
}  // namespace tc

struct tc_server {
  tc::Server* s;
};

namespace {

template <class F>
tc_status server_guard(F&& f) {
  try {
    f();
    tc::set_last_error("");
    return TC_OK;
  } catch (const tc::Error& e) {
    tc::set_last_error(e.what());
    return e.status;
  } catch (const std::bad_alloc&) {
    tc::set_last_error("tc_server: host allocation failed");
    return TC_ENOMEM;
  } catch (const std::exception& e) {
    tc::set_last_error(e.what());
    return TC_EDEVICE;
  }
}

// options: flat JSON with integer values only
void parse_options(const char* js, int& prep_threads, int& ticks, std::string& tuning) {
  // tick plans: plain launches (a new plan every tick), units in request
  // order unless "lpt": 1 (the LPT sort synchronises the tick stream)
  tuning = "{\"graph\": 0";
  if (!js) {
    tuning += ", \"order\": \"input\"}";
    return;
  }
  std::string s(js);
  auto get = [&](const char* key, int& out) {
    const std::string k = std::string("\"") + key + "\"";
    size_t p = s.find(k);
    if (p == std::string::npos) return false;
    p = s.find(':', p + k.size());
    TC_REQUIRE(p != std::string::npos, TC_EINVAL, std::string("tc_server options: ") + key);
    char* end = nullptr;
    long v = std::strtol(s.c_str() + p + 1, &end, 10);
    TC_REQUIRE(end != s.c_str() + p + 1, TC_EINVAL, std::string("tc_server options: ") + key + " not an integer");
    out = (int)v;
    return true;
  };
  int v = 0;
  if (get("prep_threads", v)) {
    TC_REQUIRE(v >= 1 && v <= 16, TC_EINVAL, "tc_server options: prep_threads outside [1, 16]");
    prep_threads = v;
  }
  if (get("lds_cap_log2", v)) {
    TC_REQUIRE(v >= 6 && v <= 14, TC_EINVAL, "tc_server options: lds_cap_log2 outside [6, 14]");
    tuning += ", \"lds_cap_log2\": " + std::to_string(v);
  }
  if (get("blocks_per_cu", v)) {
    TC_REQUIRE(v >= 0 && v <= 64, TC_EINVAL, "tc_server options: blocks_per_cu outside [0, 64]");
    tuning += ", \"blocks_per_cu\": " + std::to_string(v);
  }
  if (get("ticks", v)) {
    TC_REQUIRE(v >= 1 && v <= 2, TC_EINVAL, "tc_server options: ticks outside [1, 2]");
    ticks = v;
  }
  int lpt = 0;
  get("lpt", lpt);
  tuning += lpt ? ", \"order\": \"lpt\"}" : ", \"order\": \"input\"}";
}

}  // namespace

extern "C" {

tc_status tc_server_create(int64_t hbm_budget_bytes, int32_t max_slots, const char* options_json,
                           tc_server** out) {
  return server_guard([&] {
    TC_REQUIRE(out != nullptr, TC_EINVAL, "tc_server_create: out is NULL");
    *out = nullptr;
    TC_REQUIRE(hbm_budget_bytes > 0, TC_EINVAL, "tc_server_create: budget must be > 0");
    TC_REQUIRE(max_slots >= 1 && max_slots <= 65536, TC_EINVAL, "tc_server_create: max_slots outside [1, 65536]");
    std::unique_ptr<tc::Server> s(new tc::Server());
    s->budget = hbm_budget_bytes;
    s->max_slots = max_slots;
    parse_options(options_json, s->prep_threads, s->ticks_max, s->tuning);
    TC_HIP(hipGetDevice(&s->device));
    TC_HIP(hipStreamCreateWithFlags(&s->tick_stream, hipStreamNonBlocking));
    const size_t nc = (size_t)tc::Server::kTickSlots * 3 * (size_t)max_slots;  // counts of every tick slot
    TC_HIP(hipMalloc(&s->d_counts, sizeof(int64_t) * nc));
    TC_HIP(hipHostMalloc(reinterpret_cast<void**>(&s->h_counts), sizeof(int64_t) * nc, hipHostMallocDefault));
    tc::Server* sp = s.get();
    for (int i = 0; i < s->prep_threads; ++i) s->workers.emplace_back([sp] { sp->worker_main(); });
    s->sched = std::thread([sp] { sp->sched_main(); });
    *out = new tc_server{s.release()};
  });
}

tc_status tc_server_submit(tc_server* srv, const tc_request* req, int64_t* ticket) {
  return server_guard([&] {
    TC_REQUIRE(srv && srv->s && req && ticket, TC_EINVAL, "tc_server_submit: null argument");
    TC_REQUIRE(req->op >= TC_REQ_COUNT && req->op <= TC_REQ_SUPPORT_ORIENTED, TC_EINVAL,
               "tc_server_submit: unknown op");
    TC_REQUIRE(req->n >= 1 && req->m_raw >= 0, TC_EINVAL, "tc_server_submit: n < 1 or m_raw < 0");
    TC_REQUIRE(req->m_raw < (int64_t)0xFFFFFFFFLL, TC_EOVERFLOW, "tc_server_submit: m_raw >= 2^32 - 1");
    TC_REQUIRE(req->op == TC_REQ_COUNT || req->support_out != nullptr || req->m_raw == 0, TC_EINVAL,
               "tc_server_submit: support op without support_out");
    TC_REQUIRE(req->graph_key != 0 || req->m_raw == 0 || (req->src && req->dst), TC_EINVAL,
               "tc_server_submit: null edge list");
    tc::Server& s = *srv->s;
    auto q = std::make_unique<tc::Req>();
    q->r = *req;
    std::lock_guard<std::mutex> lk(s.mu);
    TC_REQUIRE(!s.stop, TC_EINVAL, "tc_server_submit: server is stopping");
    q->ticket = s.next_ticket++;
    q->res.t_submit = s.now();
    *ticket = q->ticket;
    s.pending.push_back(q.get());
    s.reqs[q->ticket] = std::move(q);
    ++s.n_submitted;
    s.cv_sched.notify_all();
  });
}

tc_status tc_server_poll(tc_server* srv, int64_t ticket, int32_t wait, tc_result* out) {
  if (!srv || !srv->s || !out) {
    tc::set_last_error("tc_server_poll: null argument");
    return TC_EINVAL;
  }
  tc::Server& s = *srv->s;
  std::unique_lock<std::mutex> lk(s.mu);
  auto it = s.reqs.find(ticket);
  if (it == s.reqs.end()) {
    tc::set_last_error("tc_server_poll: unknown ticket");
    return TC_EINVAL;
  }
  tc::Req* q = it->second.get();
  if (q->state != tc::Req::DONE) {
    if (!wait) return TC_EBUSY;
    s.cv_done.wait(lk, [&] { return q->state == tc::Req::DONE; });
  }
  *out = q->res;
  tc::set_last_error(q->err);
  s.reqs.erase(it);
  return TC_OK;
}

tc_status tc_server_cancel(tc_server* srv, int64_t ticket) {
  if (!srv || !srv->s) {
    tc::set_last_error("tc_server_cancel: null server");
    return TC_EINVAL;
  }
  tc::Server& s = *srv->s;
  std::lock_guard<std::mutex> lk(s.mu);
  auto it = s.reqs.find(ticket);
  if (it == s.reqs.end()) {
    tc::set_last_error("tc_server_cancel: unknown ticket");
    return TC_EINVAL;
  }
  tc::Req* q = it->second.get();
  if (q->state == tc::Req::DONE) return TC_OK;
  if (q->state != tc::Req::PENDING) return TC_EBUSY;
  s.pending.erase(std::remove(s.pending.begin(), s.pending.end(), q), s.pending.end());
  ++s.n_canceled;
  s.finish(q, TC_ECANCELED, "tc_server: cancelled");
  return TC_OK;
}

tc_status tc_server_stats(tc_server* srv, char* out, size_t cap) {
  return server_guard([&] {
    TC_REQUIRE(srv && srv->s && out, TC_EINVAL, "tc_server_stats: null argument");
    tc::Server& s = *srv->s;
    std::lock_guard<std::mutex> lk(s.mu);
    char buf[768];
    size_t resident = 0;
    int64_t cached = 0;
    for (auto& e : s.cache)
      if (!e->building && e->g) {
        resident += e->bytes;
        ++cached;
      }
    std::snprintf(buf, sizeof(buf),
                  "{\"submitted\": %lld, \"done\": %lld, \"failed\": %lld, \"canceled\": %lld, "
                  "\"cache_hits\": %lld, \"evicted\": %lld, \"cached_graphs\": %lld, \"resident_bytes\": %zu, "
                  "\"reserved_bytes\": %zu, \"peak_reserved_bytes\": %zu, \"budget_bytes\": %lld, "
                  "\"ticks\": %lld, \"tick_requests\": %lld, \"max_tick_requests\": %lld, \"tick_units\": %lld, "
                  "\"pending\": %zu, \"active\": %zu, \"prep_threads\": %d, \"max_slots\": %d, \"tick_slots\": %d}",
                  (long long)s.n_submitted, (long long)s.n_done, (long long)s.n_failed, (long long)s.n_canceled,
                  (long long)s.n_hits, (long long)s.n_evicted, (long long)cached, resident, s.reserved,
                  s.peak_reserved, (long long)s.budget, (long long)s.n_ticks, (long long)s.tick_requests,
                  (long long)s.max_tick_requests, (long long)s.tick_units, s.pending.size(), s.active.size(),
                  s.prep_threads, s.max_slots, s.ticks_max);
    TC_REQUIRE(cap > std::strlen(buf), TC_EINVAL, "tc_server_stats: buffer too small");
    std::memcpy(out, buf, std::strlen(buf) + 1);
  });
}

void tc_server_destroy(tc_server* srv) {
  if (!srv) return;
  tc::Server* s = srv->s;
  if (s) {
    {
      std::lock_guard<std::mutex> lk(s->mu);
      for (tc::Req* q : s->pending) {
        ++s->n_canceled;
        s->finish(q, TC_ECANCELED, "tc_server: destroyed");
      }
      s->pending.clear();
      s->stop = true;
      s->cv_sched.notify_all();
      s->cv_prep.notify_all();
    }
    if (s->sched.joinable()) s->sched.join();
    {
      std::lock_guard<std::mutex> lk(s->mu);
      s->cv_prep.notify_all();
    }
    for (auto& t : s->workers)
      if (t.joinable()) t.join();
    (void)hipDeviceSynchronize();
    for (auto& e : s->cache)
      if (e->g) tc::destroy_graph_idle(e->g);
    s->cache.clear();
    if (s->tick_stream) {
      tc::cache_retire_stream(s->tick_stream);
      (void)hipStreamDestroy(s->tick_stream);
    }
    if (s->d_counts) (void)hipFree(s->d_counts);
    if (s->h_counts) (void)hipHostFree(s->h_counts);
    delete s;
  }
  delete srv;
}

}  // extern "C"
