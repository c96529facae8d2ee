// tc_alloc.cpp - caching device allocator for the library's temporaries and
// graph arrays.
//
// hipFree (and hipFreeAsync of large blocks) can block the host for
// milliseconds, and every preprocessing call allocates and frees several GB
// of temporaries. Freed blocks are therefore kept per device and handed out
// again: a block is reused for a request of at least 4/5 of its size (sizes
// are rounded up to 2 MiB above 1 MiB, to powers of two below). When a block
// is freed, an event is recorded on the stream of its last use; reusing it on
// another stream first makes that stream wait for the event, on the same
// stream ordering is implicit. Among the cached blocks that fit, one last
// used on the requesting stream (or idle) is taken first: with several
// streams allocating at once (concurrent preprocessing), taking the oldest
// block of a size would make nearly every reuse wait for another stream's
// work and chain the streams into one. The HIP calls of a reuse or a free
// (event record, stream wait) run outside the cache's lock. Cached free
// bytes are bounded (a quarter of the device's memory by default); beyond
// that, and whenever hipMalloc runs out of memory, cached blocks are
// released (after their events complete).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <map>
#include <mutex>
#include <unordered_map>
#include <vector>

#include "tc_internal.h"

namespace tc {
namespace {

struct Block {
  void* p = nullptr;
  size_t size = 0;
  hipStream_t st = nullptr;
  hipEvent_t ev = nullptr;  // null: no work pending on the block
};

struct DeviceCache {
  std::multimap<size_t, Block> free;         // by size
  std::unordered_map<void*, size_t> live;    // handed-out blocks
  std::vector<hipEvent_t> events;            // recycled events
  size_t cached = 0, cap = 0, in_use = 0, peak = 0;
};

std::mutex g_mu;
std::map<int, DeviceCache> g_dev;

size_t round_size(size_t b) {
  if (b <= ((size_t)1 << 20)) {
    size_t r = 512;
    while (r < b) r <<= 1;
    return r;
  }
  const size_t g = (size_t)2 << 20;
  return (b + g - 1) / g * g;
}

DeviceCache& cache_for(int dev) {
  DeviceCache& c = g_dev[dev];
  if (c.cap == 0) {
    size_t fr = 0, tot = 0;
    c.cap = hipMemGetInfo(&fr, &tot) == hipSuccess ? tot / 4 : ((size_t)16 << 30);
  }
  return c;
}

// Release cached blocks until at most `keep` bytes stay cached. Called with
// g_mu held. Blocks with pending work are waited for by one device
// synchronisation (not through their events: the stream an event was
// recorded on may have been destroyed since).
void trim_locked(DeviceCache& c, size_t keep) {
  bool synced = false;
  while (c.cached > keep && !c.free.empty()) {
    auto it = std::prev(c.free.end());  // largest first
    Block b = it->second;
    c.free.erase(it);
    c.cached -= b.size;
    if (b.ev) {
      if (!synced) (void)hipDeviceSynchronize();
      synced = true;
      c.events.push_back(b.ev);
    }
    (void)hipFree(b.p);
  }
}

}  // namespace

// Cached blocks of one size looked at for one last used on the requesting
// stream before the smallest fitting one is taken.
constexpr int kReuseScan = 32;

void* cache_alloc(size_t bytes, hipStream_t st) {
  int dev = 0;
  TC_HIP(hipGetDevice(&dev));
  const size_t rb = round_size(bytes ? bytes : 1);
  Block b;
  {
    std::lock_guard<std::mutex> lk(g_mu);
    DeviceCache& c = cache_for(dev);
    const auto lo = c.free.lower_bound(rb);
    const auto hi = c.free.upper_bound(rb + rb / 4);
    auto pick = lo;
    int looked = 0;
    for (auto it = lo; it != hi && looked < kReuseScan; ++it, ++looked) {
      if (!it->second.ev || it->second.st == st) {
        pick = it;
        break;
      }
    }
    if (pick != hi) {
      b = pick->second;
      c.free.erase(pick);
      c.cached -= b.size;
      c.live[b.p] = b.size;
      c.in_use += b.size;
      c.peak = std::max(c.peak, c.in_use);
    }
  }
  if (b.p) {
    hipError_t e = hipSuccess;
    if (b.ev && b.st != st) e = hipStreamWaitEvent(st, b.ev, 0);
    std::lock_guard<std::mutex> lk(g_mu);
    DeviceCache& c = cache_for(dev);
    if (e != hipSuccess) {
      // back to the cache as it was
      c.live.erase(b.p);
      c.in_use -= b.size;
      c.free.emplace(b.size, b);
      c.cached += b.size;
      throw Error(TC_EDEVICE, std::string("hipStreamWaitEvent: ") + hipGetErrorString(e));
    }
    if (b.ev) c.events.push_back(b.ev);  // the wait (if any) is queued: the event is free again
    return b.p;
  }
  void* p = nullptr;
  hipError_t e = hipMalloc(&p, rb);
  if (e == hipErrorOutOfMemory) {
    (void)hipGetLastError();
    std::lock_guard<std::mutex> lk(g_mu);
    trim_locked(cache_for(dev), 0);
    e = hipMalloc(&p, rb);
  }
  if (e != hipSuccess) {
    (void)hipGetLastError();
    throw Error(e == hipErrorOutOfMemory ? TC_ENOMEM : TC_EDEVICE,
                std::string("hipMalloc(") + std::to_string(rb) + "): " + hipGetErrorString(e));
  }
  std::lock_guard<std::mutex> lk(g_mu);
  DeviceCache& c = cache_for(dev);
  c.live[p] = rb;
  c.in_use += rb;
  c.peak = std::max(c.peak, c.in_use);
  return p;
}

void cache_free(void* p, hipStream_t st, bool idle) {
  if (!p) return;
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return;
  Block b;
  b.p = p;
  b.st = st;
  {
    std::lock_guard<std::mutex> lk(g_mu);
    DeviceCache& c = cache_for(dev);
    auto it = c.live.find(p);
    if (it == c.live.end()) return;  // not ours
    b.size = it->second;
    c.live.erase(it);
    c.in_use -= b.size;
    if (!idle && !c.events.empty()) {
      b.ev = c.events.back();
      c.events.pop_back();
    }
  }
  // (the block is in neither map meanwhile: nobody else can hand it out)
  if (!idle) {
    if (!b.ev && hipEventCreateWithFlags(&b.ev, hipEventDisableTiming) != hipSuccess) b.ev = nullptr;
    if (b.ev && hipEventRecord(b.ev, st) != hipSuccess) {
      std::lock_guard<std::mutex> lk(g_mu);
      cache_for(dev).events.push_back(b.ev);
      b.ev = nullptr;
    }
    if (!b.ev) (void)hipStreamSynchronize(st);  // could not record: make the block idle
  }
  std::lock_guard<std::mutex> lk(g_mu);
  DeviceCache& c = cache_for(dev);
  c.free.emplace(b.size, b);
  c.cached += b.size;
  if (c.cached > c.cap) trim_locked(c, c.cap / 2);
}

// ---- use logs -----------------------------------------------------------------

namespace {
// A library stream per device on which freed memory waits for the events of
// its users (never destroyed; default priority).
hipStream_t release_stream() {
  static std::mutex mu;
  static std::map<int, hipStream_t> streams;
  int dev = 0;
  TC_HIP(hipGetDevice(&dev));
  std::lock_guard<std::mutex> lk(mu);
  hipStream_t& st = streams[dev];
  if (!st) TC_HIP(hipStreamCreateWithFlags(&st, hipStreamNonBlocking));
  return st;
}
}  // namespace

UseLog::~UseLog() {
  for (auto& u : uses) (void)hipEventDestroy(u.second);
}

void UseLog::note(hipStream_t st) {
  hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
  TC_HIP(hipStreamIsCapturing(st, &cs));
  std::lock_guard<std::mutex> lk(mu);
  if (cs != hipStreamCaptureStatusNone) {
    captured = true;  // the use happens when the caller launches its graph
    return;
  }
  for (auto& u : uses) {
    if (u.first == st) {
      TC_HIP(hipEventRecord(u.second, st));
      return;
    }
  }
  hipEvent_t ev = nullptr;
  TC_HIP(hipEventCreateWithFlags(&ev, hipEventDisableTiming));
  hipError_t e = hipEventRecord(ev, st);
  if (e != hipSuccess) {
    (void)hipEventDestroy(ev);
    throw Error(TC_EDEVICE, std::string("hipEventRecord: ") + hipGetErrorString(e));
  }
  uses.emplace_back(st, ev);
}

void UseLog::wait_host() {
  std::lock_guard<std::mutex> lk(mu);
  if (captured) {
    (void)hipDeviceSynchronize();
    return;
  }
  for (auto& u : uses) (void)hipEventSynchronize(u.second);
}

void UseLog::release_after_uses(Owned& owned) {
  std::lock_guard<std::mutex> lk(mu);
  if (captured) {
    (void)hipDeviceSynchronize();
    owned.release(true);
    return;
  }
  hipStream_t rel = nullptr;
  try {
    rel = release_stream();
    for (auto& u : uses) TC_HIP(hipStreamWaitEvent(rel, u.second, 0));
  } catch (const Error&) {
    (void)hipDeviceSynchronize();  // cannot order the release: wait for everything
    owned.release(true);
    return;
  }
  owned.st = rel;
  owned.release(false);  // each block's event is recorded on rel, after the waits
}

void cache_retire_stream(hipStream_t st) {
  if (!st) return;
  (void)hipStreamSynchronize(st);
  std::lock_guard<std::mutex> lk(g_mu);
  for (auto& kv : g_dev) {
    DeviceCache& c = kv.second;
    for (auto& fb : c.free) {
      Block& b = fb.second;
      if (b.st != st) continue;
      if (b.ev) c.events.push_back(b.ev);  // its record has completed: the event is free again
      b.ev = nullptr;
      b.st = nullptr;
    }
  }
}

void cache_release_all() {
  std::lock_guard<std::mutex> lk(g_mu);
  int cur = 0;
  (void)hipGetDevice(&cur);
  for (auto& kv : g_dev) {
    (void)hipSetDevice(kv.first);
    trim_locked(kv.second, 0);
  }
  (void)hipSetDevice(cur);
}

void cache_stats(int64_t* in_use, int64_t* cached, int64_t* peak) {
  int dev = 0;
  (void)hipGetDevice(&dev);
  std::lock_guard<std::mutex> lk(g_mu);
  DeviceCache& c = cache_for(dev);
  if (in_use) *in_use = (int64_t)c.in_use;
  if (cached) *cached = (int64_t)c.cached;
  if (peak) *peak = (int64_t)c.peak;
}

}  // namespace tc

extern "C" {

void tc_release_cached_memory(void) { tc::cache_release_all(); }

tc_status tc_memory_stats(int64_t* in_use_bytes, int64_t* cached_bytes, int64_t* peak_bytes) {
  try {
    tc::cache_stats(in_use_bytes, cached_bytes, peak_bytes);
    return TC_OK;
  } catch (...) {
    return TC_EDEVICE;
  }
}

}  // extern "C"
