// tc_timer.cpp - phase timers: HIP events around every library launch made
// while a timer is attached to the calling host thread.
#include <cstdlib>
#include <map>
#include <mutex>
#include <set>
#include <sstream>
#include <string>
#include <vector>

#include "tc_prims.h"

struct tc_timer {
  std::vector<hipEvent_t> ev;       // 2 per slot
  std::vector<const char*> names;   // per slot (static strings)
  int used = 0;
  int64_t dropped = 0;
  std::mutex mu;
};

namespace tc {

static thread_local tc_timer* t_active = nullptr;

const char* intern_name(const std::string& s) {
  static std::mutex mu;
  static std::set<std::string> names;
  std::lock_guard<std::mutex> lk(mu);
  return names.insert(s).first->c_str();
}

bool sort_wide_words_forced() {
  const char* v = std::getenv("TC_SORT_WIDE_WORDS");
  return v != nullptr && v[0] != '\0' && !(v[0] == '0' && v[1] == '\0');
}

TempCtx& temp_ctx() {
  static thread_local TempCtx c;
  return c;
}

TempStream::TempStream(hipStream_t st) : prev(temp_ctx()) {
  fail_word = cache_alloc(sizeof(int), st);
  TC_HIP(hipMemsetAsync(fail_word, 0, sizeof(int), st));
  temp_ctx().active = true;
  temp_ctx().st = st;
  temp_ctx().fail = static_cast<int*>(fail_word);
}

TempStream::~TempStream() {
  cache_free(fail_word, temp_ctx().st, false);
  temp_ctx() = prev;
}

LaunchScope::LaunchScope(const char* name, hipStream_t s) : st(s) {
  tc_timer* t = t_active;
  if (!t) return;
  std::lock_guard<std::mutex> lk(t->mu);
  if (t->used >= (int)t->names.size()) {
    ++t->dropped;
    return;
  }
  slot = t->used++;
  t->names[slot] = name;
  timer = t;
  (void)hipEventRecord(t->ev[2 * slot], st);
}

LaunchScope::~LaunchScope() {
  if (slot < 0) return;
  tc_timer* t = static_cast<tc_timer*>(timer);
  (void)hipEventRecord(t->ev[2 * slot + 1], st);
}

}  // namespace tc

extern "C" {

tc_status tc_timer_create(int32_t capacity, tc_timer** out) {
  if (!out || capacity < 1) {
    tc::set_last_error("tc_timer_create: bad argument");
    return TC_EINVAL;
  }
  *out = nullptr;
  tc_timer* t = new (std::nothrow) tc_timer();
  if (!t) return TC_ENOMEM;
  t->ev.resize(2 * (size_t)capacity, nullptr);
  t->names.resize((size_t)capacity, nullptr);
  for (auto& e : t->ev) {
    if (hipEventCreate(&e) != hipSuccess) {
      for (auto& x : t->ev)
        if (x) (void)hipEventDestroy(x);
      delete t;
      tc::set_last_error("tc_timer_create: hipEventCreate failed");
      return TC_EDEVICE;
    }
  }
  *out = t;
  return TC_OK;
}

tc_status tc_timer_attach(tc_timer* t) {
  tc::t_active = t;
  return TC_OK;
}

tc_status tc_timer_reset(tc_timer* t) {
  if (!t) return TC_EINVAL;
  std::lock_guard<std::mutex> lk(t->mu);
  for (int i = 0; i < 2 * t->used; ++i) (void)hipEventSynchronize(t->ev[i]);
  t->used = 0;
  t->dropped = 0;
  return TC_OK;
}

tc_status tc_timer_summary(tc_timer* t, char* buf, int64_t buf_bytes) {
  if (!t || !buf || buf_bytes < 2) {
    tc::set_last_error("tc_timer_summary: bad argument");
    return TC_EINVAL;
  }
  std::lock_guard<std::mutex> lk(t->mu);
  struct Acc {
    int64_t n = 0;
    double tot = 0, mn = 1e300, mx = 0;
  };
  std::map<std::string, Acc> acc;
  for (int i = 0; i < t->used; ++i) {
    if (hipEventSynchronize(t->ev[2 * i + 1]) != hipSuccess) {
      tc::set_last_error("tc_timer_summary: hipEventSynchronize failed");
      return TC_EDEVICE;
    }
    float ms = 0.f;
    if (hipEventElapsedTime(&ms, t->ev[2 * i], t->ev[2 * i + 1]) != hipSuccess) continue;
    Acc& a = acc[t->names[i]];
    a.n += 1;
    a.tot += ms;
    a.mn = ms < a.mn ? ms : a.mn;
    a.mx = ms > a.mx ? ms : a.mx;
  }
  std::ostringstream os;
  os.precision(9);
  os << "{";
  for (auto& kv : acc) {
    const Acc& a = kv.second;
    os << "\"" << kv.first << "\": {\"launches\": " << a.n << ", \"total_ms\": " << a.tot
       << ", \"avg_ms\": " << a.tot / (double)a.n << ", \"min_ms\": " << a.mn << ", \"max_ms\": " << a.mx
       << "}, ";
  }
  os << "\"_dropped\": " << t->dropped << "}";
  const std::string out = os.str();
  if ((int64_t)out.size() + 1 > buf_bytes) {
    tc::set_last_error("tc_timer_summary: buffer too small");
    return TC_EINVAL;
  }
  std::copy(out.begin(), out.end(), buf);
  buf[out.size()] = '\0';
  return TC_OK;
}

void tc_timer_free(tc_timer* t) {
  if (!t) return;
  if (tc::t_active == t) tc::t_active = nullptr;
  for (auto& e : t->ev)
    if (e) (void)hipEventDestroy(e);
  delete t;
}

}  // extern "C"
