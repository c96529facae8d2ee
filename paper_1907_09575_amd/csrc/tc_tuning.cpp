// tc_tuning.cpp - the tuning table (tuned row-bucket thresholds and batch
// schedules, persisted as JSON), retuned graph handles and the single-graph
// threshold autotuner.
//
// The table maps "<arch>/<CUs>cu/<kind>_e<k>" to a flat JSON object: kind
// "graph" holds the thresholds tc_preprocess uses for graphs of about 2^k
// edges, kind "batch" a tc_batch_create schedule (and thresholds) for batches
// of about 2^k edges in total. A lookup takes the entry of the same device
// tag and kind whose k is nearest (at most two classes away). The file form
// is one JSON object of such entries; TC_TUNING_FILE names a file read at the
// first lookup.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cctype>
#include <cstdlib>
#include <cstring>
#include <fstream>
#include <memory>
#include <sstream>
#include <vector>

#include "tc_internal.h"

namespace tc {

std::map<std::string, std::string> parse_flat_json(const char* js) {
  std::map<std::string, std::string> kv;
  const char* p = js;
  auto ws = [&] { while (*p && std::isspace((unsigned char)*p)) ++p; };
  auto fail = [&](const char* what) {
    throw Error(TC_EINVAL, std::string("tuning json: ") + what + " near '" + std::string(p).substr(0, 20) + "'");
  };
  auto str = [&]() {
    if (*p != '"') fail("expected a string");
    ++p;
    std::string s;
    while (*p && *p != '"') s += *p++;
    if (*p != '"') fail("unterminated string");
    ++p;
    return s;
  };
  ws();
  if (*p != '{') fail("expected '{'");
  ++p;
  ws();
  if (*p == '}') return kv;
  while (true) {
    ws();
    std::string k = str();
    ws();
    if (*p != ':') fail("expected ':'");
    ++p;
    ws();
    std::string v;
    if (*p == '"') {
      v = str();
    } else {
      while (*p && (std::isalnum((unsigned char)*p) || *p == '-' || *p == '+' || *p == '.')) v += *p++;
      if (v.empty()) fail("expected a value");
    }
    kv[k] = v;
    ws();
    if (*p == ',') {
      ++p;
      continue;
    }
    if (*p == '}') break;
    fail("expected ',' or '}'");
  }
  ++p;
  ws();
  if (*p) fail("text after the object");
  return kv;
}

namespace {

int64_t to_i64(const std::string& k, const std::string& v, int64_t lo, int64_t hi) {
  char* end = nullptr;
  const long long x = std::strtoll(v.c_str(), &end, 10);
  TC_REQUIRE(!v.empty() && end && *end == '\0', TC_EINVAL, "tuning json: " + k + " must be an integer");
  TC_REQUIRE(x >= lo && x <= hi, TC_EINVAL,
             "tuning json: " + k + " outside [" + std::to_string(lo) + ", " + std::to_string(hi) + "]");
  return (int64_t)x;
}

}  // namespace

bool parse_work_key(const std::string& k, const std::string& v, WorkParams& wp) {
  if (k == "heavy_min") {
    wp.heavy_min = (uint64_t)to_i64(k, v, 0, (int64_t)kHeavyMinMax);
  } else if (k == "pack_target") {
    wp.pack_target = (uint64_t)to_i64(k, v, (int64_t)kPackTargetMin, (int64_t)kPackTargetMax);
  } else if (k == "pack_slots") {
    wp.pack_slots = (uint32_t)to_i64(k, v, kPackSlotsMin, kPackSlotsMax);
  } else if (k == "wave_chunk") {
    wp.wave_chunk = (uint32_t)to_i64(k, v, kWaveChunkMin, kWaveChunkMax);
  } else if (k == "min_groups") {
    wp.min_groups = (uint32_t)to_i64(k, v, 0, kMinGroupsMax);
  } else {
    return false;
  }
  return true;
}

std::string work_params_json(const WorkParams& wp) {
  char buf[224];
  std::snprintf(buf, sizeof(buf),
                "\"heavy_min\": %llu, \"pack_target\": %llu, \"pack_slots\": %u, \"wave_chunk\": %u, "
                "\"min_groups\": %u",
                (unsigned long long)wp.heavy_min, (unsigned long long)wp.pack_target, wp.pack_slots,
                wp.wave_chunk, wp.min_groups);
  return buf;
}

namespace {

std::mutex g_tmu;
std::map<std::string, std::string> g_table;
bool g_env_read = false;

// An entry must parse, and the thresholds it names must be in range (so that
// a bad table fails where it is set or loaded, not in a later tc_preprocess).
void check_entry(const std::string& json) {
  WorkParams wp;
  for (const auto& kv : parse_flat_json(json.c_str())) (void)parse_work_key(kv.first, kv.second, wp);
}

// Entries of a file: one object whose values are flat objects. Each value is
// kept as its text after checking it (check_entry).
std::map<std::string, std::string> parse_table(const std::string& text) {
  std::map<std::string, std::string> out;
  size_t i = 0;
  auto ws = [&] { while (i < text.size() && std::isspace((unsigned char)text[i])) ++i; };
  auto fail = [&](const char* what) {
    throw Error(TC_EINVAL, std::string("tuning file: ") + what + " at offset " + std::to_string(i));
  };
  ws();
  if (i >= text.size() || text[i] != '{') fail("expected '{'");
  ++i;
  ws();
  if (i < text.size() && text[i] == '}') return out;
  while (true) {
    ws();
    if (i >= text.size() || text[i] != '"') fail("expected a key");
    const size_t k0 = ++i;
    while (i < text.size() && text[i] != '"') ++i;
    if (i >= text.size()) fail("unterminated key");
    const std::string key = text.substr(k0, i - k0);
    ++i;
    ws();
    if (i >= text.size() || text[i] != ':') fail("expected ':'");
    ++i;
    ws();
    if (i >= text.size() || text[i] != '{') fail("expected an object");
    const size_t v0 = i;
    while (i < text.size() && text[i] != '}') ++i;  // flat objects: the first '}' closes it
    if (i >= text.size()) fail("unterminated object");
    ++i;
    const std::string val = text.substr(v0, i - v0);
    check_entry(val);
    out[key] = val;
    ws();
    if (i < text.size() && text[i] == ',') {
      ++i;
      continue;
    }
    if (i < text.size() && text[i] == '}') break;
    fail("expected ',' or '}'");
  }
  return out;
}

void load_file_locked(const char* path) {
  std::ifstream f(path, std::ios::binary);
  TC_REQUIRE(f.good(), TC_EINVAL, std::string("tuning file: cannot read ") + path);
  std::stringstream ss;
  ss << f.rdbuf();
  for (auto& kv : parse_table(ss.str())) g_table[kv.first] = kv.second;
}

void read_env_locked() {
  if (g_env_read) return;
  g_env_read = true;
  const char* path = std::getenv("TC_TUNING_FILE");
  if (path && *path) load_file_locked(path);
}

int size_class(int64_t edges) {
  int k = 0;
  while (k < 62 && ((int64_t)1 << (k + 1)) <= edges) ++k;
  return k;
}

std::string device_tag() {
  int dev = 0;
  TC_HIP(hipGetDevice(&dev));
  hipDeviceProp_t prop;
  TC_HIP(hipGetDeviceProperties(&prop, dev));
  std::string arch(prop.gcnArchName);
  const size_t colon = arch.find(':');
  if (colon != std::string::npos) arch.resize(colon);
  return arch + "/" + std::to_string(prop.multiProcessorCount) + "cu";
}

}  // namespace

std::string tuning_key(const char* kind, int64_t edges) {
  return device_tag() + "/" + kind + "_e" + std::to_string(size_class(edges));
}

std::string tuning_lookup(const std::string& key) {
  std::lock_guard<std::mutex> lk(g_tmu);
  read_env_locked();
  auto it = g_table.find(key);
  if (it != g_table.end()) return it->second;
  const size_t e = key.rfind("_e");
  if (e == std::string::npos) return "";
  const std::string prefix = key.substr(0, e + 2);
  const int k = std::atoi(key.c_str() + e + 2);
  std::string best;
  int best_d = 3, best_k = 0;
  for (const auto& kv : g_table) {
    if (kv.first.compare(0, prefix.size(), prefix) != 0) continue;
    const std::string rest = kv.first.substr(prefix.size());
    if (rest.empty() || rest.size() > 2 || rest.find_first_not_of("0123456789") != std::string::npos) continue;
    const int kk = std::atoi(rest.c_str());
    const int d = std::abs(kk - k);
    if (d < best_d || (d == best_d && kk < best_k)) {  // ties: the smaller class
      best_d = d;
      best_k = kk;
      best = kv.second;
    }
  }
  return best;
}

void tuning_store(const std::string& key, const std::string& json) {
  check_entry(json);
  std::lock_guard<std::mutex> lk(g_tmu);
  read_env_locked();
  g_table[key] = json;
}

WorkParams default_work_params(int64_t m) {
  WorkParams wp;
  const std::string js = tuning_lookup(tuning_key("graph", m));
  if (js.empty()) return wp;
  for (const auto& kv : parse_flat_json(js.c_str())) (void)parse_work_key(kv.first, kv.second, wp);
  return wp;
}

namespace {

template <class F>
tc_status guarded(const char* where, F&& f) {
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

void copy_text(const std::string& s, char* out, size_t cap) {
  TC_REQUIRE(out != nullptr && cap > s.size(), TC_EINVAL, "output buffer too small for the text");
  std::memcpy(out, s.c_str(), s.size() + 1);
}

// Thresholds named by a flat JSON object (other keys: TC_EINVAL), starting
// from `wp`.
WorkParams parse_thresholds(const char* js, WorkParams wp, const char* where) {
  if (!js || !*js) return wp;
  for (const auto& kv : parse_flat_json(js)) {
    if (parse_work_key(kv.first, kv.second, wp)) continue;
    if (kv.first == "ms") continue;  // descriptive key of the autotuner's output
    throw Error(TC_EINVAL, std::string(where) + ": unknown key \"" + kv.first + "\"");
  }
  return wp;
}

}  // namespace

}  // namespace tc

extern "C" {

tc_status tc_tuning_load(const char* path) {
  return tc::guarded("tc_tuning_load", [&] {
    TC_REQUIRE(path != nullptr, TC_EINVAL, "tc_tuning_load: null path");
    std::lock_guard<std::mutex> lk(tc::g_tmu);
    tc::read_env_locked();
    tc::load_file_locked(path);
  });
}

tc_status tc_tuning_save(const char* path) {
  return tc::guarded("tc_tuning_save", [&] {
    TC_REQUIRE(path != nullptr, TC_EINVAL, "tc_tuning_save: null path");
    std::string text = "{\n";
    {
      std::lock_guard<std::mutex> lk(tc::g_tmu);
      tc::read_env_locked();
      bool first = true;
      for (const auto& kv : tc::g_table) {
        text += (first ? "  \"" : ",\n  \"") + kv.first + "\": " + kv.second;
        first = false;
      }
    }
    text += "\n}\n";
    const std::string tmp = std::string(path) + ".tmp";
    {
      std::ofstream f(tmp, std::ios::binary | std::ios::trunc);
      TC_REQUIRE(f.good(), TC_EINVAL, std::string("tc_tuning_save: cannot write ") + tmp);
      f << text;
      f.flush();
      TC_REQUIRE(f.good(), TC_EINVAL, std::string("tc_tuning_save: write failed: ") + tmp);
    }
    TC_REQUIRE(std::rename(tmp.c_str(), path) == 0, TC_EINVAL, std::string("tc_tuning_save: cannot rename to ") + path);
  });
}

tc_status tc_tuning_get(const char* key, char* out, size_t cap) {
  return tc::guarded("tc_tuning_get", [&] {
    TC_REQUIRE(key != nullptr, TC_EINVAL, "tc_tuning_get: null key");
    tc::copy_text(tc::tuning_lookup(key), out, cap);
  });
}

tc_status tc_tuning_set(const char* key, const char* json) {
  return tc::guarded("tc_tuning_set", [&] {
    TC_REQUIRE(key != nullptr && *key, TC_EINVAL, "tc_tuning_set: empty key");
    if (!json) {
      std::lock_guard<std::mutex> lk(tc::g_tmu);
      tc::read_env_locked();
      tc::g_table.erase(key);
      return;
    }
    tc::tuning_store(key, json);
  });
}

tc_status tc_tuning_key(const char* kind, int64_t edges, char* out, size_t cap) {
  return tc::guarded("tc_tuning_key", [&] {
    TC_REQUIRE(kind != nullptr && (std::strcmp(kind, "graph") == 0 || std::strcmp(kind, "batch") == 0), TC_EINVAL,
               "tc_tuning_key: kind must be \"graph\" or \"batch\"");
    TC_REQUIRE(edges >= 0, TC_EINVAL, "tc_tuning_key: edges < 0");
    tc::copy_text(tc::tuning_key(kind, edges), out, cap);
  });
}

tc_status tc_graph_retune(const tc_graph* gh, const char* params_json, void* stream, tc_graph** out) {
  return tc::guarded("tc_graph_retune", [&] {
    TC_REQUIRE(out != nullptr, TC_EINVAL, "tc_graph_retune: out is NULL");
    *out = nullptr;
    TC_REQUIRE(gh != nullptr, TC_EINVAL, "tc_graph_retune: null graph");
    const tc::Graph& base = *tc::G(gh);
    tc::require_plain(base, "tc_graph_retune");
    const tc::WorkParams wp = tc::parse_thresholds(params_json, base.w.wp, "tc_graph_retune");
    *out = reinterpret_cast<tc_graph*>(tc::build_variant(base, 0, wp, static_cast<hipStream_t>(stream)));
  });
}

tc_status tc_graph_work_params(const tc_graph* gh, char* out, size_t cap) {
  return tc::guarded("tc_graph_work_params", [&] {
    TC_REQUIRE(gh != nullptr, TC_EINVAL, "tc_graph_work_params: null graph");
    tc::copy_text("{" + tc::work_params_json(tc::G(gh)->w.wp) + "}", out, cap);
  });
}

tc_status tc_graph_autotune(const tc_graph* gh, void* stream, char* out_json, size_t cap) {
  return tc::guarded("tc_graph_autotune", [&] {
    TC_REQUIRE(gh != nullptr, TC_EINVAL, "tc_graph_autotune: null graph");
    const tc::Graph& g = *tc::G(gh);
    tc::require_plain(g, "tc_graph_autotune");
    hipStream_t st = static_cast<hipStream_t>(stream);
    int64_t* d_count = nullptr;
    TC_HIP(hipMalloc(&d_count, sizeof(int64_t)));
    std::unique_ptr<int64_t, void (*)(int64_t*)> hold(d_count, [](int64_t* p) { (void)hipFree(p); });
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
    // median-of-5 time of tc_count on a graph whose work is cut by wp
    auto time_count = [&](const tc::Graph& h) {
      const tc::CountView v = tc::graph_view(h);
      tc::launch_count(v, tc::MODE_COUNT, d_count, nullptr, nullptr, st);  // warm-up
      std::vector<float> t;
      for (int r = 0; r < 5; ++r) {
        TC_HIP(hipEventRecord(e0, st));
        tc::launch_count(v, tc::MODE_COUNT, d_count, nullptr, nullptr, st);
        TC_HIP(hipEventRecord(e1, st));
        TC_HIP(hipEventSynchronize(e1));
        float f = 0;
        TC_HIP(hipEventElapsedTime(&f, e0, e1));
        t.push_back(f);
      }
      tc::note_use(h, st);
      std::sort(t.begin(), t.end());
      return (double)t[t.size() / 2];
    };
    auto entry = [](const tc::WorkParams& wp, double ms) {
      char buf[64];
      std::snprintf(buf, sizeof(buf), ", \"ms\": %.4f}", ms);
      return "{" + tc::work_params_json(wp) + buf;
    };
    // coordinate descent from the graph's own thresholds: each parameter in
    // turn takes the best of its candidate values, the others held
    tc::WorkParams best = g.w.wp;
    double best_ms = time_count(g);
    std::string all = "[" + entry(best, best_ms);
    const uint64_t heavy[] = {8192, 16384, 32768, 65536, 131072};
    const uint64_t target[] = {16384, 32768, 65536, 131072, 262144};
    const uint32_t slots[] = {2048, 4096, 8192};
    const uint32_t chunk[] = {8192, 16384, 32767};
    const uint32_t groups[] = {0, 4096, 16384, 65536};
    for (int param = 0; param < 5; ++param) {
      const int nc = param <= 1 ? 5 : param == 4 ? 4 : 3;
      const tc::WorkParams start = best;
      for (int c = 0; c < nc; ++c) {
        tc::WorkParams wp = start;
        if (param == 0) wp.heavy_min = heavy[c];
        if (param == 1) wp.pack_target = target[c];
        if (param == 2) wp.pack_slots = slots[c];
        if (param == 3) wp.wave_chunk = chunk[c];
        if (param == 4) wp.min_groups = groups[c];
        if (wp == start) continue;
        std::unique_ptr<tc::Graph, void (*)(tc::Graph*)> h(tc::build_variant(g, 0, wp, st), tc::destroy_graph);
        const double ms = time_count(*h);
        all += ", " + entry(wp, ms);
        if (ms < best_ms) {
          best_ms = ms;
          best = wp;
        }
      }
    }
    all += "]";
    const std::string key = tc::tuning_key("graph", g.m);
    tc::tuning_store(key, entry(best, best_ms));
    tc::copy_text("{\"key\": \"" + key + "\", \"best\": " + entry(best, best_ms) + ", \"candidates\": " + all + "}",
                  out_json, cap);
  });
}

}  // extern "C"
