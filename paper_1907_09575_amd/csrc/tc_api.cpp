// tc_api.cpp - C ABI entry points that are thin wrappers over the internal
// graph and the count launchers (tc_preprocess lives in tc_preprocess.hip,
// block and batched counting in their own files).
#include <string>

#include "tc_internal.h"

namespace tc {

const char* const kClassNames[NUM_CLASSES] = {"pack_small", "pack_large", "wg_small", "wg_large",
                                              "wg_huge",    "wg_giant",   "global"};

static thread_local std::string g_last_error;

void set_last_error(const std::string& msg) { g_last_error = msg; }

}  // namespace tc

#define TC_API_GUARD(body)                                   \
  try {                                                      \
    body;                                                    \
    tc::set_last_error("");                                  \
    return TC_OK;                                            \
  } catch (const tc::Error& e) {                             \
    tc::set_last_error(e.what());                            \
    return e.status;                                         \
  } catch (const std::bad_alloc&) {                          \
    tc::set_last_error("host allocation failed");            \
    return TC_ENOMEM;                                        \
  } catch (const std::exception& e) {                        \
    tc::set_last_error(e.what());                            \
    return TC_EDEVICE;                                       \
  }

extern "C" {

tc_status tc_graph_info(const tc_graph* gh, tc_info* out) {
  TC_API_GUARD({
    TC_REQUIRE(gh && out, TC_EINVAL, "tc_graph_info: null argument");
    const tc::Graph& g = *tc::G(gh);
    out->n = g.n;
    out->m_raw = g.m_raw;
    out->m = g.m;
    out->wedges_plus = g.wedges_plus;
    out->probes = g.w.probes;
    out->tasks = g.w.n_tasks;
    out->max_out_degree = g.max_dplus;
    out->device_bytes = (int64_t)g.arena_bytes;
  })
}

tc_status tc_graph_export(const tc_graph* gh, int64_t* d_row_ptr, int32_t* d_col, int32_t* d_perm,
                          void* stream) {
  TC_API_GUARD({
    TC_REQUIRE(gh, TC_EINVAL, "tc_graph_export: null graph");
    const tc::Graph& g = *tc::G(gh);
    hipStream_t st = static_cast<hipStream_t>(stream);
    if (d_row_ptr)
      TC_HIP(hipMemcpyAsync(d_row_ptr, g.row_ptr, sizeof(int64_t) * (size_t)(g.n + 1),
                            hipMemcpyDeviceToDevice, st));
    if (d_col && g.m > 0)
      TC_HIP(hipMemcpyAsync(d_col, g.col, sizeof(int32_t) * (size_t)g.m, hipMemcpyDeviceToDevice, st));
    if (d_perm)
      TC_HIP(hipMemcpyAsync(d_perm, g.perm, sizeof(int32_t) * (size_t)g.n, hipMemcpyDeviceToDevice, st));
    tc::note_use(g, st);
  })
}

tc_status tc_count(const tc_graph* gh, int64_t* d_count, void* stream) {
  TC_API_GUARD({
    TC_REQUIRE(gh && d_count, TC_EINVAL, "tc_count: null argument");
    const tc::Graph& g = *tc::G(gh);
    tc::launch_count(tc::graph_view(g), tc::MODE_COUNT, d_count, nullptr, nullptr, static_cast<hipStream_t>(stream));
    tc::note_use(g, static_cast<hipStream_t>(stream));
  })
}

tc_status tc_edge_support(const tc_graph* gh, int mode, int32_t* d_support, int64_t* d_count,
                          void* stream) {
  TC_API_GUARD({
    TC_REQUIRE(gh, TC_EINVAL, "tc_edge_support: null graph");
    TC_REQUIRE(mode == TC_SUPPORT_FULL || mode == TC_SUPPORT_ORIENTED, TC_EINVAL,
               "tc_edge_support: unknown mode");
    const tc::Graph& g = *tc::G(gh);
    tc::require_plain(g, "tc_edge_support");
    TC_REQUIRE(d_support || g.m == 0, TC_EINVAL, "tc_edge_support: null support array");
    hipStream_t st = static_cast<hipStream_t>(stream);
    tc::launch_count(tc::graph_view(g),
                     mode == TC_SUPPORT_FULL ? tc::MODE_SUPPORT_FULL : tc::MODE_SUPPORT_ORIENTED, d_count,
                     d_support, nullptr, st);
    tc::note_use(g, st);
  })
}

tc_status tc_graph_class_stats(const tc_graph* gh, tc_class_stats* out) {
  TC_API_GUARD({
    TC_REQUIRE(gh && out, TC_EINVAL, "tc_graph_class_stats: null argument");
    const tc::Graph& g = *tc::G(gh);
    for (int c = 0; c < tc::NUM_CLASSES; ++c) {
      tc_class_stats& o = out[c];
      const bool pack = c == tc::CLS_PACK_SMALL || c == tc::CLS_PACK_LARGE;
      o.workgroups = pack ? g.w.n_packs[c] : g.w.n_items[c] / tc::class_waves(c);
      o.rows = g.w.cls_stats[c][0];
      o.table_keys = g.w.cls_stats[c][1];
      o.tasks = g.w.cls_stats[c][2];
      o.probes = g.w.cls_stats[c][3];
      o.table_slots = g.w.cls_stats[c][0] ? (int64_t)1 << g.w.cls_log2S[c] : 0;
    }
  })
}

const char* tc_class_name(int32_t cls) {
  return (cls >= 0 && cls < tc::NUM_CLASSES) ? tc::kClassNames[cls] : nullptr;
}

void tc_graph_free(tc_graph* gh) {
  if (!gh) return;
  tc::destroy_graph(reinterpret_cast<tc::Graph*>(gh));
}

const char* tc_status_string(tc_status s) {
  switch (s) {
    case TC_OK: return "TC_OK";
    case TC_EINVAL: return "TC_EINVAL: invalid argument";
    case TC_ENOMEM: return "TC_ENOMEM: out of memory";
    case TC_EDEVICE: return "TC_EDEVICE: HIP runtime error";
    case TC_EOVERFLOW: return "TC_EOVERFLOW: size exceeds index width";
    case TC_EBUSY: return "TC_EBUSY: no capacity";
    case TC_ECANCELED: return "TC_ECANCELED: cancelled";
  }
  return "unknown tc_status";
}

const char* tc_last_error(void) { return tc::g_last_error.c_str(); }

const char* tc_version(void) { return "tcmi 0.1.0 (gfx950)"; }

}  // extern "C"
