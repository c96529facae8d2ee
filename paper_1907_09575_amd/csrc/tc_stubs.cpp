// Temporary: entry points whose implementations are not in this build yet.
#include "tc_internal.h"

extern "C" {
tc_status tc_batch_create(const tc_graph* const*, int32_t, const char*, void*, tc_batch** out) {
  if (out) *out = nullptr;
  tc::set_last_error("tc_batch_create: not implemented in this build");
  return TC_EINVAL;
}
tc_status tc_batch_count(tc_batch*, int64_t*, void*) {
  tc::set_last_error("tc_batch_count: not implemented in this build");
  return TC_EINVAL;
}
void tc_batch_free(tc_batch*) {}
tc_status tc_count_batched(const tc_graph* const*, int32_t, int64_t*, const char*, void*) {
  tc::set_last_error("tc_count_batched: not implemented in this build");
  return TC_EINVAL;
}
}
