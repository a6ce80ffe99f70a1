// Entry points whose implementation is not in this build yet.
#include <hip/hip_runtime.h>

#include "internal.h"
#include "tune.h"

namespace fp {
int tune_lookup(const fp_ensemble_t*, int, int fallback) { return fallback; }
}  // namespace fp

using namespace fp;
extern "C" {
int fp_workspace_bytes_groups(const fp_ensemble_t*, int, const fp_group_t*, int, size_t*) {
  return set_error(FP_ENOTIMPL, "not built");
}
int fp_contract_trace_groups(const fp_ensemble_t*, int, const fp_group_t*, int, const void* const*, double*, void*,
                             size_t, void*) {
  return set_error(FP_ENOTIMPL, "not built");
}
size_t fp_autotune_workspace_bytes(const fp_ensemble_t*, int) { return 0; }
int fp_autotune(const fp_ensemble_t*, int, void*, size_t, int*, void*) { return set_error(FP_ENOTIMPL, "not built"); }
int fp_autotune_table(char* buf, size_t cap) {
  if (buf && cap) buf[0] = 0;
  return FP_OK;
}
int fp_autotune_load(const char*) { return set_error(FP_ENOTIMPL, "not built"); }
}
