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
int64_t fp_mlp_param_count(int n_in, int hidden) {
  return (int64_t)n_in * hidden + hidden + 2 * ((int64_t)hidden * hidden + hidden) + hidden + 1;
}
int64_t fp_mlp_act_floats(int64_t batch, int hidden) { return batch * hidden * 6; }
int fp_mlp_init(int, int, uint64_t, float*, void*) { return set_error(FP_ENOTIMPL, "not built"); }
int fp_mlp_features(const fp_ensemble_t*, int64_t, const void*, float*, void*) {
  return set_error(FP_ENOTIMPL, "not built");
}
int fp_mlp_forward(int, int, int64_t, const float*, const float*, float*, float*, void*) {
  return set_error(FP_ENOTIMPL, "not built");
}
int fp_mlp_backward(int, int, int64_t, const float*, const float*, const float*, const float*, float*, double*,
                    void*) {
  return set_error(FP_ENOTIMPL, "not built");
}
int fp_mlp_adam_step(int64_t, float*, const float*, float*, int, float, float, float, float, void*) {
  return set_error(FP_ENOTIMPL, "not built");
}
}
