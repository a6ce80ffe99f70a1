// Launch tuning of the persistent sweep over groups (host side).
#pragma once
#include <hip/hip_runtime.h>

#include "../../include/fp.h"

namespace fp {

// Launch choice of one group of the persistent sweep: its lane class
// (PCLASS_* of sched.h) and the algorithmic flops of work per task.
struct GroupLaunch {
  int cls;
  double task_flops;
};

// Tuned choice for (ensemble, precision) on the current device; false if none.
bool tune_group_lookup(const fp_ensemble_t* e, int precision, GroupLaunch* out);

// The persistent sweep over groups; `force` (may be NULL) overrides the
// launch choice of every group.
int contract_groups(const fp_ensemble_t* ens, int n_ens, const fp_group_t* groups, int n_groups,
                    const void* const* d_gates, double* d_trace, void* d_ws, size_t ws_bytes, hipStream_t s,
                    const GroupLaunch* force);

int contract_dispatch(const fp_ensemble_t* e, int64_t num_pairs, int precision, const void* gates, double* trace,
                      void* ws, size_t ws_bytes, hipStream_t s, int64_t trace_offset);

}  // namespace fp
