// Host-side dispatch helpers shared by the C-ABI translation units.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/fp.h"
#include "plan.h"

namespace fp {

struct DevPlan {
  PlanHeader hdr;
  Op* ops = nullptr;
  int2* wg = nullptr;
  int32_t* fac = nullptr;
  PlanHeader* dhdr = nullptr;
};

constexpr int NUM_AUX = 3;  // side streams per caller stream
struct Aux {
  hipStream_t s[NUM_AUX];
  hipEvent_t fork, join[NUM_AUX];
};

int check_ensemble(const fp_ensemble_t* e);
int check_precision(int p);
int get_brickwork_plan(int n, int depth, DevPlan* out);
int get_aux(Aux* out, hipStream_t caller);  // side streams for a call on caller (shared per device unless capturing)
int lds_bits_max(int precision);
int tile_pairs(int tile);
double hea_flops_per_pair(int n, int L);
int workspace_bytes_impl(const fp_ensemble_t* e, int64_t num_pairs, int precision, size_t* out);
int contract_brickwork(const fp_ensemble_t* e, int64_t num_pairs, int precision, const void* gates, double* trace,
                       void* ws, size_t ws_bytes, hipStream_t s, int64_t trace_offset);
int contract_local_random(const fp_ensemble_t* e, int64_t num_pairs, int precision, const void* gates, double* trace,
                          void* ws, size_t ws_bytes, hipStream_t s, int64_t trace_offset);
int contract_hea(const fp_ensemble_t* e, int64_t num_pairs, int precision, const void* gates, double* trace,
                 hipStream_t s, int64_t trace_offset);

}  // namespace fp
