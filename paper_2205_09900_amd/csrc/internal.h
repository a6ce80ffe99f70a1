// Internal declarations shared by the library's translation units.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/fp.h"

namespace fp {

// Thread-local last-error text; returns `code`.
int set_error(int code, const char* fmt, ...);
// FP_OK, or FP_EDEVICE with the launch error recorded.
int check_launch(const char* what);
int check_hip(hipError_t e, const char* what);

int launch_sample(const fp_ensemble_t* e, int64_t num_pairs, uint64_t seed, uint64_t first_pair,
                  int precision, void* d_gates, hipStream_t stream);
// Haar U(q^2) gates of a qudit brickwork (qudit.hip)
int launch_sample_qudit(const fp_ensemble_t* e, int64_t num_pairs, uint64_t seed, uint64_t first_pair, int precision,
                        void* d_gates, hipStream_t s);

}  // namespace fp
