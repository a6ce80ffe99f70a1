// Tile-shape tuning table of the persistent sweep (host side).
#pragma once
#include "../../include/fp.h"

namespace fp {
// Tuned tile for (ensemble, precision) on the current device, or `fallback`.
int tune_lookup(const fp_ensemble_t* e, int precision, int fallback);
int contract_dispatch(const fp_ensemble_t* e, int64_t num_pairs, int precision, const void* gates, double* trace,
                      void* ws, size_t ws_bytes, hipStream_t s, int64_t trace_offset, int tile_override);
}  // namespace fp
