// C-ABI of the statistics of the estimates (declared in include/fp.h): the
// bootstrap, the layers-to-epsilon fit, the Haar values, the sample-size rule
// and the adaptive estimator built on it.
#include <hip/hip_runtime.h>
#include <math.h>
#include <string.h>

#include <algorithm>
#include <chrono>

#include "dispatch.h"
#include "internal.h"
#include "layout.h"
#include "sweep.h"

namespace fp {
int run_bootstrap(const double* d_trace, int64_t n, int kmax, int R, uint64_t seed, double* d_samples,
                  double* h_median, double* h_lo, double* h_hi, double coverage, hipStream_t s);
int run_layers_to_epsilon(const double* d_F, const int32_t* h_layers, int nl, int R, double fh, double epsilon,
                          int n, int q, int k, double rel_dev_max, double* d_out, double* h_median, int* h_failed,
                          hipStream_t s);
int contract_dispatch(const fp_ensemble_t* e, int64_t num_pairs, int precision, const void* gates, double* trace,
                      void* ws, size_t ws_bytes, hipStream_t s, int64_t trace_offset);

namespace {

// Longest increasing subsequence of p[0..k) (patience sorting).
int lis(const int* p, int k) {
  int tails[16];
  int len = 0;
  for (int i = 0; i < k; ++i) {
    int lo = 0, hi = len;
    while (lo < hi) {
      const int mid = (lo + hi) / 2;
      if (tails[mid] < p[i])
        lo = mid + 1;
      else
        hi = mid;
    }
    tails[lo] = p[i];
    if (lo == len) ++len;
  }
  return len;
}

}  // namespace
}  // namespace fp

using namespace fp;

extern "C" {

int fp_haar_frame_potential(int k, double dim, double* out) {
  if (!out || k < 1 || k > 10 || !(dim >= 1.0)) return set_error(FP_EINVAL, "bad arguments");
  double f = 1.0;
  for (int i = 2; i <= k; ++i) f *= i;
  if (dim >= (double)k) {
    *out = f;
    return FP_OK;
  }
  int p[16];
  for (int i = 0; i < k; ++i) p[i] = i;
  long long cnt = 0;
  do {
    if (lis(p, k) <= (int)dim) ++cnt;
  } while (std::next_permutation(p, p + k));
  *out = (double)cnt;
  return FP_OK;
}

int fp_bootstrap(const double* d_trace, int64_t num_pairs, int k_max, int resamples, uint64_t seed,
                 double* d_samples, double* h_median, double* h_lo, double* h_hi, double coverage, void* stream) {
  if (!d_trace) return set_error(FP_EINVAL, "NULL trace");
  if (num_pairs < 1 || num_pairs > ((int64_t)1 << 40)) return set_error(FP_EINVAL, "num_pairs outside 1..2^40");
  if (k_max < 1 || k_max > 8) return set_error(FP_EINVAL, "k_max %d outside 1..8", k_max);
  if (resamples < 2 || resamples > 1024) return set_error(FP_EINVAL, "resamples %d outside 2..1024", resamples);
  if (!(coverage > 0.0 && coverage < 1.0)) return set_error(FP_EINVAL, "coverage outside (0, 1)");
  return run_bootstrap(d_trace, num_pairs, k_max, resamples, seed, d_samples, h_median, h_lo, h_hi, coverage,
                       (hipStream_t)stream);
}

int fp_layers_to_epsilon(const double* d_F, const int32_t* h_layers, int n_layers, int resamples, double F_haar,
                         double epsilon, int n_qubits, int q, int k, double rel_dev_max, double* d_out,
                         double* h_median, int* h_failed, void* stream) {
  if (!d_F || !h_layers) return set_error(FP_EINVAL, "NULL argument");
  if (n_layers < 1 || resamples < 1 || !(F_haar > 0.0) || !(epsilon > 0.0) || n_qubits < 1 || q < 2 || k < 1 ||
      !(rel_dev_max > 0.0))
    return set_error(FP_EINVAL, "bad arguments");
  return run_layers_to_epsilon(d_F, h_layers, n_layers, resamples, F_haar, epsilon, n_qubits, q, k, rel_dev_max,
                               d_out, h_median, h_failed, (hipStream_t)stream);
}

int fp_sample_size_decision(double F, double se, double F_haar, double F_lower, double z, int64_t n_done,
                            int64_t n_max, double seconds, double max_seconds, int* decision) {
  if (!decision || !(se >= 0.0) || !(z >= 0.0)) return set_error(FP_EINVAL, "bad arguments");
  if (n_done >= n_max || seconds >= max_seconds)
    *decision = FP_STOP_BUDGET;
  else if (F < F_haar || (F_lower > 0.0 && F > F_lower))
    *decision = FP_CONTINUE;
  else if (F - F_haar > z * se)
    *decision = FP_STOP_RESOLVED;
  else
    *decision = FP_CONTINUE;
  return FP_OK;
}

int fp_frame_potential_adaptive(const fp_ensemble_t* ens, int precision, int k_max, int k_rule, uint64_t seed,
                                int64_t batch_pairs, int64_t max_pairs, double max_seconds, double z, double F_haar,
                                double F_lower, void* d_gates, size_t gates_bytes, void* d_ws, size_t ws_bytes,
                                double* d_trace, double* h_F, double* h_stderr, int64_t* h_pairs_used, int* h_reason,
                                void* stream) {
  int rc = check_ensemble(ens);
  if (rc) return rc;
  if ((rc = check_precision(precision))) return rc;
  if (!d_gates || !d_trace || !h_F || !h_pairs_used || !h_reason) return set_error(FP_EINVAL, "NULL argument");
  if (k_max < 1 || k_max > 8 || k_rule < 1 || k_rule > k_max) return set_error(FP_EINVAL, "bad k");
  if (batch_pairs < 2 || max_pairs < batch_pairs) return set_error(FP_EINVAL, "bad batch or budget");
  const int64_t stride = pair_bytes(ens->ansatz, ens->n_qubits, ens->depth, precision, ens->local_dim);
  if ((int64_t)gates_bytes < batch_pairs * stride) return set_error(FP_EINVAL, "gate buffer below one batch");
  size_t need = 0;
  if ((rc = workspace_bytes_impl(ens, batch_pairs, precision, &need))) return rc;
  if (ws_bytes < need) return set_error(FP_ETOOBIG, "workspace of %zu bytes needed for one batch", need);
  hipStream_t s = (hipStream_t)stream;
  const auto t0 = std::chrono::steady_clock::now();
  double F[8], SE[8];
  int64_t done = 0;
  int decision = FP_CONTINUE;
  while (decision == FP_CONTINUE) {
    const int64_t m = max_pairs - done < batch_pairs ? max_pairs - done : batch_pairs;
    rc = fp_sample_gates(ens, m, seed, (uint64_t)done, precision, d_gates, gates_bytes, stream);
    if (!rc) rc = contract_dispatch(ens, m, precision, d_gates, d_trace, d_ws, ws_bytes, s, done);
    if (rc) return rc;
    done += m;
    rc = fp_frame_potential(d_trace, done, k_max, F, SE, stream);  // synchronises
    if (rc) return rc;
    const double secs = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    rc = fp_sample_size_decision(F[k_rule - 1], SE[k_rule - 1], F_haar, F_lower, z, done, max_pairs, secs,
                                 max_seconds, &decision);
    if (rc) return rc;
  }
  for (int k = 0; k < k_max; ++k) {
    h_F[k] = F[k];
    if (h_stderr) h_stderr[k] = SE[k];
  }
  *h_pairs_used = done;
  *h_reason = decision;
  return FP_OK;
}

}  // extern "C"
