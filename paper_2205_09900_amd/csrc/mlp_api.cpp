// C-ABI of the surrogate network (declared in include/fp.h).
#include <hip/hip_runtime.h>
#include <math.h>

#include "internal.h"
#include "layout.h"

namespace fp {
int mlp_forward(int n_in, int H, int64_t Bn, const float* params, const float* x, float* y, float* act, hipStream_t s);
int mlp_backward(int n_in, int H, int64_t Bn, const float* params, const float* x, const float* act, const float* t,
                 float* grad, double* h_loss, hipStream_t s);
int mlp_gemm_test(int M, int N, int K, const float* A, int lda, int ta, const float* B, int ldb, int tb, float* C,
                  int ldc, hipStream_t s);
int mlp_adam(int64_t n, float* p, const float* g, float* adam, int step, float lr, float b1, float b2, float eps,
             hipStream_t s);
int mlp_init(int n_in, int H, uint64_t seed, float* p, hipStream_t s);
int mlp_features(const fp_ensemble_t* e, int64_t num_pairs, const void* gates, float* x, hipStream_t s);
int run_cv_holdout(const double* tr, const float* g, int64_t n, int k, double* out6, hipStream_t s);
int run_moments_f32(const float* x, int64_t n, double* mean, double* var, hipStream_t s);
}  // namespace fp

using namespace fp;

static int check_shape(int n_in, int hidden) {
  if (n_in < 1 || hidden < 1 || n_in > (1 << 20) || hidden > 8192)
    return set_error(FP_EINVAL, "bad network shape %d x %d", n_in, hidden);
  return FP_OK;
}

extern "C" {

int64_t fp_mlp_param_count(int n_in, int hidden) {
  if (check_shape(n_in, hidden)) return 0;
  return (int64_t)n_in * hidden + hidden + 2 * ((int64_t)hidden * hidden + hidden) + hidden + 1;
}

int64_t fp_mlp_act_floats(int64_t batch, int hidden) { return batch < 0 || hidden < 1 ? 0 : 6 * batch * hidden; }

int fp_mlp_init(int n_in, int hidden, uint64_t seed, float* d_params, void* stream) {
  int rc = check_shape(n_in, hidden);
  if (rc) return rc;
  if (!d_params) return set_error(FP_EINVAL, "d_params is NULL");
  return mlp_init(n_in, hidden, seed, d_params, (hipStream_t)stream);
}

int fp_mlp_features(const fp_ensemble_t* ens, int64_t num_pairs, const void* d_gates, float* d_x, void* stream) {
  if (!ens || ens->ansatz != FP_HEA_RYRZ_CZ) return set_error(FP_EINVAL, "features are defined for the HEA ensemble");
  if (ens->n_qubits < 2 || ens->n_qubits > 64 || ens->depth < 1 || ens->depth > 64)
    return set_error(FP_EINVAL, "bad ensemble");
  if (num_pairs < 0) return set_error(FP_EINVAL, "num_pairs < 0");
  if (num_pairs == 0) return FP_OK;
  if (!d_gates || !d_x) return set_error(FP_EINVAL, "NULL buffer");
  return mlp_features(ens, num_pairs, d_gates, d_x, (hipStream_t)stream);
}

int fp_mlp_forward(int n_in, int hidden, int64_t batch, const float* d_params, const float* d_x, float* d_y,
                   float* d_act, void* stream) {
  int rc = check_shape(n_in, hidden);
  if (rc) return rc;
  if (batch < 0 || batch > (1 << 30)) return set_error(FP_EINVAL, "bad batch");
  if (batch == 0) return FP_OK;
  if (!d_params || !d_x || !d_y) return set_error(FP_EINVAL, "NULL buffer");
  return mlp_forward(n_in, hidden, batch, d_params, d_x, d_y, d_act, (hipStream_t)stream);
}

int fp_mlp_backward(int n_in, int hidden, int64_t batch, const float* d_params, const float* d_x, const float* d_act,
                    const float* d_target, float* d_grad, double* h_loss, void* stream) {
  int rc = check_shape(n_in, hidden);
  if (rc) return rc;
  if (batch < 1 || batch > (1 << 30)) return set_error(FP_EINVAL, "bad batch");
  if (!d_params || !d_x || !d_act || !d_target || !d_grad) return set_error(FP_EINVAL, "NULL buffer");
  return mlp_backward(n_in, hidden, batch, d_params, d_x, d_act, d_target, d_grad, h_loss, (hipStream_t)stream);
}

int fp_mlp_adam_step(int64_t count, float* d_params, const float* d_grad, float* d_adam, int step, float lr,
                     float beta1, float beta2, float eps, void* stream) {
  if (count < 0 || step < 1 || !(lr > 0.0f) || !(beta1 >= 0.0f && beta1 < 1.0f) || !(beta2 >= 0.0f && beta2 < 1.0f))
    return set_error(FP_EINVAL, "bad Adam arguments");
  if (count == 0) return FP_OK;
  if (!d_params || !d_grad || !d_adam) return set_error(FP_EINVAL, "NULL buffer");
  return mlp_adam(count, d_params, d_grad, d_adam, step, lr, beta1, beta2, eps, (hipStream_t)stream);
}

int fp_mlp_gemm(int M, int N, int K, const float* d_A, int lda, int trans_a, const float* d_B, int ldb, int trans_b,
                float* d_C, int ldc, void* stream) {
  if (M < 0 || N < 0 || K < 0 || !d_A || !d_B || !d_C) return set_error(FP_EINVAL, "bad GEMM arguments");
  if (M == 0 || N == 0) return FP_OK;
  return mlp_gemm_test(M, N, K, d_A, lda, trans_a ? 1 : 0, d_B, ldb, trans_b ? 1 : 0, d_C, ldc, (hipStream_t)stream);
}

// ---- control-variate statistics and the plain-or-CV choice ----------------------

int fp_cv_holdout(const double* d_trace, const float* d_g, int64_t num_pairs, int k, double* h_stats, void* stream) {
  if (!d_trace || !d_g || !h_stats) return set_error(FP_EINVAL, "NULL argument");
  if (num_pairs < 2 || k < 1 || k > 8) return set_error(FP_EINVAL, "bad arguments");
  return run_cv_holdout(d_trace, d_g, num_pairs, k, h_stats, (hipStream_t)stream);
}

int fp_moments_f32(const float* d_x, int64_t n, double* h_mean, double* h_var, void* stream) {
  if (!d_x || !h_mean || !h_var || n < 2) return set_error(FP_EINVAL, "bad arguments");
  return run_moments_f32(d_x, n, h_mean, h_var, (hipStream_t)stream);
}

int fp_cv_choose(double rho, double sec_per_exact, double sec_per_surrogate, int* use_cv, double* time_ratio) {
  if (!use_cv || !(sec_per_exact > 0.0) || !(sec_per_surrogate >= 0.0) || !(fabs(rho) <= 1.0 + 1e-12) ||
      !isfinite(sec_per_surrogate))
    return set_error(FP_EINVAL, "bad arguments");
  // Variance per unit time with the best split of the time between exact
  // pairs and surrogate draws, relative to the plain estimator's.
  const double r2 = rho * rho < 1.0 ? rho * rho : 1.0;
  const double a = sqrt((1.0 - r2) * sec_per_exact) + fabs(rho) * sqrt(sec_per_surrogate);
  const double ratio = a * a / sec_per_exact;
  *use_cv = ratio < 1.0 ? 1 : 0;
  if (time_ratio) *time_ratio = ratio;
  return FP_OK;
}

int fp_cv_time_to_rel_se(const double* stats_B, double c, double var_g_C, double rel_se, double sec_per_exact,
                         double sec_per_surrogate, double* t_plain, double* t_cv) {
  if (!stats_B || !t_plain || !t_cv || !(rel_se > 0.0) || var_g_C < 0.0 || sec_per_exact < 0.0 ||
      sec_per_surrogate < 0.0)
    return set_error(FP_EINVAL, "bad arguments");
  const double F = stats_B[2], var_f = stats_B[3], var_g = stats_B[5], rho = stats_B[1];
  if (!(F > 0.0) || var_f < 0.0 || var_g < 0.0) return set_error(FP_EINVAL, "bad statistics of the exact pairs");
  // variance of f - c g over the exact pairs
  double var_r = var_f - 2.0 * c * rho * sqrt(var_f * var_g) + c * c * var_g;
  if (var_r < 0.0) var_r = 0.0;
  const double target = (rel_se * F) * (rel_se * F);
  *t_plain = var_f / target * sec_per_exact;
  const double a = sqrt(var_r * sec_per_exact) + fabs(c) * sqrt(var_g_C * sec_per_surrogate);
  *t_cv = a * a / target;
  return FP_OK;
}

}  // extern "C"
