// Statistics of the frame-potential estimates on the device: the bootstrap
// (Supplementary Methods, bootstrapping for uncertainty quantification: N
// traces resampled with replacement, the estimate recomputed per resample),
// the exponential fit over the fit region (Supplementary Methods, choice of
// curve fitting region) with the layers needed for an epsilon-approximate
// design (main text, the exponential-decay bound), and the adaptive
// sample-size rule (Supplementary Methods, determination of sample sizes).
#include <hip/hip_runtime.h>
#include <math.h>
#include <time.h>

#include <algorithm>
#include <vector>

#include "internal.h"
#include "layout.h"
#include "philox.h"
#include "sweep.h"

namespace fp {

constexpr int ST_THREADS = 256;
constexpr int BOOT_KMAX = 8;
constexpr uint32_t BOOT_TAG = 0xB0075A3Bu;

// Largest |Tr|^2 (as its power-of-two exponent) and the count of non-finite traces.
__global__ void __launch_bounds__(ST_THREADS) boot_max_kernel(const double* __restrict__ tr, int64_t n,
                                                              unsigned long long* __restrict__ bits) {
  double m = 0.0;
  unsigned long long bad = 0;
  for (int64_t i = (int64_t)blockIdx.x * ST_THREADS + threadIdx.x; i < n; i += (int64_t)gridDim.x * ST_THREADS) {
    const double a = tr[2 * i] * tr[2 * i] + tr[2 * i + 1] * tr[2 * i + 1];
    if (!isfinite(a))
      ++bad;
    else
      m = fmax(m, a);
  }
  // non-negative doubles order as their bit patterns
  atomicMax(bits, (unsigned long long)__double_as_longlong(m));
  if (bad) atomicAdd(bits + 1, bad);
}

// Resample r = blockIdx.x, split s = blockIdx.y of S: draws i = 2 b, 2 b + 1
// for blocks b = s*per + t .. with one Philox block each; partial sums of
// (|Tr|^2 2^-e)^k, k = 1..kmax, per (r, s) in a fixed order.
__global__ void __launch_bounds__(ST_THREADS) boot_sum_kernel(const double* __restrict__ tr, int64_t n, int kmax,
                                                              uint64_t seed, const unsigned long long* __restrict__ bits,
                                                              double* __restrict__ part) {
  __shared__ double sh[ST_THREADS];
  const uint32_t r = blockIdx.x;
  const int S = gridDim.y, s = blockIdx.y;
  const int64_t nb = (n + 1) / 2;
  const int64_t per = (nb + S - 1) / S;
  const int64_t b0 = (int64_t)s * per, b1 = b0 + per < nb ? b0 + per : nb;
  int e = 0;
  const double mx = __longlong_as_double((long long)bits[0]);
  if (mx > 0.0) frexp(mx, &e);
  double acc[BOOT_KMAX];
#pragma unroll
  for (int k = 0; k < BOOT_KMAX; ++k) acc[k] = 0.0;
  const uint32_t k0 = (uint32_t)seed, k1 = (uint32_t)(seed >> 32);
  for (int64_t b = b0 + threadIdx.x; b < b1; b += ST_THREADS) {
    const u32x4 x = philox4x32_10((uint32_t)b, (uint32_t)((uint64_t)b >> 32), r, BOOT_TAG, k0, k1);
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      const int64_t i = 2 * b + h;
      if (i >= n) break;
      const uint64_t u = h == 0 ? ((uint64_t)x.v[1] << 32 | x.v[0]) : ((uint64_t)x.v[3] << 32 | x.v[2]);
      const int64_t idx = (int64_t)__umul64hi(u, (uint64_t)n);
      const double a = ldexp(tr[2 * idx] * tr[2 * idx] + tr[2 * idx + 1] * tr[2 * idx + 1], -e);
      double p = 1.0;
#pragma unroll
      for (int k = 0; k < BOOT_KMAX; ++k) {
        if (k < kmax) {
          p *= a;
          acc[k] += p;
        }
      }
    }
  }
  for (int k = 0; k < kmax; ++k) {
    sh[threadIdx.x] = acc[k];
    __syncthreads();
    for (int w = ST_THREADS / 2; w > 0; w >>= 1) {
      if (threadIdx.x < w) sh[threadIdx.x] += sh[threadIdx.x + w];
      __syncthreads();
    }
    if (threadIdx.x == 0) part[((int64_t)k * gridDim.x + r) * S + s] = sh[0];
    __syncthreads();
  }
}

// F_r^(k) = 2^(e k) (sum over the splits in order) / N.
__global__ void boot_final_kernel(const double* __restrict__ part, int R, int S, int kmax, int64_t n,
                                  const unsigned long long* __restrict__ bits, double* __restrict__ out) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= R * kmax) return;
  int e = 0;
  const double mx = __longlong_as_double((long long)bits[0]);
  if (mx > 0.0) frexp(mx, &e);
  const int k = i / R;
  double sum = 0.0;
  for (int s = 0; s < S; ++s) sum += part[(int64_t)i * S + s];
  out[i] = ldexp(sum / (double)n, e * (k + 1));
}

// One workgroup per k: bitonic sort of the R resample values (R <= 1024) in LDS.
__global__ void __launch_bounds__(512) boot_sort_kernel(const double* __restrict__ in, int R, double* __restrict__ out) {
  __shared__ double v[1024];
  const int k = blockIdx.x;
  int P = 1;
  while (P < R) P <<= 1;
  for (int i = threadIdx.x; i < P; i += blockDim.x) v[i] = i < R ? in[(int64_t)k * R + i] : INFINITY;
  __syncthreads();
  for (int size = 2; size <= P; size <<= 1) {
    for (int stride = size >> 1; stride > 0; stride >>= 1) {
      for (int i = threadIdx.x; i < P; i += blockDim.x) {
        const int j = i ^ stride;
        if (j > i) {
          const bool up = (i & size) == 0;
          const double a = v[i], b = v[j];
          if ((a > b) == up) {
            v[i] = b;
            v[j] = a;
          }
        }
      }
      __syncthreads();
    }
  }
  for (int i = threadIdx.x; i < R; i += blockDim.x) out[(int64_t)k * R + i] = v[i];
}

// Quantile with linear interpolation at position q (R - 1) of sorted values.
static double quantile_sorted(const double* v, int R, double q) {
  const double pos = q * (R - 1);
  int lo = (int)floor(pos);
  if (lo < 0) lo = 0;
  if (lo > R - 1) lo = R - 1;
  const int hi = lo + 1 < R ? lo + 1 : R - 1;
  return v[lo] + (pos - lo) * (v[hi] - v[lo]);
}

int run_bootstrap(const double* d_trace, int64_t n, int kmax, int R, uint64_t seed, double* d_samples,
                  double* h_median, double* h_lo, double* h_hi, double coverage, hipStream_t s) {
  int S = (int)((2048 + R - 1) / R);  // about 2048 workgroups in all
  const int64_t nb = (n + 1) / 2;
  const int64_t max_s = (nb + ST_THREADS - 1) / ST_THREADS;  // at least one block of draws per thread
  if (S > max_s) S = (int)max_s;
  if (S < 1) S = 1;
  const size_t part_n = (size_t)kmax * R * S;
  const size_t bytes = 256 + sizeof(double) * (part_n + 2 * (size_t)kmax * R);
  void* ws = nullptr;
  int rc = check_hip(hipMallocAsync(&ws, bytes, s), "hipMallocAsync(bootstrap)");
  if (rc) return rc;
  unsigned long long* bits = (unsigned long long*)ws;
  double* part = (double*)((unsigned char*)ws + 256);
  double* vals = part + part_n;
  double* sorted = vals + (size_t)kmax * R;
  rc = check_hip(hipMemsetAsync(bits, 0, 16, s), "memset bootstrap");
  int blocks = (int)((n + ST_THREADS - 1) / ST_THREADS);
  if (blocks > 1024) blocks = 1024;
  if (!rc) {
    hipLaunchKernelGGL(boot_max_kernel, dim3(blocks), dim3(ST_THREADS), 0, s, d_trace, n, bits);
    hipLaunchKernelGGL(boot_sum_kernel, dim3(R, S), dim3(ST_THREADS), 0, s, d_trace, n, kmax, seed, bits, part);
    hipLaunchKernelGGL(boot_final_kernel, dim3((R * kmax + 255) / 256), dim3(256), 0, s, part, R, S, kmax, n, bits,
                       vals);
    hipLaunchKernelGGL(boot_sort_kernel, dim3(kmax), dim3(512), 0, s, vals, R, sorted);
    rc = check_launch("bootstrap");
  }
  if (!rc && d_samples)
    rc = check_hip(hipMemcpyAsync(d_samples, vals, sizeof(double) * kmax * R, hipMemcpyDeviceToDevice, s),
                   "copy bootstrap samples");
  std::vector<double> host((size_t)kmax * R);
  unsigned long long hb[2] = {0, 0};
  if (!rc) rc = check_hip(hipMemcpyAsync(host.data(), sorted, sizeof(double) * host.size(), hipMemcpyDeviceToHost, s),
                          "copy sorted");
  if (!rc) rc = check_hip(hipMemcpyAsync(hb, bits, sizeof(hb), hipMemcpyDeviceToHost, s), "copy bootstrap status");
  const int rc2 = check_hip(hipFreeAsync(ws, s), "hipFreeAsync(bootstrap)");
  const int rc3 = check_hip(hipStreamSynchronize(s), "sync(bootstrap)");
  if (rc) return rc;
  if (rc2) return rc2;
  if (rc3) return rc3;
  if (hb[1] > 0) return set_error(FP_ENUMERIC, "%llu non-finite trace(s) in the batch", hb[1]);
  const double tail = 0.5 * (1.0 - coverage);
  for (int k = 0; k < kmax; ++k) {
    const double* v = host.data() + (size_t)k * R;
    if (h_median) h_median[k] = quantile_sorted(v, R, 0.5);
    if (h_lo) h_lo[k] = quantile_sorted(v, R, tail);
    if (h_hi) h_hi[k] = quantile_sorted(v, R, 1.0 - tail);
  }
  return FP_OK;
}

// ---- exponential fit and layers to epsilon -----------------------------------
// One thread per bootstrap sample r: least-squares line through
// (l_j, log(F_j - F_Haar)) over the layers with 0 < (F_j - F_Haar)/F_Haar <
// rel_dev_max; F - F_Haar = A^2 exp(-2 l / C) gives C = -2 / slope and
// log A = intercept / 2; l_eps = C (k n log q + log A + log(1/eps)).  NaN
// when fewer than two layers qualify or the line does not decay.
__global__ void fit_kernel(const double* __restrict__ F, const int32_t* __restrict__ layers, int nl, int R,
                           double fh, double rhs, double rel_dev_max, double* __restrict__ out) {
  const int r = blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= R) return;
  double sx = 0.0, sy = 0.0, sxx = 0.0, sxy = 0.0;
  int cnt = 0;
  for (int j = 0; j < nl; ++j) {
    const double f = F[(int64_t)j * R + r];
    const double d = (f - fh) / fh;
    if (!(d > 0.0 && d < rel_dev_max)) continue;
    const double x = (double)layers[j], y = log(f - fh);
    sx += x;
    sy += y;
    sxx += x * x;
    sxy += x * y;
    ++cnt;
  }
  double res = __builtin_nan("");
  if (cnt >= 2) {
    const double den = cnt * sxx - sx * sx;
    if (den > 0.0) {
      const double slope = (cnt * sxy - sx * sy) / den;
      const double icept = (sy - slope * sx) / cnt;
      if (slope < 0.0) {
        const double c = -2.0 / slope;
        res = c * (rhs + 0.5 * icept);
      }
    }
  }
  out[r] = res;
}

int run_layers_to_epsilon(const double* d_F, const int32_t* h_layers, int nl, int R, double fh, double epsilon,
                          int n, int q, int k, double rel_dev_max, double* d_out, double* h_median, int* h_failed,
                          hipStream_t s) {
  void* ws = nullptr;
  const size_t lbytes = (sizeof(int32_t) * nl + 255) & ~(size_t)255;
  int rc = check_hip(hipMallocAsync(&ws, lbytes + sizeof(double) * R, s), "hipMallocAsync(fit)");
  if (rc) return rc;
  int32_t* d_layers = (int32_t*)ws;
  double* res = (double*)((unsigned char*)ws + lbytes);
  rc = check_hip(hipMemcpyAsync(d_layers, h_layers, sizeof(int32_t) * nl, hipMemcpyHostToDevice, s), "upload layers");
  const double rhs = (double)k * n * log((double)q) + log(1.0 / epsilon);
  if (!rc) {
    hipLaunchKernelGGL(fit_kernel, dim3((R + 255) / 256), dim3(256), 0, s, d_F, d_layers, nl, R, fh, rhs,
                       rel_dev_max, res);
    rc = check_launch("layers_to_epsilon");
  }
  if (!rc && d_out) rc = check_hip(hipMemcpyAsync(d_out, res, sizeof(double) * R, hipMemcpyDeviceToDevice, s), "copy fit");
  std::vector<double> host(R);
  if (!rc) rc = check_hip(hipMemcpyAsync(host.data(), res, sizeof(double) * R, hipMemcpyDeviceToHost, s), "copy fit");
  const int rc2 = check_hip(hipFreeAsync(ws, s), "hipFreeAsync(fit)");
  const int rc3 = check_hip(hipStreamSynchronize(s), "sync(fit)");
  if (rc) return rc;
  if (rc2) return rc2;
  if (rc3) return rc3;
  std::vector<double> ok;
  for (double v : host)
    if (v == v) ok.push_back(v);
  if (h_failed) *h_failed = R - (int)ok.size();
  if (h_median) {
    if (ok.empty()) {
      *h_median = __builtin_nan("");
    } else {
      std::sort(ok.begin(), ok.end());
      *h_median = quantile_sorted(ok.data(), (int)ok.size(), 0.5);
    }
  }
  return FP_OK;
}

}  // namespace fp
