// Monte Carlo reduction of traces into frame potentials (Sec. II.A of the
// paper: F^(k) ~ mean of |Tr|^{2k}; the same traces serve every k).
//
// float64 throughout.  Each thread runs Welford's update over a fixed
// strided subset, workgroups merge by Chan's formula in a fixed tree, and a
// single workgroup merges the per-workgroup partials in index order, so the
// result is bitwise reproducible for a given N.  Terms are scaled by 2^-e,
// with 2^e the largest |Tr|^2 rounded to a power of two, so that |Tr|^{2k}
// cannot overflow before the final rescale.
#include <hip/hip_runtime.h>
#include <math.h>

#include <mutex>

#include "internal.h"

namespace fp {

constexpr int RED_THREADS = 256;
constexpr int RED_MAX_BLOCKS = 512;
constexpr int KMAX = 8;

struct Welford {
  double n, mean, m2;
};

__device__ __forceinline__ Welford chan_merge(Welford a, Welford b) {
  Welford r;
  r.n = a.n + b.n;
  if (r.n == 0.0) {
    r.mean = 0.0;
    r.m2 = 0.0;
    return r;
  }
  const double d = b.mean - a.mean;
  r.mean = a.mean + d * (b.n / r.n);
  r.m2 = a.m2 + b.m2 + d * d * (a.n * b.n / r.n);
  return r;
}

__device__ __forceinline__ void welford_add(Welford& w, double x) {
  w.n += 1.0;
  const double d = x - w.mean;
  w.mean += d / w.n;
  w.m2 += d * (x - w.mean);
}

// Pass 1: per-workgroup max of |Tr|^2 and count of non-finite traces.
__global__ void __launch_bounds__(RED_THREADS) red_max_kernel(const double* __restrict__ tr, int64_t n,
                                                              double* __restrict__ part) {
  __shared__ double smax[RED_THREADS];
  __shared__ double sbad[RED_THREADS];
  double m = 0.0, bad = 0.0;
  for (int64_t i = (int64_t)blockIdx.x * RED_THREADS + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * RED_THREADS) {
    const double re = tr[2 * i], im = tr[2 * i + 1];
    const double a = re * re + im * im;
    if (!isfinite(a))
      bad += 1.0;
    else
      m = fmax(m, a);
  }
  smax[threadIdx.x] = m;
  sbad[threadIdx.x] = bad;
  __syncthreads();
  for (int s = RED_THREADS / 2; s > 0; s >>= 1) {
    if (threadIdx.x < s) {
      smax[threadIdx.x] = fmax(smax[threadIdx.x], smax[threadIdx.x + s]);
      sbad[threadIdx.x] += sbad[threadIdx.x + s];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    part[2 * blockIdx.x] = smax[0];
    part[2 * blockIdx.x + 1] = sbad[0];
  }
}

// Pass 2 (one workgroup): global max -> scale exponent; bad count.
__global__ void __launch_bounds__(RED_THREADS) red_max_final(const double* __restrict__ part, int nb,
                                                             double* __restrict__ scale) {
  __shared__ double smax[RED_THREADS];
  __shared__ double sbad[RED_THREADS];
  double m = 0.0, bad = 0.0;
  for (int i = threadIdx.x; i < nb; i += RED_THREADS) {
    m = fmax(m, part[2 * i]);
    bad += part[2 * i + 1];
  }
  smax[threadIdx.x] = m;
  sbad[threadIdx.x] = bad;
  __syncthreads();
  for (int s = RED_THREADS / 2; s > 0; s >>= 1) {
    if (threadIdx.x < s) {
      smax[threadIdx.x] = fmax(smax[threadIdx.x], smax[threadIdx.x + s]);
      sbad[threadIdx.x] += sbad[threadIdx.x + s];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    int e = 0;
    if (smax[0] > 0.0) frexp(smax[0], &e);
    scale[0] = (double)e;  // terms are scaled by 2^-e
    scale[1] = sbad[0];
  }
}

// Pass 3: per-workgroup Welford of (|Tr|^2 2^-e)^k, k = 1..k_max.
__global__ void __launch_bounds__(RED_THREADS) red_moments_kernel(const double* __restrict__ tr, int64_t n,
                                                                  int kmax, const double* __restrict__ scale,
                                                                  Welford* __restrict__ part) {
  __shared__ Welford sw[RED_THREADS];
  const int e = (int)scale[0];
  Welford w[KMAX];
#pragma unroll
  for (int k = 0; k < KMAX; ++k) w[k] = Welford{0.0, 0.0, 0.0};
  for (int64_t i = (int64_t)blockIdx.x * RED_THREADS + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * RED_THREADS) {
    const double re = tr[2 * i], im = tr[2 * i + 1];
    const double a = ldexp(re * re + im * im, -e);
    double x = 1.0;
#pragma unroll
    for (int k = 0; k < KMAX; ++k) {
      if (k < kmax) {
        x *= a;
        welford_add(w[k], x);
      }
    }
  }
  for (int k = 0; k < kmax; ++k) {
    sw[threadIdx.x] = w[k];
    __syncthreads();
    for (int s = RED_THREADS / 2; s > 0; s >>= 1) {
      if (threadIdx.x < s) sw[threadIdx.x] = chan_merge(sw[threadIdx.x], sw[threadIdx.x + s]);
      __syncthreads();
    }
    if (threadIdx.x == 0) part[(int64_t)blockIdx.x * KMAX + k] = sw[0];
    __syncthreads();
  }
}

// Pass 4 (one workgroup of 256): merge the workgroup partials.  Thirty-two
// threads per k: thread j merges partials [j nb/32, (j+1) nb/32) in index
// order, then a fixed tree (j with j + s, s = 16, 8, .., 1) merges the 32
// results, so the order of the merges, and the result, never change.
constexpr int FINAL_THREADS = 256;
__global__ void __launch_bounds__(FINAL_THREADS) red_moments_final(const Welford* __restrict__ part, int nb, int kmax,
                                                                   const double* __restrict__ scale,
                                                                   double* __restrict__ out) {
  __shared__ Welford sw[FINAL_THREADS];
  const int t = threadIdx.x, k = t >> 5, j = t & 31;
  Welford acc{0.0, 0.0, 0.0};
  if (k < kmax) {
    const int lo = (int)((int64_t)nb * j / 32), hi = (int)((int64_t)nb * (j + 1) / 32);
    for (int b = lo; b < hi; ++b) acc = chan_merge(acc, part[(int64_t)b * KMAX + k]);
  }
  sw[t] = acc;
  __syncthreads();
  for (int s = 16; s > 0; s >>= 1) {
    if (j < s) sw[t] = chan_merge(sw[t], sw[t + s]);
    __syncthreads();
  }
  const int e = (int)scale[0];
  if (j == 0 && k < kmax) {
    const Welford w = sw[t];
    out[2 * k] = ldexp(w.mean, e * (k + 1));
    out[2 * k + 1] = w.n > 1.0 ? ldexp(sqrt(w.m2 / (w.n - 1.0) / w.n), e * (k + 1)) : 0.0;
  }
  if (t == 0) out[2 * KMAX] = scale[1];
}

static int red_blocks(int64_t n) {
  int64_t b = (n + RED_THREADS * 4 - 1) / (RED_THREADS * 4);
  if (b < 1) b = 1;
  if (b > RED_MAX_BLOCKS) b = RED_MAX_BLOCKS;
  return (int)b;
}

static size_t red_scratch_bytes(int nb) {
  return sizeof(double) * (2 * (size_t)nb + 2 + 2 * KMAX + 1) + sizeof(Welford) * nb * KMAX;
}

// The reduction on a scratch area of red_scratch_bytes(red_blocks(n)) bytes
// (no allocation; every partial is written before it is read).
static int frame_potential_on(const double* d_trace, int64_t n, int kmax, double* h_F, double* h_se, void* ws,
                              hipStream_t s, bool free_ws) {
  const int nb = red_blocks(n);
  double* part = (double*)ws;
  double* scale = part + 2 * nb;
  double* out = scale + 2;
  Welford* wpart = (Welford*)(out + 2 * KMAX + 1);
  hipLaunchKernelGGL(red_max_kernel, dim3(nb), dim3(RED_THREADS), 0, s, d_trace, n, part);
  hipLaunchKernelGGL(red_max_final, dim3(1), dim3(RED_THREADS), 0, s, part, nb, scale);
  hipLaunchKernelGGL(red_moments_kernel, dim3(nb), dim3(RED_THREADS), 0, s, d_trace, n, kmax, scale, wpart);
  hipLaunchKernelGGL(red_moments_final, dim3(1), dim3(FINAL_THREADS), 0, s, wpart, nb, kmax, scale, out);
  int rc = check_launch("frame_potential");
  double host[2 * KMAX + 1];
  if (!rc) rc = check_hip(hipMemcpyAsync(host, out, sizeof(host), hipMemcpyDeviceToHost, s), "copy F");
  int rc2 = free_ws ? check_hip(hipFreeAsync(ws, s), "hipFreeAsync(reduce)") : FP_OK;
  int rc3 = check_hip(hipStreamSynchronize(s), "sync(reduce)");
  if (rc) return rc;
  if (rc2) return rc2;
  if (rc3) return rc3;
  if (host[2 * KMAX] > 0.0)
    return set_error(FP_ENUMERIC, "%.0f non-finite trace(s) in the batch", host[2 * KMAX]);
  for (int k = 0; k < kmax; ++k) {
    h_F[k] = host[2 * k];
    if (h_se) h_se[k] = host[2 * k + 1];
  }
  return FP_OK;
}

int run_frame_potential(const double* d_trace, int64_t n, int kmax, double* h_F, double* h_se,
                        hipStream_t s) {
  void* ws = nullptr;
  int rc = check_hip(hipMallocAsync(&ws, red_scratch_bytes(red_blocks(n)), s), "hipMallocAsync(reduce)");
  if (rc) return rc;
  return frame_potential_on(d_trace, n, kmax, h_F, h_se, ws, s, true);
}

// ---- the reduction without allocation -------------------------------------------
// One file-scope scratch array per device for callers that cannot allocate.
// The largest reduction needs red_scratch_bytes(RED_MAX_BLOCKS) bytes (about
// 107 KiB) whatever the number of traces.  Host code never passes the
// array's name to a kernel: each device's address of it is taken once with
// hipGetSymbolAddress, with that device current, and kept per device.
constexpr size_t NOALLOC_SCRATCH_BYTES = 128 * 1024;
static __device__ __align__(256) unsigned char scratch[NOALLOC_SCRATCH_BYTES];

constexpr int NOALLOC_MAX_DEVICES = 64;
static std::mutex g_scratch_mu;
static void* g_scratch_ptr[NOALLOC_MAX_DEVICES] = {};

static int scratch_of_current_device(void** out) {
  int dev = 0;
  int rc = check_hip(hipGetDevice(&dev), "hipGetDevice");
  if (rc) return rc;
  if (dev < 0 || dev >= NOALLOC_MAX_DEVICES) return set_error(FP_EDEVICE, "device %d beyond %d", dev, NOALLOC_MAX_DEVICES);
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    rc = check_hip(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)), "hipGetSymbolAddress(scratch)");
    if (rc) return rc;
    if (!p) return set_error(FP_EDEVICE, "no address for the scratch array on device %d", dev);
    g_scratch_ptr[dev] = p;
  }
  *out = g_scratch_ptr[dev];
  return FP_OK;
}

int run_frame_potential_noalloc(const double* d_trace, int64_t n, int kmax, double* h_F, double* h_se,
                                hipStream_t s) {
  const size_t need = red_scratch_bytes(red_blocks(n));
  if (need > NOALLOC_SCRATCH_BYTES)
    return set_error(FP_ETOOBIG, "reduction needs %zu bytes of scratch, the static array holds %zu", need,
                     NOALLOC_SCRATCH_BYTES);
  void* ws = nullptr;
  int rc = scratch_of_current_device(&ws);
  if (rc) return rc;
  return frame_potential_on(d_trace, n, kmax, h_F, h_se, ws, s, false);
}

// ---- control variate ----------------------------------------------------------
// Welford of r_i = |Tr_i|^{2k} - c g_B[i] over B and of g_C over C.
__global__ void __launch_bounds__(RED_THREADS) cv_kernel(const double* __restrict__ trB,
                                                         const float* __restrict__ gB, int64_t nB,
                                                         const float* __restrict__ gC, int64_t nC, int k,
                                                         double c, Welford* __restrict__ part,
                                                         double* __restrict__ badp) {
  __shared__ Welford sw[RED_THREADS];
  __shared__ double sbad[RED_THREADS];
  Welford wr{0.0, 0.0, 0.0}, wg{0.0, 0.0, 0.0};
  double bad = 0.0;
  for (int64_t i = (int64_t)blockIdx.x * RED_THREADS + threadIdx.x; i < nB;
       i += (int64_t)gridDim.x * RED_THREADS) {
    const double re = trB[2 * i], im = trB[2 * i + 1];
    const double a = re * re + im * im;
    double f = 1.0;
    for (int j = 0; j < k; ++j) f *= a;
    const double r = f - c * (double)gB[i];
    if (!isfinite(r)) bad += 1.0;
    welford_add(wr, r);
  }
  for (int64_t i = (int64_t)blockIdx.x * RED_THREADS + threadIdx.x; i < nC;
       i += (int64_t)gridDim.x * RED_THREADS) {
    const double g = (double)gC[i];
    if (!isfinite(g)) bad += 1.0;
    welford_add(wg, g);
  }
  for (int which = 0; which < 2; ++which) {
    sw[threadIdx.x] = which == 0 ? wr : wg;
    sbad[threadIdx.x] = bad;
    __syncthreads();
    for (int s = RED_THREADS / 2; s > 0; s >>= 1) {
      if (threadIdx.x < s) {
        sw[threadIdx.x] = chan_merge(sw[threadIdx.x], sw[threadIdx.x + s]);
        sbad[threadIdx.x] += sbad[threadIdx.x + s];
      }
      __syncthreads();
    }
    if (threadIdx.x == 0) {
      part[2 * blockIdx.x + which] = sw[0];
      if (which == 0) badp[blockIdx.x] = sbad[0];
    }
    __syncthreads();
  }
}

__global__ void cv_final(const Welford* __restrict__ part, const double* __restrict__ badp, int nb,
                         double c, double* __restrict__ out) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  Welford r{0.0, 0.0, 0.0}, g{0.0, 0.0, 0.0};
  double bad = 0.0;
  for (int b = 0; b < nb; ++b) {
    r = chan_merge(r, part[2 * b]);
    g = chan_merge(g, part[2 * b + 1]);
    bad += badp[b];
  }
  const double est = r.mean + c * g.mean;
  double var = r.n > 1.0 ? r.m2 / (r.n - 1.0) / r.n : 0.0;
  if (g.n > 1.0) var += c * c * (g.m2 / (g.n - 1.0) / g.n);
  out[0] = est;
  out[1] = sqrt(var);
  out[2] = bad;
}

int run_frame_potential_cv(const double* trB, const float* gB, int64_t nB, const float* gC, int64_t nC,
                           int k, double c, double* h_F, double* h_se, hipStream_t s) {
  const int nb = red_blocks(nB > nC ? nB : nC);
  const size_t bytes = sizeof(Welford) * 2 * nb + sizeof(double) * (nb + 3);
  void* ws = nullptr;
  int rc = check_hip(hipMallocAsync(&ws, bytes, s), "hipMallocAsync(cv)");
  if (rc) return rc;
  Welford* part = (Welford*)ws;
  double* badp = (double*)(part + 2 * nb);
  double* out = badp + nb;
  hipLaunchKernelGGL(cv_kernel, dim3(nb), dim3(RED_THREADS), 0, s, trB, gB, nB, gC, nC, k, c, part, badp);
  hipLaunchKernelGGL(cv_final, dim3(1), dim3(64), 0, s, part, badp, nb, c, out);
  rc = check_launch("frame_potential_cv");
  double host[3];
  if (!rc) rc = check_hip(hipMemcpyAsync(host, out, sizeof(host), hipMemcpyDeviceToHost, s), "copy CV");
  int rc2 = check_hip(hipFreeAsync(ws, s), "hipFreeAsync(cv)");
  int rc3 = check_hip(hipStreamSynchronize(s), "sync(cv)");
  if (rc) return rc;
  if (rc2) return rc2;
  if (rc3) return rc3;
  if (host[2] > 0.0) return set_error(FP_ENUMERIC, "%.0f non-finite value(s) in the CV inputs", host[2]);
  *h_F = host[0];
  if (h_se) *h_se = host[1];
  return FP_OK;
}

// ---- surrogate targets and the control-variate coefficient ----------------------
__global__ void __launch_bounds__(256) targets_kernel(const double* __restrict__ tr, int64_t n, int k, double scale,
                                                      float* __restrict__ t) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const double a = tr[2 * i] * tr[2 * i] + tr[2 * i + 1] * tr[2 * i + 1];
  double f = 1.0;
  for (int j = 0; j < k; ++j) f *= a;
  t[i] = (float)(scale * f);
}

// Co-moments of (f, g): count, means, and the sums of products of deviations.
struct Co {
  double n, mf, mg, cfg, m2g, m2f;
};

__device__ __forceinline__ Co co_merge(Co a, Co b) {
  Co r;
  r.n = a.n + b.n;
  if (r.n == 0.0) return Co{0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
  const double df = b.mf - a.mf, dg = b.mg - a.mg, w = a.n * b.n / r.n;
  r.mf = a.mf + df * (b.n / r.n);
  r.mg = a.mg + dg * (b.n / r.n);
  r.cfg = a.cfg + b.cfg + df * dg * w;
  r.m2g = a.m2g + b.m2g + dg * dg * w;
  r.m2f = a.m2f + b.m2f + df * df * w;
  return r;
}

// Per-workgroup co-moments of f = |Tr|^{2k} and g.
__global__ void __launch_bounds__(RED_THREADS) cvcoef_kernel(const double* __restrict__ tr, const float* __restrict__ g,
                                                             int64_t n, int k, Co* __restrict__ part) {
  __shared__ Co sh[RED_THREADS];
  Co c{0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
  for (int64_t i = (int64_t)blockIdx.x * RED_THREADS + threadIdx.x; i < n; i += (int64_t)gridDim.x * RED_THREADS) {
    const double a = tr[2 * i] * tr[2 * i] + tr[2 * i + 1] * tr[2 * i + 1];
    double f = 1.0;
    for (int j = 0; j < k; ++j) f *= a;
    const double gv = (double)g[i];
    c.n += 1.0;
    const double df = f - c.mf, dg = gv - c.mg;
    c.mf += df / c.n;
    c.mg += dg / c.n;
    c.cfg += df * (gv - c.mg);
    c.m2g += dg * (gv - c.mg);
    c.m2f += df * (f - c.mf);
  }
  sh[threadIdx.x] = c;
  __syncthreads();
  for (int s2 = RED_THREADS / 2; s2 > 0; s2 >>= 1) {
    if (threadIdx.x < s2) sh[threadIdx.x] = co_merge(sh[threadIdx.x], sh[threadIdx.x + s2]);
    __syncthreads();
  }
  if (threadIdx.x == 0) part[blockIdx.x] = sh[0];
}

// out: c = Cov(f, g) / Var(g) (0 for constant g), the correlation rho (0
// when either is constant), mean and sample variance of f, then of g.
__global__ void cvcoef_final(const Co* __restrict__ part, int nb, double* __restrict__ out) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  Co a{0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
  for (int b = 0; b < nb; ++b) a = co_merge(a, part[b]);
  out[0] = a.m2g > 0.0 ? a.cfg / a.m2g : 0.0;
  out[1] = a.m2g > 0.0 && a.m2f > 0.0 ? a.cfg / sqrt(a.m2f * a.m2g) : 0.0;
  out[2] = a.mf;
  out[3] = a.n > 1.0 ? a.m2f / (a.n - 1.0) : 0.0;
  out[4] = a.mg;
  out[5] = a.n > 1.0 ? a.m2g / (a.n - 1.0) : 0.0;
}

int run_targets(const double* tr, int64_t n, int k, double scale, float* t, hipStream_t s) {
  hipLaunchKernelGGL(targets_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, tr, n, k, scale, t);
  return check_launch("targets");
}

int run_cv_holdout(const double* tr, const float* g, int64_t n, int k, double* out6, hipStream_t s) {
  const int nb = red_blocks(n);
  void* ws = nullptr;
  int rc = check_hip(hipMallocAsync(&ws, sizeof(Co) * nb + 8 * sizeof(double), s), "hipMallocAsync(cvcoef)");
  if (rc) return rc;
  Co* part = (Co*)ws;
  double* out = (double*)(part + nb);
  hipLaunchKernelGGL(cvcoef_kernel, dim3(nb), dim3(RED_THREADS), 0, s, tr, g, n, k, part);
  hipLaunchKernelGGL(cvcoef_final, dim3(1), dim3(64), 0, s, part, nb, out);
  rc = check_launch("cv_coefficient");
  double host[6] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
  if (!rc) rc = check_hip(hipMemcpyAsync(host, out, sizeof(host), hipMemcpyDeviceToHost, s), "copy c");
  int rc2 = check_hip(hipFreeAsync(ws, s), "hipFreeAsync(cvcoef)");
  int rc3 = check_hip(hipStreamSynchronize(s), "sync(cvcoef)");
  if (rc) return rc;
  if (rc2) return rc2;
  if (rc3) return rc3;
  for (int i = 0; i < 6; ++i) {
    if (!isfinite(host[i])) return set_error(FP_ENUMERIC, "non-finite hold-out statistic %d", i);
    out6[i] = host[i];
  }
  return FP_OK;
}

int run_cv_coefficient(const double* tr, const float* g, int64_t n, int k, double* c_out, hipStream_t s) {
  double st[6];
  int rc = run_cv_holdout(tr, g, n, k, st, s);
  if (rc) return rc;
  *c_out = st[0];
  return FP_OK;
}

// Mean and sample variance of a float array (Welford in float64, fixed order).
__global__ void __launch_bounds__(RED_THREADS) mom32_kernel(const float* __restrict__ x, int64_t n,
                                                            Welford* __restrict__ part) {
  __shared__ Welford sw[RED_THREADS];
  Welford w{0.0, 0.0, 0.0};
  for (int64_t i = (int64_t)blockIdx.x * RED_THREADS + threadIdx.x; i < n; i += (int64_t)gridDim.x * RED_THREADS)
    welford_add(w, (double)x[i]);
  sw[threadIdx.x] = w;
  __syncthreads();
  for (int s2 = RED_THREADS / 2; s2 > 0; s2 >>= 1) {
    if (threadIdx.x < s2) sw[threadIdx.x] = chan_merge(sw[threadIdx.x], sw[threadIdx.x + s2]);
    __syncthreads();
  }
  if (threadIdx.x == 0) part[blockIdx.x] = sw[0];
}

__global__ void mom32_final(const Welford* __restrict__ part, int nb, double* __restrict__ out) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  Welford a{0.0, 0.0, 0.0};
  for (int b = 0; b < nb; ++b) a = chan_merge(a, part[b]);
  out[0] = a.mean;
  out[1] = a.n > 1.0 ? a.m2 / (a.n - 1.0) : 0.0;
}

int run_moments_f32(const float* x, int64_t n, double* mean, double* var, hipStream_t s) {
  const int nb = red_blocks(n);
  void* ws = nullptr;
  int rc = check_hip(hipMallocAsync(&ws, sizeof(Welford) * nb + 2 * sizeof(double), s), "hipMallocAsync(mom32)");
  if (rc) return rc;
  Welford* part = (Welford*)ws;
  double* out = (double*)(part + nb);
  hipLaunchKernelGGL(mom32_kernel, dim3(nb), dim3(RED_THREADS), 0, s, x, n, part);
  hipLaunchKernelGGL(mom32_final, dim3(1), dim3(64), 0, s, part, nb, out);
  rc = check_launch("moments_f32");
  double host[2] = {0.0, 0.0};
  if (!rc) rc = check_hip(hipMemcpyAsync(host, out, sizeof(host), hipMemcpyDeviceToHost, s), "copy moments");
  int rc2 = check_hip(hipFreeAsync(ws, s), "hipFreeAsync(mom32)");
  int rc3 = check_hip(hipStreamSynchronize(s), "sync(mom32)");
  if (rc) return rc;
  if (rc2) return rc2;
  if (rc3) return rc3;
  if (!isfinite(host[0]) || !isfinite(host[1])) return set_error(FP_ENUMERIC, "non-finite values");
  *mean = host[0];
  *var = host[1];
  return FP_OK;
}

// ---- log-space targets of the surrogate -------------------------------------------
// Moments of L_i = log(|Tr_i|^2 + eps) (Welford, float64, fixed order).
__global__ void __launch_bounds__(RED_THREADS) logmom_kernel(const double* __restrict__ tr, int64_t n, double eps,
                                                             Welford* __restrict__ part) {
  __shared__ Welford sw[RED_THREADS];
  Welford w{0.0, 0.0, 0.0};
  for (int64_t i = (int64_t)blockIdx.x * RED_THREADS + threadIdx.x; i < n; i += (int64_t)gridDim.x * RED_THREADS)
    welford_add(w, log(tr[2 * i] * tr[2 * i] + tr[2 * i + 1] * tr[2 * i + 1] + eps));
  sw[threadIdx.x] = w;
  __syncthreads();
  for (int s2 = RED_THREADS / 2; s2 > 0; s2 >>= 1) {
    if (threadIdx.x < s2) sw[threadIdx.x] = chan_merge(sw[threadIdx.x], sw[threadIdx.x + s2]);
    __syncthreads();
  }
  if (threadIdx.x == 0) part[blockIdx.x] = sw[0];
}

__global__ void logmom_final(const Welford* __restrict__ part, int nb, double* __restrict__ out) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  Welford a{0.0, 0.0, 0.0};
  for (int b = 0; b < nb; ++b) a = chan_merge(a, part[b]);
  out[0] = a.mean;
  out[1] = a.n > 1.0 ? sqrt(a.m2 / (a.n - 1.0)) : 0.0;
}

// t_i = (log(|Tr_i|^2 + eps) - mu) / sigma
__global__ void __launch_bounds__(256) logtargets_kernel(const double* __restrict__ tr, int64_t n, double eps, double mu,
                                                         double inv_sigma, float* __restrict__ t) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  t[i] = (float)((log(tr[2 * i] * tr[2 * i] + tr[2 * i + 1] * tr[2 * i + 1] + eps) - mu) * inv_sigma);
}

// g_i = exp(k (mu + sigma y_i) - shift): |Tr|^{2k} predicted from the log-space output, in units of e^shift.
__global__ void __launch_bounds__(256) link_kernel(const float* __restrict__ y, int64_t n, int k, double mu,
                                                   double sigma, double shift, float* __restrict__ g) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const double v = (double)k * (mu + sigma * (double)y[i]) - shift;
  g[i] = (float)exp(v < 80.0 ? v : 80.0);
}

int run_log_moments(const double* tr, int64_t n, double eps, double* mu, double* sigma, hipStream_t s) {
  const int nb = red_blocks(n);
  void* ws = nullptr;
  int rc = check_hip(hipMallocAsync(&ws, sizeof(Welford) * nb + 2 * sizeof(double), s), "hipMallocAsync(logmom)");
  if (rc) return rc;
  Welford* part = (Welford*)ws;
  double* out = (double*)(part + nb);
  hipLaunchKernelGGL(logmom_kernel, dim3(nb), dim3(RED_THREADS), 0, s, tr, n, eps, part);
  hipLaunchKernelGGL(logmom_final, dim3(1), dim3(64), 0, s, part, nb, out);
  rc = check_launch("log_moments");
  double host[2] = {0.0, 0.0};
  if (!rc) rc = check_hip(hipMemcpyAsync(host, out, sizeof(host), hipMemcpyDeviceToHost, s), "copy moments");
  int rc2 = check_hip(hipFreeAsync(ws, s), "hipFreeAsync(logmom)");
  int rc3 = check_hip(hipStreamSynchronize(s), "sync(logmom)");
  if (rc) return rc;
  if (rc2) return rc2;
  if (rc3) return rc3;
  *mu = host[0];
  *sigma = host[1];
  return FP_OK;
}

int run_log_targets(const double* tr, int64_t n, double eps, double mu, double sigma, float* t, hipStream_t s) {
  hipLaunchKernelGGL(logtargets_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, tr, n, eps, mu,
                     sigma > 0.0 ? 1.0 / sigma : 1.0, t);
  return check_launch("log_targets");
}

int run_link(const float* y, int64_t n, int k, double mu, double sigma, double shift, float* g, hipStream_t s) {
  hipLaunchKernelGGL(link_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, y, n, k, mu, sigma, shift, g);
  return check_launch("link");
}

}  // namespace fp
