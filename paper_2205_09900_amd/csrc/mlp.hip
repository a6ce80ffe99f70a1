// Surrogate network of the control variate: features, forward, backward and
// Adam, float32, with the dense products on the MFMA units.
//
// Network: x (n_in) -> SiLU(x W1 + b1) -> SiLU(. W2 + b2) -> SiLU(. W3 + b3)
// -> . w4 + b4.  Loss (1/B) sum_i (y_i - t_i)^2.  Parameters are one float
// buffer: W1 (n_in x H, row-major), b1, W2 (H x H), b2, W3, b3, w4 (H), b4.
// Activations kept for the backward pass: z1, h1, z2, h2, z3, h3 (B x H each).
#include <hip/hip_runtime.h>
#include <math.h>

#include "internal.h"
#include "layout.h"
#include "philox.h"

namespace fp {

typedef float floatx16 __attribute__((ext_vector_type(16)));

__device__ __forceinline__ float sigm(float z) { return 1.0f / (1.0f + __expf(-z)); }
__device__ __forceinline__ float silu(float z) { return z * sigm(z); }
__device__ __forceinline__ float dsilu(float z) {
  const float s = sigm(z);
  return s * (1.0f + z * (1.0f - s));
}

enum { EPI_STORE = 0, EPI_BIAS_SILU = 1, EPI_DSILU = 2 };

// C (M x N) = op(A) (M x K) * op(B) (K x N).  op(A) = A (row-major, lda) or
// A^T (A stored K x M); likewise B.  One 64 x 64 tile per workgroup, four
// wavefronts of 32 x 32 each on v_mfma_f32_32x32x2f32; K in steps of 16
// staged through LDS.  Epilogues: store; z = acc + bias -> C, silu(z) -> H;
// acc * silu'(Z) -> C.
template <int EPI>
__global__ void __launch_bounds__(256) gemm_kernel(int M, int N, int K, const float* __restrict__ A, int lda, int ta,
                                                   const float* __restrict__ B, int ldb, int tb, float* __restrict__ C,
                                                   int ldc, const float* __restrict__ bias, float* __restrict__ H,
                                                   const float* __restrict__ Z) {
  __shared__ float As[16][64 + 4];
  __shared__ float Bs[16][64 + 4];
  const int m0 = blockIdx.y * 64, n0 = blockIdx.x * 64;
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
  const int wm = (wave >> 1) * 32, wn = (wave & 1) * 32;
  floatx16 acc;
#pragma unroll
  for (int r = 0; r < 16; ++r) acc[r] = 0.0f;
  for (int k0 = 0; k0 < K; k0 += 16) {
#pragma unroll
    for (int e = tid; e < 1024; e += 256) {
      int mm, kk;
      if (!ta) {
        mm = e >> 4;
        kk = e & 15;
      } else {
        kk = e >> 6;
        mm = e & 63;
      }
      const int gm = m0 + mm, gk = k0 + kk;
      float v = 0.0f;
      if (gm < M && gk < K) v = ta ? A[(size_t)gk * lda + gm] : A[(size_t)gm * lda + gk];
      As[kk][mm] = v;
    }
#pragma unroll
    for (int e = tid; e < 1024; e += 256) {
      int nn, kk;
      if (!tb) {
        kk = e >> 6;
        nn = e & 63;
      } else {
        nn = e >> 4;
        kk = e & 15;
      }
      const int gn = n0 + nn, gk = k0 + kk;
      float v = 0.0f;
      if (gn < N && gk < K) v = tb ? B[(size_t)gn * ldb + gk] : B[(size_t)gk * ldb + gn];
      Bs[kk][nn] = v;
    }
    __syncthreads();
#pragma unroll
    for (int kk = 0; kk < 16; kk += 2) {
      const float a = As[kk + (lane >> 5)][wm + (lane & 31)];
      const float b = Bs[kk + (lane >> 5)][wn + (lane & 31)];
      acc = __builtin_amdgcn_mfma_f32_32x32x2f32(a, b, acc, 0, 0, 0);
    }
    __syncthreads();
  }
#pragma unroll
  for (int r = 0; r < 16; ++r) {
    const int row = m0 + wm + (r >> 2) * 8 + (lane >> 5) * 4 + (r & 3);
    const int col = n0 + wn + (lane & 31);
    if (row < M && col < N) {
      const float v = acc[r];
      if constexpr (EPI == EPI_STORE) {
        C[(size_t)row * ldc + col] = v;
      } else if constexpr (EPI == EPI_BIAS_SILU) {
        const float z = v + bias[col];
        C[(size_t)row * ldc + col] = z;
        H[(size_t)row * ldc + col] = silu(z);
      } else {
        C[(size_t)row * ldc + col] = v * dsilu(Z[(size_t)row * ldc + col]);
      }
    }
  }
}

template <int EPI>
static void gemm(int M, int N, int K, const float* A, int lda, int ta, const float* B, int ldb, int tb, float* C, int ldc,
                 const float* bias, float* H, const float* Z, hipStream_t s) {
  dim3 grid((N + 63) / 64, (M + 63) / 64);
  hipLaunchKernelGGL((gemm_kernel<EPI>), grid, dim3(256), 0, s, M, N, K, A, lda, ta, B, ldb, tb, C, ldc, bias, H, Z);
}

// y[i] = h3[i] . w4 + b4 (one wavefront per row).
__global__ void __launch_bounds__(256) out_layer_kernel(int Bn, int H, const float* __restrict__ h3,
                                                        const float* __restrict__ w4, const float* __restrict__ b4,
                                                        float* __restrict__ y) {
  const int row = blockIdx.x * 4 + (threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  if (row >= Bn) return;
  float s = 0.0f;
  for (int j = lane; j < H; j += 64) s += h3[(size_t)row * H + j] * w4[j];
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) s += __shfl_xor(s, off, 64);
  if (lane == 0) y[row] = s + b4[0];
}

// dy_i = 2 (y_i - t_i) / B; dz3 = dy w4^T * silu'(z3); per-row squared errors.
__global__ void __launch_bounds__(256) out_backward_kernel(int Bn, int H, const float* __restrict__ y,
                                                           const float* __restrict__ t, const float* __restrict__ w4,
                                                           const float* __restrict__ z3, float* __restrict__ dy,
                                                           float* __restrict__ dz3, float* __restrict__ sq) {
  const int row = blockIdx.x;
  if (row >= Bn) return;
  const float r = y[row] - t[row];
  const float d = 2.0f * r / (float)Bn;
  if (threadIdx.x == 0) {
    dy[row] = d;
    sq[row] = r * r;
  }
  for (int j = threadIdx.x; j < H; j += blockDim.x)
    dz3[(size_t)row * H + j] = d * w4[j] * dsilu(z3[(size_t)row * H + j]);
}

// out[j] = sum_i X[i][j] (column sums, fixed order) ; optionally the sum of v.
__global__ void __launch_bounds__(256) colsum_kernel(int rows, int cols, const float* __restrict__ X,
                                                     float* __restrict__ out) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= cols) return;
  float s = 0.0f;
  for (int i = 0; i < rows; ++i) s += X[(size_t)i * cols + j];
  out[j] = s;
}

// gw4[j] = sum_i h3[i][j] dy[i]; gb4 = sum_i dy[i].
__global__ void __launch_bounds__(256) outgrad_kernel(int Bn, int H, const float* __restrict__ h3,
                                                      const float* __restrict__ dy, float* __restrict__ gw4,
                                                      float* __restrict__ gb4) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j > H) return;
  float s = 0.0f;
  if (j < H) {
    for (int i = 0; i < Bn; ++i) s += h3[(size_t)i * H + j] * dy[i];
    gw4[j] = s;
  } else {
    for (int i = 0; i < Bn; ++i) s += dy[i];
    gb4[0] = s;
  }
}

__global__ void __launch_bounds__(256) sum_kernel(int n, const float* __restrict__ v, double* __restrict__ out) {
  __shared__ double sh[256];
  double s = 0.0;
  for (int i = threadIdx.x; i < n; i += 256) s += (double)v[i];
  sh[threadIdx.x] = s;
  __syncthreads();
  for (int k = 128; k > 0; k >>= 1) {
    if (threadIdx.x < k) sh[threadIdx.x] += sh[threadIdx.x + k];
    __syncthreads();
  }
  if (threadIdx.x == 0) out[0] = sh[0];
}

__global__ void __launch_bounds__(256) adam_kernel(int64_t n, float* __restrict__ p, const float* __restrict__ g,
                                                   float* __restrict__ m, float* __restrict__ v, float lr, float b1,
                                                   float b2, float eps, float c1, float c2) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const float gi = g[i];
  const float mi = b1 * m[i] + (1.0f - b1) * gi;
  const float vi = b2 * v[i] + (1.0f - b2) * gi * gi;
  m[i] = mi;
  v[i] = vi;
  p[i] -= lr * (mi / c1) / (sqrtf(vi / c2) + eps);
}

// Uniform(-1/sqrt(fan_in), 1/sqrt(fan_in)) weights from Philox, zero biases.
__global__ void __launch_bounds__(256) init_kernel(int64_t n, int n_in, int H, uint64_t seed, float* __restrict__ p) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const int64_t s1 = (int64_t)n_in * H, s2 = s1 + H, s3 = s2 + (int64_t)H * H, s4 = s3 + H;
  const int64_t s5 = s4 + (int64_t)H * H, s6 = s5 + H, s7 = s6 + H;
  float fan;
  if (i < s1)
    fan = (float)n_in;
  else if (i < s2)
    fan = 0.0f;
  else if (i < s3)
    fan = (float)H;
  else if (i < s4)
    fan = 0.0f;
  else if (i < s5)
    fan = (float)H;
  else if (i < s6)
    fan = 0.0f;
  else if (i < s7)
    fan = (float)H;
  else
    fan = 0.0f;
  if (fan == 0.0f) {
    p[i] = 0.0f;
    return;
  }
  const u32x4 x = philox4x32_10((uint32_t)i, (uint32_t)(i >> 32), 0x4D4C5000u, 0u, (uint32_t)seed,
                                (uint32_t)(seed >> 32));
  const double u = u53(x.v[0], x.v[1]);
  p[i] = (float)((2.0 * u - 1.0) / sqrt((double)fan));
}

// Features of HEA pairs: sin and cos of every angle, circuit U then V, layer,
// qubit, (theta, phi).  Angles are float32 (FP_C64 gate layout).
__global__ void __launch_bounds__(256) features_kernel(int64_t num_pairs, int n, int L, const unsigned char* __restrict__ g,
                                                       int64_t stride, float* __restrict__ x) {
  const int64_t nang = 4 * (int64_t)n * L;  // angles per pair
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= num_pairs * nang) return;
  const int64_t p = idx / nang, a = idx % nang;
  const float ang = reinterpret_cast<const float*>(g + p * stride)[a];
  float s, c;
  sincosf(ang, &s, &c);
  x[p * 2 * nang + 2 * a] = s;
  x[p * 2 * nang + 2 * a + 1] = c;
}

struct Params {
  const float *W1, *b1, *W2, *b2, *W3, *b3, *w4, *b4;
};

static Params split(const float* p, int n_in, int H) {
  Params q;
  q.W1 = p;
  q.b1 = q.W1 + (size_t)n_in * H;
  q.W2 = q.b1 + H;
  q.b2 = q.W2 + (size_t)H * H;
  q.W3 = q.b2 + H;
  q.b3 = q.W3 + (size_t)H * H;
  q.w4 = q.b3 + H;
  q.b4 = q.w4 + H;
  return q;
}

int mlp_forward(int n_in, int H, int64_t Bn, const float* params, const float* x, float* y, float* act, hipStream_t s) {
  float* tmp = nullptr;
  if (!act) {
    int rc = check_hip(hipMallocAsync(&tmp, sizeof(float) * 6 * (size_t)Bn * H, s), "hipMallocAsync(mlp)");
    if (rc) return rc;
    act = tmp;
  }
  const Params P = split(params, n_in, H);
  float *z1 = act, *h1 = z1 + Bn * H, *z2 = h1 + Bn * H, *h2 = z2 + Bn * H, *z3 = h2 + Bn * H, *h3 = z3 + Bn * H;
  gemm<EPI_BIAS_SILU>((int)Bn, H, n_in, x, n_in, 0, P.W1, H, 0, z1, H, P.b1, h1, nullptr, s);
  gemm<EPI_BIAS_SILU>((int)Bn, H, H, h1, H, 0, P.W2, H, 0, z2, H, P.b2, h2, nullptr, s);
  gemm<EPI_BIAS_SILU>((int)Bn, H, H, h2, H, 0, P.W3, H, 0, z3, H, P.b3, h3, nullptr, s);
  hipLaunchKernelGGL(out_layer_kernel, dim3((unsigned)((Bn + 3) / 4)), dim3(256), 0, s, (int)Bn, H, h3, P.w4, P.b4, y);
  int rc = check_launch("mlp_forward");
  if (tmp) {
    int rc2 = check_hip(hipFreeAsync(tmp, s), "hipFreeAsync(mlp)");
    if (!rc) rc = rc2;
  }
  return rc;
}

int mlp_backward(int n_in, int H, int64_t Bn, const float* params, const float* x, const float* act, const float* t,
                 float* grad, double* h_loss, hipStream_t s) {
  const Params P = split(params, n_in, H);
  const float *z1 = act, *h1 = z1 + Bn * H, *z2 = h1 + Bn * H, *h2 = z2 + Bn * H, *z3 = h2 + Bn * H, *h3 = z3 + Bn * H;
  float* G = grad;
  float *gW1 = G, *gb1 = gW1 + (size_t)n_in * H, *gW2 = gb1 + H, *gb2 = gW2 + (size_t)H * H, *gW3 = gb2 + H;
  float *gb3 = gW3 + (size_t)H * H, *gw4 = gb3 + H, *gb4 = gw4 + H;
  float* tmp = nullptr;
  const size_t tmp_floats = 2 * (size_t)Bn * H + 3 * (size_t)Bn + 2;
  int rc = check_hip(hipMallocAsync(&tmp, sizeof(float) * tmp_floats, s), "hipMallocAsync(mlp)");
  if (rc) return rc;
  float *dza = tmp, *dzb = dza + Bn * H, *y = dzb + Bn * H, *dy = y + Bn, *sq = dy + Bn;
  // forward output from the stored activations
  hipLaunchKernelGGL(out_layer_kernel, dim3((unsigned)((Bn + 3) / 4)), dim3(256), 0, s, (int)Bn, H, h3, P.w4, P.b4, y);
  hipLaunchKernelGGL(out_backward_kernel, dim3((unsigned)Bn), dim3(256), 0, s, (int)Bn, H, y, t, P.w4, z3, dy, dza, sq);
  hipLaunchKernelGGL(outgrad_kernel, dim3((H + 1 + 255) / 256), dim3(256), 0, s, (int)Bn, H, h3, dy, gw4, gb4);
  // layer 3: dz3 in dza
  gemm<EPI_STORE>(H, H, (int)Bn, h2, H, 1, dza, H, 0, gW3, H, nullptr, nullptr, nullptr, s);
  hipLaunchKernelGGL(colsum_kernel, dim3((H + 255) / 256), dim3(256), 0, s, (int)Bn, H, dza, gb3);
  gemm<EPI_DSILU>((int)Bn, H, H, dza, H, 0, P.W3, H, 1, dzb, H, nullptr, nullptr, z2, s);  // dz2
  // layer 2: dz2 in dzb
  gemm<EPI_STORE>(H, H, (int)Bn, h1, H, 1, dzb, H, 0, gW2, H, nullptr, nullptr, nullptr, s);
  hipLaunchKernelGGL(colsum_kernel, dim3((H + 255) / 256), dim3(256), 0, s, (int)Bn, H, dzb, gb2);
  gemm<EPI_DSILU>((int)Bn, H, H, dzb, H, 0, P.W2, H, 1, dza, H, nullptr, nullptr, z1, s);  // dz1
  // layer 1: dz1 in dza
  gemm<EPI_STORE>(n_in, H, (int)Bn, x, n_in, 1, dza, H, 0, gW1, H, nullptr, nullptr, nullptr, s);
  hipLaunchKernelGGL(colsum_kernel, dim3((H + 255) / 256), dim3(256), 0, s, (int)Bn, H, dza, gb1);
  rc = check_launch("mlp_backward");
  double loss_sum = 0.0;
  if (!rc && h_loss) {
    double* dsum = nullptr;
    rc = check_hip(hipMallocAsync(&dsum, sizeof(double), s), "hipMallocAsync(loss)");
    if (!rc) {
      hipLaunchKernelGGL(sum_kernel, dim3(1), dim3(256), 0, s, (int)Bn, sq, dsum);
      rc = check_hip(hipMemcpyAsync(&loss_sum, dsum, sizeof(double), hipMemcpyDeviceToHost, s), "copy loss");
      int rc2 = check_hip(hipFreeAsync(dsum, s), "hipFreeAsync(loss)");
      if (!rc) rc = rc2;
    }
  }
  int rc2 = check_hip(hipFreeAsync(tmp, s), "hipFreeAsync(mlp)");
  if (!rc) rc = rc2;
  if (!rc && h_loss) {
    rc = check_hip(hipStreamSynchronize(s), "sync(loss)");
    *h_loss = loss_sum / (double)Bn;
  }
  return rc;
}

int mlp_gemm_test(int M, int N, int K, const float* A, int lda, int ta, const float* B, int ldb, int tb, float* C,
                  int ldc, hipStream_t s) {
  gemm<EPI_STORE>(M, N, K, A, lda, ta, B, ldb, tb, C, ldc, nullptr, nullptr, nullptr, s);
  return check_launch("gemm");
}

int mlp_adam(int64_t n, float* p, const float* g, float* adam, int step, float lr, float b1, float b2, float eps,
             hipStream_t s) {
  const float c1 = 1.0f - powf(b1, (float)step), c2 = 1.0f - powf(b2, (float)step);
  hipLaunchKernelGGL(adam_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, n, p, g, adam, adam + n, lr, b1,
                     b2, eps, c1, c2);
  return check_launch("adam");
}

int mlp_init(int n_in, int H, uint64_t seed, float* p, hipStream_t s) {
  const int64_t n = (int64_t)n_in * H + H + 2 * ((int64_t)H * H + H) + H + 1;
  hipLaunchKernelGGL(init_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, n, n_in, H, seed, p);
  return check_launch("mlp_init");
}

int mlp_features(const fp_ensemble_t* e, int64_t num_pairs, const void* gates, float* x, hipStream_t s) {
  const int64_t stride = pair_bytes(FP_HEA_RYRZ_CZ, e->n_qubits, e->depth, FP_C64);
  const int64_t work = num_pairs * 4 * (int64_t)e->n_qubits * e->depth;
  hipLaunchKernelGGL(features_kernel, dim3((unsigned)((work + 255) / 256)), dim3(256), 0, s, num_pairs, e->n_qubits,
                     e->depth, (const unsigned char*)gates, stride, x);
  return check_launch("mlp_features");
}

}  // namespace fp
