// fp_sample_gates kernels: the ensembles of the paper (Results, Fig. 2) drawn
// from one Philox4x32-10 counter stream (see fp.h for the counter layout).
#include <hip/hip_runtime.h>
#include <math.h>

#include "internal.h"
#include "layout.h"
#include "philox.h"

namespace fp {

struct dcplx {
  double x, y;
};

// Haar U(4): complex Gaussian (Box-Muller) -> Q factor with positive real R
// diagonal (Mezzadri 2007), computed by classical Gram-Schmidt applied twice,
// which reproduces the unique factor to rounding.
__device__ inline void haar_u4(uint64_t seed, uint64_t pair, uint32_t circuit, uint32_t gate,
                               dcplx q[4][4]) {
  dcplx z[4][4];
#pragma unroll
  for (int w = 0; w < 16; ++w) {
    u32x4 x = draw(seed, (uint32_t)w, gate, pair, circuit);
    const double u1 = u53(x.v[0], x.v[1]);
    const double u2 = u53(x.v[2], x.v[3]);
    const double r = sqrt(-2.0 * log(u1));
    double s, c;
    sincospi(2.0 * u2, &s, &c);  // sin and cos of 2 pi u2, without rounding 2 pi u2 first
    z[w >> 2][w & 3].x = r * c;
    z[w >> 2][w & 3].y = r * s;
  }
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    dcplx v[4];
#pragma unroll
    for (int a = 0; a < 4; ++a) v[a] = z[a][j];
#pragma unroll
    for (int pass = 0; pass < 2; ++pass) {
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        if (i >= j) break;
        double rr = 0.0, ri = 0.0;  // <q_i, v>
#pragma unroll
        for (int a = 0; a < 4; ++a) {
          rr += q[a][i].x * v[a].x + q[a][i].y * v[a].y;
          ri += q[a][i].x * v[a].y - q[a][i].y * v[a].x;
        }
#pragma unroll
        for (int a = 0; a < 4; ++a) {
          v[a].x -= rr * q[a][i].x - ri * q[a][i].y;
          v[a].y -= rr * q[a][i].y + ri * q[a][i].x;
        }
      }
    }
    double nrm = 0.0;
#pragma unroll
    for (int a = 0; a < 4; ++a) nrm += v[a].x * v[a].x + v[a].y * v[a].y;
    const double inv = 1.0 / sqrt(nrm);
#pragma unroll
    for (int a = 0; a < 4; ++a) {
      q[a][j].x = v[a].x * inv;
      q[a][j].y = v[a].y * inv;
    }
  }
}

template <typename Real>
__global__ void __launch_bounds__(256) sample_haar_kernel(Real* __restrict__ gates, int64_t num_pairs,
                                                          uint64_t seed, uint64_t first_pair, int ansatz,
                                                          int n, int depth, int G, int64_t stride_bytes,
                                                          int64_t bonds_off) {
  const int64_t tid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t per_pair = 2 * (int64_t)G;
  if (tid >= num_pairs * per_pair) return;
  const int64_t p = tid / per_pair;
  const int rem = (int)(tid % per_pair);
  const uint32_t circuit = (uint32_t)(rem / G);
  const uint32_t g = (uint32_t)(rem % G);
  const uint64_t pair = first_pair + (uint64_t)p;
  dcplx q[4][4];
  haar_u4(seed, pair, circuit, g, q);
  char* base = reinterpret_cast<char*>(gates) + p * stride_bytes;
  Real* dst = reinterpret_cast<Real*>(base) + ((int64_t)circuit * G + g) * 32;
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int b = 0; b < 4; ++b) {
      dst[(a * 4 + b) * 2] = (Real)q[a][b].x;
      dst[(a * 4 + b) * 2 + 1] = (Real)q[a][b].y;
    }
  if (ansatz == FP_LOCAL_RANDOM_HAAR) {
    int32_t* bonds = reinterpret_cast<int32_t*>(base + bonds_off);
    bonds[(int64_t)circuit * G + g] = sample_bond(seed, pair, circuit, g, n);
  }
}

template <typename Real>
__global__ void __launch_bounds__(256) sample_hea_kernel(Real* __restrict__ gates, int64_t num_pairs,
                                                         uint64_t seed, uint64_t first_pair, int n,
                                                         int layers, int64_t stride_bytes) {
  const int64_t tid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t per_circ = (int64_t)layers * n;
  if (tid >= num_pairs * 2 * per_circ) return;
  const int64_t p = tid / (2 * per_circ);
  const int rem = (int)(tid % (2 * per_circ));
  const uint32_t circuit = (uint32_t)(rem / per_circ);
  const uint32_t item = (uint32_t)(rem % per_circ);  // l * n + q
  const uint64_t pair = first_pair + (uint64_t)p;
  u32x4 x = draw(seed, 0u, item, pair, circuit);
  const double two_pi = 6.283185307179586;
  const double theta = two_pi * u53(x.v[0], x.v[1]);
  const double phi = two_pi * u53(x.v[2], x.v[3]);
  Real* dst = reinterpret_cast<Real*>(reinterpret_cast<char*>(gates) + p * stride_bytes) +
              ((int64_t)circuit * per_circ + item) * 2;
  dst[0] = (Real)theta;
  dst[1] = (Real)phi;
}

// Pauli-rotation HEA: one thread per (pair, circuit, layer, qubit) writes
// (theta, axis); the axis comes from the first of x0, x1 below 2^32 - 1
// (2^32 - 1 is a multiple of 3, so x mod 3 is uniform), theta from x2, x3.
template <typename Real>
__global__ void __launch_bounds__(256) sample_pauli_kernel(Real* __restrict__ gates, int64_t num_pairs,
                                                           uint64_t seed, uint64_t first_pair, int n,
                                                           int layers, int64_t stride_bytes) {
  const int64_t tid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t per_circ = (int64_t)layers * n;
  if (tid >= num_pairs * 2 * per_circ) return;
  const int64_t p = tid / (2 * per_circ);
  const int rem = (int)(tid % (2 * per_circ));
  const uint32_t circuit = (uint32_t)(rem / per_circ);
  const uint32_t item = (uint32_t)(rem % per_circ);  // l * n + q
  const uint64_t pair = first_pair + (uint64_t)p;
  u32x4 x = draw(seed, 0u, item, pair, circuit);
  const uint32_t top = 0xFFFFFFFFu;
  const uint32_t axis = x.v[0] < top ? x.v[0] % 3u : x.v[1] < top ? x.v[1] % 3u : 0u;
  const double theta = 6.283185307179586 * u53(x.v[2], x.v[3]);
  Real* dst = reinterpret_cast<Real*>(reinterpret_cast<char*>(gates) + p * stride_bytes) +
              ((int64_t)circuit * per_circ + item) * 2;
  dst[0] = (Real)theta;
  dst[1] = (Real)axis;
}

int launch_sample(const fp_ensemble_t* e, int64_t num_pairs, uint64_t seed, uint64_t first_pair,
                  int precision, void* d_gates, hipStream_t stream) {
  if (e->ansatz == FP_BRICKWORK_QUDIT) return launch_sample_qudit(e, num_pairs, seed, first_pair, precision, d_gates, stream);
  const int64_t stride = pair_bytes(e->ansatz, e->n_qubits, e->depth, precision, e->local_dim);
  const int threads = 256;
  if (is_pauli_hea(e->ansatz)) {
    const int64_t work = num_pairs * 2 * (int64_t)e->depth * e->n_qubits;
    const int64_t blocks = (work + threads - 1) / threads;
    if (precision == FP_C128)
      hipLaunchKernelGGL(sample_pauli_kernel<double>, dim3((unsigned)blocks), dim3(threads), 0, stream,
                         (double*)d_gates, num_pairs, seed, first_pair, e->n_qubits, e->depth, stride);
    else
      hipLaunchKernelGGL(sample_pauli_kernel<float>, dim3((unsigned)blocks), dim3(threads), 0, stream,
                         (float*)d_gates, num_pairs, seed, first_pair, e->n_qubits, e->depth, stride);
  } else if (e->ansatz == FP_HEA_RYRZ_CZ) {
    const int64_t work = num_pairs * 2 * (int64_t)e->depth * e->n_qubits;
    const int64_t blocks = (work + threads - 1) / threads;
    if (precision == FP_C128)
      hipLaunchKernelGGL(sample_hea_kernel<double>, dim3((unsigned)blocks), dim3(threads), 0, stream,
                         (double*)d_gates, num_pairs, seed, first_pair, e->n_qubits, e->depth, stride);
    else
      hipLaunchKernelGGL(sample_hea_kernel<float>, dim3((unsigned)blocks), dim3(threads), 0, stream,
                         (float*)d_gates, num_pairs, seed, first_pair, e->n_qubits, e->depth, stride);
  } else {
    const int G = (int)gates_per_circuit(e->ansatz, e->n_qubits, e->depth);
    const int64_t work = num_pairs * 2 * (int64_t)G;
    const int64_t blocks = (work + threads - 1) / threads;
    const int64_t boff = bonds_offset(e->n_qubits, e->depth, precision);
    if (precision == FP_C128)
      hipLaunchKernelGGL(sample_haar_kernel<double>, dim3((unsigned)blocks), dim3(threads), 0, stream,
                         (double*)d_gates, num_pairs, seed, first_pair, e->ansatz, e->n_qubits, e->depth,
                         G, stride, boff);
    else
      hipLaunchKernelGGL(sample_haar_kernel<float>, dim3((unsigned)blocks), dim3(threads), 0, stream,
                         (float*)d_gates, num_pairs, seed, first_pair, e->ansatz, e->n_qubits, e->depth,
                         G, stride, boff);
  }
  return check_launch("sample_gates");
}

}  // namespace fp
