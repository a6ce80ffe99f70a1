// Brickwork circuits of qudits (local dimension Q, Haar U(Q^2) gates): the
// paper's generalisation of the trace network to qudits (Sec. II.A: the
// generalised Hadamard and SUM gates), contracted along the qudit direction.
//
// The register program of a brickwork (plan.h) describes which wire segments
// the boundary carries, one register position per segment, whatever the
// local dimension: a qudit brickwork runs the same program with base-Q
// digits in place of bits.  GATE on digits (p, q) applies the realigned
// Q^2 x Q^2 matrix R[(y_in + Q y_out), (x_in + Q x_out)] =
// M[Q x_out + y_out][Q x_in + y_in] of the merged gate M to every group of
// Q^2 entries that differ in those digits; BELL appends two digits holding a
// delta; TRACE sums the entries whose digits p and q agree and removes both.
// The register lives in LDS (one pair per workgroup); after every column it
// is rescaled by a power of two with the exponent kept in float64.
//
// Sampling: one segment of 16 or 32 lanes per gate, lane r holding row r of a
// Q^2 x Q^2 complex Gaussian matrix (Philox4x32-10 block (w, gate, pair, circuit) for
// entry w = r Q^2 + c, Box-Muller in float64), made unitary by Gram-Schmidt
// over the columns (two projection passes per column), which gives the Q
// factor of the QR decomposition with a positive real R diagonal (Mezzadri
// 2007).
#include <hip/hip_runtime.h>
#include <math.h>

#include "dispatch.h"
#include "internal.h"
#include "layout.h"
#include "philox.h"
#include "plan.h"
#include "sweep.h"
#include "sweep_dev.h"

namespace fp {

namespace {

// Sum over the W lanes of a W-lane segment of the wavefront (W a power of two).
template <int W>
__device__ __forceinline__ double seg_sum(double v) {
#pragma unroll
  for (int off = W / 2; off > 0; off >>= 1) v += __shfl_xor(v, off, W);
  return v;
}

}  // namespace

// Lanes per gate (a power of two holding the Q^2 rows), gates per wavefront
// and wavefronts per workgroup of the sampler.
template <int Q>
struct QuditSampleShape {
  static constexpr int D = Q * Q;
  static constexpr int L = D <= 16 ? 16 : 32;
  static constexpr int S = 64 / L;
  static constexpr int WAVES = D <= 9 ? 4 : 2;  // static LDS within 64 KiB
};

// Gate buffer of one pair: [U gates][V gates], each gate Q^4 complex (row-major).
// Each L-lane segment of a wavefront draws one gate: lane r holds row r in
// LDS and every reduction over the rows is a segment shuffle.
template <typename Real, int Q>
__global__ void __launch_bounds__(64 * QuditSampleShape<Q>::WAVES)
    sample_qudit_kernel(Real* __restrict__ gates, int64_t num_pairs, uint64_t seed, uint64_t first_pair, int G,
                        int64_t stride_bytes) {
  using Sh = QuditSampleShape<Q>;
  constexpr int D = Sh::D, L = Sh::L, S = Sh::S;
  __shared__ double mre[Sh::WAVES * S][D][D + 1], mim[Sh::WAVES * S][D][D + 1];  // per gate, [row][col]
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int seg = lane / L, r = lane % L;
  const int64_t total = num_pairs * 2 * G;
  const int64_t gid0 = ((int64_t)blockIdx.x * Sh::WAVES + wave) * S + seg;  // (pair, circuit, gate)
  // a segment past the end repeats the last gate and stores nothing, so that
  // every lane of the wavefront takes part in the shuffles
  const bool valid = gid0 < total;
  const int64_t gid = valid ? gid0 : total - 1;
  const int64_t p = gid / (2 * G);
  const int rem = (int)(gid % (2 * G));
  const uint32_t circuit = (uint32_t)(rem / G), g = (uint32_t)(rem % G);
  const uint64_t pair = first_pair + (uint64_t)p;
  double(*Ar)[D + 1] = mre[wave * S + seg];
  double(*Ai)[D + 1] = mim[wave * S + seg];
  if (r < D) {
    for (int c = 0; c < D; ++c) {
      const u32x4 x = draw(seed, (uint32_t)(r * D + c), g, pair, circuit);
      const double u1 = u53(x.v[0], x.v[1]), u2 = u53(x.v[2], x.v[3]);
      const double rad = sqrt(-2.0 * log(u1));
      double sn, co;
      sincospi(2.0 * u2, &sn, &co);
      Ar[r][c] = rad * co;
      Ai[r][c] = rad * sn;
    }
  }
  __builtin_amdgcn_wave_barrier();
  // Gram-Schmidt column by column, two projection passes per column (lane r:
  // row r; a lane reads and writes only its own row, the column sums are
  // segment shuffles)
  for (int j = 0; j < D; ++j) {
    for (int pass = 0; pass < 2; ++pass) {
      for (int k = 0; k < j; ++k) {
        // c = <Q_k, A_j> = sum_r conj(Q[r][k]) A[r][j]
        double cr = 0.0, ci = 0.0;
        if (r < D) {
          cr = Ar[r][k] * Ar[r][j] + Ai[r][k] * Ai[r][j];
          ci = Ar[r][k] * Ai[r][j] - Ai[r][k] * Ar[r][j];
        }
        cr = seg_sum<L>(cr);
        ci = seg_sum<L>(ci);
        if (r < D) {
          const double qr = Ar[r][k], qi = Ai[r][k];
          Ar[r][j] -= cr * qr - ci * qi;
          Ai[r][j] -= cr * qi + ci * qr;
        }
      }
    }
    double nn = r < D ? Ar[r][j] * Ar[r][j] + Ai[r][j] * Ai[r][j] : 0.0;
    nn = seg_sum<L>(nn);
    const double inv = nn > 0.0 ? 1.0 / sqrt(nn) : 0.0;
    if (r < D) {
      Ar[r][j] *= inv;
      Ai[r][j] *= inv;
    }
  }
  if (!valid) return;
  Real* dst = reinterpret_cast<Real*>(reinterpret_cast<char*>(gates) + p * stride_bytes) +
              ((int64_t)circuit * G + g) * 2 * D * D;
  if (r < D)
    for (int c = 0; c < D; ++c) {
      dst[2 * (r * D + c)] = (Real)Ar[r][c];
      dst[2 * (r * D + c) + 1] = (Real)Ai[r][c];
    }
}

int launch_sample_qudit(const fp_ensemble_t* e, int64_t num_pairs, uint64_t seed, uint64_t first_pair, int precision,
                        void* d_gates, hipStream_t s) {
  const int q = e->local_dim;
  const int G = (int)gates_per_circuit(FP_BRICKWORK_HAAR, e->n_qubits, e->depth);
  const int64_t stride = pair_bytes(e->ansatz, e->n_qubits, e->depth, precision, e->local_dim);
  const int64_t total = num_pairs * 2 * G;
#define FP_QS(QV)                                                                                                   \
  {                                                                                                                 \
    using Sh = QuditSampleShape<QV>;                                                                                \
    const dim3 grid((unsigned)((total + Sh::WAVES * Sh::S - 1) / (Sh::WAVES * Sh::S))), block(64 * Sh::WAVES);      \
    if (precision == FP_C128)                                                                                       \
      hipLaunchKernelGGL((sample_qudit_kernel<double, QV>), grid, block, 0, s, (double*)d_gates, num_pairs, seed,   \
                         first_pair, G, stride);                                                                    \
    else                                                                                                            \
      hipLaunchKernelGGL((sample_qudit_kernel<float, QV>), grid, block, 0, s, (float*)d_gates, num_pairs, seed,     \
                         first_pair, G, stride);                                                                    \
  }
  if (q == 3) {
    FP_QS(3)
  } else if (q == 4) {
    FP_QS(4)
  } else if (q == 5) {
    FP_QS(5)
  } else {
    return set_error(FP_EINVAL, "local dimension %d outside 3..5", q);
  }
#undef FP_QS
  return check_launch("sample_qudit");
}

// ---- the column sweep -----------------------------------------------------------

constexpr int QNT = 256;  // lanes per pair (one pair per workgroup)

// Index with zero digits inserted at positions p < q (pw[k] = Q^k).
__device__ __forceinline__ int insert_digits(int j, int p, int q, const int* pw) {
  // insert at p, then at q (q counts positions of the result)
  const int lo = j % pw[p];
  int t = (j / pw[p]) * pw[p + 1] + lo;
  const int lo2 = t % pw[q];
  return (t / pw[q]) * pw[q + 1] + lo2;
}

template <typename Real, int Q, bool BF3>
__global__ void __launch_bounds__(QNT) qudit_kernel(const unsigned char* __restrict__ gates, int64_t gate_stride,
                                                    int G, const Op* __restrict__ ops, int num_ops,
                                                    const int2* __restrict__ wg, const int32_t* __restrict__ fac,
                                                    int peak, int untouched, double* __restrict__ trace,
                                                    int64_t trace_offset, int64_t num_pairs) {
  constexpr int D = Q * Q;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  __shared__ double mr[2][D * D], mi[2][D * D];  // merged-gate product, double buffer
  __shared__ Real Rr[D * D], Ri[D * D];          // realigned matrix of the current GATE
  __shared__ Real red[16];
  __shared__ int pw[24];
  const int lane = threadIdx.x;
  const int64_t pi = blockIdx.x;
  if (pi >= num_pairs) return;
  Cplx<Real>* B = reinterpret_cast<Cplx<Real>*>(smem_raw);
  const Real* pg = reinterpret_cast<const Real*>(gates + pi * gate_stride);
  if (lane <= peak + 1) {  // q^(peak+1) stays far below 2^31 for registers that fit LDS
    int v = 1;
    for (int k = 0; k < lane; ++k) v *= Q;
    pw[lane] = v;
  }
  if (lane == 0) {
    B[0].x = (Real)1;
    B[0].y = (Real)0;
  }
  __syncthreads();
  int b = 0;
  int64_t expo = 0;
  int pend = 0;
  bool prev_track = false;
  Real lmax = 0;
  for (int t = 0; t < num_ops; ++t) {
    const Op op = ops[t];
    const int type = op.type & OP_TYPE_MASK;
    const bool track = (op.type & OP_FLAG_TRACK) != 0;
    const int p = op.p, q = op.q;
    if (type == OP_GATE) {
      // merged gate M = F_last ... F_first (factors of V as stored, of U
      // conjugate-transposed), in float64
      const int2 w = wg[op.arg];
      int cur = 0;
      for (int f = 0; f < w.y; ++f) {
        const FactorRef fr = decode_factor(fac[w.x + f], G);
        const Real* gm = pg + ((int64_t)fr.circuit * G + fr.gate) * 2 * D * D;
        for (int e = lane; e < D * D; e += QNT) {
          const int row = e / D, col = e % D;
          if (f == 0) {
            const int src = fr.dagger ? col * D + row : row * D + col;
            mr[0][e] = (double)gm[2 * src];
            mi[0][e] = fr.dagger ? -(double)gm[2 * src + 1] : (double)gm[2 * src + 1];
          } else {
            double sr = 0.0, si = 0.0;
            for (int k = 0; k < D; ++k) {
              const int src = fr.dagger ? k * D + row : row * D + k;
              const double ar = (double)gm[2 * src], ai = fr.dagger ? -(double)gm[2 * src + 1] : (double)gm[2 * src + 1];
              const double br = mr[cur][k * D + col], bi = mi[cur][k * D + col];
              sr += ar * br - ai * bi;
              si += ar * bi + ai * br;
            }
            mr[cur ^ 1][e] = sr;
            mi[cur ^ 1][e] = si;
          }
        }
        if (f > 0) cur ^= 1;
        __syncthreads();
      }
      // realign, with the column's pending power of two taken out
      for (int e = lane; e < D * D; e += QNT) {
        const int jp = e / D, j = e % D;
        const int yin = jp % Q, yout = jp / Q, xin = j % Q, xout = j / Q;
        const int src = (Q * xout + yout) * D + (Q * xin + yin);
        Rr[e] = (Real)ldexp(mr[cur][src], -pend);
        Ri[e] = (Real)ldexp(mi[cur][src], -pend);
      }
      __syncthreads();
      expo += pend;
      pend = 0;
      const int ng = pw[b - 2];
      const int sp = pw[p], sq = pw[q];
      const int lo = p < q ? p : q, hi = p < q ? q : p;
      for (int gi = lane; gi < ng; gi += QNT) {
        const int base = insert_digits(gi, lo, hi, pw);
        Cplx<Real> v[D];
#pragma unroll
        for (int j = 0; j < D; ++j) v[j] = B[base + (j % Q) * sp + (j / Q) * sq];
        // the group's inputs are all in registers, so each output can be
        // stored as soon as it is formed (one output row at a time keeps the
        // register count at the inputs plus one accumulator)
#pragma unroll 1
        for (int jp = 0; jp < D; ++jp) {
          Real sr = 0, si = 0;
#pragma unroll
          for (int j = 0; j < D; ++j) cmac<Real, BF3>(Rr[jp * D + j], Ri[jp * D + j], v[j].x, v[j].y, sr, si);
          if (track) lmax = fmax(lmax, fmax(fabs(sr), fabs(si)));
          Cplx<Real> o;
          o.x = sr;
          o.y = si;
          B[base + (jp % Q) * sp + (jp / Q) * sq] = o;
        }
      }
    } else if (type == OP_BELL) {
      const int s = pw[b];
      for (int x = lane; x < s; x += QNT) {
        const Cplx<Real> v = B[x];
        Cplx<Real> z;
        z.x = (Real)0;
        z.y = (Real)0;
        for (int a = 0; a < Q; ++a)
          for (int c = 0; c < Q; ++c)
            if (a | c) B[x + a * s + c * s * Q] = a == c ? v : z;
      }
      b += 2;
    } else if (type == OP_TRACE) {  // p < q; outputs move down, read in rounds before any write of the round
      const int nout = pw[b - 2];
      const int step = pw[p] + pw[q];
      for (int j0 = 0; j0 < nout; j0 += QNT) {
        const int j = j0 + lane;
        Cplx<Real> acc;
        acc.x = (Real)0;
        acc.y = (Real)0;
        if (j < nout) {
          const int i0 = insert_digits(j, p, q, pw);
          for (int a = 0; a < Q; ++a) {
            const Cplx<Real> u = B[i0 + a * step];
            acc.x += u.x;
            acc.y += u.y;
          }
          if (track) lmax = fmax(lmax, fmax(fabs(acc.x), fabs(acc.y)));
        }
        __syncthreads();
        if (j < nout) B[j] = acc;
        __syncthreads();
      }
      b -= 2;
    } else if (prev_track) {  // COLEND after the column's last writing op
      const Real m = group_max<Real, QNT>(lmax, red);
      lmax = 0;
      pend = 0;
      if (m > (Real)0 && isfinite(m)) {
        int e;
        frexp(m, &e);
        pend = e;
      }
    }
    prev_track = track;
    __syncthreads();
  }
  if (lane == 0) {
    // a factor Q per qudit no gate touches
    double f = 1.0;
    for (int k = 0; k < untouched; ++k) f *= Q;
    double* out = trace + 2 * (trace_offset + pi);
    out[0] = f * ldexp((double)B[0].x, (int)expo);
    out[1] = f * ldexp((double)B[0].y, (int)expo);
  }
}

size_t qudit_register_bytes(int q, int peak, int precision) {
  double e = 1.0;
  for (int k = 0; k < peak; ++k) e *= q;
  return (size_t)e * (precision == FP_C128 ? 16 : 8);
}

// LDS of one workgroup: the register plus the gate tables (two float64
// products and the realigned matrix) and the small arrays.
size_t qudit_lds_bytes(int q, int peak, int precision) {
  const size_t d2 = (size_t)q * q * q * q;
  const size_t rb = precision == FP_C128 ? 8 : 4;
  return qudit_register_bytes(q, peak < 2 ? 2 : peak, precision) + 32 * d2 + 2 * rb * d2 + 16 * rb + 96;
}

int launch_qudit(const fp_ensemble_t* e, int64_t num_pairs, int precision, const void* gates, double* trace,
                 const DevPlan& dp, hipStream_t s, int64_t trace_offset) {
  const int q = e->local_dim;
  const int G = (int)gates_per_circuit(FP_BRICKWORK_HAAR, e->n_qubits, e->depth);
  const int64_t stride = pair_bytes(e->ansatz, e->n_qubits, e->depth, precision, e->local_dim);
  const int peak = dp.hdr.peak_bits < 2 ? 2 : dp.hdr.peak_bits;
  const size_t smem = qudit_register_bytes(q, peak, precision);
  if (qudit_lds_bytes(q, peak, precision) > 160 * 1024)
    return set_error(FP_ETOOBIG, "qudit register of %d digits (q = %d) exceeds LDS", peak, q);
  const dim3 grid((unsigned)num_pairs), block(QNT);
  const unsigned char* g = (const unsigned char*)gates;
  const int untouched = dp.hdr.log2_factor;
#define FP_QK(R, QV, BF)                                                                                   \
  {                                                                                                         \
    auto k = qudit_kernel<R, QV, BF>;                                                                       \
    if (smem > 32 * 1024) (void)hipFuncSetAttribute(reinterpret_cast<const void*>(k),                      \
                                                     hipFuncAttributeMaxDynamicSharedMemorySize, (int)smem); \
    (void)hipGetLastError();                                                                                \
    hipLaunchKernelGGL(k, grid, block, smem, s, g, stride, G, dp.ops, dp.hdr.num_ops, dp.wg, dp.fac, peak,  \
                       untouched, trace, trace_offset, num_pairs);                                          \
  }
#define FP_QP(QV)                           \
  if (precision == FP_C128)                 \
    FP_QK(double, QV, false)                \
  else if (precision == FP_BF16X3)          \
    FP_QK(float, QV, true)                  \
  else                                      \
    FP_QK(float, QV, false)
  if (q == 3) {
    FP_QP(3)
  } else if (q == 4) {
    FP_QP(4)
  } else if (q == 5) {
    FP_QP(5)
  } else {
    return set_error(FP_EINVAL, "local dimension %d outside 3..5", q);
  }
#undef FP_QP
#undef FP_QK
  return check_launch("qudit_sweep");
}

}  // namespace fp
