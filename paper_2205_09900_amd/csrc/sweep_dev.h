// Device routines of the column sweep for two-qubit-gate ensembles: the
// interpreter of the register programs of plan.h.  Included by the kernels
// that run it (per-ensemble launches and the persistent scheduler).
#pragma once
#include <hip/hip_runtime.h>
#include <math.h>

#include "plan.h"

namespace fp {

template <typename Real>
struct Cplx {
  Real x, y;
};

template <int NT>
__device__ __forceinline__ void group_sync() {
  if constexpr (NT <= 64) {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
  } else {
    __syncthreads();
  }
}

// x >= 0 with a zero bit inserted at position pos: the bits from pos up move
// up one place (adding the high part to itself; two instructions)
__device__ __forceinline__ int insert_zero(int x, int pos) {
  return x + (int)((unsigned)x & (~0u << pos));
}
__device__ __forceinline__ int64_t insert_zero(int64_t x, int pos) {
  return x + (int64_t)((uint64_t)x & (~0ull << pos));
}

// Place of register entry x in LDS: x XOR ((x >> 5) mod 32).  Entries whose
// indices differ in bits 5..9 (the strides that the gate bits leave to
// neighbouring lanes) fall in different LDS banks.  A bijection of [0, 2^b)
// for every b, and linear over XOR: rsw(x ^ y) = rsw(x) ^ rsw(y), so the
// partners x ^ 2^p of an entry cost one XOR with a uniform constant.
__device__ __forceinline__ int rsw(int x) { return x ^ ((x >> 5) & 31); }

// BF16x3 products: x = hi + lo with hi = bf16(x) (round to nearest even)
// and lo = bf16(x - hi); a*b is taken as hi_a hi_b + hi_a lo_b + lo_a hi_b.
// Products of bf16 values are exact in float32, so only the accumulation
// rounds, as in a bf16 matrix core product with float32 accumulation.
struct Bf3 {
  float h, l;
};

__device__ __forceinline__ float bf16_round(float x) {
  unsigned u = __float_as_uint(x);
  u += 0x7fffu + ((u >> 16) & 1u);
  return __uint_as_float(u & 0xffff0000u);
}

__device__ __forceinline__ Bf3 bf3_split(float x) {
  Bf3 s;
  s.h = bf16_round(x);
  s.l = bf16_round(x - s.h);
  return s;
}

__device__ __forceinline__ float bf3_fma(Bf3 a, Bf3 b, float c) {
  c = fma(a.h, b.h, c);
  c = fma(a.h, b.l, c);
  c = fma(a.l, b.h, c);
  return c;
}

// sr += ar br - ai bi, si += ar bi + ai br in the arithmetic of the precision
// (the same fused order for both)
template <typename Real, bool BF3>
__device__ __forceinline__ void cmac(Real ar, Real ai, Real br, Real bi, Real& sr, Real& si) {
  if constexpr (BF3 && sizeof(Real) == 4) {
    const Bf3 a = bf3_split(ar), b = bf3_split(ai), c = bf3_split(br), d = bf3_split(bi);
    const Bf3 nb = {-b.h, -b.l};
    sr = bf3_fma(a, c, sr);
    sr = bf3_fma(nb, d, sr);
    si = bf3_fma(a, d, si);
    si = bf3_fma(b, c, si);
  } else {
    sr = fma(ar, br, sr);
    sr = fma(-ai, bi, sr);
    si = fma(ar, bi, si);
    si = fma(ai, br, si);
  }
}

// Merged gate M = F_last ... F_first (product of its factors) realigned for
// the column transfer and written to dst (16 complex):
//   dst[j' * 4 + j] = M[2 x_out + y_out][2 x_in + y_in],
// j = x_in + 2 x_out (legs on qubit c), j' = y_in + 2 y_out (legs on qubit c+1).
// One 4x4 complex gate (32 reals, 16-byte aligned) into registers with
// 16-byte loads.
__device__ __forceinline__ void load_gate(const float* src, float (&g)[32]) {
  const float4* v = reinterpret_cast<const float4*>(src);
#pragma unroll
  for (int i = 0; i < 8; ++i) {
    const float4 x = v[i];
    g[4 * i] = x.x;
    g[4 * i + 1] = x.y;
    g[4 * i + 2] = x.z;
    g[4 * i + 3] = x.w;
  }
}
__device__ __forceinline__ void load_gate(const double* src, double (&g)[32]) {
  const double2* v = reinterpret_cast<const double2*>(src);
#pragma unroll
  for (int i = 0; i < 16; ++i) {
    const double2 x = v[i];
    g[2 * i] = x.x;
    g[2 * i + 1] = x.y;
  }
}

// Row a of a gate (or of its conjugate transpose) from its registers.
template <typename Real>
__device__ __forceinline__ void factor_row(const Real (&g)[32], int dagger, int a, Real (&fr)[4], Real (&fi)[4]) {
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    const Real dr = g[(k * 4 + a) * 2], di = g[(k * 4 + a) * 2 + 1];
    const Real nr = g[(a * 4 + k) * 2], ni = g[(a * 4 + k) * 2 + 1];
    fr[k] = dagger ? dr : nr;
    fi[k] = dagger ? -di : ni;
  }
}

// code_of(f) gives the factor code of the f-th factor (time order), count >= 1.
template <typename Real, bool BF3, class Codes>
__device__ void merged_gate(const Real* __restrict__ pair_gates, int G, int count, Codes code_of, Cplx<Real>* dst) {
  Real mr[16], mi[16];
  {
    const FactorRef f0 = decode_factor(code_of(0), G);
    Real g[32];
    load_gate(pair_gates + ((int64_t)f0.circuit * G + f0.gate) * 32, g);
#pragma unroll
    for (int a = 0; a < 4; ++a) {
      Real fr[4], fi[4];
      factor_row<Real>(g, f0.dagger, a, fr, fi);
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        mr[a * 4 + k] = fr[k];
        mi[a * 4 + k] = fi[k];
      }
    }
  }
  for (int f = 1; f < count; ++f) {
    const FactorRef ff = decode_factor(code_of(f), G);
    Real g[32];
    load_gate(pair_gates + ((int64_t)ff.circuit * G + ff.gate) * 32, g);
    Real nr[16], ni[16];
#pragma unroll
    for (int a = 0; a < 4; ++a) {
      Real fr[4], fi[4];
      factor_row<Real>(g, ff.dagger, a, fr, fi);
#pragma unroll
      for (int b = 0; b < 4; ++b) {
        Real sr = 0, si = 0;
#pragma unroll
        for (int k = 0; k < 4; ++k) cmac<Real, BF3>(fr[k], fi[k], mr[k * 4 + b], mi[k * 4 + b], sr, si);
        nr[a * 4 + b] = sr;
        ni[a * 4 + b] = si;
      }
    }
#pragma unroll
    for (int i = 0; i < 16; ++i) {
      mr[i] = nr[i];
      mi[i] = ni[i];
    }
  }
#pragma unroll
  for (int jp = 0; jp < 4; ++jp)
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int xin = j & 1, xout = j >> 1, yin = jp & 1, yout = jp >> 1;
      const int idx = (2 * xout + yout) * 4 + (2 * xin + yin);
      dst[jp * 4 + j].x = mr[idx];
      dst[jp * 4 + j].y = mi[idx];
    }
}

template <typename Real, bool BF3 = false>
__device__ void stage_gate(const Real* __restrict__ pair_gates, int G, const int32_t* __restrict__ factors, int2 wg,
                           Cplx<Real>* dst) {
  merged_gate<Real, BF3>(pair_gates, G, wg.y, [&](int f) { return factors[wg.x + f]; }, dst);
}

// Applies the realigned 4x4 matrix (Rr, Ri) to the groups of four entries
// g = first, first + stride, ... < ng (bits lo < hi of the group index are the
// gate's bits).  Up to U groups per round: distinct groups touch distinct
// entries, so all loads of a round are issued before its stores and their
// latencies overlap.  Same arithmetic per group as one group at a time.
template <typename Real, int U, bool BF3 = false>
__device__ __forceinline__ void gate_groups(Cplx<Real>* B, const Real (&Rr)[16], const Real (&Ri)[16], int lo,
                                            int hi, int ip, int iq, int ng, int first, int stride, bool track,
                                            Real& lmax) {
  const int sp = rsw(ip), sq = rsw(iq), spq = sp ^ sq;
  for (int g0 = first; g0 < ng; g0 += stride * U) {
    Cplx<Real> v[U][4];
    int idx[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int g = g0 + u * stride;
      idx[u] = rsw(insert_zero(insert_zero(g, lo), hi));
      if (g < ng) {
        v[u][0] = B[idx[u]];
        v[u][1] = B[idx[u] ^ sp];
        v[u][2] = B[idx[u] ^ sq];
        v[u][3] = B[idx[u] ^ spq];
      }
    }
#pragma unroll
    for (int u = 0; u < U; ++u) {
      if (g0 + u * stride >= ng) break;
      Cplx<Real> w[4];
#pragma unroll
      for (int jp = 0; jp < 4; ++jp) {
        Real sr = 0, si = 0;
#pragma unroll
        for (int j = 0; j < 4; ++j) cmac<Real, BF3>(Rr[jp * 4 + j], Ri[jp * 4 + j], v[u][j].x, v[u][j].y, sr, si);
        w[jp].x = sr;
        w[jp].y = si;
        if (track) lmax = fmax(lmax, fmax(fabs(sr), fabs(si)));
      }
      B[idx[u]] = w[0];
      B[idx[u] ^ sp] = w[1];
      B[idx[u] ^ sq] = w[2];
      B[idx[u] ^ spq] = w[3];
    }
  }
}

// gate_groups with the op's flags as template arguments, for groups whose op
// is uniform (one pair per wavefront or more): TRACK records the largest
// magnitude written, SCALE multiplies the outputs by 2^-scale (the column's
// pending power of two; exact, the same as scaling the matrix).
template <typename Real, int U, bool BF3, bool TRACK, bool SCALE>
__device__ __forceinline__ void gate_groups_u(Cplx<Real>* B, const Real (&Rr)[16], const Real (&Ri)[16], int lo,
                                              int hi, int ip, int iq, int ng, int first, int stride, int scale,
                                              Real& lmax) {
  const int sp = rsw(ip), sq = rsw(iq), spq = sp ^ sq;
  for (int g0 = first; g0 < ng; g0 += stride * U) {
    Cplx<Real> v[U][4];
    int idx[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int g = g0 + u * stride;
      idx[u] = rsw(insert_zero(insert_zero(g, lo), hi));
      if (g < ng) {
        v[u][0] = B[idx[u]];
        v[u][1] = B[idx[u] ^ sp];
        v[u][2] = B[idx[u] ^ sq];
        v[u][3] = B[idx[u] ^ spq];
      }
    }
#pragma unroll
    for (int u = 0; u < U; ++u) {
      if (g0 + u * stride >= ng) break;
      Cplx<Real> w[4];
#pragma unroll
      for (int jp = 0; jp < 4; ++jp) {
        Real sr = 0, si = 0;
#pragma unroll
        for (int j = 0; j < 4; ++j) cmac<Real, BF3>(Rr[jp * 4 + j], Ri[jp * 4 + j], v[u][j].x, v[u][j].y, sr, si);
        if (SCALE) {
          sr = ldexp(sr, -scale);
          si = ldexp(si, -scale);
        }
        w[jp].x = sr;
        w[jp].y = si;
        if (TRACK) lmax = fmax(lmax, fmax(fabs(sr), fabs(si)));
      }
      B[idx[u]] = w[0];
      B[idx[u] ^ sp] = w[1];
      B[idx[u] ^ sq] = w[2];
      B[idx[u] ^ spq] = w[3];
    }
  }
}

// Two GATEs on four distinct register bits, consecutive in a program, act
// as one 16x16 complex block F: the Kronecker product of their realigned
// matrices (they commute).  In the BF16x3 arithmetic the block is applied by
// bf16 matrix cores (v_mfma_f32_32x32x16_bf16): F and the register entries
// are split into bf16 hi + lo parts and hi*hi + hi*lo + lo*hi accumulate in
// float32, the same three products per real product as the vector path.  The
// complex product is the real product of the 32x32 block [[Fr, -Fi], [Fi, Fr]]
// with the stacked real and imaginary parts of X, where X[r][c] is the
// register entry whose gate bits (pa, qa, pb, qb) spell bits 0..3 of r and
// whose other bits spell c.  The group first writes F's four bf16 planes
// (Re hi, Re lo, Im hi, Im lo; 16x16 each, MFMA_BLOCK_BYTES) to LDS; then a
// wavefront takes 32 columns c at a time, reads all of them before writing
// any, and no two wavefronts share a column.  Fragment layouts (one
// wavefront, lane l, h = l / 32, n = l % 32): A[m][k] with m = n, k = 8h + j;
// B[k][c] with k = 8h + j, c = n; the accumulator element i holds
// D[8 (i / 4) + 4h + i % 4][n].
typedef __bf16 bf16x2_t __attribute__((ext_vector_type(2)));
typedef __bf16 bf16x8_t __attribute__((ext_vector_type(8)));
typedef float f32x16_t __attribute__((ext_vector_type(16)));
typedef unsigned u32x4_t __attribute__((ext_vector_type(4)));

constexpr size_t MFMA_BLOCK_BYTES = 4 * 256 * 2;

// x0, x1 as packed bf16 pairs: hi = bf16(x) (round to nearest even) and
// lo = bf16(x - hi); element 0 in the low half
__device__ __forceinline__ void bf16_split2(float x0, float x1, unsigned& hi, unsigned& lo) {
  hi = __builtin_bit_cast(unsigned, __builtin_convertvector((float __attribute__((ext_vector_type(2)))){x0, x1},
                                                            bf16x2_t));
  const float h0 = __uint_as_float(hi << 16), h1 = __uint_as_float(hi & 0xffff0000u);
  lo = __builtin_bit_cast(unsigned,
                          __builtin_convertvector((float __attribute__((ext_vector_type(2)))){x0 - h0, x1 - h1},
                                                  bf16x2_t));
}

__device__ __forceinline__ int gate_bits_offset(int r, int pa, int qa, int pb, int qb) {
  return ((r & 1) << pa) + (((r >> 1) & 1) << qa) + (((r >> 2) & 1) << pb) + (((r >> 3) & 1) << qb);
}

// Registers of 2^b entries, b >= 9 (at least one block of 32 columns); every
// lane of the group calls it (lane in [0, NT)); fblk: the group's
// MFMA_BLOCK_BYTES of LDS; scale: the column's pending power of two, taken
// out of the block (exact).  SINGLE: one GATE (Ma on bits pa, qa) as the
// block Ma x identity on two further bits pb, qb.
template <int NT, bool TRACK, bool SCALE, bool SINGLE = false>
__device__ __forceinline__ void gate_pair_mfma(Cplx<float>* B, const Cplx<float>* Ma, const Cplx<float>* Mb,
                                               unsigned short* fblk, int pa, int qa, int pb, int qb, int b, int lane,
                                               int scale, float& lmax) {
  constexpr int NW = NT / 64;
  // F[r'][r] = Ma[r' % 4][r % 4] Mb[r' / 4][r / 4], planes at e = 16 r' + r
  for (int e = lane; e < 256; e += NT) {
    const int ro = e >> 4, k = e & 15;
    const Cplx<float> x = Ma[(ro & 3) * 4 + (k & 3)];
    float fr, fi;
    if constexpr (SINGLE) {
      const bool on = (ro >> 2) == (k >> 2);
      fr = on ? x.x : 0.0f;
      fi = on ? x.y : 0.0f;
    } else {
      const Cplx<float> y = Mb[(ro >> 2) * 4 + (k >> 2)];
      fr = fmaf(x.x, y.x, -x.y * y.y);
      fi = fmaf(x.x, y.y, x.y * y.x);
    }
    if (SCALE) {
      fr = ldexpf(fr, -scale);
      fi = ldexpf(fi, -scale);
    }
    unsigned hi, lo;
    bf16_split2(fr, fi, hi, lo);
    fblk[e] = (unsigned short)hi;
    fblk[256 + e] = (unsigned short)lo;
    fblk[512 + e] = (unsigned short)(hi >> 16);
    fblk[768 + e] = (unsigned short)(lo >> 16);
  }
  group_sync<NT>();
  const int wave = lane >> 6, h = (lane >> 5) & 1, n = lane & 31;
  bf16x8_t a0h, a0l, a1h, a1l;  // k-step 0 multiplies Re X, k-step 1 Im X
  {
    // rows 0..15 of the 32x32 block: (Fr | -Fi), rows 16..31: (Fi | Fr)
    const int row = (n & 15) * 16 + 8 * h;
    const bool top = n < 16;
    const unsigned neg = top ? 0x80008000u : 0u;
    const u32x4_t* pl = reinterpret_cast<const u32x4_t*>(fblk);
    const u32x4_t r0h = pl[((top ? 0 : 512) + row) >> 3], r0l = pl[((top ? 256 : 768) + row) >> 3];
    const u32x4_t r1h = pl[((top ? 512 : 0) + row) >> 3], r1l = pl[((top ? 768 : 256) + row) >> 3];
    a0h = __builtin_bit_cast(bf16x8_t, r0h);
    a0l = __builtin_bit_cast(bf16x8_t, r0l);
    a1h = __builtin_bit_cast(bf16x8_t, r1h ^ neg);
    a1l = __builtin_bit_cast(bf16x8_t, r1l ^ neg);
  }
  // entry offsets of the rows a lane reads (8h + j) and writes
  // (8 (j / 4) + 4h + j % 4): uniform parts, and the lane's half h as one
  // gate bit (qb for the reads, pb for the writes)
  int off_in[8], off_out[8];
#pragma unroll
  for (int j = 0; j < 8; ++j) {
    off_in[j] = rsw(gate_bits_offset(j, pa, qa, pb, qb));
    off_out[j] = rsw(gate_bits_offset(8 * (j >> 2) + (j & 3), pa, qa, pb, qb));
  }
  const int h_in = h ? rsw(1 << qb) : 0, h_out = h ? rsw(1 << pb) : 0;
  // the four gate bits in increasing order
  int s0 = pa < qa ? pa : qa, s1 = pa < qa ? qa : pa, s2 = pb < qb ? pb : qb, s3 = pb < qb ? qb : pb;
  if (s2 < s0) { const int t = s0; s0 = s2; s2 = t; }
  if (s3 < s1) { const int t = s1; s1 = s3; s3 = t; }
  if (s2 < s1) { const int t = s1; s1 = s2; s2 = t; }
  const int ntile = 1 << (b - 9);
  for (int t = wave; t < ntile; t += NW) {
    const int c = t * 32 + n;
    const int base = rsw(insert_zero(insert_zero(insert_zero(insert_zero(c, s0), s1), s2), s3));
    const int bin = base ^ h_in, bout = base ^ h_out;
    Cplx<float> x[8];
#pragma unroll
    for (int j = 0; j < 8; ++j) x[j] = B[bin ^ off_in[j]];
    u32x4_t rh, rl, ih, il;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      unsigned hh, ll;
      bf16_split2(x[2 * j].x, x[2 * j + 1].x, hh, ll);
      rh[j] = hh;
      rl[j] = ll;
      bf16_split2(x[2 * j].y, x[2 * j + 1].y, hh, ll);
      ih[j] = hh;
      il[j] = ll;
    }
    const bf16x8_t xrh = __builtin_bit_cast(bf16x8_t, rh), xrl = __builtin_bit_cast(bf16x8_t, rl);
    const bf16x8_t xih = __builtin_bit_cast(bf16x8_t, ih), xil = __builtin_bit_cast(bf16x8_t, il);
    f32x16_t acc = {};
    acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a0l, xrh, acc, 0, 0, 0);
    acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a0h, xrl, acc, 0, 0, 0);
    acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a1l, xih, acc, 0, 0, 0);
    acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a1h, xil, acc, 0, 0, 0);
    acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a0h, xrh, acc, 0, 0, 0);
    acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a1h, xih, acc, 0, 0, 0);
#pragma unroll
    for (int j = 0; j < 8; ++j) {
      Cplx<float> y;
      y.x = acc[j];
      y.y = acc[j + 8];
      if (TRACK) lmax = fmax(lmax, fmax(fabs(y.x), fabs(y.y)));
      B[bout ^ off_out[j]] = y;
    }
  }
}

// Groups per round of gate_groups: one (measured: batching several raised the
// register count and lost more to occupancy than the overlapped loads gained).
template <typename Real>
constexpr int gate_batch() {
  return 1;
}

template <typename Real, int NT>
__device__ __forceinline__ Real group_max(Real v, Real* red) {
  constexpr int W = NT < 64 ? NT : 64;
#pragma unroll
  for (int off = W / 2; off > 0; off >>= 1) v = fmax(v, __shfl_xor(v, off, W));
  if constexpr (NT > 64) {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    __syncthreads();
    if (lane == 0) red[wave] = v;
    __syncthreads();
    v = red[0];
#pragma unroll
    for (int w = 1; w < NT / 64; ++w) v = fmax(v, red[w]);
  }
  return v;
}

template <int NT>
constexpr int chunk_ops() {
  return NT <= 16 ? 16 : NT <= 64 ? 32 : 64;
}

// Runs one pair's program on boundary B (LDS or global).  The program is
// processed in chunks of K ops: the group first stages the chunk's op records
// and the realigned matrices of its GATE ops in LDS (one lane per op, in
// parallel; the matrices are copied when they come precomputed, else formed
// from the factors), then executes the ops from LDS.  The per-column rescale is
// lazy: the op that ends a column records the largest magnitude it writes,
// the column end turns it into an exponent P, and the next GATE multiplies
// its matrix by 2^-P (exact), so no extra pass over the boundary is made.
// MX: BF16x3 GATEs on registers of 2^9 entries or more go to the matrix
// cores (a caller whose registers are already at the limit keeps them on
// the vector path).
template <typename Real, int NT, bool BF3 = false, bool MX = true>
__device__ __forceinline__ void run_program(Cplx<Real>* B, Cplx<Real>* mats_s, Op* ops_s, const Op* __restrict__ ops,
                                            int num_ops, const int2* __restrict__ wgates,
                                            const int32_t* __restrict__ factors, const Real* pair_gates, int G,
                                            int log2_factor, int lane, Real* red, double* tr_re, double* tr_im,
                                            const Real* __restrict__ wmat = nullptr, int num_gate_ops = 0) {
  constexpr int K = chunk_ops<NT>();
  // BF16x3 matrix-core blocks: MFMA_BLOCK_BYTES after the staged op records
  unsigned short* fblk = reinterpret_cast<unsigned short*>(ops_s + K);
  // with the matrices precomputed in program order (wmat), the first
  // wavefront stages a chunk and numbers its GATEs with a ballot
  const bool pre = NT >= 64 && wmat != nullptr;
  int gate_base = 0;  // GATE ops before the chunk (first wavefront only)
  int b = 0;
  int64_t expo = 0;  // true boundary = stored boundary * 2^expo
  int pend = 0;      // exponent to remove at the next GATE
  Real lmax = 0;
  if (lane == 0) {
    B[0].x = (Real)1;
    B[0].y = (Real)0;
  }
  for (int t0 = 0; t0 < num_ops; t0 += K) {
    const int nk = num_ops - t0 < K ? num_ops - t0 : K;
    if (pre) {
      if (lane < 64) {
        const bool here = lane < nk;
        Op op;
        if (here) op = ops[t0 + lane];
        const bool is_gate = here && (op.type & OP_TYPE_MASK) == OP_GATE;
        const unsigned long long m = __ballot(is_gate);
        const unsigned long long below = lane ? (~0ull >> (64 - lane)) : 0ull;
        const int k = gate_base + __popcll(m & below);
        gate_base += __popcll(m);
        if (here) ops_s[lane] = op;
        if (is_gate && k < num_gate_ops) {
          const float4* src = reinterpret_cast<const float4*>(wmat + 32 * (int64_t)k);
          float4* dst = reinterpret_cast<float4*>(mats_s + 16 * lane);
#pragma unroll
          for (int r = 0; r < 8 * (int)sizeof(Real) / 4; ++r) dst[r] = src[r];
        }
      }
    } else {
      for (int i = lane; i < nk; i += NT) {
        const Op op = ops[t0 + i];
        ops_s[i] = op;
        if ((op.type & OP_TYPE_MASK) == OP_GATE)
          stage_gate<Real, BF3>(pair_gates, G, factors, wgates[op.arg], mats_s + 16 * i);
      }
    }
    group_sync<NT>();
    for (int i = 0; i < nk; ++i) {
      Op op = ops_s[i];
      if constexpr (NT >= 64) {  // one pair per wavefront or more: the op is uniform
        const unsigned w0 = (unsigned)__builtin_amdgcn_readfirstlane(*reinterpret_cast<const int*>(&op));
        op.type = (uint8_t)w0;
        op.p = (uint8_t)(w0 >> 8);
        op.q = (uint8_t)(w0 >> 16);
      }
      const int type = op.type & OP_TYPE_MASK;
      const bool track = (op.type & OP_FLAG_TRACK) != 0;
      bool fused = false, single = false;
      if constexpr (BF3 && MX && NT >= 64) {
        // this GATE and the next on four distinct bits: one matrix-core block
        if (type == OP_GATE && !track && b >= 9 && i + 1 < nk) {
          const unsigned w1 = (unsigned)__builtin_amdgcn_readfirstlane(*reinterpret_cast<const int*>(&ops_s[i + 1]));
          const int p2 = (int)((w1 >> 8) & 0xff), q2 = (int)((w1 >> 16) & 0xff);
          if ((int)(w1 & OP_TYPE_MASK) == OP_GATE && p2 != op.p && p2 != op.q && q2 != op.p && q2 != op.q) {
            const bool track2 = (w1 & OP_FLAG_TRACK) != 0;
            const int sc = __builtin_amdgcn_readfirstlane(pend);
            const Cplx<float>* ma = reinterpret_cast<const Cplx<float>*>(mats_s + 16 * i);
            Cplx<float>* Bf = reinterpret_cast<Cplx<float>*>(B);
            float lm = (float)lmax;
            if (track2) {
              if (sc) gate_pair_mfma<NT, true, true>(Bf, ma, ma + 16, fblk, op.p, op.q, p2, q2, b, lane, sc, lm);
              else gate_pair_mfma<NT, true, false>(Bf, ma, ma + 16, fblk, op.p, op.q, p2, q2, b, lane, 0, lm);
            } else {
              if (sc) gate_pair_mfma<NT, false, true>(Bf, ma, ma + 16, fblk, op.p, op.q, p2, q2, b, lane, sc, lm);
              else gate_pair_mfma<NT, false, false>(Bf, ma, ma + 16, fblk, op.p, op.q, p2, q2, b, lane, 0, lm);
            }
            lmax = (Real)lm;
            expo += pend;
            pend = 0;
            fused = true;
          }
        }
        if (!fused && type == OP_GATE && b >= 9) {
          // a GATE without a partner: its matrix times the identity on the two
          // lowest other bits
          const int pa = op.p, qa = op.q;
          int pb = 0;
          while (pb == pa || pb == qa) ++pb;
          int qb = pb + 1;
          while (qb == pa || qb == qa) ++qb;
          const int sc = __builtin_amdgcn_readfirstlane(pend);
          const Cplx<float>* ma = reinterpret_cast<const Cplx<float>*>(mats_s + 16 * i);
          Cplx<float>* Bf = reinterpret_cast<Cplx<float>*>(B);
          float lm = (float)lmax;
          if (track) {
            if (sc) gate_pair_mfma<NT, true, true, true>(Bf, ma, ma, fblk, pa, qa, pb, qb, b, lane, sc, lm);
            else gate_pair_mfma<NT, true, false, true>(Bf, ma, ma, fblk, pa, qa, pb, qb, b, lane, 0, lm);
          } else {
            if (sc) gate_pair_mfma<NT, false, true, true>(Bf, ma, ma, fblk, pa, qa, pb, qb, b, lane, sc, lm);
            else gate_pair_mfma<NT, false, false, true>(Bf, ma, ma, fblk, pa, qa, pb, qb, b, lane, 0, lm);
          }
          lmax = (Real)lm;
          expo += pend;
          pend = 0;
          single = true;
        }
      }
      if (fused) {
        ++i;  // the next GATE is applied too
      } else if (single) {
      } else if (type == OP_GATE) {
        const int p = op.p, q = op.q;
        const int lo = p < q ? p : q, hi = p < q ? q : p;
        const int ip = 1 << p, iq = 1 << q;
        // (BF16x3 with 1024 lanes: one group per round, within 128 registers)
        constexpr int U = BF3 && NT < 1024 ? 2 : gate_batch<Real>();
        Real Rr[16], Ri[16];
        if constexpr (NT >= 64) {
#pragma unroll
          for (int k = 0; k < 16; ++k) {
            const Cplx<Real> r = mats_s[16 * i + k];
            Rr[k] = r.x;
            Ri[k] = r.y;
          }
          const int sc = __builtin_amdgcn_readfirstlane(pend);
          const int ng = 1 << (b - 2);
          if (track) {
            if (sc) gate_groups_u<Real, U, BF3, true, true>(B, Rr, Ri, lo, hi, ip, iq, ng, lane, NT, sc, lmax);
            else gate_groups_u<Real, U, BF3, true, false>(B, Rr, Ri, lo, hi, ip, iq, ng, lane, NT, 0, lmax);
          } else {
            if (sc) gate_groups_u<Real, U, BF3, false, true>(B, Rr, Ri, lo, hi, ip, iq, ng, lane, NT, sc, lmax);
            else gate_groups_u<Real, U, BF3, false, false>(B, Rr, Ri, lo, hi, ip, iq, ng, lane, NT, 0, lmax);
          }
        } else {
#pragma unroll
          for (int k = 0; k < 16; ++k) {
            const Cplx<Real> r = mats_s[16 * i + k];
            Rr[k] = pend ? ldexp(r.x, -pend) : r.x;
            Ri[k] = pend ? ldexp(r.y, -pend) : r.y;
          }
          gate_groups<Real, U, BF3>(B, Rr, Ri, lo, hi, ip, iq, 1 << (b - 2), lane, NT, track, lmax);
        }
        expo += pend;
        pend = 0;
      } else if (type == OP_BELL) {
        const int s = 1 << b;
        const int s1 = rsw(s), s2 = rsw(2 * s), s3 = s1 ^ s2;
        for (int k = lane; k < s; k += NT) {
          const int ks = rsw(k);
          const Cplx<Real> v = B[ks];
          Cplx<Real> z;
          z.x = (Real)0;
          z.y = (Real)0;
          B[ks ^ s1] = z;
          B[ks ^ s2] = z;
          B[ks ^ s3] = v;
        }
        b += 2;
      } else if (type == OP_TRACE) {
        const int p = op.p, q = op.q;  // p < q
        const int nout = 1 << (b - 2);
        const int step = rsw((1 << p) + (1 << q));
        for (int j0 = 0; j0 < nout; j0 += NT) {
          const int j = j0 + lane;
          Cplx<Real> acc;
          acc.x = (Real)0;
          acc.y = (Real)0;
          if (j < nout) {
            const int i0 = rsw(insert_zero(insert_zero(j, p), q));
            const Cplx<Real> a0 = B[i0], a1 = B[i0 ^ step];
            acc.x = a0.x + a1.x;
            acc.y = a0.y + a1.y;
            if (track) lmax = fmax(lmax, fmax(fabs(acc.x), fabs(acc.y)));
          }
          group_sync<NT>();
          if (j < nout) B[rsw(j)] = acc;
          group_sync<NT>();
        }
        b -= 2;
      } else {  // OP_COLEND
        if (i > 0 ? (ops_s[i - 1].type & OP_FLAG_TRACK) != 0 : false) {
          const Real m = group_max<Real, NT>(lmax, red);
          lmax = 0;
          pend = 0;
          if (m > (Real)0 && isfinite(m)) {
            int e;
            frexp(m, &e);
            pend = e;
          }
        } else if (i == 0 && t0 > 0) {
          // the column's last writing op ended the previous chunk
          const Op prev = ops[t0 - 1];
          if (prev.type & OP_FLAG_TRACK) {
            const Real m = group_max<Real, NT>(lmax, red);
            lmax = 0;
            pend = 0;
            if (m > (Real)0 && isfinite(m)) {
              int e;
              frexp(m, &e);
              pend = e;
            }
          }
        }
      }
      group_sync<NT>();
    }
  }
  const Cplx<Real> v = B[0];
  *tr_re = ldexp((double)v.x, (int)(expo + log2_factor));
  *tr_im = ldexp((double)v.y, (int)(expo + log2_factor));
}

// staged matrices and op records of a chunk, then (BF16x3 with a group of
// 64 lanes or more) the matrix-core block
template <typename Real, int NT, bool BF3 = false>
constexpr size_t stage_bytes() {
  return (size_t)chunk_ops<NT>() * (16 * sizeof(Cplx<Real>) + sizeof(Op)) + (BF3 && NT >= 64 ? MFMA_BLOCK_BYTES : 0);
}

}  // namespace fp
