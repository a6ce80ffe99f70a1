// Column sweep with one wavefront per pair, for registers of up to 2^10
// entries (the bulk of local random pairs).  Same register programs and the
// same arithmetic as the LDS sweep of sweep_dev.h (Sec. II.A of the paper,
// trace as a contraction along the qubits; Methods A).  The kernel is bound
// by vector-instruction issue, so it is organised to spend as few vector
// instructions per op as it can:
//   * the op stream is uniform across the wavefront: op records are read 64
//     at a time into lanes and taken with readlane, so decoding and branching
//     are scalar;
//   * the realigned matrices of the GATE ops come precomputed in program
//     order, prefetched four GATEs ahead by lanes 0..31 and passed through
//     two 32-entry LDS stages that hold the real parts before the imaginary
//     ones, so 16-byte LDS reads land in the registers the products use; the
//     next GATE's matrix is staged during the current one, so a GATE costs
//     one LDS fence, and a column's rescale is applied to the staged matrix;
//   * a column's largest magnitude is reduced across lanes with DPP moves;
//   * registers of up to 64 entries give each lane one output entry of the
//     gate (one matrix row, four inputs); larger ones give each lane whole
//     groups of four entries;
//   * the ops that record a column's largest magnitude and those that do not
//     are separate code paths (a scalar branch, not a select per output).
// The boundary stays in LDS; pairs are independent, so waves never wait for
// each other.
#include <hip/hip_runtime.h>
#include <math.h>

#include "internal.h"
#include "plan.h"
#include "sweep.h"
#include "sweep_dev.h"

namespace fp {

namespace {

__device__ __forceinline__ void wave_fence() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Lane movement within rows of 16 lanes by DPP (no LDS round trip).
template <int CTRL>
__device__ __forceinline__ float dpp_move(float v) {
  return __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, v), CTRL, 0xf, 0xf, false));
}
template <int CTRL>
__device__ __forceinline__ double dpp_move(double v) {
  const long long x = __builtin_bit_cast(long long, v);
  const int lo = __builtin_amdgcn_update_dpp(0, (int)x, CTRL, 0xf, 0xf, false);
  const int hi = __builtin_amdgcn_update_dpp(0, (int)(x >> 32), CTRL, 0xf, 0xf, false);
  return __builtin_bit_cast(double, ((long long)hi << 32) | (unsigned)lo);
}
__device__ __forceinline__ float lane_value(float v, int l) {
  return __builtin_bit_cast(float, __builtin_amdgcn_readlane(__builtin_bit_cast(int, v), l));
}
__device__ __forceinline__ double lane_value(double v, int l) {
  const long long x = __builtin_bit_cast(long long, v);
  const unsigned lo = (unsigned)__builtin_amdgcn_readlane((int)x, l);
  const unsigned hi = (unsigned)__builtin_amdgcn_readlane((int)(x >> 32), l);
  return __builtin_bit_cast(double, ((unsigned long long)hi << 32) | lo);
}

// Largest value over the wavefront (every lane active): swaps within quads,
// rotations by 4 and 8 within rows of 16, then the four rows' results.
template <typename Real>
__device__ __forceinline__ Real wave_max(Real v) {
  v = fmax(v, dpp_move<0xB1>(v));   // quad_perm [1, 0, 3, 2]
  v = fmax(v, dpp_move<0x4E>(v));   // quad_perm [2, 3, 0, 1]
  v = fmax(v, dpp_move<0x124>(v));  // row_ror 4
  v = fmax(v, dpp_move<0x128>(v));  // row_ror 8
  return fmax(fmax(lane_value(v, 0), lane_value(v, 16)), fmax(lane_value(v, 32), lane_value(v, 48)));
}

constexpr int TOUCH = 4;  // GATEs between a matrix's cache touch and its load

// Registers of up to 64 entries: lane = 4 g + jp computes output jp of group
// g (g < 2^(b-2)), i.e. row jp of the matrix (stage: real parts at 0..15,
// imaginary parts at 16..31) against the group's four entries.
template <typename Real, bool BF3, bool TRACK>
__device__ __forceinline__ void gate_small(Cplx<Real>* B, const Real* stage, int b, int lo, int hi, int ip, int iq,
                                           int sp, int sq, int lane, Real& lmax) {
  const int g = lane >> 2, jp = lane & 3;
  Real Rr[4], Ri[4];
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    Rr[j] = stage[jp * 4 + j];
    Ri[j] = stage[16 + jp * 4 + j];
  }
  if (g < (1 << (b - 2))) {
    const int idx = insert_zero(insert_zero(g, lo), hi);
    Cplx<Real> v[4];
    v[0] = B[idx];
    v[1] = B[idx + ip];
    v[2] = B[idx + iq];
    v[3] = B[idx + ip + iq];
    Real sr = 0, si = 0;
#pragma unroll
    for (int j = 0; j < 4; ++j) cmac<Real, BF3>(Rr[j], Ri[j], v[j].x, v[j].y, sr, si);
    if (TRACK) lmax = fmax(lmax, fmax(fabs(sr), fabs(si)));
    // the store follows the four loads of every lane (one instruction
    // stream), so no lane overwrites an input another lane still needs
    Cplx<Real> w;
    w.x = sr;
    w.y = si;
    B[idx + ((jp & 1) << sp) + ((jp >> 1) << sq)] = w;
  }
}

// Larger registers: each lane applies the whole matrix to groups of four
// entries, lane, lane + 64, ...
template <typename Real, bool BF3, bool TRACK>
__device__ __forceinline__ void gate_big(Cplx<Real>* B, const Real* stage, int b, int lo, int hi, int ip, int iq,
                                         int lane, Real& lmax) {
  Real Rr[16], Ri[16];
#pragma unroll
  for (int k = 0; k < 16; ++k) {
    Rr[k] = stage[k];
    Ri[k] = stage[16 + k];
  }
  const int ng = 1 << (b - 2);
  for (int g = lane; g < ng; g += 64) {
    const int idx = insert_zero(insert_zero(g, lo), hi);
    Cplx<Real> v[4];
    v[0] = B[idx];
    v[1] = B[idx + ip];
    v[2] = B[idx + iq];
    v[3] = B[idx + ip + iq];
    Cplx<Real> w[4];
#pragma unroll
    for (int jp = 0; jp < 4; ++jp) {
      Real sr = 0, si = 0;
#pragma unroll
      for (int j = 0; j < 4; ++j) cmac<Real, BF3>(Rr[jp * 4 + j], Ri[jp * 4 + j], v[j].x, v[j].y, sr, si);
      if (TRACK) lmax = fmax(lmax, fmax(fabs(sr), fabs(si)));
      w[jp].x = sr;
      w[jp].y = si;
    }
    B[idx] = w[0];
    B[idx + ip] = w[1];
    B[idx + iq] = w[2];
    B[idx + ip + iq] = w[3];
  }
}

// TRACE over bits p < q: entries move down in increasing order, and every
// read of an iteration precedes its writes, so the compaction is in place.
template <typename Real, bool TRACK>
__device__ __forceinline__ void trace_wave(Cplx<Real>* B, int b, int p, int q, int lane, Real& lmax) {
  const int nout = 1 << (b - 2);
  const int step = (1 << p) + (1 << q);
  for (int j = lane; j < nout; j += 64) {
    const int i0 = insert_zero(insert_zero(j, p), q);
    const Cplx<Real> a0 = B[i0], a1 = B[i0 + step];
    Cplx<Real> acc;
    acc.x = a0.x + a1.x;
    acc.y = a0.y + a1.y;
    if (TRACK) lmax = fmax(lmax, fmax(fabs(acc.x), fabs(acc.y)));
    B[j] = acc;
  }
}

}  // namespace

// register of 2^CAP entries, then two 32-real matrix stages
template <typename Real, int CAP>
constexpr size_t wave_slot_bytes() {
  return ((size_t)sizeof(Cplx<Real>) << CAP) + 64 * sizeof(Real);
}

// One pair (index pidx) on one wavefront, its register in LDS slot `wave`.
template <typename Real, int CAP, bool BF3>
__device__ __forceinline__ void wave_pair(const SweepArgs& a, int64_t pidx, int wave, int lane,
                                          unsigned char* smem_raw) {
  const PlanHeader* hdr = a.hdr + pidx * a.hdr_stride;
  const int status = __builtin_amdgcn_readfirstlane(hdr->status);
  const int peak = __builtin_amdgcn_readfirstlane(hdr->peak_bits);
  double* out = a.trace + 2 * (a.trace_offset + pidx);
  if (status != 0) {
    if (lane == 0) {
      out[0] = __builtin_nan("");
      out[1] = __builtin_nan("");
    }
    return;
  }
  if (peak > CAP || peak <= a.min_bits) return;  // another launch's pair
  const int num_ops = __builtin_amdgcn_readfirstlane(hdr->num_ops);
  const int ngate = __builtin_amdgcn_readfirstlane(hdr->num_gate_ops);
  const int log2f = __builtin_amdgcn_readfirstlane(hdr->log2_factor);
  Cplx<Real>* B = reinterpret_cast<Cplx<Real>*>(smem_raw + wave_slot_bytes<Real, CAP>() * wave);
  // two stages: the next GATE's matrix is staged while the current one is
  // applied, so the fence that ends an op also publishes the next matrix
  Real* stage = reinterpret_cast<Real*>(B + (1 << CAP));
  const uint2* ops = reinterpret_cast<const uint2*>(a.ops + pidx * a.ops_stride);
  const Real* mats = reinterpret_cast<const Real*>(a.wmat + pidx * a.wmat_stride);
  // lane l < 32 carries real l of a matrix (interleaved re, im) and stages it
  // de-interleaved
  const int my_off = (lane & 1) * 16 + ((lane & 31) >> 1);
  const int ml = lane & 31;  // lanes 32..63 load a copy and never stage it

  // Matrices reach the stage through one register, `nxt`, reloaded at the
  // end of every op: lanes 0..31 load the matrix the next GATE stages,
  // lanes 32..63 touch the one TOUCH GATEs later so that the reload finds
  // it in cache.  Loaded on every op, `nxt` is never copied (a copy of a
  // loaded value waits for the load).  Indices are clamped to
  // [0, ngate - 1]; matrix 0 lies inside the pair's region even when the
  // program has no GATE.
  const int last = ngate > 0 ? ngate - 1 : 0;
  auto mat_index = [&](int m) -> int64_t {
    const int t = lane < 32 ? m : m + TOUCH;
    return (int64_t)(t < last ? t : last) * 32 + ml;
  };
  Real nxt = mats[mat_index(0)];
  uint2 cur = lane < num_ops ? ops[lane] : make_uint2(0u, 0u);
  uint2 ahead = 64 + lane < num_ops ? ops[64 + lane] : make_uint2(0u, 0u);

  int b = 0;
  int64_t expo = 0;  // true boundary = stored boundary * 2^expo
  // exponent taken out of the staged matrix, added to expo when that matrix
  // is applied (uniform)
  int pend = 0;
  int sb = 0;  // stage holding the next GATE's matrix
  bool prev_track = false;
  Real lmax = 0;
  if (lane == 0) {
    B[0].x = (Real)1;
    B[0].y = (Real)0;
  }
  // the set-up loads land before the op loop, which otherwise waits for
  // every outstanding load (the ring's too) at each op
  __builtin_amdgcn_s_waitcnt(0x0F70);  // vmcnt(0)
  if (lane < 32) stage[my_off] = nxt;
  int jst = 1;  // matrix the next GATE stages
  nxt = mats[mat_index(jst)];
  wave_fence();
  for (int t0 = 0; t0 < num_ops; t0 += 64) {
    const int lim = num_ops - t0 < 64 ? num_ops - t0 : 64;
    for (int tt = 0; tt < lim; ++tt) {
      const unsigned w0 = (unsigned)__builtin_amdgcn_readlane((int)cur.x, tt);
      const int type = (int)(w0 & OP_TYPE_MASK);
      const bool track = (w0 & OP_FLAG_TRACK) != 0;
      const int p = (int)((w0 >> 8) & 0xff), q = (int)((w0 >> 16) & 0xff);
      if (type == OP_GATE) {
        const int lo = p < q ? p : q, hi = p < q ? q : p;
        const int ip = 1 << p, iq = 1 << q;
        const Real* st = stage + 32 * sb;
        if (b <= 6) {
          if (track) gate_small<Real, BF3, true>(B, st, b, lo, hi, ip, iq, p, q, lane, lmax);
          else gate_small<Real, BF3, false>(B, st, b, lo, hi, ip, iq, p, q, lane, lmax);
        } else {
          if (track) gate_big<Real, BF3, true>(B, st, b, lo, hi, ip, iq, lane, lmax);
          else gate_big<Real, BF3, false>(B, st, b, lo, hi, ip, iq, lane, lmax);
        }
        // the other stage was last read by the previous GATE, before its fence
        sb ^= 1;
        if (lane < 32) stage[32 * sb + my_off] = nxt;
        ++jst;
        expo += pend;
        pend = 0;
      } else if (type == OP_BELL) {
        const int s = 1 << b;
        for (int k = lane; k < s; k += 64) {
          const Cplx<Real> v = B[k];
          Cplx<Real> z;
          z.x = (Real)0;
          z.y = (Real)0;
          B[k + s] = z;
          B[k + 2 * s] = z;
          B[k + 3 * s] = v;
        }
        b += 2;
      } else if (type == OP_TRACE) {
        if (track) trace_wave<Real, true>(B, b, p, q, lane, lmax);
        else trace_wave<Real, false>(B, b, p, q, lane, lmax);
        b -= 2;
      } else {  // OP_COLEND: the op before it recorded the column's largest magnitude
        if (prev_track) {
          const Real m = wave_max<Real>(lmax);
          lmax = 0;
          int e = 0;
          if (m > (Real)0 && isfinite(m)) {
            frexp(m, &e);
            e = __builtin_amdgcn_readfirstlane(e);
          }
          // the next GATE's staged matrix takes out 2^e instead of 2^pend
          // (exact: powers of two)
          if (e != pend && lane < 32) {
            Real* x = stage + 32 * sb + my_off;
            *x = ldexp(*x, pend - e);
          }
          pend = e;
        }
      }
      prev_track = track;
      wave_fence();
      nxt = mats[mat_index(jst)];
    }
    cur = ahead;
    __builtin_amdgcn_sched_barrier(0);
    // unconditional, clamped to the last op (records past it are never
    // decoded), and after the copy above, so the load writes `ahead` itself
    const int na = t0 + 128 + lane;
    ahead = ops[na < num_ops ? na : num_ops - 1];
  }
  const Cplx<Real> v = B[0];
  if (lane == 0) {
    out[0] = ldexp((double)v.x, (int)(expo + log2f));
    out[1] = ldexp((double)v.y, (int)(expo + log2f));
  }
  wave_fence();  // B is reused by the wavefront's next pair
}

// One wavefront per pair: pair blockIdx * WPB + wave of the launch, or, with
// a range on the device, pairs taken in turn from its counter until none is
// left (each wavefront on its own; no workgroup barrier is involved).
template <typename Real, int CAP, int WPB, bool BF3>
__global__ void __launch_bounds__(64 * WPB) sweep_wave_kernel(SweepArgs a) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  const int wave = threadIdx.x >> 6;
  const int lane = threadIdx.x & 63;
  if (a.range == nullptr) {
    const int64_t pi = (int64_t)blockIdx.x * WPB + wave;
    if (pi < a.num_pairs) wave_pair<Real, CAP, BF3>(a, a.order ? (int64_t)a.order[pi] : pi, wave, lane, smem_raw);
    return;
  }
  const int32_t* order = a.order + a.range[0];
  const long long n = a.range[1];
  for (;;) {
    unsigned long long c = 0;
    if (lane == 0) c = atomicAdd(a.claim, 1ull);
    const long long pi = (long long)__shfl(c, 0, 64);
    if (pi >= n) break;
    wave_pair<Real, CAP, BF3>(a, (int64_t)order[pi], wave, lane, smem_raw);
  }
}

// Waves per workgroup: the LDS slots of 2^10-entry registers (8.3 KB per
// wavefront) fill a CU's 160 KB best in workgroups of two (18 wavefronts; four
// per workgroup leave room for only 16).
template <typename Real, int CAP, bool BF3>
static int launch_wave_t(const SweepArgs& a, hipStream_t s) {
  constexpr int WPB = CAP >= 10 ? 2 : 4;
  const size_t smem = WPB * wave_slot_bytes<Real, CAP>();
  if (smem > 64 * 1024) {
    hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(sweep_wave_kernel<Real, CAP, WPB, BF3>),
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)smem);
    if (e != hipSuccess) (void)hipGetLastError();
  }
  int64_t blocks = (a.num_pairs + WPB - 1) / WPB;
  if (a.range != nullptr) {  // claimed pairs: sized for grid_pairs, or as many workgroups as stay resident
    blocks = a.grid_pairs > 0 ? (a.grid_pairs + WPB - 1) / WPB
                              : (int64_t)resident_per_cu(reinterpret_cast<const void*>(
                                                             sweep_wave_kernel<Real, CAP, WPB, BF3>),
                                                         64 * WPB, smem) *
                                    device_cus();
  }
  hipLaunchKernelGGL((sweep_wave_kernel<Real, CAP, WPB, BF3>), dim3((unsigned)blocks), dim3(64 * WPB), smem, s, a);
  return check_launch("sweep_wave");
}

template <int CAP>
static int launch_wave_cap(const SweepArgs& a, int precision, hipStream_t s) {
  if (precision == FP_C128) return launch_wave_t<double, CAP, false>(a, s);
  return a.bf3 ? launch_wave_t<float, CAP, true>(a, s) : launch_wave_t<float, CAP, false>(a, s);
}

int launch_sweep_wave(const SweepArgs& a, int precision, int cap_bits, hipStream_t s) {
  if (a.num_pairs <= 0) return FP_OK;
  if (!a.wmat) return set_error(FP_EINVAL, "wave sweep needs precomputed gate matrices");
  if (cap_bits <= 8) return launch_wave_cap<8>(a, precision, s);
  if (cap_bits <= 10) return launch_wave_cap<10>(a, precision, s);
  return set_error(FP_EINVAL, "wave sweep holds at most 2^10 entries per pair");
}

}  // namespace fp
