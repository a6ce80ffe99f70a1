// Column-sweep kernels for ensembles of two-qubit gates (brickwork, local
// random).  They execute the register program of plan.h on one pair's
// boundary tensor: the tensor-network contraction of Tr(U^dagger V) along
// the qubit direction (Sec. II.A of the paper; Methods A).
//
// Layout: the boundary of a pair is 2^b complex numbers, index bit i = one
// wire segment.  Small and medium boundaries live in LDS (one group of NT
// lanes per pair); large ones in an HBM slot owned by a workgroup.  After
// every column the boundary is scaled by an exact power of two so that its
// largest component lies in [0.5, 1); the exponents are summed into a
// float64 scale.
#include <hip/hip_runtime.h>
#include <math.h>
#include <string.h>

#include "internal.h"
#include "layout.h"
#include "plan.h"
#include "plan_wave.h"
#include "sweep.h"
#include "sweep_dev.h"

namespace fp {

// One group of NT lanes per pair, PB pairs per workgroup, boundary in LDS
// (2^cap_bits complex per pair) next to the staging area of the group.
// Pairs whose plan needs more are left to the next launch; failed plans give NaN.
template <typename Real, int NT, bool BF3>
__device__ __forceinline__ void lds_pair(const SweepArgs& a, int64_t pidx, int slot, int lane,
                                         unsigned char* smem_raw, Real* red) {
  const PlanHeader* hdr = a.hdr + pidx * a.hdr_stride;
  const int status = hdr->status, peak = hdr->peak_bits;
  double* out = a.trace + 2 * (a.trace_offset + pidx);
  if (status != 0) {
    if (lane == 0) {
      out[0] = __builtin_nan("");
      out[1] = __builtin_nan("");
    }
    return;
  }
  if (peak > a.cap_bits || peak <= a.min_bits) return;
  const size_t per_pair = ((size_t)sizeof(Cplx<Real>) << a.cap_bits) + stage_bytes<Real, NT, BF3>();
  unsigned char* base = smem_raw + per_pair * slot;
  Cplx<Real>* B = reinterpret_cast<Cplx<Real>*>(base);
  Cplx<Real>* mats = reinterpret_cast<Cplx<Real>*>(base + ((size_t)sizeof(Cplx<Real>) << a.cap_bits));
  Op* ops_s = reinterpret_cast<Op*>(mats + 16 * chunk_ops<NT>());
  const Real* pg = reinterpret_cast<const Real*>(a.gates + pidx * a.gate_stride);
  double re, im;
  const Real* wm = a.wmat ? reinterpret_cast<const Real*>(a.wmat + pidx * a.wmat_stride) : nullptr;
  run_program<Real, NT, BF3>(B, mats, ops_s, a.ops + pidx * a.ops_stride, hdr->num_ops,
                             a.wgates + pidx * a.wg_stride, a.factors + pidx * a.f_stride, pg, a.G, hdr->log2_factor,
                             lane, red, &re, &im, wm, hdr->num_gate_ops);
  if (lane == 0) {
    out[0] = re;
    out[1] = im;
  }
}

// Pair blockIdx * PB + slot of the launch, or, with a range on the device
// (one pair per workgroup), pairs taken in turn from its counter until none
// is left.
template <typename Real, int NT, int PB, bool BF3>
__global__ void __launch_bounds__(NT* PB) sweep_lds_kernel(SweepArgs a) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  __shared__ Real red[16];
  __shared__ unsigned long long claimed;
  const int slot = threadIdx.x / NT;
  const int lane = threadIdx.x % NT;
  if (PB > 1 || a.range == nullptr) {
    const int64_t pi = (int64_t)blockIdx.x * PB + slot;
    if (pi < a.num_pairs) lds_pair<Real, NT, BF3>(a, a.order ? (int64_t)a.order[pi] : pi, slot, lane, smem_raw, red);
    return;
  }
  const int32_t* order = a.order + a.range[0];
  const unsigned long long n = (unsigned long long)a.range[1];
  for (;;) {
    if (threadIdx.x == 0) claimed = atomicAdd(a.claim, 1ull);
    __syncthreads();
    const unsigned long long pi = claimed;
    __syncthreads();
    if (pi >= n) break;
    lds_pair<Real, NT, BF3>(a, (int64_t)order[pi], 0, lane, smem_raw, red);
    __syncthreads();  // the register and staging area are reused by the next pair
  }
}

// Large boundaries: one workgroup per pair at a time, pairs taken from a
// shared counter.  The boundary lives in LDS (2^14 complex64 or 2^13
// complex128 entries, 128 KiB) while it fits and in the workgroup's HBM slot
// (2^slot_bits entries) only while it does not: the BELL that grows it past
// LDS writes its result into the slot, the TRACE that brings it back writes
// its result into LDS.  In a local random pair at 200 steps on 50 qubits some
// 390 of 400 ops stay in LDS; the few beyond carry most of the entries.
// The interpreter runs the same programs with the same arithmetic as
// run_program, organised for memory latency:
//   * every lane keeps U groups (GATE), outputs (TRACE) or entries (BELL) in
//     flight, all loads of a round issued before its stores;
//   * op fields are read once per wavefront (scalar), so branching is uniform;
//   * the realigned matrices come precomputed in program order when the
//     caller has them (local random), else they are staged from the factors.
// 512 lanes with 8 (float), 6 (float, bf16x3 products) or 3 (double) items
// each: the most loads in flight without spilling registers.
constexpr int HBM_NT = 512;
template <typename Real, bool BF3>
constexpr int hbm_u() {
  return sizeof(Real) == 8 ? 3 : BF3 ? 6 : 8;
}
template <typename Real>
constexpr int hbm_lds_bits() {
  return sizeof(Real) == 8 ? 13 : 14;
}

// The helpers below work in rounds of NT * U items (groups, outputs,
// entries; the item counts are powers of two).  Past the end of the range the
// item index wraps around: every load is valid and issued unconditionally, so
// all loads of a round are in flight together, and only the owner of an item
// (index below the count) stores it or counts it in the column maximum.
// Without wrapping (count a multiple of NT * U) every lane owns its items.
// The *_any entry points halve U while a round would be larger than the
// range, and with U = 1 a wavefront that owns no item does nothing.

// GATE: the realigned matrix (Rr, Ri) on the 2^(b-2) groups of four entries
// (bits lo < hi of the group index are the gate's bits).
// I: the index type of the register, int up to 2^31 entries, int64_t beyond.
template <typename Real, int NT, int U, bool BF3, typename I>
__device__ __forceinline__ void gate_rounds(Cplx<Real>* B, const Real (&Rr)[16], const Real (&Ri)[16], int lo, int hi,
                                            I ip, I iq, I ng, int lane, bool track, Real& lmax, I base = 0) {
  const bool whole = ng % (NT * U) == 0;
  if (U == 1 && (I)(lane & ~63) >= ng) return;
  for (I g0 = 0; g0 < ng; g0 += NT * U) {
    Cplx<Real> v[U][4];
    I idx[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const I g = base + ((g0 + lane + u * NT) & (ng - 1));
      idx[u] = insert_zero(insert_zero(g, lo), hi);
      v[u][0] = B[idx[u]];
      v[u][1] = B[idx[u] + ip];
      v[u][2] = B[idx[u] + iq];
      v[u][3] = B[idx[u] + ip + iq];
    }
    Cplx<Real> w[U][4];
#pragma unroll
    for (int u = 0; u < U; ++u) {
#pragma unroll
      for (int jp = 0; jp < 4; ++jp) {
        Real sr = 0, si = 0;
#pragma unroll
        for (int j = 0; j < 4; ++j) cmac<Real, BF3>(Rr[jp * 4 + j], Ri[jp * 4 + j], v[u][j].x, v[u][j].y, sr, si);
        w[u][jp].x = sr;
        w[u][jp].y = si;
        if (track && (whole || g0 + lane + u * NT < ng)) lmax = fmax(lmax, fmax(fabs(sr), fabs(si)));
      }
    }
#pragma unroll
    for (int u = 0; u < U; ++u) {
      if (whole || g0 + lane + u * NT < ng) {
        B[idx[u]] = w[u][0];
        B[idx[u] + ip] = w[u][1];
        B[idx[u] + iq] = w[u][2];
        B[idx[u] + ip + iq] = w[u][3];
      }
    }
  }
}

template <typename Real, int NT, int U, bool BF3, typename I>
__device__ __forceinline__ void gate_any(Cplx<Real>* B, const Real (&Rr)[16], const Real (&Ri)[16], int lo, int hi,
                                         I ip, I iq, I ng, int lane, bool track, Real& lmax) {
  if constexpr (U > 1) {
    if (ng < NT * U) {
      gate_any<Real, NT, U / 2, BF3, I>(B, Rr, Ri, lo, hi, ip, iq, ng, lane, track, lmax);
      return;
    }
  }
  gate_rounds<Real, NT, U, BF3, I>(B, Rr, Ri, lo, hi, ip, iq, ng, lane, track, lmax);
}

// A run of m consecutive GATEs on a register of 2^b entries in global memory
// (H), applied tile by tile through LDS (L): the tile bits are the bits the
// run touches, topped up with the lowest other bits to nb = log2(entries of
// L) bits; a tile holds the 2^nb entries that agree on every other bit.  Each
// tile is read once, takes every GATE of the run in LDS (in order; entries
// at rsw(local index), as the LDS sweep keeps them), and is written back
// once: one pass over the register for the run instead of one per GATE.
// mats/ops: the run's staged matrices and op records; the first matrix comes
// scaled in (Rr0, Ri0).  Every lane of the workgroup calls it (NT lanes);
// b > nb.
template <typename Real, int NT, int NB, bool BF3, typename I>
__device__ void gate_run_tiled(Cplx<Real>* H, Cplx<Real>* L, const Real (&Rr0)[16], const Real (&Ri0)[16],
                               const Cplx<Real>* mats, const uint2* ops, int m, int b, bool track_last, int lane,
                               Real& lmax, int sc) {
  constexpr int LANE_BITS = NT == 512 ? 9 : NT == 256 ? 8 : 10;
  static_assert((1 << LANE_BITS) == NT, "tiles take NT lanes per row");
  constexpr int nb = NB;

  uint64_t tmask = 0;
  for (int g = 0; g < m; ++g) {
    const unsigned w = (unsigned)__builtin_amdgcn_readfirstlane((int)ops[g].x);
    tmask |= (1ull << ((w >> 8) & 0xff)) | (1ull << ((w >> 16) & 0xff));
  }
  for (int bit = 0; __popcll(tmask) < nb; ++bit) tmask |= 1ull << bit;
  const uint64_t omask = ((b >= 64 ? ~0ull : (1ull << b) - 1)) & ~tmask;
  // the lane's bits of a local index, deposited at the lowest tile bits
  I dep_lane = 0;
  uint64_t hi_mask = tmask;  // tile bits above the lane's
  for (int j = 0; j < LANE_BITS; ++j) {
    const int pos = __ffsll((long long)hi_mask) - 1;
    hi_mask &= hi_mask - 1;
    if ((lane >> j) & 1) dep_lane += (I)1 << pos;
  }
  constexpr int per_lane = 1 << (NB - LANE_BITS);
  const I ntiles = (I)1 << (b - nb);
  constexpr int V = per_lane < 8 ? per_lane : 8;  // loads in flight per lane
  for (I tau = 0; tau < ntiles; ++tau) {
    I base = 0;  // tau's bits deposited at the other bits (uniform)
    {
      uint64_t mm = omask;
      for (I t = tau; t != 0; t >>= 1) {
        const int pos = __ffsll((long long)mm) - 1;
        mm &= mm - 1;
        if (t & 1) base += (I)1 << pos;
      }
    }
    for (int pass = 0; pass < 2; ++pass) {  // 0: read the tile, 1: write it back
      if (pass == 1) {
       if constexpr (BF3) {
        // BF16x3: the run's GATEs as matrix-core blocks on the tile (pairs on
        // four distinct bits, else one GATE times the identity); the first
        // block takes out the column's power of two
        __shared__ __align__(16) unsigned short fblk[MFMA_BLOCK_BYTES / 2];  // the block planes
        const Cplx<float>* mf = reinterpret_cast<const Cplx<float>*>(mats);
        Cplx<float>* Lf = reinterpret_cast<Cplx<float>*>(L);
        float lm = (float)lmax;
        for (int g = 0; g < m;) {
          const unsigned w = (unsigned)__builtin_amdgcn_readfirstlane((int)ops[g].x);
          const int p = (int)((w >> 8) & 0xff), q = (int)((w >> 16) & 0xff);
          const int lp = __popcll(tmask & ((1ull << p) - 1)), lq = __popcll(tmask & ((1ull << q) - 1));
          const int s0 = g == 0 ? sc : 0;
          bool paired = false;
          if (g + 1 < m) {
            const unsigned w2 = (unsigned)__builtin_amdgcn_readfirstlane((int)ops[g + 1].x);
            const int p2 = (int)((w2 >> 8) & 0xff), q2 = (int)((w2 >> 16) & 0xff);
            if (p2 != p && p2 != q && q2 != p && q2 != q) {
              const int lp2 = __popcll(tmask & ((1ull << p2) - 1)), lq2 = __popcll(tmask & ((1ull << q2) - 1));
              const bool tr = track_last && g + 2 == m;
              if (tr) gate_pair_mfma<NT, true, true>(Lf, mf + 16 * g, mf + 16 * (g + 1), fblk, lp, lq, lp2, lq2, nb,
                                                     lane, s0, lm);
              else gate_pair_mfma<NT, false, true>(Lf, mf + 16 * g, mf + 16 * (g + 1), fblk, lp, lq, lp2, lq2, nb,
                                                   lane, s0, lm);
              paired = true;
            }
          }
          if (!paired) {
            int lb = 0;
            while (lb == lp || lb == lq) ++lb;
            int lc = lb + 1;
            while (lc == lp || lc == lq) ++lc;
            const bool tr = track_last && g + 1 == m;
            if (tr) gate_pair_mfma<NT, true, true, true>(Lf, mf + 16 * g, mf + 16 * g, fblk, lp, lq, lb, lc, nb, lane,
                                                         s0, lm);
            else gate_pair_mfma<NT, false, true, true>(Lf, mf + 16 * g, mf + 16 * g, fblk, lp, lq, lb, lc, nb, lane,
                                                       s0, lm);
          }
          __syncthreads();
          g += paired ? 2 : 1;
        }
        lmax = (Real)lm;
       } else {
        for (int g = 0; g < m; ++g) {
          const unsigned w = (unsigned)__builtin_amdgcn_readfirstlane((int)ops[g].x);
          const int p = (int)((w >> 8) & 0xff), q = (int)((w >> 16) & 0xff);
          const int lp = __popcll(tmask & ((1ull << p) - 1)), lq = __popcll(tmask & ((1ull << q) - 1));
          Real Rr[16], Ri[16];
#pragma unroll
          for (int k = 0; k < 16; ++k) {
            const Cplx<Real> r = mats[16 * g + k];
            Rr[k] = g == 0 ? Rr0[k] : r.x;
            Ri[k] = g == 0 ? Ri0[k] : r.y;
          }
          const int lo = lp < lq ? lp : lq, hi = lp < lq ? lq : lp;
          if (track_last && g == m - 1)
            gate_groups_u<Real, 1, BF3, true, false>(L, Rr, Ri, lo, hi, 1 << lp, 1 << lq, 1 << (nb - 2), lane, NT, 0,
                                                     lmax);
          else
            gate_groups_u<Real, 1, BF3, false, false>(L, Rr, Ri, lo, hi, 1 << lp, 1 << lq, 1 << (nb - 2), lane, NT,
                                                      0, lmax);
          __syncthreads();
        }
       }
      }
      for (int k0 = 0; k0 < per_lane; k0 += V) {
        I addr[V];
#pragma unroll
        for (int u = 0; u < V; ++u) {
          I dk = 0;  // (k0 + u)'s bits deposited at the tile bits above the lane's (uniform)
          uint64_t mm = hi_mask;
          for (int kk = k0 + u; kk != 0; kk >>= 1) {
            const int pos = __ffsll((long long)mm) - 1;
            mm &= mm - 1;
            if (kk & 1) dk += (I)1 << pos;
          }
          addr[u] = base + dep_lane + dk;
        }
        if (pass == 0) {
          Cplx<Real> v[V];
#pragma unroll
          for (int u = 0; u < V; ++u)
            if (k0 + u < per_lane) v[u] = H[addr[u]];
#pragma unroll
          for (int u = 0; u < V; ++u)
            if (k0 + u < per_lane) L[rsw(lane + (k0 + u) * NT)] = v[u];
        } else {
#pragma unroll
          for (int u = 0; u < V; ++u)
            if (k0 + u < per_lane) H[addr[u]] = L[rsw(lane + (k0 + u) * NT)];
        }
      }
      __syncthreads();
    }
  }
}

// BELL from b to b + 2 bits: dst[k + 3s] = src[k], dst[k + s] = dst[k + 2s] = 0
// (s = 2^b), and dst[k] = src[k] when the boundary moves (COPY); entries
// k = base .. base + n - 1.
template <typename Real, int NT, int U, bool COPY, typename I>
__device__ __forceinline__ void bell_rounds(const Cplx<Real>* src, Cplx<Real>* dst, I s, int lane, I n, I base) {
  const bool whole = n % (NT * U) == 0;
  if (U == 1 && (I)(lane & ~63) >= n) return;
  Cplx<Real> z;
  z.x = (Real)0;
  z.y = (Real)0;
  for (I k0 = 0; k0 < n; k0 += NT * U) {
    Cplx<Real> v[U];
#pragma unroll
    for (int u = 0; u < U; ++u) v[u] = src[base + ((k0 + lane + u * NT) & (n - 1))];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const I k = base + k0 + lane + u * NT;
      if (whole || k0 + lane + u * NT < n) {
        if (COPY) dst[k] = v[u];
        dst[k + s] = z;
        dst[k + 2 * s] = z;
        dst[k + 3 * s] = v[u];
      }
    }
  }
}

template <typename Real, int NT, int U, bool COPY, typename I>
__device__ __forceinline__ void bell_op(const Cplx<Real>* src, Cplx<Real>* dst, int b, int lane) {
  const I s = (I)1 << b;
  if constexpr (U > 1) {
    if (s < NT * U) {
      bell_op<Real, NT, U / 2, COPY, I>(src, dst, b, lane);
      return;
    }
  }
  bell_rounds<Real, NT, U, COPY, I>(src, dst, s, lane, s, (I)0);
}

// TRACE over bits p < q of a 2^b register: dst[j] = src[i0] + src[i0 + 2^p + 2^q],
// i0 = j with zeros inserted at p and q.  In place (src == dst) every round
// reads all its inputs before anyone writes (a barrier between); every input
// of a round lies at or above its outputs, and later rounds read above what
// earlier ones wrote.  The barriers are reached by every lane.
template <typename Real, int NT, int U, bool INPLACE, typename I>
__device__ __forceinline__ void trace_rounds(const Cplx<Real>* src, Cplx<Real>* dst, I nout, int p, int q, int lane,
                                             bool track, Real& lmax, I base = 0) {
  const I step = ((I)1 << p) + ((I)1 << q);
  const bool whole = nout % (NT * U) == 0;
  const bool idle = U == 1 && (I)(lane & ~63) >= nout;  // wavefront-uniform
  for (I j0 = 0; j0 < nout; j0 += NT * U) {
    Cplx<Real> acc[U];
    if (!idle) {
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const I i0 = insert_zero(insert_zero(base + ((j0 + lane + u * NT) & (nout - 1)), p), q);
        const Cplx<Real> a0 = src[i0], a1 = src[i0 + step];
        acc[u].x = a0.x + a1.x;
        acc[u].y = a0.y + a1.y;
        if (track && (whole || j0 + lane + u * NT < nout))
          lmax = fmax(lmax, fmax(fabs(acc[u].x), fabs(acc[u].y)));
      }
    }
    if (INPLACE) __syncthreads();
    if (!idle) {
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const I j = j0 + lane + u * NT;
        if (whole || j < nout) dst[base + j] = acc[u];
      }
    }
    if (INPLACE && j0 + NT * U < nout) __syncthreads();  // the last round ends at the op's barrier
  }
}

template <typename Real, int NT, int U, bool INPLACE, typename I>
__device__ __forceinline__ void trace_op(const Cplx<Real>* src, Cplx<Real>* dst, int b, int p, int q, int lane,
                                         bool track, Real& lmax) {
  const I nout = (I)1 << (b - 2);
  if constexpr (U > 1) {
    if (nout < NT * U) {
      trace_op<Real, NT, U / 2, INPLACE, I>(src, dst, b, p, q, lane, track, lmax);
      return;
    }
  }
  trace_rounds<Real, NT, U, INPLACE, I>(src, dst, nout, p, q, lane, track, lmax);
}

// TRACE outputs base .. base + nout - 1 (nout a power of two) in place with
// no barrier between reads and writes: for ranges where no output lands on
// an input of another output of the range (the rounds of a shared TRACE).
template <typename Real, int NT, int U, typename I>
__device__ __forceinline__ void trace_range(Cplx<Real>* B, I nout, int p, int q, int lane, bool track, Real& lmax,
                                            I base) {
  if constexpr (U > 1) {
    if (nout < NT * U) {
      trace_range<Real, NT, U / 2, I>(B, nout, p, q, lane, track, lmax, base);
      return;
    }
  }
  trace_rounds<Real, NT, U, false, I>(B, B, nout, p, q, lane, track, lmax, base);
}

// ---- work sharing among workgroups (widest pairs) ----
// Publication follows release/acquire at device scope: the owner fences its
// boundary writes and the record before it opens a task, a helper fences
// after claiming a chunk (before reading) and after writing it (before
// counting it done), and the owner fences after the count is complete.  Every
// wait is bounded: an owner waits only for chunks that running helpers hold,
// and helpers leave once every pair with a record has finished.
constexpr int HELP_WAIT_POLLS = 1 << 20;  // owner: polls for its helpers' chunks (each sleeps; about a second)
constexpr int HELP_IDLE_POLLS = 1 << 21;  // helper: polls in a row that found no open task (a few seconds)

__device__ __forceinline__ unsigned long long claim_word(unsigned seq, unsigned nch) {
  return ((unsigned long long)seq << 40) | ((unsigned long long)nch << 20);
}
__device__ __forceinline__ unsigned claim_next(unsigned long long w) { return (unsigned)(w & 0xFFFFFull); }
__device__ __forceinline__ unsigned claim_count(unsigned long long w) { return (unsigned)((w >> 20) & 0xFFFFFull); }

template <typename T>
__device__ __forceinline__ T load_agent(const T* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Items base .. base + n - 1 of a shared op (groups of GATE, entries of BELL,
// outputs of TRACE); BELL stays in place, TRACE goes from src to dst.
template <typename Real, int NT, int U, bool BF3, typename I>
__device__ __forceinline__ void shared_chunk(int type, int b, int p, int q, bool track, const Real (&Rr)[16],
                                             const Real (&Ri)[16], Cplx<Real>* src, Cplx<Real>* dst, I base, I n,
                                             int lane, Real& lmax) {
  if (type == OP_GATE) {
    const int lo = p < q ? p : q, hi = p < q ? q : p;
    gate_rounds<Real, NT, U, BF3, I>(src, Rr, Ri, lo, hi, (I)1 << p, (I)1 << q, n, lane, track, lmax, base);
  } else if (type == OP_BELL) {
    bell_rounds<Real, NT, U, false, I>(src, src, (I)1 << b, lane, n, base);
  } else {
    trace_rounds<Real, NT, U, false, I>(src, dst, n, p, q, lane, track, lmax, base);
  }
}

// Whether workgroups without a pair may exist: the pair counter (low 32 bits
// of the claim word) has run out.  Read by one lane and broadcast, so every
// wavefront takes the same branch.
__device__ __forceinline__ bool pairs_exhausted(const unsigned long long* counter, long long num_pairs, int lane,
                                                unsigned long long* sh) {
  if (lane == 0) sh[1] = (load_agent(counter) & 0xFFFFFFFFull) >= (unsigned long long)num_pairs ? 1ull : 0ull;
  __syncthreads();
  const bool r = sh[1] != 0;
  __syncthreads();
  return r;
}

// The owner's side of a shared op, called by every lane of its workgroup.
// GATE: (Rr, Ri) is the scaled matrix in registers, `mat` the unscaled one in
// LDS and sc the scale exponent removed from it.  The task covers items
// base .. base + 2^ibits - 1 with base = 2^base_bits (0 for base_bits < 0);
// ibits < 0: all of the op's items, from 0; ibits >= 12 otherwise.  Returns
// false if the helpers' chunks did not all finish within the wait bound.
template <typename Real, int NT, int U, bool BF3, typename I>
__device__ bool run_shared(HelpRec* rec, unsigned& seq, int type, int b, int p, int q, bool track,
                           const Real (&Rr)[16], const Real (&Ri)[16], const Cplx<Real>* mat, int sc,
                           Cplx<Real>* src, Cplx<Real>* dst, int lane, unsigned long long* sh, Real& lmax,
                           int base_bits = -1, int ibits = -1) {
  const I base = base_bits < 0 ? (I)0 : (I)1 << base_bits;
  const int cbits = ibits >= 0 ? ibits : type == OP_BELL ? b : b - 2;  // log2 of the task's items
  int chb = cbits - 8;                            // at most 256 chunks of 2^12 .. 2^15 items,
  chb = chb < 12 ? 12 : chb > 15 ? 15 : chb;      // more for the widest registers
  if (cbits - chb > 19) chb = cbits - 19;         // (the claim word counts up to 2^20 chunks)
  const unsigned nch = 1u << (cbits - chb);
  seq = (seq + 1) & 0xFFFFFFu;
  if (seq == 0) seq = 1;
  if (type == OP_GATE && lane < 32) {
    const Cplx<Real> r = mat[lane >> 1];
    const Real v = ldexp((lane & 1) ? r.y : r.x, -sc);  // the value the owner holds in Rr / Ri
    rec->mat[lane] = (unsigned long long)__double_as_longlong((double)v);
  }
  if (lane == 0) {
    rec->type = type;
    rec->b = b;
    rec->p = p;
    rec->q = q;
    rec->track = track ? 1 : 0;
    rec->chunk_bits = chb;
    rec->src = (unsigned long long)src;
    rec->dst = (unsigned long long)dst;
    rec->base_bits = base_bits;
    rec->maxbits = 0;
    rec->done = 0;
  }
  __threadfence();  // the boundary and the record reach device scope before the task opens
  __syncthreads();
  if (lane == 0) __hip_atomic_exchange(&rec->claim, claim_word(seq, nch), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  unsigned mine = 0;
  for (;;) {
    if (lane == 0) sh[0] = atomicAdd(&rec->claim, 1ull);
    __syncthreads();
    const unsigned c = claim_next(sh[0]);
    __syncthreads();
    if (c >= nch) break;
    shared_chunk<Real, NT, U, BF3, I>(type, b, p, q, track, Rr, Ri, src, dst, base + ((I)c << chb), (I)1 << chb, lane,
                                      lmax);
    ++mine;
  }
  if (lane == 0) {
    unsigned done = atomicAdd(&rec->done, mine) + mine;
    for (int polls = 0; done < nch && polls < HELP_WAIT_POLLS; ++polls) {
      __builtin_amdgcn_s_sleep(2);
      done = load_agent(&rec->done);
    }
    sh[1] = done >= nch ? 1ull : 0ull;
  }
  __syncthreads();
  __threadfence();  // every lane sees the helpers' entries
  const bool ok = sh[1] != 0;
  if (track) lmax = fmax(lmax, (Real)__longlong_as_double((long long)load_agent(&rec->maxbits)));
  __syncthreads();  // sh is reused
  return ok;
}

// A helper's chunk of the task in `rec`, claimed with word w.
template <typename Real, int NT, int U, bool BF3, typename I>
__device__ void help_chunk(HelpRec* rec, unsigned long long w, int lane, Real* red, Real* hmat) {
  __threadfence();  // acquire: the record and the boundary as the owner published them
  if (lane < 32) hmat[lane] = (Real)__longlong_as_double((long long)load_agent(&rec->mat[lane]));
  const int type = load_agent(&rec->type), b = load_agent(&rec->b), p = load_agent(&rec->p),
            q = load_agent(&rec->q), chb = load_agent(&rec->chunk_bits);
  const bool track = load_agent(&rec->track) != 0;
  Cplx<Real>* src = reinterpret_cast<Cplx<Real>*>(load_agent(&rec->src));
  Cplx<Real>* dst = reinterpret_cast<Cplx<Real>*>(load_agent(&rec->dst));
  const int base_bits = load_agent(&rec->base_bits);
  const I base = base_bits < 0 ? (I)0 : (I)1 << base_bits;
  __syncthreads();
  Real Rr[16], Ri[16];
#pragma unroll
  for (int k = 0; k < 16; ++k) {
    Rr[k] = hmat[2 * k];
    Ri[k] = hmat[2 * k + 1];
  }
  Real lmax = 0;
  shared_chunk<Real, NT, U, BF3, I>(type, b, p, q, track, Rr, Ri, src, dst, base + ((I)claim_next(w) << chb),
                                    (I)1 << chb, lane, lmax);
  if (track) {
    const Real m = group_max<Real, NT>(lmax, red);
    if (lane == 0) atomicMax(&rec->maxbits, (unsigned long long)__double_as_longlong((double)m));
  }
  __threadfence();  // release the chunk's entries before it counts as done
  __syncthreads();
  if (lane == 0) atomicAdd(&rec->done, 1u);
}

// TILED: runs of GATEs on a register in HBM go through gate_run_tiled (its
// registers cost the LDS-resident path some speed, so batches whose
// registers never leave LDS take the variant without it).
template <typename Real, int NT, int U, bool BF3, typename I, bool TILED>
__device__ __forceinline__ void run_program_big(Cplx<Real>* L, Cplx<Real>* H, Cplx<Real>* mats_s, uint2* ops_s,
                                                const Op* __restrict__ ops, int num_ops, int num_gate_ops,
                                                const Real* __restrict__ wmat, const int2* __restrict__ wgates,
                                                const int32_t* __restrict__ factors, const Real* pair_gates, int G,
                                                int log2_factor, int lane, Real* red, double* tr_re, double* tr_im,
                                                HelpRec* rec, Cplx<Real>* H2, int help_bits, bool helpers,
                                                const unsigned long long* counter, long long num_pairs,
                                                unsigned long long* sh) {
  constexpr int K = 64;  // ops staged per chunk: one per lane of the first wavefront
  constexpr int LB = hbm_lds_bits<Real>();
  const Real Rr0[16] = {}, Ri0[16] = {};  // matrix argument of shared ops other than GATE (unused)
  int b = 0;
  bool in_lds = true;
  int64_t expo = 0;  // true boundary = stored boundary * 2^expo
  int pend = 0;      // exponent to remove at the next GATE
  bool prev_track = false;
  int gate_base = 0;  // GATE ops before the chunk (first wavefront only)
  Real lmax = 0;
  unsigned seq = 0;       // tasks published in rec
  bool failed = false;    // a shared op was not completed
  bool exhausted = helpers;  // workgroups that only help exist, or the pair counter has run out
  // share an op of this pair with idle workgroups (uniform: every input is)
  auto share = [&](int reg_bits) {
    if (rec == nullptr || in_lds || reg_bits < help_bits || failed) return false;
    if (!exhausted) exhausted = pairs_exhausted(counter, num_pairs, lane, sh);
    return exhausted;
  };
  if (lane == 0) {
    L[0].x = (Real)1;
    L[0].y = (Real)0;
  }
  for (int t0 = 0; t0 < num_ops; t0 += K) {
    const int nk = num_ops - t0 < K ? num_ops - t0 : K;
    if (lane < K) {
      const uint2 w = lane < nk ? reinterpret_cast<const uint2*>(ops)[t0 + lane] : make_uint2(0u, 0u);
      const bool is_gate = lane < nk && (w.x & OP_TYPE_MASK) == OP_GATE;
      if (wmat) {
        const unsigned long long m = __ballot(is_gate);
        const unsigned long long below = lane ? (~0ull >> (64 - lane)) : 0ull;
        const int k = gate_base + __popcll(m & below);
        gate_base += __popcll(m);
        if (is_gate && k < num_gate_ops) {
          const Real* src = wmat + 32 * (int64_t)k;
          Real* dst = reinterpret_cast<Real*>(mats_s + 16 * lane);
#pragma unroll
          for (int r = 0; r < 32; ++r) dst[r] = src[r];
        }
      } else if (is_gate) {
        stage_gate<Real, BF3>(pair_gates, G, factors, wgates[(int)w.y], mats_s + 16 * lane);  // y: Op::arg
      }
      if (lane < nk) ops_s[lane] = w;
    }
    __syncthreads();
    for (int i = 0; i < nk; ++i) {
      const unsigned w0 = (unsigned)__builtin_amdgcn_readfirstlane((int)ops_s[i].x);
      const int type = (int)(w0 & OP_TYPE_MASK);
      const bool track = (w0 & OP_FLAG_TRACK) != 0;
      const int p = (int)((w0 >> 8) & 0xff), q = (int)((w0 >> 16) & 0xff);
      if (type == OP_GATE) {
        Real Rr[16], Ri[16];
        const int sc = __builtin_amdgcn_readfirstlane(pend);
#pragma unroll
        for (int k = 0; k < 16; ++k) {  // ldexp by 0 is the identity
          const Cplx<Real> r = mats_s[16 * i + k];
          Rr[k] = ldexp(r.x, -sc);
          Ri[k] = ldexp(r.y, -sc);
        }
        expo += pend;
        pend = 0;
        const int lo = p < q ? p : q, hi = p < q ? q : p;
        // consecutive GATEs that a tile of LB bits holds; registers of 2^18
        // entries or more (past what L2 keeps of them) hold bits 0..3 in the
        // tile too, so that its rows are whole 128-byte lines (measured at
        // brickwork n = 20: D = 10 8 % faster, D = 9, 2^16 entries, 11 % slower
        // with the low bits) (uniform)
        int run = 1;
        if (TILED && !in_lds && !track) {
          const uint64_t low = b >= 18 ? 0xFull : 0ull;
          uint64_t mask = (1ull << p) | (1ull << q);
          while (i + run < nk) {
            const unsigned w1 = (unsigned)__builtin_amdgcn_readfirstlane((int)ops_s[i + run].x);
            if ((int)(w1 & OP_TYPE_MASK) != OP_GATE) break;
            const uint64_t m2 = mask | (1ull << ((w1 >> 8) & 0xff)) | (1ull << ((w1 >> 16) & 0xff));
            if (__popcll(m2 | low) > LB) break;
            mask = m2;
            ++run;
            if (w1 & OP_FLAG_TRACK) break;  // the column's last writing op
          }
        }
        if (in_lds) {
          gate_any<Real, NT, U, BF3, int>(L, Rr, Ri, lo, hi, 1 << p, 1 << q, 1 << (b - 2), lane, track, lmax);
        } else if (share(b)) {
          failed |= !run_shared<Real, NT, U, BF3, I>(rec, seq, OP_GATE, b, p, q, track, Rr, Ri, mats_s + 16 * i, sc, H,
                                                     H, lane, sh, lmax);
        } else if (TILED && run >= 2) {
          const unsigned wl = (unsigned)__builtin_amdgcn_readfirstlane((int)ops_s[i + run - 1].x);
          const bool tl = (wl & OP_FLAG_TRACK) != 0;
          gate_run_tiled<Real, NT, LB, BF3, I>(H, L, Rr, Ri, mats_s + 16 * i, ops_s + i, run, b, tl, lane, lmax, sc);
          i += run - 1;
          prev_track = tl;
          continue;  // the tiled pass ended at a barrier
        } else {
          gate_any<Real, NT, U, BF3, I>(H, Rr, Ri, lo, hi, (I)1 << p, (I)1 << q, (I)1 << (b - 2), lane, track, lmax);
        }
      } else if (type == OP_BELL) {
        if (!in_lds && share(b + 2)) {
          failed |= !run_shared<Real, NT, U, BF3, I>(rec, seq, OP_BELL, b, p, q, false, Rr0, Ri0, mats_s, 0, H, H,
                                                     lane, sh, lmax);
        } else if (!in_lds) {
          bell_op<Real, NT, U, false, I>(H, H, b, lane);
        } else if (b + 2 <= LB) {
          bell_op<Real, NT, U, false, int>(L, L, b, lane);
        } else {
          bell_op<Real, NT, U, true, int>(L, H, b, lane);
          in_lds = false;
        }
        b += 2;
      } else if (type == OP_TRACE) {  // p < q
        if (in_lds) {
          trace_op<Real, NT, U, true, int>(L, L, b, p, q, lane, track, lmax);
        } else if (b - 2 > LB && H2 != nullptr && share(b)) {  // out of place, into the other buffer
          failed |= !run_shared<Real, NT, U, BF3, I>(rec, seq, OP_TRACE, b, p, q, track, Rr0, Ri0, mats_s, 0, H, H2,
                                                     lane, sh, lmax);
          Cplx<Real>* t = H;
          H = H2;
          H2 = t;
        } else if (b - 2 > LB && share(b)) {
          // In place, in rounds of outputs: [0, 2^(p+1)), then [2^k, 2^(k+1))
          // for k = p+1 .. b-3.  Output j lands on entry j; the inputs of
          // output j are entries i0(j) and i0(j) + 2^p + 2^q, both >= j.  An
          // entry y of round k that some other output reads belongs to output
          // y with bits p and q removed, which is below 2^k (an earlier round,
          // already done); below 2^(p+1) such entries are either the output's
          // own first input (j < 2^p) or read by no one.  So the outputs of a
          // round are independent and the rounds run one after another.
          const int nb = b - 2;
          const int k0 = p + 1 < nb ? p + 1 : nb;
          for (int k = k0 - 1; k < nb; ++k) {
            const int rbase = k < k0 ? -1 : k;  // the round's first output: 2^rbase (0 for -1)
            const int rbits = k < k0 ? k0 : k;  // log2 of its outputs
            if (rbits >= 16 && share(b))
              failed |= !run_shared<Real, NT, U, BF3, I>(rec, seq, OP_TRACE, b, p, q, track, Rr0, Ri0, mats_s, 0, H,
                                                         H, lane, sh, lmax, rbase, rbits);
            else
              trace_range<Real, NT, U, I>(H, (I)1 << rbits, p, q, lane, track, lmax,
                                          rbase < 0 ? (I)0 : (I)1 << rbase);
            __syncthreads();
          }
        } else if (b - 2 > LB) {
          trace_op<Real, NT, U, true, I>(H, H, b, p, q, lane, track, lmax);
        } else {
          trace_op<Real, NT, U, false, int>(H, L, b, p, q, lane, track, lmax);
          in_lds = true;
        }
        b -= 2;
      } else if (prev_track) {  // OP_COLEND after the column's last writing op
        const Real m = group_max<Real, NT>(lmax, red);
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
  }
  const Cplx<Real> v = in_lds ? L[0] : H[0];
  *tr_re = failed ? __builtin_nan("") : ldexp((double)v.x, (int)(expo + log2_factor));
  *tr_im = failed ? __builtin_nan("") : ldexp((double)v.y, (int)(expo + log2_factor));
}

template <typename Real>
constexpr size_t hbm_lds_bytes() {
  return (size_t)sizeof(Cplx<Real>) << hbm_lds_bits<Real>();
}

__device__ __forceinline__ int slot_bits_of(const SlotArgs& sl, int j) {
  int b = SLOT_BITS;
  while (b > 0 && sl.ge[b] <= j) --b;
  return b;
}

// Owners take pairs with one atomic on the claim word: the low 32 bits count
// pairs, the high 32 bits first claims, so the j-th first claim has taken a
// pair of rank >= j, no wider than slot j.  Every pair below wide_pairs
// counts in `finished` whatever its path, and helpers leave once all have.
template <typename Real, int NT, bool BF3, typename I, bool TILED>
__global__ void __launch_bounds__(NT) sweep_hbm_kernel(SweepArgs a, unsigned long long* counter, SlotArgs sl_arg,
                                                       HelpArgs h_arg, const LrDev* dev, int phase) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  __shared__ Real red[16];
  __shared__ unsigned long long next;
  __shared__ __align__(16) Cplx<Real> mats[16 * 64];
  __shared__ uint2 ops_s[64];
  __shared__ unsigned long long sh[2];
  __shared__ Real hmat[32];
  constexpr int U = hbm_u<Real, BF3>();
  const int lane = threadIdx.x;
  // launch arguments, or the set-up the device wrote for this phase of the class
  const HbmPhase* ph = dev != nullptr ? &dev->ph[phase] : nullptr;
  const SlotArgs& sl = ph != nullptr ? ph->sl : sl_arg;
  const HelpArgs& h = ph != nullptr ? ph->help : h_arg;
  const long long np = ph != nullptr ? ph->count : a.num_pairs;
  const int32_t* order = ph != nullptr ? a.order + dev->range[4][0] + ph->first : a.order;
  const int wgs = ph != nullptr ? ph->workgroups : (int)gridDim.x;
  const int owners = sl.owners;
  if ((int)blockIdx.x >= wgs) return;
  if (owners == 0) {  // no slot fits the pool: every pair of the class gets NaN
    for (long long pi = (long long)blockIdx.x * NT + lane; pi < np; pi += (long long)wgs * NT) {
      const int64_t pidx = order ? (int64_t)order[pi] : (int64_t)pi;
      double* out = a.trace + 2 * (a.trace_offset + pidx);
      out[0] = __builtin_nan("");
      out[1] = __builtin_nan("");
    }
    return;
  }
  const int nrec = h.recs == nullptr ? 0 : owners < HELP_MAX ? owners : HELP_MAX;
  const bool helpers = nrec > 0 && wgs > owners;  // workgroups that only help
  Cplx<Real>* L = reinterpret_cast<Cplx<Real>*>(smem_raw);
  if ((int)blockIdx.x < owners) {
    Cplx<Real>* S = nullptr;
    Cplx<Real>* A = nullptr;
    HelpRec* rec = nullptr;
    int sbits = -1;
    // Once a shared op of this owner's pair did not complete, a helper may
    // still write into its slot: the slot is not used again, and the owner's
    // later pairs that would need it get NaN.
    bool poisoned = false;
    for (;;) {
      if (lane == 0) next = atomicAdd(counter, sbits < 0 ? (1ull << 32) + 1ull : 1ull);
      __syncthreads();
      const unsigned long long w = next;
      __syncthreads();
      if (sbits < 0) {  // first claim: this workgroup's slot
        const int j = (int)(w >> 32);
        const int b = slot_bits_of(sl, j);
        const long long k = (long long)(j - sl.ge[b + 1]) << b;
        sbits = b;
        S = reinterpret_cast<Cplx<Real>*>(sl.base) + sl.off[b] + k;
        if (j < nrec) {
          rec = h.recs + j;
          if (sl.alt != nullptr) A = reinterpret_cast<Cplx<Real>*>(sl.alt) + sl.alt_off[b] + k;
        }
      }
      const long long pi = (long long)(w & 0xFFFFFFFFull);
      if (pi >= np) break;
      const int64_t pidx = order ? (int64_t)order[pi] : (int64_t)pi;
      const PlanHeader* hdr = a.hdr + pidx * a.hdr_stride;
      if (hdr->status == 0 && hdr->peak_bits > a.cap_bits) {
        double* out = a.trace + 2 * (a.trace_offset + pidx);
        const bool uses_slot = hdr->peak_bits > hbm_lds_bits<Real>();
        const bool fits_index = sizeof(I) == 8 || hdr->peak_bits <= 31;  // 32-bit indices: up to 2^31 entries
        if (uses_slot && (hdr->peak_bits > sbits || poisoned || !fits_index)) {  // a wider slot or wider indices needed,
                                                                                  // or a slot it may not use
          if (lane == 0) {
            out[0] = __builtin_nan("");
            out[1] = __builtin_nan("");
          }
        } else {
          const Real* pg = reinterpret_cast<const Real*>(a.gates + pidx * a.gate_stride);
          const Real* wm = a.wmat ? reinterpret_cast<const Real*>(a.wmat + pidx * a.wmat_stride) : nullptr;
          double re, im;
          run_program_big<Real, NT, U, BF3, I, TILED>(L, S, mats, ops_s, a.ops + pidx * a.ops_stride, hdr->num_ops,
                                               hdr->num_gate_ops, wm, a.wgates + pidx * a.wg_stride,
                                               a.factors + pidx * a.f_stride, pg, a.G, hdr->log2_factor, lane, red,
                                               &re, &im, rec, A, h.help_bits, helpers, counter, np, sh);
          if (re != re) poisoned = true;  // uniform: every lane holds the same result
          if (lane == 0) {
            out[0] = re;
            out[1] = im;
          }
        }
      }
      if (nrec > 0 && pi < h.wide_pairs && lane == 0) atomicAdd(h.finished, 1u);
      __syncthreads();
    }
  }
  // a quarter of the owners stay to help (with the helpers-only workgroups,
  // enough to saturate HBM); the others free their compute unit
  if (nrec == 0 || ((int)blockIdx.x < owners && (blockIdx.x & 3) != 0)) return;
  // helping: take a chunk of any open task, starting from a record that
  // depends on the workgroup, until every pair of the launch has finished
  for (int idle = 0;;) {
    if (lane < 64) {
      const unsigned long long cw = lane < nrec ? load_agent(&h.recs[lane].claim) : 0ull;
      const bool open = (cw >> 40) != 0 && claim_next(cw) < claim_count(cw);
      const unsigned long long m = __ballot(open);
      unsigned long long got = 0, flag = 0;  // flag: 1 + record, or 1 << 32 to leave
      if (m != 0) {
        const int st = (int)(blockIdx.x % (unsigned)nrec);
        const unsigned long long from = m & (~0ull << st);
        const int r = __ffsll((long long)(from != 0 ? from : m)) - 1;
        if (lane == r) got = atomicAdd(&h.recs[r].claim, 1ull);
        got = __shfl(got, r, 64);
        if (claim_next(got) < claim_count(got)) flag = 1 + (unsigned long long)r;
      } else if (idle >= HELP_IDLE_POLLS || load_agent(h.finished) >= (unsigned long long)h.wide_pairs) {
        flag = 1ull << 32;
      }
      if (lane == 0) {
        sh[0] = got;
        sh[1] = flag;
      }
    }
    __syncthreads();
    const unsigned long long w = sh[0], flag = sh[1];
    __syncthreads();
    if (flag >> 32) break;
    if (flag == 0) {
      ++idle;
      __builtin_amdgcn_s_sleep(8);
      continue;
    }
    idle = 0;  // the bound is on polls in a row without a task
    help_chunk<Real, NT, U, BF3, I>(h.recs + (flag - 1), w, lane, red, hmat);
  }
}

// Device planner for local random pairs: one wavefront per pair.  The lanes
// copy the pair's bond list into LDS in the order of W (V's steps, then U's
// steps reversed); the wavefront then plans it cooperatively, with its
// scratch in LDS and the per-qubit and register tables in lane registers.
__global__ void __launch_bounds__(64) plan_local_random_kernel(PlanJob j) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  const int64_t pi = blockIdx.x;
  if (pi >= j.num_pairs) return;
  const int G = j.G;
  int16_t* scratch = reinterpret_cast<int16_t*>(smem_raw);
  int16_t* bw = scratch + PLAN_BOND_SLOT * 2 * G;  // shares a slot the planner fills only after reading it
  const int32_t* src = reinterpret_cast<const int32_t*>(j.gates + pi * j.gate_stride + j.bonds_off);
  for (int i = threadIdx.x; i < 2 * G; i += 64) {
    const int32_t b = i < G ? src[G + i] : src[2 * G - 1 - i];  // [U bonds][V bonds]
    bw[i] = (b >= 0 && b <= j.n - 2) ? (int16_t)b : (int16_t)-1;
  }
  WaveDev w;
  w.sync();
  const PlanHeader h = plan_pair_wave(w, j.n, G, bw, scratch, j.ops + pi * j.ops_stride,
                                      j.wgates + pi * j.wg_stride, j.factors + pi * j.f_stride,
                                      j.gseq + pi * j.gseq_stride);
  if (threadIdx.x != 0) return;
  j.hdr[pi] = h;
  if (h.status == 0) {
    atomicMax(j.max_peak, h.peak_bits);
    atomicAdd(&j.hist[h.peak_bits < PLAN_HIST ? h.peak_bits : PLAN_HIST - 1], 1);
    if (h.peak_bits > j.cap_bits) atomicAdd(j.num_large, 1);
    const int cls = h.peak_bits <= j.tiny_bits    ? 0
                    : h.peak_bits <= j.small_bits ? 1
                    : h.peak_bits <= j.mid_bits   ? 2
                    : h.peak_bits <= j.cap_bits   ? 3
                                                  : 4;
    atomicAdd(&j.class_macs[cls], h.macs);
  } else {
    atomicAdd(j.num_failed, 1);
  }
}

__global__ void __launch_bounds__(256) order_pairs_kernel(OrderJob j) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  int b = -1;
  if (i < j.num_pairs) {
    const PlanHeader* h = j.hdr + i * j.hdr_stride;
    if (h->status != 0) {
      double* out = j.trace + 2 * (j.trace_offset + i);
      out[0] = __builtin_nan("");
      out[1] = __builtin_nan("");
    } else {
      b = h->peak_bits < PLAN_HIST ? h->peak_bits : PLAN_HIST - 1;
    }
  }
  // one atomic per distinct width and wavefront: the lanes of equal width
  // take consecutive places after the block reserved by their leader
  const int lane = threadIdx.x & 63;
  const unsigned long long below = lane ? (~0ull >> (64 - lane)) : 0ull;
  unsigned long long todo = __ballot(b >= 0);
  while (todo) {
    const int leader = __ffsll((long long)todo) - 1;
    const int v = __shfl(b, leader, 64);
    const unsigned long long same = __ballot(b == v);
    int base = 0;
    if (lane == leader) base = atomicAdd(&j.cursor[v], __popcll(same));
    base = __shfl(base, leader, 64);
    if (b == v) j.order[j.first[v] + base + __popcll(same & below)] = (int32_t)i;
    todo &= ~same;
  }
}

int launch_order_pairs(const OrderJob& j, hipStream_t s) {
  if (j.num_pairs <= 0) return FP_OK;
  const int64_t blocks = (j.num_pairs + 255) / 256;
  hipLaunchKernelGGL(order_pairs_kernel, dim3((unsigned)blocks), dim3(256), 0, s, j);
  return check_launch("order_pairs");
}

size_t plan_lds_bytes(int G, int n) {
  (void)n;
  return 2 * (size_t)plan_wave_scratch_elems(G);
}

// ---- launchers --------------------------------------------------------------

template <typename Real, int NT, int PB, bool BF3>
static int launch_lds_t(const SweepArgs& a, hipStream_t s) {
  const size_t smem = (size_t)PB * ((((size_t)1 << a.cap_bits) * sizeof(Cplx<Real>)) + stage_bytes<Real, NT, BF3>());
  int64_t blocks = (a.num_pairs + PB - 1) / PB;
  if (smem > 64 * 1024) {
    hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(sweep_lds_kernel<Real, NT, PB, BF3>),
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)smem);
    if (e != hipSuccess) (void)hipGetLastError();  // the limit may already allow it
  }
  if (a.range != nullptr) {  // claimed pairs, one per workgroup
    if (PB > 1) return set_error(FP_EINVAL, "claimed pairs need one pair per workgroup");
    blocks = a.grid_pairs > 0 ? a.grid_pairs
                              : (int64_t)resident_per_cu(reinterpret_cast<const void*>(
                                                             sweep_lds_kernel<Real, NT, PB, BF3>),
                                                         NT * PB, smem) *
                                    device_cus();
  }
  hipLaunchKernelGGL((sweep_lds_kernel<Real, NT, PB, BF3>), dim3((unsigned)blocks), dim3(NT * PB), smem, s, a);
  return check_launch("sweep_lds");
}

// Tile choice -> (lanes per pair, pairs per workgroup); LDS bits come from the caller.
template <typename Real, bool BF3>
static int launch_lds_real(const SweepArgs& a, int tile, hipStream_t s) {
  switch (tile) {
    case TILE_16x16: return launch_lds_t<Real, 16, 16, BF3>(a, s);
    case TILE_64x4: return launch_lds_t<Real, 64, 4, BF3>(a, s);
    case TILE_64x1: return launch_lds_t<Real, 64, 1, BF3>(a, s);
    case TILE_256x1: return launch_lds_t<Real, 256, 1, BF3>(a, s);
    case TILE_512x1: return launch_lds_t<Real, 512, 1, BF3>(a, s);
    case TILE_1024x1:
      // float64 needs more than the 128 registers a 1024-lane workgroup allows
      if constexpr (sizeof(Real) == 8) return launch_lds_t<Real, 512, 1, BF3>(a, s);
      else return launch_lds_t<Real, 1024, 1, BF3>(a, s);
    default: return set_error(FP_EINVAL, "unknown sweep tile %d", tile);
  }
}

int launch_sweep_lds(const SweepArgs& a, int precision, int tile, hipStream_t s) {
  if (a.num_pairs <= 0) return FP_OK;
  if (precision == FP_C128) return launch_lds_real<double, false>(a, tile, s);
  return a.bf3 ? launch_lds_real<float, true>(a, tile, s) : launch_lds_real<float, false>(a, tile, s);
}

template <typename Real, bool BF3, typename I, bool TILED>
static void launch_hbm_t(const SweepArgs& a, unsigned long long* counter, const SlotArgs& sl, int grid,
                         const HelpArgs& h, const LrDev* dev, int phase, hipStream_t s) {
  const auto k = sweep_hbm_kernel<Real, HBM_NT, BF3, I, TILED>;
  const size_t smem = hbm_lds_bytes<Real>();
  hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(k), hipFuncAttributeMaxDynamicSharedMemorySize,
                                     (int)smem);
  if (e != hipSuccess) (void)hipGetLastError();  // the limit may already allow it
  hipLaunchKernelGGL(k, dim3(grid), dim3(HBM_NT), smem, s, a, counter, sl, h, dev, phase);
}

void make_slot_args(SlotArgs* sl, unsigned char* base, const int* width, int count, bool with_alt, int elem) {
  memset(sl, 0, sizeof(*sl));
  sl->base = base;
  sl->owners = count;
  for (int b = 0; b <= SLOT_TOP; ++b) {
    int c = 0;
    while (c < count && width[c] >= b) ++c;  // widths do not increase
    sl->ge[b] = b == SLOT_TOP ? 0 : c;
  }
  const int nalt = with_alt ? (count < HELP_MAX ? count : HELP_MAX) : 0;
  long long off = 0, aoff = 0;
  for (int b = SLOT_BITS; b >= 0; --b) {
    sl->off[b] = off;
    sl->alt_off[b] = aoff;
    const int lo = sl->ge[b + 1], hi = sl->ge[b];
    off += (long long)(hi - lo) << b;
    const int alo = lo < nalt ? lo : nalt, ahi = hi < nalt ? hi : nalt;
    aoff += (long long)(ahi - alo) << b;
  }
  sl->off[SLOT_TOP] = off;       // entries of the slots
  sl->alt_off[SLOT_TOP] = aoff;  // entries of the second slots, which follow them
  sl->alt = nalt > 0 ? base + off * elem : nullptr;
}

int64_t slot_args_entries(const SlotArgs& sl) {
  return sl.off[SLOT_TOP] + (sl.alt != nullptr ? sl.alt_off[SLOT_TOP] : 0);
}

// Width of the widest slot (0 without slots).
int slot_bits_host(const SlotArgs& sl) {
  int b = SLOT_BITS;
  while (b > 0 && sl.ge[b] == 0) --b;
  return b;
}

template <typename I, bool TILED>
static void launch_hbm_prec(const SweepArgs& a, int precision, unsigned long long* counter, const SlotArgs& sl,
                            int grid, const HelpArgs& h, const LrDev* dev, int phase, hipStream_t s) {
  if (precision == FP_C128)
    launch_hbm_t<double, false, I, TILED>(a, counter, sl, grid, h, dev, phase, s);
  else if (a.bf3)
    launch_hbm_t<float, true, I, TILED>(a, counter, sl, grid, h, dev, phase, s);
  else
    launch_hbm_t<float, false, I, TILED>(a, counter, sl, grid, h, dev, phase, s);
}

int launch_sweep_hbm(const SweepArgs& a, int precision, unsigned long long* counter, const SlotArgs& sl, int grid,
                     hipStream_t s, const HelpArgs* help) {
  if (a.num_pairs <= 0 || sl.owners <= 0) return FP_OK;
  if (a.num_pairs >= (1ll << 31)) return set_error(FP_EINVAL, "too many pairs for one launch");
  HelpArgs h = {nullptr, nullptr, 0, 0};
  if (help != nullptr && help->recs != nullptr && help->wide_pairs > 0) {
    // chunks of at least 2^12 items: GATE and TRACE registers from 2^14 entries, BELL inputs from 2^14
    if (!help->finished || help->help_bits < 16 || help->wide_pairs > a.num_pairs)
      return set_error(FP_EINVAL, "bad work-sharing arguments");
    h = *help;
  }
  if (grid < sl.owners || (grid > sl.owners && h.recs == nullptr)) return set_error(FP_EINVAL, "bad HBM grid");
  const int top = slot_bits_host(sl);
  if (top > 31)
    launch_hbm_prec<int64_t, true>(a, precision, counter, sl, grid, h, nullptr, 0, s);
  else if (top > (precision == FP_C128 ? hbm_lds_bits<double>() : hbm_lds_bits<float>()))
    launch_hbm_prec<int, true>(a, precision, counter, sl, grid, h, nullptr, 0, s);
  else
    launch_hbm_prec<int, false>(a, precision, counter, sl, grid, h, nullptr, 0, s);
  return check_launch("sweep_hbm");
}

int launch_sweep_hbm_dev(const SweepArgs& a, int precision, unsigned long long* counter, const LrDev* dev, int phase,
                         int grid, hipStream_t s, bool wide, bool tiled) {
  if (grid <= 0) return FP_OK;
  if (phase < 0 || phase >= HBM_PHASES) return set_error(FP_EINVAL, "bad HBM phase");
  SlotArgs sl;
  memset(&sl, 0, sizeof(sl));
  const HelpArgs h = {nullptr, nullptr, 0, 0};
  if (wide)
    launch_hbm_prec<int64_t, true>(a, precision, counter, sl, grid, h, dev, phase, s);
  else if (tiled)
    launch_hbm_prec<int, true>(a, precision, counter, sl, grid, h, dev, phase, s);
  else
    launch_hbm_prec<int, false>(a, precision, counter, sl, grid, h, dev, phase, s);
  return check_launch("sweep_hbm");
}

// One wavefront derives a local random chunk's launches from the planner's
// width histogram: the ordering pass's first positions, the class ranges, and
// for each launch of the HBM class its slots (slot j as wide as the launch's
// j-th widest pair, widths clipped to 2^SLOT_BITS entries; as many owners as
// the pool holds, up to max_owners; second slots for the first HELP_MAX when
// that keeps at least half of the owners; helpers-only workgroups on the
// compute units the owners leave free, where the pool limits the owners or a
// register is very wide).  It also clears the chunk's HBM counters and
// work-sharing records.  Lane b holds width b; sums over widths are
// wavefront reductions.
__device__ __forceinline__ long long wave_sum_ll(long long v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

__global__ void __launch_bounds__(64) lr_setup_kernel(LrSetupJob j) {
  const int lane = threadIdx.x;
  LrDev* d = j.dev;
  // above[b] (lane b): pairs whose peak is at least b, by a suffix scan
  long long above = j.hist[lane];
#pragma unroll
  for (int off = 1; off < 64; off <<= 1) {
    const long long t = __shfl_down(above, off, 64);
    if (lane + off < 64) above += t;
  }
  auto pos = [&](int b) -> long long {  // above[b], with above[< 0] = all and above[>= 64] = 0
    const long long v = __shfl(above, b < 0 ? 0 : b > 63 ? 63 : b, 64);
    return b >= PLAN_HIST ? 0ll : v;
  };
  const long long next = __shfl_down(above, 1, 64);
  d->first[lane] = (int32_t)(lane == 63 ? 0 : next);
  const int lo[5] = {-1, j.tiny_bits, j.small_bits, j.mid_bits, j.cap_bits};
  const int hi[5] = {j.tiny_bits, j.small_bits, j.mid_bits, j.cap_bits, PLAN_HIST - 1};
  long long rf[5], rc[5];
#pragma unroll
  for (int k = 0; k < 5; ++k) {
    const bool some = hi[k] > lo[k];
    const long long a = pos(hi[k] + 1), b = pos(lo[k] + 1);
    rf[k] = some ? a : 0;
    rc[k] = some ? b - a : 0;
  }
  if (lane < 5) {
    d->range[lane][0] = rf[lane];
    d->range[lane][1] = rc[lane];
    d->claim[lane] = 0;
  }
  // the chunk's HBM counters and work-sharing records start at zero
  for (int i = lane; i < (int)(HELP_AREA_BYTES / 8); i += 64) reinterpret_cast<unsigned long long*>(j.recs)[i] = 0ull;
  if (lane < HBM_PHASES) j.hbm_counter[lane] = 0ull;
  const long long pool_entries = j.pool_bytes > 0 ? j.pool_bytes >> j.elem_shift : 0;
  // The class's pairs wider than a compute unit's share of the pool run in
  // a launch of their own, before the others: slots as wide as theirs would
  // leave few owners for the rest of the class.
  int split = -1;
  {
    const long long share = j.num_cus > 0 ? pool_entries / j.num_cus : 0;
    const int sb = share > 0 ? 63 - __clzll(share) : 0;
    const long long above = pos(sb + 1);
    if (sb > j.lds_bits && sb < PLAN_HIST - 1 && above > 0 && above < rc[4]) split = sb;
  }
  int status = 0;
  // phase k: the class's pairs of widths wlo .. whi (every lane calls it)
  auto phase_setup = [&](int k, int wlo, int whi, long long first) {
    // cnt(b): the phase's pairs of width >= b
    auto cnt = [&](int b) -> long long { return b > whi ? 0ll : pos(b > wlo ? b : wlo) - pos(whi + 1); };
    const long long count = whi >= wlo ? cnt(wlo) : 0;
    const int wmax = count < j.max_owners ? (int)count : j.max_owners;
    // slot widths: a pair's register width, 0 for a pair that stays in LDS
    // (at most 2^lds_bits entries); lane b <= SLOT_BITS holds ge[b], pairs of
    // clipped slot width >= b (ge[0] = count)
    const long long wide_ge = cnt(j.lds_bits + 1);
    const long long pa = cnt(lane), pa1 = cnt(lane + 1);
    const long long ge = lane > SLOT_BITS ? 0 : lane == 0 ? count : lane <= j.lds_bits + 1 ? wide_ge : pa;
    const long long ge1 = lane >= SLOT_BITS ? 0 : lane + 1 <= j.lds_bits + 1 ? wide_ge : pa1;
    // entries of w slots, plus second slots for the first HELP_MAX of them
    // (slots of width 0 take none)
    auto entries = [&](int w, bool alt) {
      const long long na = alt ? (w < HELP_MAX ? w : HELP_MAX) : 0;
      const long long g0 = ge < w ? ge : w, g1 = ge1 < w ? ge1 : w;
      const long long a0 = g0 < na ? g0 : na, a1 = g1 < na ? g1 : na;
      return wave_sum_ll(lane >= 1 && lane <= SLOT_BITS ? ((g0 - g1) + (a0 - a1)) << lane : 0ll);
    };
    auto largest = [&](bool alt) {
      int l = 0, h = wmax;
      while (l < h) {
        const int m = (l + h + 1) / 2;
        if (entries(m, alt) <= pool_entries) l = m;
        else h = m - 1;
      }
      return l;
    };
    int owners = 0;
    bool alt = false, none = false;
    if (count > 0) {
      const int w0 = largest(false);
      const int w1 = largest(true);
      alt = w1 >= 1 && 2 * w1 >= w0;
      owners = alt ? w1 : w0;
      if (owners == 0) {  // no room for the widest pair's slot: all slots of width 0, pairs
        owners = wmax;    // that stay in LDS still run and the others get NaN
        none = true;
      }
    }
    // slot layout: ge, then offsets from the widest down (the sums above b, by a suffix scan)
    const int g0 = none ? (lane == 0 ? owners : 0) : (int)(ge < owners ? ge : owners);
    const int g1 = none ? 0 : (int)(ge1 < owners ? ge1 : owners);
    const int nalt = alt ? (owners < HELP_MAX ? owners : HELP_MAX) : 0;
    long long mine = lane >= 1 && lane <= SLOT_BITS ? (long long)(g0 - g1) << lane : 0;
    long long amine =
        lane >= 1 && lane <= SLOT_BITS ? (long long)((g0 < nalt ? g0 : nalt) - (g1 < nalt ? g1 : nalt)) << lane : 0;
    long long suf = mine, asuf = amine;  // inclusive sums over widths >= lane
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
      const long long t = __shfl_down(suf, off, 64), u = __shfl_down(asuf, off, 64);
      if (lane + off < 64) {
        suf += t;
        asuf += u;
      }
    }
    // cross-lane reads first, with every lane active
    const long long total = __shfl(suf, 0, 64), atotal = __shfl(asuf, 0, 64);
    const long long wide = count > 0 ? cnt(j.help_bits) : 0;
    const long long beyond = cnt(SLOT_BITS + 1);  // pairs wider than the widest slot
    const long long widest = cnt(j.wide_bits);    // pairs of 2^wide_bits entries or more
    const unsigned long long m = __ballot(lane >= wlo && lane <= whi && lane < PLAN_HIST && j.hist[lane] > 0);
    HbmPhase& P = d->ph[k];
    SlotArgs& sl = P.sl;
    if (lane <= SLOT_TOP) {
      sl.ge[lane] = lane < SLOT_TOP ? g0 : 0;
      sl.off[lane] = lane < SLOT_TOP ? suf - mine : total;  // entries of wider slots; [SLOT_TOP]: all
      sl.alt_off[lane] = lane < SLOT_TOP ? asuf - amine : atotal;
    }
    if (lane == 0) {
      sl.owners = owners;
      sl.base = j.pool;
      sl.alt = nalt > 0 ? j.pool + (total << j.elem_shift) : nullptr;
      HelpArgs& h = P.help;
      h.recs = owners > 0 && wide > 0 && !none ? j.recs : nullptr;
      h.finished = reinterpret_cast<unsigned int*>(reinterpret_cast<unsigned char*>(j.recs) +
                                                   HELP_MAX * sizeof(HelpRec)) + k;
      h.wide_pairs = wide;
      h.help_bits = j.help_bits;
      // the compute units the owners leave free help the widest pairs: where
      // the pool limits the owners, or where a register has 2^wide_bits
      // entries or more (narrower shared registers are left to the owners'
      // quarter that helps: helpers-only workgroups would hold compute units
      // the batch's LDS sweeps run on)
      int extra = 0;
      if (h.recs != nullptr && (owners < wmax || widest > 0)) {
        extra = j.num_cus - owners;
        extra = extra < 0 ? 0 : extra > j.max_helpers ? j.max_helpers : extra;
      }
      P.first = first;
      P.count = count;
      P.workgroups = owners == 0 ? (count > 0 ? 1 : 0) : owners + extra;
      P.max_bits = m == 0 ? 0 : 63 - __clzll((long long)m);
      status |= (beyond > 0 ? 1 : 0) | (none ? 2 : 0);
    }
    return count;
  };
  if (split >= 0) {
    const long long c0 = phase_setup(0, split + 1, PLAN_HIST - 1, 0);
    phase_setup(1, j.cap_bits + 1, split, c0);
  } else {
    phase_setup(0, j.cap_bits + 1, PLAN_HIST - 1, 0);
    phase_setup(1, 1, 0, rc[4]);  // empty
  }
  if (lane == 0) {
    const int w0 = d->ph[0].workgroups, w1 = d->ph[1].workgroups;
    d->hbm_workgroups = w0 > w1 ? w0 : w1;
    d->status = status;
  }
  {  // widest register: the highest width with pairs
    const unsigned long long m = __ballot(lane < PLAN_HIST && j.hist[lane] > 0);
    if (lane == 0) d->max_bits = m == 0 ? 0 : 63 - __clzll((long long)m);
  }
}

int launch_lr_setup(const LrSetupJob& j, hipStream_t s) {
  if (j.help_bits < 16 || j.wide_bits < j.help_bits || j.max_owners < 1 || j.elem_shift < 3 || !j.recs ||
      !j.hbm_counter || j.lds_bits < j.cap_bits)
    return set_error(FP_EINVAL, "bad set-up arguments");
  hipLaunchKernelGGL(lr_setup_kernel, dim3(1), dim3(64), 0, s, j);
  return check_launch("lr_setup");
}

__global__ void __launch_bounds__(256) zero_words_kernel(unsigned int* p, int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256) p[i] = 0u;
}

int launch_zero_words(void* p, int64_t n, hipStream_t s) {
  if (n <= 0) return FP_OK;
  int64_t blocks = (n + 255) / 256;
  if (blocks > 1024) blocks = 1024;
  hipLaunchKernelGGL(zero_words_kernel, dim3((unsigned)blocks), dim3(256), 0, s, (unsigned int*)p, n);
  return check_launch("zero_words");
}

int resident_per_cu(const void* kernel, int block, size_t smem) {
  int n = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, kernel, block, smem) != hipSuccess || n < 1) {
    (void)hipGetLastError();
    return 1;
  }
  return n;
}

int device_cus() {
  int dev = 0, n = 0;
  if (hipGetDevice(&dev) != hipSuccess ||
      hipDeviceGetAttribute(&n, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || n <= 0) {
    (void)hipGetLastError();
    return 256;
  }
  return n;
}

int launch_plan_local_random(const PlanJob& j, int precision, hipStream_t s) {
  (void)precision;
  if (j.num_pairs <= 0) return FP_OK;
  const size_t smem = plan_lds_bytes(j.G, j.n);
  if (smem > 160 * 1024) return set_error(FP_ETOOBIG, "%d steps per circuit exceed the planner's LDS", j.G);
  if (smem > 64 * 1024) {
    hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(plan_local_random_kernel),
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)smem);
    if (e != hipSuccess) (void)hipGetLastError();
  }
  hipLaunchKernelGGL(plan_local_random_kernel, dim3((unsigned)j.num_pairs), dim3(64), smem, s, j);
  return check_launch("plan_local_random");
}

__device__ __forceinline__ void store_matrix(const Cplx<float> (&m)[16], float* dst) {
  float4* v = reinterpret_cast<float4*>(dst);
#pragma unroll
  for (int i = 0; i < 8; ++i) v[i] = make_float4(m[2 * i].x, m[2 * i].y, m[2 * i + 1].x, m[2 * i + 1].y);
}
__device__ __forceinline__ void store_matrix(const Cplx<double> (&m)[16], double* dst) {
  double2* v = reinterpret_cast<double2*>(dst);
#pragma unroll
  for (int i = 0; i < 16; ++i) v[i] = make_double2(m[i].x, m[i].y);
}

// The realigned matrix of every GATE op, in program order: one thread per
// (pair, GATE op), the product of the merged gate's factors (same arithmetic
// as the staging of the LDS sweep).
template <typename Real, bool BF3>
__global__ void __launch_bounds__(256) gate_matrices_kernel(PlanJob j) {
  const int64_t tid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t per = 2 * (int64_t)j.G;
  const int64_t pi = tid / per;
  const int jj = (int)(tid - pi * per);
  if (pi >= j.num_pairs) return;
  const PlanHeader* h = j.hdr + pi;
  if (h->status != 0 || jj >= h->num_gate_ops) return;
  const int k = j.gseq[pi * j.gseq_stride + jj];
  const Real* pg = reinterpret_cast<const Real*>(j.gates + pi * j.gate_stride);
  Cplx<Real> m[16];
  stage_gate<Real, BF3>(pg, j.G, j.factors + pi * j.f_stride, j.wgates[pi * j.wg_stride + k], m);
  store_matrix(m, reinterpret_cast<Real*>(j.wmat + pi * j.wmat_stride) + 32 * (int64_t)jj);
}

// The same matrices with one workgroup per pair: the pair's gate block
// (2G gates, contiguous) is first copied to LDS with coalesced 16-byte
// loads, and every thread then multiplies its merged gate's factors from LDS
// (the per-thread form reads each 128-byte gate in eight strided pieces).
constexpr int PREP_NT = 256;
template <typename Real, bool BF3>
__global__ void __launch_bounds__(PREP_NT) gate_matrices_lds_kernel(PlanJob j) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  const int64_t pi = blockIdx.x;
  const PlanHeader* h = j.hdr + pi;
  const int ng = h->status != 0 ? 0 : h->num_gate_ops;  // uniform over the workgroup
  if (ng <= 0) return;
  const int n16 = (int)(2 * (int64_t)j.G * 32 * (int64_t)sizeof(Real) / 16);
  const float4* src = reinterpret_cast<const float4*>(j.gates + pi * j.gate_stride);
  float4* lds = reinterpret_cast<float4*>(smem_raw);
  for (int i = threadIdx.x; i < n16; i += PREP_NT) lds[i] = src[i];
  __syncthreads();
  const Real* pg = reinterpret_cast<const Real*>(smem_raw);
  Real* out = reinterpret_cast<Real*>(j.wmat + pi * j.wmat_stride);
  if (ng > PREP_NT) {  // several matrices per thread: stored as they are made
    for (int jj = threadIdx.x; jj < ng; jj += PREP_NT) {
      const int k = j.gseq[pi * j.gseq_stride + jj];
      Cplx<Real> m[16];
      stage_gate<Real, BF3>(pg, j.G, j.factors + pi * j.f_stride, j.wgates[pi * j.wg_stride + k], m);
      store_matrix(m, out + 32 * (int64_t)jj);
    }
    return;
  }
  // one matrix per thread: the matrices replace the gate block in LDS (ng <=
  // 2G blocks of the same size) once every thread has read its factors, and
  // leave with coalesced stores
  const int jj = threadIdx.x;
  Cplx<Real> m[16];
  if (jj < ng) {
    const int k = j.gseq[pi * j.gseq_stride + jj];
    stage_gate<Real, BF3>(pg, j.G, j.factors + pi * j.f_stride, j.wgates[pi * j.wg_stride + k], m);
  }
  __syncthreads();
  if (jj < ng) store_matrix(m, reinterpret_cast<Real*>(smem_raw) + 32 * jj);
  __syncthreads();
  const int o16 = (int)((int64_t)ng * 32 * (int64_t)sizeof(Real) / 16);
  float4* dst = reinterpret_cast<float4*>(out);
  for (int i = threadIdx.x; i < o16; i += PREP_NT) dst[i] = lds[i];
}

int launch_gate_matrices(const PlanJob& j, int precision, hipStream_t s) {
  if (j.num_pairs <= 0) return FP_OK;
  const size_t elem = precision == FP_C128 ? sizeof(double) : sizeof(float);
  const size_t smem = 2 * (size_t)j.G * 32 * elem;  // the pair's gate block
  if (smem <= 64 * 1024) {
    const dim3 grid((unsigned)j.num_pairs);
    if (precision == FP_C128)
      hipLaunchKernelGGL((gate_matrices_lds_kernel<double, false>), grid, dim3(PREP_NT), smem, s, j);
    else if (j.bf3)
      hipLaunchKernelGGL((gate_matrices_lds_kernel<float, true>), grid, dim3(PREP_NT), smem, s, j);
    else
      hipLaunchKernelGGL((gate_matrices_lds_kernel<float, false>), grid, dim3(PREP_NT), smem, s, j);
    return check_launch("gate_matrices");
  }
  const int64_t threads = j.num_pairs * 2 * (int64_t)j.G;
  const int64_t blocks = (threads + 255) / 256;
  if (precision == FP_C128)
    hipLaunchKernelGGL((gate_matrices_kernel<double, false>), dim3((unsigned)blocks), dim3(256), 0, s, j);
  else if (j.bf3)
    hipLaunchKernelGGL((gate_matrices_kernel<float, true>), dim3((unsigned)blocks), dim3(256), 0, s, j);
  else
    hipLaunchKernelGGL((gate_matrices_kernel<float, false>), dim3((unsigned)blocks), dim3(256), 0, s, j);
  return check_launch("gate_matrices");
}

int sweep_elem_bytes(int precision) { return precision == FP_C128 ? 16 : 8; }

}  // namespace fp
