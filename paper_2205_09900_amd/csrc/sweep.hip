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

#include "internal.h"
#include "layout.h"
#include "plan.h"
#include "sweep.h"

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

__device__ __forceinline__ int insert_zero(int x, int pos) {
  return ((x >> pos) << (pos + 1)) | (x & ((1 << pos) - 1));
}

// Merged gate M = F_last ... F_first (product of its factors) realigned for
// the column transfer and written to dst (16 complex):
//   dst[j' * 4 + j] = M[2 x_out + y_out][2 x_in + y_in],
// j = x_in + 2 x_out (legs on qubit c), j' = y_in + 2 y_out (legs on qubit c+1).
// dst doubles as the row buffer of the running product.
template <typename Real>
__device__ __forceinline__ void load_factor_row(const Real* src, int dagger, int a, Real (&fr)[4], Real (&fi)[4]) {
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    if (dagger) {
      fr[k] = src[(k * 4 + a) * 2];
      fi[k] = -src[(k * 4 + a) * 2 + 1];
    } else {
      fr[k] = src[(a * 4 + k) * 2];
      fi[k] = src[(a * 4 + k) * 2 + 1];
    }
  }
}

template <typename Real>
__device__ void stage_gate(const Real* __restrict__ pair_gates, int G, const int32_t* __restrict__ factors, int2 wg,
                           Cplx<Real>* dst) {
  Real mr[16], mi[16];
  {
    const FactorRef f0 = decode_factor(factors[wg.x], G);
    const Real* src = pair_gates + ((int64_t)f0.circuit * G + f0.gate) * 32;
#pragma unroll
    for (int a = 0; a < 4; ++a) {
      Real fr[4], fi[4];
      load_factor_row<Real>(src, f0.dagger, a, fr, fi);
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        mr[a * 4 + k] = fr[k];
        mi[a * 4 + k] = fi[k];
      }
    }
  }
  for (int f = 1; f < wg.y; ++f) {
    const FactorRef ff = decode_factor(factors[wg.x + f], G);
    const Real* src = pair_gates + ((int64_t)ff.circuit * G + ff.gate) * 32;
#pragma unroll
    for (int a = 0; a < 4; ++a) {
      Real fr[4], fi[4];
      load_factor_row<Real>(src, ff.dagger, a, fr, fi);
#pragma unroll
      for (int b = 0; b < 4; ++b) {
        Real sr = 0, si = 0;
#pragma unroll
        for (int k = 0; k < 4; ++k) {
          sr = fma(fr[k], mr[k * 4 + b], sr);
          sr = fma(-fi[k], mi[k * 4 + b], sr);
          si = fma(fr[k], mi[k * 4 + b], si);
          si = fma(fi[k], mr[k * 4 + b], si);
        }
        dst[a * 4 + b].x = sr;
        dst[a * 4 + b].y = si;
      }
    }
#pragma unroll
    for (int i = 0; i < 16; ++i) {
      mr[i] = dst[i].x;
      mi[i] = dst[i].y;
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
// parallel), then executes the ops from LDS.  The per-column rescale is
// lazy: the op that ends a column records the largest magnitude it writes,
// the column end turns it into an exponent P, and the next GATE multiplies
// its matrix by 2^-P (exact), so no extra pass over the boundary is made.
template <typename Real, int NT>
__device__ __forceinline__ void run_program(Cplx<Real>* B, Cplx<Real>* mats_s, Op* ops_s, const Op* __restrict__ ops,
                                            int num_ops, const int2* __restrict__ wgates,
                                            const int32_t* __restrict__ factors, const Real* pair_gates, int G,
                                            int log2_factor, int lane, Real* red, double* tr_re, double* tr_im) {
  constexpr int K = chunk_ops<NT>();
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
    for (int i = lane; i < nk; i += NT) {
      const Op op = ops[t0 + i];
      ops_s[i] = op;
      if ((op.type & OP_TYPE_MASK) == OP_GATE) stage_gate<Real>(pair_gates, G, factors, wgates[op.arg], mats_s + 16 * i);
    }
    group_sync<NT>();
    for (int i = 0; i < nk; ++i) {
      const Op op = ops_s[i];
      const int type = op.type & OP_TYPE_MASK;
      const bool track = (op.type & OP_FLAG_TRACK) != 0;
      if (type == OP_GATE) {
        Real Rr[16], Ri[16];
#pragma unroll
        for (int k = 0; k < 16; ++k) {
          const Cplx<Real> r = mats_s[16 * i + k];
          Rr[k] = pend ? ldexp(r.x, -pend) : r.x;
          Ri[k] = pend ? ldexp(r.y, -pend) : r.y;
        }
        expo += pend;
        pend = 0;
        const int p = op.p, q = op.q;
        const int lo = p < q ? p : q, hi = p < q ? q : p;
        const int ip = 1 << p, iq = 1 << q;
        const int ng = 1 << (b - 2);
        for (int g = lane; g < ng; g += NT) {
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
            for (int j = 0; j < 4; ++j) {
              sr = fma(Rr[jp * 4 + j], v[j].x, sr);
              sr = fma(-Ri[jp * 4 + j], v[j].y, sr);
              si = fma(Rr[jp * 4 + j], v[j].y, si);
              si = fma(Ri[jp * 4 + j], v[j].x, si);
            }
            w[jp].x = sr;
            w[jp].y = si;
            if (track) lmax = fmax(lmax, fmax(fabs(sr), fabs(si)));
          }
          B[idx] = w[0];
          B[idx + ip] = w[1];
          B[idx + iq] = w[2];
          B[idx + ip + iq] = w[3];
        }
      } else if (type == OP_BELL) {
        const int s = 1 << b;
        for (int k = lane; k < s; k += NT) {
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
        const int p = op.p, q = op.q;  // p < q
        const int nout = 1 << (b - 2);
        const int step = (1 << p) + (1 << q);
        for (int j0 = 0; j0 < nout; j0 += NT) {
          const int j = j0 + lane;
          Cplx<Real> acc;
          acc.x = (Real)0;
          acc.y = (Real)0;
          if (j < nout) {
            const int i0 = insert_zero(insert_zero(j, p), q);
            const Cplx<Real> a0 = B[i0], a1 = B[i0 + step];
            acc.x = a0.x + a1.x;
            acc.y = a0.y + a1.y;
            if (track) lmax = fmax(lmax, fmax(fabs(acc.x), fabs(acc.y)));
          }
          group_sync<NT>();
          if (j < nout) B[j] = acc;
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

template <typename Real, int NT>
constexpr size_t stage_bytes() {
  return (size_t)chunk_ops<NT>() * (16 * sizeof(Cplx<Real>) + sizeof(Op));
}

// One group of NT lanes per pair, PB pairs per workgroup, boundary in LDS
// (2^cap_bits complex per pair) next to the staging area of the group.
// Pairs whose plan needs more are left to the next launch; failed plans give NaN.
template <typename Real, int NT, int PB>
__global__ void __launch_bounds__(NT* PB) sweep_lds_kernel(SweepArgs a) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  __shared__ Real red[16];
  const int slot = threadIdx.x / NT;
  const int lane = threadIdx.x % NT;
  const int64_t pi = (int64_t)blockIdx.x * PB + slot;
  if (pi >= a.num_pairs) return;
  const int64_t pidx = pi;
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
  const size_t per_pair = ((size_t)sizeof(Cplx<Real>) << a.cap_bits) + stage_bytes<Real, NT>();
  unsigned char* base = smem_raw + per_pair * slot;
  Cplx<Real>* B = reinterpret_cast<Cplx<Real>*>(base);
  Cplx<Real>* mats = reinterpret_cast<Cplx<Real>*>(base + ((size_t)sizeof(Cplx<Real>) << a.cap_bits));
  Op* ops_s = reinterpret_cast<Op*>(mats + 16 * chunk_ops<NT>());
  const Real* pg = reinterpret_cast<const Real*>(a.gates + pidx * a.gate_stride);
  double re, im;
  run_program<Real, NT>(B, mats, ops_s, a.ops + pidx * a.ops_stride, hdr->num_ops, a.wgates + pidx * a.wg_stride,
                        a.factors + pidx * a.f_stride, pg, a.G, hdr->log2_factor, lane, red, &re, &im);
  if (lane == 0) {
    out[0] = re;
    out[1] = im;
  }
}

// Large boundaries: one workgroup per pair at a time, boundary in the HBM
// slot of the workgroup, staging in LDS, pairs taken from a shared counter.
template <typename Real, int NT>
__global__ void __launch_bounds__(NT) sweep_hbm_kernel(SweepArgs a, unsigned long long* counter,
                                                       unsigned char* slots, int slot_bits) {
  __shared__ Real red[16];
  __shared__ long long next;
  __shared__ __align__(16) Cplx<Real> mats[16 * chunk_ops<NT>()];
  __shared__ Op ops_s[chunk_ops<NT>()];
  const int lane = threadIdx.x;
  Cplx<Real>* B = reinterpret_cast<Cplx<Real>*>(slots) + ((int64_t)blockIdx.x << slot_bits);
  for (;;) {
    if (lane == 0) next = (long long)atomicAdd(counter, 1ull);
    __syncthreads();
    const long long pidx = next;
    __syncthreads();
    if (pidx >= a.num_pairs) break;
    const PlanHeader* hdr = a.hdr + pidx * a.hdr_stride;
    if (hdr->status != 0 || hdr->peak_bits <= a.cap_bits) continue;
    double* out = a.trace + 2 * (a.trace_offset + pidx);
    if (hdr->peak_bits > slot_bits) {
      if (lane == 0) {
        out[0] = __builtin_nan("");
        out[1] = __builtin_nan("");
      }
      continue;
    }
    const Real* pg = reinterpret_cast<const Real*>(a.gates + pidx * a.gate_stride);
    double re, im;
    run_program<Real, NT>(B, mats, ops_s, a.ops + pidx * a.ops_stride, hdr->num_ops, a.wgates + pidx * a.wg_stride,
                          a.factors + pidx * a.f_stride, pg, a.G, hdr->log2_factor, lane, red, &re, &im);
    if (lane == 0) {
      out[0] = re;
      out[1] = im;
    }
    __syncthreads();
  }
}

// Device planner for local random pairs: one wavefront per pair.  The lanes
// copy the pair's bond lists into LDS; lane 0 then runs the planner with all
// of its scratch in LDS (16-bit entries), so its sequential bookkeeping waits
// on LDS rather than on global memory.
__global__ void __launch_bounds__(64) plan_local_random_kernel(PlanJob j) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  const int64_t pi = blockIdx.x;
  if (pi >= j.num_pairs) return;
  const int G = j.G;
  int32_t* tags = reinterpret_cast<int32_t*>(smem_raw);
  int16_t* bonds = reinterpret_cast<int16_t*>(smem_raw + 256);
  int16_t* scratch = bonds + ((2 * G + 7) & ~7);
  const int32_t* src = reinterpret_cast<const int32_t*>(j.gates + pi * j.gate_stride + j.bonds_off);
  for (int i = threadIdx.x; i < 2 * G; i += 64) {
    const int32_t b = src[i];
    bonds[i] = (b >= 0 && b <= j.n - 2) ? (int16_t)b : (int16_t)-1;
  }
  __syncthreads();
  if (threadIdx.x != 0) return;
  PlanHeader h = plan_haar_pair(j.n, G, bonds, bonds + G, scratch, j.ops + pi * j.ops_stride,
                                j.wgates + pi * j.wg_stride, j.factors + pi * j.f_stride, tags);
  j.hdr[pi] = h;
  if (h.status == 0) {
    atomicMax(j.max_peak, h.peak_bits);
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

size_t plan_lds_bytes(int G, int n) {
  return 256 + 2 * (size_t)((2 * G + 7) & ~7) + 2 * (size_t)plan_scratch_elems(G, n);
}

// ---- launchers --------------------------------------------------------------

template <typename Real, int NT, int PB>
static int launch_lds_t(const SweepArgs& a, hipStream_t s) {
  const size_t smem = (size_t)PB * ((((size_t)1 << a.cap_bits) * sizeof(Cplx<Real>)) + stage_bytes<Real, NT>());
  const int64_t blocks = (a.num_pairs + PB - 1) / PB;
  if (smem > 64 * 1024) {
    hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(sweep_lds_kernel<Real, NT, PB>),
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)smem);
    if (e != hipSuccess) (void)hipGetLastError();  // the limit may already allow it
  }
  hipLaunchKernelGGL((sweep_lds_kernel<Real, NT, PB>), dim3((unsigned)blocks), dim3(NT * PB), smem, s, a);
  return check_launch("sweep_lds");
}

// Tile choice -> (lanes per pair, pairs per workgroup); LDS bits come from the caller.
template <typename Real>
static int launch_lds_real(const SweepArgs& a, int tile, hipStream_t s) {
  switch (tile) {
    case TILE_16x16: return launch_lds_t<Real, 16, 16>(a, s);
    case TILE_64x4: return launch_lds_t<Real, 64, 4>(a, s);
    case TILE_64x1: return launch_lds_t<Real, 64, 1>(a, s);
    case TILE_256x1: return launch_lds_t<Real, 256, 1>(a, s);
    case TILE_512x1: return launch_lds_t<Real, 512, 1>(a, s);
    case TILE_1024x1:
      // float64 needs more than the 128 registers a 1024-lane workgroup allows
      if constexpr (sizeof(Real) == 8) return launch_lds_t<Real, 512, 1>(a, s);
      else return launch_lds_t<Real, 1024, 1>(a, s);
    default: return set_error(FP_EINVAL, "unknown sweep tile %d", tile);
  }
}

int launch_sweep_lds(const SweepArgs& a, int precision, int tile, hipStream_t s) {
  if (a.num_pairs <= 0) return FP_OK;
  return precision == FP_C128 ? launch_lds_real<double>(a, tile, s) : launch_lds_real<float>(a, tile, s);
}

int launch_sweep_hbm(const SweepArgs& a, int precision, unsigned long long* counter, void* slots,
                     int slot_bits, int num_slots, hipStream_t s) {
  if (a.num_pairs <= 0 || num_slots <= 0) return FP_OK;
  if (precision == FP_C128)
    hipLaunchKernelGGL((sweep_hbm_kernel<double, 512>), dim3(num_slots), dim3(512), 0, s, a, counter,
                       (unsigned char*)slots, slot_bits);
  else
    hipLaunchKernelGGL((sweep_hbm_kernel<float, 1024>), dim3(num_slots), dim3(1024), 0, s, a, counter,
                       (unsigned char*)slots, slot_bits);
  return check_launch("sweep_hbm");
}

int launch_plan_local_random(const PlanJob& j, hipStream_t s) {
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

int sweep_elem_bytes(int precision) { return precision == FP_C128 ? 16 : 8; }

}  // namespace fp
