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

// Merged gate (product of its factors, float64) realigned for the column
// transfer: R[j'][j], j = x_in + 2 x_out (qubit c legs), j' = y_in + 2 y_out
// (qubit c+1 legs), R[j'][j] = M[2 x_out + y_out][2 x_in + y_in].
template <typename Real>
__device__ __forceinline__ void load_realigned(const Real* __restrict__ pair_gates, int G,
                                               const int32_t* __restrict__ factors, int2 wg,
                                               Real (&Rr)[16], Real (&Ri)[16]) {
  double mr[16], mi[16];
  for (int f = 0; f < wg.y; ++f) {
    const FactorRef fr = decode_factor(factors[wg.x + f], G);
    const Real* src = pair_gates + ((int64_t)fr.circuit * G + fr.gate) * 32;
    double fr_[16], fi_[16];
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
      for (int b = 0; b < 4; ++b) {
        if (fr.dagger) {
          fr_[a * 4 + b] = (double)src[(b * 4 + a) * 2];
          fi_[a * 4 + b] = -(double)src[(b * 4 + a) * 2 + 1];
        } else {
          fr_[a * 4 + b] = (double)src[(a * 4 + b) * 2];
          fi_[a * 4 + b] = (double)src[(a * 4 + b) * 2 + 1];
        }
      }
    if (f == 0) {
#pragma unroll
      for (int i = 0; i < 16; ++i) {
        mr[i] = fr_[i];
        mi[i] = fi_[i];
      }
    } else {
      double nr[16], ni[16];
#pragma unroll
      for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int b = 0; b < 4; ++b) {
          double sr = 0.0, si = 0.0;
#pragma unroll
          for (int k = 0; k < 4; ++k) {
            sr += fr_[a * 4 + k] * mr[k * 4 + b] - fi_[a * 4 + k] * mi[k * 4 + b];
            si += fr_[a * 4 + k] * mi[k * 4 + b] + fi_[a * 4 + k] * mr[k * 4 + b];
          }
          nr[a * 4 + b] = sr;
          ni[a * 4 + b] = si;
        }
#pragma unroll
      for (int i = 0; i < 16; ++i) {
        mr[i] = nr[i];
        mi[i] = ni[i];
      }
    }
  }
#pragma unroll
  for (int jp = 0; jp < 4; ++jp)
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int xin = j & 1, xout = j >> 1, yin = jp & 1, yout = jp >> 1;
      const int idx = (2 * xout + yout) * 4 + (2 * xin + yin);
      Rr[jp * 4 + j] = (Real)mr[idx];
      Ri[jp * 4 + j] = (Real)mi[idx];
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

// Runs one pair's program on boundary B (LDS or global).  Returns the trace
// (float64 parts) on every lane.
template <typename Real, int NT>
__device__ __forceinline__ void run_program(Cplx<Real>* B, const Op* __restrict__ ops, int num_ops,
                                            const int2* __restrict__ wgates,
                                            const int32_t* __restrict__ factors, const Real* pair_gates,
                                            int G, int log2_factor, int lane, Real* red, double* tr_re,
                                            double* tr_im) {
  int b = 0;
  int64_t expo = 0;
  if (lane == 0) {
    B[0].x = (Real)1;
    B[0].y = (Real)0;
  }
  group_sync<NT>();
  for (int t = 0; t < num_ops; ++t) {
    const Op op = ops[t];
    if (op.type == OP_GATE) {
      Real Rr[16], Ri[16];
      load_realigned<Real>(pair_gates, G, factors, wgates[op.arg], Rr, Ri);
      const int p = op.p, q = op.q;
      const int lo = p < q ? p : q, hi = p < q ? q : p;
      const int ip = 1 << p, iq = 1 << q;
      const int ng = 1 << (b - 2);
      for (int g = lane; g < ng; g += NT) {
        const int i = insert_zero(insert_zero(g, lo), hi);
        Cplx<Real> v[4];
        v[0] = B[i];
        v[1] = B[i + ip];
        v[2] = B[i + iq];
        v[3] = B[i + ip + iq];
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
        }
        B[i] = w[0];
        B[i + ip] = w[1];
        B[i + iq] = w[2];
        B[i + ip + iq] = w[3];
      }
    } else if (op.type == OP_BELL) {
      const int s = 1 << b;
      for (int i = lane; i < s; i += NT) {
        const Cplx<Real> v = B[i];
        Cplx<Real> z;
        z.x = (Real)0;
        z.y = (Real)0;
        B[i + s] = z;
        B[i + 2 * s] = z;
        B[i + 3 * s] = v;
      }
      b += 2;
    } else if (op.type == OP_TRACE) {
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
        }
        group_sync<NT>();
        if (j < nout) B[j] = acc;
        group_sync<NT>();
      }
      b -= 2;
    } else {  // OP_COLEND: exact power-of-two rescale
      const int s = 1 << b;
      Real m = 0;
      for (int i = lane; i < s; i += NT) m = fmax(m, fmax(fabs(B[i].x), fabs(B[i].y)));
      m = group_max<Real, NT>(m, red);
      if (m > (Real)0 && isfinite(m)) {
        int e;
        frexp(m, &e);
        for (int i = lane; i < s; i += NT) {
          B[i].x = ldexp(B[i].x, -e);
          B[i].y = ldexp(B[i].y, -e);
        }
        expo += e;
      }
    }
    group_sync<NT>();
  }
  const Cplx<Real> v = B[0];
  *tr_re = ldexp((double)v.x, (int)(expo + log2_factor));
  *tr_im = ldexp((double)v.y, (int)(expo + log2_factor));
}

// One group of NT lanes per pair, PB pairs per workgroup, boundary in LDS
// (2^cap_bits complex per pair).  Pairs whose plan needs more are left to
// the HBM kernel; failed plans give NaN.
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
  Cplx<Real>* B = reinterpret_cast<Cplx<Real>*>(smem_raw) + ((int64_t)slot << a.cap_bits);
  const Real* pg = reinterpret_cast<const Real*>(a.gates + pidx * a.gate_stride);
  double re, im;
  run_program<Real, NT>(B, a.ops + pidx * a.ops_stride, hdr->num_ops, a.wgates + pidx * a.wg_stride,
                        a.factors + pidx * a.f_stride, pg, a.G, hdr->log2_factor, lane, red, &re, &im);
  if (lane == 0) {
    out[0] = re;
    out[1] = im;
  }
}

// Large boundaries: one workgroup per pair at a time, boundary in the HBM
// slot of the workgroup, pairs taken from a shared counter.
template <typename Real, int NT>
__global__ void __launch_bounds__(NT) sweep_hbm_kernel(SweepArgs a, unsigned long long* counter,
                                                       unsigned char* slots, int slot_bits) {
  __shared__ Real red[16];
  __shared__ long long next;
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
    run_program<Real, NT>(B, a.ops + pidx * a.ops_stride, hdr->num_ops, a.wgates + pidx * a.wg_stride,
                          a.factors + pidx * a.f_stride, pg, a.G, hdr->log2_factor, lane, red, &re, &im);
    if (lane == 0) {
      out[0] = re;
      out[1] = im;
    }
    __syncthreads();
  }
}

// Device planner for local random pairs: one thread per pair.
__global__ void __launch_bounds__(64) plan_local_random_kernel(PlanJob j) {
  const int64_t pi = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (pi >= j.num_pairs) return;
  const unsigned char* pair = j.gates + pi * j.gate_stride;
  const int32_t* bu = reinterpret_cast<const int32_t*>(pair + j.bonds_off);
  const int32_t* bv = bu + j.G;
  PlanHeader h = plan_haar_pair(j.n, j.G, bu, bv, j.scratch + pi * j.scratch_stride,
                                j.ops + pi * j.ops_stride, j.wgates + pi * j.wg_stride,
                                j.factors + pi * j.f_stride);
  j.hdr[pi] = h;
  if (h.status == 0) {
    atomicMax(j.max_peak, h.peak_bits);
    if (h.peak_bits > j.cap_bits) atomicAdd(j.num_large, 1);
    const int cls = h.peak_bits <= j.small_bits ? 0 : h.peak_bits <= j.cap_bits ? 1 : 2;
    atomicAdd(&j.class_macs[cls], h.macs);
  } else {
    atomicAdd(j.num_failed, 1);
  }
}

// ---- launchers --------------------------------------------------------------

template <typename Real, int NT, int PB>
static int launch_lds_t(const SweepArgs& a, hipStream_t s) {
  const size_t smem = (size_t)PB * ((size_t)1 << a.cap_bits) * sizeof(Cplx<Real>);
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
    case TILE_1024x1: return launch_lds_t<Real, 1024, 1>(a, s);
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
    hipLaunchKernelGGL((sweep_hbm_kernel<double, 1024>), dim3(num_slots), dim3(1024), 0, s, a, counter,
                       (unsigned char*)slots, slot_bits);
  else
    hipLaunchKernelGGL((sweep_hbm_kernel<float, 1024>), dim3(num_slots), dim3(1024), 0, s, a, counter,
                       (unsigned char*)slots, slot_bits);
  return check_launch("sweep_hbm");
}

int launch_plan_local_random(const PlanJob& j, hipStream_t s) {
  if (j.num_pairs <= 0) return FP_OK;
  const int64_t blocks = (j.num_pairs + 63) / 64;
  hipLaunchKernelGGL(plan_local_random_kernel, dim3((unsigned)blocks), dim3(64), 0, s, j);
  return check_launch("plan_local_random");
}

int sweep_elem_bytes(int precision) { return precision == FP_C128 ? 16 : 8; }

}  // namespace fp
