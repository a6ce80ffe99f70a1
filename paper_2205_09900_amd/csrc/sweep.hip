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
#include "plan_wave.h"
#include "sweep.h"
#include "sweep_dev.h"

namespace fp {

// One group of NT lanes per pair, PB pairs per workgroup, boundary in LDS
// (2^cap_bits complex per pair) next to the staging area of the group.
// Pairs whose plan needs more are left to the next launch; failed plans give NaN.
template <typename Real, int NT, int PB, bool BF3>
__global__ void __launch_bounds__(NT* PB) sweep_lds_kernel(SweepArgs a) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  __shared__ Real red[16];
  const int slot = threadIdx.x / NT;
  const int lane = threadIdx.x % NT;
  const int64_t pi = (int64_t)blockIdx.x * PB + slot;
  if (pi >= a.num_pairs) return;
  const int64_t pidx = a.order ? (int64_t)a.order[pi] : pi;
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
  run_program<Real, NT, BF3>(B, mats, ops_s, a.ops + pidx * a.ops_stride, hdr->num_ops,
                             a.wgates + pidx * a.wg_stride, a.factors + pidx * a.f_stride, pg, a.G, hdr->log2_factor,
                             lane, red, &re, &im);
  if (lane == 0) {
    out[0] = re;
    out[1] = im;
  }
}

// Large boundaries: one workgroup per pair at a time, boundary in the HBM
// slot of the workgroup (2^slot_bits entries), pairs taken from a shared
// counter.  The interpreter runs the same programs with the same arithmetic
// as run_program, organised for global-memory latency:
//   * every lane keeps U groups (GATE), outputs (TRACE) or entries (BELL) in
//     flight, all loads of a round issued before its stores, so a TRACE needs
//     two barriers per NT * U outputs;
//   * op fields are read once per wavefront (scalar), so branching is uniform;
//   * the realigned matrices come precomputed in program order when the
//     caller has them (local random), else they are staged from the factors.
// 512 lanes with 8 (float) or 3 (double) groups each: the most loads in
// flight without spilling registers.
constexpr int HBM_NT = 512;
template <typename Real>
constexpr int hbm_u() {
  return sizeof(Real) == 8 ? 3 : 8;
}

template <typename Real, int NT, int U, bool BF3>
__device__ __forceinline__ void run_program_hbm(Cplx<Real>* B, Cplx<Real>* mats_s, uint2* ops_s,
                                                const Op* __restrict__ ops, int num_ops, int num_gate_ops,
                                                const Real* __restrict__ wmat, const int2* __restrict__ wgates,
                                                const int32_t* __restrict__ factors, const Real* pair_gates, int G,
                                                int log2_factor, int lane, Real* red, double* tr_re, double* tr_im) {
  constexpr int K = 64;  // ops staged per chunk: one per lane of the first wavefront
  int b = 0;
  int64_t expo = 0;  // true boundary = stored boundary * 2^expo
  int pend = 0;      // exponent to remove at the next GATE
  bool prev_track = false;
  int gate_base = 0;  // GATE ops before the chunk (first wavefront only)
  Real lmax = 0;
  if (lane == 0) {
    B[0].x = (Real)1;
    B[0].y = (Real)0;
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
#pragma unroll
        for (int k = 0; k < 16; ++k) {
          const Cplx<Real> r = mats_s[16 * i + k];
          Rr[k] = pend ? ldexp(r.x, -pend) : r.x;
          Ri[k] = pend ? ldexp(r.y, -pend) : r.y;
        }
        expo += pend;
        pend = 0;
        const int lo = p < q ? p : q, hi = p < q ? q : p;
        gate_groups<Real, U, BF3>(B, Rr, Ri, lo, hi, 1 << p, 1 << q, 1 << (b - 2), lane, NT, track, lmax);
      } else if (type == OP_BELL) {
        const int s = 1 << b;
        for (int k0 = lane; k0 < s; k0 += NT * U) {
          Cplx<Real> v[U];
#pragma unroll
          for (int u = 0; u < U; ++u)
            if (k0 + u * NT < s) v[u] = B[k0 + u * NT];
          Cplx<Real> z;
          z.x = (Real)0;
          z.y = (Real)0;
#pragma unroll
          for (int u = 0; u < U; ++u) {
            const int k = k0 + u * NT;
            if (k < s) {
              B[k + s] = z;
              B[k + 2 * s] = z;
              B[k + 3 * s] = v[u];
            }
          }
        }
        b += 2;
      } else if (type == OP_TRACE) {
        // p < q; in place, in chunks of NT * U outputs: every input of a
        // chunk lies at or above its output, so the chunk reads everything
        // before anyone writes, and later chunks read above what it wrote
        const int nout = 1 << (b - 2);
        const int step = (1 << p) + (1 << q);
        for (int j0 = 0; j0 < nout; j0 += NT * U) {
          Cplx<Real> a0[U], a1[U];
#pragma unroll
          for (int u = 0; u < U; ++u) {
            const int j = j0 + lane + u * NT;
            if (j < nout) {
              const int i0 = insert_zero(insert_zero(j, p), q);
              a0[u] = B[i0];
              a1[u] = B[i0 + step];
            }
          }
          __syncthreads();
#pragma unroll
          for (int u = 0; u < U; ++u) {
            const int j = j0 + lane + u * NT;
            if (j < nout) {
              Cplx<Real> acc;
              acc.x = a0[u].x + a1[u].x;
              acc.y = a0[u].y + a1[u].y;
              if (track) lmax = fmax(lmax, fmax(fabs(acc.x), fabs(acc.y)));
              B[j] = acc;
            }
          }
          if (j0 + NT * U < nout) __syncthreads();  // the last chunk ends at the op's barrier
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
  const Cplx<Real> v = B[0];
  *tr_re = ldexp((double)v.x, (int)(expo + log2_factor));
  *tr_im = ldexp((double)v.y, (int)(expo + log2_factor));
}

template <typename Real, int NT, bool BF3>
__global__ void __launch_bounds__(NT) sweep_hbm_kernel(SweepArgs a, unsigned long long* counter,
                                                       unsigned char* slots, int slot_bits) {
  __shared__ Real red[16];
  __shared__ long long next;
  __shared__ __align__(16) Cplx<Real> mats[16 * 64];
  __shared__ uint2 ops_s[64];
  const int lane = threadIdx.x;
  Cplx<Real>* B = reinterpret_cast<Cplx<Real>*>(slots) + ((int64_t)blockIdx.x << slot_bits);
  for (;;) {
    if (lane == 0) next = (long long)atomicAdd(counter, 1ull);
    __syncthreads();
    const long long pi = next;
    __syncthreads();
    if (pi >= a.num_pairs) break;
    const int64_t pidx = a.order ? (int64_t)a.order[pi] : (int64_t)pi;
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
    const Real* wm = a.wmat ? reinterpret_cast<const Real*>(a.wmat + pidx * a.wmat_stride) : nullptr;
    double re, im;
    run_program_hbm<Real, NT, hbm_u<Real>(), BF3>(B, mats, ops_s, a.ops + pidx * a.ops_stride,
                                          hdr->num_ops, hdr->num_gate_ops, wm, a.wgates + pidx * a.wg_stride,
                                          a.factors + pidx * a.f_stride, pg, a.G, hdr->log2_factor, lane, red, &re,
                                          &im);
    if (lane == 0) {
      out[0] = re;
      out[1] = im;
    }
    __syncthreads();
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
  int16_t* bw = reinterpret_cast<int16_t*>(smem_raw);
  int16_t* scratch = bw + ((2 * G + 7) & ~7);
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
  return 2 * (size_t)((2 * G + 7) & ~7) + 2 * (size_t)plan_wave_scratch_elems(G);
}

// ---- launchers --------------------------------------------------------------

template <typename Real, int NT, int PB, bool BF3>
static int launch_lds_t(const SweepArgs& a, hipStream_t s) {
  const size_t smem = (size_t)PB * ((((size_t)1 << a.cap_bits) * sizeof(Cplx<Real>)) + stage_bytes<Real, NT>());
  const int64_t blocks = (a.num_pairs + PB - 1) / PB;
  if (smem > 64 * 1024) {
    hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(sweep_lds_kernel<Real, NT, PB, BF3>),
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)smem);
    if (e != hipSuccess) (void)hipGetLastError();  // the limit may already allow it
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

int launch_sweep_hbm(const SweepArgs& a, int precision, unsigned long long* counter, void* slots,
                     int slot_bits, int num_slots, hipStream_t s) {
  if (a.num_pairs <= 0 || num_slots <= 0) return FP_OK;
  if (precision == FP_C128)
    hipLaunchKernelGGL((sweep_hbm_kernel<double, HBM_NT, false>), dim3(num_slots), dim3(HBM_NT), 0, s, a,
                       counter, (unsigned char*)slots, slot_bits);
  else if (a.bf3)
    hipLaunchKernelGGL((sweep_hbm_kernel<float, HBM_NT, true>), dim3(num_slots), dim3(HBM_NT), 0, s, a,
                       counter, (unsigned char*)slots, slot_bits);
  else
    hipLaunchKernelGGL((sweep_hbm_kernel<float, HBM_NT, false>), dim3(num_slots), dim3(HBM_NT), 0, s, a,
                       counter, (unsigned char*)slots, slot_bits);
  return check_launch("sweep_hbm");
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

int launch_gate_matrices(const PlanJob& j, int precision, hipStream_t s) {
  if (j.num_pairs <= 0) return FP_OK;
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
