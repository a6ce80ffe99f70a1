// Persistent sweep over groups of pairs with different ensembles (uneven
// work: different depths and qubit counts in one launch).
//
// The host cuts every group into tasks of consecutive pairs, orders the
// tasks by planned cost, largest first, and launches a grid sized to the
// device.  Each lane group (NT lanes) takes the next task from a counter and
// contracts its pairs with the HEA transform or the register-program
// interpreter; the loop ends when the counter passes the last task, so every
// group of lanes exits.
#include <hip/hip_runtime.h>

#include "hea_dev.h"
#include "internal.h"
#include "sched.h"
#include "sweep_dev.h"

namespace fp {

// KIND (GROUP_HEA or GROUP_PROGRAM) is the kind of every group of the launch,
// so each instance holds one contraction path.
template <typename Real, int NT, int PB, bool BF3, int KIND>
__global__ void __launch_bounds__(NT* PB) persistent_kernel(const GroupDesc* __restrict__ groups,
                                                            const Task* __restrict__ tasks, int ntasks,
                                                            unsigned int* counter, double* trace, int slot_bytes) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  __shared__ Real red[16];
  __shared__ double redd[16];
  __shared__ int grab[PB];
  const int slot = threadIdx.x / NT;
  const int lane = threadIdx.x % NT;
  unsigned char* my = smem_raw + (size_t)slot * slot_bytes;
  for (;;) {
    int t;
    if constexpr (NT <= 64) {
      int v = 0;
      if (lane == 0) v = (int)atomicAdd(counter, 1u);
      t = __shfl(v, 0, NT);
    } else {
      if (lane == 0) grab[slot] = (int)atomicAdd(counter, 1u);
      __syncthreads();
      t = grab[slot];
      __syncthreads();
    }
    if (t >= ntasks) break;
    const Task tk = tasks[t];
    const GroupDesc& g = groups[tk.group];
    for (int i = 0; i < tk.count; ++i) {
      const int64_t pair = tk.first + i;
      const unsigned char* pg = g.gates + (g.gate_first + pair) * g.stride;
      double* out = trace + 2 * (g.trace_offset + pair);
      if constexpr (KIND == GROUP_HEA) {
        const Real* angU = reinterpret_cast<const Real*>(pg);
        const Real* angV = angU + (int64_t)g.depth * g.n * 2;
        hea_pair<Real, NT, BF3>(angU, angV, g.n, g.depth, g.m, my, lane, red, redd, out);
      } else {
        const PlanHeader* hdr = g.hdr + pair * g.hdr_stride;
        Cplx<Real>* B = reinterpret_cast<Cplx<Real>*>(my);
        Cplx<Real>* mats = reinterpret_cast<Cplx<Real>*>(my + ((size_t)sizeof(Cplx<Real>) << g.m));
        Op* ops_s = reinterpret_cast<Op*>(mats + 16 * chunk_ops<NT>());
        double re, im;
        // 1024 lanes: the task loop's state leaves no registers for the
        // matrix-core blocks
        run_program<Real, NT, BF3, (NT < 1024)>(B, mats, ops_s, g.ops + pair * g.ops_stride, hdr->num_ops, g.wg + pair * g.wg_stride,
                              g.fac + pair * g.f_stride, reinterpret_cast<const Real*>(pg), g.G, hdr->log2_factor,
                              lane, red, &re, &im);
        if (lane == 0) {
          out[0] = re;
          out[1] = im;
        }
      }
      if constexpr (NT <= 64) {
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
      } else {
        __syncthreads();
      }
    }
  }
}

size_t program_slot_bytes(int bits, int nt, int real_bytes, bool bf3) {
  const size_t cb = 2 * (size_t)real_bytes;
  const int k = nt <= 16 ? 16 : nt <= 64 ? 32 : 64;
  const size_t blk = bf3 && nt >= 64 ? MFMA_BLOCK_BYTES : 0;  // as stage_bytes
  return ((cb << bits) + (size_t)k * (16 * cb + sizeof(Op)) + blk + 15) & ~(size_t)15;
}

template <typename Real, int NT, int PB, bool BF3, int KIND>
static int launch_t(const GroupDesc* groups, const Task* tasks, int ntasks, unsigned int* counter, double* trace,
                    int slot_bytes, int num_cus, hipStream_t s) {
  const size_t smem = (size_t)PB * slot_bytes;
  if (smem > 160 * 1024) return set_error(FP_ETOOBIG, "persistent sweep needs %zu bytes of LDS", smem);
  if (smem > 64 * 1024) {
    hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(persistent_kernel<Real, NT, PB, BF3, KIND>),
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)smem);
    if (e != hipSuccess) (void)hipGetLastError();
  }
  int per_cu = 0;
  hipError_t e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, persistent_kernel<Real, NT, PB, BF3, KIND>, NT * PB, smem);
  if (e != hipSuccess || per_cu < 1) {
    (void)hipGetLastError();
    per_cu = 1;
  }
  // four times the resident count the runtime reports (workgroups beyond the
  // resident ones start as others finish and leave once the counter has run
  // out), so that an underestimate does not leave compute units idle
  int64_t blocks = 4 * (int64_t)per_cu * num_cus;
  const int64_t need = ((int64_t)ntasks + PB - 1) / PB;
  if (blocks > need) blocks = need;
  if (blocks < 1) blocks = 1;
  hipLaunchKernelGGL((persistent_kernel<Real, NT, PB, BF3, KIND>), dim3((unsigned)blocks), dim3(NT * PB), smem, s, groups, tasks,
                     ntasks, counter, trace, slot_bytes);
  return check_launch("persistent_sweep");
}

int pclass_lanes(int cls, int precision) {
  switch (cls) {
    case PCLASS_TINY: return 16;
    case PCLASS_SMALL: return 64;
    case PCLASS_MID: return 256;
    default: return precision == FP_C128 ? 512 : 1024;
  }
}

int pclass_pairs(int cls) { return cls == PCLASS_TINY ? 16 : cls == PCLASS_SMALL ? 4 : 1; }

size_t pclass_slot_bytes(int cls, int bits, bool hea, int precision) {
  const int nt = pclass_lanes(cls, precision);
  const size_t rb = precision == FP_C128 ? 8 : 4;
  return hea ? ((hea_smem_bytes(bits, nt, rb) + 15) & ~(size_t)15)
             : program_slot_bytes(bits, nt, (int)rb, precision == FP_BF16X3);
}

bool pclass_fits(int cls, int bits, bool hea, int precision) {
  return (size_t)pclass_pairs(cls) * pclass_slot_bytes(cls, bits, hea, precision) <= 160 * 1024;
}

int pclass_default(int bits, int precision) {
  const int small_bits = precision == FP_C128 ? 9 : 10;
  if (bits <= 6) return PCLASS_TINY;
  if (bits <= small_bits) return PCLASS_SMALL;
  if (bits <= 12) return PCLASS_MID;
  return PCLASS_LARGE;
}

template <typename Real, bool BF3, int KIND>
static int launch_cls(int cls, const GroupDesc* groups, const Task* tasks, int ntasks, unsigned int* counter,
                      double* trace, int slot_bytes, int num_cus, hipStream_t s) {
  switch (cls) {
    case PCLASS_TINY:
      return launch_t<Real, 16, 16, BF3, KIND>(groups, tasks, ntasks, counter, trace, slot_bytes, num_cus, s);
    case PCLASS_SMALL:
      return launch_t<Real, 64, 4, BF3, KIND>(groups, tasks, ntasks, counter, trace, slot_bytes, num_cus, s);
    case PCLASS_MID:
      return launch_t<Real, 256, 1, BF3, KIND>(groups, tasks, ntasks, counter, trace, slot_bytes, num_cus, s);
    default:
      if constexpr (sizeof(Real) == 8)
        return launch_t<Real, 512, 1, BF3, KIND>(groups, tasks, ntasks, counter, trace, slot_bytes, num_cus, s);
      else
        return launch_t<Real, 1024, 1, BF3, KIND>(groups, tasks, ntasks, counter, trace, slot_bytes, num_cus, s);
  }
}

template <typename Real, bool BF3>
static int launch_kind(int kind, int cls, const GroupDesc* groups, const Task* tasks, int ntasks,
                       unsigned int* counter, double* trace, int slot_bytes, int num_cus, hipStream_t s) {
  if (kind == GROUP_HEA)
    return launch_cls<Real, BF3, GROUP_HEA>(cls, groups, tasks, ntasks, counter, trace, slot_bytes, num_cus, s);
  return launch_cls<Real, BF3, GROUP_PROGRAM>(cls, groups, tasks, ntasks, counter, trace, slot_bytes, num_cus, s);
}

int launch_persistent(int precision, int kind, int cls, const GroupDesc* groups, const Task* tasks, int ntasks,
                      unsigned int* counter, double* trace, int slot_bytes, int num_cus, hipStream_t s) {
  if (ntasks <= 0) return FP_OK;
  if (precision == FP_C128)
    return launch_kind<double, false>(kind, cls, groups, tasks, ntasks, counter, trace, slot_bytes, num_cus, s);
  if (precision == FP_BF16X3)
    return launch_kind<float, true>(kind, cls, groups, tasks, ntasks, counter, trace, slot_bytes, num_cus, s);
  return launch_kind<float, false>(kind, cls, groups, tasks, ntasks, counter, trace, slot_bytes, num_cus, s);
}

}  // namespace fp
