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

template <typename Real, int NT, int PB, bool BF3>
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
      if (g.kind == GROUP_HEA) {
        const Real* angU = reinterpret_cast<const Real*>(pg);
        const Real* angV = angU + (int64_t)g.depth * g.n * 2;
        hea_pair<Real, NT, BF3>(angU, angV, g.n, g.depth, g.m, my, lane, red, redd, out);
      } else {
        const PlanHeader* hdr = g.hdr + pair * g.hdr_stride;
        Cplx<Real>* B = reinterpret_cast<Cplx<Real>*>(my);
        Cplx<Real>* mats = reinterpret_cast<Cplx<Real>*>(my + ((size_t)sizeof(Cplx<Real>) << g.m));
        Op* ops_s = reinterpret_cast<Op*>(mats + 16 * chunk_ops<NT>());
        double re, im;
        run_program<Real, NT, BF3>(B, mats, ops_s, g.ops + pair * g.ops_stride, hdr->num_ops, g.wg + pair * g.wg_stride,
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

size_t program_slot_bytes(int bits, int nt, int real_bytes) {
  const size_t cb = 2 * (size_t)real_bytes;
  const int k = nt <= 16 ? 16 : nt <= 64 ? 32 : 64;
  return ((cb << bits) + (size_t)k * (16 * cb + sizeof(Op)) + 15) & ~(size_t)15;
}

template <typename Real, int NT, int PB, bool BF3>
static int launch_t(const GroupDesc* groups, const Task* tasks, int ntasks, unsigned int* counter, double* trace,
                    int slot_bytes, int num_cus, hipStream_t s) {
  const size_t smem = (size_t)PB * slot_bytes;
  if (smem > 160 * 1024) return set_error(FP_ETOOBIG, "persistent sweep needs %zu bytes of LDS", smem);
  if (smem > 64 * 1024) {
    hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(persistent_kernel<Real, NT, PB, BF3>),
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)smem);
    if (e != hipSuccess) (void)hipGetLastError();
  }
  int per_cu = 0;
  hipError_t e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, persistent_kernel<Real, NT, PB, BF3>, NT * PB, smem);
  if (e != hipSuccess || per_cu < 1) {
    (void)hipGetLastError();
    per_cu = 1;
  }
  int64_t blocks = (int64_t)per_cu * num_cus;
  const int64_t need = ((int64_t)ntasks + PB - 1) / PB;
  if (blocks > need) blocks = need;
  if (blocks < 1) blocks = 1;
  hipLaunchKernelGGL((persistent_kernel<Real, NT, PB, BF3>), dim3((unsigned)blocks), dim3(NT * PB), smem, s, groups, tasks,
                     ntasks, counter, trace, slot_bytes);
  return check_launch("persistent_sweep");
}

int launch_persistent(int precision, int cls, const GroupDesc* groups, const Task* tasks, int ntasks,
                      unsigned int* counter, double* trace, int slot_bytes, int num_cus, hipStream_t s) {
  if (ntasks <= 0) return FP_OK;
  if (precision == FP_C128) {
    if (cls == PCLASS_SMALL)
      return launch_t<double, 64, 4, false>(groups, tasks, ntasks, counter, trace, slot_bytes, num_cus, s);
    return launch_t<double, 512, 1, false>(groups, tasks, ntasks, counter, trace, slot_bytes, num_cus, s);
  }
  if (precision == FP_BF16X3) {
    if (cls == PCLASS_SMALL)
      return launch_t<float, 64, 4, true>(groups, tasks, ntasks, counter, trace, slot_bytes, num_cus, s);
    return launch_t<float, 1024, 1, true>(groups, tasks, ntasks, counter, trace, slot_bytes, num_cus, s);
  }
  if (cls == PCLASS_SMALL)
    return launch_t<float, 64, 4, false>(groups, tasks, ntasks, counter, trace, slot_bytes, num_cus, s);
  return launch_t<float, 1024, 1, false>(groups, tasks, ntasks, counter, trace, slot_bytes, num_cus, s);
}

}  // namespace fp
