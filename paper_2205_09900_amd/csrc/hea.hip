// Column sweep for the hardware-efficient ansatz (RY RZ layers, CZ ladders).
//
// W = U^dagger V of two L-layer circuits: the CZ ladders at the junction
// cancel, and the rotation layers that meet at the junction and across the
// wrap of the trace merge.  Around the loop W is m = 2L-2 slots, slot t being
// a layer of single-qubit gates A_t followed by CZ ladder t:
//   A_0 = R^V_0 (R^U_0)^dag,  A_t = R^V_t (1 <= t <= L-2),
//   A_{L-1} = (R^U_{L-1})^dag R^V_{L-1},  A_t = (R^U_{2L-2-t})^dag (L <= t <= 2L-3),
// with R = RZ(phi) RY(theta) per qubit.  CZ is diagonal, so qubit q keeps
// one value x_{q,t} across ladder t (one boundary bit per ladder), and
//   Tr = sum_x prod_q f_q(x_q) prod_{t,q} (-1)^{x_{q,t} x_{q+1,t}},
//   f_q(x) = prod_t A_{t+1,q}[x_{t+1}, x_t]  (slot indices mod m).
// Sweeping the qubits (Sec. II.A of the paper: contraction along the qubit
// direction; memory exponential in depth, Methods A):
//   B_0 = f_0,  B_q = f_q . WHT(B_{q-1}),  Tr = sum_x B_{n-1}(x),
// where WHT is the unnormalised Walsh-Hadamard transform over the m bits.
// f_q is evaluated from two tables over the low and high halves of the bits.
// L = 1 has no ladder left: Tr = prod_q Tr(A_{0,q}).
#include <hip/hip_runtime.h>
#include <math.h>

#include "internal.h"
#include "layout.h"
#include "sweep.h"
#include "hea_dev.h"

namespace fp {

template <typename Real, int NT, int PB, bool BF3>
__global__ void __launch_bounds__(NT* PB) hea_kernel(HeaArgs a, int m, int per_pair_bytes) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  __shared__ Real red[16];
  __shared__ double redd[16];
  const int slot = threadIdx.x / NT;
  const int lane = threadIdx.x % NT;
  const int64_t pi = (int64_t)blockIdx.x * PB + slot;
  if (pi >= a.num_pairs) return;
  const Real* angU = reinterpret_cast<const Real*>(a.gates + pi * a.gate_stride);
  const Real* angV = angU + (int64_t)a.L * a.n * 2;
  hea_pair<Real, NT, BF3>(angU, angV, a.n, a.L, m, smem_raw + (size_t)slot * per_pair_bytes, lane, red, redd,
                          a.trace + 2 * (a.trace_offset + pi));
}

int hea_bits(int L) { return L <= 1 ? 0 : 2 * L - 2; }


template <typename Real, int NT, int PB, bool BF3>
static int launch_hea_t(const HeaArgs& a, hipStream_t s) {
  const int m = hea_bits(a.L);
  const size_t per_pair = (hea_smem_bytes(m, NT, sizeof(Real)) + 15) & ~(size_t)15;
  const size_t smem = (size_t)PB * per_pair;
  if (smem > 160 * 1024) return set_error(FP_ETOOBIG, "HEA boundary of %d bits does not fit LDS", m);
  if (smem > 64 * 1024) {
    hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(hea_kernel<Real, NT, PB, BF3>),
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)smem);
    if (e != hipSuccess) (void)hipGetLastError();  // the limit may already allow it
  }
  const int64_t blocks = (a.num_pairs + PB - 1) / PB;
  hipLaunchKernelGGL((hea_kernel<Real, NT, PB, BF3>), dim3((unsigned)blocks), dim3(NT * PB), smem, s, a, m, (int)per_pair);
  return check_launch("hea_sweep");
}

template <typename Real, bool BF3>
static int launch_hea_real(const HeaArgs& a, int tile, hipStream_t s) {
  switch (tile) {
    case TILE_16x16: return launch_hea_t<Real, 16, 16, BF3>(a, s);
    case TILE_64x4: return launch_hea_t<Real, 64, 4, BF3>(a, s);
    case TILE_64x1: return launch_hea_t<Real, 64, 1, BF3>(a, s);
    case TILE_256x1: return launch_hea_t<Real, 256, 1, BF3>(a, s);
    case TILE_512x1: return launch_hea_t<Real, 512, 1, BF3>(a, s);
    case TILE_1024x1: return launch_hea_t<Real, 1024, 1, BF3>(a, s);
    default: return set_error(FP_EINVAL, "unknown HEA tile %d", tile);
  }
}

int launch_hea(const HeaArgs& a, int precision, int tile, hipStream_t s) {
  if (a.num_pairs <= 0) return FP_OK;
  if (precision == FP_C128) return launch_hea_real<double, false>(a, tile, s);
  return a.bf3 ? launch_hea_real<float, true>(a, tile, s) : launch_hea_real<float, false>(a, tile, s);
}

}  // namespace fp
