// Column sweep for the paper's hardware-efficient ansatz (Fig. 2c; Sec. II.C):
// a wall of RY(pi/4), then per layer a random Pauli rotation on every qubit
// and two walls of CNOT (control q, target q+1; even bonds, then odd bonds),
// or of CZ.
//
// In W = U^dagger V the fixed RY(pi/4) walls cancel around the trace, the
// entangling walls of the two circuits cancel at the junction (every wall
// is its own inverse), and the rotation layers that meet at the junction and
// across the wrap merge.  Around the loop W is m = 2L-2 slots, slot t being a
// rotation layer A_t followed by both entangling walls; slots 0 .. L-2 come
// from V (even wall first), slots L-1 .. 2L-3 from U^dagger (odd wall first):
//   A_0 = R^V_0 (R^U_0)^dag,  A_t = R^V_t (1 <= t <= L-2),
//   A_{L-1} = (R^U_{L-1})^dag R^V_{L-1},  A_t = (R^U_{2L-2-t})^dag (t >= L).
// A CNOT leaves its control's value unchanged, so that value is one boundary
// label per slot and bond (as the CZ ladders of the other ansatz): the
// boundary after qubit q is B_q(b), b = (b_0 .. b_{m-1}) the values of qubit
// q at its controls.  Qubit q's wire around the loop meets, in slot t, A_t,
// then its control event (bond q) and its target event (bond q-1) in the
// order of the walls.  The column transfer B_{q-1}(a) -> B_q(b) follows the
// wire: a register R(labels, w) with the wire value w as bit m; a control
// event copies w into label b_t, a target event flips w by a_t and drops
// a_t.  Starting the walk inside a control event (where the wire value is the
// new label, so no separate start value is kept) and ending there closes the
// loop by selecting w = b_{t0}.  Per slot, on groups of four entries
// (label t, wire):
//   rotation:  (R[l,0], R[l,1]) <- A_t (R[l,0], R[l,1]) for l = 0, 1
//   control then target:  R'[b,w'] = R[b^w', b]         (a permutation)
//   target then control:  R'[b,w'] = delta(b,w') sum_a R[a, w'^a]
//   CZ (either order):    R'[b,w]  = delta(b,w) sum_a (-1)^(a w) R[a, w]
// B_{-1} is the unit vector at a = 0 (qubit 0 has no target events); the last
// qubit's control events are emitted and summed at the end, which is the same
// as having none.  Tr = sum_b B_{n-1}(b).  One layer (m = 0) leaves
// Tr = prod_q Tr(A_{0,q}).  The register (2^(m+1) entries) lives in LDS; each
// column is rescaled by a power of two with the exponent kept in float64.
#include <hip/hip_runtime.h>
#include <math.h>

#include "hea_dev.h"
#include "internal.h"
#include "layout.h"
#include "sweep.h"

namespace fp {

// exp(-i theta P / 2) = cos(theta/2) I - i sin(theta/2) P as [out][in]; P = X, Y, Z for axis 0, 1, 2.
__device__ __forceinline__ void pauli_rot(double theta, int axis, D2 r[2][2]) {
  double s, c;
  sincos(0.5 * theta, &s, &c);
  if (axis == 0) {
    r[0][0] = D2{c, 0.0};
    r[0][1] = D2{0.0, -s};
    r[1][0] = D2{0.0, -s};
    r[1][1] = D2{c, 0.0};
  } else if (axis == 1) {
    r[0][0] = D2{c, 0.0};
    r[0][1] = D2{-s, 0.0};
    r[1][0] = D2{s, 0.0};
    r[1][1] = D2{c, 0.0};
  } else {
    r[0][0] = D2{c, -s};
    r[0][1] = D2{0.0, 0.0};
    r[1][0] = D2{0.0, 0.0};
    r[1][1] = D2{c, s};
  }
}

// Rotation of (circuit parameters p, layer l, qubit q): p holds (theta, axis) per (l, q).
template <typename Real>
__device__ __forceinline__ void pauli_rot_of(const Real* p, int n, int l, int q, D2 r[2][2]) {
  const Real* e = p + ((int64_t)l * n + q) * 2;
  int axis = (int)e[1];
  axis = axis < 0 ? 0 : axis > 2 ? 2 : axis;
  pauli_rot((double)e[0], axis, r);
}

// Slot matrix A_t of qubit q (see the header).
template <typename Real>
__device__ void pauli_slot_matrix(const Real* pU, const Real* pV, int n, int L, int t, int q, D2 out[2][2]) {
  D2 ru[2][2], rv[2][2], rud[2][2];
  if (t == 0) {
    pauli_rot_of(pV, n, 0, q, rv);
    pauli_rot_of(pU, n, 0, q, ru);
    dag(ru, rud);
    mat2(rv, rud, out);
  } else if (t < L - 1) {
    pauli_rot_of(pV, n, t, q, out);
  } else if (t == L - 1) {
    pauli_rot_of(pV, n, L - 1, q, rv);
    pauli_rot_of(pU, n, L - 1, q, ru);
    dag(ru, rud);
    mat2(rud, rv, out);
  } else {
    pauli_rot_of(pU, n, 2 * L - 2 - t, q, ru);
    dag(ru, out);
  }
}

enum { EV_CT = 0, EV_TC = 1, EV_CZ = 2 };

// One slot on the register (2^(m+1) entries, wire = bit m): the rotation
// (unless rot is false), then the event on label bit t.  scale: the column's
// pending power of two, taken out as the entries are read (exact).
template <typename Real, int NT, bool BF3>
__device__ __forceinline__ void slot_pass(HC<Real>* R, int m, int t, int ev, bool rot, const D2* A, int lane) {
  Real ar[4], ai[4];
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    ar[k] = (Real)A[k].x;
    ai[k] = (Real)A[k].y;
  }
  const int half = 1 << m, bt = 1 << t;
  const int ng = half >> 1;
  for (int g = lane; g < ng; g += NT) {
    const int base = ((g >> t) << (t + 1)) | (g & (bt - 1));
    const int i00 = base, i10 = base | bt, i01 = base | half, i11 = base | bt | half;  // [label, wire]
    HC<Real> v00 = R[i00], v10 = R[i10], v01 = R[i01], v11 = R[i11];
    if (rot) {
      HC<Real> w00, w01, w10, w11;
      w00.x = w00.y = w01.x = w01.y = w10.x = w10.y = w11.x = w11.y = (Real)0;
      cmac<Real, BF3>(ar[0], ai[0], v00.x, v00.y, w00.x, w00.y);
      cmac<Real, BF3>(ar[1], ai[1], v01.x, v01.y, w00.x, w00.y);
      cmac<Real, BF3>(ar[2], ai[2], v00.x, v00.y, w01.x, w01.y);
      cmac<Real, BF3>(ar[3], ai[3], v01.x, v01.y, w01.x, w01.y);
      cmac<Real, BF3>(ar[0], ai[0], v10.x, v10.y, w10.x, w10.y);
      cmac<Real, BF3>(ar[1], ai[1], v11.x, v11.y, w10.x, w10.y);
      cmac<Real, BF3>(ar[2], ai[2], v10.x, v10.y, w11.x, w11.y);
      cmac<Real, BF3>(ar[3], ai[3], v11.x, v11.y, w11.x, w11.y);
      v00 = w00;
      v01 = w01;
      v10 = w10;
      v11 = w11;
    }
    HC<Real> z;
    z.x = z.y = (Real)0;
    if (ev == EV_CT) {
      R[i00] = v00;
      R[i01] = v10;
      R[i10] = v11;
      R[i11] = v01;
    } else if (ev == EV_TC) {
      HC<Real> s0, s1;
      s0.x = v00.x + v11.x;
      s0.y = v00.y + v11.y;
      s1.x = v01.x + v10.x;
      s1.y = v01.y + v10.y;
      R[i00] = s0;
      R[i11] = s1;
      R[i01] = z;
      R[i10] = z;
    } else {
      HC<Real> s0, s1;
      s0.x = v00.x + v10.x;
      s0.y = v00.y + v10.y;
      s1.x = v01.x - v11.x;
      s1.y = v01.y - v11.y;
      R[i00] = s0;
      R[i11] = s1;
      R[i01] = z;
      R[i10] = z;
    }
  }
}

// The wire's rotation A (2x2 on bit m) alone.
template <typename Real, int NT, bool BF3>
__device__ __forceinline__ void wire_rot(HC<Real>* R, int m, const D2* A, int lane) {
  Real ar[4], ai[4];
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    ar[k] = (Real)A[k].x;
    ai[k] = (Real)A[k].y;
  }
  const int half = 1 << m;
  for (int x = lane; x < half; x += NT) {
    const HC<Real> v0 = R[x], v1 = R[x + half];
    HC<Real> w0, w1;
    w0.x = w0.y = w1.x = w1.y = (Real)0;
    cmac<Real, BF3>(ar[0], ai[0], v0.x, v0.y, w0.x, w0.y);
    cmac<Real, BF3>(ar[1], ai[1], v1.x, v1.y, w0.x, w0.y);
    cmac<Real, BF3>(ar[2], ai[2], v0.x, v0.y, w1.x, w1.y);
    cmac<Real, BF3>(ar[3], ai[3], v1.x, v1.y, w1.x, w1.y);
    R[x] = w0;
    R[x + half] = w1;
  }
}

// Event order of qubit q in slot t: V's slots (t <= L-2) run the even wall
// first, U^dagger's the odd wall first; qubit q is the control of bond q
// (in the even wall when q is even) and the target of bond q-1.
__device__ __forceinline__ int pauli_event(bool cnot, int q, int t, int L) {
  if (!cnot) return EV_CZ;
  const bool v_slot = t <= L - 2;
  return (v_slot == ((q & 1) == 0)) ? EV_CT : EV_TC;
}

// LDS bytes of one pair.
__host__ __device__ inline size_t pauli_smem_bytes(int m, int nt, size_t real_bytes) {
  if (m == 0) return (size_t)nt * 16;
  const size_t reg = ((size_t)2 << m) * 2 * real_bytes;
  return reg + (size_t)m * 4 * sizeof(D2);
}

// Trace of one pair with NT lanes; smem is the pair's LDS area
// (pauli_smem_bytes).  Lane 0 writes out[0], out[1].
template <typename Real, int NT, bool BF3>
__device__ void pauli_pair(const Real* pU, const Real* pV, int n, int L, bool cnot, unsigned char* smem, int lane,
                           Real* red, double* redd, double* out) {
  if (L == 1) {
    double lr = 1.0, li = 0.0;
    for (int q = lane; q < n; q += NT) {
      D2 A[2][2];
      pauli_slot_matrix<Real>(pU, pV, n, 1, 0, q, A);
      const double tr_ = A[0][0].x + A[1][1].x, ti_ = A[0][0].y + A[1][1].y;
      const double nr = lr * tr_ - li * ti_, ni = lr * ti_ + li * tr_;
      lr = nr;
      li = ni;
    }
    HC<double>* sc = reinterpret_cast<HC<double>*>(smem);
    sc[lane].x = lr;
    sc[lane].y = li;
    hsync<NT>();
    if (lane == 0) {
      double pr = 1.0, pim = 0.0;
      for (int i = 0; i < NT; ++i) {
        const double nr = pr * sc[i].x - pim * sc[i].y, ni = pr * sc[i].y + pim * sc[i].x;
        pr = nr;
        pim = ni;
      }
      out[0] = pr;
      out[1] = pim;
    }
    return;
  }
  const int m = 2 * L - 2;
  const int half = 1 << m;
  HC<Real>* R = reinterpret_cast<HC<Real>*>(smem);
  D2* As = reinterpret_cast<D2*>(smem + ((size_t)2 << m) * sizeof(HC<Real>));  // m slots x 4 entries
  int64_t expo = 0;
  int pending = 0;
  for (int x = lane; x < half; x += NT) {  // B_{-1}: the unit vector at label 0
    R[x].x = x == 0 ? (Real)1 : (Real)0;
    R[x].y = (Real)0;
  }
  for (int q = 0; q < n; ++q) {
    for (int t = lane; t < m; t += NT) {
      D2 A[2][2];
      pauli_slot_matrix<Real>(pU, pV, n, L, t, q, A);
      As[t * 4 + 0] = A[0][0];
      As[t * 4 + 1] = A[0][1];
      As[t * 4 + 2] = A[1][0];
      As[t * 4 + 3] = A[1][1];
    }
    // both wire values start from B_{q-1}(a), scaled by the pending power of two
    for (int x = lane; x < half; x += NT) {
      HC<Real> v = R[x];
      if (pending) {
        v.x = ldexp(v.x, -pending);
        v.y = ldexp(v.y, -pending);
      }
      R[x] = v;
      R[x + half] = v;
    }
    hsync<NT>();
    // the walk starts inside a control event: of a slot where the control
    // comes first (CNOT), or of slot 0 (CZ, where the order is free)
    const int t0 = !cnot ? 0 : ((q & 1) == 0 ? 0 : L - 1);
    slot_pass<Real, NT, BF3>(R, m, t0, pauli_event(cnot, q, t0, L), false, As + 4 * t0, lane);
    hsync<NT>();
    for (int j = 1; j < m; ++j) {
      const int t = t0 + j < m ? t0 + j : t0 + j - m;
      slot_pass<Real, NT, BF3>(R, m, t, pauli_event(cnot, q, t, L), true, As + 4 * t, lane);
      hsync<NT>();
    }
    wire_rot<Real, NT, BF3>(R, m, As + 4 * t0, lane);
    hsync<NT>();
    // closing the loop at the start: the wire equals label b_{t0}
    Real mx = 0;
    const int bt0 = 1 << t0;
    for (int b = lane; b < half; b += NT) {
      HC<Real> v = R[b];
      if (b & bt0) {
        v = R[b + half];
        R[b] = v;
      }
      mx = fmax(mx, fmax(fabs(v.x), fabs(v.y)));
    }
    mx = hmax<Real, NT>(mx, red);
    pending = 0;
    if (mx > (Real)0 && isfinite(mx)) {
      int e;
      frexp(mx, &e);
      pending = e;
      expo += e;
    }
    hsync<NT>();
  }
  double sr = 0.0, si = 0.0;
  for (int b = lane; b < half; b += NT) {
    sr += ldexp((double)R[b].x, -pending);
    si += ldexp((double)R[b].y, -pending);
  }
  sr = hsum<double, NT>(sr, redd);
  si = hsum<double, NT>(si, redd);
  if (lane == 0) {
    out[0] = ldexp(sr, (int)expo);
    out[1] = ldexp(si, (int)expo);
  }
}

template <typename Real, int NT, int PB, bool BF3>
__global__ void __launch_bounds__(NT* PB) pauli_hea_kernel(HeaArgs a, int cnot, int per_pair_bytes) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  __shared__ Real red[16];
  __shared__ double redd[16];
  const int slot = threadIdx.x / NT;
  const int lane = threadIdx.x % NT;
  const int64_t pi = (int64_t)blockIdx.x * PB + slot;
  if (pi >= a.num_pairs) return;
  const Real* pU = reinterpret_cast<const Real*>(a.gates + pi * a.gate_stride);
  const Real* pV = pU + (int64_t)a.L * a.n * 2;
  pauli_pair<Real, NT, BF3>(pU, pV, a.n, a.L, cnot != 0, smem_raw + (size_t)slot * per_pair_bytes, lane, red, redd,
                            a.trace + 2 * (a.trace_offset + pi));
}

int pauli_bits(int L) { return L <= 1 ? 0 : 2 * L - 2; }

// Algorithmic flops of one trace: per column and slot, the rotation's two
// complex multiply-adds per register entry (8 flops each) and the event's
// complex additions (2 flops per pair of entries); one layer: n 2x2 traces.
double pauli_flops_per_pair(int n, int L) {
  const int m = pauli_bits(L);
  if (m == 0) return 8.0 * n;
  const double reg = (double)(2ull << m);
  return (double)n * m * (reg * 2.0 * 8.0 + reg);
}

template <typename Real, int NT, int PB, bool BF3>
static int launch_pauli_t(const HeaArgs& a, int cnot, hipStream_t s) {
  const int m = pauli_bits(a.L);
  const size_t per_pair = (pauli_smem_bytes(m, NT, sizeof(Real)) + 15) & ~(size_t)15;
  const size_t smem = (size_t)PB * per_pair;
  if (smem > 160 * 1024) return set_error(FP_ETOOBIG, "Pauli HEA register of %d bits does not fit LDS", m + 1);
  if (smem > 64 * 1024) {
    hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(pauli_hea_kernel<Real, NT, PB, BF3>),
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)smem);
    if (e != hipSuccess) (void)hipGetLastError();  // the limit may already allow it
  }
  const int64_t blocks = (a.num_pairs + PB - 1) / PB;
  hipLaunchKernelGGL((pauli_hea_kernel<Real, NT, PB, BF3>), dim3((unsigned)blocks), dim3(NT * PB), smem, s, a, cnot,
                     (int)per_pair);
  return check_launch("pauli_hea_sweep");
}

// Lanes per pair by register size: up to 2^7 entries 16 lanes (16 pairs per
// workgroup), up to 2^11 64 lanes (4 pairs), beyond 256 lanes.
template <typename Real, bool BF3>
static int launch_pauli_real(const HeaArgs& a, int cnot, hipStream_t s) {
  const int m = pauli_bits(a.L);
  if (m <= 6) return launch_pauli_t<Real, 16, 16, BF3>(a, cnot, s);
  if (m <= 10) return launch_pauli_t<Real, 64, 4, BF3>(a, cnot, s);
  return launch_pauli_t<Real, 256, 1, BF3>(a, cnot, s);
}

int launch_pauli_hea(const HeaArgs& a, int precision, int cnot, hipStream_t s) {
  if (a.num_pairs <= 0) return FP_OK;
  if (precision == FP_C128) return launch_pauli_real<double, false>(a, cnot, s);
  return a.bf3 ? launch_pauli_real<float, true>(a, cnot, s) : launch_pauli_real<float, false>(a, cnot, s);
}

}  // namespace fp
