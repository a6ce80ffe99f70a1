// Device routines of the hardware-efficient-ansatz sweep (Walsh-Hadamard
// column transfer).  Included by the kernels that run it.
#pragma once
#include <hip/hip_runtime.h>
#include <math.h>

#include "sweep_dev.h"

namespace fp {

template <typename Real>
struct HC {
  Real x, y;
};

struct D2 {
  double x, y;
};

__device__ __forceinline__ D2 dmul(D2 a, D2 b) { return D2{a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x}; }

// R = RZ(phi) RY(theta) as [out][in].
__device__ __forceinline__ void rot(double theta, double phi, D2 r[2][2]) {
  double s, c, sp, cp;
  sincos(0.5 * theta, &s, &c);
  sincos(0.5 * phi, &sp, &cp);
  const D2 em{cp, -sp}, ep{cp, sp};  // e^{-i phi/2}, e^{+i phi/2}
  r[0][0] = D2{em.x * c, em.y * c};
  r[0][1] = D2{-em.x * s, -em.y * s};
  r[1][0] = D2{ep.x * s, ep.y * s};
  r[1][1] = D2{ep.x * c, ep.y * c};
}

__device__ __forceinline__ void dag(const D2 a[2][2], D2 r[2][2]) {
  for (int i = 0; i < 2; ++i)
    for (int j = 0; j < 2; ++j) r[i][j] = D2{a[j][i].x, -a[j][i].y};
}

__device__ __forceinline__ void mat2(const D2 a[2][2], const D2 b[2][2], D2 r[2][2]) {
  for (int i = 0; i < 2; ++i)
    for (int j = 0; j < 2; ++j) {
      D2 s0 = dmul(a[i][0], b[0][j]), s1 = dmul(a[i][1], b[1][j]);
      r[i][j] = D2{s0.x + s1.x, s0.y + s1.y};
    }
}

// Slot matrix A_t of qubit q.  ang(c, l, q) -> (theta, phi) of circuit c.
template <typename Real>
__device__ void slot_matrix(const Real* angU, const Real* angV, int n, int L, int t, int q, D2 out[2][2]) {
  D2 ru[2][2], rv[2][2], rud[2][2];
  auto th = [&](const Real* a, int l) { return (double)a[((int64_t)l * n + q) * 2]; };
  auto ph = [&](const Real* a, int l) { return (double)a[((int64_t)l * n + q) * 2 + 1]; };
  if (t == 0) {
    rot(th(angV, 0), ph(angV, 0), rv);
    rot(th(angU, 0), ph(angU, 0), ru);
    dag(ru, rud);
    mat2(rv, rud, out);
  } else if (t < L - 1) {
    rot(th(angV, t), ph(angV, t), out);
  } else if (t == L - 1) {
    rot(th(angV, L - 1), ph(angV, L - 1), rv);
    rot(th(angU, L - 1), ph(angU, L - 1), ru);
    dag(ru, rud);
    mat2(rud, rv, out);
  } else {
    const int l = 2 * L - 2 - t;
    rot(th(angU, l), ph(angU, l), ru);
    dag(ru, out);
  }
}

template <int NT>
__device__ __forceinline__ void hsync() {
  if constexpr (NT <= 64) {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
  } else {
    __syncthreads();
  }
}

template <typename Real, int NT>
__device__ __forceinline__ Real hmax(Real v, Real* red) {
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

template <typename T, int NT>
__device__ __forceinline__ T hsum(T v, T* red) {
  constexpr int W = NT < 64 ? NT : 64;
#pragma unroll
  for (int off = W / 2; off > 0; off >>= 1) v += __shfl_xor(v, off, W);
  if constexpr (NT > 64) {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    __syncthreads();
    if (lane == 0) red[wave] = v;
    __syncthreads();
    T s = red[0];
#pragma unroll
    for (int w = 1; w < NT / 64; ++w) s += red[w];
    v = s;
  }
  return v;
}

// Position of register entry x in LDS: its low four bits XORed with the next
// four.  The transform's first pass gives each lane 16 consecutive entries;
// unswizzled, the lanes of a wavefront would read them 128 bytes apart, all
// in the same banks.  Only bits 0..3 change, so the position stays below 2^m.
__device__ __forceinline__ int hsw(int x) { return x ^ ((x >> 4) & 15); }

__device__ __forceinline__ int ins_bits(int g, int s0, int r) {
  return ((g >> s0) << (s0 + r)) | (g & ((1 << s0) - 1));
}

// In-place WHT over bits [s0, s0+r) of B (2^m entries); optional scale 2^-e.
template <typename Real, int NT, int R>
__device__ __forceinline__ void wht_pass(HC<Real>* B, int m, int s0, int lane, int scale_e) {
  const int ng = 1 << (m - R);
  for (int g = lane; g < ng; g += NT) {
    const int base = ins_bits(g, s0, R);
    HC<Real> v[1 << R];
#pragma unroll
    for (int k = 0; k < (1 << R); ++k) v[k] = B[hsw(base + (k << s0))];
    if (scale_e != 0) {
#pragma unroll
      for (int k = 0; k < (1 << R); ++k) {
        v[k].x = ldexp(v[k].x, -scale_e);
        v[k].y = ldexp(v[k].y, -scale_e);
      }
    }
#pragma unroll
    for (int st = 0; st < R; ++st) {
#pragma unroll
      for (int k = 0; k < (1 << R); ++k) {
        if (k & (1 << st)) continue;
        const HC<Real> a = v[k], b = v[k | (1 << st)];
        v[k].x = a.x + b.x;
        v[k].y = a.y + b.y;
        v[k | (1 << st)].x = a.x - b.x;
        v[k | (1 << st)].y = a.y - b.y;
      }
    }
#pragma unroll
    for (int k = 0; k < (1 << R); ++k) B[hsw(base + (k << s0))] = v[k];
  }
}

template <typename Real, int NT>
__device__ void wht(HC<Real>* B, int m, int lane, int scale_e) {
  int s0 = 0;
  bool first = true;
  while (s0 < m) {
    const int r = (m - s0) >= 4 ? 4 : (m - s0);
    const int e = first ? scale_e : 0;
    switch (r) {
      case 4: wht_pass<Real, NT, 4>(B, m, s0, lane, e); break;
      case 3: wht_pass<Real, NT, 3>(B, m, s0, lane, e); break;
      case 2: wht_pass<Real, NT, 2>(B, m, s0, lane, e); break;
      default: wht_pass<Real, NT, 1>(B, m, s0, lane, e); break;
    }
    hsync<NT>();
    s0 += r;
    first = false;
  }
}

// Trace of one HEA pair (angles of U and V as stored by the sampler) with
// NT lanes; smem is the pair's LDS area (hea_smem_bytes(m, NT)).  The result
// is written to out[0], out[1] by lane 0.
template <typename Real, int NT, bool BF3 = false>
__device__ void hea_pair(const Real* angU, const Real* angV, int n, int L, int m, unsigned char* smem, int lane,
                         Real* red, double* redd, double* out) {
  if (L == 1) {
    // Tr = prod_q Tr(A_0,q): product in float64 over lanes.
    double lr = 1.0, li = 0.0;
    for (int q = lane; q < n; q += NT) {
      D2 A[2][2];
      slot_matrix<Real>(angU, angV, n, 1, 0, q, A);
      const double tr_ = A[0][0].x + A[1][1].x, ti_ = A[0][0].y + A[1][1].y;
      const double nr = lr * tr_ - li * ti_, ni = lr * ti_ + li * tr_;
      lr = nr;
      li = ni;
    }
    // ordered product across lanes via LDS (lane order)
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
  const int h = m / 2;
  const int nlo = 1 << (h + 1), nhi = 1 << (m - h + 1);
  HC<Real>* B = reinterpret_cast<HC<Real>*>(smem);
  HC<Real>* Tlo = B + (1 << m);
  HC<Real>* Thi = Tlo + nlo;
  D2* As = reinterpret_cast<D2*>(Thi + nhi);  // m slots x 4 entries, float64
  int64_t expo = 0;
  int pending = 0;
  for (int q = 0; q < n; ++q) {
    // slot matrices of this qubit
    for (int t = lane; t < m; t += NT) {
      D2 A[2][2];
      slot_matrix<Real>(angU, angV, n, L, t, q, A);
      As[t * 4 + 0] = A[0][0];
      As[t * 4 + 1] = A[0][1];
      As[t * 4 + 2] = A[1][0];
      As[t * 4 + 3] = A[1][1];
    }
    hsync<NT>();
    // tables over the low and high halves of the bits
    for (int e = lane; e < nlo + nhi; e += NT) {
      D2 acc{1.0, 0.0};
      if (e < nlo) {
        for (int t = 0; t < h; ++t) {
          const int xt = (e >> t) & 1, xt1 = (e >> (t + 1)) & 1;
          acc = dmul(acc, As[(t + 1) * 4 + xt1 * 2 + xt]);
        }
        Tlo[e].x = (Real)acc.x;
        Tlo[e].y = (Real)acc.y;
      } else {
        const int f = e - nlo;
        for (int t = h; t < m; ++t) {
          const int xt = (f >> (t - h)) & 1;
          const int t1 = (t + 1) % m;
          const int xt1 = t1 == 0 ? ((f >> (m - h)) & 1) : ((f >> (t1 - h)) & 1);
          acc = dmul(acc, As[t1 * 4 + xt1 * 2 + xt]);
        }
        Thi[f].x = (Real)acc.x;
        Thi[f].y = (Real)acc.y;
      }
    }
    hsync<NT>();
    if (q > 0) wht<Real, NT>(B, m, lane, pending);
    // pointwise product with f_q and max
    Real mx = 0;
    const int mlo = nlo - 1;
    for (int x = lane; x < (1 << m); x += NT) {
      const HC<Real> tl = Tlo[x & mlo];
      const HC<Real> th = Thi[(x >> h) | ((x & 1) << (m - h))];
      HC<Real> f, v;
      if constexpr (BF3) {  // both products as three bf16 products each (float32 storage)
        f.x = 0;
        f.y = 0;
        cmac<Real, true>(tl.x, tl.y, th.x, th.y, f.x, f.y);
        if (q == 0) {
          v = f;
        } else {
          const HC<Real> b = B[hsw(x)];
          v.x = 0;
          v.y = 0;
          cmac<Real, true>(b.x, b.y, f.x, f.y, v.x, v.y);
        }
      } else {
        f.x = tl.x * th.x - tl.y * th.y;
        f.y = tl.x * th.y + tl.y * th.x;
        if (q == 0) {
          v = f;
        } else {
          const HC<Real> b = B[hsw(x)];
          v.x = b.x * f.x - b.y * f.y;
          v.y = b.x * f.y + b.y * f.x;
        }
      }
      B[hsw(x)] = v;
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
  // Tr = 2^expo * sum_x B(x) 2^-pending
  double sr = 0.0, si = 0.0;
  for (int x = lane; x < (1 << m); x += NT) {
    sr += ldexp((double)B[hsw(x)].x, -pending);
    si += ldexp((double)B[hsw(x)].y, -pending);
  }
  sr = hsum<double, NT>(sr, redd);
  si = hsum<double, NT>(si, redd);
  if (lane == 0) {
    out[0] = ldexp(sr, (int)expo);
    out[1] = ldexp(si, (int)expo);
  }
}

// LDS bytes of one pair of the HEA sweep.
__host__ __device__ inline size_t hea_smem_bytes(int m, int nt, size_t real_bytes) {
  if (m == 0) return (size_t)nt * 16;
  const int h = m / 2;
  const size_t elems = ((size_t)1 << m) + ((size_t)1 << (h + 1)) + ((size_t)1 << (m - h + 1));
  const size_t cbytes = 2 * real_bytes;
  return elems * cbytes + (((size_t)m * 4 * 16 + cbytes - 1) / cbytes) * cbytes;
}

}  // namespace fp
