// Philox4x32-10 counter-based generator (Salmon, Moraes, Dror, Shaw,
// "Parallel random numbers: as easy as 1, 2, 3", SC'11), host and device.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace fp {

struct u32x4 {
  uint32_t v[4];
};

__host__ __device__ inline void mulhilo32(uint32_t a, uint32_t b, uint32_t* hi, uint32_t* lo) {
  uint64_t p = (uint64_t)a * (uint64_t)b;
  *hi = (uint32_t)(p >> 32);
  *lo = (uint32_t)p;
}

__host__ __device__ inline u32x4 philox4x32_10(uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3,
                                               uint32_t k0, uint32_t k1) {
  const uint32_t M0 = 0xD2511F53u, M1 = 0xCD9E8D57u;
  const uint32_t W0 = 0x9E3779B9u, W1 = 0xBB67AE85u;
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    if (r > 0) {
      k0 += W0;
      k1 += W1;
    }
    uint32_t hi0, lo0, hi1, lo1;
    mulhilo32(M0, c0, &hi0, &lo0);
    mulhilo32(M1, c2, &hi1, &lo1);
    uint32_t n0 = hi1 ^ c1 ^ k0;
    uint32_t n2 = hi0 ^ c3 ^ k1;
    c0 = n0;
    c1 = lo1;
    c2 = n2;
    c3 = lo0;
  }
  u32x4 r;
  r.v[0] = c0;
  r.v[1] = c1;
  r.v[2] = c2;
  r.v[3] = c3;
  return r;
}

// One draw of the sampler's stream: counter (word, item, pair lo, pair hi | circuit << 31).
__host__ __device__ inline u32x4 draw(uint64_t seed, uint32_t word, uint32_t item, uint64_t pair,
                                      uint32_t circuit) {
  return philox4x32_10(word, item, (uint32_t)pair,
                       ((uint32_t)(pair >> 32) & 0x7FFFFFFFu) | (circuit << 31), (uint32_t)seed,
                       (uint32_t)(seed >> 32));
}

// ((a >> 5) * 2^26 + (b >> 6) + 1) * 2^-53, exact in float64, in (0, 1].
__host__ __device__ inline double u53(uint32_t a, uint32_t b) {
  return ((double)(a >> 5) * 67108864.0 + (double)(b >> 6) + 1.0) * 1.1102230246251565e-16;
}

// Unbiased bond in [0, n-2] for local random step `step` of one circuit:
// the first 32-bit output below the largest multiple of n-1, reduced mod n-1.
// A word is rejected with probability < 2^-26 (n <= 64), so the scan of at
// most 4096 words never ends by its bound in practice; the bound exists so
// that every GPU thread has an exit.
__host__ __device__ inline int32_t sample_bond(uint64_t seed, uint64_t pair, uint32_t circuit,
                                               uint32_t step, int32_t n) {
  const uint32_t m = (uint32_t)(n - 1);
  const uint64_t limit = 4294967296ull - (4294967296ull % m);
  uint32_t last = 0;
  for (uint32_t w = 16; w < 16 + 1024; ++w) {
    u32x4 x = draw(seed, w, step, pair, circuit);
    for (int i = 0; i < 4; ++i) {
      if ((uint64_t)x.v[i] < limit) return (int32_t)(x.v[i] % m);
      last = x.v[i];
    }
  }
  return (int32_t)(last % m);
}

}  // namespace fp
