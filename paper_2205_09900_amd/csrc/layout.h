// Gate-buffer layout and small shared definitions (host and device).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/fp.h"

namespace fp {

__host__ __device__ inline int real_bytes(int precision) { return precision == FP_C128 ? 8 : 4; }

// The paper's hardware-efficient ansatz (Pauli rotations, CNOT or CZ walls).
__host__ __device__ inline bool is_pauli_hea(int ansatz) {
  return ansatz == FP_HEA_PAULI_CNOT || ansatz == FP_HEA_PAULI_CZ;
}

// Two-qubit gates per circuit (Haar ensembles).
__host__ __device__ inline int64_t gates_per_circuit(int ansatz, int n, int depth) {
  if (ansatz == FP_LOCAL_RANDOM_HAAR) return depth;
  if (ansatz == FP_BRICKWORK_HAAR || ansatz == FP_BRICKWORK_QUDIT) {
    int64_t even = n / 2, odd = (n - 1) / 2;  // bonds 0,2,.. and 1,3,..
    return even * ((depth + 1) / 2) + odd * (depth / 2);
  }
  return 0;
}

// Bond of gate g of a brickwork circuit.
__host__ __device__ inline int brickwork_bond(int n, int g) {
  const int even = n / 2, odd = (n - 1) / 2, two = even + odd;
  const int blk = g / two, r = g % two;
  (void)blk;
  return r < even ? 2 * r : 2 * (r - even) + 1;
}

__host__ __device__ inline int64_t pad64(int64_t x) { return (x + 63) & ~(int64_t)63; }

// local_dim: q of a qudit brickwork (ignored otherwise)
__host__ __device__ inline int64_t pair_bytes(int ansatz, int n, int depth, int precision, int local_dim = 0) {
  const int64_t rb = real_bytes(precision);
  if (ansatz == FP_BRICKWORK_QUDIT) {
    const int64_t d2 = (int64_t)local_dim * local_dim;
    return pad64(2 * gates_per_circuit(ansatz, n, depth) * d2 * d2 * 2 * rb);
  }
  if (ansatz == FP_HEA_RYRZ_CZ || is_pauli_hea(ansatz)) return pad64(2 * (int64_t)depth * n * 2 * rb);
  const int64_t G = gates_per_circuit(ansatz, n, depth);
  int64_t b = 2 * G * 32 * rb;
  if (ansatz == FP_LOCAL_RANDOM_HAAR) b += 2 * G * 4;
  return pad64(b);
}

// Byte offset of the bond arrays inside a local random pair.
__host__ __device__ inline int64_t bonds_offset(int n, int depth, int precision) {
  return 2 * (int64_t)depth * 32 * real_bytes(precision);
}

}  // namespace fp
