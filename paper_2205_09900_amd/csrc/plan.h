// Register programs of the column sweep for ensembles of two-qubit gates
// (brickwork, local random).
//
// The trace of W = U^dagger V is a tensor network (Sec. II.A of the paper,
// trace as a contraction).  It is contracted one qubit column at a time, in
// the qubit direction, so that the exposed indices are few (Sec. II.A; cost
// exponential in depth and linear in n, Methods A).
//
// W as a cyclic gate list: V's gates in time order, then U's gates in
// reverse order, each conjugate-transposed; the trace closes the list into a
// loop.  Cyclically adjacent gates on the same bond with no gate touching
// either qubit in between are merged into one gate (a product of factors).
//
// Column c absorbs the gates on bond c.  Its input is the boundary over the
// wire segments of qubit c that join a bond-(c-1) gate to a bond-c gate; its
// output is the boundary over the segments of qubit c+1 that join a bond-c
// gate to a bond-(c+1) gate.  Each boundary index is one register bit.  With
// the gate G (row = 2 out_c + out_{c+1}, column = 2 in_c + in_{c+1}) a column
// is a sequence of register operations:
//   GATE(p, q, g): bits p, q hold (in_c, out_c) of gate g and are replaced in
//                  place by (in_{c+1}, out_{c+1}):
//                  B'[y_in, y_out] = sum_{x_in, x_out} G[2 x_out + y_out, 2 x_in + y_in] B[x_in, x_out]
//   BELL:          append two bits holding a delta (an internal wire segment of
//                  qubit c whose two ends are consumed by two gates)
//   TRACE(p, q):   sum over p = q and remove both bits (an internal segment of
//                  qubit c+1 between two bond-c gates); higher bits move down
//   COLEND:        end of column (the kernels rescale here)
// The walk around each column starts at the gate that minimises the largest
// register.  This header holds the program format and the column rules; the
// planner itself (plan_wave.h) compiles for host and device, so one source
// plans fixed topologies on the host and local random pairs on the GPU.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace fp {

enum : uint8_t { OP_GATE = 0, OP_BELL = 1, OP_TRACE = 2, OP_COLEND = 3 };
// Flag in Op::type: the next op ends the column, so the kernels record the
// largest magnitude this op writes (for the column's power-of-two rescale).
constexpr uint8_t OP_TYPE_MASK = 0x3;
constexpr uint8_t OP_FLAG_TRACK = 0x80;

struct Op {
  uint8_t type;
  uint8_t p;
  uint8_t q;
  uint8_t bits;  // register exponent after the op
  int32_t arg;   // GATE: merged-gate index
};

struct PlanHeader {
  int32_t num_ops;
  int32_t num_wgates;
  int32_t num_factors;
  int32_t peak_bits;
  int32_t log2_factor;  // qubits no gate touches contribute a factor 2 each
  int32_t status;       // 0 ok, 1 capacity exceeded, 2 register too wide, 3 internal
  int32_t num_gate_ops; // GATE ops (one per live merged gate)
  double macs;          // complex multiply-adds of all GATE ops
  double elems;         // sum over ops of the register size (memory traffic proxy)
};

enum { PLAN_OK = 0, PLAN_ECAP = 1, PLAN_EWIDE = 2, PLAN_EINTERNAL = 3 };

constexpr int PLAN_MAX_BITS = 60;

// Factor code: the raw W position i; i < G -> V gate i, else U gate 2G-1-i, daggered.
struct FactorRef {
  int32_t circuit;  // 0 = U, 1 = V
  int32_t gate;
  int32_t dagger;
};

__host__ __device__ inline FactorRef decode_factor(int32_t code, int32_t G) {
  FactorRef f;
  if (code < G) {
    f.circuit = 1;
    f.gate = code;
    f.dagger = 0;
  } else {
    f.circuit = 0;
    f.gate = 2 * G - 1 - code;
    f.dagger = 1;
  }
  return f;
}

// Gates per circuit the planner accepts (its indices are 16-bit).
constexpr int PLAN_MAX_GATES = 16000;

__host__ __device__ inline int64_t plan_max_ops(int G, int n) { return 10 * (int64_t)G + n + 8; }

constexpr int32_t TAG_OUT = 1 << 27;
constexpr int32_t TAG_PEND = 1 << 28;
constexpr int32_t TAG_FIRST = 1 << 29;
constexpr int32_t TAG_TMP = 1 << 30;
constexpr int32_t TAG_KEY = TAG_OUT - 1;

__host__ __device__ inline int32_t seg_key(int e, int side) { return 2 * e + side; }

// Per-gate flags of a column: which of the gate's four legs sit on internal
// segments (ends on another gate of the same bond).
enum { GF_IN = 1, GF_OUT = 2, GF_C1IN = 4, GF_C1OUT = 8 };

// Largest register along the walk of the column started at gate index s.
__host__ __device__ inline int walk_peak(const int16_t* fl, int m, int s, int b0) {
  int b = b0, peak = b0;
  for (int t = 0; t < m; ++t) {
    const int i = s + t < m ? s + t : s + t - m;
    const int f = fl[i];
    const int nxt = i + 1 < m ? i + 1 : 0;
    if ((f & GF_IN) && t == 0) b += 2;
    if ((f & GF_OUT) && nxt != s) b += 2;
    if (b > peak) peak = b;
    if ((f & GF_C1IN) && t != 0) b -= 2;
    if ((f & GF_C1OUT) && nxt == s) b -= 2;
  }
  return peak;
}

}  // namespace fp
