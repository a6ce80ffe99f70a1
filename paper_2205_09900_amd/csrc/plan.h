// Sweep planner for ensembles of two-qubit gates (brickwork, local random).
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
// register.  Everything here is integer bookkeeping; it compiles for host and
// device so one source plans fixed topologies on the host and local random
// pairs on the GPU.
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

// Scratch of one pair, in 16-bit entries.
__host__ __device__ inline int64_t plan_scratch_elems(int G, int n) {
  const int64_t W = 2 * (int64_t)G;
  return 17 * W + 6 * (int64_t)(n + 2) + 16;
}

__host__ __device__ inline int64_t plan_max_ops(int G, int n) { return 10 * (int64_t)G + n + 8; }

struct PlanCtx {
  int n, G, W;
  int nw;  // merged gates
  int16_t *mbond, *head, *tail, *cnt, *nextf, *dead;
  int16_t *non0, *non1, *pon0, *pon1;  // next / previous gate on lower (0) / upper (1) qubit
  int16_t *colgates;                   // gates of each bond in time order
  int16_t *lastq, *firstq, *colstart, *colfill, *lastb, *firstb;
  // register: tags of the live bits and, per tag, its bit position (-1 = none)
  int32_t* tag;
  int b;
  int16_t *lab, *outp, *pendp;  // plain labels (2 per gate), Bell out-ends, pending legs
  int16_t *gflags;              // per gate of the current column: internal-segment flags
  int16_t first_pos, tmp_pos;
  // outputs
  Op* ops;
  int2* wgates;  // (first factor, count)
  int32_t* factors;
  int64_t max_ops;
  int num_ops;
  int status;
  double macs, elems;
  int peak;
};

constexpr int32_t TAG_OUT = 1 << 27;
constexpr int32_t TAG_PEND = 1 << 28;
constexpr int32_t TAG_FIRST = 1 << 29;
constexpr int32_t TAG_TMP = 1 << 30;
constexpr int32_t TAG_KEY = TAG_OUT - 1;

// ---- register: positions are looked up through per-tag tables (O(1)) ----
__host__ __device__ inline int16_t* reg_slot(PlanCtx& c, int32_t t) {
  if (t & TAG_TMP) return &c.tmp_pos;
  if (t & TAG_FIRST) return &c.first_pos;
  const int k = t & TAG_KEY;
  if (t & TAG_OUT) return &c.outp[k >> 1];
  if (t & TAG_PEND) return &c.pendp[k >> 1];
  return &c.lab[k];
}

__host__ __device__ inline int reg_find(PlanCtx& c, int32_t t) { return *reg_slot(c, t); }

__host__ __device__ inline void reg_set(PlanCtx& c, int pos, int32_t t) {
  c.tag[pos] = t;
  *reg_slot(c, t) = (int16_t)pos;
}

// Retag bit `pos` (its old tag no longer names it).
__host__ __device__ inline void reg_retag(PlanCtx& c, int pos, int32_t t) {
  *reg_slot(c, c.tag[pos]) = -1;
  reg_set(c, pos, t);
}

// Remove bits lo < hi; the bits above move down.
__host__ __device__ inline void reg_remove2(PlanCtx& c, int lo, int hi) {
  *reg_slot(c, c.tag[lo]) = -1;
  *reg_slot(c, c.tag[hi]) = -1;
  int w = lo;
  for (int i = lo + 1; i < c.b; ++i) {
    if (i == hi) continue;
    reg_set(c, w++, c.tag[i]);
  }
  c.b = w;
}

__host__ __device__ inline int32_t seg_key(int e, int side) { return 2 * e + side; }

__host__ __device__ inline void emit(PlanCtx& c, uint8_t type, int p, int q, int bits, int32_t arg) {
  if (c.num_ops >= c.max_ops) {
    c.status = PLAN_ECAP;
    return;
  }
  if (type == OP_COLEND && c.num_ops > 0) c.ops[c.num_ops - 1].type |= OP_FLAG_TRACK;
  Op o;
  o.type = type;
  o.p = (uint8_t)p;
  o.q = (uint8_t)q;
  o.bits = (uint8_t)bits;
  o.arg = arg;
  c.ops[c.num_ops++] = o;
  double sz = (double)(1ull << bits);
  c.elems += sz;
  if (type == OP_GATE) c.macs += 4.0 * sz;
}

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

__host__ __device__ inline void plan_column(PlanCtx& c, int col) {
  const int m = c.colstart[col + 1] - c.colstart[col];
  const int16_t* cg = c.colgates + c.colstart[col];
  if (m == 0) {
    if (c.b != 0) c.status = PLAN_EINTERNAL;
    emit(c, OP_COLEND, 0, 0, c.b, col);
    return;
  }
  for (int i = 0; i < m; ++i) {
    const int g = cg[i];
    c.gflags[i] = (int16_t)((c.mbond[c.pon0[g]] == col ? GF_IN : 0) | (c.mbond[c.non0[g]] == col ? GF_OUT : 0) |
                            (c.mbond[c.pon1[g]] == col ? GF_C1IN : 0) | (c.mbond[c.non1[g]] == col ? GF_C1OUT : 0));
  }
  int best = 0, bestpeak = 1 << 30;
  for (int s = 0; s < m; ++s) {
    const int pk = walk_peak(c.gflags, m, s, c.b);
    if (pk < bestpeak) {
      bestpeak = pk;
      best = s;
    }
  }
  if (bestpeak > PLAN_MAX_BITS) {
    c.status = PLAN_EWIDE;
    return;
  }
  const int first = cg[best];
  for (int t = 0; t < m && c.status == PLAN_OK; ++t) {
    const int g = cg[(best + t) % m];
    if (c.b + 4 > 64) {
      c.status = PLAN_EWIDE;
      return;
    }
    // input leg on qubit col
    int pin = reg_find(c, seg_key(g, 0));
    if (pin < 0) {
      if (!(t == 0 && c.mbond[c.pon0[g]] == col)) {
        c.status = PLAN_EINTERNAL;
        return;
      }
      reg_set(c, c.b, seg_key(g, 0));
      reg_set(c, c.b + 1, seg_key(g, 0) | TAG_OUT);
      pin = c.b;
      c.b += 2;
      emit(c, OP_BELL, 0, 0, c.b, 0);
    }
    // output leg on qubit col
    const int X = c.non0[g];
    int pout;
    if (c.mbond[X] == col - 1) {
      pout = reg_find(c, seg_key(X, 1));
      if (pout < 0) {
        c.status = PLAN_EINTERNAL;
        return;
      }
    } else {
      pout = reg_find(c, seg_key(X, 0) | TAG_OUT);
      if (pout < 0) {
        reg_set(c, c.b, seg_key(X, 0));
        reg_set(c, c.b + 1, seg_key(X, 0) | TAG_OUT);
        pout = c.b + 1;
        c.b += 2;
        emit(c, OP_BELL, 0, 0, c.b, 0);
      }
    }
    if (c.b > c.peak) c.peak = c.b;
    emit(c, OP_GATE, pin, pout, c.b, g);
    // pin now holds the input leg on qubit col+1, pout the output leg.
    reg_retag(c, pout, TAG_TMP);
    const int Y = c.pon1[g];
    if (c.mbond[Y] == col + 1) {
      reg_retag(c, pin, seg_key(g, 1));
    } else {
      const int partner = reg_find(c, seg_key(g, 1) | TAG_PEND);
      if (partner >= 0) {
        const int lo = pin < partner ? pin : partner, hi = pin < partner ? partner : pin;
        reg_remove2(c, lo, hi);
        emit(c, OP_TRACE, lo, hi, c.b, 0);
      } else {
        reg_retag(c, pin, seg_key(g, 1) | TAG_FIRST);
      }
    }
    pout = reg_find(c, TAG_TMP);
    const int Z = c.non1[g];
    if (c.mbond[Z] == col + 1) {
      reg_retag(c, pout, seg_key(Z, 0));
    } else if (Z == first) {
      const int partner = reg_find(c, seg_key(Z, 1) | TAG_FIRST);
      if (partner < 0) {
        c.status = PLAN_EINTERNAL;
        return;
      }
      const int lo = pout < partner ? pout : partner, hi = pout < partner ? partner : pout;
      reg_remove2(c, lo, hi);
      emit(c, OP_TRACE, lo, hi, c.b, 0);
    } else {
      reg_retag(c, pout, seg_key(Z, 1) | TAG_PEND);
    }
  }
  // only labels for the next column may remain
  for (int i = 0; i < c.b; ++i)
    if (c.tag[i] & (TAG_OUT | TAG_PEND | TAG_FIRST | TAG_TMP)) c.status = PLAN_EINTERNAL;
  emit(c, OP_COLEND, 0, 0, c.b, col);
}

// Plan one pair.  bond_u, bond_v: G bonds each (time order; G <= PLAN_MAX_GATES).
// scratch: plan_scratch_elems(G, n) entries; tag_store: 64 entries.  ops:
// plan_max_ops(G, n) entries; wgates: 2G; factors: 2G.  Returns the header
// (status != 0 on failure).
__host__ __device__ inline PlanHeader plan_haar_pair(int n, int G, const int16_t* bond_u,
                                                     const int16_t* bond_v, int16_t* scratch, Op* ops,
                                                     int2* wgates, int32_t* factors, int32_t* tag_store) {
  PlanCtx c;
  c.n = n;
  c.G = G;
  c.W = 2 * G;
  const int W = c.W;
  int16_t* s = scratch;
  c.mbond = s;
  s += W;
  c.head = s;
  s += W;
  c.tail = s;
  s += W;
  c.cnt = s;
  s += W;
  c.nextf = s;
  s += W;
  c.dead = s;
  s += W;
  c.non0 = s;
  s += W;
  c.non1 = s;
  s += W;
  c.pon0 = s;
  s += W;
  c.pon1 = s;
  s += W;
  c.colgates = s;
  s += W;
  c.lastq = s;
  s += n + 2;
  c.firstq = s;
  s += n + 2;
  c.colstart = s;
  s += n + 2;
  c.colfill = s;
  s += n + 2;
  c.lastb = s;
  s += n + 2;
  c.firstb = s;
  s += n + 2;
  c.lab = s;
  s += 2 * W;
  c.outp = s;
  s += W;
  c.pendp = s;
  s += W;
  c.gflags = s;
  s += W;
  for (int i = 0; i < 4 * W; ++i) c.lab[i] = -1;  // lab, outp, pendp
  c.first_pos = -1;
  c.tmp_pos = -1;
  c.tag = tag_store;
  c.b = 0;
  c.ops = ops;
  c.wgates = wgates;
  c.factors = factors;
  c.max_ops = plan_max_ops(G, n);
  c.num_ops = 0;
  c.status = PLAN_OK;
  c.macs = 0.0;
  c.elems = 0.0;
  c.peak = 0;
  c.nw = 0;

  PlanHeader h;
  h.num_ops = 0;
  h.num_wgates = 0;
  h.num_factors = 0;
  h.peak_bits = 0;
  h.log2_factor = 0;
  h.status = PLAN_OK;
  h.macs = 0.0;
  h.elems = 0.0;

  if (G > PLAN_MAX_GATES) {
    h.status = PLAN_ECAP;
    return h;
  }
  for (int i = 0; i < W; ++i) {
    int b = i < G ? bond_v[i] : bond_u[2 * G - 1 - i];
    if (b < 0 || b > n - 2) {
      h.status = PLAN_EINTERNAL;
      return h;
    }
  }
  // ---- merge pass: linear, then across the wrap of the trace ----
  for (int q = 0; q < n; ++q) {
    c.lastq[q] = -1;
    c.firstq[q] = -1;
  }
  for (int i = 0; i < W; ++i) {
    const int b = i < G ? bond_v[i] : bond_u[2 * G - 1 - i];
    c.nextf[i] = -1;
    const int kp = c.lastq[b];
    if (kp >= 0 && c.lastq[b + 1] == kp && c.mbond[kp] == b) {
      c.nextf[c.tail[kp]] = i;
      c.tail[kp] = i;
      c.cnt[kp] += 1;
    } else {
      const int k = c.nw++;
      c.mbond[k] = b;
      c.head[k] = i;
      c.tail[k] = i;
      c.cnt[k] = 1;
      c.dead[k] = 0;
      if (c.firstq[b] < 0) c.firstq[b] = k;
      if (c.firstq[b + 1] < 0) c.firstq[b + 1] = k;
      c.lastq[b] = k;
      c.lastq[b + 1] = k;
    }
  }
  for (int b = 0; b < n - 1; ++b) {
    const int x = c.firstq[b], y = c.lastq[b];
    if (x < 0 || x == y) continue;
    if (c.firstq[b + 1] != x || c.lastq[b + 1] != y) continue;
    if (c.mbond[x] != b || c.mbond[y] != b) continue;
    // y precedes x around the loop: factors of y, then of x, at x's position.
    c.nextf[c.tail[y]] = c.head[x];
    c.head[x] = c.head[y];
    c.cnt[x] += c.cnt[y];
    c.dead[y] = 1;
  }
  // ---- per-qubit neighbours of every surviving gate, cyclic ----
  for (int q = 0; q < n; ++q) {
    c.lastq[q] = -1;
    c.firstq[q] = -1;
  }
  int touched = 0;
  for (int k = 0; k < c.nw; ++k) {
    if (c.dead[k]) continue;
    const int b = c.mbond[k];
    for (int side = 0; side < 2; ++side) {
      const int q = b + side;
      const int pk = c.lastq[q];
      if (pk >= 0) {
        const int pside = (c.mbond[pk] == q) ? 0 : 1;
        (pside == 0 ? c.non0 : c.non1)[pk] = k;
        (side == 0 ? c.pon0 : c.pon1)[k] = pk;
      } else {
        c.firstq[q] = k;
      }
      c.lastq[q] = k;
    }
  }
  for (int q = 0; q < n; ++q) {
    const int f = c.firstq[q], l = c.lastq[q];
    if (f < 0) continue;
    ++touched;
    const int lside = (c.mbond[l] == q) ? 0 : 1;
    const int fside = (c.mbond[f] == q) ? 0 : 1;
    (lside == 0 ? c.non0 : c.non1)[l] = f;
    (fside == 0 ? c.pon0 : c.pon1)[f] = l;
  }
  // ---- bucket gates by bond, time order kept ----
  for (int b = 0; b <= n; ++b) c.colstart[b] = 0;
  for (int k = 0; k < c.nw; ++k)
    if (!c.dead[k]) c.colstart[c.mbond[k] + 1] += 1;
  for (int b = 0; b < n; ++b) c.colstart[b + 1] += c.colstart[b];
  for (int b = 0; b < n; ++b) c.colfill[b] = c.colstart[b];
  for (int k = 0; k < c.nw; ++k)
    if (!c.dead[k]) c.colgates[c.colfill[c.mbond[k]]++] = k;
  // ---- merged-gate table ----
  int nf = 0;
  for (int k = 0; k < c.nw; ++k) {
    if (c.dead[k]) {
      wgates[k] = make_int2(0, 0);
      continue;
    }
    wgates[k] = make_int2(nf, c.cnt[k]);
    for (int f = c.head[k]; f >= 0; f = c.nextf[f]) factors[nf++] = f;
  }
  // ---- columns ----
  for (int col = 0; col < n - 1 && c.status == PLAN_OK; ++col) plan_column(c, col);
  if (c.status == PLAN_OK && c.b != 0) c.status = PLAN_EINTERNAL;

  h.num_ops = c.num_ops;
  h.num_wgates = c.nw;
  h.num_factors = nf;
  h.peak_bits = c.peak;
  h.log2_factor = n - touched;
  h.status = c.status;
  h.macs = c.macs;
  h.elems = c.elems;
  return h;
}

}  // namespace fp
