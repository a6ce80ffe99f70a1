// The sweep planner for two-qubit-gate ensembles (program format and column
// rules in plan.h), written for one wavefront per pair.
//
// Steps, in order: merge cyclically adjacent gates of W on the same bond
// (one pass in time order, then across the wrap of the trace); link every
// surviving gate to its cyclic neighbours on both of its qubits; bucket the
// gates by bond; lay out the factor list of each merged gate; then walk every
// column from the start that keeps the register smallest and emit its
// GATE / BELL / TRACE / COLEND ops.
//
// State that a sequential planner keeps in lookup tables lives in the 64
// lanes of the wavefront:
//   * per-qubit tables (last gate touching a qubit, its bond, first gate,
//     gates per bond, column starts) hold one qubit per lane and are read
//     with readlane;
//   * the register's bit tags hold one register position per lane, so a
//     tag lookup is a ballot and removing two bits is one lane shuffle;
//   * per-gate and per-walk-start passes run one item per lane.
// The same source compiles for the host, where the wavefront is emulated by
// 64-entry arrays and the per-lane loops run in order; the host form plans
// the fixed topologies and is what the CPU tests check.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "plan.h"

namespace fp {

constexpr int WAVE = 64;

// ---- the host emulation -------------------------------------------------------
struct LanesHost {
  int a[WAVE];
  int get(int q) const { return a[q]; }
  void set(int q, int x) { a[q] = x; }
  void fill(int x) {
    for (int i = 0; i < WAVE; ++i) a[i] = x;
  }
  template <class F>
  void fill_by(F f) {
    for (int i = 0; i < WAVE; ++i) a[i] = f(i);
  }
  int at(int q) const { return a[q]; }
  int shfl_at(int q) const { return a[q & (WAVE - 1)]; }
  int find(int t, int b) const {
    for (int i = 0; i < b; ++i)
      if (a[i] == t) return i;
    return -1;
  }
  int find_flag(int f, int b) const {
    for (int i = 0; i < b; ++i)
      if (a[i] >= 0 && (a[i] & f)) return i;
    return -1;
  }
  bool any_flag(int f, int b) const { return find_flag(f, b) >= 0; }
  int count_nonneg(int lim) const {
    int c = 0;
    for (int i = 0; i < lim; ++i) c += a[i] >= 0 ? 1 : 0;
    return c;
  }
  void remove2(int lo, int hi, int b) {
    int t[WAVE];
    for (int i = 0; i < WAVE; ++i) {
      const int src = i < lo ? i : (i + 1 < hi ? i + 1 : i + 2);
      t[i] = (i < b - 2) ? a[src] : -1;
    }
    for (int i = 0; i < WAVE; ++i) a[i] = t[i];
  }
  LanesHost scan_excl() const {
    LanesHost r;
    int s = 0;
    for (int i = 0; i < WAVE; ++i) {
      r.a[i] = s;
      s += a[i];
    }
    return r;
  }
};

struct WaveHost {
  using Lanes = LanesHost;
  static constexpr int step = 1;
  int first() const { return 0; }
  void sync() const {}
  template <class F>
  void single(F f) const {
    f();
  }
  int min_i32(int v) const { return v; }
  int scan_excl(int v, int* total) const {
    *total = v;
    return 0;
  }
  bool any(bool p) const { return p; }
};

// ---- the device form ---------------------------------------------------------------
// One wavefront per workgroup.  Lanes exchange data through LDS only, and a
// wavefront's LDS operations complete in order, so a wavefront-scope fence
// (a compiler barrier) orders them; a workgroup barrier would also wait for
// the global stores of the emitted ops.
struct LanesDev {
  int v;
  __device__ static int lane() { return (int)__lane_id(); }
  __device__ int get(int q) const { return __builtin_amdgcn_readlane(v, q); }
  __device__ void set(int q, int x) { v = lane() == q ? x : v; }
  __device__ void fill(int x) { v = x; }
  template <class F>
  __device__ void fill_by(F f) {
    v = f(lane());
  }
  __device__ int at(int) const { return v; }
  __device__ int shfl_at(int q) const { return __shfl(v, q & (WAVE - 1), WAVE); }
  __device__ int find(int t, int b) const {
    const unsigned long long m = __ballot(v == t && lane() < b);
    return m ? __ffsll((long long)m) - 1 : -1;
  }
  __device__ int find_flag(int f, int b) const {
    const unsigned long long m = __ballot(v >= 0 && (v & f) != 0 && lane() < b);
    return m ? __ffsll((long long)m) - 1 : -1;
  }
  __device__ bool any_flag(int f, int b) const { return __ballot(v >= 0 && (v & f) != 0 && lane() < b) != 0ull; }
  __device__ int count_nonneg(int lim) const { return __popcll(__ballot(v >= 0 && lane() < lim)); }
  __device__ void remove2(int lo, int hi, int b) {
    const int i = lane();
    const int src = i < lo ? i : (i + 1 < hi ? i + 1 : i + 2);
    const int nv = __shfl(v, src & (WAVE - 1), WAVE);
    v = (i < b - 2) ? nv : -1;
  }
  __device__ LanesDev scan_excl() const {
    int x = v;
#pragma unroll
    for (int off = 1; off < WAVE; off <<= 1) {
      const int y = __shfl_up(x, off, WAVE);
      if (lane() >= off) x += y;
    }
    LanesDev r;
    r.v = x - v;
    return r;
  }
};

struct WaveDev {
  using Lanes = LanesDev;
  static constexpr int step = WAVE;
  __device__ int first() const { return (int)__lane_id(); }
  __device__ void sync() const {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
  }
  template <class F>
  __device__ void single(F f) const {
    if (__lane_id() == 0) f();
  }
  __device__ int min_i32(int v) const {
#pragma unroll
    for (int off = WAVE / 2; off > 0; off >>= 1) {
      const int o = __shfl_xor(v, off, WAVE);
      v = o < v ? o : v;
    }
    return v;
  }
  __device__ int scan_excl(int v, int* total) const {
    int x = v;
#pragma unroll
    for (int off = 1; off < WAVE; off <<= 1) {
      const int y = __shfl_up(x, off, WAVE);
      if ((int)__lane_id() >= off) x += y;
    }
    *total = __shfl(x, WAVE - 1, WAVE);
    return x - v;
  }
  __device__ bool any(bool p) const { return __ballot(p) != 0ull; }
};

// Scratch of the wave planner, in 16-bit entries (W = 2G merged-gate slots).
__host__ __device__ inline int64_t plan_wave_scratch_elems(int G) { return 12 * 2 * (int64_t)G; }

// Ops are written one behind, so that the end of a column can mark the op
// before it (OP_FLAG_TRACK) without reading it back.
struct WaveEmitter {
  Op* ops;
  int16_t* gseq;  // merged gate of each GATE op (optional)
  int64_t max_ops;
  int num;
  int ngate;
  bool has;
  Op pend;
  double macs, elems;
};

template <class P>
__host__ __device__ inline void wave_emit(const P& w, WaveEmitter& e, int& status, uint8_t type, int p, int q,
                                          int bits, int32_t arg) {
  if (e.num >= e.max_ops) {
    status = PLAN_ECAP;
    return;
  }
  if (e.has) {
    if (type == OP_COLEND) e.pend.type |= OP_FLAG_TRACK;
    const Op o = e.pend;
    Op* dst = e.ops + e.num - 1;
    w.single([&] { *dst = o; });
  }
  e.pend.type = type;
  e.pend.p = (uint8_t)p;
  e.pend.q = (uint8_t)q;
  e.pend.bits = (uint8_t)bits;
  e.pend.arg = arg;
  e.has = true;
  e.num += 1;
  const double sz = (double)(1ull << bits);
  e.elems += sz;
  if (type == OP_GATE) {
    e.macs += 4.0 * sz;
    if (e.gseq) {
      int16_t* gs = e.gseq + e.ngate;
      w.single([&] { *gs = (int16_t)arg; });
    }
    e.ngate += 1;
  }
}

template <class P>
__host__ __device__ inline void wave_flush(const P& w, WaveEmitter& e) {
  if (e.has) {
    const Op o = e.pend;
    Op* dst = e.ops + e.num - 1;
    w.single([&] { *dst = o; });
    e.has = false;
  }
}

// Plan one pair.  bw: bond of each position of W (2G entries: V's gates in
// time order, then U's gates in reverse order); scratch: plan_wave_scratch_elems(G)
// entries; ops: plan_max_ops(G, n); wgates, factors: 2G each; gseq (may be
// null): 2G entries, the merged gate applied by each GATE op in program order.
// n <= 64.
template <class P>
__host__ __device__ inline PlanHeader plan_pair_wave(const P& w, int n, int G, const int16_t* bw, int16_t* scratch,
                                                     Op* ops, int2* wgates, int32_t* factors, int16_t* gseq) {
  using Lanes = typename P::Lanes;
  const int W = 2 * G;
  int16_t* mbond = scratch;
  int16_t* head = scratch + W;
  int16_t* tail = scratch + 2 * W;
  int16_t* cnt = scratch + 3 * W;
  int16_t* dead = scratch + 4 * W;
  int16_t* nextf = scratch + 5 * W;
  int16_t* non0 = scratch + 6 * W;
  int16_t* non1 = scratch + 7 * W;
  int16_t* pon0 = scratch + 8 * W;
  int16_t* pon1 = scratch + 9 * W;
  int16_t* colg = scratch + 10 * W;
  int16_t* gfl = scratch + 11 * W;

  PlanHeader h;
  h.num_ops = 0;
  h.num_wgates = 0;
  h.num_factors = 0;
  h.peak_bits = 0;
  h.log2_factor = 0;
  h.status = PLAN_OK;
  h.num_gate_ops = 0;
  h.macs = 0.0;
  h.elems = 0.0;
  if (G > PLAN_MAX_GATES || n < 2 || n > WAVE) {
    h.status = PLAN_ECAP;
    return h;
  }
  {
    bool bad = false;
    for (int i = w.first(); i < W; i += P::step) bad |= (bw[i] < 0 || bw[i] > n - 2);
    if (w.any(bad)) {
      h.status = PLAN_EINTERNAL;
      return h;
    }
  }

  // ---- merge pass over W in time order; per-qubit state in lanes ----
  // lastg[q]: gate holding the last position that touches q; lastb[q]: its
  // bond; lastp[q]: that position; lastc[q]: that gate's factor count.
  Lanes lastg, lastb, lastp, lastc, firstg;
  lastg.fill(-1);
  lastb.fill(-1);
  lastp.fill(-1);
  lastc.fill(0);
  firstg.fill(-1);
  int nw = 0;
  for (int i0 = 0; i0 < W; i0 += WAVE) {
    Lanes bch;
    bch.fill_by([&](int j) { return i0 + j < W ? (int)bw[i0 + j] : -1; });
    const int lim = W - i0 < WAVE ? W - i0 : WAVE;
    for (int jj = 0; jj < lim; ++jj) {
      const int i = i0 + jj;
      const int b = bch.get(jj);
      const int kp = lastg.get(b);
      if (kp >= 0 && lastg.get(b + 1) == kp && lastb.get(b) == b) {
        const int tp = lastp.get(b);
        const int c1 = lastc.get(b) + 1;
        w.single([&] {
          nextf[tp] = (int16_t)i;
          nextf[i] = -1;
          tail[kp] = (int16_t)i;
          cnt[kp] = (int16_t)c1;
        });
        lastp.set(b, i);
        lastp.set(b + 1, i);
        lastc.set(b, c1);
        lastc.set(b + 1, c1);
      } else {
        const int k = nw++;
        w.single([&] {
          mbond[k] = (int16_t)b;
          head[k] = (int16_t)i;
          tail[k] = (int16_t)i;
          cnt[k] = 1;
          dead[k] = 0;
          nextf[i] = -1;
        });
        if (firstg.get(b) < 0) firstg.set(b, k);
        if (firstg.get(b + 1) < 0) firstg.set(b + 1, k);
        lastg.set(b, k);
        lastg.set(b + 1, k);
        lastb.set(b, b);
        lastb.set(b + 1, b);
        lastp.set(b, i);
        lastp.set(b + 1, i);
        lastc.set(b, 1);
        lastc.set(b + 1, 1);
      }
    }
  }
  w.sync();
  // ---- merge across the wrap of the trace, one bond per lane ----
  for (int q = w.first(); q < WAVE; q += P::step) {
    const int x = firstg.at(q), y = lastg.at(q);
    const int x1 = firstg.shfl_at(q + 1), y1 = lastg.shfl_at(q + 1);
    if (q < n - 1 && x >= 0 && x != y && x1 == x && y1 == y && mbond[x] == q && mbond[y] == q) {
      // y precedes x around the loop: factors of y, then of x, at x's position
      nextf[tail[y]] = head[x];
      head[x] = head[y];
      cnt[x] = (int16_t)(cnt[x] + cnt[y]);
      dead[y] = 1;
    }
  }
  w.sync();
  // ---- cyclic neighbours of the surviving gates on each qubit ----
  Lanes lg, lgb, fg, fgb, ccount;
  lg.fill(-1);
  lgb.fill(-1);
  fg.fill(-1);
  fgb.fill(-1);
  ccount.fill(0);
  for (int k0 = 0; k0 < nw; k0 += WAVE) {
    Lanes bk;
    bk.fill_by([&](int j) { return k0 + j < nw && !dead[k0 + j] ? (int)mbond[k0 + j] : -1; });
    const int lim = nw - k0 < WAVE ? nw - k0 : WAVE;
    for (int jj = 0; jj < lim; ++jj) {
      const int b = bk.get(jj);
      if (b < 0) continue;
      const int k = k0 + jj;
      for (int side = 0; side < 2; ++side) {
        const int q = b + side;
        const int pk = lg.get(q);
        if (pk >= 0) {
          const int pside = lgb.get(q) == q ? 0 : 1;
          w.single([&] {
            (pside == 0 ? non0 : non1)[pk] = (int16_t)k;
            (side == 0 ? pon0 : pon1)[k] = (int16_t)pk;
          });
        } else {
          fg.set(q, k);
          fgb.set(q, b);
        }
        lg.set(q, k);
        lgb.set(q, b);
      }
      ccount.set(b, ccount.get(b) + 1);
    }
  }
  w.sync();
  for (int q = w.first(); q < WAVE; q += P::step) {
    const int f = fg.at(q), l = lg.at(q);
    if (q < n && f >= 0) {
      const int lside = lgb.at(q) == q ? 0 : 1;
      const int fside = fgb.at(q) == q ? 0 : 1;
      (lside == 0 ? non0 : non1)[l] = (int16_t)f;
      (fside == 0 ? pon0 : pon1)[f] = (int16_t)l;
    }
  }
  const int touched = fg.count_nonneg(n);
  // ---- gates of each bond, in time order ----
  const Lanes cstart = ccount.scan_excl();
  Lanes cfill = cstart;
  for (int k0 = 0; k0 < nw; k0 += WAVE) {
    Lanes bk;
    bk.fill_by([&](int j) { return k0 + j < nw && !dead[k0 + j] ? (int)mbond[k0 + j] : -1; });
    const int lim = nw - k0 < WAVE ? nw - k0 : WAVE;
    for (int jj = 0; jj < lim; ++jj) {
      const int b = bk.get(jj);
      if (b < 0) continue;
      const int pos = cfill.get(b);
      const int k = k0 + jj;
      w.single([&] { colg[pos] = (int16_t)k; });
      cfill.set(b, pos + 1);
    }
  }
  // ---- merged-gate table: factor lists in gate order ----
  int carry = 0;
  for (int k0 = 0; k0 < nw; k0 += P::step) {
    const int k = k0 + w.first();
    const bool live = k < nw && !dead[k];
    const int c = live ? (int)cnt[k] : 0;
    int tot;
    const int ex = w.scan_excl(c, &tot);
    if (k < nw) {
      if (!live) {
        wgates[k] = make_int2(0, 0);
      } else {
        const int start = carry + ex;
        wgates[k] = make_int2(start, c);
        int j = 0;
        for (int f = head[k]; f >= 0 && j < c; f = nextf[f]) factors[start + j++] = f;
      }
    }
    carry += tot;
  }
  w.sync();

  // ---- columns ----
  WaveEmitter e;
  e.ops = ops;
  e.gseq = gseq;
  e.max_ops = plan_max_ops(G, n);
  e.num = 0;
  e.ngate = 0;
  e.has = false;
  e.macs = 0.0;
  e.elems = 0.0;
  int status = PLAN_OK;
  int b = 0, peak = 0;
  Lanes tag;  // tag of each register position (-1: none)
  tag.fill(-1);
  for (int col = 0; col < n - 1 && status == PLAN_OK; ++col) {
    const int m = ccount.get(col);
    const int cs = cstart.get(col);
    if (m == 0) {
      if (b != 0) status = PLAN_EINTERNAL;
      wave_emit(w, e, status, OP_COLEND, 0, 0, b, col);
      continue;
    }
    // flags of the column's gates: which legs end on another gate of this bond
    for (int i = w.first(); i < m; i += P::step) {
      const int g = colg[cs + i];
      gfl[i] = (int16_t)((mbond[pon0[g]] == col ? GF_IN : 0) | (mbond[non0[g]] == col ? GF_OUT : 0) |
                         (mbond[pon1[g]] == col ? GF_C1IN : 0) | (mbond[non1[g]] == col ? GF_C1OUT : 0));
    }
    w.sync();
    // walk start with the smallest peak (first such start on ties)
    int key = 0x7fffffff;
    for (int s = w.first(); s < m; s += P::step) {
      int pk = walk_peak(gfl, m, s, b);
      if (pk > 0x7ffe) pk = 0x7ffe;
      const int kk = (pk << 16) | s;
      key = kk < key ? kk : key;
    }
    key = w.min_i32(key);
    const int best = key & 0xffff, bestpeak = key >> 16;
    if (bestpeak > PLAN_MAX_BITS) {
      status = PLAN_EWIDE;
      break;
    }
    const int first = colg[cs + best];
    for (int t0 = 0; t0 < m && status == PLAN_OK; t0 += WAVE) {
      // per-gate facts of the next (up to) 64 gates of the walk
      Lanes ig, iX, iZ, ifl;
      ig.fill_by([&](int j) {
        const int t = t0 + j;
        if (t >= m) return -1;
        const int idx = best + t < m ? best + t : best + t - m;
        return (int)colg[cs + idx];
      });
      iX.fill_by([&](int j) { return t0 + j < m ? (int)non0[ig.at(j)] : -1; });
      iZ.fill_by([&](int j) { return t0 + j < m ? (int)non1[ig.at(j)] : -1; });
      ifl.fill_by([&](int j) {
        if (t0 + j >= m) return 0;
        const int g = ig.at(j);
        return (mbond[pon0[g]] == col ? 1 : 0) | (mbond[non0[g]] == col - 1 ? 2 : 0) |
               (mbond[pon1[g]] == col + 1 ? 4 : 0) | (mbond[non1[g]] == col + 1 ? 8 : 0);
      });
      const int lim = m - t0 < WAVE ? m - t0 : WAVE;
      for (int jj = 0; jj < lim && status == PLAN_OK; ++jj) {
        const int t = t0 + jj;
        const int g = ig.get(jj), X = iX.get(jj), Z = iZ.get(jj), fl = ifl.get(jj);
        if (b + 4 > WAVE) {
          status = PLAN_EWIDE;
          break;
        }
        // input leg on qubit col
        int pin = tag.find(seg_key(g, 0), b);
        if (pin < 0) {
          if (!(t == 0 && (fl & 1))) {
            status = PLAN_EINTERNAL;
            break;
          }
          tag.set(b, seg_key(g, 0));
          tag.set(b + 1, seg_key(g, 0) | TAG_OUT);
          pin = b;
          b += 2;
          wave_emit(w, e, status, OP_BELL, 0, 0, b, 0);
        }
        // output leg on qubit col
        int pout;
        if (fl & 2) {
          pout = tag.find(seg_key(X, 1), b);
          if (pout < 0) {
            status = PLAN_EINTERNAL;
            break;
          }
        } else {
          pout = tag.find(seg_key(X, 0) | TAG_OUT, b);
          if (pout < 0) {
            tag.set(b, seg_key(X, 0));
            tag.set(b + 1, seg_key(X, 0) | TAG_OUT);
            pout = b + 1;
            b += 2;
            wave_emit(w, e, status, OP_BELL, 0, 0, b, 0);
          }
        }
        if (pin >= b || pout >= b || pin == pout) {
          status = PLAN_EINTERNAL;
          break;
        }
        if (b > peak) peak = b;
        wave_emit(w, e, status, OP_GATE, pin, pout, b, g);
        // pin now holds the input leg on qubit col+1, pout the output leg
        tag.set(pout, TAG_TMP);
        if (fl & 4) {
          tag.set(pin, seg_key(g, 1));
        } else {
          const int partner = tag.find(seg_key(g, 1) | TAG_PEND, b);
          if (partner >= 0) {
            const int lo = pin < partner ? pin : partner, hi = pin < partner ? partner : pin;
            tag.remove2(lo, hi, b);
            b -= 2;
            wave_emit(w, e, status, OP_TRACE, lo, hi, b, 0);
          } else {
            tag.set(pin, seg_key(g, 1) | TAG_FIRST);
          }
        }
        pout = tag.find_flag(TAG_TMP, b);
        if (pout < 0) {
          status = PLAN_EINTERNAL;
          break;
        }
        if (fl & 8) {
          tag.set(pout, seg_key(Z, 0));
        } else if (Z == first) {
          const int partner = tag.find_flag(TAG_FIRST, b);
          if (partner < 0 || partner == pout) {
            status = PLAN_EINTERNAL;
            break;
          }
          const int lo = pout < partner ? pout : partner, hi = pout < partner ? partner : pout;
          tag.remove2(lo, hi, b);
          b -= 2;
          wave_emit(w, e, status, OP_TRACE, lo, hi, b, 0);
        } else {
          tag.set(pout, seg_key(Z, 1) | TAG_PEND);
        }
      }
    }
    if (status != PLAN_OK) break;
    // only labels for the next column may remain
    if (tag.any_flag(TAG_OUT | TAG_PEND | TAG_FIRST | TAG_TMP, b)) status = PLAN_EINTERNAL;
    wave_emit(w, e, status, OP_COLEND, 0, 0, b, col);
    w.sync();
  }
  if (status == PLAN_OK && b != 0) status = PLAN_EINTERNAL;
  wave_flush(w, e);

  h.num_ops = e.num;
  h.num_wgates = nw;
  h.num_factors = carry;
  h.peak_bits = peak;
  h.log2_factor = n - touched;
  h.status = status;
  h.num_gate_ops = e.ngate;
  h.macs = e.macs;
  h.elems = e.elems;
  return h;
}

}  // namespace fp
