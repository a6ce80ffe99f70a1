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
  void put(int q, int x) { a[q] = x; }
  void or_at(int q, int x) { a[q] |= x; }
  void add_at(int q, int x) { a[q] += x; }
  // sum over lanes of a[i] * 2^i (exact while below 2^53)
  double pow2_sum() const {
    double s = 0.0;
    for (int i = 0; i < WAVE; ++i) s += (double)a[i] * (double)(1ull << i);
    return s;
  }
  void set2(int q1, int q2, int x) {
    a[q1] = x;
    a[q2] = x;
  }
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
  void atomic_add(int32_t* p, int v) const { *p += v; }
};

// ---- the device form ---------------------------------------------------------------
// One wavefront per workgroup.  Lanes exchange data through LDS only, and a
// wavefront's LDS operations complete in order, so a wavefront-scope fence
// (a compiler barrier) orders them; a workgroup barrier would also wait for
// the global stores of the emitted ops.
// v_writelane: x (uniform) into lane q of v.  Clang has no builtin for it,
// so the LLVM intrinsic is named directly.
__device__ int lane_write(int x, int q, int v) __asm("llvm.amdgcn.writelane.i32");

// Writes to one lane take a lane index in [0, 64) (writelane uses its low six
// bits); every caller's index is a qubit, a register position or a chunk slot.
struct LanesDev {
  int v;
  __device__ static int lane() { return (int)__lane_id(); }
  // lanes below b, as a ballot mask (b in [0, 64])
  __device__ static unsigned long long below(int b) { return b >= WAVE ? ~0ull : ((1ull << b) - 1ull); }
  __device__ int get(int q) const { return __builtin_amdgcn_readlane(v, q); }
  __device__ void set(int q, int x) { v = lane_write(x, q, v); }
  __device__ void fill(int x) { v = x; }
  template <class F>
  __device__ void fill_by(F f) {
    v = f(lane());
  }
  __device__ int at(int) const { return v; }
  __device__ void put(int, int x) { v = x; }
  __device__ void or_at(int q, int x) { set(q, get(q) | x); }
  __device__ void add_at(int q, int x) { set(q, get(q) + x); }
  __device__ double pow2_sum() const {
    double s = (double)v * (double)(1ull << lane());
#pragma unroll
    for (int off = WAVE / 2; off > 0; off >>= 1) s += __shfl_xor(s, off, WAVE);
    return s;
  }
  __device__ void set2(int q1, int q2, int x) {
    set(q1, x);
    set(q2, x);
  }
  __device__ int shfl_at(int q) const { return __shfl(v, q & (WAVE - 1), WAVE); }
  __device__ int find(int t, int b) const {
    const unsigned long long m = __ballot(v == t) & below(b);
    return m ? __ffsll((long long)m) - 1 : -1;
  }
  __device__ int find_flag(int f, int b) const {
    const unsigned long long m = __ballot(v >= 0 && (v & f) != 0) & below(b);
    return m ? __ffsll((long long)m) - 1 : -1;
  }
  __device__ bool any_flag(int f, int b) const { return (__ballot(v >= 0 && (v & f) != 0) & below(b)) != 0ull; }
  __device__ int count_nonneg(int lim) const { return __popcll(__ballot(v >= 0) & below(lim)); }
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
  __device__ void atomic_add(int32_t* p, int v) const { atomicAdd(p, v); }
};

// Scratch of the wave planner, in 16-bit entries: 13 slots of W = 2G entries
// (arrays whose lifetimes do not overlap share a slot) and per-qubit tables.
// The bond list may live in slot 11 (it is not read after step 2, and the
// slot's next array is first written in step 4).
constexpr int PLAN_SLOTS = 13;
constexpr int PLAN_BOND_SLOT = 11;
__host__ __device__ inline int64_t plan_wave_scratch_elems(int G) { return PLAN_SLOTS * 2 * (int64_t)G + 256; }

// Emitted ops are buffered in lanes, 64 at a time (lane j holds op j of the
// chunk), and stored together; the end of a column marks the op before it
// (OP_FLAG_TRACK) in the buffer.  The merged gate of each GATE op is buffered
// the same way.  MACs and register sizes are counted per register width.
template <class P>
struct WaveEmitter {
  using Lanes = typename P::Lanes;
  Op* ops;
  int16_t* gseq;  // merged gate of each GATE op (optional)
  int64_t max_ops;
  int num;    // ops emitted
  int ngate;  // GATE ops emitted
  Lanes w0, w1;           // chunk of packed ops: type | p << 8 | q << 16 | bits << 24, arg
  Lanes gq;               // chunk of merged-gate indices
  Lanes nops, ngates;     // ops and GATE ops per register width
};

template <class P>
__host__ __device__ inline void wave_store_ops(const P& w, WaveEmitter<P>& e, int first, int count) {
  for (int j = w.first(); j < count; j += P::step) {
    const unsigned x = (unsigned)e.w0.at(j);
    Op o;
    o.type = (uint8_t)(x & 0xff);
    o.p = (uint8_t)((x >> 8) & 0xff);
    o.q = (uint8_t)((x >> 16) & 0xff);
    o.bits = (uint8_t)(x >> 24);
    o.arg = e.w1.at(j);
    e.ops[first + j] = o;
  }
}

template <class P>
__host__ __device__ inline void wave_store_gseq(const P& w, WaveEmitter<P>& e, int first, int count) {
  if (!e.gseq) return;
  for (int j = w.first(); j < count; j += P::step) e.gseq[first + j] = (int16_t)e.gq.at(j);
}

template <class P>
__host__ __device__ inline void wave_emit(const P& w, WaveEmitter<P>& e, int& status, uint8_t type, int p, int q,
                                          int bits, int32_t arg) {
  if (e.num >= e.max_ops) {
    status = PLAN_ECAP;
    return;
  }
  const int slot = e.num & (WAVE - 1);
  if (slot == 0 && e.num > 0) {  // the chunk is full: finish its last op, store it
    if (type == OP_COLEND) e.w0.or_at(WAVE - 1, OP_FLAG_TRACK);
    wave_store_ops(w, e, e.num - WAVE, WAVE);
  } else if (type == OP_COLEND && e.num > 0) {
    e.w0.or_at(slot - 1, OP_FLAG_TRACK);
  }
  e.w0.set(slot, (int)((unsigned)type | ((unsigned)p << 8) | ((unsigned)q << 16) | ((unsigned)bits << 24)));
  e.w1.set(slot, arg);
  e.nops.add_at(bits, 1);
  if (type == OP_GATE) {
    const int gs = e.ngate & (WAVE - 1);
    e.gq.set(gs, arg);
    if (gs == WAVE - 1) wave_store_gseq(w, e, e.ngate - (WAVE - 1), WAVE);
    e.ngate += 1;
    e.ngates.add_at(bits, 1);
  }
  e.num += 1;
}

template <class P>
__host__ __device__ inline void wave_flush(const P& w, WaveEmitter<P>& e) {
  if (e.num > 0) {
    const int rem = ((e.num - 1) & (WAVE - 1)) + 1;
    wave_store_ops(w, e, e.num - rem, rem);
  }
  const int grem = e.ngate & (WAVE - 1);
  if (grem) wave_store_gseq(w, e, e.ngate - grem, grem);
}

// Plan one pair.  bw: bond of each position of W (2G entries: V's gates in
// time order, then U's gates in reverse order; may be slot PLAN_BOND_SLOT of
// the scratch); scratch: plan_wave_scratch_elems(G) entries (4-byte aligned);
// ops: plan_max_ops(G, n); wgates, factors: 2G each;
// gseq (may be null): 2G entries, the merged gate applied by each GATE op in
// program order.  n <= 64.
//
// A position of W belongs to the same merged gate as the previous position on
// its lower qubit when that position is also the previous one on its upper
// qubit and lies on the same bond; merged gates are numbered by their first
// position.  Neighbours on a qubit follow from the previous position on that
// qubit; the gate merged across the wrap of the trace (the last gate of a bond
// whose qubits see no other gate after it nor before the bond's first gate)
// drops out of the neighbour lists, its factors going in front of the first.
template <class P>
__host__ __device__ inline PlanHeader plan_pair_wave(const P& w, int n, int G, const int16_t* bw, int16_t* scratch,
                                                     Op* ops, int2* wgates, int32_t* factors, int16_t* gseq) {
  using Lanes = typename P::Lanes;
  const int W = 2 * G;
  // slots and the steps their arrays live in
  int16_t* prev0 = scratch;             // 1-4: previous position on the lower qubit of a position
  int16_t* prev1 = scratch + W;         // 1-4: ... on the upper qubit
  int16_t* gid = scratch + 2 * W;       // 2-4: merged gate of a position
  int16_t* root = scratch + 3 * W;      // 2: first position of its merged gate
  int16_t* mbond = scratch + 4 * W;     // 2-7
  int16_t* head = scratch + 5 * W;      // 2-6
  int16_t* tail = scratch + 6 * W;      // 2-4
  int16_t* dead = scratch + 7 * W;      // 2-6
  int16_t* nextf = scratch + 8 * W;     // 2-6
  int32_t* cnt32 = reinterpret_cast<int32_t*>(scratch + 9 * W);  // 2 (slots 9 and 10)
  int16_t* pon1 = scratch + PLAN_BOND_SLOT * W;                  // 4-7 (the bond list in 1-2)
  int16_t* cnt = scratch + 12 * W;      // 2-6
  int16_t* non0 = root;                 // 4-7
  int16_t* non1 = scratch + 9 * W;      // 4-7
  int16_t* pon0 = scratch + 10 * W;     // 4-7
  int16_t* colg = gid;                  // 5-7
  int16_t* gfl = tail;                  // 7
  int16_t* firstpos = scratch + PLAN_SLOTS * W;
  int16_t* larr = firstpos + WAVE;
  int32_t* bcnt32 = reinterpret_cast<int32_t*>(larr + WAVE);
  // walk tables of the columns (written in 7, read in 8)
  int16_t* wk_g = prev0;
  int16_t* wk_X = prev1;
  int16_t* wk_Z = head;
  int16_t* wk_f = dead;

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

  // ---- 1. previous position on each qubit, one qubit per lane ----
  Lanes lastp;
  lastp.fill(-1);
  for (int i0 = 0; i0 < W; i0 += WAVE) {
    Lanes bch, pv0, pv1;
    bch.fill_by([&](int j) { return i0 + j < W ? (int)bw[i0 + j] : -1; });
    pv0.fill(-1);
    pv1.fill(-1);
    const int lim = W - i0 < WAVE ? W - i0 : WAVE;
    for (int jj = 0; jj < lim; ++jj) {
      const int b = bch.get(jj);
      pv0.set(jj, lastp.get(b));
      pv1.set(jj, lastp.get(b + 1));
      lastp.set2(b, b + 1, i0 + jj);
    }
    for (int j = w.first(); j < lim; j += P::step) {
      prev0[i0 + j] = (int16_t)pv0.at(j);
      prev1[i0 + j] = (int16_t)pv1.at(j);
    }
  }
  for (int q = w.first(); q < WAVE; q += P::step) {
    firstpos[q] = -1;
    bcnt32[q] = 0;
  }
  w.sync();
  // ---- 2. merged gates: flags, numbering by first position, chains ----
  int nw = 0;
  for (int i0 = 0; i0 < W; i0 += P::step) {
    const int i = i0 + w.first();
    int hd = 0;
    if (i < W) {
      const int b = bw[i], p0 = prev0[i];
      const bool mf = p0 >= 0 && p0 == prev1[i] && bw[p0] == b;
      hd = mf ? 0 : 1;
      root[i] = (int16_t)(mf ? p0 : i);
      nextf[i] = -1;
      if (prev0[i] < 0) firstpos[b] = (int16_t)i;
      if (prev1[i] < 0) firstpos[b + 1] = (int16_t)i;
    }
    int tot;
    const int ex = w.scan_excl(hd, &tot);
    if (i < W && hd) gid[i] = (int16_t)(nw + ex);
    nw += tot;
  }
  w.sync();
  for (;;) {  // pointer jumping to the first position of each chain
    bool ch = false;
    for (int i = w.first(); i < W; i += P::step) {
      const int r = root[i], rr = root[r];
      if (rr != r) {
        root[i] = (int16_t)rr;
        ch = true;
      }
    }
    w.sync();
    if (!w.any(ch)) break;
  }
  for (int i = w.first(); i < W; i += P::step) {
    const int r = root[i];
    if (r != i) {
      gid[i] = gid[r];
      nextf[prev0[i]] = (int16_t)i;
    } else {
      const int k = gid[i];
      mbond[k] = bw[i];
      head[k] = (int16_t)i;
      dead[k] = 0;
      cnt32[k] = 0;
    }
  }
  w.sync();
  for (int i = w.first(); i < W; i += P::step) {
    w.atomic_add(&cnt32[gid[i]], 1);
    if (nextf[i] < 0) tail[gid[i]] = (int16_t)i;
  }
  w.sync();
  for (int k = w.first(); k < nw; k += P::step) cnt[k] = (int16_t)cnt32[k];
  Lanes firstg, lastg;
  firstg.fill_by([&](int q) { return q < n && firstpos[q] >= 0 ? (int)gid[firstpos[q]] : -1; });
  lastg.fill_by([&](int q) { return q < n && lastp.at(q) >= 0 ? (int)gid[lastp.at(q)] : -1; });
  // ---- 3. merges across the wrap of the trace, one bond per lane ----
  Lanes wx, wy;
  for (int q = w.first(); q < WAVE; q += P::step) {
    const int x = firstg.at(q), y = lastg.at(q);
    const int x1 = firstg.shfl_at(q + 1), y1 = lastg.shfl_at(q + 1);
    int mx = -1, my = -1;
    if (q < n - 1 && x >= 0 && x != y && x1 == x && y1 == y && mbond[x] == q && mbond[y] == q) {
      mx = x;
      my = y;
      dead[y] = 1;
    }
    wx.put(q, mx);
    wy.put(q, my);
  }
  w.sync();
  // last surviving gate on each qubit
  for (int q = w.first(); q < WAVE; q += P::step) {
    int L = -1;
    const int y = lastg.at(q);
    if (q < n && y >= 0) {
      if (!dead[y]) {
        L = y;
      } else {
        const int pp = (mbond[y] == q ? prev0 : prev1)[head[y]];
        L = pp >= 0 ? (int)gid[pp] : -1;
      }
    }
    larr[q] = (int16_t)L;
  }
  w.sync();
  // ---- 4. cyclic neighbours of the surviving gates on each qubit ----
  for (int k = w.first(); k < nw; k += P::step) {
    if (dead[k]) continue;
    const int b = mbond[k], hp = head[k];
    for (int side = 0; side < 2; ++side) {
      const int q = b + side;
      const int pp = (side == 0 ? prev0 : prev1)[hp];
      const int pk = pp >= 0 ? (int)gid[pp] : (int)larr[q];
      (side == 0 ? pon0 : pon1)[k] = (int16_t)pk;
      const int pside = mbond[pk] == q ? 0 : 1;
      (pside == 0 ? non0 : non1)[pk] = (int16_t)k;
    }
    w.atomic_add(&bcnt32[b], 1);
  }
  w.sync();
  for (int q = w.first(); q < WAVE; q += P::step) {
    const int x = wx.at(q), y = wy.at(q);
    if (x >= 0) {  // y precedes x around the loop: factors of y, then of x
      nextf[tail[y]] = head[x];
      head[x] = head[y];
      cnt[x] = (int16_t)(cnt[x] + cnt[y]);
    }
  }
  const int touched = firstg.count_nonneg(n);
  w.sync();
  // ---- 5. gates of each bond in gate order ----
  Lanes ccount;
  ccount.fill_by([&](int q) { return (int)bcnt32[q]; });
  const Lanes cstart = ccount.scan_excl();
  {
    Lanes cfill = cstart;
    for (int k0 = 0; k0 < nw; k0 += WAVE) {
      Lanes bk, posl;
      bk.fill_by([&](int j) { return k0 + j < nw && !dead[k0 + j] ? (int)mbond[k0 + j] : -1; });
      posl.fill(0);
      const int lim = nw - k0 < WAVE ? nw - k0 : WAVE;
      for (int jj = 0; jj < lim; ++jj) {
        const int b = bk.get(jj);
        if (b < 0) continue;
        const int pos = cfill.get(b);
        posl.set(jj, pos);
        cfill.set(b, pos + 1);
      }
      for (int j = w.first(); j < lim; j += P::step)
        if (bk.at(j) >= 0) colg[posl.at(j)] = (int16_t)(k0 + j);
    }
  }
  // ---- 6. merged-gate table: factor lists in gate order ----
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
  // ---- 7. per column: walk start with the smallest peak, walk tables ----
  Lanes relpk, firstc;
  for (int c = w.first(); c < WAVE; c += P::step) {
    int rp = 0, fg = -1;
    const int m = ccount.at(c), cs = cstart.at(c);
    if (c < n - 1 && m > 0) {
      for (int i = 0; i < m; ++i) {
        const int g = colg[cs + i];
        gfl[cs + i] = (int16_t)((mbond[pon0[g]] == c ? GF_IN : 0) | (mbond[non0[g]] == c ? GF_OUT : 0) |
                                (mbond[pon1[g]] == c ? GF_C1IN : 0) | (mbond[non1[g]] == c ? GF_C1OUT : 0));
      }
      int best = 0, bestpk = 0x7fffffff;
      for (int st = 0; st < m; ++st) {
        const int pk = walk_peak(gfl + cs, m, st, 0);
        if (pk < bestpk) {
          bestpk = pk;
          best = st;
        }
      }
      for (int t = 0; t < m; ++t) {
        const int idx = best + t < m ? best + t : best + t - m;
        const int g = colg[cs + idx];
        wk_g[cs + t] = (int16_t)g;
        wk_X[cs + t] = non0[g];
        wk_Z[cs + t] = non1[g];
        wk_f[cs + t] = (int16_t)((mbond[pon0[g]] == c ? 1 : 0) | (mbond[non0[g]] == c - 1 ? 2 : 0) |
                                 (mbond[pon1[g]] == c + 1 ? 4 : 0) | (mbond[non1[g]] == c + 1 ? 8 : 0));
      }
      rp = bestpk;
      fg = colg[cs + best];
    }
    relpk.put(c, rp);
    firstc.put(c, fg);
  }
  w.sync();

  // ---- 8. the walks: register programs ----
  WaveEmitter<P> e;
  e.ops = ops;
  e.gseq = gseq;
  e.max_ops = plan_max_ops(G, n);
  e.num = 0;
  e.ngate = 0;
  e.w0.fill(0);
  e.w1.fill(0);
  e.gq.fill(0);
  e.nops.fill(0);
  e.ngates.fill(0);
  int status = PLAN_OK;
  int b = 0, peak = 0;
  Lanes tag;  // tag of each register position (-1: none)
  tag.fill(-1);
  Lanes ig, iX, iZ, ifl;  // walk tables from flat index c0
  int c0 = -WAVE;
  for (int col = 0; col < n - 1 && status == PLAN_OK; ++col) {
    const int m = ccount.get(col);
    const int cs = cstart.get(col);
    if (m == 0) {
      if (b != 0) status = PLAN_EINTERNAL;
      wave_emit(w, e, status, OP_COLEND, 0, 0, b, col);
      continue;
    }
    if (b + relpk.get(col) > PLAN_MAX_BITS) {
      status = PLAN_EWIDE;
      break;
    }
    const int first = firstc.get(col);
    for (int t = 0; t < m && status == PLAN_OK; ++t) {
      const int ft = cs + t;
      if (ft >= c0 + WAVE) {
        c0 = ft;
        ig.fill_by([&](int j) { return c0 + j < W ? (int)wk_g[c0 + j] : -1; });
        iX.fill_by([&](int j) { return c0 + j < W ? (int)wk_X[c0 + j] : -1; });
        iZ.fill_by([&](int j) { return c0 + j < W ? (int)wk_Z[c0 + j] : -1; });
        ifl.fill_by([&](int j) { return c0 + j < W ? (int)wk_f[c0 + j] : 0; });
      }
      const int jj = ft - c0;
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
    if (status != PLAN_OK) break;
    // only labels for the next column may remain
    if (tag.any_flag(TAG_OUT | TAG_PEND | TAG_FIRST | TAG_TMP, b)) status = PLAN_EINTERNAL;
    wave_emit(w, e, status, OP_COLEND, 0, 0, b, col);
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
  h.macs = 4.0 * e.ngates.pow2_sum();
  h.elems = e.nops.pow2_sum();
  return h;
}

}  // namespace fp
