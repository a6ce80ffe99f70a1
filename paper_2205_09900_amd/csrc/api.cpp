// C-ABI entry points of libfp.so (declared in include/fp.h): argument
// checks, plan cache, workspace partitioning and kernel dispatch.
#include <hip/hip_runtime.h>
#include <stdarg.h>
#include <stdio.h>
#include <string.h>

#include <atomic>
#include <map>
#include <mutex>
#include <tuple>
#include <vector>

#include "internal.h"
#include "plan_wave.h"
#include "layout.h"
#include "plan.h"
#include "sweep.h"
#include "tune.h"
#include "dispatch.h"

namespace fp {

static thread_local char g_err[512] = "";

int set_error(int code, const char* fmt, ...) {
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(g_err, sizeof(g_err), fmt, ap);
  va_end(ap);
  return code;
}

int check_hip(hipError_t e, const char* what) {
  if (e == hipSuccess) return FP_OK;
  return set_error(FP_EDEVICE, "%s: %s", what, hipGetErrorString(e));
}

int check_launch(const char* what) { return check_hip(hipGetLastError(), what); }

int check_ensemble(const fp_ensemble_t* e) {
  if (!e) return set_error(FP_EINVAL, "ensemble is NULL");
  if (e->ansatz < FP_BRICKWORK_HAAR || e->ansatz > FP_BRICKWORK_QUDIT)
    return set_error(FP_EINVAL, "unknown ansatz %d", e->ansatz);
  if (e->n_qubits < 2 || e->n_qubits > 64) return set_error(FP_EINVAL, "n_qubits %d outside 2..64", e->n_qubits);
  if (e->depth < 1) return set_error(FP_EINVAL, "depth %d < 1", e->depth);
  if (e->ansatz == FP_BRICKWORK_QUDIT) {
    if (e->local_dim < 3 || e->local_dim > 5)
      return set_error(FP_EINVAL, "local_dim %d outside 3..5", e->local_dim);
  } else if (e->local_dim != 0) {
    return set_error(FP_EINVAL, "local_dim must be 0 for qubit ensembles");
  }
  const bool hea = e->ansatz == FP_HEA_RYRZ_CZ || is_pauli_hea(e->ansatz);
  if (!hea && gates_per_circuit(e->ansatz, e->n_qubits, e->depth) > PLAN_MAX_GATES)
    return set_error(FP_EINVAL, "more than %d gates per circuit", PLAN_MAX_GATES);
  if (hea && e->depth > 64) return set_error(FP_EINVAL, "depth %d too large", e->depth);
  return FP_OK;
}

int check_precision(int p) {
  if (p < FP_C128 || p > FP_BF16X3) return set_error(FP_EINVAL, "unknown precision %d", p);
  return FP_OK;
}

// ---- plans of fixed-topology ensembles (host planner, cached on device) ----
struct HostPlan {
  PlanHeader hdr;
  std::vector<Op> ops;
  std::vector<int2> wg;
  std::vector<int32_t> fac;
  std::vector<int32_t> bits;  // register exponent after each column
};

static int host_plan_pair(int n, int G, const int32_t* bu, const int32_t* bv, HostPlan* out) {
  if (G > PLAN_MAX_GATES) return set_error(FP_EINVAL, "%d gates per circuit exceed %d", G, PLAN_MAX_GATES);
  std::vector<int16_t> scratch((size_t)plan_wave_scratch_elems(G));
  // bond of each position of W: V's gates in time order, then U's reversed;
  // kept in the planner's scratch as the device planner keeps it
  int16_t* bw = scratch.data() + (size_t)PLAN_BOND_SLOT * 2 * G;
  for (int i = 0; i < 2 * G; ++i) {
    const int32_t b = i < G ? bv[i] : bu[2 * G - 1 - i];
    bw[i] = (b >= 0 && b <= n - 2) ? (int16_t)b : (int16_t)-1;
  }
  out->ops.resize((size_t)plan_max_ops(G, n));
  out->wg.resize(2 * (size_t)G);
  out->fac.resize(2 * (size_t)G);
  WaveHost wh;
  out->hdr = plan_pair_wave(wh, n, G, bw, scratch.data(), out->ops.data(), out->wg.data(), out->fac.data(), nullptr);
  if (out->hdr.status != PLAN_OK) {
    if (out->hdr.status == PLAN_EWIDE)
      return set_error(FP_ETOOBIG, "boundary wider than %d bits", PLAN_MAX_BITS);
    return set_error(FP_EINVAL, "planner failed (status %d)", out->hdr.status);
  }
  out->ops.resize(out->hdr.num_ops);
  out->bits.clear();
  for (const Op& o : out->ops)
    if ((o.type & OP_TYPE_MASK) == OP_COLEND) out->bits.push_back(o.bits);
  return FP_OK;
}

static int host_plan_brickwork(int n, int depth, HostPlan* out) {
  const int G = (int)gates_per_circuit(FP_BRICKWORK_HAAR, n, depth);
  std::vector<int32_t> b(G);
  for (int g = 0; g < G; ++g) b[g] = brickwork_bond(n, g);
  return host_plan_pair(n, G, b.data(), b.data(), out);
}


static std::mutex g_plan_mu;
static std::map<std::tuple<int, int, int>, DevPlan> g_plans;  // (device, n, depth)

int get_brickwork_plan(int n, int depth, DevPlan* out) {
  int dev = 0;
  int rc = check_hip(hipGetDevice(&dev), "hipGetDevice");
  if (rc) return rc;
  std::lock_guard<std::mutex> lk(g_plan_mu);
  auto key = std::make_tuple(dev, n, depth);
  auto it = g_plans.find(key);
  if (it != g_plans.end()) {
    *out = it->second;
    return FP_OK;
  }
  HostPlan hp;
  rc = host_plan_brickwork(n, depth, &hp);
  if (rc) return rc;
  DevPlan dp;
  dp.hdr = hp.hdr;
  const size_t bo = sizeof(Op) * hp.ops.size(), bw = sizeof(int2) * hp.wg.size(), bf = sizeof(int32_t) * hp.fac.size();
  rc = check_hip(hipMalloc(&dp.ops, bo + 1), "hipMalloc(plan)");
  if (!rc) rc = check_hip(hipMalloc(&dp.wg, bw + 1), "hipMalloc(plan)");
  if (!rc) rc = check_hip(hipMalloc(&dp.fac, bf + 1), "hipMalloc(plan)");
  if (!rc) rc = check_hip(hipMalloc(&dp.dhdr, sizeof(PlanHeader)), "hipMalloc(plan)");
  if (!rc) rc = check_hip(hipMemcpy(dp.ops, hp.ops.data(), bo, hipMemcpyHostToDevice), "upload plan");
  if (!rc) rc = check_hip(hipMemcpy(dp.wg, hp.wg.data(), bw, hipMemcpyHostToDevice), "upload plan");
  if (!rc) rc = check_hip(hipMemcpy(dp.fac, hp.fac.data(), bf, hipMemcpyHostToDevice), "upload plan");
  if (!rc) rc = check_hip(hipMemcpy(dp.dhdr, &dp.hdr, sizeof(PlanHeader), hipMemcpyHostToDevice), "upload plan");
  if (rc) return rc;
  g_plans[key] = dp;
  *out = dp;
  return FP_OK;
}

// ---- auxiliary streams: the sweep classes of one batch touch disjoint pairs
// and run side by side (all streams at the default priority).  Eager calls on
// a device share one set of side streams: with the four hardware queues a
// process gets, few streams keep each caller stream on a queue of its own, so
// that a caller's wait for its side streams stalls no other caller's work
// (the sweeps of batches issued one after another on different streams seldom
// overlap, so sharing costs little).  A call under stream capture takes side
// streams of its caller's own, so that a capture never draws in another
// caller's work.  Fork and join events always belong to the caller stream. ---
struct CallerAux {
  Aux a;              // the caller's events (a.s: filled per call)
  bool own = false;   // own side streams created (capture)
  hipStream_t own_s[NUM_AUX];
};
static std::mutex g_aux_mu;
static std::map<std::pair<int, hipStream_t>, CallerAux> g_aux;
static std::map<int, Aux> g_shared;  // device -> shared side streams (s only)

static int create_streams(hipStream_t* out) {
  for (int i = 0; i < NUM_AUX; ++i) {
    int rc = check_hip(hipStreamCreateWithFlags(&out[i], hipStreamNonBlocking), "hipStreamCreate");
    if (rc) return rc;
  }
  return FP_OK;
}

int get_aux(Aux* out, hipStream_t caller) {
  int dev = 0;
  int rc = check_hip(hipGetDevice(&dev), "hipGetDevice");
  if (rc) return rc;
  hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
  bool capture = true;  // unknown: as under capture
  if (hipStreamIsCapturing(caller, &cs) == hipSuccess)
    capture = cs != hipStreamCaptureStatusNone;
  else
    (void)hipGetLastError();
  std::lock_guard<std::mutex> lk(g_aux_mu);
  const auto key = std::make_pair(dev, caller);
  auto it = g_aux.find(key);
  if (it == g_aux.end()) {
    CallerAux c;
    for (int i = 0; i < NUM_AUX; ++i) {
      rc = check_hip(hipEventCreateWithFlags(&c.a.join[i], hipEventDisableTiming), "hipEventCreate");
      if (rc) return rc;
    }
    rc = check_hip(hipEventCreateWithFlags(&c.a.fork, hipEventDisableTiming), "hipEventCreate");
    if (rc) return rc;
    it = g_aux.emplace(key, c).first;
  }
  CallerAux& c = it->second;
  if (capture) {
    if (!c.own) {
      rc = create_streams(c.own_s);
      if (rc) return rc;
      c.own = true;
    }
    for (int i = 0; i < NUM_AUX; ++i) c.a.s[i] = c.own_s[i];
  } else {
    auto sh = g_shared.find(dev);
    if (sh == g_shared.end()) {
      Aux a;
      rc = create_streams(a.s);
      if (rc) return rc;
      sh = g_shared.emplace(dev, a).first;
    }
    for (int i = 0; i < NUM_AUX; ++i) c.a.s[i] = sh->second.s[i];
  }
  *out = c.a;
  return FP_OK;
}

// ---- sizes -------------------------------------------------------------------
int lds_bits_max(int precision) { return precision == FP_C128 ? 13 : 14; }

// Local random: per-pair plan region.
struct LrLayout {
  int64_t hdr, ops, wg, fac, gseq, mat, per_pair;
};

// mat: realigned matrix of every GATE op (at most 2G), 16 complex each
static LrLayout lr_layout(int n, int G, int precision) {
  LrLayout l;
  l.hdr = 64;
  l.ops = pad64(plan_max_ops(G, n) * (int64_t)sizeof(Op));
  l.wg = pad64(2 * (int64_t)G * (int64_t)sizeof(int2));
  l.fac = pad64(2 * (int64_t)G * 4);
  l.gseq = pad64(2 * (int64_t)G * 2);
  l.mat = pad64(2 * (int64_t)G * 16 * sweep_elem_bytes(precision));
  l.per_pair = l.hdr + l.ops + l.wg + l.fac + l.gseq + l.mat;
  return l;
}

// Local random workspace: LR_CHUNKS chunk headers of LR_HEAD bytes (zeroed
// per chunk up to the set-up), then the pair order (int32 per pair), the
// per-pair plans, the work-sharing records and the HBM slots.  Chunk header:
//   +0   int max_peak, num_large, num_failed
//   +16  double class MACs[5]
//   +64  uint64 counters of the HBM launches (one per phase)
//   +128 int hist[PLAN_HIST]   pairs per peak width
//   +384 int cursor[PLAN_HIST] fill counters of the ordering pass
//   +1024 LrDev  launch set-up written on the device
constexpr int64_t LR_HEAD = 4096;
constexpr int64_t LR_DEV_OFF = 1024;
static_assert(LR_DEV_OFF + (int64_t)sizeof(LrDev) <= LR_HEAD, "set-up fits the chunk header");
constexpr int LR_CHUNKS = 4;
// Pairs per chunk at least: a chunk must fill the device by itself (planning
// and the large classes are latency-bound per pair), so only batches far
// larger than one wave of the device are split.
constexpr int64_t LR_MIN_CHUNK = 65536;

// ... one work-sharing area of the HBM-slot sweep per chunk, then its slot pool
static int64_t lr_fixed_bytes(int64_t num_pairs, const LrLayout& l) {
  return LR_CHUNKS * LR_HEAD + pad64(4 * num_pairs) + num_pairs * l.per_pair + LR_CHUNKS * HELP_AREA_BYTES;
}

constexpr int LR_SMALL_BITS = 10;  // wave per pair
constexpr int LR_MAX_OWNERS = 512;  // owner workgroups of the HBM-slot sweep at most
constexpr int LR_HELP_BITS = 18;    // owners with a task record share ops on registers from 2^18 entries
constexpr int LR_HELPERS = 256;     // workgroups that only help, at most (one per compute unit)
// helpers-only workgroups where the pairs, not the pool, limit the owners,
// once a register has 2^LR_WIDE_HELP_BITS entries: a 2^34-entry pair alone
// 80 s -> 2.5 s; at S = 100, where a rare pair reaches 2^18, they took
// compute units from the LDS sweeps (0.39 -> 0.48 ms per wavefront sweep)
constexpr int LR_WIDE_HELP_BITS = 24;
constexpr int LR_MID_BITS = 12;    // 256 lanes per pair
// HBM-slot sweep with tiled GATE runs when a batch's widest register has
// more than 2^LR_TILED_BITS entries.  Local random columns interleave BELL
// and TRACE with short runs of GATEs, and the tiled variant runs the rest of
// the kernel slower; measured at n = 50 (10^4 pairs): S = 150 and 200 (widest
// 2^22) 9 and 18 % slower with tiles, S = 250 (2^28) unchanged, S = 300
// (2^32) 36 % faster.
constexpr int LR_TILED_BITS = 22;
constexpr int64_t POOL_BUDGET = (int64_t)48 << 30;        // registers predicted up to 2^31 entries
constexpr int64_t POOL_BUDGET_DEEP = (int64_t)192 << 30;  // beyond: most of the device's 288 GB

static int64_t slot_count(int bits, int elem, int64_t large_pairs, int64_t budget = POOL_BUDGET) {
  int64_t per = hbm_slot_bytes(bits, elem);
  int64_t s = budget / per;
  if (s > 512) s = 512;
  if (s > large_pairs) s = large_pairs;
  if (s < 1) s = 1;
  return s;
}

// predicted largest boundary of a local random batch (bits), unclipped
static int lr_predicted_bits_raw(int n, int S) { return (int)(4.0 * S / (n - 1)) + 10; }
// the same, clipped to the slot width the workspace is sized in
static int lr_predicted_bits(int n, int S) {
  const int b = lr_predicted_bits_raw(n, S);
  return b > 30 ? 30 : b;
}

int workspace_bytes_impl(const fp_ensemble_t* e, int64_t num_pairs, int precision, size_t* out) {
  const int elem = sweep_elem_bytes(precision);
  if (e->ansatz == FP_HEA_RYRZ_CZ) {
    *out = 0;
    return FP_OK;
  }
  if (is_pauli_hea(e->ansatz)) {
    if (pauli_bits(e->depth) + 1 > lds_bits_max(precision))
      return set_error(FP_ETOOBIG, "Pauli HEA of %d layers: its register exceeds LDS", e->depth);
    *out = 0;
    return FP_OK;
  }
  if (e->ansatz == FP_BRICKWORK_QUDIT) {
    HostPlan hp;
    int rc = host_plan_brickwork(e->n_qubits, e->depth, &hp);
    if (rc) return rc;
    if (qudit_lds_bytes(e->local_dim, hp.hdr.peak_bits, precision) > 160 * 1024)
      return set_error(FP_ETOOBIG, "qudit boundary of %d digits (q = %d) exceeds LDS", hp.hdr.peak_bits,
                       e->local_dim);
    *out = 0;
    return FP_OK;
  }
  if (e->ansatz == FP_BRICKWORK_HAAR) {
    DevPlan dp;
    HostPlan hp;
    int rc = host_plan_brickwork(e->n_qubits, e->depth, &hp);
    if (rc) return rc;
    (void)dp;
    if (hp.hdr.peak_bits <= lds_bits_max(precision) || num_pairs == 0) {
      *out = 0;
      return FP_OK;
    }
    if (hp.hdr.peak_bits > SLOT_BITS) return set_error(FP_ETOOBIG, "boundary of %d bits", hp.hdr.peak_bits);
    int64_t slots = slot_count(hp.hdr.peak_bits, elem, num_pairs);
    *out = (size_t)(256 + slots * hbm_slot_bytes(hp.hdr.peak_bits, elem));
    return FP_OK;
  }
  const int G = e->depth;
  LrLayout l = lr_layout(e->n_qubits, G, precision);
  const int bits = lr_predicted_bits(e->n_qubits, e->depth);
  // the deep pool where registers beyond 2^31 entries are expected: wide
  // circuits (the prediction is made for them; narrow ones stay far below it)
  const bool deep = e->n_qubits >= 32 && lr_predicted_bits_raw(e->n_qubits, e->depth) > 31;
  const int64_t budget = deep ? POOL_BUDGET_DEEP : POOL_BUDGET;
  int64_t pool = 0;
  if (bits > LR_SMALL_BITS) pool = slot_count(bits, elem, num_pairs, budget) * hbm_slot_bytes(bits, elem);
  *out = (size_t)(lr_fixed_bytes(num_pairs, l) + pool);
  return FP_OK;
}

static int choose_lds_tile(int bits) {
  if (bits <= 6) return TILE_16x16;
  if (bits <= 10) return TILE_64x4;
  if (bits <= 12) return TILE_256x1;
  return TILE_1024x1;
}

// LDS bytes of one workgroup for (tile, bits) must stay within 160 KiB.
int tile_pairs(int tile) { return tile == TILE_16x16 ? 16 : tile == TILE_64x4 ? 4 : 1; }

int contract_brickwork(const fp_ensemble_t* e, int64_t num_pairs, int precision, const void* gates,
                              double* trace, void* ws, size_t ws_bytes, hipStream_t s, int64_t trace_offset) {
  DevPlan dp;
  int rc = get_brickwork_plan(e->n_qubits, e->depth, &dp);
  if (rc) return rc;
  SweepArgs a;
  memset(&a, 0, sizeof(a));
  a.gates = (const unsigned char*)gates;
  a.gate_stride = pair_bytes(e->ansatz, e->n_qubits, e->depth, precision, e->local_dim);
  a.G = (int)gates_per_circuit(e->ansatz, e->n_qubits, e->depth);
  a.ops = dp.ops;
  a.wgates = dp.wg;
  a.factors = dp.fac;
  a.hdr = dp.dhdr;
  a.trace = trace;
  a.trace_offset = trace_offset;
  a.num_pairs = num_pairs;
  a.bf3 = precision == FP_BF16X3 ? 1 : 0;
  const int peak = dp.hdr.peak_bits;
  const int elem = sweep_elem_bytes(precision);
  if (peak <= lds_bits_max(precision)) {
    int tile = choose_lds_tile(peak);
    int cap = peak < 2 ? 2 : peak;
    if ((int64_t)tile_pairs(tile) * ((int64_t)elem << cap) > 160 * 1024) tile = choose_lds_tile(peak);
    a.cap_bits = cap;
    a.min_bits = -1;
    const int kc = tile == TILE_16x16   ? KCLASS_LDS16
                   : tile == TILE_64x4  ? KCLASS_LDS64
                   : tile == TILE_256x1 ? KCLASS_LDS256
                                        : KCLASS_LDS1024;
    profile_launch_begin(kc, s);
    rc = launch_sweep_lds(a, precision, tile, s);
    profile_launch_end(kc, 8.0 * dp.hdr.macs * (double)num_pairs, s);
    return rc;
  }
  // HBM slots (registers up to 2^SLOT_BITS entries)
  if (peak > SLOT_BITS) return set_error(FP_ETOOBIG, "boundary of %d bits", peak);
  const int64_t slots = slot_count(peak, elem, num_pairs);
  const size_t need = (size_t)(256 + slots * hbm_slot_bytes(peak, elem));
  if (!ws || ws_bytes < need)
    return set_error(FP_ETOOBIG, "workspace of %zu bytes needed for %d-bit boundaries", need, peak);
  unsigned long long* counter = (unsigned long long*)ws;
  rc = check_hip(hipMemsetAsync(counter, 0, 8, s), "memset counter");
  if (rc) return rc;
  a.cap_bits = 0;
  a.min_bits = -1;
  profile_launch_begin(KCLASS_HBM, s);
  SlotArgs sl;
  int width[512];
  for (int k = 0; k < (int)slots; ++k) width[k] = peak;
  make_slot_args(&sl, (unsigned char*)ws + 256, width, (int)slots, false, elem);
  rc = launch_sweep_hbm(a, precision, counter, sl, (int)slots, s);
  profile_launch_end(KCLASS_HBM, 8.0 * dp.hdr.macs * (double)num_pairs, s);
  return rc;
}

// Launch sizes for local random batches under stream capture: the class
// sizes of the last eager batch of the same ensemble (per pair of the batch).
// The captured sweeps take their pairs through counters, so any size is
// correct; a hint keeps the launches close to the work, which lets the
// dispatcher interleave the classes as it does with one workgroup per pair.
struct LrHint {
  double frac[5];  // class sizes per pair of the batch
  int hbm_workgroups;
  int max_bits;    // widest register of the batch (log2 entries)
};
constexpr double LR_WAIT_FREE_HBM_FRAC = 0.2;  // HBM-slot share of the pairs beyond which eager batches do not wait
static std::mutex g_hint_mu;
static std::map<long long, LrHint> g_hints;

static long long hint_key(const fp_ensemble_t* e, int precision) {
  int dev = 0;
  (void)hipGetDevice(&dev);
  return ((long long)dev << 48) | ((long long)e->n_qubits << 32) | ((long long)e->depth << 4) | precision;
}

static bool capturing(hipStream_t s) {
  hipStreamCaptureStatus st = hipStreamCaptureStatusNone;
  if (hipStreamIsCapturing(s, &st) != hipSuccess) {
    (void)hipGetLastError();
    return true;  // unknown: behave as under capture
  }
  return st != hipStreamCaptureStatusNone;
}

static std::atomic<int> g_launch_mode{FP_LAUNCH_AUTO};

static LrHint hint_of(const LrDev& d, int64_t np) {
  LrHint h;
  for (int k = 0; k < 5; ++k) h.frac[k] = (double)d.range[k][1] / (double)np;
  h.hbm_workgroups = d.hbm_workgroups;
  h.max_bits = d.max_bits;
  return h;
}

// A set-up read back without waiting: a pinned copy and the event after it.
struct PendingHint {
  LrDev* host = nullptr;
  hipEvent_t done = nullptr;
  int64_t np = 0;
  bool pending = false;
};
static std::map<long long, PendingHint> g_pending;

// take_pending: take up a pending read-back (never under stream capture,
// where querying an event would invalidate the capture).
static bool lr_hint(long long key, LrHint* out, bool take_pending) {
  std::lock_guard<std::mutex> lk(g_hint_mu);
  auto p = g_pending.find(key);
  if (take_pending && p != g_pending.end() && p->second.pending && hipEventQuery(p->second.done) == hipSuccess) {
    g_hints[key] = hint_of(*p->second.host, p->second.np);
    p->second.pending = false;
  }
  auto it = g_hints.find(key);
  if (it == g_hints.end()) return false;
  *out = it->second;
  return true;
}

static void lr_hint_set(long long key, const LrDev& d, int64_t np) {
  std::lock_guard<std::mutex> lk(g_hint_mu);
  g_hints[key] = hint_of(d, np);
  auto p = g_pending.find(key);
  if (p != g_pending.end()) p->second.pending = false;  // superseded
}

// Queue the copy of a batch's set-up on s; the next lr_hint of the key takes
// it up once it has landed.  A copy still in flight from an earlier batch
// is left to finish and this one is skipped.
static int lr_hint_post(long long key, const LrDev* dev, int64_t np, hipStream_t s) {
  std::lock_guard<std::mutex> lk(g_hint_mu);
  PendingHint& p = g_pending[key];
  if (!p.host) {
    if (hipHostMalloc((void**)&p.host, sizeof(LrDev), hipHostMallocDefault) != hipSuccess) {
      p.host = nullptr;
      (void)hipGetLastError();
      return FP_OK;  // no refresh; the hint stays as it was
    }
    if (hipEventCreateWithFlags(&p.done, hipEventDisableTiming) != hipSuccess) {
      (void)hipGetLastError();
      (void)hipHostFree(p.host);
      p.host = nullptr;
      return FP_OK;
    }
  }
  if (p.pending && hipEventQuery(p.done) != hipSuccess) {
    (void)hipGetLastError();
    return FP_OK;
  }
  int rc = check_hip(hipMemcpyAsync(p.host, dev, sizeof(LrDev), hipMemcpyDeviceToHost, s), "copy set-up (hint)");
  if (!rc) rc = check_hip(hipEventRecord(p.done, s), "hint event");
  p.np = np;
  p.pending = rc == FP_OK;
  return rc;
}

// One chunk of a local random batch: plan its pairs (on s), derive its
// launches on the device, order the pairs by peak width, and launch the
// sweep classes, most on side streams that s does not wait for here, so the
// next chunk's planning overlaps this chunk's sweep.
struct LrCtx {
  const fp_ensemble_t* e;
  int precision, elem;
  LrLayout l;
  const unsigned char* gates;
  int64_t gate_stride, bonds_off;
  double* trace;
  int64_t trace_offset;
  unsigned char* w;      // workspace
  size_t ws_bytes, fixed_bytes;
  int64_t num_pairs;     // whole batch
  Aux aux;
  bool used[NUM_AUX];
  long long key;  // grid hints
  int hbm_slot;   // eager: stream of the HBM class (-2: none yet); all chunks share one slot pool
};

static int lr_chunk(LrCtx& c, int chunk, int64_t p0, int64_t np, hipStream_t s) {
  const int n = c.e->n_qubits, G = c.e->depth;
  unsigned char* hw = c.w + (int64_t)chunk * LR_HEAD;
  int* counters = (int*)hw;
  unsigned long long* hbm_counter = (unsigned long long*)(hw + 64);
  int* hist = (int*)(hw + 128);
  int* cursor = (int*)(hw + 128 + 4 * PLAN_HIST);
  int32_t* order = (int32_t*)(c.w + LR_CHUNKS * LR_HEAD) + p0;
  unsigned char* base = c.w + LR_CHUNKS * LR_HEAD + pad64(4 * c.num_pairs);
  const LrLayout& l = c.l;
  PlanJob j;
  memset(&j, 0, sizeof(j));
  j.gates = c.gates + p0 * c.gate_stride;
  j.gate_stride = c.gate_stride;
  j.bonds_off = c.bonds_off;
  j.n = n;
  j.G = G;
  j.num_pairs = np;
  j.hdr = (PlanHeader*)base + p0;
  j.ops = (Op*)(base + c.num_pairs * l.hdr) + p0 * (l.ops / (int64_t)sizeof(Op));
  j.wgates = (int2*)(base + c.num_pairs * (l.hdr + l.ops)) + p0 * (l.wg / (int64_t)sizeof(int2));
  j.factors = (int32_t*)(base + c.num_pairs * (l.hdr + l.ops + l.wg)) + p0 * (l.fac / 4);
  j.ops_stride = l.ops / (int64_t)sizeof(Op);
  j.wg_stride = l.wg / (int64_t)sizeof(int2);
  j.f_stride = l.fac / 4;
  j.max_peak = counters;
  j.num_large = counters + 1;
  j.num_failed = counters + 2;
  // registers up to 2^12 entries: the LDS sweeps; wider: the HBM-slot sweep,
  // whose interpreter keeps a register in LDS up to 2^14 (c64) entries and
  // runs such pairs several times faster than 1024 lanes of the LDS sweep
  j.cap_bits = LR_MID_BITS < lds_bits_max(c.precision) ? LR_MID_BITS : lds_bits_max(c.precision);
  j.small_bits = LR_SMALL_BITS < j.cap_bits ? LR_SMALL_BITS : j.cap_bits;
  j.tiny_bits = -1;  // registers up to 2^10 entries form one class (one wavefront per pair)
  j.mid_bits = LR_MID_BITS < j.cap_bits ? LR_MID_BITS : j.cap_bits;
  j.class_macs = (double*)(hw + 16);
  j.hist = hist;
  j.gseq = (int16_t*)(base + c.num_pairs * (l.hdr + l.ops + l.wg + l.fac)) + p0 * (l.gseq / 2);
  j.gseq_stride = l.gseq / 2;
  j.wmat = base + c.num_pairs * (l.hdr + l.ops + l.wg + l.fac + l.gseq) + p0 * l.mat;
  j.wmat_stride = l.mat;
  j.bf3 = c.precision == FP_BF16X3 ? 1 : 0;
  static_assert(sizeof(PlanHeader) <= 64, "plan header fits its slot");
  LrDev* dev = (LrDev*)(hw + LR_DEV_OFF);
  int rc = launch_zero_words(hw, LR_DEV_OFF / 4, s);  // counters, histogram, cursors (the set-up writes dev)
  if (rc) return rc;
  // algorithmic bytes: the planner reads the bond lists and writes the plans;
  // the preparation reads the gate buffer and writes one matrix per GATE op
  const double gate_bytes = (double)np * (double)c.gate_stride;
  profile_launch_begin(KCLASS_PLAN, s);
  rc = launch_plan_local_random(j, c.precision, s);
  profile_launch_end(KCLASS_PLAN, 0.0, s, (double)np * (8.0 * G + (double)(l.hdr + l.ops + l.wg + l.fac + l.gseq)));
  if (rc) return rc;
  profile_launch_begin(KCLASS_PREP, s);
  rc = launch_gate_matrices(j, c.precision, s);
  profile_launch_end(KCLASS_PREP, 0.0, s, gate_bytes + (double)np * (double)l.mat);
  if (rc) return rc;
  // Launches derived on the device from the planner's width histogram.  A
  // pair that cannot be contracted (a failed plan, a register beyond 2^31
  // entries, no room in the pool) gets a NaN trace.
  unsigned char* help_area = c.w + c.fixed_bytes - (LR_CHUNKS - chunk) * HELP_AREA_BYTES;
  LrSetupJob sj;
  memset(&sj, 0, sizeof(sj));
  sj.hist = hist;
  sj.tiny_bits = j.tiny_bits;
  sj.small_bits = j.small_bits;
  sj.mid_bits = j.mid_bits;
  sj.cap_bits = j.cap_bits;
  sj.lds_bits = c.precision == FP_C128 ? 13 : 14;  // registers the HBM-slot sweep keeps in LDS
  sj.pool = c.w + c.fixed_bytes;
  sj.pool_bytes = (long long)c.ws_bytes - (long long)c.fixed_bytes;
  sj.elem_shift = c.elem == 16 ? 4 : 3;
  sj.max_owners = LR_MAX_OWNERS;
  sj.max_helpers = LR_HELPERS;
  sj.num_cus = device_cus();
  sj.help_bits = LR_HELP_BITS;
  sj.wide_bits = LR_WIDE_HELP_BITS;
  sj.recs = (HelpRec*)help_area;
  sj.hbm_counter = hbm_counter;
  sj.dev = dev;
  rc = launch_lr_setup(sj, s);
  if (rc) return rc;
  // Order the pairs by decreasing peak width, so that every class below is
  // one contiguous range of the order and each class takes its costliest
  // pairs first.
  OrderJob oj;
  memset(&oj, 0, sizeof(oj));
  oj.hdr = j.hdr;
  oj.hdr_stride = l.hdr / (int64_t)sizeof(PlanHeader);
  oj.num_pairs = np;
  oj.cursor = cursor;
  oj.order = order;
  oj.trace = c.trace;
  oj.trace_offset = c.trace_offset + p0;
  oj.first = dev->first;
  rc = launch_order_pairs(oj, s);
  if (rc) return rc;
  SweepArgs a;
  memset(&a, 0, sizeof(a));
  a.gates = j.gates;
  a.gate_stride = j.gate_stride;
  a.G = G;
  a.ops = j.ops;
  a.ops_stride = j.ops_stride;
  a.wgates = j.wgates;
  a.wg_stride = j.wg_stride;
  a.factors = j.factors;
  a.f_stride = j.f_stride;
  a.hdr = j.hdr;
  a.hdr_stride = oj.hdr_stride;
  a.trace = c.trace;
  a.trace_offset = c.trace_offset + p0;
  a.wmat = j.wmat;
  a.wmat_stride = j.wmat_stride;
  a.bf3 = j.bf3;
  a.order = order;
  a.num_pairs = np;  // upper bound; each class takes its range from the set-up
  int64_t dev_first[5] = {0, 0, 0, 0, 0};  // class starts in the order, when read back
  // Classes by the largest register of a pair: up to 2^10 entries with one
  // wavefront per pair (class 0 stays empty: the VGPRs of the wavefront
  // sweep, not its LDS, bound its occupancy, so one class serves all small
  // registers), up to 2^12 and 2^14 with 256 and 1024 lanes per pair
  // (boundary in LDS), then HBM slots, each class on its own stream.
  struct Cls {
    int lo, hi, tile, kclass;
  };
  const Cls cls[5] = {{-1, j.tiny_bits, TILE_16x16, KCLASS_LDS16},
                      {j.tiny_bits, j.small_bits, TILE_64x4, KCLASS_LDS64},
                      {j.small_bits, j.mid_bits, TILE_256x1, KCLASS_LDS256},
                      {j.mid_bits, j.cap_bits, TILE_1024x1, KCLASS_LDS1024},
                      {j.cap_bits, PLAN_HIST - 1, 0, KCLASS_HBM}};
  rc = check_hip(hipEventRecord(c.aux.fork, s), "fork");
  if (rc) return rc;
  bool waited[NUM_AUX] = {false, false, false};
  auto side = [&](int ai, hipStream_t* out) -> int {
    if (ai < 0) {
      *out = s;
      return FP_OK;
    }
    if (!waited[ai]) {
      int r = check_hip(hipStreamWaitEvent(c.aux.s[ai], c.aux.fork, 0), "fork wait");
      if (r) return r;
      waited[ai] = true;
    }
    c.used[ai] = true;
    *out = c.aux.s[ai];
    return FP_OK;
  };
  // The HBM-slot sweep runs with 64-bit entry indices when a register may
  // exceed 2^31 entries: known exactly once the set-up is read back, else
  // from the last batch of the ensemble or, for the first, from the depth.
  bool wide_hbm = n >= 32 && lr_predicted_bits_raw(n, G) > 27;
  // and with the tiled runs of GATEs for the widest batches (both variants
  // give the same results)
  bool tiled_hbm = lr_predicted_bits_raw(n, G) > LR_TILED_BITS;
  // flops < 0: the class's MAC count is read from the device afterwards
  // phase: the HBM class's launch (k = 4 only)
  auto launch_class = [&](int k, int ai, const long long* range, int64_t count, int64_t grid_pairs,
                          double flops, int phase = 0) -> int {
    hipStream_t sx;
    int r = side(ai, &sx);
    if (r) return r;
    SweepArgs ax = a;
    ax.min_bits = cls[k].lo;
    ax.cap_bits = cls[k].hi;
    if (k == 4) {
      // the HBM sweep contracts the pairs beyond the LDS capacity, and takes
      // its range (and slots) from the set-up itself: order base, no offset
      ax.cap_bits = j.cap_bits;
    } else if (range != nullptr) {  // pairs taken from the device range
      ax.range = range;
      ax.claim = &dev->claim[k];
      ax.grid_pairs = grid_pairs;
    } else {  // the class's pairs at a known place: one launch slot per pair
      ax.order = order + dev_first[k];
      ax.num_pairs = count;
    }
    profile_launch_begin(cls[k].kclass, sx);
    if (k == 4)
      r = launch_sweep_hbm_dev(ax, c.precision, hbm_counter + phase, dev, phase, (int)grid_pairs, sx, wide_hbm,
                               tiled_hbm);
    else  // up to 2^10 entries: one wavefront per pair; larger: the LDS sweep
      r = cls[k].hi <= 10 ? launch_sweep_wave(ax, c.precision, cls[k].hi, sx)
                          : launch_sweep_lds(ax, c.precision, cls[k].tile, sx);
    if (flops < 0.0)
      profile_launch_end_dev(cls[k].kclass, j.class_macs + k, sx);
    else
      profile_launch_end(cls[k].kclass, flops, sx);
    return r;
  };
  // An eager batch also goes without waiting when the previous eager batch
  // of the ensemble had a fifth of its pairs or more in the HBM-slot class: there the
  // sweeps, not the planner, set the pace, and not waiting lets the next
  // batch's planner run beside them (S = 200: 1.9 -> 2.4 x 10^5
  // contractions/s; at S = 100 waiting is faster, 1.19 against 1.36 ms).
  LrHint hint;
  const bool captured = capturing(s);
  const bool hinted = lr_hint(c.key, &hint, !captured);
  const int mode = g_launch_mode.load();
  const bool wait_free = captured || mode == FP_LAUNCH_WAIT_FREE ||
                         (mode == FP_LAUNCH_AUTO && hinted && hint.frac[4] > LR_WAIT_FREE_HBM_FRAC);
  if (!wait_free) {
    // Eager: read the set-up back (one wait for the plans, as the launch
    // sizes depend on them), then launch every class at its exact size, the
    // costliest by planned MACs on s and the HBM class on the same stream in
    // every chunk (the chunks share its slot pool); launched widest class
    // first, so their long pairs start first.
    struct {
      LrDev d;
      double macs[5];
    } h;
    rc = check_hip(hipMemcpyAsync(&h.d, dev, sizeof(LrDev), hipMemcpyDeviceToHost, s), "copy set-up");
    if (!rc) rc = check_hip(hipMemcpyAsync(h.macs, j.class_macs, sizeof(h.macs), hipMemcpyDeviceToHost, s), "copy MACs");
    if (!rc) rc = check_hip(hipStreamSynchronize(s), "sync(plan)");
    if (rc) return rc;
    lr_hint_set(c.key, h.d, np);
    for (int k = 0; k < 5; ++k) dev_first[k] = h.d.range[k][0];
    int slot_of[5] = {-1, -1, -1, -1, -1};  // -1: s; 0..2: side streams
    int act[5], na = 0;
    for (int k = 0; k < 5; ++k)
      if (h.d.range[k][1] > 0) act[na++] = k;
    for (int x = 1; x < na; ++x)  // by MACs, heaviest first
      for (int y = x; y > 0 && h.macs[act[y]] > h.macs[act[y - 1]]; --y) {
        const int t = act[y];
        act[y] = act[y - 1];
        act[y - 1] = t;
      }
    for (int x = 0; x < na; ++x) slot_of[act[x]] = x < 4 ? x - 1 : slot_of[act[3]];
    if (h.d.range[4][1] > 0) {
      if (c.hbm_slot == -2) c.hbm_slot = slot_of[4];
      slot_of[4] = c.hbm_slot;
    }
    for (int k = 4; k >= 1; --k) {
      const int64_t count = h.d.range[k][1];
      if (count <= 0) continue;
      if (k == 4) {  // its launches in order on one stream, each with the whole slot pool
        for (int ph = 0; ph < HBM_PHASES && !rc; ++ph) {
          if (h.d.ph[ph].count <= 0) continue;
          wide_hbm = h.d.ph[ph].max_bits > 31;
          tiled_hbm = h.d.ph[ph].max_bits > LR_TILED_BITS;
          rc = launch_class(4, slot_of[4], nullptr, count, h.d.ph[ph].workgroups, ph == 0 ? 8.0 * h.macs[4] : 0.0,
                            ph);
        }
      } else {
        rc = launch_class(k, slot_of[k], nullptr, count, 0, 8.0 * h.macs[k]);
      }
      if (rc) return rc;
    }
    return FP_OK;
  }
  // Under stream capture (or as above): no waiting.  Every class takes its pairs from the
  // device range through a counter, so any launch size is correct; the sizes
  // come from the last eager batch of the ensemble when there was one (else
  // as many workgroups as stay resident).  The HBM class goes on s, whose
  // order needs no cross-stream wait, so its long pairs start first.
  int grid = LR_MAX_OWNERS + LR_HELPERS;
  if (hinted) wide_hbm = hint.max_bits > 31 || wide_hbm;
  if (hinted) tiled_hbm = hint.max_bits > LR_TILED_BITS;
  if (hinted) {
    const int want = hint.hbm_workgroups + hint.hbm_workgroups / 8 + 4;
    grid = want < grid ? want : grid;
  }
  // the HBM class's launches: the second (narrower pairs, when the set-up
  // split the class) never needs 64-bit indices
  rc = launch_class(4, -1, dev->range[4], 0, grid, -1.0, 0);
  wide_hbm = false;
  if (!rc) rc = launch_class(4, -1, dev->range[4], 0, grid, 0.0, 1);
  for (int k = 3; k >= 1 && !rc; --k) {
    if (cls[k].hi <= cls[k].lo) continue;
    const int64_t gp = hinted ? (int64_t)(hint.frac[k] * 1.05 * (double)np) + 2 : 0;
    rc = launch_class(k, k == 1 ? 2 : k - 2, dev->range[k], 0, gp, -1.0);
  }
  // An uncaptured batch refreshes the hint from its own set-up, read back
  // without a wait and taken up by the next batch of the ensemble.
  if (!rc && !captured) rc = lr_hint_post(c.key, dev, np, s);
  return rc;
}

int contract_local_random(const fp_ensemble_t* e, int64_t num_pairs, int precision, const void* gates,
                          double* trace, void* ws, size_t ws_bytes, hipStream_t s, int64_t trace_offset) {
  LrCtx c;
  c.e = e;
  c.precision = precision;
  c.elem = sweep_elem_bytes(precision);
  c.l = lr_layout(e->n_qubits, e->depth, precision);
  c.gates = (const unsigned char*)gates;
  c.gate_stride = pair_bytes(e->ansatz, e->n_qubits, e->depth, precision, e->local_dim);
  c.bonds_off = bonds_offset(e->n_qubits, e->depth, precision);
  c.trace = trace;
  c.trace_offset = trace_offset;
  c.w = (unsigned char*)ws;
  c.ws_bytes = ws_bytes;
  c.fixed_bytes = (size_t)lr_fixed_bytes(num_pairs, c.l);
  c.num_pairs = num_pairs;
  for (int i = 0; i < NUM_AUX; ++i) c.used[i] = false;
  c.key = hint_key(e, precision);
  c.hbm_slot = -2;
  if (!ws || ws_bytes < c.fixed_bytes)
    return set_error(FP_ETOOBIG, "workspace of %zu bytes needed for the plans", c.fixed_bytes);
  int rc = get_aux(&c.aux, s);
  if (rc) return rc;
  int64_t chunks = num_pairs / LR_MIN_CHUNK;
  if (chunks < 1) chunks = 1;
  if (chunks > LR_CHUNKS) chunks = LR_CHUNKS;
  const int64_t per = (num_pairs + chunks - 1) / chunks;
  for (int k = 0; k < chunks && !rc; ++k) {
    const int64_t p0 = k * per;
    const int64_t np = num_pairs - p0 < per ? num_pairs - p0 : per;
    if (np > 0) rc = lr_chunk(c, k, p0, np, s);
  }
  // join every side stream that took work, also after an error
  for (int i = 0; i < NUM_AUX; ++i) {
    if (!c.used[i]) continue;
    int r = check_hip(hipEventRecord(c.aux.join[i], c.aux.s[i]), "join");
    if (!r) r = check_hip(hipStreamWaitEvent(s, c.aux.join[i], 0), "join wait");
    if (!rc) rc = r;
  }
  return rc;
}

// Algorithmic flops of one HEA trace: n-1 transforms of m butterfly stages
// (one complex addition, 2 flops, per entry and stage) and n pointwise
// complex products (6 flops per entry).
double hea_flops_per_pair(int n, int L) {
  const int m = hea_bits(L);
  if (m == 0) return 6.0 * n;
  const double chi = (double)(1ull << m);
  return (double)(n - 1) * m * chi * 2.0 + (double)n * chi * 6.0;
}

int contract_hea(const fp_ensemble_t* e, int64_t num_pairs, int precision, const void* gates, double* trace,
                        hipStream_t s, int64_t trace_offset) {
  HeaArgs a;
  a.gates = (const unsigned char*)gates;
  a.gate_stride = pair_bytes(e->ansatz, e->n_qubits, e->depth, precision, e->local_dim);
  a.n = e->n_qubits;
  a.L = e->depth;
  a.trace = trace;
  a.trace_offset = trace_offset;
  a.num_pairs = num_pairs;
  a.bf3 = precision == FP_BF16X3 ? 1 : 0;
  const int m = hea_bits(e->depth);
  if (m > lds_bits_max(precision)) return set_error(FP_ETOOBIG, "HEA boundary of %d bits exceeds LDS", m);
  const int tile = m <= 6 ? TILE_16x16 : m <= 10 ? TILE_64x4 : m <= 12 ? TILE_256x1 : TILE_1024x1;
  profile_launch_begin(KCLASS_HEA, s);
  int rc = launch_hea(a, precision, tile, s);
  profile_launch_end(KCLASS_HEA, hea_flops_per_pair(e->n_qubits, e->depth) * (double)num_pairs, s);
  return rc;
}

int contract_pauli_hea(const fp_ensemble_t* e, int64_t num_pairs, int precision, const void* gates, double* trace,
                       hipStream_t s, int64_t trace_offset) {
  size_t ws = 0;
  int rc = workspace_bytes_impl(e, num_pairs, precision, &ws);
  if (rc) return rc;
  HeaArgs a;
  a.gates = (const unsigned char*)gates;
  a.gate_stride = pair_bytes(e->ansatz, e->n_qubits, e->depth, precision, e->local_dim);
  a.n = e->n_qubits;
  a.L = e->depth;
  a.trace = trace;
  a.trace_offset = trace_offset;
  a.num_pairs = num_pairs;
  a.bf3 = precision == FP_BF16X3 ? 1 : 0;
  profile_launch_begin(KCLASS_HEA, s);
  rc = launch_pauli_hea(a, precision, e->ansatz == FP_HEA_PAULI_CNOT ? 1 : 0, s);
  profile_launch_end(KCLASS_HEA, pauli_flops_per_pair(e->n_qubits, e->depth) * (double)num_pairs, s);
  return rc;
}

// Complex multiply-adds of the GATE ops of a qudit brickwork pair: a GATE on a
// register of b digits updates q^(b-2) groups with a q^2 x q^2 matrix.
static double qudit_macs(const HostPlan& hp, int q) {
  double m = 0.0;
  for (const Op& o : hp.ops)
    if ((o.type & OP_TYPE_MASK) == OP_GATE) m += pow((double)q, (double)o.bits + 2.0);
  return m;
}

int contract_qudit(const fp_ensemble_t* e, int64_t num_pairs, int precision, const void* gates, double* trace,
                   hipStream_t s, int64_t trace_offset) {
  DevPlan dp;
  int rc = get_brickwork_plan(e->n_qubits, e->depth, &dp);
  if (rc) return rc;
  double macs = 0.0;
  if (profiling()) {
    HostPlan hp;
    if ((rc = host_plan_brickwork(e->n_qubits, e->depth, &hp))) return rc;
    macs = qudit_macs(hp, e->local_dim);
  }
  profile_launch_begin(KCLASS_LDS256, s);
  rc = launch_qudit(e, num_pairs, precision, gates, trace, dp, s, trace_offset);
  profile_launch_end(KCLASS_LDS256, 8.0 * macs * (double)num_pairs, s);
  return rc;
}

int contract_dispatch(const fp_ensemble_t* e, int64_t num_pairs, int precision, const void* gates, double* trace,
                      void* ws, size_t ws_bytes, hipStream_t s, int64_t trace_offset) {
  if (e->ansatz == FP_BRICKWORK_QUDIT) return contract_qudit(e, num_pairs, precision, gates, trace, s, trace_offset);
  if (is_pauli_hea(e->ansatz)) return contract_pauli_hea(e, num_pairs, precision, gates, trace, s, trace_offset);
  if (e->ansatz == FP_BRICKWORK_HAAR)
    return contract_brickwork(e, num_pairs, precision, gates, trace, ws, ws_bytes, s, trace_offset);
  if (e->ansatz == FP_LOCAL_RANDOM_HAAR)
    return contract_local_random(e, num_pairs, precision, gates, trace, ws, ws_bytes, s, trace_offset);
  return contract_hea(e, num_pairs, precision, gates, trace, s, trace_offset);
}

}  // namespace fp

using namespace fp;

extern "C" {

const char* fp_last_error(void) { return g_err; }
int fp_version(void) { return 1; }

size_t fp_gate_bytes_per_pair(const fp_ensemble_t* ens, int precision) {
  if (check_ensemble(ens) || check_precision(precision)) return 0;
  return (size_t)pair_bytes(ens->ansatz, ens->n_qubits, ens->depth, precision, ens->local_dim);
}

int fp_sample_gates(const fp_ensemble_t* ens, int64_t num_pairs, uint64_t seed, uint64_t first_pair, int precision,
                    void* d_gates, size_t gates_bytes, void* stream) {
  int rc = check_ensemble(ens);
  if (rc) return rc;
  if ((rc = check_precision(precision))) return rc;
  if (num_pairs < 0) return set_error(FP_EINVAL, "num_pairs < 0");
  if (num_pairs == 0) return FP_OK;
  if (!d_gates) return set_error(FP_EINVAL, "d_gates is NULL");
  const int64_t need = num_pairs * pair_bytes(ens->ansatz, ens->n_qubits, ens->depth, precision, ens->local_dim);
  if ((int64_t)gates_bytes < need) return set_error(FP_EINVAL, "gates_bytes %zu < %lld", gates_bytes, (long long)need);
  if (first_pair + (uint64_t)num_pairs > (1ull << 62)) return set_error(FP_EINVAL, "pair index beyond 2^62");
  profile_launch_begin(KCLASS_SAMPLE, (hipStream_t)stream);
  rc = launch_sample(ens, num_pairs, seed, first_pair, precision, d_gates, (hipStream_t)stream);
  profile_launch_end(KCLASS_SAMPLE, 0.0, (hipStream_t)stream, (double)need);
  return rc;
}

int fp_workspace_bytes(const fp_ensemble_t* ens, int64_t num_pairs, int precision, size_t* out_bytes) {
  int rc = check_ensemble(ens);
  if (rc) return rc;
  if ((rc = check_precision(precision))) return rc;
  if (!out_bytes) return set_error(FP_EINVAL, "out_bytes is NULL");
  if (num_pairs < 0) return set_error(FP_EINVAL, "num_pairs < 0");
  return workspace_bytes_impl(ens, num_pairs, precision, out_bytes);
}

int fp_contract_trace_batch(const fp_ensemble_t* ens, int64_t num_pairs, int precision, const void* d_gates,
                            double* d_trace, void* d_workspace, size_t workspace_bytes, void* stream) {
  int rc = check_ensemble(ens);
  if (rc) return rc;
  if ((rc = check_precision(precision))) return rc;
  if (num_pairs < 0) return set_error(FP_EINVAL, "num_pairs < 0");
  if (num_pairs == 0) return FP_OK;
  if (!d_gates || !d_trace) return set_error(FP_EINVAL, "NULL gates or trace buffer");
  return contract_dispatch(ens, num_pairs, precision, d_gates, d_trace, d_workspace, workspace_bytes,
                           (hipStream_t)stream, 0);
}

int fp_set_launch_mode(int mode) {
  if (mode != FP_LAUNCH_AUTO && mode != FP_LAUNCH_WAIT && mode != FP_LAUNCH_WAIT_FREE)
    return set_error(FP_EINVAL, "unknown launch mode %d", mode);
  g_launch_mode.store(mode);
  return FP_OK;
}

int fp_frame_potential(const double* d_trace, int64_t num_pairs, int k_max, double* h_F, double* h_stderr,
                       void* stream) {
  if (!d_trace || !h_F) return set_error(FP_EINVAL, "NULL trace or output");
  if (num_pairs < 1) return set_error(FP_EINVAL, "num_pairs must be >= 1");
  if (k_max < 1 || k_max > 8) return set_error(FP_EINVAL, "k_max %d outside 1..8", k_max);
  return run_frame_potential(d_trace, num_pairs, k_max, h_F, h_stderr, (hipStream_t)stream);
}

int fp_frame_potential_noalloc(const double* d_trace, int64_t num_pairs, int k_max, double* h_F, double* h_stderr,
                               void* stream) {
  if (!d_trace || !h_F) return set_error(FP_EINVAL, "NULL trace or output");
  if (num_pairs < 1) return set_error(FP_EINVAL, "num_pairs must be >= 1");
  if (k_max < 1 || k_max > 8) return set_error(FP_EINVAL, "k_max %d outside 1..8", k_max);
  return run_frame_potential_noalloc(d_trace, num_pairs, k_max, h_F, h_stderr, (hipStream_t)stream);
}

int fp_frame_potential_cv(const double* d_trace_B, const float* d_g_B, int64_t nB, const float* d_g_C, int64_t nC,
                          int k, double c, double* h_F, double* h_stderr, void* stream) {
  if (!d_trace_B || !d_g_B || !h_F) return set_error(FP_EINVAL, "NULL argument");
  if (nB < 1) return set_error(FP_EINVAL, "nB must be >= 1");
  if (nC < 0 || (nC > 0 && !d_g_C)) return set_error(FP_EINVAL, "bad surrogate set");
  if (nC == 0 && c != 0.0) return set_error(FP_EINVAL, "c != 0 needs surrogate values");
  if (k < 1 || k > 8) return set_error(FP_EINVAL, "k %d outside 1..8", k);
  return run_frame_potential_cv(d_trace_B, d_g_B, nB, d_g_C, nC, k, c, h_F, h_stderr, (hipStream_t)stream);
}

int fp_mlp_targets(const double* d_trace, int64_t num_pairs, int k, double scale, float* d_t, void* stream) {
  if (!d_trace || !d_t) return set_error(FP_EINVAL, "NULL buffer");
  if (num_pairs < 0 || k < 1 || k > 8) return set_error(FP_EINVAL, "bad arguments");
  if (num_pairs == 0) return FP_OK;
  return run_targets(d_trace, num_pairs, k, scale, d_t, (hipStream_t)stream);
}

int fp_log_moments(const double* d_trace, int64_t num_pairs, double eps, double* h_mean, double* h_std,
                   void* stream) {
  if (!d_trace || !h_mean || !h_std || num_pairs < 2 || !(eps >= 0.0)) return set_error(FP_EINVAL, "bad arguments");
  return run_log_moments(d_trace, num_pairs, eps, h_mean, h_std, (hipStream_t)stream);
}

int fp_mlp_log_targets(const double* d_trace, int64_t num_pairs, double eps, double mean, double std_dev, float* d_t,
                       void* stream) {
  if (!d_trace || !d_t || num_pairs < 0 || !(eps >= 0.0)) return set_error(FP_EINVAL, "bad arguments");
  if (num_pairs == 0) return FP_OK;
  return run_log_targets(d_trace, num_pairs, eps, mean, std_dev, d_t, (hipStream_t)stream);
}

int fp_mlp_link(const float* d_y, int64_t n, int k, double mean, double std_dev, double shift, float* d_g,
                void* stream) {
  if (!d_y || !d_g || n < 0 || k < 1 || k > 8) return set_error(FP_EINVAL, "bad arguments");
  if (n == 0) return FP_OK;
  return run_link(d_y, n, k, mean, std_dev, shift, d_g, (hipStream_t)stream);
}

int fp_cv_coefficient(const double* d_trace, const float* d_g, int64_t num_pairs, int k, double* h_c, void* stream) {
  if (!d_trace || !d_g || !h_c) return set_error(FP_EINVAL, "NULL argument");
  if (num_pairs < 2 || k < 1 || k > 8) return set_error(FP_EINVAL, "bad arguments");
  return run_cv_coefficient(d_trace, d_g, num_pairs, k, h_c, (hipStream_t)stream);
}

int fp_plan_info(const fp_ensemble_t* ens, int32_t* out_bits, int32_t* peak_bits, double* macs, int64_t* ops) {
  int rc = check_ensemble(ens);
  if (rc) return rc;
  const int n = ens->n_qubits;
  if (ens->ansatz == FP_LOCAL_RANDOM_HAAR)
    return set_error(FP_ENOTIMPL, "local random ensembles are planned per pair");
  if (is_pauli_hea(ens->ansatz)) {
    const int m = pauli_bits(ens->depth);
    if (out_bits)
      for (int j = 0; j < n - 1; ++j) out_bits[j] = m;
    if (peak_bits) *peak_bits = m == 0 ? 0 : m + 1;  // the register adds the wire's bit
    // complex multiply-adds of the rotations (two per register entry and slot)
    if (macs) *macs = m == 0 ? (double)n : (double)n * m * 2.0 * (double)(2ull << m);
    if (ops) *ops = (int64_t)n * m;
    return FP_OK;
  }
  if (ens->ansatz == FP_HEA_RYRZ_CZ) {
    const int m = hea_bits(ens->depth);
    if (out_bits)
      for (int j = 0; j < n - 1; ++j) out_bits[j] = m;
    if (peak_bits) *peak_bits = m;
    // complex additions of the transforms + products with f_q, per pair
    if (macs) *macs = (double)(n - 1) * m * (double)(1ull << m) + (double)n * (double)(1ull << m);
    if (ops) *ops = n;
    return FP_OK;
  }
  HostPlan hp;
  rc = host_plan_brickwork(n, ens->depth, &hp);
  if (rc) return rc;
  if (out_bits)
    for (int j = 0; j < n - 1 && j < (int)hp.bits.size(); ++j) out_bits[j] = hp.bits[j];
  if (peak_bits) *peak_bits = hp.hdr.peak_bits;
  if (macs) *macs = ens->ansatz == FP_BRICKWORK_QUDIT ? qudit_macs(hp, ens->local_dim) : hp.hdr.macs;
  if (ops) *ops = hp.hdr.num_ops;
  return FP_OK;
}

int fp_plan_local_random_host(int n_qubits, int steps, const int32_t* bonds_u, const int32_t* bonds_v,
                              int32_t* out_bits, int32_t* peak_bits, double* macs, int64_t* ops) {
  if (n_qubits < 2 || n_qubits > 64 || steps < 1 || !bonds_u || !bonds_v)
    return set_error(FP_EINVAL, "bad arguments");
  HostPlan hp;
  int rc = host_plan_pair(n_qubits, steps, bonds_u, bonds_v, &hp);
  if (rc) return rc;
  if (out_bits)
    for (int j = 0; j < n_qubits - 1 && j < (int)hp.bits.size(); ++j) out_bits[j] = hp.bits[j];
  if (peak_bits) *peak_bits = hp.hdr.peak_bits;
  if (macs) *macs = hp.hdr.macs;
  if (ops) *ops = hp.hdr.num_ops;
  return FP_OK;
}

int fp_plan_program_host(int n_qubits, int steps, const int32_t* bonds_u, const int32_t* bonds_v, void* ops,
                         int64_t max_ops, int32_t* wgates, int32_t* factors, int64_t* num_ops, int32_t* log2_factor) {
  if (n_qubits < 2 || n_qubits > 64 || steps < 1 || !bonds_u || !bonds_v || !ops || !wgates || !factors)
    return set_error(FP_EINVAL, "bad arguments");
  HostPlan hp;
  int rc = host_plan_pair(n_qubits, steps, bonds_u, bonds_v, &hp);
  if (rc) return rc;
  if ((int64_t)hp.ops.size() > max_ops) return set_error(FP_EINVAL, "max_ops %lld < %zu", (long long)max_ops, hp.ops.size());
  memcpy(ops, hp.ops.data(), hp.ops.size() * sizeof(Op));
  for (int k = 0; k < hp.hdr.num_wgates; ++k) {
    wgates[2 * k] = hp.wg[k].x;
    wgates[2 * k + 1] = hp.wg[k].y;
  }
  memcpy(factors, hp.fac.data(), sizeof(int32_t) * hp.hdr.num_factors);
  if (num_ops) *num_ops = (int64_t)hp.ops.size();
  if (log2_factor) *log2_factor = hp.hdr.log2_factor;
  return FP_OK;
}

}  // extern "C"
