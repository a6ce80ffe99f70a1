// Launch descriptors shared between the sweep kernels and the host API.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "plan.h"

namespace fp {

// Tile shapes of the LDS sweep: lanes per pair x pairs per workgroup.
enum { TILE_16x16 = 0, TILE_64x4 = 1, TILE_64x1 = 2, TILE_256x1 = 3, TILE_512x1 = 4, TILE_1024x1 = 5,
       NUM_TILES = 6 };

struct SweepArgs {
  const unsigned char* gates;
  int64_t gate_stride;  // bytes per pair
  int G;                // gates per circuit
  const Op* ops;
  int64_t ops_stride;   // per pair (0: one program shared by all pairs)
  const int2* wgates;
  int64_t wg_stride;
  const int32_t* factors;
  int64_t f_stride;
  const PlanHeader* hdr;
  int64_t hdr_stride;
  double* trace;
  int64_t trace_offset;
  int64_t num_pairs;
  int cap_bits;         // LDS capacity per pair (log2 of complex entries)
  int min_bits;         // pairs whose peak is <= min_bits belong to another launch
  const int32_t* order; // if set: slot i contracts pair order[i] (num_pairs = length of the list)
  const unsigned char* wmat;  // realigned GATE matrices in program order (wave sweep), per pair
  int64_t wmat_stride;        // bytes per pair
  int bf3;                    // float32 storage with BF16x3 products
  // Pairs given on the device (local random): if range is set, the launch
  // contracts pairs order[range[0] + i], i < range[1], taken in turn through
  // the counter *claim (zero at launch) by workgroups (or wavefronts) that
  // loop until none is left; num_pairs is then only the launch's upper bound.
  const long long* range;
  unsigned long long* claim;
  int64_t grid_pairs;  // with range: pairs the launch is sized for (0: as many workgroups as stay resident)
};

struct PlanJob {
  const unsigned char* gates;
  int64_t gate_stride;
  int64_t bonds_off;
  int n, G;
  int64_t num_pairs;
  Op* ops;
  int64_t ops_stride;
  int2* wgates;
  int64_t wg_stride;
  int32_t* factors;
  int64_t f_stride;
  PlanHeader* hdr;
  int* max_peak;
  int* num_large;
  int* num_failed;
  int cap_bits;    // largest boundary run in LDS
  int tiny_bits;   // largest boundary run with 16 lanes per pair
  int small_bits;  // largest boundary run with one wavefront per pair
  int mid_bits;    // largest boundary run with 256 lanes per pair
  double* class_macs;  // complex MACs per launch class (16, 64, 256, 1024 lanes, HBM), then GATE ops
  int* hist;           // pairs per peak register width (PLAN_HIST entries)
  int16_t* gseq;       // merged gate of each GATE op, per pair
  int64_t gseq_stride; // entries per pair
  unsigned char* wmat; // realigned GATE matrices in program order, per pair
  int64_t wmat_stride; // bytes per pair
  int bf3;             // float32 storage with BF16x3 products
};

// Pair order by decreasing peak register width: pair i with peak b goes to
// position first[b] + (arrival rank among pairs of width b).  Failed plans
// get NaN traces and no position.
constexpr int PLAN_HIST = 64;
struct OrderJob {
  const PlanHeader* hdr;
  int64_t hdr_stride;
  int64_t num_pairs;
  int* cursor;        // PLAN_HIST counters, zero at launch
  int32_t* order;
  double* trace;
  int64_t trace_offset;
  const int32_t* first;  // PLAN_HIST first positions (device)
};
int launch_order_pairs(const OrderJob& j, hipStream_t s);

int launch_sweep_lds(const SweepArgs& a, int precision, int tile, hipStream_t s);
// HBM slots of the large-register sweep.  Owner workgroups (blockIdx below
// `owners`) take pairs from the launch's list in order; the j-th of them to
// make its first claim gets slot j (width 0 for a pair that stays in LDS), which has 2^b entries for the b with
// ge[b + 1] <= j < ge[b] (ge[b]: slots of at least 2^b entries, non-increasing
// in b, ge[32] = 0), at entry offset off[b] + (j - ge[b + 1]) * 2^b of base.
// The list is ordered by decreasing width and slot j is as wide as its j-th
// pair, so every pair an owner takes fits its slot.  alt (or null) holds a
// second slot for each j < min(owners, HELP_MAX), at alt_off[b] + (j - ge[b + 1])
// * 2^b.  Workgroups from `owners` on only help (needs HelpArgs).
// Widest HBM slot: 2^SLOT_BITS entries (registers beyond 2^31 entries run
// with 64-bit entry indices).  Slot arrays are indexed by width 0..SLOT_BITS
// with one more entry (SLOT_TOP) for the totals.
constexpr int SLOT_BITS = 36;
constexpr int SLOT_TOP = SLOT_BITS + 1;
struct SlotArgs {
  unsigned char* base;
  unsigned char* alt;
  int owners;
  int ge[SLOT_TOP + 1];
  long long off[SLOT_TOP + 1];
  long long alt_off[SLOT_TOP + 1];
};

// Work sharing: owner slots j < min(owners, HELP_MAX) have a task record.
// While an owner's boundary is in HBM and an op's register has at least
// 2^help_bits entries, it publishes the op there in chunks (once workgroups
// without pairs can exist).  Helpers (the workgroups from `owners` on, and a
// quarter of the owners once the pairs have run out) take chunks until the
// launch's first wide_pairs pairs, the only ones with such registers, have
// finished.
struct HelpRec {
  unsigned long long claim;    // task number (bits 40..63), chunks (20..39), next unclaimed chunk (0..19)
  unsigned long long maxbits;  // largest |entry| the helpers wrote (bits of a non-negative double)
  unsigned int done;           // chunks finished
  int type, b, p, q, track, chunk_bits;
  int base_bits;                // first item of the task: 2^base_bits (-1: item 0)
  unsigned long long src, dst;  // device addresses of the boundary before and after the op
  unsigned long long mat[32];   // realigned GATE matrix, pending scale applied (bits of doubles)
};
constexpr int HELP_MAX = 32;  // records per launch
struct HelpArgs {
  HelpRec* recs;           // HELP_MAX records, zero at launch
  unsigned int* finished;  // pairs below wide_pairs that have ended, zero at launch
  long long wide_pairs;    // pairs of the launch with a register of 2^help_bits entries or more (the first)
  int help_bits;           // smallest register (log2 entries) of a shared op
};
constexpr int64_t HELP_AREA_BYTES = HELP_MAX * (int64_t)sizeof(HelpRec) + 256;

// counter: zero at launch.  grid: workgroups (owners, then helpers).
int slot_bits_host(const SlotArgs& sl);
int launch_sweep_hbm(const SweepArgs& a, int precision, unsigned long long* counter, const SlotArgs& slots,
                     int grid, hipStream_t s, const HelpArgs* help = nullptr);

// Launch set-up of a local random chunk on the device: written by
// lr_setup_kernel from the planner's statistics and read by the ordering pass
// and the sweeps, so that the host enqueues the whole chunk without waiting.
// Classes k = 0..4 as the planner's class MACs: registers up to tiny, small,
// mid and cap bits, then HBM slots.  The HBM class runs as up to two launches
// on one stream, each with the whole slot pool: the pairs wider than a
// compute unit's share of the pool first (their slots would leave few owners
// for the rest), then the others.
struct HbmPhase {
  SlotArgs sl;             // slots (owners 0: the phase's pairs get NaN)
  HelpArgs help;           // work sharing (recs null: none)
  long long first, count;  // positions in the class's range of the order
  int workgroups;          // owners plus helpers-only workgroups (0: nothing to do)
  int max_bits;            // widest register of the phase's pairs (log2 entries)
};
constexpr int HBM_PHASES = 2;
struct LrDev {
  int32_t first[PLAN_HIST];     // ordering pass: first position of each width
  long long range[5][2];        // class k: first position in the order and count
  unsigned long long claim[5];  // class k: pair counter of its sweep (zero after set-up)
  HbmPhase ph[HBM_PHASES];      // the HBM class's launches, in order
  int hbm_workgroups;           // the larger launch's workgroups
  int max_bits;                 // widest register of the chunk's pairs (log2 entries)
  int status;                   // bit 0: a pair wider than 2^SLOT_BITS entries; bit 1: a pair without room in the pool
};
struct LrSetupJob {
  const int* hist;                 // pairs per peak width (PLAN_HIST)
  int tiny_bits, small_bits, mid_bits, cap_bits;
  unsigned char* pool;             // HBM slot pool
  long long pool_bytes;
  int elem_shift;                  // log2 of the bytes per complex entry
  int lds_bits;                    // pairs up to 2^lds_bits entries never use their HBM slot
  int max_owners, max_helpers, num_cus, help_bits;
  int wide_bits;                   // helpers-only workgroups also where the pairs limit the owners, once
                                   // the widest register has 2^wide_bits entries (>= help_bits)
  HelpRec* recs;                   // the chunk's work-sharing area (HELP_AREA_BYTES, cleared here)
  unsigned long long* hbm_counter; // the chunk's HBM claim words, one per phase (cleared here)
  LrDev* dev;
};
int launch_lr_setup(const LrSetupJob& j, hipStream_t s);
// HBM-slot sweep of phase `phase` of a local random class set up on the
// device (launch `grid` workgroups; those beyond the phase's workgroups
// return at once).  counter: the phase's claim word.  wide: 64-bit entry
// indices; tiled: some register may leave LDS (runs of GATEs on it then go
// tile by tile; either choice gives the same results).
int launch_sweep_hbm_dev(const SweepArgs& a, int precision, unsigned long long* counter, const LrDev* dev, int phase,
                         int grid, hipStream_t s, bool wide, bool tiled);
// Zero n 32-bit words (a kernel, so that stream capture records no memset node).
int launch_zero_words(void* p, int64_t n, hipStream_t s);
// Workgroups of a kernel resident per compute unit (occupancy query, no device work),
// and the current device's compute units.
int resident_per_cu(const void* kernel, int block, size_t smem);
int device_cus();
// Slot layout for `count` slots of non-increasing widths width[0 .. count)
// (log2 entries) of elem bytes each, from base; with_alt: the second slots
// follow.  slot_args_entries: entries of both.
void make_slot_args(SlotArgs* sl, unsigned char* base, const int* width, int count, bool with_alt, int elem);
int64_t slot_args_entries(const SlotArgs& sl);
inline int64_t hbm_slot_bytes(int bits, int elem) { return (int64_t)elem << bits; }
int launch_plan_local_random(const PlanJob& j, int precision, hipStream_t s);
int launch_gate_matrices(const PlanJob& j, int precision, hipStream_t s);
int launch_sweep_wave(const SweepArgs& a, int precision, int cap_bits, hipStream_t s);
size_t plan_lds_bytes(int G, int n);
int sweep_elem_bytes(int precision);

// Event timing of the sweep launches (enabled by fp_profile_begin).
enum { KCLASS_LDS16 = 0, KCLASS_LDS64 = 1, KCLASS_LDS256 = 2, KCLASS_LDS1024 = 3, KCLASS_HBM = 4, KCLASS_HEA = 5,
       KCLASS_PLAN = 6, KCLASS_PREP = 7, KCLASS_SAMPLE = 8, KCLASS_COUNT = 9 };
bool profiling();
void profile_launch_begin(int kclass, hipStream_t s);
void profile_launch_end(int kclass, double flops, hipStream_t s, double bytes = 0.0);
// As profile_launch_end, with the launch's complex MAC count read from device
// memory once the launch's stream reaches this point (flops = 8 x MACs).
void profile_launch_end_dev(int kclass, const double* d_macs, hipStream_t s);

// HEA (diagonal CZ ladders -> Walsh-Hadamard column transfer)
struct HeaArgs {
  const unsigned char* gates;
  int64_t gate_stride;
  int n, L;
  int bf3;  // float32 storage with BF16x3 products
  double* trace;
  int64_t trace_offset;
  int64_t num_pairs;
};
int launch_hea(const HeaArgs& a, int precision, int tile, hipStream_t s);
int hea_bits(int L);
// The paper's hardware-efficient ansatz (Pauli rotations; cnot = 1: CNOT
// walls, 0: CZ walls): boundary of 2L-2 labels, register of one more bit.
int launch_pauli_hea(const HeaArgs& a, int precision, int cnot, hipStream_t s);
int pauli_bits(int L);

// Qudit brickwork (qudit.hip): sampler, LDS budget and the column sweep on
// the brickwork program with base-q digits.
struct DevPlan;
size_t qudit_lds_bytes(int q, int peak, int precision);
int launch_qudit(const fp_ensemble_t* e, int64_t num_pairs, int precision, const void* gates, double* trace,
                 const DevPlan& dp, hipStream_t s, int64_t trace_offset);
double pauli_flops_per_pair(int n, int L);

int run_frame_potential(const double* d_trace, int64_t n, int kmax, double* h_F, double* h_se,
                        hipStream_t s);
// As run_frame_potential, on the library's static scratch array of the
// current device (no allocation).
int run_frame_potential_noalloc(const double* d_trace, int64_t n, int kmax, double* h_F, double* h_se,
                                hipStream_t s);
int run_log_moments(const double* tr, int64_t n, double eps, double* mu, double* sigma, hipStream_t s);
int run_log_targets(const double* tr, int64_t n, double eps, double mu, double sigma, float* t, hipStream_t s);
int run_link(const float* y, int64_t n, int k, double mu, double sigma, double shift, float* g, hipStream_t s);
int run_targets(const double* tr, int64_t n, int k, double scale, float* t, hipStream_t s);
int run_cv_coefficient(const double* tr, const float* g, int64_t n, int k, double* c_out, hipStream_t s);
int run_cv_holdout(const double* tr, const float* g, int64_t n, int k, double* out6, hipStream_t s);
int run_moments_f32(const float* x, int64_t n, double* mean, double* var, hipStream_t s);
int run_frame_potential_cv(const double* trB, const float* gB, int64_t nB, const float* gC, int64_t nC,
                           int k, double c, double* h_F, double* h_se, hipStream_t s);

}  // namespace fp
