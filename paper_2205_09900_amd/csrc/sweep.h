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
  int32_t first[PLAN_HIST];
};
int launch_order_pairs(const OrderJob& j, hipStream_t s);

int launch_sweep_lds(const SweepArgs& a, int precision, int tile, hipStream_t s);
// Slots of num_slots * hbm_slot_bytes(slot_bits, element bytes): 2^slot_bits entries each, one per
// workgroup; the first nbig pairs of the launch (its widest, the pairs being ordered by decreasing
// width) use big_slots instead, nbig * hbm_slot_bytes(big_bits, element bytes).
int launch_sweep_hbm(const SweepArgs& a, int precision, unsigned long long* counter, void* slots,
                     int slot_bits, int num_slots, void* big_slots, int big_bits, int nbig, hipStream_t s);
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

int run_frame_potential(const double* d_trace, int64_t n, int kmax, double* h_F, double* h_se,
                        hipStream_t s);
int run_log_moments(const double* tr, int64_t n, double eps, double* mu, double* sigma, hipStream_t s);
int run_log_targets(const double* tr, int64_t n, double eps, double mu, double sigma, float* t, hipStream_t s);
int run_link(const float* y, int64_t n, int k, double mu, double sigma, double shift, float* g, hipStream_t s);
int run_targets(const double* tr, int64_t n, int k, double scale, float* t, hipStream_t s);
int run_cv_coefficient(const double* tr, const float* g, int64_t n, int k, double* c_out, hipStream_t s);
int run_frame_potential_cv(const double* trB, const float* gB, int64_t nB, const float* gC, int64_t nC,
                           int k, double c, double* h_F, double* h_se, hipStream_t s);

}  // namespace fp
