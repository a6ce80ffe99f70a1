// Descriptors of the persistent sweep over groups of pairs.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "plan.h"

namespace fp {

enum { GROUP_PROGRAM = 0, GROUP_HEA = 1 };
enum { PCLASS_SMALL = 0, PCLASS_LARGE = 1 };  // lanes per pair 64 (4 per workgroup) or a whole workgroup

struct GroupDesc {
  int32_t kind;
  int32_t n, depth, G, m;  // m: boundary bits held in LDS (HEA: 2L-2; programs: the plan's peak)
  const unsigned char* gates;
  int64_t stride;
  int64_t gate_first;    // first pair of the group inside its gate buffer
  int64_t trace_offset;  // first output slot of the group
  const Op* ops;
  int64_t ops_stride;
  const int2* wg;
  int64_t wg_stride;
  const int32_t* fac;
  int64_t f_stride;
  const PlanHeader* hdr;
  int64_t hdr_stride;
  int32_t bf3;  // float32 storage with BF16x3 products (also selects the launch)
};

struct Task {
  int32_t group;
  int32_t count;   // pairs
  int64_t first;   // first pair, relative to the group
};

size_t program_slot_bytes(int bits, int nt, int real_bytes);
int launch_persistent(int precision, int cls, const GroupDesc* groups, const Task* tasks, int ntasks,
                      unsigned int* counter, double* trace, int slot_bytes, int num_cus, hipStream_t s);

}  // namespace fp
