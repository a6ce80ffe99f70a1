// Descriptors of the persistent sweep over groups of pairs.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "plan.h"

namespace fp {

enum { GROUP_PROGRAM = 0, GROUP_HEA = 1 };
// Lane classes of the persistent sweep: lanes per pair and pairs per
// workgroup, as the per-ensemble launches choose them by register width.
//   PCLASS_TINY:  16 lanes, 16 pairs per workgroup
//   PCLASS_SMALL: 64 lanes, 4 pairs per workgroup
//   PCLASS_MID:   256 lanes, one pair per workgroup
//   PCLASS_LARGE: 1024 lanes (512 in complex128), one pair per workgroup
enum { PCLASS_TINY = 0, PCLASS_SMALL = 1, PCLASS_MID = 2, PCLASS_LARGE = 3, PCLASS_COUNT = 4 };
int pclass_lanes(int cls, int precision);
int pclass_pairs(int cls);
// LDS bytes of one pair slot (register of 2^bits entries, staging) of the class
size_t pclass_slot_bytes(int cls, int bits, bool hea, int precision);
// whether the class's workgroup holds its pairs' slots in LDS
bool pclass_fits(int cls, int bits, bool hea, int precision);
// the class a register of 2^bits entries gets without tuning
int pclass_default(int bits, int precision);

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

size_t program_slot_bytes(int bits, int nt, int real_bytes, bool bf3);
// One persistent launch over tasks whose groups are all of `kind` (GROUP_*).
int launch_persistent(int precision, int kind, int cls, const GroupDesc* groups, const Task* tasks, int ntasks,
                      unsigned int* counter, double* trace, int slot_bytes, int num_cus, hipStream_t s);

}  // namespace fp
