// fp_contract_trace_groups: uneven batches (different depths and qubit
// counts) in one persistent launch per lane class and register-size bucket
// (so that a workgroup's LDS slot is sized for the registers it runs, not for
// the widest group of the call), tasks ordered by cost.
#include <hip/hip_runtime.h>
#include <string.h>

#include <algorithm>
#include <vector>

#include "dispatch.h"
#include "hea_dev.h"
#include "internal.h"
#include "layout.h"
#include "sched.h"
#include "sweep.h"
#include "tune.h"

namespace fp {

namespace {

enum Route { ROUTE_PERSISTENT = 0, ROUTE_SEPARATE = 1 };

struct GroupPlan {
  int route;
  int cls;           // PCLASS_* for the persistent route
  int bits;          // LDS boundary bits
  double pair_cost;  // algorithmic flops of one pair
  double task_flops; // algorithmic flops per task
  int per_task;      // pairs per task
  int64_t ntasks;
  size_t sep_ws;     // workspace of the separate route
  DevPlan plan;      // brickwork
};

constexpr double DEFAULT_TASK_FLOPS = 2e7;

// Register-size buckets of the persistent launches: bucket k holds groups of
// 2k - 1 or 2k register bits (bits 0 .. 2 in bucket 1).
constexpr int NBUCKET = 9;
constexpr int NLISTS = 3 * PCLASS_COUNT * 2 * NBUCKET;  // precision x lane class x group kind x bucket
constexpr size_t COUNTER_BYTES = 4 * 4 * NLISTS;  // one 16-byte counter per list
inline int size_bucket(int bits) {
  const int k = (bits + 1) / 2;
  return k < 1 ? 1 : (k >= NBUCKET ? NBUCKET - 1 : k);
}

// Pairs per task: about task_flops of work per task, between 1 and 256 pairs.
int pairs_per_task(double cost, double task_flops) {
  double c = task_flops / (cost > 1.0 ? cost : 1.0);
  if (c < 1.0) c = 1.0;
  if (c > 256.0) c = 256.0;
  return (int)c;
}

// Lane class and task size of a persistent group: `force` if given, else the
// tuning table's entry, else the class the per-ensemble launches take for the
// register width (pclass_default), with DEFAULT_TASK_FLOPS per task.  A class
// whose workgroup cannot hold its pairs' registers falls back to the default.
void choose_launch(const fp_ensemble_t* e, int prec, int bits, const GroupLaunch* force, GroupPlan* gp) {
  const bool hea = e->ansatz == FP_HEA_RYRZ_CZ;
  GroupLaunch c{pclass_default(bits, prec), DEFAULT_TASK_FLOPS};
  GroupLaunch t;
  if (force)
    c = *force;
  else if (tune_group_lookup(e, prec, &t))
    c = t;
  if (c.cls < 0 || c.cls >= PCLASS_COUNT || !pclass_fits(c.cls, bits, hea, prec)) c.cls = pclass_default(bits, prec);
  gp->cls = c.cls;
  gp->task_flops = c.task_flops > 0.0 ? c.task_flops : DEFAULT_TASK_FLOPS;
}

int plan_group(const fp_ensemble_t* e, const fp_group_t* g, bool upload_plan, const GroupLaunch* force,
               GroupPlan* gp) {
  memset(gp, 0, sizeof(*gp));
  const int prec = g->precision;
  if (e->ansatz == FP_HEA_RYRZ_CZ) {
    gp->bits = hea_bits(e->depth);
    gp->pair_cost = hea_flops_per_pair(e->n_qubits, e->depth);
    if (gp->bits > lds_bits_max(prec)) return set_error(FP_ETOOBIG, "HEA boundary of %d bits exceeds LDS", gp->bits);
    gp->route = ROUTE_PERSISTENT;
    choose_launch(e, prec, gp->bits, force, gp);
  } else if (e->ansatz == FP_BRICKWORK_HAAR) {
    int rc = 0;
    if (upload_plan) {
      rc = get_brickwork_plan(e->n_qubits, e->depth, &gp->plan);
      if (rc) return rc;
      gp->bits = gp->plan.hdr.peak_bits;
      gp->pair_cost = 8.0 * gp->plan.hdr.macs;
    } else {
      int32_t peak = 0;
      double macs = 0.0;
      rc = fp_plan_info(e, nullptr, &peak, &macs, nullptr);
      if (rc) return rc;
      gp->bits = peak;
      gp->pair_cost = 8.0 * macs;
    }
    if (gp->bits <= lds_bits_max(prec)) {
      gp->route = ROUTE_PERSISTENT;
      choose_launch(e, prec, gp->bits < 2 ? 2 : gp->bits, force, gp);
    } else {
      gp->route = ROUTE_SEPARATE;
    }
  } else {
    gp->route = ROUTE_SEPARATE;
    gp->pair_cost = 0.0;
  }
  if (gp->route == ROUTE_SEPARATE) {
    size_t b = 0;
    int rc = workspace_bytes_impl(e, g->num_pairs, prec, &b);
    if (rc) return rc;
    gp->sep_ws = (b + 255) & ~(size_t)255;
  } else {
    gp->per_task = pairs_per_task(gp->pair_cost, gp->task_flops);
    // and small enough that every lane group of the class on every compute
    // unit gets tasks several times over (cheap pairs otherwise leave a few
    // groups working through long tasks alone)
    const int64_t target = (int64_t)device_cus() * pclass_pairs(gp->cls) * 16;
    const int64_t cap = (g->num_pairs + target - 1) / target;
    if (gp->per_task > cap) gp->per_task = (int)(cap > 1 ? cap : 1);
    gp->ntasks = (g->num_pairs + gp->per_task - 1) / gp->per_task;
  }
  return FP_OK;
}

int check_groups(const fp_ensemble_t* ens, int n_ens, const fp_group_t* groups, int n_groups) {
  if (!ens || !groups || n_ens < 1 || n_groups < 0) return set_error(FP_EINVAL, "bad group arguments");
  for (int i = 0; i < n_ens; ++i) {
    int rc = check_ensemble(&ens[i]);
    if (rc) return rc;
  }
  for (int g = 0; g < n_groups; ++g) {
    const fp_group_t& gr = groups[g];
    if (gr.ensemble_index < 0 || gr.ensemble_index >= n_ens) return set_error(FP_EINVAL, "group %d: bad ensemble", g);
    if (check_precision(gr.precision)) return set_error(FP_EINVAL, "group %d: unknown precision %d", g, gr.precision);
    if (gr.num_pairs < 0 || gr.first_pair < 0) return set_error(FP_EINVAL, "group %d: bad pair range", g);
  }
  return FP_OK;
}

}  // namespace

}  // namespace fp

using namespace fp;

extern "C" {

int fp_workspace_bytes_groups(const fp_ensemble_t* ens, int n_ens, const fp_group_t* groups, int n_groups,
                              size_t* out_bytes) {
  int rc = check_groups(ens, n_ens, groups, n_groups);
  if (rc) return rc;
  if (!out_bytes) return set_error(FP_EINVAL, "out_bytes is NULL");
  size_t total = ((COUNTER_BYTES + 255) & ~(size_t)255) + (size_t)n_groups * sizeof(GroupDesc);
  total = (total + 255) & ~(size_t)255;
  int64_t ntasks = 0;  // at most one task per pair, whatever the launch choice
  for (int g = 0; g < n_groups; ++g) {
    GroupPlan gp;
    rc = plan_group(&ens[groups[g].ensemble_index], &groups[g], false, nullptr, &gp);
    if (rc) return rc;
    if (gp.route == ROUTE_SEPARATE)
      total += gp.sep_ws;
    else
      ntasks += groups[g].num_pairs;
  }
  total += (size_t)ntasks * sizeof(Task) + NLISTS * 256;
  *out_bytes = total;
  return FP_OK;
}

int fp_contract_trace_groups(const fp_ensemble_t* ens, int n_ens, const fp_group_t* groups, int n_groups,
                             const void* const* d_gates, double* d_trace, void* d_ws, size_t ws_bytes, void* stream) {
  return contract_groups(ens, n_ens, groups, n_groups, d_gates, d_trace, d_ws, ws_bytes, (hipStream_t)stream,
                         nullptr);
}

}  // extern "C"

namespace fp {

int contract_groups(const fp_ensemble_t* ens, int n_ens, const fp_group_t* groups, int n_groups,
                    const void* const* d_gates, double* d_trace, void* d_ws, size_t ws_bytes, hipStream_t s,
                    const GroupLaunch* force) {
  int rc = check_groups(ens, n_ens, groups, n_groups);
  if (rc) return rc;
  if (n_groups == 0) return FP_OK;
  if (!d_gates || !d_trace) return set_error(FP_EINVAL, "NULL gates or trace");
  size_t need = 0;
  rc = fp_workspace_bytes_groups(ens, n_ens, groups, n_groups, &need);
  if (rc) return rc;
  if (!d_ws || ws_bytes < need) return set_error(FP_ETOOBIG, "workspace of %zu bytes needed", need);

  std::vector<GroupPlan> gps(n_groups);
  std::vector<GroupDesc> descs(n_groups);
  // tasks per (precision index, class, size bucket): precision index 0 = c128, 1 = c64, 2 = bf16x3
  std::vector<Task> tasks[3][PCLASS_COUNT][2][NBUCKET];  // [.][.][GROUP_PROGRAM or GROUP_HEA][.]
  int slot_bytes[3][PCLASS_COUNT][2][NBUCKET] = {};
  int64_t offset = 0;
  for (int g = 0; g < n_groups; ++g) {
    const fp_ensemble_t* e = &ens[groups[g].ensemble_index];
    const fp_group_t& gr = groups[g];
    if (gr.num_pairs > 0 && !d_gates[g]) return set_error(FP_EINVAL, "group %d: NULL gate buffer", g);
    GroupPlan& gp = gps[g];
    rc = plan_group(e, &gr, true, force, &gp);
    if (rc) return rc;
    GroupDesc& d = descs[g];
    memset(&d, 0, sizeof(d));
    d.n = e->n_qubits;
    d.depth = e->depth;
    d.G = (int)gates_per_circuit(e->ansatz, e->n_qubits, e->depth);
    d.m = gp.bits < 2 && e->ansatz != FP_HEA_RYRZ_CZ ? 2 : gp.bits;
    d.gates = (const unsigned char*)d_gates[g];
    d.stride = pair_bytes(e->ansatz, e->n_qubits, e->depth, gr.precision, e->local_dim);
    d.gate_first = gr.first_pair;
    d.trace_offset = offset;
    d.bf3 = gr.precision == FP_BF16X3 ? 1 : 0;
    if (e->ansatz == FP_HEA_RYRZ_CZ) {
      d.kind = GROUP_HEA;
    } else {
      d.kind = GROUP_PROGRAM;
      d.ops = gp.plan.ops;
      d.wg = gp.plan.wg;
      d.fac = gp.plan.fac;
      d.hdr = gp.plan.dhdr;
    }
    if (gp.route == ROUTE_PERSISTENT && gr.num_pairs > 0) {
      const int pi = gr.precision == FP_C128 ? 0 : gr.precision == FP_C64 ? 1 : 2;
      const size_t sb = e->ansatz == FP_HEA_RYRZ_CZ ? pclass_slot_bytes(gp.cls, gp.bits, true, gr.precision)
                                                      : pclass_slot_bytes(gp.cls, d.m, false, gr.precision);
      const int bk = size_bucket(gp.bits);
      const int kd = d.kind;
      if ((int)sb > slot_bytes[pi][gp.cls][kd][bk]) slot_bytes[pi][gp.cls][kd][bk] = (int)sb;
      for (int64_t p = 0; p < gr.num_pairs; p += gp.per_task) {
        Task t;
        t.group = g;
        t.first = p;
        t.count = (int32_t)std::min<int64_t>(gp.per_task, gr.num_pairs - p);
        tasks[pi][gp.cls][kd][bk].push_back(t);
      }
    }
    offset += gr.num_pairs;
  }
  // largest first
  for (int pi = 0; pi < 3; ++pi)
    for (int c = 0; c < PCLASS_COUNT; ++c)
      for (int kd = 0; kd < 2; ++kd)
        for (int bk = 0; bk < NBUCKET; ++bk)
          std::stable_sort(tasks[pi][c][kd][bk].begin(), tasks[pi][c][kd][bk].end(),
                           [&](const Task& a, const Task& b) {
                             return gps[a.group].pair_cost * a.count > gps[b.group].pair_cost * b.count;
                           });
  // workspace: counters | descriptors | task lists | separate-route slices
  unsigned char* w = (unsigned char*)d_ws;
  unsigned int* counters = (unsigned int*)w;
  const size_t desc_off = (COUNTER_BYTES + 255) & ~(size_t)255;
  GroupDesc* d_desc = (GroupDesc*)(w + desc_off);
  size_t off = (desc_off + (size_t)n_groups * sizeof(GroupDesc) + 255) & ~(size_t)255;
  Task* d_tasks[3][PCLASS_COUNT][2][NBUCKET];
  for (int pi = 0; pi < 3; ++pi)
    for (int c = 0; c < PCLASS_COUNT; ++c)
      for (int kd = 0; kd < 2; ++kd)
        for (int bk = 0; bk < NBUCKET; ++bk) {
          d_tasks[pi][c][kd][bk] = (Task*)(w + off);
          off += ((tasks[pi][c][kd][bk].size() * sizeof(Task)) + 255) & ~(size_t)255;
        }
  rc = check_hip(hipMemsetAsync(counters, 0, COUNTER_BYTES, s), "memset counters");
  if (!rc) rc = check_hip(hipMemcpyAsync(d_desc, descs.data(), sizeof(GroupDesc) * n_groups, hipMemcpyHostToDevice, s),
                          "upload groups");
  for (int pi = 0; pi < 3 && !rc; ++pi)
    for (int c = 0; c < PCLASS_COUNT && !rc; ++c)
      for (int kd = 0; kd < 2 && !rc; ++kd)
        for (int bk = 0; bk < NBUCKET && !rc; ++bk)
          if (!tasks[pi][c][kd][bk].empty())
            rc = check_hip(hipMemcpyAsync(d_tasks[pi][c][kd][bk], tasks[pi][c][kd][bk].data(),
                                          sizeof(Task) * tasks[pi][c][kd][bk].size(), hipMemcpyHostToDevice, s),
                           "upload tasks");
  // the host vectors are released when this call returns
  if (!rc) rc = check_hip(hipStreamSynchronize(s), "sync(upload)");
  if (rc) return rc;
  int dev = 0, num_cus = 1;
  rc = check_hip(hipGetDevice(&dev), "hipGetDevice");
  if (!rc) rc = check_hip(hipDeviceGetAttribute(&num_cus, hipDeviceAttributeMultiprocessorCount, dev), "CU count");
  if (rc) return rc;
  // persistent launches, one after another on s, widest registers first
  // (launches of different slot sizes side by side were slower: a workgroup
  // of the widest bucket needs a whole compute unit's LDS)
  for (int c = PCLASS_COUNT - 1; c >= 0; --c) {
    const int kc = c == PCLASS_TINY    ? KCLASS_LDS16
                   : c == PCLASS_SMALL ? KCLASS_LDS64
                   : c == PCLASS_MID   ? KCLASS_LDS256
                                       : KCLASS_LDS1024;
    for (int pi = 0; pi < 3; ++pi) {
      for (int kd = 0; kd < 2; ++kd) {
        for (int bk = NBUCKET - 1; bk >= 0; --bk) {
          const std::vector<Task>& tl = tasks[pi][c][kd][bk];
          if (tl.empty()) continue;
          const int prec = pi == 0 ? FP_C128 : pi == 1 ? FP_C64 : FP_BF16X3;
          const int list = ((pi * PCLASS_COUNT + c) * 2 + kd) * NBUCKET + bk;
          profile_launch_begin(kc, s);
          rc = launch_persistent(prec, kd, c, d_desc, d_tasks[pi][c][kd][bk], (int)tl.size(), counters + 4 * list,
                                 d_trace, slot_bytes[pi][c][kd][bk], num_cus, s);
          double fl = 0.0;
          for (const Task& t : tl) fl += gps[t.group].pair_cost * t.count;
          profile_launch_end(kc, fl, s);
          if (rc) return rc;
        }
      }
    }
  }
  // groups that need per-pair plans or HBM boundaries: after the persistent launches, on s
  // (their own launches fork from s and join back into s)
  for (int g = 0; g < n_groups && !rc; ++g) {
    if (gps[g].route != ROUTE_SEPARATE || groups[g].num_pairs == 0) continue;
    const fp_ensemble_t* e = &ens[groups[g].ensemble_index];
    const unsigned char* gg = (const unsigned char*)d_gates[g] +
                              groups[g].first_pair * pair_bytes(e->ansatz, e->n_qubits, e->depth, groups[g].precision, e->local_dim);
    rc = contract_dispatch(e, groups[g].num_pairs, groups[g].precision, gg, d_trace, w + off, gps[g].sep_ws, s,
                           descs[g].trace_offset);
    off += gps[g].sep_ws;
  }
  return rc;
}

}  // namespace fp
