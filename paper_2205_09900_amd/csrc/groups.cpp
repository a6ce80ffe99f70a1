// fp_contract_trace_groups: uneven batches (different depths and qubit
// counts) in one persistent launch per LDS class, tasks ordered by cost.
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

// Pairs per task: about task_flops of work per task, between 1 and 256 pairs.
int pairs_per_task(double cost, double task_flops) {
  double c = task_flops / (cost > 1.0 ? cost : 1.0);
  if (c < 1.0) c = 1.0;
  if (c > 256.0) c = 256.0;
  return (int)c;
}

// Lane class and task size of a persistent group: `force` if given, else the
// tuning table's entry, else 64 lanes for registers up to 2^small_bits
// entries and a whole workgroup beyond, with DEFAULT_TASK_FLOPS per task.
void choose_launch(const fp_ensemble_t* e, int prec, int bits, const GroupLaunch* force, GroupPlan* gp) {
  const int small_bits = prec == FP_C128 ? 9 : 10;  // 64 lanes x 4 pairs per workgroup
  GroupLaunch c{bits <= small_bits ? PCLASS_SMALL : PCLASS_LARGE, DEFAULT_TASK_FLOPS};
  GroupLaunch t;
  if (force)
    c = *force;
  else if (tune_group_lookup(e, prec, &t))
    c = t;
  if (c.cls == PCLASS_SMALL && bits > small_bits) c.cls = PCLASS_LARGE;  // the register must fit 4 per workgroup
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
  size_t total = 256 + (size_t)n_groups * sizeof(GroupDesc);
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
  total += (size_t)ntasks * sizeof(Task) + 6 * 256;
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
  // tasks per (precision index, class): precision index 0 = c128, 1 = c64, 2 = bf16x3
  std::vector<Task> tasks[3][2];
  int slot_bytes[3][2] = {{0, 0}, {0, 0}, {0, 0}};
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
      const int rb = gr.precision == FP_C128 ? 8 : 4;
      const int nt = gp.cls == PCLASS_SMALL ? 64 : (gr.precision == FP_C128 ? 512 : 1024);
      const size_t sb = e->ansatz == FP_HEA_RYRZ_CZ ? ((hea_smem_bytes(gp.bits, nt, rb) + 15) & ~(size_t)15)
                                                      : program_slot_bytes(d.m, nt, rb);
      if ((int)sb > slot_bytes[pi][gp.cls]) slot_bytes[pi][gp.cls] = (int)sb;
      for (int64_t p = 0; p < gr.num_pairs; p += gp.per_task) {
        Task t;
        t.group = g;
        t.first = p;
        t.count = (int32_t)std::min<int64_t>(gp.per_task, gr.num_pairs - p);
        tasks[pi][gp.cls].push_back(t);
      }
    }
    offset += gr.num_pairs;
  }
  // largest first
  for (int pi = 0; pi < 3; ++pi)
    for (int c = 0; c < 2; ++c)
      std::stable_sort(tasks[pi][c].begin(), tasks[pi][c].end(), [&](const Task& a, const Task& b) {
        return gps[a.group].pair_cost * a.count > gps[b.group].pair_cost * b.count;
      });
  // workspace: counters | descriptors | task lists | separate-route slices
  unsigned char* w = (unsigned char*)d_ws;
  unsigned int* counters = (unsigned int*)w;
  GroupDesc* d_desc = (GroupDesc*)(w + 256);
  size_t off = (256 + (size_t)n_groups * sizeof(GroupDesc) + 255) & ~(size_t)255;
  Task* d_tasks[3][2];
  for (int pi = 0; pi < 3; ++pi)
    for (int c = 0; c < 2; ++c) {
      d_tasks[pi][c] = (Task*)(w + off);
      off += ((tasks[pi][c].size() * sizeof(Task)) + 255) & ~(size_t)255;
    }
  rc = check_hip(hipMemsetAsync(counters, 0, 256, s), "memset counters");
  if (!rc) rc = check_hip(hipMemcpyAsync(d_desc, descs.data(), sizeof(GroupDesc) * n_groups, hipMemcpyHostToDevice, s),
                          "upload groups");
  for (int pi = 0; pi < 3 && !rc; ++pi)
    for (int c = 0; c < 2 && !rc; ++c)
      if (!tasks[pi][c].empty())
        rc = check_hip(hipMemcpyAsync(d_tasks[pi][c], tasks[pi][c].data(), sizeof(Task) * tasks[pi][c].size(),
                                      hipMemcpyHostToDevice, s),
                       "upload tasks");
  // the host vectors are released when this call returns
  if (!rc) rc = check_hip(hipStreamSynchronize(s), "sync(upload)");
  if (rc) return rc;
  int dev = 0, num_cus = 1;
  rc = check_hip(hipGetDevice(&dev), "hipGetDevice");
  if (!rc) rc = check_hip(hipDeviceGetAttribute(&num_cus, hipDeviceAttributeMultiprocessorCount, dev), "CU count");
  if (rc) return rc;
  Aux aux;
  rc = get_aux(&aux, s);
  if (rc) return rc;
  rc = check_hip(hipEventRecord(aux.fork, s), "fork");
  if (rc) return rc;
  // persistent launches: class SMALL on s, LARGE on aux stream 0 (both precisions)
  int used = 0;
  for (int c = 0; c < 2; ++c) {
    hipStream_t sx = c == 0 ? s : aux.s[0];
    if (c == 1) {
      rc = check_hip(hipStreamWaitEvent(sx, aux.fork, 0), "fork wait");
      if (rc) return rc;
    }
    for (int pi = 0; pi < 3; ++pi) {
      if (tasks[pi][c].empty()) continue;
      const int prec = pi == 0 ? FP_C128 : pi == 1 ? FP_C64 : FP_BF16X3;
      profile_launch_begin(c == 0 ? KCLASS_LDS64 : KCLASS_LDS1024, sx);
      rc = launch_persistent(prec, c, d_desc, d_tasks[pi][c], (int)tasks[pi][c].size(), counters + 4 * (2 * pi + c),
                             d_trace, slot_bytes[pi][c], num_cus, sx);
      double fl = 0.0;
      for (const Task& t : tasks[pi][c]) fl += gps[t.group].pair_cost * t.count;
      profile_launch_end(c == 0 ? KCLASS_LDS64 : KCLASS_LDS1024, fl, sx);
      if (rc) return rc;
    }
    if (c == 1) {
      rc = check_hip(hipEventRecord(aux.join[0], sx), "join");
      if (rc) return rc;
      used = 1;
    }
  }
  if (used) rc = check_hip(hipStreamWaitEvent(s, aux.join[0], 0), "join wait");
  if (rc) return rc;
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
