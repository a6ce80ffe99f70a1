// Autotuner of the persistent sweep over groups (fp_contract_trace_groups).
//
// For one ensemble and precision it times the candidate launch choices of a
// group on the device -- the lane class (16 lanes with 16 pairs per
// workgroup, 64 lanes with four, 256 lanes, or 1024 (512 in complex128); a
// class only while its workgroup holds its pairs' registers in LDS) and the
// work per task the persistent workgroups take from their counter -- on synthetic pairs drawn by
// fp_sample_gates, and keeps the fastest in a table keyed by the device
// architecture, the ensemble and the precision.  fp_contract_trace_groups
// reads the table for every group it launches.  The table can be written
// out and read back as text.  Every candidate runs the same kernels, with the
// same shapes, as untuned launches of some register width.
#include <hip/hip_runtime.h>
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <map>
#include <mutex>
#include <string>
#include <tuple>
#include <vector>

#include "dispatch.h"
#include "internal.h"
#include "layout.h"
#include "sched.h"
#include "sweep.h"
#include "tune.h"

namespace fp {

namespace {

using Key = std::tuple<std::string, int, int, int, int>;  // arch, ansatz, n, depth, precision
struct Entry {
  GroupLaunch launch;
  double ms;
};
std::mutex g_mu;
std::map<Key, Entry> g_table;

// Candidates: choice = 3 * class + task size index.
constexpr double TASK_FLOPS[3] = {5e6, 2e7, 8e7};
constexpr int NUM_CHOICES = 3 * PCLASS_COUNT;

GroupLaunch choice_launch(int c) { return GroupLaunch{c / 3, TASK_FLOPS[c % 3]}; }

std::string arch_name() {
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) {
    (void)hipGetLastError();
    return "unknown";
  }
  hipDeviceProp_t prop;
  if (hipGetDeviceProperties(&prop, dev) != hipSuccess) {
    (void)hipGetLastError();
    return "unknown";
  }
  std::string a = prop.gcnArchName;
  const size_t c = a.find(':');
  return c == std::string::npos ? a : a.substr(0, c);
}

// Register width and algorithmic flops of one pair of a fixed-topology ensemble.
int ensemble_bits(const fp_ensemble_t* e, int* bits, double* cost) {
  if (e->ansatz == FP_HEA_RYRZ_CZ) {
    *bits = hea_bits(e->depth);
    *cost = hea_flops_per_pair(e->n_qubits, e->depth);
    return FP_OK;
  }
  int32_t peak = 0;
  double macs = 0.0;
  int rc = fp_plan_info(e, nullptr, &peak, &macs, nullptr);
  *bits = peak < 2 ? 2 : peak;
  *cost = 8.0 * macs;
  return rc;
}

// Pairs timed per candidate: about 4e9 flops of work, 2^12 .. 2^16 pairs.
int64_t tune_pairs(double cost) {
  double p = 4e9 / (cost > 1.0 ? cost : 1.0);
  if (p < 4096) p = 4096;
  if (p > 65536) p = 65536;
  return (int64_t)p;
}

size_t round256(size_t x) { return (x + 255) & ~(size_t)255; }

const char* const CLASS_NAMES[PCLASS_COUNT] = {"tiny", "small", "mid", "large"};
const char* class_name(int c) { return c >= 0 && c < PCLASS_COUNT ? CLASS_NAMES[c] : "large"; }

}  // namespace

bool tune_group_lookup(const fp_ensemble_t* e, int precision, GroupLaunch* out) {
  std::lock_guard<std::mutex> lk(g_mu);
  if (g_table.empty()) return false;
  auto it = g_table.find(Key(arch_name(), e->ansatz, e->n_qubits, e->depth, precision));
  if (it == g_table.end()) return false;
  *out = it->second.launch;
  return true;
}

}  // namespace fp

using namespace fp;

extern "C" {

size_t fp_autotune_workspace_bytes(const fp_ensemble_t* ens, int precision) {
  if (check_ensemble(ens) || check_precision(precision) || ens->ansatz == FP_LOCAL_RANDOM_HAAR ||
      ens->ansatz == FP_BRICKWORK_QUDIT)
    return 0;
  int bits = 0;
  double cost = 0.0;
  if (ensemble_bits(ens, &bits, &cost)) return 0;
  const int64_t np = tune_pairs(cost);
  fp_group_t g{0, precision, 0, np};
  size_t ws = 0;
  if (fp_workspace_bytes_groups(ens, 1, &g, 1, &ws)) return 0;
  return round256((size_t)np * (size_t)pair_bytes(ens->ansatz, ens->n_qubits, ens->depth, precision, ens->local_dim)) +
         round256(16 * (size_t)np) + round256(ws);
}

int fp_autotune(const fp_ensemble_t* ens, int precision, void* d_ws, size_t ws_bytes, int* out_choice, void* stream) {
  int rc = check_ensemble(ens);
  if (rc) return rc;
  if ((rc = check_precision(precision))) return rc;
  if (ens->ansatz == FP_LOCAL_RANDOM_HAAR)
    return set_error(FP_ENOTIMPL, "local random pairs are planned per pair and launched by register width");
  if (ens->ansatz == FP_BRICKWORK_QUDIT)
    return set_error(FP_ENOTIMPL, "qudit brickworks have one launch shape (one pair per workgroup)");
  if (!out_choice) return set_error(FP_EINVAL, "out_choice is NULL");
  int bits = 0;
  double cost = 0.0;
  if ((rc = ensemble_bits(ens, &bits, &cost))) return rc;
  if (bits > lds_bits_max(precision))
    return set_error(FP_ENOTIMPL, "boundaries beyond LDS do not run in the persistent sweep");
  const size_t need = fp_autotune_workspace_bytes(ens, precision);
  if (need == 0) return set_error(FP_EINVAL, "no workspace size for this ensemble");
  if (!d_ws || ws_bytes < need) return set_error(FP_ETOOBIG, "autotune needs %zu bytes of workspace", need);
  hipStream_t s = (hipStream_t)stream;
  const int64_t np = tune_pairs(cost);
  unsigned char* w = (unsigned char*)d_ws;
  const size_t gbytes = (size_t)np * (size_t)pair_bytes(ens->ansatz, ens->n_qubits, ens->depth, precision, ens->local_dim);
  void* gates = w;
  double* trace = (double*)(w + round256(gbytes));
  unsigned char* gws = (unsigned char*)trace + round256(16 * (size_t)np);
  const size_t gws_bytes = ws_bytes - (size_t)(gws - w);
  rc = fp_sample_gates(ens, np, 0x7E57ull, 0, precision, gates, gbytes, stream);
  if (rc) return rc;
  const fp_group_t grp{0, precision, 0, np};
  const void* gptr[1] = {gates};
  const bool hea = ens->ansatz == FP_HEA_RYRZ_CZ;
  hipEvent_t a, b;
  if ((rc = check_hip(hipEventCreate(&a), "event"))) return rc;
  if ((rc = check_hip(hipEventCreate(&b), "event"))) {
    (void)hipEventDestroy(a);
    return rc;
  }
  int best = -1;
  double best_ms = 1e300;
  for (int c = 0; c < NUM_CHOICES && !rc; ++c) {
    const GroupLaunch gl = choice_launch(c);
    if (!pclass_fits(gl.cls, bits, hea, precision)) continue;  // the workgroup must hold its pairs' registers
    // warm-up, then the median of three timed runs
    rc = contract_groups(ens, 1, &grp, 1, gptr, trace, gws, gws_bytes, s, &gl);
    std::vector<double> ms;
    for (int r = 0; r < 3 && !rc; ++r) {
      rc = check_hip(hipEventRecord(a, s), "record");
      if (!rc) rc = contract_groups(ens, 1, &grp, 1, gptr, trace, gws, gws_bytes, s, &gl);
      if (!rc) rc = check_hip(hipEventRecord(b, s), "record");
      if (!rc) rc = check_hip(hipEventSynchronize(b), "sync");
      float el = 0.f;
      if (!rc) rc = check_hip(hipEventElapsedTime(&el, a, b), "elapsed");
      ms.push_back(el);
    }
    if (rc) break;
    std::sort(ms.begin(), ms.end());
    if (ms[1] < best_ms) {
      best_ms = ms[1];
      best = c;
    }
  }
  (void)hipEventDestroy(a);
  (void)hipEventDestroy(b);
  if (rc) return rc;
  if (best < 0) return set_error(FP_ENOTIMPL, "no launch choice fits");
  {
    std::lock_guard<std::mutex> lk(g_mu);
    g_table[Key(arch_name(), ens->ansatz, ens->n_qubits, ens->depth, precision)] = Entry{choice_launch(best), best_ms};
  }
  *out_choice = best;
  return FP_OK;
}

int fp_autotune_table(char* buf, size_t cap) {
  if (!buf || cap == 0) return set_error(FP_EINVAL, "NULL buffer");
  std::string out;
  {
    std::lock_guard<std::mutex> lk(g_mu);
    for (const auto& kv : g_table) {
      char line[256];
      snprintf(line, sizeof(line), "%s %d %d %d %d %s %.0f %.6f\n", std::get<0>(kv.first).c_str(),
               std::get<1>(kv.first), std::get<2>(kv.first), std::get<3>(kv.first), std::get<4>(kv.first),
               class_name(kv.second.launch.cls), kv.second.launch.task_flops, kv.second.ms);
      out += line;
    }
  }
  if (out.size() + 1 > cap) return set_error(FP_EINVAL, "buffer of %zu bytes too small (%zu needed)", cap, out.size() + 1);
  memcpy(buf, out.c_str(), out.size() + 1);
  return FP_OK;
}

int fp_autotune_load(const char* text) {
  if (!text) return set_error(FP_EINVAL, "NULL text");
  std::map<Key, Entry> add;
  const char* p = text;
  while (*p) {
    const char* e = strchr(p, '\n');
    std::string line = e ? std::string(p, e - p) : std::string(p);
    p = e ? e + 1 : p + line.size();
    if (line.empty() || line[0] == '#') continue;
    char arch[64], cname[16];
    int an, n, d, pr;
    double tf, ms;
    if (sscanf(line.c_str(), "%63s %d %d %d %d %15s %lf %lf", arch, &an, &n, &d, &pr, cname, &tf, &ms) != 8)
      return set_error(FP_EINVAL, "bad tuning line: %s", line.c_str());
    int c = -1;
    for (int k = 0; k < PCLASS_COUNT; ++k)
      if (strcmp(cname, CLASS_NAMES[k]) == 0) c = k;
    if (c < 0) return set_error(FP_EINVAL, "unknown lane class %s", cname);
    if (!(tf >= 1.0 && tf <= 1e12)) return set_error(FP_EINVAL, "task flops %g outside 1 .. 1e12", tf);
    add[Key(arch, an, n, d, pr)] = Entry{GroupLaunch{c, tf}, ms};
  }
  std::lock_guard<std::mutex> lk(g_mu);
  for (const auto& kv : add) g_table[kv.first] = kv.second;
  return FP_OK;
}

}  // extern "C"
