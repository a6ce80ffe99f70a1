// Optional HIP-event timing of the launches of the hot path, for roofline
// reporting.  While enabled, every sweep, planning, matrix-preparation and
// sampling launch is bracketed by a pair of events on its stream, and its
// algorithmic flop and byte counts are recorded with it.
#include <hip/hip_runtime.h>

#include <mutex>
#include <vector>

#include "internal.h"
#include "sweep.h"

namespace fp {

struct Rec {
  int kclass;
  hipEvent_t a, b;
  double flops, bytes;
};

static std::mutex g_mu;
static bool g_on = false;
static std::vector<Rec> g_recs;
static Rec g_open;
static bool g_has_open = false;

bool profiling() { return g_on; }

void profile_launch_begin(int kclass, hipStream_t s) {
  if (!g_on) return;
  std::lock_guard<std::mutex> lk(g_mu);
  g_open.kclass = kclass;
  g_open.flops = 0.0;
  g_open.bytes = 0.0;
  (void)hipEventCreate(&g_open.a);
  (void)hipEventCreate(&g_open.b);
  (void)hipEventRecord(g_open.a, s);
  g_has_open = true;
}

void profile_launch_end(int kclass, double flops, hipStream_t s, double bytes) {
  if (!g_on) return;
  std::lock_guard<std::mutex> lk(g_mu);
  if (!g_has_open || g_open.kclass != kclass) return;
  (void)hipEventRecord(g_open.b, s);
  g_open.flops = flops;
  g_open.bytes = bytes;
  g_recs.push_back(g_open);
  g_has_open = false;
}

}  // namespace fp

using namespace fp;

extern "C" {

int fp_profile_begin(void) {
  std::lock_guard<std::mutex> lk(g_mu);
  for (Rec& r : g_recs) {
    (void)hipEventDestroy(r.a);
    (void)hipEventDestroy(r.b);
  }
  g_recs.clear();
  g_on = true;
  return FP_OK;
}

int fp_profile_end(double* kernel_ms, int64_t* launches, double* flops, double* bytes) {
  std::lock_guard<std::mutex> lk(g_mu);
  g_on = false;
  for (int c = 0; c < KCLASS_COUNT; ++c) {
    if (kernel_ms) kernel_ms[c] = 0.0;
    if (launches) launches[c] = 0;
    if (flops) flops[c] = 0.0;
    if (bytes) bytes[c] = 0.0;
  }
  int rc = FP_OK;
  for (Rec& r : g_recs) {
    hipError_t e = hipEventSynchronize(r.b);
    if (e != hipSuccess && !rc) rc = check_hip(e, "profile sync");
    float ms = 0.f;
    e = hipEventElapsedTime(&ms, r.a, r.b);
    if (e != hipSuccess && !rc) rc = check_hip(e, "profile elapsed");
    const double f = r.flops;
    if (kernel_ms) kernel_ms[r.kclass] += ms;
    if (launches) launches[r.kclass] += 1;
    if (flops) flops[r.kclass] += f;
    if (bytes) bytes[r.kclass] += r.bytes;
    (void)hipEventDestroy(r.a);
    (void)hipEventDestroy(r.b);
  }
  g_recs.clear();
  return rc;
}

}  // extern "C"
