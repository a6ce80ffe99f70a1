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
  int deferred;  // index into g_pinned of a MAC count copied from the device, or -1
};

// Pinned host slots that receive MAC counts known only on the device (the
// launches that do not wait for their plans); read at fp_profile_end.
constexpr int PINNED_SLOTS = 1 << 14;
static double* g_pinned = nullptr;
static int g_pinned_used = 0;

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
  g_open.deferred = -1;
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

void profile_launch_end_dev(int kclass, const double* d_macs, hipStream_t s) {
  if (!g_on) return;
  std::lock_guard<std::mutex> lk(g_mu);
  if (!g_has_open || g_open.kclass != kclass) return;
  (void)hipEventRecord(g_open.b, s);
  g_open.flops = 0.0;
  g_open.bytes = 0.0;
  g_open.deferred = -1;
  if (!g_pinned) (void)hipHostMalloc((void**)&g_pinned, sizeof(double) * PINNED_SLOTS, hipHostMallocDefault);
  if (g_pinned && g_pinned_used < PINNED_SLOTS &&
      hipMemcpyAsync(g_pinned + g_pinned_used, d_macs, sizeof(double), hipMemcpyDeviceToHost, s) == hipSuccess)
    g_open.deferred = g_pinned_used++;
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
  g_pinned_used = 0;
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
  if (g_pinned_used > 0) {  // the deferred counts are copied after their launches' end events
    hipError_t e = hipDeviceSynchronize();
    if (e != hipSuccess) rc = check_hip(e, "profile sync (deferred counts)");
  }
  for (Rec& r : g_recs) {
    hipError_t e = hipEventSynchronize(r.b);
    if (e != hipSuccess && !rc) rc = check_hip(e, "profile sync");
    float ms = 0.f;
    e = hipEventElapsedTime(&ms, r.a, r.b);
    if (e != hipSuccess && !rc) rc = check_hip(e, "profile elapsed");
    // 8 real flops per complex MAC
    const double f = r.deferred >= 0 ? 8.0 * g_pinned[r.deferred] : r.flops;
    if (kernel_ms) kernel_ms[r.kclass] += ms;
    if (launches) launches[r.kclass] += 1;
    if (flops) flops[r.kclass] += f;
    if (bytes) bytes[r.kclass] += r.bytes;
    (void)hipEventDestroy(r.a);
    (void)hipEventDestroy(r.b);
  }
  g_recs.clear();
  g_pinned_used = 0;
  return rc;
}

}  // extern "C"
