// Optional per-kernel timing: when enabled for a kernel class, the launchers of
// that class bracket each launch with a pair of HIP events on the launch stream
// and record the algorithmic bytes that launch must move.  Reading the totals
// synchronizes on the recorded events.  Disabled by default (no events).  Each
// event pair adds a few microseconds between dependent launches, so a timing
// run enables only the classes it reports.
#include <hip/hip_runtime.h>

#include <mutex>
#include <vector>

#include "helm.h"
#include "lib.h"
#include "prof.h"

namespace helm {

namespace {
struct Rec {
  hipEvent_t a, b;
  double bytes;
};
struct Prof {
  unsigned mask = 0;
  std::vector<Rec> recs[KP_COUNT];
  std::vector<hipEvent_t> pool;
  std::mutex mu;
  hipEvent_t take() {
    if (!pool.empty()) {
      hipEvent_t e = pool.back();
      pool.pop_back();
      return e;
    }
    // timing-only events: no system-scope cache writeback and invalidation at
    // each record, which would otherwise sit inside the measured interval and
    // slow the kernel that follows
    hipEvent_t e = nullptr;
    (void)hipEventCreateWithFlags(&e, hipEventDisableSystemFence);
    return e;
  }
  void clear() {
    for (auto& v : recs) {
      for (auto& r : v) {
        pool.push_back(r.a);
        pool.push_back(r.b);
      }
      v.clear();
    }
  }
};
Prof g_prof;
thread_local hipEvent_t t_start = nullptr;
}  // namespace

bool kprof_on() { return g_prof.mask != 0; }

void kprof_begin(int kind, hipStream_t st) {
  if (!((g_prof.mask >> kind) & 1u)) return;
  std::lock_guard<std::mutex> lk(g_prof.mu);
  t_start = g_prof.take();
  (void)hipEventRecord(t_start, st);
}

void kprof_end(int kind, double bytes, hipStream_t st) {
  if (!((g_prof.mask >> kind) & 1u) || !t_start) return;
  std::lock_guard<std::mutex> lk(g_prof.mu);
  hipEvent_t e = g_prof.take();
  (void)hipEventRecord(e, st);
  g_prof.recs[kind].push_back(Rec{t_start, e, bytes});
  t_start = nullptr;
}

}  // namespace helm

using namespace helm;

extern "C" {

helm_status helm_kprof_enable(int mask) {
  std::lock_guard<std::mutex> lk(g_prof.mu);
  if (hipDeviceSynchronize() != hipSuccess) return fail(HELM_E_HIP, "helm_kprof_enable: device sync failed");
  g_prof.clear();
  g_prof.mask = (unsigned)mask & ((1u << KP_COUNT) - 1u);
  return HELM_OK;
}

helm_status helm_kprof_read(int kind, int* count, double* total_ms, double* total_bytes) {
  if (kind < 0 || kind >= KP_COUNT || !count || !total_ms || !total_bytes)
    return fail(HELM_E_INVAL, "helm_kprof_read: bad argument");
  std::lock_guard<std::mutex> lk(g_prof.mu);
  double ms = 0.0, by = 0.0;
  for (auto& r : g_prof.recs[kind]) {
    if (hipEventSynchronize(r.b) != hipSuccess) return fail(HELM_E_HIP, "helm_kprof_read: event sync");
    float t = 0.f;
    if (hipEventElapsedTime(&t, r.a, r.b) != hipSuccess) return fail(HELM_E_HIP, "helm_kprof_read: elapsed");
    ms += t;
    by += r.bytes;
  }
  *count = (int)g_prof.recs[kind].size();
  *total_ms = ms;
  *total_bytes = by;
  return HELM_OK;
}

}  // extern "C"
