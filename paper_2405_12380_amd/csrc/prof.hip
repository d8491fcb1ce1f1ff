// Optional per-kernel timing: when enabled for a kernel class, the launchers of
// that class bracket each launch with a pair of HIP events on the launch stream
// and record the algorithmic bytes that launch must move.  Reading the totals
// synchronizes on the recorded events.  Disabled by default (no events).  Each
// event pair adds a few microseconds between dependent launches, so a timing
// run enables only the classes it reports.
#include <hip/hip_runtime.h>

#include <mutex>
#include <stdint.h>
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

// dst = src, 16 bytes per lane per step, non-temporal loads and stores (the
// copy streams past the caches, as a bandwidth ceiling should)
typedef unsigned int cp_u4 __attribute__((ext_vector_type(4)));
__global__ __launch_bounds__(256) void k_stream_copy(size_t n16, const cp_u4* __restrict__ src, cp_u4* __restrict__ dst) {
  const size_t stride = (size_t)gridDim.x * blockDim.x;
  size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x;
  for (; i + 3 * stride < n16; i += 4 * stride) {  // four loads in flight per lane
    cp_u4 v[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) v[u] = __builtin_nontemporal_load(src + i + u * stride);
#pragma unroll
    for (int u = 0; u < 4; ++u) __builtin_nontemporal_store(v[u], dst + i + u * stride);
  }
  for (; i < n16; i += stride) __builtin_nontemporal_store(__builtin_nontemporal_load(src + i), dst + i);
}

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

helm_status helm_stream_copy(const void* src, void* dst, size_t bytes, void* stream) {
  if (!src || !dst || bytes == 0 || bytes % 16 != 0 || ((uintptr_t)src | (uintptr_t)dst) % 16 != 0)
    return fail(HELM_E_INVAL, "helm_stream_copy: NULL pointer, or size or address not a multiple of 16");
  if ((const char*)src < (const char*)dst + bytes && (const char*)dst < (const char*)src + bytes)
    return fail(HELM_E_INVAL, "helm_stream_copy: the buffers overlap");
  const size_t n16 = bytes / 16;
  size_t nb = (n16 + 4 * 256 - 1) / (4 * 256);
  if (nb > 8192) nb = 8192;  // 32 workgroups per CU; the loop strides over the rest
  hipLaunchKernelGGL(k_stream_copy, dim3((unsigned)nb), dim3(256), 0, (hipStream_t)stream, n16, (const cp_u4*)src,
                     (cp_u4*)dst);
  return launch_check("helm_stream_copy");
}

}  // extern "C"
