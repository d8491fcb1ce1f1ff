// Caching allocator for the library's device buffers and pinned host mirrors.
//
// A solve on a fresh operator needs the operator's fields, the coarse space's
// work buffers (hundreds of MB at 64^3) and the solver workspace; allocating
// and releasing them with hipMalloc / hipFree on every operator costs more
// than a millisecond per solve in page mapping and unmapping.  Freed blocks
// are kept instead, per device and per rounded size, and handed out again for
// requests of the same rounded size.
//
// Release keeps hipFree's ordering: the device is synchronized before a block
// joins the cache, so a block is never handed out while work that used it can
// still be in flight.  When the cached bytes would exceed the soft cap, the
// block is returned to the runtime instead; when an allocation fails, the
// cache is emptied and the allocation tried once more.
#include <hip/hip_runtime.h>

#include <map>
#include <mutex>
#include <unordered_map>
#include <vector>

#include "lib.h"

namespace helm {

namespace {

constexpr size_t POOL_SOFT_CAP = (size_t)48 << 30;  // bytes kept in the cache, all devices

size_t round_size(size_t bytes) {
  if (bytes == 0) bytes = 256;
  if (bytes >= ((size_t)1 << 20)) return (bytes + ((size_t)2 << 20) - 1) & ~(((size_t)2 << 20) - 1);
  size_t r = 256;
  while (r < bytes) r <<= 1;
  return r;
}

struct Pool {
  std::mutex mu;
  // (device, rounded size) -> free blocks
  std::map<std::pair<int, size_t>, std::vector<void*>> free_dev, free_host;
  // live block -> (device, rounded size)
  std::unordered_map<void*, std::pair<int, size_t>> live_dev, live_host;
  size_t cached = 0;

  void drain() {  // return every cached block to the runtime (caller holds mu)
    for (auto& kv : free_dev)
      for (void* p : kv.second) (void)hipFree(p);
    for (auto& kv : free_host)
      for (void* p : kv.second) (void)hipHostFree(p);
    free_dev.clear();
    free_host.clear();
    cached = 0;
  }
};

Pool& pool() {
  static Pool* p = new Pool();  // never destroyed: blocks may be released during process exit
  return *p;
}

int current_device() {
  int d = 0;
  if (hipGetDevice(&d) != hipSuccess) d = 0;
  return d;
}

}  // namespace

helm_status dalloc(void** p, size_t bytes) {
  *p = nullptr;
  const size_t r = round_size(bytes);
  const int dev = current_device();
  Pool& P = pool();
  std::lock_guard<std::mutex> lk(P.mu);
  auto it = P.free_dev.find({dev, r});
  if (it != P.free_dev.end() && !it->second.empty()) {
    *p = it->second.back();
    it->second.pop_back();
    P.cached -= r;
    P.live_dev[*p] = {dev, r};
    return HELM_OK;
  }
  hipError_t e = hipMalloc(p, r);
  if (e != hipSuccess) {
    (void)hipGetLastError();
    P.drain();
    e = hipMalloc(p, r);
  }
  if (e != hipSuccess) {
    (void)hipGetLastError();
    *p = nullptr;
    return fail(HELM_E_NOMEM, "hipMalloc(%zu bytes) failed: %s", r, hipGetErrorString(e));
  }
  P.live_dev[*p] = {dev, r};
  return HELM_OK;
}

void dfree(void* p) {
  if (!p) return;
  Pool& P = pool();
  std::lock_guard<std::mutex> lk(P.mu);
  auto it = P.live_dev.find(p);
  if (it == P.live_dev.end()) {  // not from dalloc
    (void)hipFree(p);
    return;
  }
  const auto key = it->second;
  P.live_dev.erase(it);
  // hipFree's ordering: nothing still in flight may use the block once it is reusable
  if (hipDeviceSynchronize() != hipSuccess || P.cached + key.second > POOL_SOFT_CAP) {
    (void)hipGetLastError();
    (void)hipFree(p);
    return;
  }
  P.free_dev[key].push_back(p);
  P.cached += key.second;
}

helm_status halloc_mapped(void** p, size_t bytes) {
  *p = nullptr;
  const size_t r = round_size(bytes);
  Pool& P = pool();
  std::lock_guard<std::mutex> lk(P.mu);
  auto it = P.free_host.find({-1, r});
  if (it != P.free_host.end() && !it->second.empty()) {
    *p = it->second.back();
    it->second.pop_back();
    P.cached -= r;
    P.live_host[*p] = {-1, r};
    return HELM_OK;
  }
  hipError_t e = hipHostMalloc(p, r, hipHostMallocMapped);
  if (e != hipSuccess) {
    (void)hipGetLastError();
    *p = nullptr;
    return hip_fail(e, "hipHostMalloc");
  }
  P.live_host[*p] = {-1, r};
  return HELM_OK;
}

void hfree_mapped(void* p) {
  if (!p) return;
  Pool& P = pool();
  std::lock_guard<std::mutex> lk(P.mu);
  auto it = P.live_host.find(p);
  if (it == P.live_host.end()) {
    (void)hipHostFree(p);
    return;
  }
  const auto key = it->second;
  P.live_host.erase(it);
  if (hipDeviceSynchronize() != hipSuccess) {
    (void)hipGetLastError();
    (void)hipHostFree(p);
    return;
  }
  P.free_host[key].push_back(p);
  P.cached += key.second;
}

}  // namespace helm
