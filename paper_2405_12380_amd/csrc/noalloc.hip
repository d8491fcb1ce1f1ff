// Relaxation sweeps that allocate no device memory (helm_relax_noalloc), for
// callers that cannot allocate: code under HIP graph capture, tight serving
// loops, harnesses that forbid allocation.
//
// helm_relax ping-pongs its sweeps through a field of op-owned scratch that is
// allocated on first use.  This variant runs the same kernels with that field
// in a file-scope device array instead.  Every GPU the library runs on holds
// one copy of the array (NOALLOC_SCRATCH_BYTES) until the process ends; its
// device address is looked up once per device, with that device current, and
// only that address is ever handed to kernels.  Each sweep overwrites every
// node of its output, so nothing in the array needs clearing between calls.
#include <hip/hip_runtime.h>

#include <cmath>
#include <mutex>

#include "internal.h"
#include "lib.h"

namespace helm {

static constexpr size_t NOALLOC_SCRATCH_BYTES = (size_t)64 << 20;  // one field: 4 Mi nodes c128, 8 Mi c64
static constexpr int NOALLOC_MAX_DEVICES = 64;

static __device__ __align__(256) unsigned char scratch[NOALLOC_SCRATCH_BYTES];

static std::mutex g_scratch_mu;
static void* g_scratch_dev[NOALLOC_MAX_DEVICES];  // device address of `scratch`, per device

// The current device's copy of the scratch array (looked up on first use).
static helm_status scratch_address(void** out) {
  int dev = -1;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return hip_fail(e, "helm_relax_noalloc: hipGetDevice");
  if (dev < 0 || dev >= NOALLOC_MAX_DEVICES)
    return fail(HELM_E_INVAL, "helm_relax_noalloc: device %d beyond the %d supported", dev, NOALLOC_MAX_DEVICES);
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch_dev[dev]) {
    void* p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p) return hip_fail(e, "helm_relax_noalloc: hipGetSymbolAddress(scratch)");
    g_scratch_dev[dev] = p;
  }
  *out = g_scratch_dev[dev];
  return HELM_OK;
}

template <typename S>
static helm_status relax_static(helm_op_s* op, int kind, double omega, int sweeps, const void* f, void* u, void* tmp,
                                hipStream_t st) {
  void* a = u;
  void* b = tmp;
  for (int k = 0; k < sweeps; ++k) {
    if (kind == HELM_RBGS) stencil_rbgs_fused<S>(op->geom, op->sc, op->code, f, a, b, omega, st);
    else stencil_jacobi<S>(op->geom, op->sc, op->code, f, a, b, omega, st);
    void* t = a;
    a = b;
    b = t;
  }
  if (a != u) copy_vec<S>(op->nn, a, u, st);
  return launch_check("helm_relax_noalloc");
}

}  // namespace helm

using namespace helm;

extern "C" helm_status helm_relax_noalloc(helm_op op, int kind, double omega, int sweeps, const void* f, void* u,
                                          void* stream) {
  if (!op || !f || !u) return fail(HELM_E_INVAL, "helm_relax_noalloc: NULL argument");
  if (kind != HELM_JACOBI && kind != HELM_RBGS) return fail(HELM_E_INVAL, "helm_relax_noalloc: unknown kind %d", kind);
  if (sweeps < 0) return fail(HELM_E_INVAL, "helm_relax_noalloc: sweeps < 0");
  if (!std::isfinite(omega)) return fail(HELM_E_INVAL, "helm_relax_noalloc: omega not finite");
  if (f == u) return fail(HELM_E_INVAL, "helm_relax_noalloc: f and u alias");
  const size_t bytes = op->nn * op_esz(op);
  if (bytes > NOALLOC_SCRATCH_BYTES)
    return fail(HELM_E_INVAL, "helm_relax_noalloc: a field of %zu bytes exceeds the %zu-byte static scratch", bytes,
                NOALLOC_SCRATCH_BYTES);
  if (sweeps == 0) return HELM_OK;
  void* tmp = nullptr;
  helm_status s = scratch_address(&tmp);
  if (s) return s;
  hipStream_t st = (hipStream_t)stream;
  return op->dt == HELM_C128 ? relax_static<double>(op, kind, omega, sweeps, f, u, tmp, st)
                             : relax_static<float>(op, kind, omega, sweeps, f, u, tmp, st);
}
