// C ABI of libhelm: handles, argument validation, workspace, and the solver
// drivers (relaxation, GMRES(m)-CGS2, BiCGStab, the relaxation meta-solver of
// eq. 3 and the trunk-basis Krylov meta-solvers of §3.1.2 / App. C).
//
// Every numerical step runs in the HIP kernels of this library; host code
// only sequences launches and reads back the scalars that decide control flow
// (convergence flags, breakdown flags).
#include "helm.h"

#include <hip/hip_runtime.h>

#include <chrono>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "internal.h"
#include "lib.h"

namespace helm {

thread_local std::string g_last_error;

helm_status fail(helm_status s, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  g_last_error = buf;
  return s;
}

helm_status hip_fail(hipError_t e, const char* what) {
  return fail(HELM_E_HIP, "%s: %s", what, hipGetErrorString(e));
}

helm_status Buffer::ensure(size_t bytes) {
  if (bytes <= cap) return HELM_OK;
  dfree(ptr);
  ptr = nullptr;
  cap = 0;
  helm_status s = dalloc(&ptr, bytes);
  if (s == HELM_OK) cap = bytes;
  return s;
}
void Buffer::release() {
  dfree(ptr);
  ptr = nullptr;
  cap = 0;
}

helm_status launch_check(const char* what) {
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return hip_fail(e, what);
  return HELM_OK;
}

helm_status sync_stream(hipStream_t st, const char* what) {
  hipError_t e = hipStreamSynchronize(st);
  if (e != hipSuccess) return hip_fail(e, what);
  return launch_check(what);
}

}  // namespace helm

using namespace helm;

// ---------------------------------------------------------------------------
// helpers on the op
// ---------------------------------------------------------------------------
namespace helm {

size_t op_esz(const helm_op_s* op) { return op->dt == HELM_C128 ? 16 : 8; }

// Partial-sum scratch big enough for `doubles` values.
helm_status op_part(helm_op_s* op, size_t doubles, double** out) {
  helm_status s = op->part.ensure(doubles * sizeof(double));
  *out = (double*)op->part.ptr;
  return s;
}

}  // namespace helm

// ---------------------------------------------------------------------------
// C ABI: operator
// ---------------------------------------------------------------------------
extern "C" {

const char* helm_strerror(helm_status s) {
  switch (s) {
    case HELM_OK: return "ok";
    case HELM_NOT_CONVERGED: return "not converged";
    case HELM_E_INVAL: return "invalid argument";
    case HELM_E_NOMEM: return "out of device memory";
    case HELM_E_HIP: return "HIP runtime error";
    case HELM_E_BREAKDOWN: return "Krylov breakdown";
    case HELM_E_NONFINITE: return "non-finite residual";
    case HELM_E_SINGULAR: return "singular coarse matrix";
  }
  return "unknown status";
}

const char* helm_last_error(void) { return g_last_error.c_str(); }

helm_status helm_setup(const helm_grid* g, helm_dtype dt, const double* ksq, const double* alpha,
                       const uint8_t* mask, void* stream, helm_op* out) {
  if (!out) return fail(HELM_E_INVAL, "helm_setup: out is NULL");
  *out = nullptr;
  if (!g || !ksq || !alpha || !mask) return fail(HELM_E_INVAL, "helm_setup: NULL argument");
  if (g->dim != 2 && g->dim != 3) return fail(HELM_E_INVAL, "helm_setup: dim must be 2 or 3 (got %d)", g->dim);
  if (dt != HELM_C64 && dt != HELM_C128) return fail(HELM_E_INVAL, "helm_setup: unknown dtype %d", (int)dt);
  size_t nn = 1;
  for (int a = 0; a < g->dim; ++a) {
    if (g->n[a] < 3) return fail(HELM_E_INVAL, "helm_setup: n[%d] = %d < 3", a, g->n[a]);
    nn *= (size_t)g->n[a];
  }
  if (nn > ((size_t)1 << 31)) return fail(HELM_E_INVAL, "helm_setup: %zu nodes exceeds 2^31", nn);
  hipStream_t st = (hipStream_t)stream;
  helm_op_s* op = new helm_op_s();
  op->dim = g->dim;
  for (int a = 0; a < 3; ++a) op->n[a] = a < g->dim ? g->n[a] : 1;
  op->nn = nn;
  op->dt = dt;
  op->geom = make_geom(g->dim, op->n, 0);
  helm_status s;
  if ((s = dalloc(&op->sc, nn * op_esz(op))) || (s = dalloc((void**)&op->mask, nn)) ||
      (s = dalloc((void**)&op->alpha, nn * sizeof(double))) || (s = dalloc((void**)&op->code, (nn + 3) & ~(size_t)3)) ||
      (s = dalloc((void**)&op->red, 4096 * sizeof(double)))) {
    helm_destroy(op);
    return s;
  }
  if ((s = halloc_mapped((void**)&op->host, 4096 * sizeof(double)))) {
    helm_destroy(op);
    return s;
  }
  hipError_t e = hipHostGetDevicePointer((void**)&op->host_dev, op->host, 0);
  if (e != hipSuccess) {
    helm_destroy(op);
    return hip_fail(e, "hipHostGetDevicePointer");
  }
  // inputs in host (the documented case) or device memory: each copy takes its
  // direction from the pointer; k^2 is staged in the op's field scratch
  if ((s = op->tmp.ensure(nn * op_esz(op)))) {
    helm_destroy(op);
    return s;
  }
  double* ksq_dev = (double*)op->tmp.ptr;
  e = hipMemcpyAsync(op->mask, mask, nn, hipMemcpyDefault, st);
  if (e == hipSuccess) e = hipMemcpyAsync(op->alpha, alpha, nn * sizeof(double), hipMemcpyDefault, st);
  if (e == hipSuccess) e = hipMemcpyAsync(ksq_dev, ksq, nn * sizeof(double), hipMemcpyDefault, st);
  if (e != hipSuccess) {
    helm_destroy(op);
    return hip_fail(e, "helm_setup: input copy");
  }
  if (dt == HELM_C128) build_s<double>(nn, ksq_dev, op->alpha, op->sc, st);
  else build_s<float>(nn, ksq_dev, op->alpha, op->sc, st);
  build_codes(op->geom, op->mask, op->code, st);
  if ((s = sync_stream(st, "helm_setup"))) {
    helm_destroy(op);
    return s;
  }
  *out = op;
  return HELM_OK;
}

helm_status helm_set_ksq(helm_op op, const double* ksq, void* stream) {
  if (!op || !ksq) return fail(HELM_E_INVAL, "helm_set_ksq: NULL argument");
  hipStream_t st = (hipStream_t)stream;
  if (op->dt == HELM_C128) build_s<double>(op->nn, ksq, op->alpha, op->sc, st);
  else build_s<float>(op->nn, ksq, op->alpha, op->sc, st);
  helm_status s = sync_stream(st, "helm_set_ksq");
  if (s) return s;
  op->ksq_version++;
  return HELM_OK;
}

void helm_destroy(helm_op op) {
  if (!op) return;
  mg_release(op);
  coarse_release(op);
  dfree(op->sc);
  dfree(op->mask);
  dfree(op->code);
  dfree(op->alpha);
  dfree(op->red);
  hfree_mapped(op->host);
  op->tmp.release();
  op->part.release();
  op->ws.release();
  op->adj.release();
  delete op;
}

size_t helm_size(helm_op op) { return op ? op->nn : 0; }

helm_status helm_apply(helm_op op, const void* x, void* y, void* stream) {
  if (!op || !x || !y) return fail(HELM_E_INVAL, "helm_apply: NULL argument");
  if (x == y) return fail(HELM_E_INVAL, "helm_apply: x and y alias");
  hipStream_t st = (hipStream_t)stream;
  if (op->dt == HELM_C128) stencil_apply<double>(op->geom, op->sc, op->code, x, y, st);
  else stencil_apply<float>(op->geom, op->sc, op->code, x, y, st);
  return launch_check("helm_apply");
}

helm_status helm_residual(helm_op op, const void* f, const void* u, void* r, double* rnorm, void* stream) {
  if (!op || !f || !u || !r) return fail(HELM_E_INVAL, "helm_residual: NULL argument");
  if (r == f || r == u) return fail(HELM_E_INVAL, "helm_residual: r aliases an input");
  hipStream_t st = (hipStream_t)stream;
  return op->dt == HELM_C128 ? residual_norm<double>(op, f, u, r, rnorm, st)
                             : residual_norm<float>(op, f, u, r, rnorm, st);
}

helm_status helm_tune(helm_op op, int fixed_ty, void* stream, int* ty_out, int* zb_out, double* us_out) {
  if (!op) return fail(HELM_E_INVAL, "helm_tune: NULL op");
  if (fixed_ty != 0 && fixed_ty != 4 && fixed_ty != 8) return fail(HELM_E_INVAL, "helm_tune: tile height %d", fixed_ty);
  hipStream_t st = (hipStream_t)stream;
  const size_t fld = op->nn * op_esz(op);
  helm_status s;
  if ((s = op->tmp.ensure(fld)) || (s = op->ws.ensure(fld))) return s;
  void* x = op->tmp.ptr;
  void* y = op->ws.ptr;
  const bool c128 = op->dt == HELM_C128;
  if (c128) zero_vec<double>(op->nn, x, st);
  else zero_vec<float>(op->nn, x, st);
  hipEvent_t e0, e1;
  if (hipEventCreate(&e0) != hipSuccess) return fail(HELM_E_HIP, "helm_tune: event");
  if (hipEventCreate(&e1) != hipSuccess) {
    (void)hipEventDestroy(e0);
    return fail(HELM_E_HIP, "helm_tune: event");
  }
  StencilGeom best = op->geom;
  double best_us = INFINITY;
  const int tys[2] = {4, 8};
  const int zbs[6] = {1, 2, 4, 8, 16, 32};
  for (int a = 0; a < 2; ++a) {
    if (fixed_ty && tys[a] != fixed_ty) continue;
    for (int b = 0; b < 6; ++b) {
      if (op->dim == 2 && zbs[b] != 1) continue;
      if (zbs[b] > op->geom.nz) continue;
      for (int v = 0; v < 4; ++v) {  // plain / non-temporal stores, one / two rows per thread
        const int nt = v & 1, rows = 1 + (v >> 1);
        if (rows == 2 && op->dim != 3) continue;
        StencilGeom g = op->geom;
        g.ty = tys[a];
        g.zb = zbs[b];
        g.nt = nt != 0;
        g.rows = rows;
        auto run = [&]() {
          if (c128) stencil_apply<double>(g, op->sc, op->code, x, y, st);
          else stencil_apply<float>(g, op->sc, op->code, x, y, st);
        };
        run();
        run();
        (void)hipEventRecord(e0, st);
        for (int k = 0; k < 8; ++k) run();
        (void)hipEventRecord(e1, st);
        if (hipEventSynchronize(e1) != hipSuccess) {
          (void)hipEventDestroy(e0);
          (void)hipEventDestroy(e1);
          return launch_check("helm_tune");
        }
        float ms = 0.f;
        (void)hipEventElapsedTime(&ms, e0, e1);
        const double us = 1e3 * ms / 8;
        if (us < best_us) {
          best_us = us;
          best = g;
        }
      }
    }
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if ((s = launch_check("helm_tune"))) return s;
  op->geom = best;
  if (ty_out) *ty_out = best.ty;
  if (zb_out) *zb_out = best.zb;
  if (us_out) *us_out = best_us;
  return HELM_OK;
}

helm_status helm_set_rbgs_kernel(helm_op op, int which) {
  if (!op) return fail(HELM_E_INVAL, "helm_set_rbgs_kernel: NULL op");
  if (which < HELM_RB_AUTO || which > HELM_RB_PAIRS)
    return fail(HELM_E_INVAL, "helm_set_rbgs_kernel: unknown kernel %d", which);
  if (which == HELM_RB_RING) {
    if (op->dim != 3) return fail(HELM_E_INVAL, "helm_set_rbgs_kernel: the ring kernel is 3D only");
    if ((double)op->nn * op_esz(op) >= 2147483648.0)
      return fail(HELM_E_INVAL, "helm_set_rbgs_kernel: the ring kernel needs fields under 2 GiB");
  }
  op->geom.rb = which;
  return HELM_OK;
}

helm_status helm_relax(helm_op op, int kind, double omega, int sweeps, const void* f, void* u, void* stream) {
  if (!op || !f || !u) return fail(HELM_E_INVAL, "helm_relax: NULL argument");
  if (kind != HELM_JACOBI && kind != HELM_RBGS) return fail(HELM_E_INVAL, "helm_relax: unknown kind %d", kind);
  if (sweeps < 0) return fail(HELM_E_INVAL, "helm_relax: sweeps < 0");
  if (!std::isfinite(omega)) return fail(HELM_E_INVAL, "helm_relax: omega not finite");
  if (f == u) return fail(HELM_E_INVAL, "helm_relax: f and u alias");
  hipStream_t st = (hipStream_t)stream;
  return op->dt == HELM_C128 ? relax<double>(op, kind, omega, sweeps, f, u, st)
                             : relax<float>(op, kind, omega, sweeps, f, u, st);
}

helm_status helm_dot(helm_op op, const void* x, const void* y, double out[2], void* stream) {
  if (!op || !x || !y || !out) return fail(HELM_E_INVAL, "helm_dot: NULL argument");
  hipStream_t st = (hipStream_t)stream;
  double* part;
  const int nb = red_nblocks(op->nn);
  helm_status s = op_part(op, 2 * (size_t)nb, &part);
  if (s) return s;
  if (op->dt == HELM_C128) dot_part<double>(op->nn, x, y, part, st);
  else dot_part<float>(op->nn, x, y, part, st);
  reduce_cols(part, nb, 2, op->red, st);
  hipError_t e = hipMemcpyAsync(op->host, op->red, 2 * sizeof(double), hipMemcpyDeviceToHost, st);
  if (e != hipSuccess) return hip_fail(e, "helm_dot readback");
  if ((s = sync_stream(st, "helm_dot"))) return s;
  out[0] = op->host[0];
  out[1] = op->host[1];
  return HELM_OK;
}

helm_status helm_nrm2(helm_op op, const void* x, double* out, void* stream) {
  if (!op || !x || !out) return fail(HELM_E_INVAL, "helm_nrm2: NULL argument");
  hipStream_t st = (hipStream_t)stream;
  return op->dt == HELM_C128 ? vec_norm<double>(op, x, out, st) : vec_norm<float>(op, x, out, st);
}

}  // extern "C"
