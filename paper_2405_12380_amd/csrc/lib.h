// Host-side internals of libhelm: handle layouts, device buffers, error
// helpers, and the driver entry points shared by the translation units.
#pragma once

#include <hip/hip_runtime.h>

#include <cmath>
#include <string>
#include <vector>

#include "helm.h"
#include "internal.h"

namespace helm {

struct Mg;
helm_status fail(helm_status s, const char* fmt, ...);
helm_status hip_fail(hipError_t e, const char* what);
// Device buffers and pinned host mirrors from the library's caching pool
// (pool.hip): released blocks are kept for reuse; a release synchronizes the
// device first, as hipFree does.
helm_status dalloc(void** p, size_t bytes);
void dfree(void* p);
helm_status halloc_mapped(void** p, size_t bytes);
void hfree_mapped(void* p);
helm_status launch_check(const char* what);
helm_status sync_stream(hipStream_t st, const char* what);

// A growable device allocation (contents are not preserved on growth).
struct Buffer {
  void* ptr = nullptr;
  size_t cap = 0;
  helm_status ensure(size_t bytes);
  void release();
};

// Cached trunk-basis coarse space of one op (App. C).
struct Coarse {
  int net_serial = -1;  // network the space was built from
  int p_used = 0;
  int ksq_version = -1;
  bool valid = false;
  bool q_f32 = false;  // basis stored in fp32
  bool pass1 = false;  // stored basis is the first CholeskyQR pass's Q1 (fp64 path)
  bool pending = false;  // built, but the inverse's record is not yet checked (coarse_finish)
  hipEvent_t ev0 = nullptr, ev1 = nullptr;  // set-up start and end while pending
  int rank = 0;
  double cond_est = 0.0;
  double setup_ms = 0.0;
  Buffer Q;      // n x rank, real (dtype's precision), row-major: the basis the solves use
  Buffer Ainv;   // rank x rank complex128, row-major: inverse of the Galerkin matrix in that basis
  Buffer Ac;     // rank x rank complex128, row-major: that Galerkin matrix
  Buffer T;      // trunk matrix at the op's nodes, n x p (dtype's precision)
  int T_serial = -1;
  Buffer W1, W2;  // setup work (n x p_used fp64 each)
  Buffer small;   // setup work: Gram partials, factors, coarse matrices
  Buffer qpart;   // per-application partials of Q^T r (own buffer: drivers hold op->part)
};

}  // namespace helm

struct helm_op_s {
  int dim = 0;
  int n[3] = {1, 1, 1};
  size_t nn = 0;
  helm_dtype dt = HELM_C128;
  helm::StencilGeom geom{};
  void* sc = nullptr;        // s = k^2 (1 + i alpha), complex in the dtype's precision
  uint8_t* mask = nullptr;   // scatterer indicator
  uint8_t* code = nullptr;   // per-node neighbour code for the stencil kernels
  double* alpha = nullptr;   // sponge profile (kept to rebuild s after helm_set_ksq)
  double* red = nullptr;     // small reduced results (device, 4096 doubles)
  double* host = nullptr;    // pinned host mirror for scalar read-backs (4096 doubles)
  double* host_dev = nullptr;  // the same pinned buffer as seen from the device
  int ksq_version = 0;
  helm::Buffer tmp;          // one field: Jacobi ping-pong
  helm::Buffer part;         // reduction partials
  helm::Buffer ws;           // solver workspace
  helm::Buffer adj;          // one field: the conjugated right-hand side of an adjoint solve
  helm::Coarse coarse;
  helm::Mg* mg = nullptr;    // multigrid hierarchy (mg.hip), built on demand
};

// A loaded DeepONet (deeponet.hip): widths, weights on the device in the
// dtype's real precision (W_l is in x out, row-major), and inference scratch.
// A C64 network also keeps its trunk weights widened to fp64 (tW64, tB64:
// the same values as the fp32 copies), since the trunk matrix is evaluated in
// fp64 arithmetic for both dtypes.
struct don_s {
  helm_dtype dt = HELM_C128;
  int act = DON_TANH, head = DON_SPLIT_OUTPUT, p = 0, k_input = 0;
  int bgrid[3] = {1, 1, 1};
  std::vector<int> bw, tw;
  std::vector<void*> bW, bB, tW, tB;
  std::vector<void*> tW64, tB64;
  int serial = 0;
  helm::Buffer act0, act1;  // branch activations (small) and trunk chunks
  helm::Buffer tact0, tact1;
  helm::Buffer part;
  helm::Buffer coef;        // 2p doubles
};

namespace helm {
size_t op_esz(const helm_op_s* op);
helm_status op_part(helm_op_s* op, size_t doubles, double** out);

// ---- DeepONet (deeponet.hip) ----
// Validate that `net` can act on `op` (grid dimension, dtype) with p_used columns.
helm_status check_net_for_op(const don_s* net, const helm_op_s* op, int p_used);
int don_p(const don_s* net);
int don_serial(const don_s* net);
// A fresh serial number (weights changed: cached trunk matrices and coarse spaces go stale).
void don_touch(don_s* net);
// du = s N(r/s), masked (DON_FULL); async on st
helm_status don_full(don_s* net, helm_op_s* op, const void* r, double k, void* du, hipStream_t st);
// T = trunk(node coordinates) into `out` (n x p real, dtype precision), fp64
// arithmetic for both dtypes; async
helm_status don_trunk(don_s* net, helm_op_s* op, void* out, hipStream_t st);

// ---- coarse space (coarse.hip) ----
// Build or reuse the coarse space; HELM_E_SINGULAR if no_drop and a column was dropped.
// Builds (or reuses) the trunk-basis coarse space.  With defer set, a fresh
// build returns without waiting for the Galerkin inverse: the space is then
// pending and must be settled by coarse_finish before its results are trusted
// (the solver does so at its first wait on later work).
helm_status coarse_ensure(helm_op_s* op, don_s* net, int p_used, bool q_fp32, bool no_drop, hipStream_t st,
                          bool defer = false);
// Settles a pending space: waits for the set-up, checks the inverse's record
// (HELM_E_SINGULAR on a zero pivot or a lost rank), sets cond_est and
// setup_ms.  A no-op when nothing is pending.
helm_status coarse_finish(helm_op_s* op);
// doubles into the op's pinned host buffer where the set-up's inverse record lands
constexpr size_t COARSE_REC = 1024;
template <typename S>
helm_status coarse_correct(helm_op_s* op, const void* r1, void* z, hipStream_t st);  // z += Q A_c^-1 Q^T r1
void coarse_release(helm_op_s* op);
// The orthonormal basis Q (device, n x r fp64, may be NULL) and its Galerkin
// matrix A_c = Q^T A Q (host, complex r x r, may be NULL) of a built coarse
// space whose stored basis is the first CholeskyQR pass's: the second pass is
// run here, for inspection.  Synchronous.
helm_status coarse_orthonormal(helm_op_s* op, double* Q, double* Ac, hipStream_t st);
// Free the setup work buffers and the cached trunk matrix, keeping Q and A_c^{-1}.
void coarse_trim(helm_op_s* op);
// Validation of meta_opts against an op and a network (meta.hip).
helm_status check_opts(helm_op_s* op, don_s* net, const meta_opts* o);
// Multigrid (mg.hip): option checks, hierarchy (cached on the op), one V-cycle.
helm_status mg_check(const helm_op_s* op, const meta_opts* o);
helm_status mg_ensure(helm_op_s* op, don_s* net, const meta_opts* o, hipStream_t st);
template <typename S>
helm_status mg_apply(helm_op_s* op, don_s* net, const meta_opts* o, const void* v, void* z, hipStream_t st);
void mg_release(helm_op_s* op);

// ---- shared driver pieces ----
template <typename S>
helm_status residual_norm(helm_op_s* op, const void* f, const void* u, void* r, double* norm, hipStream_t st) {
  double* part;
  const int nb = stencil_nblocks(op->geom);
  helm_status s = op_part(op, (size_t)nb, &part);
  if (s) return s;
  stencil_resid<S>(op->geom, op->sc, op->code, f, u, r, part, st);
  if (norm) {
    reduce_cols(part, nb, 1, op->red, st);
    hipError_t e = hipMemcpyAsync(op->host, op->red, sizeof(double), hipMemcpyDeviceToHost, st);
    if (e != hipSuccess) return hip_fail(e, "residual readback");
    if ((s = sync_stream(st, "residual"))) return s;
    *norm = std::sqrt(op->host[0]);
  }
  return launch_check("residual");
}

template <typename S>
helm_status vec_norm(helm_op_s* op, const void* x, double* out, hipStream_t st) {
  double* part;
  const int nb = red_nblocks(op->nn);
  helm_status s = op_part(op, (size_t)nb, &part);
  if (s) return s;
  nrm2_part<S>(op->nn, x, part, st);
  reduce_cols(part, nb, 1, op->red, st);
  hipError_t e = hipMemcpyAsync(op->host, op->red, sizeof(double), hipMemcpyDeviceToHost, st);
  if (e != hipSuccess) return hip_fail(e, "norm readback");
  if ((s = sync_stream(st, "norm"))) return s;
  *out = std::sqrt(op->host[0]);
  return HELM_OK;
}

// `sweeps` relaxation steps in place on u; both kinds ping-pong through op->tmp
// (a red-black sweep is one fused out-of-place pass).
template <typename S>
helm_status relax(helm_op_s* op, int kind, double omega, int sweeps, const void* f, void* u, hipStream_t st) {
  if (sweeps <= 0) return HELM_OK;
  helm_status s = op->tmp.ensure(op->nn * op_esz(op));
  if (s) return s;
  void* a = u;
  void* b = op->tmp.ptr;
  for (int k = 0; k < sweeps; ++k) {
    if (kind == HELM_RBGS) stencil_rbgs_fused<S>(op->geom, op->sc, op->code, f, a, b, omega, st);
    else stencil_jacobi<S>(op->geom, op->sc, op->code, f, a, b, omega, st);
    void* t = a;
    a = b;
    b = t;
  }
  if (a != u) copy_vec<S>(op->nn, a, u, st);
  return launch_check("relax");
}

}  // namespace helm
