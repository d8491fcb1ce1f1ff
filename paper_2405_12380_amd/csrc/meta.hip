// Solver drivers and the meta-solver C ABI.
//
//  * relaxation meta-solver (eq. 3): cycles of n_r smoother sweeps followed by
//    one DeepONet correction of the residual, optionally handing a diverging
//    iteration to standalone GMRES;
//  * restarted GMRES(m) with CGS2 and BiCGStab, right-preconditioned, stopping
//    on the true relative residual (§3.1.2);
//  * the Krylov preconditioner M(r) = eq. 3 from z = 0 with the linear
//    trunk-basis M2 = Q A_c^{-1} Q^T of App. C.
//
// The host sequences kernel launches; per iteration it reads back one small
// status record (residual estimate, breakdown flag) to decide control flow.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstring>

#include "internal.h"
#include "lib.h"

namespace helm {

struct Carve {
  char* base;
  size_t off = 0;
  explicit Carve(void* b) : base((char*)b) {}
  void* take(size_t bytes) {
    void* p = base + off;
    off += (bytes + 255) & ~(size_t)255;
    return p;
  }
  static size_t need(size_t bytes) { return (bytes + 255) & ~(size_t)255; }
};

// Two timing-free events, destroyed with the scope.
// Status events of the iteration loops.  With system_fence false the event
// carries no system-scope release: the kernel that writes the status record to
// pinned host memory must make it visible itself (the GMRES step does).
struct EventPair {
  hipEvent_t e[2] = {nullptr, nullptr};
  explicit EventPair(bool system_fence = true) {
    const unsigned fl = hipEventDisableTiming | (system_fence ? 0u : (unsigned)hipEventDisableSystemFence);
    for (auto& x : e)
      if (hipEventCreateWithFlags(&x, fl) != hipSuccess) x = nullptr;
  }
  ~EventPair() {
    for (auto& x : e)
      if (x) (void)hipEventDestroy(x);
  }
  bool ok() const { return e[0] && e[1]; }
  hipEvent_t operator[](int i) const { return e[i]; }
};

struct MetaCtx {
  const meta_opts* o;
  don_s* net;
  bool use_M;  // Krylov: apply the preconditioner (net != NULL)
  void* r1;    // scratch field for the preconditioner residual
};

// z = M(v): n_r smoother sweeps on A z = v from z = 0, then the coarse
// correction z += Q A_c^{-1} Q^T (v - A z).
// With vscale (device scalar) the input is vscale[0] * v, and that scaled
// vector is also written to vout (the GMRES basis vector, normalized on the
// way in): the two-sweep Jacobi kernel scales as it loads, other paths scale
// in a separate pass first.
template <typename S>
helm_status precond_apply(helm_op_s* op, const MetaCtx& c, const void* v, void* z, hipStream_t st,
                          const double* vscale = nullptr, void* vout = nullptr) {
  const meta_opts* o = c.o;
  const size_t n = op->nn;
  if (vscale && !(o->mg_levels == 0 && o->n_r >= 2 && o->smoother == HELM_JACOBI)) {
    scale_dev<S>(n, v, vscale, vout, st);
    v = vout;
    vscale = nullptr;
  }
  if (o->mg_levels > 0) return mg_apply<S>(op, c.net, o, v, z, st);
  helm_status s;
  if (o->n_r > 0) {
    if (o->smoother == HELM_JACOBI) {
      if (o->n_r == 1) {
        jacobi_from_zero<S>(n, op->geom.dsum, op->sc, op->mask, v, z, o->omega, st);
      } else {
        // first two sweeps fused; the remaining n_r - 2 ping-pong through op->tmp
        // so that the last one lands in z
        if ((s = op->tmp.ensure(n * op_esz(op)))) return s;
        const int rest = o->n_r - 2;
        void* a = (rest & 1) ? op->tmp.ptr : z;
        void* b = (rest & 1) ? z : op->tmp.ptr;
        jacobi2_from_zero<S>(op->geom, op->sc, op->code, v, a, o->omega, st, vscale, vout);
        if (vscale) v = vout;  // the later sweeps and the residual read the scaled vector
        for (int k = 0; k < rest; ++k) {
          stencil_jacobi<S>(op->geom, op->sc, op->code, v, a, b, o->omega, st);
          void* t = a;
          a = b;
          b = t;
        }
      }
    } else {
      // red-black sweeps from zero, ping-ponging so that the last lands in z
      if ((s = op->tmp.ensure(n * op_esz(op)))) return s;
      void* a = (o->n_r & 1) ? op->tmp.ptr : z;
      void* b = (o->n_r & 1) ? z : op->tmp.ptr;
      zero_vec<S>(n, a, st);
      for (int k = 0; k < o->n_r; ++k) {
        stencil_rbgs_fused<S>(op->geom, op->sc, op->code, v, a, b, o->omega, st);
        void* t = a;
        a = b;
        b = t;
      }
    }
  } else {
    zero_vec<S>(n, z, st);
  }
  if (c.net) {
    double* part;
    if ((s = op_part(op, (size_t)stencil_nblocks(op->geom), &part))) return s;
    stencil_resid<S>(op->geom, op->sc, op->code, v, z, c.r1, part, st);
    if ((s = coarse_correct<S>(op, c.r1, z, st))) return s;
  }
  return launch_check("precond");
}

// ---------------------------------------------------------------------------
// GMRES(m), CGS2, right preconditioning
// ---------------------------------------------------------------------------
template <typename S>
helm_status gmres_drive(helm_op_s* op, MetaCtx& c, const void* f, void* u, meta_stats* out, hipStream_t st) {
  const meta_opts* o = c.o;
  const int m = o->restart;
  const bool one_pass = o->gs_passes == 1;
  const size_t n = op->nn, esz = op_esz(op);
  const size_t fld = Carve::need(n * esz);
  const size_t dsm = Carve::need(sizeof(double) * (2 * (size_t)(m + 1) * m + 8 * (size_t)(m + 1) + 64));
  helm_status s = op->ws.ensure(fld * (size_t)(m + 1 + 4) + dsm + Carve::need(sizeof(GmState)));
  if (s) return s;
  Carve cv(op->ws.ptr);
  char* V = (char*)cv.take(fld * (m + 1));
  void* W = cv.take(n * esz);  // the new Arnoldi vector before normalization
  void* z = cv.take(n * esz);
  void* t = cv.take(n * esz);
  c.r1 = cv.take(n * esz);
  double* H = (double*)cv.take(sizeof(double) * 2 * (m + 1) * m);
  double* g = (double*)cv.take(sizeof(double) * 2 * (m + 1));
  double* cs = (double*)cv.take(sizeof(double) * (m + 1));
  double* sn = (double*)cv.take(sizeof(double) * 2 * (m + 1));
  double* y = (double*)cv.take(sizeof(double) * 2 * (m + 1));
  double* h1 = (double*)cv.take(sizeof(double) * 2 * (m + 1));
  double* h2 = (double*)cv.take(sizeof(double) * 2 * (m + 1));
  double* nrm = (double*)cv.take(sizeof(double) * 8);
  GmState* gs = (GmState*)cv.take(sizeof(GmState));
  const size_t ldv = fld / esz;  // elements between basis vectors
  auto Vj = [&](int j) { return (void*)(V + (size_t)j * fld); };

  const int mdb = multidot_nblocks(n), rdb = red_nblocks(n), stb = stencil_nblocks(op->geom);
  const int cfb = cgs_fused_nblocks(n, 1);  // the largest block count of the fused CGS pass
  size_t pneed = (size_t)mdb * 2 * (m + 1);
  const size_t cneed = (size_t)cfb * 2 * (m + 1 < cgs_fused_max_nv() ? m + 1 : cgs_fused_max_nv());
  if (cneed > pneed) pneed = cneed;
  if ((size_t)rdb > pneed) pneed = rdb;
  if ((size_t)stb > pneed) pneed = stb;
  double* part;
  if ((s = op_part(op, pneed, &part))) return s;

  // status records land directly in pinned host memory (written by the kernel)
  GmState* slot[2] = {(GmState*)(op->host + 64), (GmState*)(op->host + 128)};
  GmState* slot_dev[2] = {(GmState*)(op->host_dev + 64), (GmState*)(op->host_dev + 128)};
  EventPair ev(false);
  if (!ev.ok()) return fail(HELM_E_HIP, "gmres: event creation failed");

  // No host round trip at a cycle start that follows a restart (or opens
  // the solve): ||f||^2 (once) and ||r||^2 are reduced on the device, the
  // start kernel sets g = beta e_1 and 1/beta and copies both squares to the
  // pinned record crec, and the cycle's first Arnoldi steps are queued behind
  // it.  The host reads the record at its first wait in the cycle; if the
  // cycle should not have started (beta at or below the tolerance, or not
  // finite) the queued steps are discarded: they touch V, W, H, g and the
  // status slots, never u.  After a cycle whose estimate met the tolerance
  // the true residual most likely does too, so that start waits for its
  // record before queueing anything.
  double* crec = op->host + 192;
  double* crec_dev = op->host_dev + 192;
  nrm2_part<S>(n, f, part, st);
  reduce_cols(part, rdb, 1, nrm + 1, st);
  bool first = true;
  double fs = 1.0, thr = 0.0;
  int count = 0, matvecs = 0, papps = 0, hlen = 0;
  helm_status status = HELM_NOT_CONVERGED;
  double beta = 0.0;
  bool est_met = false;  // the last cycle ended on its residual estimate
  // reads the cycle-start record once the work behind it has completed; true
  // when the solve ends at this cycle start (status set, or *err on failure)
  auto start_ends = [&](helm_status* err) -> bool {
    *err = HELM_OK;
    beta = std::sqrt(crec[0]);
    if (first) {
      first = false;
      const double fn = std::sqrt(crec[1]);
      if (!std::isfinite(fn)) {
        *err = fail(HELM_E_NONFINITE, "gmres: ||f|| is not finite");
        return true;
      }
      fs = fn > 0 ? fn : 1.0;  // residual scale: absolute residual when f = 0
      thr = o->tol * fs;
      if ((*err = coarse_finish(op))) return true;
    }
    if (o->history && hlen == 0) o->history[hlen++] = beta / fs;
    if (!std::isfinite(beta)) {
      status = HELM_E_NONFINITE;
      return true;
    }
    if (beta <= thr) {
      status = HELM_OK;
      return true;
    }
    return false;
  };
  for (;;) {
    // r = f - A u into V_0, beta = ||r||, V_0 = r / beta
    stencil_resid<S>(op->geom, op->sc, op->code, f, u, Vj(0), part, st);
    matvecs++;
    reduce_cols(part, stb, 1, nrm, st);
    gmres_start(nrm, g, m, crec_dev, st);
    scale_dev<S>(n, Vj(0), nrm + 2, Vj(0), st);
    bool checked = false;  // the start record has been read
    if (count >= o->max_iters || est_met) {
      // no Arnoldi step will run, or the cycle most likely ends here: read the record now
      if ((s = sync_stream(st, "gmres: residual"))) return s;
      helm_status e2;
      if (start_ends(&e2)) {
        if (e2) return e2;
        break;
      }
      if (count >= o->max_iters) break;
      checked = true;
    }
    // One Arnoldi step: z = M v_j, w = A z into W, CGS2 (or one classical
    // Gram-Schmidt pass with gs_passes = 1), Givens.  W stays
    // unnormalized; the next step forms v_{j+1} = W / ||W|| as its first kernel
    // reads it (inside the two-sweep Jacobi kernel, or a scaling pass).
    // Its status record is copied to pinned slot j & 1 and an event marks it.
    auto enqueue_step = [&](int j) -> helm_status {
      const void* zj = Vj(j);
      const double* vsc = j > 0 ? &gs->inv_hn : nullptr;
      if (c.use_M) {
        helm_status e2 = j > 0 ? precond_apply<S>(op, c, W, z, st, vsc, Vj(j)) : precond_apply<S>(op, c, Vj(j), z, st);
        if (e2) return e2;
        zj = z;
      } else if (j > 0) {
        scale_dev<S>(n, W, vsc, Vj(j), st);
      }
      void* w = W;
      multidot_apply<S>(op->geom, op->sc, op->code, zj, V, ldv, j + 1, w, part, st);  // w = A z_j and V^H w
      reduce_cols(part, mdb, 2 * (j + 1), h1, st);
      if (one_pass) {
        // one classical Gram-Schmidt projection, then ||w||^2
        multi_axpy<S>(n, V, ldv, j + 1, h1, -1.0, w, w, part, st);
        arnoldi_finish(j, m, H, g, cs, sn, h1, nullptr, part, rdb, gs, slot_dev[j & 1], st);
        hipError_t e1 = hipEventRecord(ev[j & 1], st);
        if (e1 != hipSuccess) return hip_fail(e1, "gmres: status event");
        return launch_check("gmres: arnoldi step");
      }
      if (j + 1 <= cgs_fused_max_nv()) {
        // first projection and second inner products in one pass over V
        const int nb = cgs_fused<S>(n, V, ldv, j + 1, h1, w, part, st);
        reduce_cols(part, nb, 2 * (j + 1), h2, st);
      } else {
        multi_axpy<S>(n, V, ldv, j + 1, h1, -1.0, w, w, nullptr, st);
        multidot_part<S>(n, V, ldv, j + 1, w, part, st);
        reduce_cols(part, mdb, 2 * (j + 1), h2, st);
      }
      multi_axpy<S>(n, V, ldv, j + 1, h2, -1.0, w, w, part, st);
      arnoldi_finish(j, m, H, g, cs, sn, h1, h2, part, rdb, gs, slot_dev[j & 1], st);
      hipError_t e1 = hipEventRecord(ev[j & 1], st);
      if (e1 != hipSuccess) return hip_fail(e1, "gmres: status event");
      return launch_check("gmres: arnoldi step");
    };
    int k = 0, queued = 0;  // steps 0 .. queued-1 are enqueued
    double g1 = -1.0, g2 = -1.0;  // the cycle's last two residual estimates
    bool ended = false;           // the solve ended at this cycle's start
    for (int j = 0; j < m; ++j) {
      if (queued == j) {
        if ((s = enqueue_step(j))) return s;
        queued = j + 1;
      }
      // look ahead: queue step j+1 before waiting for step j's status; if step j
      // ends the cycle the queued step is discarded (it only touches V_{j+1}, W,
      // column j+1 of H and g[j+1..j+2], none of which the back-solve and the
      // update u += M(V_{0..j} y) read).  When the last two estimates, extended
      // at their ratio, put step j at or below the tolerance, step j+1 would
      // most likely be discarded and is not queued ahead (a wrong guess costs
      // one wait for step j before step j+1 starts).
      bool ahead = j + 1 < m && count + 1 < o->max_iters;
      if (ahead && g1 > 0.0 && g2 > 0.0 && g1 * (g1 / g2) <= thr) ahead = false;
      if (ahead) {
        if ((s = enqueue_step(j + 1))) return s;
        queued = j + 2;
      }
      hipError_t e1 = hipEventSynchronize(ev[j & 1]);
      if (e1 != hipSuccess) return hip_fail(e1, "gmres: status wait");
      if (j == 0 && !checked) {
        helm_status e2;
        if (start_ends(&e2)) {
          if (e2) return e2;
          ended = true;
          break;
        }
      }
      const GmState hs = *slot[j & 1];
      g2 = g1;
      g1 = hs.gabs;
      count++;
      matvecs++;
      if (c.use_M) papps++;
      k = j + 1;
      if (o->history && hlen <= o->max_iters) o->history[hlen++] = hs.gabs / fs;
      if (hs.flag) {
        status = HELM_E_NONFINITE;
        break;
      }
      est_met = hs.gabs <= thr;
      if (est_met || count >= o->max_iters || hs.hn == 0.0) break;
    }
    if (ended || status == HELM_E_NONFINITE) break;
    // u += M (V_k y)
    gmres_backsolve(k, m, H, g, y, st);
    multi_axpy<S>(n, V, ldv, k, y, 1.0, nullptr, t, nullptr, st);
    if (c.use_M) {
      if ((s = precond_apply<S>(op, c, t, z, st))) return s;
      papps++;
      add_inplace<S>(n, z, u, st);
    } else {
      add_inplace<S>(n, t, u, st);
    }
  }
  if ((s = launch_check("gmres"))) return s;
  // true final residual
  double rn;
  if ((s = residual_norm<S>(op, f, u, Vj(0), &rn, st))) return s;
  out->iters = count;
  out->matvecs = matvecs;
  out->precond_apps = papps;
  out->rel_res = rn / fs;
  out->history_len = hlen;
  if (status == HELM_NOT_CONVERGED && rn <= thr) status = HELM_OK;
  out->converged = status == HELM_OK;
  return status;
}

// ---------------------------------------------------------------------------
// BiCGStab, right preconditioning
// ---------------------------------------------------------------------------
template <typename S>
helm_status bicgstab_drive(helm_op_s* op, MetaCtx& c, const void* f, void* u, meta_stats* out, hipStream_t st) {
  const meta_opts* o = c.o;
  const size_t n = op->nn, esz = op_esz(op);
  const size_t fld = Carve::need(n * esz);
  helm_status s = op->ws.ensure(fld * 9 + Carve::need(sizeof(BiState)) + Carve::need(64 * sizeof(double)));
  if (s) return s;
  Carve cv(op->ws.ptr);
  void* r = cv.take(n * esz);
  void* rh = cv.take(n * esz);
  void* p = cv.take(n * esz);
  void* v = cv.take(n * esz);
  void* sv = cv.take(n * esz);
  void* t = cv.take(n * esz);
  void* ph = cv.take(n * esz);
  void* sh = cv.take(n * esz);
  c.r1 = cv.take(n * esz);
  BiState* bs = (BiState*)cv.take(sizeof(BiState));
  double* red = (double*)cv.take(64 * sizeof(double));
  const int rdb = red_nblocks(n), stb = stencil_nblocks(op->geom);
  EventPair ev(false);
  if (!ev.ok()) return fail(HELM_E_HIP, "bicgstab: event creation failed");
  double* part;
  if ((s = op_part(op, (size_t)(3 * rdb > stb ? 3 * rdb : stb), &part))) return s;
  if (!c.use_M) {
    ph = p;
    sh = sv;
  }

  // ||f||^2 and the first ||r||^2 are reduced on the device and reach the
  // host in the first sweep's start record (pinned memory), read at the first
  // wait: the first half 1 is queued behind them without a round trip, and
  // is discarded if the solve should not have started (it touches neither u
  // nor r).
  BiState* hI = (BiState*)(op->host + 384);
  BiState* dI = (BiState*)(op->host_dev + 384);
  nrm2_part<S>(n, f, part, st);
  reduce_cols(part, rdb, 1, red + 12, st);
  stencil_resid<S>(op->geom, op->sc, op->code, f, u, r, part, st);
  reduce_cols(part, stb, 1, red + 13, st);
  int count = 0, matvecs = 1, papps = 0, hlen = 0;
  helm_status status = HELM_NOT_CONVERGED;
  double fs = 1.0, thr = 0.0, rn = 0.0;
  bool start_read = false;
  // reads the start record (once the work behind it has completed): the
  // residual scale, the tolerance and the status at the start
  auto read_start = [&]() -> helm_status {
    start_read = true;
    const double fn = std::sqrt(hI->fn);
    if (!std::isfinite(fn)) return fail(HELM_E_NONFINITE, "bicgstab: ||f|| is not finite");
    fs = fn > 0 ? fn : 1.0;  // residual scale: absolute residual when f = 0
    thr = o->tol * fs;
    rn = std::sqrt(hI->rr);
    if (o->history) o->history[hlen++] = rn / fs;
    if (!std::isfinite(rn)) status = HELM_E_NONFINITE;
    else if (rn <= thr) status = HELM_OK;
    return coarse_finish(op);
  };
  bool first_sweep = true;
  for (;;) {
    copy_vec<S>(n, r, rh, st);
    bicg_scalar(BI_INIT, bs, red + 12, st, first_sweep ? dI : nullptr);
    if (first_sweep && count >= o->max_iters) {
      // no iteration will run: read the record now
      if ((s = sync_stream(st, "bicgstab: residual"))) return s;
      if ((s = read_start())) return s;
    }
    first_sweep = false;
    if (status != HELM_NOT_CONVERGED) break;
    // rho for the first iteration of this sweep
    dot_part<S>(n, rh, r, part, st);
    reduce_cols(part, rdb, 2, red + 8, st);
    // One iteration = half 1 (rho, p, M p, v = A M p, alpha, s, ||s||) and
    // half 2 (M s, t = A M s, omega, the updates of u and r, ||r||).  Each half
    // ends by writing the state record to pinned memory behind an event.  Half 1
    // of the next iteration is queued before the host looks at ||r||: if ||r||
    // ends the sweep, that half is discarded (it writes only p, v, s, their
    // preconditioned copies and the scalar record, which a new sweep resets).
    BiState* hS = (BiState*)(op->host + 256);
    BiState* hR = (BiState*)(op->host + 320);
    BiState* dS = (BiState*)(op->host_dev + 256);  // the same records, as the kernels address them
    BiState* dR = (BiState*)(op->host_dev + 320);
    auto half1 = [&](bool first_) -> helm_status {
      bicg_scalar(BI_RHO, bs, red + 8, st);
      bicg_p<S>(n, r, v, p, bs, first_ ? 1 : 0, st);
      if (c.use_M) {
        helm_status e2 = precond_apply<S>(op, c, p, ph, st);
        if (e2) return e2;
      }
      stencil_apply<S>(op->geom, op->sc, op->code, ph, v, st);
      dot_part<S>(n, rh, v, part, st);
      reduce_cols(part, rdb, 2, red, st);
      bicg_scalar(BI_ALPHA, bs, red, st);
      bicg_s<S>(n, r, v, sv, bs, part, st);
      reduce_cols(part, rdb, 1, red + 2, st);
      bicg_scalar(BI_SS, bs, red + 2, st, dS);
      hipError_t e1 = hipEventRecord(ev[0], st);
      return e1 == hipSuccess ? launch_check("bicgstab: half 1") : hip_fail(e1, "bicgstab: half 1 record");
    };
    bool stopped = false, pending = false;
    double half2_ratio = -1.0;  // ||r|| / ||s|| of the last iteration's second half
    if (count < o->max_iters) {
      if ((s = half1(true))) return s;
      pending = true;
    }
    while (pending) {
      pending = false;
      hipError_t e1 = hipEventSynchronize(ev[0]);
      if (e1 != hipSuccess) return hip_fail(e1, "bicgstab: s");
      if (!start_read) {
        if ((s = read_start())) return s;
        if (status != HELM_NOT_CONVERGED) {
          stopped = true;
          break;
        }
      }
      BiState hb = *hS;
      const double ss_now = hb.ss;
      matvecs++;
      if (c.use_M) papps++;
      count++;
      if (hb.flag) {
        status = hb.flag == -4 ? HELM_E_BREAKDOWN : HELM_E_NONFINITE;
        stopped = true;
        break;
      }
      if (!std::isfinite(hb.ss)) {
        status = HELM_E_NONFINITE;
        stopped = true;
        break;
      }
      if (hb.ss <= thr) {
        axpy_dev<S>(n, ph, u, bs->alpha, st);
        if (o->history && hlen <= o->max_iters) o->history[hlen++] = hb.ss / fs;
        break;
      }
      if (c.use_M) {
        if ((s = precond_apply<S>(op, c, sv, sh, st))) return s;
        papps++;
      }
      stencil_apply<S>(op->geom, op->sc, op->code, sh, t, st);
      matvecs++;
      two_dot_part<S>(n, t, sv, part, st);
      reduce_cols(part, rdb, 3, red + 4, st);
      bicg_scalar(BI_OMEGA, bs, red + 4, st);
      bicg_update<S>(n, ph, sh, sv, t, rh, u, r, bs, part, st);
      reduce_cols(part, rdb, 3, red + 8 - 1, st);  // red[7] = ||r||^2, red[8..9] = r_hat^H r (next rho)
      bicg_scalar(BI_RR, bs, red + 7, st, dR);
      e1 = hipEventRecord(ev[1], st);
      if (e1 != hipSuccess) return hip_fail(e1, "bicgstab: half 2 record");
      // look ahead: the next half 1, unless ||s|| scaled by the last second
      // half's reduction predicts ||r|| at or below the tolerance (then the
      // queued half would most likely be discarded)
      const bool near = half2_ratio > 0.0 && ss_now * half2_ratio <= thr;
      if (count < o->max_iters && !near) {
        if ((s = half1(false))) return s;
        pending = true;
      }
      e1 = hipEventSynchronize(ev[1]);
      if (e1 != hipSuccess) return hip_fail(e1, "bicgstab: r");
      hb = *hR;
      if (ss_now > 0.0) half2_ratio = hb.rr / ss_now;
      if (hb.flag) {
        status = hb.flag == -4 ? HELM_E_BREAKDOWN : HELM_E_NONFINITE;
        stopped = true;
        break;
      }
      if (o->history && hlen <= o->max_iters) o->history[hlen++] = hb.rr / fs;
      if (!std::isfinite(hb.rr)) {
        status = HELM_E_NONFINITE;
        stopped = true;
        break;
      }
      if (hb.rr <= thr) break;
      if (!pending && count < o->max_iters) {  // the guess was wrong: queue the next half 1 now
        if ((s = half1(false))) return s;
        pending = true;
      }
    }
    if (stopped) break;
    if ((s = residual_norm<S>(op, f, u, r, &rn, st))) return s;
    matvecs++;
    if (!std::isfinite(rn)) status = HELM_E_NONFINITE;
    else if (rn <= thr) status = HELM_OK;
    else if (count >= o->max_iters) break;
    if (status != HELM_NOT_CONVERGED) break;
  }
  if ((s = launch_check("bicgstab"))) return s;
  if ((s = residual_norm<S>(op, f, u, c.r1, &rn, st))) return s;
  out->iters = count;
  out->matvecs = matvecs;
  out->precond_apps = papps;
  out->rel_res = rn / fs;
  out->history_len = hlen;
  out->converged = status == HELM_OK;
  return status;
}

// ---------------------------------------------------------------------------
// relaxation meta-solver, eq. 3
// ---------------------------------------------------------------------------
template <typename S>
helm_status relax_meta_drive(helm_op_s* op, MetaCtx& c, const void* f, void* u, meta_stats* out, hipStream_t st) {
  const meta_opts* o = c.o;
  const size_t n = op->nn, esz = op_esz(op);
  // Krylov fallback: the iterate before each cycle is kept, so a cycle whose
  // residual grows (or is not finite) can be undone and handed to GMRES
  const bool fb = o->fallback_restart > 0;
  helm_status s = op->ws.ensure(Carve::need(n * esz) * (fb ? 3 : 2));
  if (s) return s;
  Carve cv(op->ws.ptr);
  void* r = cv.take(n * esz);
  void* du = cv.take(n * esz);
  void* keep = fb ? cv.take(n * esz) : nullptr;
  const int kind = o->kind == META_JACOBI ? HELM_JACOBI : HELM_RBGS;
  double fn;
  if ((s = vec_norm<S>(op, f, &fn, st))) return s;
  const double fs = fn > 0 ? fn : 1.0;  // residual scale: absolute residual when f = 0
  int count = 0, ncorr = 0, hlen = 0, matvecs = 0;
  helm_status status = HELM_NOT_CONVERGED;
  double rn = 0.0, prev = 0.0;
  if (fb) {
    if ((s = residual_norm<S>(op, f, u, r, &rn, st))) return s;
    matvecs++;
    prev = rn / fs;
    copy_vec<S>(n, u, keep, st);
  }
  bool diverged = false;
  while (count < o->max_iters) {
    int cyc = o->nn_every > 0 ? o->nn_every : o->max_iters - count;
    if (cyc > o->max_iters - count) cyc = o->max_iters - count;
    if ((s = relax<S>(op, kind, o->omega, cyc, f, u, st))) return s;
    count += cyc;
    matvecs += cyc;
    if (c.net && o->nn_every > 0 && cyc == o->nn_every) {
      if ((s = residual_norm<S>(op, f, u, r, nullptr, st))) return s;
      matvecs++;
      if ((s = don_full(c.net, op, r, o->k, du, st))) return s;
      add_inplace<S>(n, du, u, st);
      ncorr++;
    }
    if ((s = residual_norm<S>(op, f, u, r, &rn, st))) return s;
    matvecs++;
    const double rel = rn / fs;
    if (o->history && hlen <= o->max_iters) o->history[hlen++] = rel;
    if (fb && !(rel <= prev)) {  // grew, or not finite
      diverged = true;
      break;
    }
    if (!std::isfinite(rel)) {
      status = HELM_E_NONFINITE;
      break;
    }
    if (rel <= o->tol) {
      status = HELM_OK;
      break;
    }
    if (fb) {
      copy_vec<S>(n, u, keep, st);
      prev = rel;
    }
  }
  if (diverged) {
    // standalone GMRES(fallback_restart), M = I, from the iterate before the
    // cycle that grew; its workspace may replace op->ws, so wait for the copy
    copy_vec<S>(n, keep, u, st);
    if ((s = sync_stream(st, "relaxation fallback"))) return s;
    meta_opts g = *o;
    g.kind = META_GMRES;
    g.restart = o->fallback_restart;
    g.history = nullptr;
    g.mg_levels = 0;
    MetaCtx gc{&g, nullptr, false, nullptr};
    meta_stats gst;
    std::memset(&gst, 0, sizeof gst);
    status = gmres_drive<S>(op, gc, f, u, &gst, st);
    out->iters = count;
    out->matvecs = matvecs + gst.matvecs;
    out->precond_apps = ncorr;
    out->rel_res = gst.rel_res;
    out->history_len = hlen;
    out->fallback_iters = gst.iters;
    out->converged = status == HELM_OK;
    return status;
  }
  if (count == 0) {
    if ((s = residual_norm<S>(op, f, u, r, &rn, st))) return s;
    if (rn <= o->tol * fs) status = HELM_OK;
  }
  out->iters = count;
  out->matvecs = matvecs;
  out->precond_apps = ncorr;
  out->rel_res = rn / fs;
  out->history_len = hlen;
  out->converged = status == HELM_OK;
  return status;
}

template <typename S>
helm_status meta_dispatch(helm_op_s* op, don_s* net, const meta_opts* o, const void* f, void* u, meta_stats* st_out,
                          hipStream_t st) {
  MetaCtx c{o, net, net != nullptr, nullptr};
  helm_status s;
  hipEvent_t e0, e1, e2;
  (void)hipEventCreate(&e0);
  (void)hipEventCreate(&e1);
  (void)hipEventCreate(&e2);
  (void)hipEventRecord(e0, st);
  if (net && (o->kind == META_GMRES || o->kind == META_BICGSTAB)) {
    // the Krylov drivers settle the space at their first wait, so the set-up's last
    // read-back does not stall the queue ahead of the first Arnoldi steps
    const bool defer = o->kind == META_GMRES || o->kind == META_BICGSTAB;
    if ((s = coarse_ensure(op, net, o->p_used, o->q_fp32 != 0, o->no_drop != 0, st, defer))) {
      if (op->coarse.valid) st_out->rank_used = op->coarse.rank;
      (void)hipEventDestroy(e0);
      (void)hipEventDestroy(e1);
      (void)hipEventDestroy(e2);
      return s;
    }
    st_out->rank_used = op->coarse.rank;
  }
  if (o->mg_levels > 0 && (s = mg_ensure(op, net, o, st))) {
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    (void)hipEventDestroy(e2);
    return s;
  }
  if (o->mg_levels > 0) c.use_M = true;
  (void)hipEventRecord(e1, st);
  if (o->kind == META_GMRES) s = gmres_drive<S>(op, c, f, u, st_out, st);
  else if (o->kind == META_BICGSTAB) s = bicgstab_drive<S>(op, c, f, u, st_out, st);
  else s = relax_meta_drive<S>(op, c, f, u, st_out, st);
  (void)hipEventRecord(e2, st);
  (void)hipEventSynchronize(e2);
  if (net && (o->kind == META_GMRES || o->kind == META_BICGSTAB)) {
    const helm_status s2 = coarse_finish(op);  // still pending only if the solve ended early
    if (!s) s = s2;
    st_out->cond_Ac_est = op->coarse.cond_est;
  }
  float a = 0.f, b = 0.f;
  (void)hipEventElapsedTime(&a, e0, e1);
  (void)hipEventElapsedTime(&b, e1, e2);
  st_out->setup_ms = a;
  st_out->solve_ms = b;
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  (void)hipEventDestroy(e2);
  return s;
}

helm_status check_opts(helm_op_s* op, don_s* net, const meta_opts* o) {
  if (!o) return fail(HELM_E_INVAL, "meta: opts is NULL");
  if (o->kind < META_JACOBI || o->kind > META_BICGSTAB) return fail(HELM_E_INVAL, "meta: unknown kind %d", o->kind);
  if (!(o->tol >= 0.0) || !std::isfinite(o->tol)) return fail(HELM_E_INVAL, "meta: tol must be finite and >= 0");
  if (o->max_iters < 0) return fail(HELM_E_INVAL, "meta: max_iters < 0");
  if (o->kind == META_GMRES && (o->restart < 1 || o->restart > 1000))
    return fail(HELM_E_INVAL, "meta: restart must be in [1, 1000]");
  if (o->smoother != HELM_JACOBI && o->smoother != HELM_RBGS)
    return fail(HELM_E_INVAL, "meta: unknown smoother %d", o->smoother);
  if (o->n_r < 0) return fail(HELM_E_INVAL, "meta: n_r < 0");
  if (!std::isfinite(o->omega)) return fail(HELM_E_INVAL, "meta: omega not finite");
  if (o->fallback_restart < 0 || o->fallback_restart > 1000)
    return fail(HELM_E_INVAL, "meta: fallback_restart must be in [0, 1000]");
  if (o->gs_passes < 0 || o->gs_passes > 2) return fail(HELM_E_INVAL, "meta: gs_passes must be 0, 1 or 2");
  if (net && (o->kind == META_GMRES || o->kind == META_BICGSTAB)) {
    helm_status s = check_net_for_op(net, op, o->p_used);
    if (s) return s;
  }
  if (net && (o->kind == META_JACOBI || o->kind == META_GS)) {
    helm_status s = check_net_for_op(net, op, 1);
    if (s) return s;
  }
  return mg_check(op, o);
}

}  // namespace helm

using namespace helm;

extern "C" {

helm_status meta_solve(helm_op op, don_net net, const meta_opts* o, const void* f, void* u, meta_stats* st,
                       void* stream) {
  if (!op || !f || !u || !st) return fail(HELM_E_INVAL, "meta_solve: NULL argument");
  if (f == u) return fail(HELM_E_INVAL, "meta_solve: f and u alias");
  helm_status s = check_opts(op, net, o);
  if (s) return s;
  std::memset(st, 0, sizeof *st);
  hipStream_t hs = (hipStream_t)stream;
  return op->dt == HELM_C128 ? meta_dispatch<double>(op, net, o, f, u, st, hs)
                             : meta_dispatch<float>(op, net, o, f, u, st, hs);
}

helm_status meta_solve_adjoint(helm_op op, don_net net, const meta_opts* o, const void* g, void* lam, meta_stats* st,
                               void* stream) {
  if (!op || !g || !lam || !st) return fail(HELM_E_INVAL, "meta_solve_adjoint: NULL argument");
  if (g == lam) return fail(HELM_E_INVAL, "meta_solve_adjoint: g and lam alias");
  helm_status s = check_opts(op, net, o);
  if (s) return s;
  std::memset(st, 0, sizeof *st);
  hipStream_t hs = (hipStream_t)stream;
  if ((s = op->adj.ensure(op->nn * op_esz(op)))) return s;
  // A is complex symmetric, so A^H lam = g  <=>  A conj(lam) = conj(g): the same
  // solver (and its cached coarse space) on conjugated data.  The preconditioner
  // this applies to the adjoint system is conj(M(conj(.))), i.e. M built from A^H.
  const bool c128 = op->dt == HELM_C128;
  if (c128) {
    conj_vec<double>(op->nn, g, op->adj.ptr, hs);
    conj_vec<double>(op->nn, lam, lam, hs);
    s = meta_dispatch<double>(op, net, o, op->adj.ptr, lam, st, hs);
    conj_vec<double>(op->nn, lam, lam, hs);
  } else {
    conj_vec<float>(op->nn, g, op->adj.ptr, hs);
    conj_vec<float>(op->nn, lam, lam, hs);
    s = meta_dispatch<float>(op, net, o, op->adj.ptr, lam, st, hs);
    conj_vec<float>(op->nn, lam, lam, hs);
  }
  helm_status s2 = sync_stream(hs, "meta_solve_adjoint");
  return s ? s : s2;
}

helm_status meta_precond(helm_op op, don_net net, const meta_opts* o, const void* r, void* z, void* stream) {
  if (!op || !r || !z) return fail(HELM_E_INVAL, "meta_precond: NULL argument");
  if (r == z) return fail(HELM_E_INVAL, "meta_precond: r and z alias");
  helm_status s = check_opts(op, net, o);
  if (s) return s;
  hipStream_t hs = (hipStream_t)stream;
  if (net && (s = coarse_ensure(op, net, o->p_used, o->q_fp32 != 0, o->no_drop != 0, hs))) return s;
  if (o->mg_levels > 0 && (s = mg_ensure(op, net, o, hs))) return s;
  const size_t fld = op->nn * op_esz(op);
  if ((s = op->ws.ensure(fld))) return s;
  MetaCtx c{o, net, true, op->ws.ptr};
  s = op->dt == HELM_C128 ? precond_apply<double>(op, c, r, z, hs) : precond_apply<float>(op, c, r, z, hs);
  if (s) return s;
  return sync_stream(hs, "meta_precond");
}

helm_status meta_coarse_info(helm_op op, don_net net, const meta_opts* o, int* rank, double* Ac, size_t ac_cap,
                             void* Q, size_t q_cap, void* stream) {
  if (!op || !net || !o || !rank) return fail(HELM_E_INVAL, "meta_coarse_info: NULL argument");
  helm_status s = check_net_for_op(net, op, o->p_used);
  if (s) return s;
  hipStream_t hs = (hipStream_t)stream;
  if ((s = coarse_ensure(op, net, o->p_used, o->q_fp32 != 0, o->no_drop != 0, hs))) return s;
  const int r = op->coarse.rank;
  *rank = r;
  if (op->coarse.pass1 && r > 0) {
    // the solves use the first-pass basis; the orthonormal one is formed here
    if (Ac && ac_cap < (size_t)r * r) return fail(HELM_E_INVAL, "meta_coarse_info: Ac capacity %zu < %d", ac_cap, r * r);
    if (Q && q_cap < op->nn * (size_t)r) return fail(HELM_E_INVAL, "meta_coarse_info: Q capacity too small");
    return coarse_orthonormal(op, (double*)Q, Ac, hs);
  }
  if (Ac) {
    if (ac_cap < (size_t)r * r) return fail(HELM_E_INVAL, "meta_coarse_info: Ac capacity %zu < %d", ac_cap, r * r);
    hipError_t e = hipMemcpyAsync(Ac, op->coarse.Ac.ptr, sizeof(double) * 2 * r * r, hipMemcpyDeviceToHost, hs);
    if (e != hipSuccess) return hip_fail(e, "meta_coarse_info: Ac");
  }
  if (Q) {
    if (q_cap < op->nn * (size_t)r) return fail(HELM_E_INVAL, "meta_coarse_info: Q capacity too small");
    const size_t rs = op->coarse.q_f32 ? sizeof(float) : sizeof(double);
    hipError_t e = hipMemcpyAsync(Q, op->coarse.Q.ptr, rs * op->nn * r, hipMemcpyDeviceToDevice, hs);
    if (e != hipSuccess) return hip_fail(e, "meta_coarse_info: Q");
  }
  return sync_stream(hs, "meta_coarse_info");
}

}  // extern "C"
