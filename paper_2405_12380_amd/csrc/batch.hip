// Many independent solves in one launch sequence: BiCGStab (optionally with
// the trunk-basis Krylov preconditioner of §3.1.2 / App. C) over a batch of
// problems with their own grids, wave numbers, scatterers and sources.
//
// Every kernel covers all problems: a workgroup belongs to exactly one problem
// (per-family block maps give its index), reads that problem's descriptor and
// BiCGStab state, and exits at once when the problem is not iterating, so
// convergence is decided on the device.  The per-problem scalar recurrences
// run in one workgroup per problem, which also reduces that problem's
// partials in a fixed order.  A chunk of iterations is captured once as a
// HIP graph on a library stream and replayed; between replays the host reads
// the states, checks the true residual of problems whose recurrence stopped
// (restarting those that are not converged, as the single-problem driver
// does) and repacks the block maps when the active set has shrunk.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <vector>

#include "coarse_dev.h"
#include "common.h"
#include "internal.h"
#include "lib.h"
#include "stencil_dev.h"

namespace helm {

namespace {

constexpr int EB_CH = 2048;     // elements per element-wise workgroup (256 threads x 8)
constexpr size_t QB_ROWS = 2048;  // basis rows per skinny-product workgroup
constexpr int SEG_ALIGN = 256;  // element alignment of each problem's segment
constexpr int ITERS_PER_GRAPH = 4;

struct BProb {
  StencilGeom g;
  const void* sc;
  const uint8_t* code;
  const uint8_t* mask;
  void* u;              // caller's iterate
  const void* Q;        // n x rank basis (fp64 or fp32)
  const double* Ainv;   // rank x rank complex128
  int rank;
  int pad;
  size_t n, off;        // nodes; element offset of the segment in the work vectors
  int sb0, sbn;         // stencil workgroups [sb0, sb0 + sbn) in the current packing
  int eb0, ebn;         // element-wise workgroups
  int qb0, qbn;         // basis workgroups
};

struct BState {
  double rho[2], rho0[2], alpha[2], omega[2], beta[2];
  double rr, ss, thr;
  int active;   // iterating
  int phase;    // 1: stopped on ||s|| in the current iteration
  int first;    // the next p-update is p = r
  int flag;     // 0, -4 breakdown, -5 non-finite
  int iters, max_iters, s_stops, pad;
};

enum { B_RHO = 0, B_ALPHA = 1, B_SS = 2, B_OMEGA = 3, B_RR = 4 };

__device__ __forceinline__ bool running(const BState& b) { return b.active && !b.phase; }
__device__ __forceinline__ bool finite2(double2 a) { return isfinite(a.x) && isfinite(a.y); }

// ---- stencils --------------------------------------------------------------
template <typename S, int DIM, int MODE>
__global__ __launch_bounds__(512) void kb_stencil(const BProb* __restrict__ P, const BState* __restrict__ B,
                                                  const int* __restrict__ smap, const cplx_t<S>* x,
                                                  const cplx_t<S>* __restrict__ f, cplx_t<S>* y, double omega,
                                                  double* __restrict__ scratch) {
  const int p = smap[blockIdx.x];
  if (!running(B[p])) return;
  const BProb& q = P[p];
  const size_t o = q.off;
  stencil_tile<S, DIM, MODE>(q.g, blockIdx.x - q.sb0, (const cplx_t<S>*)q.sc, q.code, x + o, f ? f + o : nullptr,
                             y + o, omega, 0, MODE == ST_RESID ? scratch + blockIdx.x : nullptr);
}

template <typename S, int DIM>
__global__ __launch_bounds__(512) void kb_jacobi2z(const BProb* __restrict__ P, const BState* __restrict__ B,
                                                   const int* __restrict__ smap, const cplx_t<S>* __restrict__ f,
                                                   cplx_t<S>* __restrict__ y, double omega) {
  const int p = smap[blockIdx.x];
  if (!running(B[p])) return;
  const BProb& q = P[p];
  jacobi2z_tile<S, DIM>(q.g, blockIdx.x - q.sb0, (const cplx_t<S>*)q.sc, q.code, f + q.off, y + q.off, omega);
}

// ---- element-wise and reductions ---------------------------------------------
// Element range of workgroup b of problem q: [lb EB_CH, min(n, (lb + 1) EB_CH)).
#define EW_RANGE(q)                                                      \
  const size_t e0 = (size_t)(blockIdx.x - (q).eb0) * EB_CH;              \
  const size_t e1 = min((q).n, e0 + EB_CH);                              \
  const size_t o = (q).off

// z = omega D^{-1} v (one Jacobi sweep from zero)
template <typename S>
__global__ __launch_bounds__(256) void kb_jacobi0(const BProb* __restrict__ P, const BState* __restrict__ B,
                                                  const int* __restrict__ emap, const cplx_t<S>* __restrict__ v,
                                                  cplx_t<S>* __restrict__ z, double omega) {
  const int p = emap[blockIdx.x];
  if (!running(B[p])) return;
  const BProb& q = P[p];
  EW_RANGE(q);
  const cplx_t<S>* sc = (const cplx_t<S>*)q.sc;
  for (size_t e = e0 + threadIdx.x; e < e1; e += 256) {
    const double2 s = ldc(sc, e);
    const double2 d = q.mask[e] ? make_double2(1.0, 0.0) : make_double2(q.g.dsum - s.x, -s.y);
    const double2 w = ddiv(ldc(v, o + e), d);
    stc(z, o + e, make_double2(omega * w.x, omega * w.y));
  }
}

template <typename S>
__global__ __launch_bounds__(256) void kb_zero(const BProb* __restrict__ P, const BState* __restrict__ B,
                                               const int* __restrict__ emap, cplx_t<S>* __restrict__ z) {
  const int p = emap[blockIdx.x];
  if (!running(B[p])) return;
  const BProb& q = P[p];
  EW_RANGE(q);
  for (size_t e = e0 + threadIdx.x; e < e1; e += 256) stc(z, o + e, czero());
}

// partial of conj(x)^T y  (only < 0: every running problem; otherwise that problem alone)
template <typename S>
__global__ __launch_bounds__(256) void kb_dot(const BProb* __restrict__ P, const BState* __restrict__ B,
                                              const int* __restrict__ emap, int only, const cplx_t<S>* __restrict__ x,
                                              const cplx_t<S>* __restrict__ y, double* __restrict__ part) {
  __shared__ double sh[32];
  const int p = emap[blockIdx.x];
  if (!running(B[p]) || (only >= 0 && p != only)) return;
  const BProb& q = P[p];
  EW_RANGE(q);
  double2 acc = czero();
  for (size_t e = e0 + threadIdx.x; e < e1; e += 256) acc = cadd(acc, cconjmul(ldc(x, o + e), ldc(y, o + e)));
  acc = block_sum2(acc, sh);
  if (threadIdx.x == 0) {
    part[2 * blockIdx.x] = acc.x;
    part[2 * blockIdx.x + 1] = acc.y;
  }
}

// p = r (first) or r + beta (p - omega v)
template <typename S>
__global__ __launch_bounds__(256) void kb_p(const BProb* __restrict__ P, const BState* __restrict__ B,
                                            const int* __restrict__ emap, const cplx_t<S>* __restrict__ r,
                                            const cplx_t<S>* __restrict__ v, cplx_t<S>* __restrict__ pv) {
  const int p = emap[blockIdx.x];
  const BState& b = B[p];
  if (!running(b)) return;
  const BProb& q = P[p];
  EW_RANGE(q);
  const double2 beta = make_double2(b.beta[0], b.beta[1]);
  const double2 om = make_double2(b.omega[0], b.omega[1]);
  const bool first = b.first;
  for (size_t e = e0 + threadIdx.x; e < e1; e += 256) {
    const double2 re = ldc(r, o + e);
    if (first) {
      stc(pv, o + e, re);
    } else {
      const double2 t = csub(ldc(pv, o + e), cmul(om, ldc(v, o + e)));
      stc(pv, o + e, cadd(re, cmul(beta, t)));
    }
  }
}

// s = r - alpha v, partial of ||s||^2
template <typename S>
__global__ __launch_bounds__(256) void kb_s(const BProb* __restrict__ P, const BState* __restrict__ B,
                                            const int* __restrict__ emap, const cplx_t<S>* __restrict__ r,
                                            const cplx_t<S>* __restrict__ v, cplx_t<S>* __restrict__ s,
                                            double* __restrict__ part) {
  __shared__ double sh[16];
  const int p = emap[blockIdx.x];
  const BState& b = B[p];
  if (!running(b)) return;
  const BProb& q = P[p];
  EW_RANGE(q);
  const double2 al = make_double2(b.alpha[0], b.alpha[1]);
  double nrm = 0.0;
  for (size_t e = e0 + threadIdx.x; e < e1; e += 256) {
    const double2 w = csub(ldc(r, o + e), cmul(al, ldc(v, o + e)));
    stc(s, o + e, w);
    nrm += w.x * w.x + w.y * w.y;
  }
  nrm = block_sum(nrm, sh);
  if (threadIdx.x == 0) part[blockIdx.x] = nrm;
}

// partials of t^H s and t^H t
template <typename S>
__global__ __launch_bounds__(256) void kb_two_dot(const BProb* __restrict__ P, const BState* __restrict__ B,
                                                  const int* __restrict__ emap, const cplx_t<S>* __restrict__ t,
                                                  const cplx_t<S>* __restrict__ s, double* __restrict__ part) {
  __shared__ double sh[32];
  const int p = emap[blockIdx.x];
  if (!running(B[p])) return;
  const BProb& q = P[p];
  EW_RANGE(q);
  double2 ts = czero();
  double tt = 0.0;
  for (size_t e = e0 + threadIdx.x; e < e1; e += 256) {
    const double2 te = ldc(t, o + e);
    ts = cadd(ts, cconjmul(te, ldc(s, o + e)));
    tt += te.x * te.x + te.y * te.y;
  }
  ts = block_sum2(ts, sh);
  tt = block_sum(tt, sh);
  if (threadIdx.x == 0) {
    part[3 * blockIdx.x] = ts.x;
    part[3 * blockIdx.x + 1] = ts.y;
    part[3 * blockIdx.x + 2] = tt;
  }
}

// phase 0: u += alpha p_hat + omega s_hat; r = s - omega t; partials of ||r||^2
// and r_hat^H r.  phase 1 (stopped on ||s||): u += alpha p_hat.
template <typename S>
__global__ __launch_bounds__(256) void kb_update(const BProb* __restrict__ P, const BState* __restrict__ B,
                                                 const int* __restrict__ emap, const cplx_t<S>* __restrict__ ph,
                                                 const cplx_t<S>* __restrict__ shat, const cplx_t<S>* __restrict__ s,
                                                 const cplx_t<S>* __restrict__ t, const cplx_t<S>* __restrict__ rhat,
                                                 cplx_t<S>* __restrict__ r, double* __restrict__ prr,
                                                 double* __restrict__ prho) {
  __shared__ double sh[32];
  const int p = emap[blockIdx.x];
  const BState& b = B[p];
  if (!b.active) return;
  const BProb& q = P[p];
  EW_RANGE(q);
  cplx_t<S>* u = (cplx_t<S>*)q.u;
  const double2 al = make_double2(b.alpha[0], b.alpha[1]);
  if (b.phase) {
    for (size_t e = e0 + threadIdx.x; e < e1; e += 256) stc(u, e, cadd(ldc(u, e), cmul(al, ldc(ph, o + e))));
    return;
  }
  const double2 om = make_double2(b.omega[0], b.omega[1]);
  double rr = 0.0;
  double2 rho = czero();
  for (size_t e = e0 + threadIdx.x; e < e1; e += 256) {
    const double2 ue = cadd(ldc(u, e), cadd(cmul(al, ldc(ph, o + e)), cmul(om, ldc(shat, o + e))));
    stc(u, e, ue);
    const double2 re = csub(ldc(s, o + e), cmul(om, ldc(t, o + e)));
    stc(r, o + e, re);
    rr += re.x * re.x + re.y * re.y;
    rho = cadd(rho, cconjmul(ldc(rhat, o + e), re));
  }
  rr = block_sum(rr, sh);
  rho = block_sum2(rho, sh);
  if (threadIdx.x == 0) {
    prr[blockIdx.x] = rr;
    prho[2 * blockIdx.x] = rho.x;
    prho[2 * blockIdx.x + 1] = rho.y;
  }
}

// ---- per-problem recurrences (one workgroup per problem) ---------------------
// Sum of `width` interleaved values over the problem's element-wise partials,
// in a fixed order (thread t takes blocks t, t + 256, ..., then a fixed tree).
__device__ double seg_sum(const double* part, int width, int k, int b0, int nb, double* sh) {
  double a = 0.0;
  for (int bb = 0; bb < nb; bb += 4 * 256) {  // four loads in flight, added in index order
    double v[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int b = bb + threadIdx.x + 256 * q;
      v[q] = b < nb ? part[(size_t)(b0 + b) * width + k] : 0.0;
    }
#pragma unroll
    for (int q = 0; q < 4; ++q) a += v[q];
  }
  return block_sum(a, sh);
}

__global__ __launch_bounds__(256) void kb_state(int step, const BProb* __restrict__ P, BState* __restrict__ B,
                                                const double* __restrict__ part) {
  __shared__ double sh[16];
  __shared__ double v[3];
  const int p = blockIdx.x;
  BState& b = B[p];
  const bool need = step == B_RR ? (bool)b.active : running(b);
  if (!need) return;
  const BProb& q = P[p];
  const bool reduce = !(step == B_RR && b.phase);
  if (reduce) {
    const int width = step == B_OMEGA ? 3 : (step == B_SS || step == B_RR) ? 1 : 2;
    for (int k = 0; k < width; ++k) {
      const double s = seg_sum(part, width, k, q.eb0, q.ebn, sh);
      if (threadIdx.x == 0) v[k] = s;
      __syncthreads();
    }
  }
  if (threadIdx.x != 0) return;
  if (step == B_RHO) {
    const double2 rho = make_double2(v[0], v[1]);
    if (!finite2(rho)) {
      b.flag = -5;
      b.active = 0;
      return;
    }
    if (rho.x == 0.0 && rho.y == 0.0) {
      b.flag = -4;
      b.active = 0;
      return;
    }
    const double2 beta = cmul(cdiv(rho, make_double2(b.rho0[0], b.rho0[1])),
                              cdiv(make_double2(b.alpha[0], b.alpha[1]), make_double2(b.omega[0], b.omega[1])));
    b.beta[0] = beta.x;
    b.beta[1] = beta.y;
    b.rho[0] = rho.x;
    b.rho[1] = rho.y;
  } else if (step == B_ALPHA) {
    const double2 den = make_double2(v[0], v[1]);
    b.first = 0;
    if (!finite2(den)) {
      b.flag = -5;
      b.active = 0;
      return;
    }
    if (den.x == 0.0 && den.y == 0.0) {
      b.flag = -4;
      b.active = 0;
      return;
    }
    const double2 al = cdiv(make_double2(b.rho[0], b.rho[1]), den);
    b.alpha[0] = al.x;
    b.alpha[1] = al.y;
  } else if (step == B_SS) {
    b.ss = sqrt(v[0]);
    b.iters++;
    if (!isfinite(b.ss)) {
      b.flag = -5;
      b.active = 0;
    } else if (b.ss <= b.thr) {
      b.phase = 1;
      b.s_stops++;
    }
  } else if (step == B_OMEGA) {
    const double2 ts = make_double2(v[0], v[1]);
    const double tt = v[2];
    double2 om = czero();
    if (tt != 0.0) om = make_double2(ts.x / tt, ts.y / tt);
    if (!finite2(om)) {
      b.flag = -5;
      b.active = 0;
      return;
    }
    if (om.x == 0.0 && om.y == 0.0) {
      b.flag = -4;
      b.active = 0;
      return;
    }
    b.omega[0] = om.x;
    b.omega[1] = om.y;
  } else {  // B_RR
    if (b.phase) {
      b.active = 0;
      return;
    }
    b.rr = sqrt(v[0]);
    b.rho0[0] = b.rho[0];
    b.rho0[1] = b.rho[1];
    if (!isfinite(b.rr)) {
      b.flag = -5;
      b.active = 0;
    } else if (b.rr <= b.thr || b.iters >= b.max_iters) {
      b.active = 0;
    }
  }
}

// ---- trunk-basis correction ----------------------------------------------------
template <typename T, typename S>
__global__ __launch_bounds__(256) void kb_qt(const BProb* __restrict__ P, const BState* __restrict__ B,
                                             const int* __restrict__ qmap, const cplx_t<S>* __restrict__ x,
                                             double* __restrict__ part) {
  const int p = qmap[blockIdx.x];
  if (!running(B[p])) return;
  const BProb& q = P[p];
  const size_t i0 = (size_t)(blockIdx.x - q.qb0) * QB_ROWS;
  qt_rows<T, S>(q.rank, (const T*)q.Q, x + q.off, i0, min(q.n, i0 + QB_ROWS), part + (size_t)blockIdx.x * 256);
}

// y_p = sum of the problem's Q^T partials (fixed order), then c_p = A_c^{-1} y_p
__global__ __launch_bounds__(256) void kb_qreduce(const BProb* __restrict__ P, const BState* __restrict__ B,
                                                  const double* __restrict__ part, double* __restrict__ y) {
  const int p = blockIdx.x;
  if (!running(B[p])) return;
  const BProb& q = P[p];
  const int e = threadIdx.x;
  if (e >= 2 * q.rank) return;
  double a = 0.0;
  for (int bb = 0; bb < q.qbn; bb += 8) {  // eight loads in flight, added in index order
    double v[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) v[u] = bb + u < q.qbn ? part[(size_t)(q.qb0 + bb + u) * 256 + e] : 0.0;
#pragma unroll
    for (int u = 0; u < 8; ++u) a += v[u];
  }
  y[(size_t)p * 256 + e] = a;
}

__global__ __launch_bounds__(64) void kb_ainv(const BProb* __restrict__ P, const BState* __restrict__ B,
                                              const double* __restrict__ y, double* __restrict__ c) {
  const int p = blockIdx.x >> 7, j = blockIdx.x & 127, l = threadIdx.x;
  if (!running(B[p])) return;
  const BProb& q = P[p];
  const int r = q.rank;
  if (j >= r) return;
  const double* yp = y + (size_t)p * 256;
  double2 acc = czero();
  for (int k = l; k < r; k += 64) {
    const size_t o = 2 * ((size_t)j * r + k);
    acc = cadd(acc, cmul(make_double2(q.Ainv[o], q.Ainv[o + 1]), make_double2(yp[2 * k], yp[2 * k + 1])));
  }
  acc.x = wave_sum(acc.x);
  acc.y = wave_sum(acc.y);
  if (l == 0) {
    c[(size_t)p * 256 + 2 * j] = acc.x;
    c[(size_t)p * 256 + 2 * j + 1] = acc.y;
  }
}

template <typename T, typename S>
__global__ __launch_bounds__(256) void kb_skinny(const BProb* __restrict__ P, const BState* __restrict__ B,
                                                 const int* __restrict__ qmap, const double* __restrict__ c,
                                                 cplx_t<S>* __restrict__ z) {
  const int p = qmap[blockIdx.x];
  if (!running(B[p])) return;
  const BProb& q = P[p];
  const size_t wave = 4 * (size_t)(blockIdx.x - q.qb0) + (threadIdx.x >> 6);
  skinny_rows<T, S, SK_ADD>(q.n, q.rank, (const T*)q.Q, c + (size_t)p * 256, z + q.off, q.mask, nullptr, wave,
                            4 * (size_t)q.qbn);
}

// ---- host side -------------------------------------------------------------------
struct DevMem {
  void* p = nullptr;
  ~DevMem() { dfree(p); }
};

struct Packing {
  std::vector<int> smap, emap, qmap;
};

// Block ranges of the problems in `list` (others get empty ranges).
static void pack(std::vector<BProb>& pr, const std::vector<int>& list, Packing& pk) {
  pk.smap.clear();
  pk.emap.clear();
  pk.qmap.clear();
  for (auto& q : pr) q.sbn = q.ebn = q.qbn = 0;
  for (int i : list) {
    BProb& q = pr[i];
    q.sb0 = (int)pk.smap.size();
    q.sbn = stencil_nblocks(q.g);
    pk.smap.insert(pk.smap.end(), q.sbn, i);
    q.eb0 = (int)pk.emap.size();
    q.ebn = (int)((q.n + EB_CH - 1) / EB_CH);
    pk.emap.insert(pk.emap.end(), q.ebn, i);
    q.qb0 = (int)pk.qmap.size();
    q.qbn = q.rank > 0 ? (int)((q.n + QB_ROWS - 1) / QB_ROWS) : 0;
    pk.qmap.insert(pk.qmap.end(), q.qbn, i);
  }
}

template <typename S, typename T, int DIM>
struct BatchRun {
  using C = cplx_t<S>;
  const meta_opts* o;
  bool use_M;
  int np;
  BProb* dP;
  BState* dB;
  int *dsmap, *demap, *dqmap;
  int nsb, neb, nqb;
  C *r, *rh, *pv, *v, *s, *t, *ph, *sh, *r1, *tmp;
  double *pe, *pts, *prr, *prho, *pq, *ybuf, *cbuf, *scratch;
  int ty;

  void stencil_launch(int mode, const C* x, const C* f, C* y, hipStream_t st) {
    dim3 blk(64, ty);
    if (nsb == 0) return;
    switch (mode) {
      case ST_APPLY:
        hipLaunchKernelGGL((kb_stencil<S, DIM, ST_APPLY>), dim3(nsb), blk, 0, st, dP, dB, dsmap, x, f, y, 0.0, scratch);
        break;
      case ST_RESID:
        hipLaunchKernelGGL((kb_stencil<S, DIM, ST_RESID>), dim3(nsb), blk, 0, st, dP, dB, dsmap, x, f, y, 0.0, scratch);
        break;
      default:
        hipLaunchKernelGGL((kb_stencil<S, DIM, ST_JACOBI>), dim3(nsb), blk, 0, st, dP, dB, dsmap, x, f, y, o->omega,
                           scratch);
    }
  }

  // z = M(v): n_r Jacobi sweeps from zero, then z += Q A_c^{-1} Q^T (v - A z)
  void precond(const C* vin, C* z, hipStream_t st) {
    const int nr = o->n_r;
    if (nr <= 0) {
      hipLaunchKernelGGL((kb_zero<S>), dim3(neb), dim3(256), 0, st, dP, dB, demap, z);
    } else if (nr == 1) {
      hipLaunchKernelGGL((kb_jacobi0<S>), dim3(neb), dim3(256), 0, st, dP, dB, demap, vin, z, o->omega);
    } else {
      const int rest = nr - 2;
      C* a = (rest & 1) ? tmp : z;
      C* b = (rest & 1) ? z : tmp;
      hipLaunchKernelGGL((kb_jacobi2z<S, DIM>), dim3(nsb), dim3(64, ty), 0, st, dP, dB, dsmap, vin, a, o->omega);
      for (int k = 0; k < rest; ++k) {
        stencil_launch(ST_JACOBI, a, vin, b, st);
        std::swap(a, b);
      }
    }
    if (nqb > 0) {
      stencil_launch(ST_RESID, z, vin, r1, st);
      hipLaunchKernelGGL((kb_qt<T, S>), dim3(nqb), dim3(256), 0, st, dP, dB, dqmap, r1, pq);
      hipLaunchKernelGGL(kb_qreduce, dim3(np), dim3(256), 0, st, dP, dB, pq, ybuf);
      hipLaunchKernelGGL(kb_ainv, dim3(np * 128), dim3(64), 0, st, dP, dB, ybuf, cbuf);
      hipLaunchKernelGGL((kb_skinny<T, S>), dim3(nqb), dim3(256), 0, st, dP, dB, dqmap, cbuf, z);
    }
  }

  // one BiCGStab iteration for every running problem (M = I without a network)
  void iteration(hipStream_t st) {
    C* PH = use_M ? ph : pv;
    C* SH = use_M ? sh : s;
    hipLaunchKernelGGL(kb_state, dim3(np), dim3(256), 0, st, B_RHO, dP, dB, prho);
    hipLaunchKernelGGL((kb_p<S>), dim3(neb), dim3(256), 0, st, dP, dB, demap, r, v, pv);
    if (use_M) precond(pv, ph, st);
    stencil_launch(ST_APPLY, PH, nullptr, v, st);
    hipLaunchKernelGGL((kb_dot<S>), dim3(neb), dim3(256), 0, st, dP, dB, demap, -1, rh, v, pe);
    hipLaunchKernelGGL(kb_state, dim3(np), dim3(256), 0, st, B_ALPHA, dP, dB, pe);
    hipLaunchKernelGGL((kb_s<S>), dim3(neb), dim3(256), 0, st, dP, dB, demap, r, v, s, prr);
    hipLaunchKernelGGL(kb_state, dim3(np), dim3(256), 0, st, B_SS, dP, dB, prr);
    if (use_M) precond(s, sh, st);
    stencil_launch(ST_APPLY, SH, nullptr, t, st);
    hipLaunchKernelGGL((kb_two_dot<S>), dim3(neb), dim3(256), 0, st, dP, dB, demap, t, s, pts);
    hipLaunchKernelGGL(kb_state, dim3(np), dim3(256), 0, st, B_OMEGA, dP, dB, pts);
    hipLaunchKernelGGL((kb_update<S>), dim3(neb), dim3(256), 0, st, dP, dB, demap, PH, SH, s, t, rh, r, prr, prho);
    hipLaunchKernelGGL(kb_state, dim3(np), dim3(256), 0, st, B_RR, dP, dB, prr);
  }
};

template <typename S, typename T, int DIM>
helm_status batch_drive(int np, helm_op_s* const* ops, don_s* net, const meta_opts* o, const void* const* f,
                        void* const* u, meta_stats* stats, hipStream_t user_st) {
  using C = cplx_t<S>;
  const bool use_M = net != nullptr;
  const size_t esz = sizeof(C);
  helm_status s;
  // build (or reuse) the coarse spaces one problem at a time, releasing the
  // setup work buffers so that only the bases stay resident
  for (int i = 0; i < np; ++i) {
    std::memset(&stats[i], 0, sizeof stats[i]);
    if (!use_M) continue;
    hipEvent_t e0, e1;
    (void)hipEventCreate(&e0);
    (void)hipEventCreate(&e1);
    (void)hipEventRecord(e0, user_st);
    s = coarse_ensure(ops[i], net, o->p_used, o->q_fp32 != 0, o->no_drop != 0, user_st);
    (void)hipEventRecord(e1, user_st);
    if (!s) s = sync_stream(user_st, "meta_solve_batch: coarse setup");
    float ms = 0.f;
    (void)hipEventElapsedTime(&ms, e0, e1);
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (s) return s;
    coarse_trim(ops[i]);
    stats[i].setup_ms = ms;
    stats[i].rank_used = ops[i]->coarse.rank;
    stats[i].cond_Ac_est = ops[i]->coarse.cond_est;
  }
  // problem descriptors; a uniform workgroup height for the batch: the ops'
  // own (tuned) one when they agree, else 4
  int ty = ops[0]->geom.ty;
  for (int i = 1; i < np; ++i)
    if (ops[i]->geom.ty != ty) ty = 4;
  std::vector<BProb> pr(np);
  size_t tot = 0;
  for (int i = 0; i < np; ++i) {
    BProb& q = pr[i];
    std::memset(&q, 0, sizeof q);
    q.g = ops[i]->geom;
    q.g.ty = ty;
    q.g.rows = 1;  // the batched kernels run one row per thread
    q.sc = ops[i]->sc;
    q.code = ops[i]->code;
    q.mask = ops[i]->mask;
    q.u = u[i];
    q.n = ops[i]->nn;
    q.off = tot;
    tot += (q.n + SEG_ALIGN - 1) / SEG_ALIGN * SEG_ALIGN;
    if (use_M) {
      q.Q = ops[i]->coarse.Q.ptr;
      q.Ainv = (const double*)ops[i]->coarse.Ainv.ptr;
      q.rank = ops[i]->coarse.rank;
    }
  }
  std::vector<int> all(np);
  for (int i = 0; i < np; ++i) all[i] = i;
  Packing pk;
  pack(pr, all, pk);
  const size_t max_sb = pk.smap.size(), max_eb = pk.emap.size(), max_qb = pk.qmap.size();

  // device memory: 10 work vectors, partials, maps, descriptors and states
  DevMem work, small;
  const size_t vecb = tot * esz;
  if ((s = dalloc(&work.p, vecb * 10))) return s;
  const size_t nsmall = 2 * max_eb + 3 * max_eb + max_eb + 2 * max_eb + 256 * (max_qb + 1) + 512 * (size_t)np +
                        (max_sb + 1);
  const size_t bytes_small = sizeof(double) * nsmall + sizeof(int) * (max_sb + max_eb + max_qb + 3) +
                             sizeof(BProb) * np + sizeof(BState) * np + 4096;
  if ((s = dalloc(&small.p, bytes_small))) return s;
  BatchRun<S, T, DIM> R;
  R.o = o;
  R.use_M = use_M;
  R.np = np;
  R.ty = ty;
  C* base = (C*)work.p;
  C** vecs[10] = {&R.r, &R.rh, &R.pv, &R.v, &R.s, &R.t, &R.ph, &R.sh, &R.r1, &R.tmp};
  for (int k = 0; k < 10; ++k) *vecs[k] = base + (size_t)k * tot;
  double* dp = (double*)small.p;
  R.pe = dp;
  dp += 2 * max_eb;
  R.pts = dp;
  dp += 3 * max_eb;
  R.prr = dp;
  dp += max_eb;
  R.prho = dp;
  dp += 2 * max_eb;
  R.pq = dp;
  dp += 256 * (max_qb + 1);
  R.ybuf = dp;
  dp += 256 * (size_t)np;
  R.cbuf = dp;
  dp += 256 * (size_t)np;
  R.scratch = dp;
  dp += max_sb + 1;
  char* cp = (char*)(((uintptr_t)dp + 255) & ~(uintptr_t)255);
  R.dP = (BProb*)cp;
  cp += (sizeof(BProb) * np + 255) & ~(size_t)255;
  R.dB = (BState*)cp;
  cp += (sizeof(BState) * np + 255) & ~(size_t)255;
  R.dsmap = (int*)cp;
  R.demap = R.dsmap + max_sb + 1;
  R.dqmap = R.demap + max_eb + 1;

  // a library stream for capture and replay (the caller's may be the null stream)
  if ((s = sync_stream(user_st, "meta_solve_batch"))) return s;
  hipStream_t st;
  if (hipStreamCreateWithFlags(&st, hipStreamNonBlocking) != hipSuccess)
    return fail(HELM_E_HIP, "meta_solve_batch: stream creation failed");
  struct StreamGuard {
    hipStream_t s;
    ~StreamGuard() { (void)hipStreamDestroy(s); }
  } sguard{st};
  BState* hB = nullptr;
  if (hipHostMalloc((void**)&hB, sizeof(BState) * np, hipHostMallocDefault) != hipSuccess)
    return fail(HELM_E_NOMEM, "meta_solve_batch: pinned state");
  struct HostGuard {
    void* p;
    ~HostGuard() { (void)hipHostFree(p); }
  } hguard{hB};

  auto upload = [&](const Packing& k) -> helm_status {
    hipError_t e = hipMemcpyAsync(R.dP, pr.data(), sizeof(BProb) * np, hipMemcpyHostToDevice, st);
    if (e == hipSuccess && !k.smap.empty())
      e = hipMemcpyAsync(R.dsmap, k.smap.data(), sizeof(int) * k.smap.size(), hipMemcpyHostToDevice, st);
    if (e == hipSuccess && !k.emap.empty())
      e = hipMemcpyAsync(R.demap, k.emap.data(), sizeof(int) * k.emap.size(), hipMemcpyHostToDevice, st);
    if (e == hipSuccess && !k.qmap.empty())
      e = hipMemcpyAsync(R.dqmap, k.qmap.data(), sizeof(int) * k.qmap.size(), hipMemcpyHostToDevice, st);
    if (e != hipSuccess) return hip_fail(e, "meta_solve_batch: descriptors");
    R.nsb = (int)k.smap.size();
    R.neb = (int)k.emap.size();
    R.nqb = (int)k.qmap.size();
    return sync_stream(st, "meta_solve_batch: descriptors");
  };
  if ((s = upload(pk))) return s;

  // initial residuals (per problem, with the op's own kernels) and states
  std::vector<double> fn(np);
  std::vector<int> status(np, HELM_NOT_CONVERGED), checks(np, 0);
  for (int i = 0; i < np; ++i) {
    if ((s = vec_norm<S>(ops[i], f[i], &fn[i], st))) return s;
    if (!std::isfinite(fn[i])) return fail(HELM_E_NONFINITE, "meta_solve_batch: ||f|| of problem %d is not finite", i);
    if (!(fn[i] > 0)) fn[i] = 1.0;  // residual scale: absolute residual when f = 0
  }
  auto restart = [&](int i, double rn) -> helm_status {
    // r (already in its segment) becomes r_hat; fresh recurrence
    copy_vec<S>(pr[i].n, R.r + pr[i].off, R.rh + pr[i].off, st);
    BState b;
    std::memset(&b, 0, sizeof b);
    b.rho0[0] = b.alpha[0] = b.omega[0] = 1.0;
    b.thr = o->tol * fn[i];
    b.active = 1;
    b.first = 1;
    b.iters = hB[i].iters;
    b.s_stops = hB[i].s_stops;
    b.max_iters = o->max_iters;
    b.rr = rn;
    hB[i] = b;
    hipError_t e = hipMemcpyAsync(R.dB + i, &hB[i], sizeof(BState), hipMemcpyHostToDevice, st);
    if (e != hipSuccess) return hip_fail(e, "meta_solve_batch: state");
    return HELM_OK;
  };
  // rho = r_hat^H r into the element-wise partial slots of the current packing
  auto first_dot = [&](int only) {
    hipLaunchKernelGGL((kb_dot<S>), dim3(R.neb), dim3(256), 0, st, R.dP, R.dB, R.demap, only, R.rh, R.r, R.prho);
  };
  std::memset(hB, 0, sizeof(BState) * np);
  if (hipMemcpyAsync(R.dB, hB, sizeof(BState) * np, hipMemcpyHostToDevice, st) != hipSuccess)
    return fail(HELM_E_HIP, "meta_solve_batch: states");
  for (int i = 0; i < np; ++i) {
    double rn;
    if ((s = residual_norm<S>(ops[i], f[i], u[i], R.r + pr[i].off, &rn, st))) return s;
    stats[i].matvecs = 1;
    checks[i] = 1;
    if (!std::isfinite(rn)) status[i] = HELM_E_NONFINITE;
    else if (rn <= o->tol * fn[i]) status[i] = HELM_OK;
    else if (o->max_iters <= 0) status[i] = HELM_NOT_CONVERGED;
    else if ((s = restart(i, rn))) return s;
    stats[i].rel_res = rn / fn[i];
  }
  if ((s = sync_stream(st, "meta_solve_batch: init"))) return s;

  // capture a chunk of iterations once per packing
  hipGraphExec_t exec = nullptr;
  struct ExecGuard {
    hipGraphExec_t* e;
    ~ExecGuard() {
      if (*e) (void)hipGraphExecDestroy(*e);
    }
  } eguard{&exec};
  auto capture = [&]() -> helm_status {
    if (exec) {
      (void)hipGraphExecDestroy(exec);
      exec = nullptr;
    }
    hipGraph_t g;
    if (hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal) != hipSuccess)
      return fail(HELM_E_HIP, "meta_solve_batch: begin capture");
    for (int k = 0; k < ITERS_PER_GRAPH; ++k) R.iteration(st);
    hipError_t e = hipStreamEndCapture(st, &g);
    if (e != hipSuccess) return hip_fail(e, "meta_solve_batch: end capture");
    e = hipGraphInstantiate(&exec, g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    if (e != hipSuccess) return hip_fail(e, "meta_solve_batch: instantiate");
    return HELM_OK;
  };
  std::vector<int> live;
  for (int i = 0; i < np; ++i)
    if (status[i] == HELM_NOT_CONVERGED && hB[i].active) live.push_back(i);
  size_t packed = live.size();
  if (!live.empty()) {
    pack(pr, live, pk);
    if ((s = upload(pk))) return s;
    first_dot(-1);
    if ((s = capture())) return s;
  }
  hipEvent_t t0, t1;
  (void)hipEventCreate(&t0);
  (void)hipEventCreate(&t1);
  (void)hipEventRecord(t0, st);
  while (!live.empty()) {
    hipError_t e = hipGraphLaunch(exec, st);
    if (e == hipSuccess) e = hipMemcpyAsync(hB, R.dB, sizeof(BState) * np, hipMemcpyDeviceToHost, st);
    if (e != hipSuccess) {
      (void)hipEventDestroy(t0);
      (void)hipEventDestroy(t1);
      return hip_fail(e, "meta_solve_batch: replay");
    }
    if ((s = sync_stream(st, "meta_solve_batch: replay"))) {
      (void)hipEventDestroy(t0);
      (void)hipEventDestroy(t1);
      return s;
    }
    std::vector<int> next, restarted;
    for (int i : live) {
      const BState& b = hB[i];
      if (b.active) {
        next.push_back(i);
        continue;
      }
      if (b.flag) {
        status[i] = b.flag == -4 ? HELM_E_BREAKDOWN : HELM_E_NONFINITE;
        continue;
      }
      // recurrence stopped: true residual, then done or restart
      double rn;
      if ((s = residual_norm<S>(ops[i], f[i], u[i], R.r + pr[i].off, &rn, st))) return s;
      checks[i]++;
      stats[i].rel_res = rn / fn[i];
      if (!std::isfinite(rn)) status[i] = HELM_E_NONFINITE;
      else if (rn <= o->tol * fn[i]) status[i] = HELM_OK;
      else if (b.iters >= o->max_iters) status[i] = HELM_NOT_CONVERGED;
      else {
        if ((s = restart(i, rn))) return s;
        next.push_back(i);
        restarted.push_back(i);
      }
    }
    live.swap(next);
    if (!live.empty() && 2 * live.size() <= packed) {
      // repack: only the remaining problems' workgroups are launched; rho is
      // recomputed into the new partial slots (the same per-block sums)
      if ((s = sync_stream(st, "meta_solve_batch: repack"))) return s;
      pack(pr, live, pk);
      if ((s = upload(pk))) return s;
      first_dot(-1);
      if ((s = capture())) return s;
      packed = live.size();
    } else {
      for (int i : restarted) first_dot(i);
    }
  }
  (void)hipEventRecord(t1, st);
  (void)hipEventSynchronize(t1);
  float solve_ms = 0.f;
  (void)hipEventElapsedTime(&solve_ms, t0, t1);
  (void)hipEventDestroy(t0);
  (void)hipEventDestroy(t1);
  if ((s = sync_stream(st, "meta_solve_batch"))) return s;
  helm_status worst = HELM_OK;
  for (int i = 0; i < np; ++i) {
    const BState& b = hB[i];
    meta_stats& m = stats[i];
    m.iters = b.iters;
    m.matvecs = checks[i] + 2 * b.iters - b.s_stops;
    m.precond_apps = use_M ? 2 * b.iters - b.s_stops : 0;
    m.solve_ms = solve_ms;
    m.converged = status[i] == HELM_OK;
    if (status[i] < 0 && (worst >= 0 || status[i] < worst)) worst = (helm_status)status[i];
    else if (status[i] == HELM_NOT_CONVERGED && worst == HELM_OK) worst = HELM_NOT_CONVERGED;
  }
  return worst;
}

}  // namespace

}  // namespace helm

using namespace helm;

extern "C" helm_status meta_solve_batch(int count, const helm_op* ops, don_net net, const meta_opts* o,
                                        const void* const* f, void* const* u, meta_stats* st, void* stream) {
  if (count <= 0 || !ops || !o || !f || !u || !st) return fail(HELM_E_INVAL, "meta_solve_batch: bad argument");
  if (o->kind != META_BICGSTAB) return fail(HELM_E_INVAL, "meta_solve_batch: kind must be META_BICGSTAB");
  if (o->smoother != HELM_JACOBI) return fail(HELM_E_INVAL, "meta_solve_batch: the smoother must be HELM_JACOBI");
  if (o->mg_levels != 0) return fail(HELM_E_INVAL, "meta_solve_batch: the multigrid preconditioner is not batched");
  for (int i = 0; i < count; ++i) {
    if (!ops[i] || !f[i] || !u[i]) return fail(HELM_E_INVAL, "meta_solve_batch: NULL entry %d", i);
    if (f[i] == u[i]) return fail(HELM_E_INVAL, "meta_solve_batch: f and u alias in problem %d", i);
    if (ops[i]->dt != ops[0]->dt || ops[i]->dim != ops[0]->dim)
      return fail(HELM_E_INVAL, "meta_solve_batch: problems must share dtype and dimension");
    for (int j = 0; j < i; ++j)
      if (ops[j] == ops[i]) return fail(HELM_E_INVAL, "meta_solve_batch: op %d repeats op %d", i, j);
    helm_status s = check_opts(ops[i], net, o);
    if (s) return s;
  }
  hipStream_t hs = (hipStream_t)stream;
  const bool c128 = ops[0]->dt == HELM_C128;
  const bool q32 = !c128 || o->q_fp32;
  helm_op_s* const* P = ops;
  if (ops[0]->dim == 3) {
    if (c128) return q32 ? batch_drive<double, float, 3>(count, P, net, o, f, u, st, hs)
                         : batch_drive<double, double, 3>(count, P, net, o, f, u, st, hs);
    return batch_drive<float, float, 3>(count, P, net, o, f, u, st, hs);
  }
  if (c128) return q32 ? batch_drive<double, float, 2>(count, P, net, o, f, u, st, hs)
                       : batch_drive<double, double, 2>(count, P, net, o, f, u, st, hs);
  return batch_drive<float, float, 2>(count, P, net, o, f, u, st, hs);
}
