// Geometric multigrid preconditioner with the DeepONet-Jacobi smoother (§4.3,
// DeepONet-MG-Krylov): one V-cycle from zero per application.
//
// Level l + 1 keeps every second node of level l (coarse node j on fine node
// 2 j + 1, h' = 2 h); its operator is the rediscretisation with the
// coefficient and the scatterer mask injected.  Transfers: full weighting
// (3^dim fine neighbours, weights prod (1/2)^{|d|} / 2^dim, zero on coarse
// scatterer nodes) and multilinear prolongation with zero ghosts (zero on fine
// scatterer nodes).  Smoothing: nu damped Jacobi sweeps, or with a network
// a Jacobi sweeps, one trunk-basis correction of that level, b sweeps
// (a = nu / 2, b = nu - a - 1), before and after the coarse-grid correction.
// The coarsest level (at most 128 nodes) is solved with an explicit inverse.
// Every level is an op of its own, so the stencil, residual and trunk-basis
// kernels of the single-grid path are reused unchanged.
#include <hip/hip_runtime.h>

#include <cmath>
#include <complex>
#include <vector>

#include "common.h"
#include "dense.h"
#include "internal.h"
#include "lib.h"

namespace helm {

struct Mg {
  int levels = 0, nu = 0, p_used = 0, net_serial = -1, ksq_version = -1, dt = 0;
  std::vector<helm_op_s*> ops;  // ops[0] is the caller's op (not owned)
  std::vector<Buffer> f, u, r;  // per level >= 1: right-hand side, iterate; residual per level
  Buffer Ainv, work;            // coarsest inverse (complex128) and its scratch
  int nc = 0;
  ~Mg() {
    for (size_t l = 1; l < ops.size(); ++l) helm_destroy(ops[l]);
    for (auto* v : {&f, &u, &r})
      for (auto& b : *v) b.release();
    Ainv.release();
    work.release();
  }
};

namespace {

template <typename S>
__global__ void k_inject(int dim, int fx, int fy, int cx, int cy, int cz, const cplx_t<S>* __restrict__ sf,
                         const uint8_t* __restrict__ mf, const double* __restrict__ af, cplx_t<S>* __restrict__ sc,
                         uint8_t* __restrict__ mc, double* __restrict__ ac) {
  const size_t n = (size_t)cx * cy * cz;
  for (size_t p = blockIdx.x * (size_t)blockDim.x + threadIdx.x; p < n; p += (size_t)gridDim.x * blockDim.x) {
    const int i = (int)(p % cx), j = (int)((p / cx) % cy), k = (int)(p / ((size_t)cx * cy));
    const size_t q = (size_t)(2 * i + 1) + (size_t)fx * ((size_t)(2 * j + 1) + (size_t)fy * (dim == 3 ? 2 * k + 1 : 0));
    sc[p] = sf[q];
    mc[p] = mf[q];
    ac[p] = af ? af[q] : 0.0;
  }
}

// full weighting of r (fine fx x fy x fz) onto the coarse grid
template <typename S>
__global__ __launch_bounds__(256) void k_restrict(int dim, int fx, int fy, int cx, int cy, int cz,
                                                  const cplx_t<S>* __restrict__ r, const uint8_t* __restrict__ mc,
                                                  cplx_t<S>* __restrict__ out) {
  const size_t n = (size_t)cx * cy * cz;
  for (size_t p = blockIdx.x * (size_t)blockDim.x + threadIdx.x; p < n; p += (size_t)gridDim.x * blockDim.x) {
    if (mc[p]) {
      stc(out, p, czero());
      continue;
    }
    const int i = (int)(p % cx), j = (int)((p / cx) % cy), k = (int)(p / ((size_t)cx * cy));
    const int I = 2 * i + 1, J = 2 * j + 1, K = dim == 3 ? 2 * k + 1 : 0;
    double2 a = czero();
    const int dz0 = dim == 3 ? -1 : 0, dz1 = dim == 3 ? 1 : 0;
    for (int dz = dz0; dz <= dz1; ++dz)
      for (int dy = -1; dy <= 1; ++dy)
        for (int dx = -1; dx <= 1; ++dx) {
          const double w = (dx ? 0.5 : 1.0) * (dy ? 0.5 : 1.0) * (dz ? 0.5 : 1.0) / (dim == 3 ? 8.0 : 4.0);
          const size_t q = (size_t)(I + dx) + (size_t)fx * ((size_t)(J + dy) + (size_t)fy * (K + dz));
          const double2 v = ldc(r, q);
          a.x += w * v.x;
          a.y += w * v.y;
        }
    stc(out, p, a);
  }
}

// u_f += P e (multilinear, zero coarse ghosts), skipping fine scatterer nodes
template <typename S>
__global__ __launch_bounds__(256) void k_prolong_add(int dim, int fx, int fy, int fz, int cx, int cy, int cz,
                                                     const cplx_t<S>* __restrict__ e, const uint8_t* __restrict__ mf,
                                                     cplx_t<S>* __restrict__ u) {
  const size_t n = (size_t)fx * fy * fz;
  for (size_t p = blockIdx.x * (size_t)blockDim.x + threadIdx.x; p < n; p += (size_t)gridDim.x * blockDim.x) {
    if (mf[p]) continue;
    const int idx[3] = {(int)(p % fx), (int)((p / fx) % fy), (int)(p / ((size_t)fx * fy))};
    const int cn[3] = {cx, cy, cz};
    int lo[3], hi[3];
    double wl[3], wh[3];
    for (int a = 0; a < 3; ++a) {
      if (a >= dim) {
        lo[a] = hi[a] = 0;
        wl[a] = 1.0;
        wh[a] = 0.0;
      } else if (idx[a] & 1) {
        lo[a] = hi[a] = (idx[a] - 1) / 2;
        wl[a] = 1.0;
        wh[a] = 0.0;
      } else {
        lo[a] = idx[a] / 2 - 1;
        hi[a] = idx[a] / 2;
        wl[a] = wh[a] = 0.5;
      }
    }
    double2 acc = czero();
    for (int c = 0; c < 8; ++c) {
      const int pick[3] = {c & 1, (c >> 1) & 1, (c >> 2) & 1};
      double w = 1.0;
      int J[3];
      bool ok = true;
      for (int a = 0; a < 3; ++a) {
        w *= pick[a] ? wh[a] : wl[a];
        J[a] = pick[a] ? hi[a] : lo[a];
        if (J[a] < 0 || J[a] >= cn[a]) ok = false;
      }
      if (w == 0.0 || !ok) continue;
      const double2 v = ldc(e, (size_t)J[0] + (size_t)cx * ((size_t)J[1] + (size_t)cy * J[2]));
      acc.x += w * v.x;
      acc.y += w * v.y;
    }
    stc(u, p, cadd(ldc(u, p), acc));
  }
}

// out = A^{-1} f on the coarsest level (A^{-1} complex128 row-major, nc <= 128)
template <typename S>
__global__ __launch_bounds__(64) void k_dense_apply(int nc, const double* __restrict__ Ainv,
                                                    const cplx_t<S>* __restrict__ f, cplx_t<S>* __restrict__ out) {
  const int j = blockIdx.x, l = threadIdx.x;
  double2 acc = czero();
  for (int k = l; k < nc; k += 64) {
    const size_t o = 2 * ((size_t)j * nc + k);
    acc = cadd(acc, cmul(make_double2(Ainv[o], Ainv[o + 1]), ldc(f, k)));
  }
  acc.x = wave_sum(acc.x);
  acc.y = wave_sum(acc.y);
  if (l == 0) stc(out, j, acc);
}

unsigned grid_for(size_t n) {
  size_t b = (n + 255) / 256;
  if (b > 8192) b = 8192;
  return (unsigned)(b ? b : 1);
}

// A coarse op (every second node) of `fine`, coefficient, alpha and mask injected.
helm_status coarse_op(const helm_op_s* fine, hipStream_t st, helm_op_s** out) {
  helm_op_s* op = new helm_op_s();
  op->dim = fine->dim;
  op->n[0] = (fine->n[0] + 1) / 2 - 1;
  op->n[1] = (fine->n[1] + 1) / 2 - 1;
  op->n[2] = fine->dim == 3 ? (fine->n[2] + 1) / 2 - 1 : 1;
  op->nn = (size_t)op->n[0] * op->n[1] * op->n[2];
  op->dt = fine->dt;
  op->geom = make_geom(op->dim, op->n, 0);
  helm_status s;
  if ((s = dalloc(&op->sc, op->nn * op_esz(op))) || (s = dalloc((void**)&op->mask, op->nn)) ||
      (s = dalloc((void**)&op->alpha, op->nn * sizeof(double))) || (s = dalloc((void**)&op->code, (op->nn + 3) & ~(size_t)3)) ||
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
    return hip_fail(e, "multigrid: pinned scalars");
  }
  if (op->dt == HELM_C128)
    hipLaunchKernelGGL(k_inject<double>, dim3(grid_for(op->nn)), dim3(256), 0, st, op->dim, fine->n[0], fine->n[1],
                       op->n[0], op->n[1], op->n[2], (const double2*)fine->sc, fine->mask, fine->alpha,
                       (double2*)op->sc, op->mask, op->alpha);
  else
    hipLaunchKernelGGL(k_inject<float>, dim3(grid_for(op->nn)), dim3(256), 0, st, op->dim, fine->n[0], fine->n[1],
                       op->n[0], op->n[1], op->n[2], (const float2*)fine->sc, fine->mask, fine->alpha,
                       (float2*)op->sc, op->mask, op->alpha);
  build_codes(op->geom, op->mask, op->code, st);
  if ((s = sync_stream(st, "multigrid: coarse op"))) {
    helm_destroy(op);
    return s;
  }
  *out = op;
  return HELM_OK;
}

// Dense matrix of a (small) op from its coefficients, by the definition of eq. 1.
template <typename S>
helm_status dense_of(const helm_op_s* op, std::vector<double>& A, hipStream_t st) {
  const size_t n = op->nn;
  std::vector<cplx_t<S>> sh(n);
  std::vector<uint8_t> mh(n);
  hipError_t e = hipMemcpyAsync(sh.data(), op->sc, n * sizeof(cplx_t<S>), hipMemcpyDeviceToHost, st);
  if (e == hipSuccess) e = hipMemcpyAsync(mh.data(), op->mask, n, hipMemcpyDeviceToHost, st);
  if (e != hipSuccess) return hip_fail(e, "multigrid: coarsest coefficients");
  helm_status s = sync_stream(st, "multigrid: coarsest coefficients");
  if (s) return s;
  A.assign(2 * n * n, 0.0);
  const int nx = op->n[0], ny = op->n[1], nz = op->n[2];
  double ih2[3] = {0, 0, 0};
  for (int a = 0; a < op->dim; ++a) {
    const double h = 1.0 / (op->n[a] + 1);
    ih2[a] = 1.0 / (h * h);
  }
  for (size_t p = 0; p < n; ++p) {
    if (mh[p]) {
      A[2 * (p * n + p)] = 1.0;
      continue;
    }
    const int idx[3] = {(int)(p % nx), (int)((p / nx) % ny), (int)(p / ((size_t)nx * ny))};
    const int dims[3] = {nx, ny, nz};
    const size_t stride[3] = {1, (size_t)nx, (size_t)nx * ny};
    double diag = 0.0;
    for (int a = 0; a < op->dim; ++a) {
      diag += 2.0 * ih2[a];
      for (int step = -1; step <= 1; step += 2) {
        const int qa = idx[a] + step;
        if (qa < 0 || qa >= dims[a]) continue;
        const size_t q = step < 0 ? p - stride[a] : p + stride[a];
        if (mh[q]) continue;
        A[2 * (p * n + q)] -= ih2[a];
      }
    }
    A[2 * (p * n + p)] = diag - (double)sh[p].x;
    A[2 * (p * n + p) + 1] = -(double)sh[p].y;
  }
  return HELM_OK;
}

template <typename S>
helm_status smooth(Mg& m, int l, const meta_opts* o, don_s* net, const void* f, void* u, bool from_zero,
                   void* r, hipStream_t st) {
  helm_op_s* op = m.ops[l];
  const size_t n = op->nn;
  helm_status s;
  if ((s = op->tmp.ensure(n * op_esz(op)))) return s;
  // `count` Jacobi sweeps on u (from zero when z0), ending in u
  auto sweeps = [&](int count, bool z0) {
    if (count <= 0) {
      if (z0) zero_vec<S>(n, u, st);
      return;
    }
    void* a = u;
    void* b = op->tmp.ptr;
    int rest = count;
    if (z0) {
      if (count == 1) {
        jacobi_from_zero<S>(n, op->geom.dsum, op->sc, op->mask, f, u, o->omega, st);
        return;
      }
      // the first two sweeps fused; the rest ping-pong so that the last lands in u
      rest = count - 2;
      a = (rest & 1) ? op->tmp.ptr : u;
      b = (rest & 1) ? u : op->tmp.ptr;
      jacobi2_from_zero<S>(op->geom, op->sc, op->code, f, a, o->omega, st);
    }
    for (int k = 0; k < rest; ++k) {
      stencil_jacobi<S>(op->geom, op->sc, op->code, f, a, b, o->omega, st);
      void* t = a;
      a = b;
      b = t;
    }
    if (a != u) copy_vec<S>(n, a, u, st);
  };
  if (!net) {
    sweeps(m.nu, from_zero);
    return launch_check("multigrid smoother");
  }
  const int a = m.nu / 2, b = m.nu - a - 1;
  sweeps(a, from_zero);
  double* part;
  if ((s = op_part(op, (size_t)stencil_nblocks(op->geom), &part))) return s;
  stencil_resid<S>(op->geom, op->sc, op->code, f, u, r, part, st);
  if ((s = coarse_correct<S>(op, r, u, st))) return s;
  sweeps(b, false);
  return launch_check("multigrid smoother");
}

template <typename S>
helm_status vcycle(Mg& m, int l, const meta_opts* o, don_s* net, const void* f, void* u, hipStream_t st) {
  using C = cplx_t<S>;
  helm_op_s* op = m.ops[l];
  if (l == m.levels) {
    hipLaunchKernelGGL(k_dense_apply<S>, dim3(m.nc), dim3(64), 0, st, m.nc, (const double*)m.Ainv.ptr, (const C*)f,
                       (C*)u);
    return launch_check("multigrid coarsest solve");
  }
  void* r = m.r[l].ptr;
  helm_status s;
  if ((s = smooth<S>(m, l, o, net, f, u, true, r, st))) return s;
  double* part;
  if ((s = op_part(op, (size_t)stencil_nblocks(op->geom), &part))) return s;
  stencil_resid<S>(op->geom, op->sc, op->code, f, u, r, part, st);
  helm_op_s* cop = m.ops[l + 1];
  hipLaunchKernelGGL(k_restrict<S>, dim3(grid_for(cop->nn)), dim3(256), 0, st, op->dim, op->n[0], op->n[1], cop->n[0],
                     cop->n[1], cop->n[2], (const C*)r, cop->mask, (C*)m.f[l + 1].ptr);
  if ((s = vcycle<S>(m, l + 1, o, net, m.f[l + 1].ptr, m.u[l + 1].ptr, st))) return s;
  hipLaunchKernelGGL(k_prolong_add<S>, dim3(grid_for(op->nn)), dim3(256), 0, st, op->dim, op->n[0], op->n[1],
                     op->n[2], cop->n[0], cop->n[1], cop->n[2], (const C*)m.u[l + 1].ptr, op->mask, (C*)u);
  return smooth<S>(m, l, o, net, f, u, false, r, st);
}

}  // namespace

void mg_release(helm_op_s* op) {
  delete op->mg;
  op->mg = nullptr;
}

helm_status mg_check(const helm_op_s* op, const meta_opts* o) {
  const int L = o->mg_levels;
  if (L < 0 || L > 8) return fail(HELM_E_INVAL, "multigrid: mg_levels %d outside [0, 8]", L);
  if (L == 0) return HELM_OK;
  if (o->kind != META_GMRES && o->kind != META_BICGSTAB)
    return fail(HELM_E_INVAL, "multigrid: the V-cycle preconditions META_GMRES or META_BICGSTAB");
  if (o->smoother != HELM_JACOBI) return fail(HELM_E_INVAL, "multigrid: the smoother must be HELM_JACOBI");
  if (o->mg_nu < 1 || o->mg_nu > 64) return fail(HELM_E_INVAL, "multigrid: mg_nu %d outside [1, 64]", o->mg_nu);
  size_t nc = 1;
  for (int a = 0; a < op->dim; ++a) {
    if ((op->n[a] + 1) % (1 << L))
      return fail(HELM_E_INVAL, "multigrid: n[%d] + 1 = %d is not divisible by 2^%d", a, op->n[a] + 1, L);
    const int c = (op->n[a] + 1) / (1 << L) - 1;
    if (c < 1) return fail(HELM_E_INVAL, "multigrid: %d levels leave no coarse nodes on axis %d", L, a);
    nc *= (size_t)c;
  }
  if (nc > 128) return fail(HELM_E_INVAL, "multigrid: the coarsest grid has %zu > 128 nodes; use more levels", nc);
  return HELM_OK;
}

// Build (or reuse) the hierarchy of op for opts o and network net.
helm_status mg_ensure(helm_op_s* op, don_s* net, const meta_opts* o, hipStream_t st) {
  Mg* m = op->mg;
  const int serial = net ? don_serial(net) : 0;
  if (m && m->levels == o->mg_levels && m->nu == o->mg_nu && m->net_serial == serial &&
      m->ksq_version == op->ksq_version && m->p_used == o->p_used && m->dt == op->dt)
    return HELM_OK;
  mg_release(op);
  m = new Mg();
  op->mg = m;
  m->levels = o->mg_levels;
  m->nu = o->mg_nu;
  m->p_used = o->p_used;
  m->net_serial = serial;
  m->ksq_version = op->ksq_version;
  m->dt = op->dt;
  m->ops.push_back(op);
  helm_status s;
  for (int l = 1; l <= m->levels; ++l) {
    helm_op_s* c;
    if ((s = coarse_op(m->ops[l - 1], st, &c))) {
      mg_release(op);
      return s;
    }
    m->ops.push_back(c);
  }
  m->f.resize(m->levels + 1);
  m->u.resize(m->levels + 1);
  m->r.resize(m->levels + 1);
  for (int l = 0; l <= m->levels; ++l) {
    const size_t fb = m->ops[l]->nn * op_esz(op);
    if ((s = m->r[l].ensure(fb)) || (l > 0 && ((s = m->f[l].ensure(fb)) || (s = m->u[l].ensure(fb))))) {
      mg_release(op);
      return s;
    }
  }
  // trunk-basis spaces of the smoothing levels
  if (net)
    for (int l = 0; l < m->levels; ++l) {
      const int pu = (size_t)o->p_used < m->ops[l]->nn ? o->p_used : (int)m->ops[l]->nn;
      if ((s = coarse_ensure(m->ops[l], net, pu, o->q_fp32 != 0, o->no_drop != 0, st))) {
        mg_release(op);
        return s;
      }
    }
  // coarsest inverse
  helm_op_s* cop = m->ops[m->levels];
  m->nc = (int)cop->nn;
  std::vector<double> A;
  s = op->dt == HELM_C128 ? dense_of<double>(cop, A, st) : dense_of<float>(cop, A, st);
  if (!s) s = m->Ainv.ensure(A.size() * sizeof(double));
  if (!s) s = m->work.ensure(A.size() * sizeof(double) + 64 * sizeof(double));
  if (s) {
    mg_release(op);
    return s;
  }
  hipError_t e = hipMemcpyAsync(m->work.ptr, A.data(), A.size() * sizeof(double), hipMemcpyHostToDevice, st);
  if (e != hipSuccess) {
    mg_release(op);
    return hip_fail(e, "multigrid: coarsest matrix");
  }
  double* info = (double*)m->work.ptr + A.size();
  gj_inverse(m->nc, (const double*)m->work.ptr, nullptr, (double*)m->Ainv.ptr, (int*)info, info + 2, st);
  int hinfo = 0;
  e = hipMemcpyAsync(&hinfo, info, sizeof(int), hipMemcpyDeviceToHost, st);
  if (e != hipSuccess || (s = sync_stream(st, "multigrid: coarsest inverse"))) {
    mg_release(op);
    return e != hipSuccess ? hip_fail(e, "multigrid: coarsest inverse") : s;
  }
  if (hinfo) {
    mg_release(op);
    return fail(HELM_E_SINGULAR, "multigrid: the coarsest operator is singular");
  }
  return HELM_OK;
}

// z = one V-cycle on A z = v from zero; r1 is a field of scratch on the finest level.
template <typename S>
helm_status mg_apply(helm_op_s* op, don_s* net, const meta_opts* o, const void* v, void* z, hipStream_t st) {
  Mg* m = op->mg;
  if (!m) return fail(HELM_E_INVAL, "multigrid: hierarchy not built");
  return vcycle<S>(*m, 0, o, net, v, z, st);
}

template helm_status mg_apply<double>(helm_op_s*, don_s*, const meta_opts*, const void*, void*, hipStream_t);
template helm_status mg_apply<float>(helm_op_s*, don_s*, const meta_opts*, const void*, void*, hipStream_t);

}  // namespace helm
