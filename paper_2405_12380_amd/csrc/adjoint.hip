// Pieces of the k^2 gradient of a receiver misfit (§2 eq. 1 differentiated):
// complex conjugation (A is complex symmetric, so A^H x = conj(A conj(x))),
// the receiver misfit with its adjoint source, and the pointwise gradient
// Re(conj(lam) (1 + i alpha) u).  All HBM-bound streaming kernels.
#include "common.h"
#include "internal.h"
#include "lib.h"

namespace helm {

template <typename S>
__global__ __launch_bounds__(256) void k_conj(size_t n, const cplx_t<S>* __restrict__ x, cplx_t<S>* y) {
  const size_t e = blockIdx.x * (size_t)blockDim.x + threadIdx.x;
  if (e >= n) return;
  cplx_t<S> v = x[e];
  v.y = -v.y;
  y[e] = v;
}

// One thread per receiver: plane entry j = a + na b sits at node
// base + a sa + b sb.  r = u - d; g = r off the scatterer (0 on it); per-block
// partial sums of |r|^2.  g must be zero elsewhere (cleared by the caller).
template <typename S>
__global__ __launch_bounds__(256) void k_misfit(int m, int na, size_t base, size_t sa, size_t sb,
                                                const cplx_t<S>* __restrict__ u, const cplx_t<S>* __restrict__ d,
                                                const uint8_t* __restrict__ mask, cplx_t<S>* __restrict__ g,
                                                double* __restrict__ part) {
  __shared__ double sh[16];
  const int j = blockIdx.x * 256 + threadIdx.x;
  double acc = 0.0;
  if (j < m) {
    const int a = j % na, b = j / na;
    const size_t node = base + (size_t)a * sa + (size_t)b * sb;
    const double2 r = csub(ldc(u, node), ldc(d, (size_t)j));
    acc = r.x * r.x + r.y * r.y;
    stc(g, node, mask[node] ? czero() : r);
  }
  acc = block_sum(acc, sh);
  if (threadIdx.x == 0) part[blockIdx.x] = acc;
}

// grad_p = Re(conj(lam_p) (1 + i alpha_p) u_p) = Re(w) - alpha_p Im(w), w = conj(lam_p) u_p; 0 on the scatterer.
template <typename S>
__global__ __launch_bounds__(256) void k_ksq_grad(size_t n, const cplx_t<S>* __restrict__ u,
                                                  const cplx_t<S>* __restrict__ lam, const double* __restrict__ alpha,
                                                  const uint8_t* __restrict__ mask, S* __restrict__ grad) {
  const size_t e = blockIdx.x * (size_t)blockDim.x + threadIdx.x;
  if (e >= n) return;
  const double2 w = cconjmul(ldc(lam, e), ldc(u, e));
  grad[e] = mask[e] ? (S)0 : (S)(w.x - alpha[e] * w.y);
}

static unsigned ew_blocks(size_t n) { return (unsigned)((n + 255) / 256); }

template <typename S>
void conj_vec(size_t n, const void* x, void* y, hipStream_t st) {
  using C = cplx_t<S>;
  if (n) hipLaunchKernelGGL((k_conj<S>), dim3(ew_blocks(n)), dim3(256), 0, st, n, (const C*)x, (C*)y);
}

template <typename S>
static helm_status misfit_t(helm_op_s* op, int axis, int index, const void* u, const void* d, void* g, double* loss,
                            hipStream_t st) {
  using C = cplx_t<S>;
  const size_t stride[3] = {1, (size_t)op->n[0], (size_t)op->n[0] * op->n[1]};
  int r0 = -1, r1 = -1;
  for (int a = 0; a < 3; ++a)
    if (a != axis) (r0 < 0 ? r0 : r1) = a;
  const int na = op->n[r0], nb = op->n[r1];  // n[2] = 1 on 2D grids
  const int m = na * nb;
  const int nblk = (m + 255) / 256;
  double* part;
  helm_status s = op_part(op, (size_t)nblk, &part);
  if (s) return s;
  zero_vec<S>(op->nn, g, st);
  hipLaunchKernelGGL((k_misfit<S>), dim3(nblk), dim3(256), 0, st, m, na, (size_t)index * stride[axis], stride[r0],
                     stride[r1], (const C*)u, (const C*)d, op->mask, (C*)g, part);
  if (!loss) return launch_check("helm_misfit");
  reduce_cols(part, nblk, 1, op->red, st);
  hipError_t e = hipMemcpyAsync(op->host, op->red, sizeof(double), hipMemcpyDeviceToHost, st);
  if (e != hipSuccess) return hip_fail(e, "helm_misfit: readback");
  if ((s = sync_stream(st, "helm_misfit"))) return s;
  *loss = 0.5 * op->host[0];
  return HELM_OK;
}

#define HELM_ADJ_INST(S) template void conj_vec<S>(size_t, const void*, void*, hipStream_t);
HELM_ADJ_INST(double)
HELM_ADJ_INST(float)
#undef HELM_ADJ_INST

}  // namespace helm

using namespace helm;

extern "C" {

helm_status helm_misfit(helm_op op, int axis, int index, const void* u, const void* d, void* g, double* loss,
                        void* stream) {
  if (!op || !u || !d || !g) return fail(HELM_E_INVAL, "helm_misfit: NULL argument");
  if (axis < 0 || axis >= op->dim) return fail(HELM_E_INVAL, "helm_misfit: axis %d outside the grid's %d axes", axis,
                                               op->dim);
  if (index < 0 || index >= op->n[axis])
    return fail(HELM_E_INVAL, "helm_misfit: plane index %d outside [0, %d)", index, op->n[axis]);
  if (g == u || g == d) return fail(HELM_E_INVAL, "helm_misfit: g aliases an input");
  hipStream_t st = (hipStream_t)stream;
  return op->dt == HELM_C128 ? misfit_t<double>(op, axis, index, u, d, g, loss, st)
                             : misfit_t<float>(op, axis, index, u, d, g, loss, st);
}

helm_status helm_ksq_gradient(helm_op op, const void* u, const void* lam, void* grad, void* stream) {
  if (!op || !u || !lam || !grad) return fail(HELM_E_INVAL, "helm_ksq_gradient: NULL argument");
  if (grad == u || grad == lam) return fail(HELM_E_INVAL, "helm_ksq_gradient: grad aliases an input");
  hipStream_t st = (hipStream_t)stream;
  const size_t n = op->nn;
  if (op->dt == HELM_C128)
    hipLaunchKernelGGL((k_ksq_grad<double>), dim3(ew_blocks(n)), dim3(256), 0, st, n, (const double2*)u,
                       (const double2*)lam, op->alpha, op->mask, (double*)grad);
  else
    hipLaunchKernelGGL((k_ksq_grad<float>), dim3(ew_blocks(n)), dim3(256), 0, st, n, (const float2*)u,
                       (const float2*)lam, op->alpha, op->mask, (float*)grad);
  return launch_check("helm_ksq_gradient");
}

}  // extern "C"
