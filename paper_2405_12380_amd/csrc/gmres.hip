// Small dense GMRES work on the device: completion of an Arnoldi column
// (CGS2 coefficients, complex Givens rotations, residual estimate) and the
// upper-triangular back-solve.  O(m) / O(m^2) work in fp64, one thread: the
// host never touches H, so a cycle needs no host round trip except the
// convergence flag.
#include "common.h"
#include "internal.h"

namespace helm {

__device__ static inline double2 H_at(const double* H, int m, int i, int j) {
  const size_t o = 2 * ((size_t)j * (m + 1) + i);
  return make_double2(H[o], H[o + 1]);
}
__device__ static inline void H_set(double* H, int m, int i, int j, double2 v) {
  const size_t o = 2 * ((size_t)j * (m + 1) + i);
  H[o] = v.x;
  H[o + 1] = v.y;
}
__device__ static inline double cabs2(double2 a) { return hypot(a.x, a.y); }

__global__ void k_arnoldi_finish(int j, int m, double* H, double* g, double* cs, double* sn, const double* h1,
                                 const double* h2, const double* nrm2, GmState* gs) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  for (int i = 0; i <= j; ++i)
    H_set(H, m, i, j, make_double2(h1[2 * i] + h2[2 * i], h1[2 * i + 1] + h2[2 * i + 1]));
  const double hn = sqrt(nrm2[0]);
  gs->hn = hn;
  gs->inv_hn = hn != 0.0 ? 1.0 / hn : 0.0;
  // previous rotations G_i = [[c, s], [-conj(s), c]] on rows (i, i+1)
  for (int i = 0; i < j; ++i) {
    const double2 a = H_at(H, m, i, j), b = H_at(H, m, i + 1, j);
    const double c = cs[i];
    const double2 s = make_double2(sn[2 * i], sn[2 * i + 1]);
    const double2 sconj = make_double2(s.x, -s.y);
    H_set(H, m, i, j, cadd(cscale(a, c), cmul(s, b)));
    H_set(H, m, i + 1, j, csub(cscale(b, c), cmul(sconj, a)));
  }
  const double2 a = H_at(H, m, j, j);
  const double b = hn;
  double c;
  double2 s;
  if (b == 0.0) {
    c = 1.0;
    s = czero();
  } else if (a.x == 0.0 && a.y == 0.0) {
    c = 0.0;
    s = make_double2(1.0, 0.0);
  } else {
    const double aa = cabs2(a);
    const double nu = sqrt(aa * aa + b * b);
    c = aa / nu;
    s = cscale(make_double2(a.x / aa, a.y / aa), b / nu);
  }
  cs[j] = c;
  sn[2 * j] = s.x;
  sn[2 * j + 1] = s.y;
  H_set(H, m, j, j, cadd(cscale(a, c), cscale(s, b)));
  H_set(H, m, j + 1, j, czero());
  const double2 gj = make_double2(g[2 * j], g[2 * j + 1]);
  const double2 gn = cmul(make_double2(-s.x, s.y), gj);  // -conj(s) g_j
  g[2 * (j + 1)] = gn.x;
  g[2 * (j + 1) + 1] = gn.y;
  g[2 * j] = c * gj.x;
  g[2 * j + 1] = c * gj.y;
  gs->gabs = cabs2(gn);
  gs->flag = (isfinite(hn) && isfinite(gs->gabs)) ? 0 : -5;
}

__global__ void k_backsolve(int k, int m, const double* H, const double* g, double* y) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  for (int i = k - 1; i >= 0; --i) {
    double2 acc = czero();
    for (int l = i + 1; l < k; ++l) acc = cadd(acc, cmul(H_at(H, m, i, l), make_double2(y[2 * l], y[2 * l + 1])));
    const double2 v = cdiv(csub(make_double2(g[2 * i], g[2 * i + 1]), acc), H_at(H, m, i, i));
    y[2 * i] = v.x;
    y[2 * i + 1] = v.y;
  }
}

__global__ void k_gmres_init(double beta, double* g, int m) {
  for (int i = threadIdx.x; i < 2 * (m + 1); i += blockDim.x) g[i] = 0.0;
  __syncthreads();
  if (threadIdx.x == 0) g[0] = beta;
}

void arnoldi_finish(int j, int m, double* H, double* g, double* cs, double* sn, const double* h1, const double* h2,
                    const double* nrm2, GmState* gs, hipStream_t st) {
  hipLaunchKernelGGL(k_arnoldi_finish, dim3(1), dim3(64), 0, st, j, m, H, g, cs, sn, h1, h2, nrm2, gs);
}
void gmres_backsolve(int k, int m, const double* H, const double* g, double* y, hipStream_t st) {
  hipLaunchKernelGGL(k_backsolve, dim3(1), dim3(64), 0, st, k, m, H, g, y);
}
void gmres_init(double beta, double* g, int m, hipStream_t st) {
  hipLaunchKernelGGL(k_gmres_init, dim3(1), dim3(256), 0, st, beta, g, m);
}

}  // namespace helm
