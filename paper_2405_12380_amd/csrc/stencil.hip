// Stencil kernels of the discrete Helmholtz operator (§2 eq. 1) and of the
// point relaxations of eq. 2 (damped Jacobi, red-black Gauss-Seidel).
//
// Mapping: a workgroup is 64 x ty threads (ty = 4, or 8 on large grids),
// lanes along x (a wavefront reads
// one contiguous 1 KiB (complex128) row segment per load), 4 rows in y, and
// each thread marches over `zb` consecutive z-planes keeping the z-1, z, z+1
// values of its column in registers, so every node is loaded from HBM once;
// x/y neighbours are re-read from L1/L2.  Masks enter through one neighbour
// code byte per node, so all loads of a node are independent and issued
// together.  Logical blocks are laid out x-, y-,
// then z-fastest and remapped so that each XCD owns one contiguous range of
// them (one z-slab), keeping halo re-reads inside that XCD's L2.
//
// Per-node arithmetic is fixed (independent of the tiling): the axis terms
// ((c - x_minus) + (c - x_plus)) / h_a^2 are accumulated x, y, z in turn and
// s_p c is subtracted last, in fp64 for both storage precisions.
#include "common.h"
#include "internal.h"
#include "prof.h"
#include "stencil_dev.h"

namespace helm {

__global__ void k_build_codes(int dim, int nx, int ny, int nz, const uint8_t* __restrict__ mask,
                              uint8_t* __restrict__ code) {
  const size_t n = (size_t)nx * ny * nz, plane = (size_t)nx * ny;
  for (size_t p = blockIdx.x * (size_t)blockDim.x + threadIdx.x; p < n; p += (size_t)gridDim.x * blockDim.x) {
    const int i = (int)(p % nx), j = (int)((p / nx) % ny), l = (int)(p / plane);
    uint8_t c = mask[p] ? NB_SELF : 0;
    if (i == 0 || mask[p - 1]) c |= NB_XM;
    if (i + 1 == nx || mask[p + 1]) c |= NB_XP;
    if (j == 0 || mask[p - nx]) c |= NB_YM;
    if (j + 1 == ny || mask[p + nx]) c |= NB_YP;
    if (dim == 3) {
      if (l == 0 || mask[p - plane]) c |= NB_ZM;
      if (l + 1 == nz || mask[p + plane]) c |= NB_ZP;
    }
    code[p] = c;
  }
}

static int stencil_blocks(const StencilGeom& g) {
  const int nbx = (g.nx + 63) / 64, nby = (g.ny + g.ty - 1) / g.ty, nbz = (g.nz + g.zb - 1) / g.zb;
  return nbx * nby * nbz;
}

template <typename S, int DIM, int MODE>
__global__ __launch_bounds__(512) void k_stencil(StencilGeom g, const cplx_t<S>* __restrict__ sc,
                                                 const uint8_t* __restrict__ code, const cplx_t<S>* x,
                                                 const cplx_t<S>* __restrict__ f, cplx_t<S>* y,
                                                 double omega, int color, double* __restrict__ partials) {
  const unsigned lb = xcd_remap(blockIdx.x, gridDim.x);
  stencil_tile<S, DIM, MODE>(g, lb, sc, code, x, f, y, omega, color, MODE == ST_RESID ? partials + lb : nullptr);
}

template <typename S, int DIM>
__global__ __launch_bounds__(512) void k_jacobi2z(StencilGeom g, const cplx_t<S>* __restrict__ sc,
                                                  const uint8_t* __restrict__ code, const cplx_t<S>* __restrict__ f,
                                                  cplx_t<S>* __restrict__ y, double omega) {
  jacobi2z_tile<S, DIM>(g, xcd_remap(blockIdx.x, gridDim.x), sc, code, f, y, omega);
}

template <typename S>
void jacobi2_from_zero(const StencilGeom& g, const void* sc, const uint8_t* code, const void* f, void* z, double omega,
                       hipStream_t st) {
  using C = cplx_t<S>;
  const int nb = stencil_blocks(g);
  const double n = (double)g.nx * g.ny * g.nz, esz = 2.0 * sizeof(S);
  kprof_begin(st);
  if (g.dim == 3)
    hipLaunchKernelGGL((k_jacobi2z<S, 3>), dim3(nb), dim3(64, g.ty), 0, st, g, (const C*)sc, code, (const C*)f, (C*)z,
                       omega);
  else
    hipLaunchKernelGGL((k_jacobi2z<S, 2>), dim3(nb), dim3(64, g.ty), 0, st, g, (const C*)sc, code, (const C*)f, (C*)z,
                       omega);
  kprof_end(KP_STENCIL, n * (3 * esz + 1), st);
}

// z = omega D^{-1} f: a Jacobi sweep started from z = 0 (no stencil needed).
template <typename S>
__global__ __launch_bounds__(256) void k_jacobi0(size_t n, double dsum, const cplx_t<S>* __restrict__ sc,
                                                 const uint8_t* __restrict__ mask,
                                                 const cplx_t<S>* __restrict__ f, cplx_t<S>* __restrict__ z,
                                                 double omega) {
  for (size_t p = blockIdx.x * (size_t)blockDim.x + threadIdx.x; p < n; p += (size_t)gridDim.x * blockDim.x) {
    const double2 r = ldc(f, p);
    double2 d = make_double2(1.0, 0.0);
    if (!mask[p]) {
      const double2 sp = ldc(sc, p);
      d = make_double2(dsum - sp.x, -sp.y);
    }
    const double2 q = cdiv(r, d);
    stc(z, p, make_double2(omega * q.x, omega * q.y));
  }
}

// s = ksq (1 + i alpha), stored in the op's precision.
template <typename S>
__global__ void k_build_s(size_t n, const double* __restrict__ ksq, const double* __restrict__ alpha,
                          cplx_t<S>* __restrict__ sc) {
  for (size_t p = blockIdx.x * (size_t)blockDim.x + threadIdx.x; p < n; p += (size_t)gridDim.x * blockDim.x)
    stc(sc, p, make_double2(ksq[p], ksq[p] * alpha[p]));
}


StencilGeom make_geom(int dim, const int n[3], int zb) {
  StencilGeom g;
  g.nx = n[0];
  g.ny = n[1];
  g.nz = dim == 3 ? n[2] : 1;
  g.dim = dim;
  g.dsum = 0.0;
  for (int a = 0; a < 3; ++a) g.ih2[a] = 0.0;
  for (int a = 0; a < dim; ++a) {
    const double h = 1.0 / (n[a] + 1);
    g.ih2[a] = 1.0 / (h * h);
    g.dsum += 2.0 * g.ih2[a];
  }
  // taller tiles (fewer y-halo re-reads) on large grids; 64 x 4 keeps enough
  // workgroups on small ones
  const size_t nn = (size_t)g.nx * g.ny * g.nz;
  g.ty = (g.ny >= 128 && nn >= ((size_t)1 << 22)) ? 8 : 4;
  g.nt = nn >= ((size_t)1 << 23);
  if (zb <= 0) {
    // enough blocks to fill 256 CUs several times over, long z-marches otherwise
    const long nxy = (long)((g.nx + 63) / 64) * ((g.ny + g.ty - 1) / g.ty);
    long target = 2048;
    zb = (int)((nxy * g.nz) / target);
    if (zb < 1) zb = 1;
    if (zb > 16) zb = 16;
  }
  g.zb = dim == 3 ? zb : 1;
  return g;
}

int stencil_nblocks(const StencilGeom& g) { return stencil_blocks(g); }

void build_codes(const StencilGeom& g, const uint8_t* mask, uint8_t* code, hipStream_t st) {
  size_t n = (size_t)g.nx * g.ny * g.nz;
  size_t nb = (n + 255) / 256;
  if (nb > 8192) nb = 8192;
  hipLaunchKernelGGL(k_build_codes, dim3((unsigned)nb), dim3(256), 0, st, g.dim, g.nx, g.ny, g.nz, mask, code);
}

template <typename S, int MODE>
static void launch_mode(const StencilGeom& g, const void* sc, const uint8_t* code, const void* x, const void* f,
                        void* y, double omega, int color, double* part, hipStream_t st) {
  using C = cplx_t<S>;
  dim3 blk(64, g.ty);
  const int nb = stencil_blocks(g);
  const double n = (double)g.nx * g.ny * g.nz, esz = 2.0 * sizeof(S);
  // algorithmic bytes: x, s, the code byte, y (+ f); a red-black colour pass is half a sweep
  const double bytes = MODE == ST_APPLY ? n * (3 * esz + 1) : MODE == ST_RBGS ? n * (4 * esz + 1) / 2 : n * (4 * esz + 1);
  kprof_begin(st);
  if (g.dim == 3)
    hipLaunchKernelGGL((k_stencil<S, 3, MODE>), dim3(nb), blk, 0, st, g, (const C*)sc, code, (const C*)x,
                       (const C*)f, (C*)y, omega, color, part);
  else
    hipLaunchKernelGGL((k_stencil<S, 2, MODE>), dim3(nb), blk, 0, st, g, (const C*)sc, code, (const C*)x,
                       (const C*)f, (C*)y, omega, color, part);
  kprof_end(KP_STENCIL, bytes, st);
}

template <typename S>
void stencil_apply(const StencilGeom& g, const void* sc, const uint8_t* code, const void* x, void* y,
                   hipStream_t st) {
  launch_mode<S, ST_APPLY>(g, sc, code, x, nullptr, y, 0.0, 0, nullptr, st);
}
template <typename S>
void stencil_resid(const StencilGeom& g, const void* sc, const uint8_t* code, const void* f, const void* u,
                   void* r, double* part, hipStream_t st) {
  launch_mode<S, ST_RESID>(g, sc, code, u, f, r, 0.0, 0, part, st);
}
template <typename S>
void stencil_jacobi(const StencilGeom& g, const void* sc, const uint8_t* code, const void* f, const void* u,
                    void* unew, double omega, hipStream_t st) {
  launch_mode<S, ST_JACOBI>(g, sc, code, u, f, unew, omega, 0, nullptr, st);
}
template <typename S>
void stencil_rbgs(const StencilGeom& g, const void* sc, const uint8_t* code, const void* f, void* u, double omega,
                  hipStream_t st) {
  launch_mode<S, ST_RBGS>(g, sc, code, u, f, u, omega, 0, nullptr, st);
  launch_mode<S, ST_RBGS>(g, sc, code, u, f, u, omega, 1, nullptr, st);
}
template <typename S>
void jacobi_from_zero(size_t n, double dsum, const void* sc, const uint8_t* mask, const void* f, void* z,
                      double omega, hipStream_t st) {
  using C = cplx_t<S>;
  int nb = (int)((n + 255) / 256);
  if (nb > 8192) nb = 8192;
  hipLaunchKernelGGL((k_jacobi0<S>), dim3(nb), dim3(256), 0, st, n, dsum, (const C*)sc, mask, (const C*)f, (C*)z,
                     omega);
}
template <typename S>
void build_s(size_t n, const double* ksq, const double* alpha, void* sc, hipStream_t st) {
  int nb = (int)((n + 255) / 256);
  if (nb > 8192) nb = 8192;
  hipLaunchKernelGGL((k_build_s<S>), dim3(nb), dim3(256), 0, st, n, ksq, alpha, (cplx_t<S>*)sc);
}

#define HELM_INST(S)                                                                                        \
  template void stencil_apply<S>(const StencilGeom&, const void*, const uint8_t*, const void*, void*,        \
                                 hipStream_t);                                                              \
  template void stencil_resid<S>(const StencilGeom&, const void*, const uint8_t*, const void*, const void*,  \
                                 void*, double*, hipStream_t);                                              \
  template void stencil_jacobi<S>(const StencilGeom&, const void*, const uint8_t*, const void*, const void*, \
                                  void*, double, hipStream_t);                                              \
  template void stencil_rbgs<S>(const StencilGeom&, const void*, const uint8_t*, const void*, void*, double, \
                                hipStream_t);                                                               \
  template void jacobi_from_zero<S>(size_t, double, const void*, const uint8_t*, const void*, void*, double,  \
                                    hipStream_t);                                                           \
  template void jacobi2_from_zero<S>(const StencilGeom&, const void*, const uint8_t*, const void*, void*,     \
                                     double, hipStream_t);                                                  \
  template void build_s<S>(size_t, const double*, const double*, void*, hipStream_t);
HELM_INST(double)
HELM_INST(float)
#undef HELM_INST

}  // namespace helm
