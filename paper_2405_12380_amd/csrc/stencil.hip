// Stencil kernels of the discrete Helmholtz operator (§2 eq. 1) and of the
// point relaxations of eq. 2 (damped Jacobi, red-black Gauss-Seidel).
//
// Mapping: a workgroup is 64 x 4 threads, lanes along x (a wavefront reads
// one contiguous 1 KiB (complex128) row segment per load), 4 rows in y, and
// each thread marches over `zb` consecutive z-planes keeping the z-1, z, z+1
// values of its column in registers, so every node is loaded from HBM once;
// x/y neighbours are re-read from L1/L2.  Logical blocks are laid out x-, y-,
// then z-fastest and remapped so that each XCD owns one contiguous range of
// them (one z-slab), keeping halo re-reads inside that XCD's L2.
//
// Per-node arithmetic is fixed (independent of the tiling): the axis terms
// ((c - x_minus) + (c - x_plus)) / h_a^2 are accumulated x, y, z in turn and
// s_p c is subtracted last, in fp64 for both storage precisions.
#include "common.h"
#include "internal.h"
#include "prof.h"

namespace helm {

enum { ST_APPLY = 0, ST_JACOBI = 1, ST_RESID = 2, ST_RBGS = 3 };

template <typename S, int DIM, int MODE>
__global__ __launch_bounds__(256) void k_stencil(StencilGeom g, const cplx_t<S>* __restrict__ sc,
                                                 const uint8_t* __restrict__ mask, const cplx_t<S>* x,
                                                 const cplx_t<S>* __restrict__ f, cplx_t<S>* y,
                                                 double omega, int color, double* __restrict__ partials) {
  __shared__ double sh[16];
  const unsigned lb = xcd_remap(blockIdx.x, gridDim.x);
  const unsigned nbx = (g.nx + 63) / 64, nby = (g.ny + 3) / 4;
  const unsigned bx = lb % nbx, by = (lb / nbx) % nby, bz = lb / (nbx * nby);
  const int i = bx * 64 + threadIdx.x;
  const int j = by * 4 + threadIdx.y;
  const int z0 = bz * g.zb;
  const int z1 = min(g.nz, z0 + g.zb);
  const bool active = (i < g.nx) && (j < g.ny);
  const size_t plane = (size_t)g.nx * g.ny;
  double nrm = 0.0;
  if (active && z0 < z1) {
    size_t p = (size_t)i + (size_t)g.nx * ((size_t)j + (size_t)g.ny * z0);
    double2 c = ldc(x, p);
    bool mc = mask[p] != 0;
    double2 zm = czero();
    if (DIM == 3 && z0 > 0) {
      if (!mask[p - plane]) zm = ldc(x, p - plane);
    }
    for (int z = z0; z < z1; ++z, p += plane) {
      double2 znext = czero();
      bool mnext = false;
      if (DIM == 3 && z + 1 < g.nz) {
        znext = ldc(x, p + plane);
        mnext = mask[p + plane] != 0;
      }
      const bool upd = (MODE != ST_RBGS) || (((i + j + z) & 1) == color);
      if (upd) {
        double2 ax;
        if (mc) {
          ax = c;
        } else {
          double2 xm = czero(), xp = czero(), ym = czero(), yp = czero();
          if (i > 0 && !mask[p - 1]) xm = ldc(x, p - 1);
          if (i + 1 < g.nx && !mask[p + 1]) xp = ldc(x, p + 1);
          if (j > 0 && !mask[p - g.nx]) ym = ldc(x, p - g.nx);
          if (j + 1 < g.ny && !mask[p + g.nx]) yp = ldc(x, p + g.nx);
          double2 acc;
          acc.x = ((c.x - xm.x) + (c.x - xp.x)) * g.ih2[0];
          acc.y = ((c.y - xm.y) + (c.y - xp.y)) * g.ih2[0];
          acc.x = acc.x + ((c.x - ym.x) + (c.x - yp.x)) * g.ih2[1];
          acc.y = acc.y + ((c.y - ym.y) + (c.y - yp.y)) * g.ih2[1];
          if (DIM == 3) {
            const double2 zp = mnext ? czero() : znext;
            acc.x = acc.x + ((c.x - zm.x) + (c.x - zp.x)) * g.ih2[2];
            acc.y = acc.y + ((c.y - zm.y) + (c.y - zp.y)) * g.ih2[2];
          }
          ax = csub(acc, cmul(ldc(sc, p), c));
        }
        if (MODE == ST_APPLY) {
          stc(y, p, ax);
        } else if (MODE == ST_RESID) {
          const double2 r = csub(ldc(f, p), ax);
          nrm += r.x * r.x + r.y * r.y;
          stc(y, p, r);
        } else {  // Jacobi / RB-GS update
          const double2 r = csub(ldc(f, p), ax);
          double2 d = make_double2(1.0, 0.0);
          if (!mc) {
            const double2 sp = ldc(sc, p);
            d = make_double2(g.dsum - sp.x, -sp.y);
          }
          const double2 q = cdiv(r, d);
          stc(y, p, make_double2(c.x + omega * q.x, c.y + omega * q.y));
        }
      }
      if (DIM == 3) {
        zm = mc ? czero() : c;
        c = znext;
        mc = mnext;
      }
    }
  }
  if (MODE == ST_RESID) {
    // deterministic per-block partial of ||r||^2
    __shared__ double shr[16];
    const int t = threadIdx.x + 64 * threadIdx.y;
    double v = wave_sum(nrm);
    if ((t & 63) == 0) shr[t >> 6] = v;
    __syncthreads();
    if (t == 0) partials[lb] = (shr[0] + shr[1]) + (shr[2] + shr[3]);
  }
  (void)sh;
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

static int stencil_blocks(const StencilGeom& g) {
  const int nbx = (g.nx + 63) / 64, nby = (g.ny + 3) / 4, nbz = (g.nz + g.zb - 1) / g.zb;
  return nbx * nby * nbz;
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
  if (zb <= 0) {
    // enough blocks to fill 256 CUs several times over, long z-marches otherwise
    const long nxy = (long)((g.nx + 63) / 64) * ((g.ny + 3) / 4);
    long target = 2048;
    zb = (int)((nxy * g.nz) / target);
    if (zb < 1) zb = 1;
    if (zb > 16) zb = 16;
  }
  g.zb = dim == 3 ? zb : 1;
  return g;
}

int stencil_nblocks(const StencilGeom& g) { return stencil_blocks(g); }

template <typename S, int MODE>
static void launch_mode(const StencilGeom& g, const void* sc, const uint8_t* mask, const void* x, const void* f,
                        void* y, double omega, int color, double* part, hipStream_t st) {
  using C = cplx_t<S>;
  dim3 blk(64, 4);
  const int nb = stencil_blocks(g);
  const double n = (double)g.nx * g.ny * g.nz, esz = 2.0 * sizeof(S);
  // algorithmic bytes: x, s, mask, y (+ f); a red-black colour pass is half a sweep
  const double bytes = MODE == ST_APPLY ? n * (3 * esz + 1) : MODE == ST_RBGS ? n * (4 * esz + 1) / 2 : n * (4 * esz + 1);
  kprof_begin(st);
  if (g.dim == 3)
    hipLaunchKernelGGL((k_stencil<S, 3, MODE>), dim3(nb), blk, 0, st, g, (const C*)sc, mask, (const C*)x,
                       (const C*)f, (C*)y, omega, color, part);
  else
    hipLaunchKernelGGL((k_stencil<S, 2, MODE>), dim3(nb), blk, 0, st, g, (const C*)sc, mask, (const C*)x,
                       (const C*)f, (C*)y, omega, color, part);
  kprof_end(KP_STENCIL, bytes, st);
}

template <typename S>
void stencil_apply(const StencilGeom& g, const void* sc, const uint8_t* mask, const void* x, void* y,
                   hipStream_t st) {
  launch_mode<S, ST_APPLY>(g, sc, mask, x, nullptr, y, 0.0, 0, nullptr, st);
}
template <typename S>
void stencil_resid(const StencilGeom& g, const void* sc, const uint8_t* mask, const void* f, const void* u,
                   void* r, double* part, hipStream_t st) {
  launch_mode<S, ST_RESID>(g, sc, mask, u, f, r, 0.0, 0, part, st);
}
template <typename S>
void stencil_jacobi(const StencilGeom& g, const void* sc, const uint8_t* mask, const void* f, const void* u,
                    void* unew, double omega, hipStream_t st) {
  launch_mode<S, ST_JACOBI>(g, sc, mask, u, f, unew, omega, 0, nullptr, st);
}
template <typename S>
void stencil_rbgs(const StencilGeom& g, const void* sc, const uint8_t* mask, const void* f, void* u, double omega,
                  hipStream_t st) {
  launch_mode<S, ST_RBGS>(g, sc, mask, u, f, u, omega, 0, nullptr, st);
  launch_mode<S, ST_RBGS>(g, sc, mask, u, f, u, omega, 1, nullptr, st);
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
  template void build_s<S>(size_t, const double*, const double*, void*, hipStream_t);
HELM_INST(double)
HELM_INST(float)
#undef HELM_INST

}  // namespace helm
