// Device bodies of the stencil kernels (§2 eq. 1, §3.1.1 eq. 2), shared by the
// single-grid kernels and the batched ones: a workgroup of 64 x ty threads
// handles logical tile lb of a geometry (the mapping and the fixed per-node
// arithmetic are described in stencil.hip).
#pragma once

#include "common.h"
#include "internal.h"

namespace helm {

enum { ST_APPLY = 0, ST_JACOBI = 1, ST_RESID = 2, ST_RBGS = 3 };

// Neighbour code of a node (built once per op): bit 0 = the node is masked;
// bits 1..6 = its x-, x+, y-, y+, z-, z+ neighbour is absent (ghost or masked)
// and contributes 0.  One byte replaces seven mask reads per node, and lets
// every neighbour load be issued unconditionally (clamped inside the grid).
enum { NB_SELF = 1, NB_XM = 2, NB_XP = 4, NB_YM = 8, NB_YP = 16, NB_ZM = 32, NB_ZP = 64 };

__device__ __forceinline__ double2 sel0(bool absent, double2 v) { return absent ? czero() : v; }

// Output store: non-temporal (streaming, not kept in L2/MALL) when the grid is
// far larger than the caches, so neighbour rows stay resident.
typedef double dv2 __attribute__((ext_vector_type(2)));
typedef float fv2 __attribute__((ext_vector_type(2)));
__device__ __forceinline__ void stc_out(double2* p, size_t i, double2 v, bool nt) {
  if (nt) __builtin_nontemporal_store(dv2{v.x, v.y}, reinterpret_cast<dv2*>(p + i));
  else p[i] = v;
}
__device__ __forceinline__ void stc_out(float2* p, size_t i, double2 v, bool nt) {
  if (nt) __builtin_nontemporal_store(fv2{(float)v.x, (float)v.y}, reinterpret_cast<fv2*>(p + i));
  else p[i] = make_float2((float)v.x, (float)v.y);
}

// Inputs read once per sweep (s, f and the code byte): on grids far larger than
// the caches these are non-temporal loads, so the caches keep the field whose
// neighbour rows are read again by the adjacent rows of the tile.
__device__ __forceinline__ double2 ldc_once(const double2* p, size_t i, bool nt) {
  if (nt) {
    const dv2 v = __builtin_nontemporal_load(reinterpret_cast<const dv2*>(p + i));
    return make_double2(v.x, v.y);
  }
  return p[i];
}
__device__ __forceinline__ double2 ldc_once(const float2* p, size_t i, bool nt) {
  if (nt) {
    const fv2 v = __builtin_nontemporal_load(reinterpret_cast<const fv2*>(p + i));
    return make_double2((double)v.x, (double)v.y);
  }
  return ldc(p, i);
}
__device__ __forceinline__ unsigned ldcode(const uint8_t* p, size_t i, bool nt) {
  return nt ? (unsigned)__builtin_nontemporal_load(p + i) : (unsigned)p[i];
}

// One workgroup's tile: logical block lb of geometry g (64 x ty threads, each
// owning R consecutive rows, so a tile is 64 x ty R nodes of zb planes).  A
// thread keeps its rows' values of planes z - 1, z and z + 1 in registers; the
// rows inside its block of R are each other's y neighbours, so only the rows
// just below and above it are loaded for y (a 64 x 16 tile at R = 2 re-reads
// 2 of 18 rows instead of 2 of 10).  RESID writes the block's partial of
// ||r||^2 to *partial.
template <typename S, int DIM, int MODE, int R = 1>
__device__ __forceinline__ void stencil_tile(const StencilGeom& g, unsigned lb, const cplx_t<S>* __restrict__ sc,
                                             const uint8_t* __restrict__ code, const cplx_t<S>* x,
                                             const cplx_t<S>* __restrict__ f, cplx_t<S>* y, double omega, int color,
                                             double* __restrict__ partial) {
  const unsigned nbx = (g.nx + 63) / 64, nby = (g.ny + g.ty * R - 1) / (g.ty * R);
  const unsigned bx = lb % nbx, by = (lb / nbx) % nby, bz = lb / (nbx * nby);
  const int i = bx * 64 + threadIdx.x;
  const int j0 = (by * g.ty + threadIdx.y) * R;
  const int z0 = bz * g.zb;
  const int z1 = min(g.nz, z0 + g.zb);
  const bool active = (i < g.nx) && (j0 < g.ny);
  const size_t plane = (size_t)g.nx * g.ny;
  // clamped x offsets (an absent neighbour is read from the node itself and
  // then replaced by 0 through the code bits)
  const ptrdiff_t oxm = i > 0 ? -1 : 0, oxp = i + 1 < g.nx ? 1 : 0;
  double nrm = 0.0;
  if (active && z0 < z1) {
    const size_t pb = (size_t)i + (size_t)g.nx * ((size_t)j0 + (size_t)g.ny * z0);
    double2 c[R], zm[R];
#pragma unroll
    for (int r = 0; r < R; ++r) {
      const bool in = j0 + r < g.ny;
      c[r] = in ? ldc(x, pb + (size_t)r * g.nx) : czero();
      zm[r] = (DIM == 3 && z0 > 0 && in) ? ldc(x, pb + (size_t)r * g.nx - plane) : czero();
    }
    size_t p = pb;
    for (int z = z0; z < z1; ++z, p += plane) {
      double2 zn[R], xm[R], xp[R];
#pragma unroll
      for (int r = 0; r < R; ++r) {
        const bool in = j0 + r < g.ny;
        const size_t q = p + (size_t)r * g.nx;
        zn[r] = (DIM == 3 && z + 1 < g.nz && in) ? ldc(x, q + plane) : czero();
        xm[r] = in ? ldc(x, q + oxm) : czero();
        xp[r] = in ? ldc(x, q + oxp) : czero();
      }
      const double2 ybelow = j0 > 0 ? ldc(x, p - g.nx) : czero();               // row j0 - 1
      const double2 yabove = j0 + R < g.ny ? ldc(x, p + (size_t)R * g.nx) : czero();  // row j0 + R
#pragma unroll
      for (int r = 0; r < R; ++r) {
        if (j0 + r >= g.ny) break;
        const size_t q = p + (size_t)r * g.nx;
        const bool upd = (MODE != ST_RBGS) || (((i + j0 + r + z) & 1) == color);
        if (!upd) continue;
        const unsigned cd = ldcode(code, q, g.nt);
        const double2 ym = r == 0 ? ybelow : c[r - 1], yp = r == R - 1 ? yabove : c[r + 1];
        const double2 sp = ldc_once(sc, q, g.nt);
        double2 fp = czero();
        if (MODE != ST_APPLY) fp = ldc_once(f, q, g.nt);
        const double2 cc = c[r];
        double2 ax;
        if (cd & NB_SELF) {
          ax = cc;
        } else {
          const double2 a = sel0(cd & NB_XM, xm[r]), b = sel0(cd & NB_XP, xp[r]);
          const double2 e = sel0(cd & NB_YM, ym), h = sel0(cd & NB_YP, yp);
          double2 acc;
          acc.x = ((cc.x - a.x) + (cc.x - b.x)) * g.ih2[0];
          acc.y = ((cc.y - a.y) + (cc.y - b.y)) * g.ih2[0];
          acc.x = acc.x + ((cc.x - e.x) + (cc.x - h.x)) * g.ih2[1];
          acc.y = acc.y + ((cc.y - e.y) + (cc.y - h.y)) * g.ih2[1];
          if (DIM == 3) {
            const double2 qq = sel0(cd & NB_ZM, zm[r]), w = sel0(cd & NB_ZP, zn[r]);
            acc.x = acc.x + ((cc.x - qq.x) + (cc.x - w.x)) * g.ih2[2];
            acc.y = acc.y + ((cc.y - qq.y) + (cc.y - w.y)) * g.ih2[2];
          }
          ax = csub(acc, cmul(sp, cc));
        }
        if (MODE == ST_APPLY) {
          stc_out(y, q, ax, g.nt);
        } else if (MODE == ST_RESID) {
          const double2 rr = csub(fp, ax);
          nrm += rr.x * rr.x + rr.y * rr.y;
          stc_out(y, q, rr, g.nt);
        } else {  // Jacobi / RB-GS update (red-black updates in place: plain stores)
          const double2 rr = csub(fp, ax);
          const double2 d = (cd & NB_SELF) ? make_double2(1.0, 0.0) : make_double2(g.dsum - sp.x, -sp.y);
          const double2 qd = ddiv(rr, d);
          stc_out(y, q, make_double2(cc.x + omega * qd.x, cc.y + omega * qd.y), MODE == ST_JACOBI && g.nt);
        }
      }
#pragma unroll
      for (int r = 0; r < R; ++r) {
        zm[r] = c[r];
        c[r] = zn[r];
      }
    }
  }
  if (MODE == ST_RESID) {
    // deterministic per-block partial of ||r||^2 (one value per row-wavefront)
    __shared__ double shr[16];
    const int t = threadIdx.x + 64 * threadIdx.y;
    double v = wave_sum(nrm);
    if ((t & 63) == 0) shr[t >> 6] = v;
    __syncthreads();
    if (t == 0) {
      double a = 0.0;
      for (int w = 0; w < g.ty; ++w) a += shr[w];
      *partial = a;
    }
  }
}

// Two damped Jacobi sweeps on A z = f started from z = 0, in one pass:
// z1 = omega D^{-1} f is formed on the fly at the node and its neighbours (f and
// s re-read from cache), then z2 = z1 + omega D^{-1} (f - A z1).  The per-node
// arithmetic is that of two separate sweeps; the HBM traffic is that of one
// (f, s, code in; z2 out).
__device__ __forceinline__ double2 jac0(double2 f, double2 s, double dsum, bool masked, double omega) {
  const double2 d = masked ? make_double2(1.0, 0.0) : make_double2(dsum - s.x, -s.y);
  const double2 q = ddiv(f, d);
  return make_double2(omega * q.x, omega * q.y);
}

// Right-hand side value at node q, optionally scaled on load by fs (the
// scaled value rounded to the storage precision, exactly what a separate
// scaling pass would have stored).
template <typename S>
__device__ __forceinline__ double2 ldf(const cplx_t<S>* __restrict__ f, size_t q, double fs, bool scaled) {
  double2 v = ldc(f, q);
  if (scaled) {
    v = make_double2(v.x * fs, v.y * fs);
    if (sizeof(S) == sizeof(float)) v = make_double2((double)(float)v.x, (double)(float)v.y);
  }
  return v;
}

// fscale (optional): the right-hand side is fscale[0] * f; fout (optional,
// requires fscale) receives that scaled right-hand side, each node written once
// by the thread that owns it.
template <typename S, int DIM, int R = 1>
__device__ __forceinline__ void jacobi2z_tile(const StencilGeom& g, unsigned lb, const cplx_t<S>* __restrict__ sc,
                                              const uint8_t* __restrict__ code, const cplx_t<S>* __restrict__ f,
                                              cplx_t<S>* __restrict__ y, double omega,
                                              const double* __restrict__ fscale = nullptr,
                                              cplx_t<S>* __restrict__ fout = nullptr) {
  const bool scaled = fscale != nullptr;
  const double fs = scaled ? fscale[0] : 1.0;
  const unsigned nbx = (g.nx + 63) / 64, nby = (g.ny + g.ty * R - 1) / (g.ty * R);
  const unsigned bx = lb % nbx, by = (lb / nbx) % nby, bz = lb / (nbx * nby);
  const int i = bx * 64 + threadIdx.x;
  const int j0 = (by * g.ty + threadIdx.y) * R;
  const int z0 = bz * g.zb;
  const int z1e = min(g.nz, z0 + g.zb);
  if (!(i < g.nx && j0 < g.ny) || z0 >= z1e) return;
  const size_t plane = (size_t)g.nx * g.ny;
  const ptrdiff_t oxm = i > 0 ? -1 : 0, oxp = i + 1 < g.nx ? 1 : 0;
  // each of the thread's R rows is marched on its own (the per-node values are
  // those of a one-row tile)
  double2 zc[R], zmv[R];
#pragma unroll
  for (int r = 0; r < R; ++r) {
    zc[r] = czero();
    zmv[r] = czero();
    const int j = j0 + r;
    if (j >= g.ny) continue;
    const size_t p = (size_t)i + (size_t)g.nx * ((size_t)j + (size_t)g.ny * z0);
    // z1 of the column at z-1, z (the z-1 value only matters when present)
    zc[r] = jac0(ldf<S>(f, p, fs, scaled), ldc(sc, p), g.dsum, code[p] & NB_SELF, omega);
    if (DIM == 3 && z0 > 0) zmv[r] = jac0(ldf<S>(f, p - plane, fs, scaled), ldc(sc, p - plane), g.dsum, false, omega);
  }
  for (int z = z0; z < z1e; ++z) {
#pragma unroll
    for (int r = 0; r < R; ++r) {
      const int j = j0 + r;
      if (j >= g.ny) continue;
      const size_t p = (size_t)i + (size_t)g.nx * ((size_t)j + (size_t)g.ny * z);
      const ptrdiff_t oym = j > 0 ? -(ptrdiff_t)g.nx : 0, oyp = j + 1 < g.ny ? (ptrdiff_t)g.nx : 0;
      double2 znv = czero();
      if (DIM == 3 && z + 1 < g.nz)
        znv = jac0(ldf<S>(f, p + plane, fs, scaled), ldc(sc, p + plane), g.dsum, false, omega);
      const unsigned cd = code[p];
      const double2 fp = ldf<S>(f, p, fs, scaled), sp = ldc(sc, p);
      if (fout) stc(fout, p, fp);
      double2 ax;
      if (cd & NB_SELF) {
        ax = zc[r];
      } else {
        const double2 a = (cd & NB_XM) ? czero() : jac0(ldf<S>(f, p + oxm, fs, scaled), ldc(sc, p + oxm), g.dsum, false, omega);
        const double2 b = (cd & NB_XP) ? czero() : jac0(ldf<S>(f, p + oxp, fs, scaled), ldc(sc, p + oxp), g.dsum, false, omega);
        const double2 e = (cd & NB_YM) ? czero() : jac0(ldf<S>(f, p + oym, fs, scaled), ldc(sc, p + oym), g.dsum, false, omega);
        const double2 h = (cd & NB_YP) ? czero() : jac0(ldf<S>(f, p + oyp, fs, scaled), ldc(sc, p + oyp), g.dsum, false, omega);
        const double2 zz = zc[r];
        double2 acc;
        acc.x = ((zz.x - a.x) + (zz.x - b.x)) * g.ih2[0];
        acc.y = ((zz.y - a.y) + (zz.y - b.y)) * g.ih2[0];
        acc.x = acc.x + ((zz.x - e.x) + (zz.x - h.x)) * g.ih2[1];
        acc.y = acc.y + ((zz.y - e.y) + (zz.y - h.y)) * g.ih2[1];
        if (DIM == 3) {
          const double2 q = (cd & NB_ZM) ? czero() : zmv[r], w = (cd & NB_ZP) ? czero() : znv;
          acc.x = acc.x + ((zz.x - q.x) + (zz.x - w.x)) * g.ih2[2];
          acc.y = acc.y + ((zz.y - q.y) + (zz.y - w.y)) * g.ih2[2];
        }
        ax = csub(acc, cmul(sp, zz));
      }
      const double2 rr = csub(fp, ax);
      const double2 d = (cd & NB_SELF) ? make_double2(1.0, 0.0) : make_double2(g.dsum - sp.x, -sp.y);
      const double2 q = ddiv(rr, d);
      stc(y, p, make_double2(zc[r].x + omega * q.x, zc[r].y + omega * q.y));
      if (DIM == 3) {
        zmv[r] = zc[r];
        zc[r] = znv;
        // the next node's own z1 needs its own mask bit; recompute if it is masked
        if (z + 1 < z1e && (code[p + plane] & NB_SELF))
          zc[r] = jac0(ldf<S>(f, p + plane, fs, scaled), ldc(sc, p + plane), g.dsum, true, omega);
      }
    }
  }
}

}  // namespace helm
