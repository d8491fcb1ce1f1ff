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
  const int rows = g.ty * g.rows;
  const int nbx = (g.nx + 63) / 64, nby = (g.ny + rows - 1) / rows, nbz = (g.nz + g.zb - 1) / g.zb;
  return nbx * nby * nbz;
}

template <typename S, int DIM, int MODE, int R>
__global__ __launch_bounds__(512) void k_stencil(StencilGeom g, const cplx_t<S>* __restrict__ sc,
                                                 const uint8_t* __restrict__ code, const cplx_t<S>* x,
                                                 const cplx_t<S>* __restrict__ f, cplx_t<S>* y,
                                                 double omega, int color, double* __restrict__ partials) {
  const unsigned lb = xcd_remap(blockIdx.x, gridDim.x);
  stencil_tile<S, DIM, MODE, R>(g, lb, sc, code, x, f, y, omega, color, MODE == ST_RESID ? partials + lb : nullptr);
}

template <typename S, int DIM, int R>
__global__ __launch_bounds__(512) void k_jacobi2z(StencilGeom g, const cplx_t<S>* __restrict__ sc,
                                                  const uint8_t* __restrict__ code, const cplx_t<S>* __restrict__ f,
                                                  cplx_t<S>* __restrict__ y, double omega,
                                                  const double* __restrict__ fscale, cplx_t<S>* __restrict__ fout) {
  jacobi2z_tile<S, DIM, R>(g, xcd_remap(blockIdx.x, gridDim.x), sc, code, f, y, omega, fscale, fout);
}

// One red-black Gauss-Seidel sweep in a single pass, out of place (uin -> uout):
// red nodes ((i + j + z) even) get the relaxation update from uin; black nodes
// get it from the red values just computed at their six neighbours.  Every
// thread keeps the new red values of its own column at z - 1, z and z + 1 in
// registers; the in-plane ones are exchanged through LDS, and threads on the
// tile's rim recompute the red value of the neighbouring tile's node (from uin,
// so no other workgroup's output is ever read).  The per-node arithmetic is that
// of the two colour passes of k_stencil<RBGS>, so the result is the same; HBM
// sees one pass (uin, f, s and the code byte read, uout written).
template <typename S>
__device__ __forceinline__ double2 relax_upd(const StencilGeom& g, unsigned cd, double2 c, double2 a, double2 b,
                                             double2 e, double2 h, double2 q, double2 w, double2 sp, double2 fp,
                                             double omega, bool dim3) {
  double2 ax;
  if (cd & NB_SELF) {
    ax = c;
  } else {
    a = sel0(cd & NB_XM, a);
    b = sel0(cd & NB_XP, b);
    e = sel0(cd & NB_YM, e);
    h = sel0(cd & NB_YP, h);
    double2 acc;
    acc.x = ((c.x - a.x) + (c.x - b.x)) * g.ih2[0];
    acc.y = ((c.y - a.y) + (c.y - b.y)) * g.ih2[0];
    acc.x = acc.x + ((c.x - e.x) + (c.x - h.x)) * g.ih2[1];
    acc.y = acc.y + ((c.y - e.y) + (c.y - h.y)) * g.ih2[1];
    if (dim3) {
      q = sel0(cd & NB_ZM, q);
      w = sel0(cd & NB_ZP, w);
      acc.x = acc.x + ((c.x - q.x) + (c.x - w.x)) * g.ih2[2];
      acc.y = acc.y + ((c.y - q.y) + (c.y - w.y)) * g.ih2[2];
    }
    ax = csub(acc, cmul(sp, c));
  }
  const double2 r = csub(fp, ax);
  const double2 d = (cd & NB_SELF) ? make_double2(1.0, 0.0) : make_double2(g.dsum - sp.x, -sp.y);
  const double2 qq = ddiv(r, d);
  return make_double2(c.x + omega * qq.x, c.y + omega * qq.y);
}

// a value rounded to the storage precision (what a pass through memory gives)
template <typename S>
__device__ __forceinline__ double2 rnd_store(double2 v) {
  if (sizeof(S) == sizeof(float)) return make_double2((double)(float)v.x, (double)(float)v.y);
  return v;
}

// the relaxation update at node (i, j, z) from the values of x alone (a red
// node), rounded to the storage precision: the black updates read red values
// as if the two colours were separate passes through memory
template <typename S, int DIM>
__device__ __forceinline__ double2 red_at(const StencilGeom& g, const cplx_t<S>* __restrict__ sc,
                                          const uint8_t* __restrict__ code, const cplx_t<S>* __restrict__ x,
                                          const cplx_t<S>* __restrict__ f, int i, int j, int z, double omega) {
  const size_t plane = (size_t)g.nx * g.ny;
  const size_t p = (size_t)i + (size_t)g.nx * ((size_t)j + (size_t)g.ny * z);
  const unsigned cd = code[p];
  const ptrdiff_t oxm = i > 0 ? -1 : 0, oxp = i + 1 < g.nx ? 1 : 0;
  const ptrdiff_t oym = j > 0 ? -(ptrdiff_t)g.nx : 0, oyp = j + 1 < g.ny ? (ptrdiff_t)g.nx : 0;
  double2 q = czero(), w = czero();
  if (DIM == 3) {
    if (z > 0) q = ldc(x, p - plane);
    if (z + 1 < g.nz) w = ldc(x, p + plane);
  }
  return rnd_store<S>(relax_upd<S>(g, cd, ldc(x, p), ldc(x, p + oxm), ldc(x, p + oxp), ldc(x, p + oym),
                                   ldc(x, p + oyp), q, w, ldc(sc, p), ldc(f, p), omega, DIM == 3));
}

// Thread (tx, ty) owns the node pair x = 2 tx, 2 tx + 1 of row j in a 128 x ty
// tile: in every plane one of the pair is red and the other black, so every
// lane does one red and one black update (no checkerboard divergence).  The
// black node's red neighbours: along x its own red node and the neighbouring
// lane's (a wavefront is one row; the tile's outer neighbours are recomputed by
// lanes 0 and 63), along y the red nodes of the rows above and below (LDS; the
// tile's outer rows recomputed by the first and last row), along z the red
// values of its own column below and above (the one above is also the red node
// of the next plane, computed once).
template <typename S, int DIM>
__global__ __launch_bounds__(512) void k_rbgs_fused(StencilGeom g, const cplx_t<S>* __restrict__ sc,
                                                    const uint8_t* __restrict__ code, const cplx_t<S>* __restrict__ uin,
                                                    const cplx_t<S>* __restrict__ f, cplx_t<S>* __restrict__ uout,
                                                    double omega) {
  __shared__ double2 red[8][128];  // new red values of the current plane (ty <= 8)
  const unsigned lb = xcd_remap(blockIdx.x, gridDim.x);
  const unsigned nbx = (g.nx + 127) / 128, nby = (g.ny + g.ty - 1) / g.ty;
  const unsigned bx = lb % nbx, by = (lb / nbx) % nby, bz = lb / (nbx * nby);
  const int tx = threadIdx.x, tyi = threadIdx.y;
  const int x0 = bx * 128 + 2 * tx;
  const int j = by * g.ty + tyi;
  const int z0 = bz * g.zb;
  const int z1 = min(g.nz, z0 + g.zb);
  const bool rowin = j < g.ny;
  // the pair's red node sits at x0 + ((x0 + j + z) & 1); its black node at the other
  auto xr = [&](int z) { return x0 + ((x0 + j + z) & 1); };
  auto xb = [&](int z) { return x0 + 1 - ((x0 + j + z) & 1); };
  auto in = [&](int x) { return rowin && x < g.nx; };
  // red value of this plane's red node, and of the red node below this plane's black node
  double2 rcur = czero(), rbelow = czero();
  if (z0 < z1) {
    if (in(xr(z0))) rcur = red_at<S, DIM>(g, sc, code, uin, f, xr(z0), j, z0, omega);
    if (DIM == 3 && z0 > 0 && in(xb(z0))) rbelow = red_at<S, DIM>(g, sc, code, uin, f, xb(z0), j, z0 - 1, omega);
  }
  for (int z = z0; z < z1; ++z) {
    const int r_x = xr(z), b_x = xb(z);
    // the black node's own inputs, issued first
    const bool bin = in(b_x);
    const size_t pb = (size_t)b_x + (size_t)g.nx * ((size_t)j + (size_t)g.ny * z);
    unsigned cdb = 0;
    double2 ub = czero(), sb = czero(), fb = czero();
    if (bin) {
      cdb = code[pb];
      ub = ldc(uin, pb);
      sb = ldc(sc, pb);
      fb = ldc(f, pb);
    }
    // red of the column above the black node: next plane's red node of this pair
    double2 rabove = czero();
    if (DIM == 3 && z + 1 < g.nz && in(b_x)) rabove = red_at<S, DIM>(g, sc, code, uin, f, b_x, j, z + 1, omega);
    // x neighbours of the black node: its own pair's red node and the adjacent lane's
    const bool red_left = r_x < b_x;  // red at x0, black at x0 + 1: the right neighbour is lane tx + 1's red
    const double2 nb = make_double2(__shfl(rcur.x, red_left ? (tx + 1) & 63 : (tx + 63) & 63, 64),
                                    __shfl(rcur.y, red_left ? (tx + 1) & 63 : (tx + 63) & 63, 64));
    double2 xo = nb;  // the red node on the far side of the black node
    if (red_left && tx == 63 && in(b_x + 1)) xo = red_at<S, DIM>(g, sc, code, uin, f, b_x + 1, j, z, omega);
    if (!red_left && tx == 0 && b_x > 0 && rowin) xo = red_at<S, DIM>(g, sc, code, uin, f, b_x - 1, j, z, omega);
    // y neighbours (same x as the black node) through LDS; the tile's outer rows recomputed
    red[tyi][r_x - bx * 128] = rcur;
    double2 ym = czero(), yp = czero();
    if (tyi == 0 && j > 0 && in(b_x)) ym = red_at<S, DIM>(g, sc, code, uin, f, b_x, j - 1, z, omega);
    if (tyi == g.ty - 1 && j + 1 < g.ny && in(b_x)) yp = red_at<S, DIM>(g, sc, code, uin, f, b_x, j + 1, z, omega);
    __syncthreads();
    if (tyi > 0) ym = red[tyi - 1][b_x - bx * 128];
    if (tyi < g.ty - 1) yp = red[tyi + 1][b_x - bx * 128];
    if (in(r_x)) {
      const size_t pr = (size_t)r_x + (size_t)g.nx * ((size_t)j + (size_t)g.ny * z);
      stc_out(uout, pr, rcur, g.nt);
    }
    if (bin) {
      const double2 a = red_left ? rcur : xo;   // x - 1
      const double2 b = red_left ? xo : rcur;   // x + 1
      const double2 out = relax_upd<S>(g, cdb, ub, a, b, ym, yp, rbelow, rabove, sb, fb, omega, DIM == 3);
      stc_out(uout, pb, out, g.nt);
    }
    __syncthreads();
    // next plane: this plane's red node is below the next black node (same x), and
    // the red node above this black node is the next plane's red node
    rbelow = rcur;
    rcur = rabove;
  }
}

// ---- red-black sweep through an LDS ring of planes (3D) -------------------------
// A workgroup owns a 64 x 8 column tile and marches over zb planes.  Each plane
// of uin is staged once in LDS with a two-node rim (68 x 12 values); a ring of
// six staged planes is kept.  In step z the red half-sweep of plane z + 1 runs
// on the tile and a one-node rim (the rim's red values are the neighbouring
// tile's, recomputed here from uin, so no other workgroup's output is read) and
// overwrites the red positions of the staged plane; then the black half-sweep
// of plane z reads its six red neighbours (planes z - 1, z, z + 1) and its own
// old value from LDS.  Black positions in LDS always keep their uin values, which
// is what the red updates read.  Plane z + 4 is loaded into registers one step
// ahead and the node data (code byte, s, f) of the next step's updates as well;
// one barrier per step.  Stores go through the caches: a colour's stores fill
// every other 16-byte slot of a line, and the other colour's stores of the same
// line follow a step later, so they merge in L2 (non-temporal stores of these
// half lines cost 8% at 256^3 and 13% at 384^3).  Every global access is a buffer load or store whose
// offset is pushed past the end of the buffer where the node is absent (loads
// give 0, stores are dropped), so a step issues the same memory operations on
// every path and waiting for the prefetched data never waits for the step's
// stores.  Red values are rounded to the storage precision before the black
// updates read them, as if the two colours were separate passes through
// memory; the per-node arithmetic is relax_upd's.  Buffers must be under 2 GiB.
constexpr int RB_TX = 64, RB_TY = 8, RB_LX = RB_TX + 4, RB_LY = RB_TY + 4, RB_PL = RB_LX * RB_LY, RB_NS = 6;
constexpr int RB_RROW = (RB_TX + 2) / 2, RB_NRED = RB_RROW * (RB_TY + 2);  // red nodes of the tile and its rim (330)
constexpr unsigned RB_OOB = 0x80000000u;  // byte offset past the end of every buffer the kernel is given
// 384 threads: one red update per thread and step (330 on the tile and its
// rim), one black update on the first 256 (the tile's 256 black nodes), the
// staged plane three positions per thread
constexpr int RB_NT = 384, RB_NB = RB_TX * RB_TY / 2;
constexpr int RB_QP = (RB_PL + RB_NT - 1) / RB_NT, RB_RU = (RB_NRED + RB_NT - 1) / RB_NT;
static_assert(RB_NB <= RB_NT && RB_RU == 1, "ring tile sizes");

typedef unsigned int rb_u4 __attribute__((ext_vector_type(4)));
typedef unsigned int rb_u2 __attribute__((ext_vector_type(2)));

__device__ __forceinline__ __amdgpu_buffer_rsrc_t rb_rsrc(const void* p, size_t bytes) {
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(p), 0, (int)bytes, 0x00020000);
}
__device__ __forceinline__ double2 rb_ld(__amdgpu_buffer_rsrc_t r, unsigned off, const double2*) {
  return __builtin_bit_cast(double2, __builtin_amdgcn_raw_buffer_load_b128(r, off, 0, 0));
}
__device__ __forceinline__ double2 rb_ld(__amdgpu_buffer_rsrc_t r, unsigned off, const float2*) {
  const float2 v = __builtin_bit_cast(float2, __builtin_amdgcn_raw_buffer_load_b64(r, off, 0, 0));
  return make_double2((double)v.x, (double)v.y);
}
__device__ __forceinline__ void rb_st(__amdgpu_buffer_rsrc_t r, unsigned off, double2 v, double2*) {
  __builtin_amdgcn_raw_buffer_store_b128(__builtin_bit_cast(rb_u4, v), r, off, 0, 0);
}
__device__ __forceinline__ void rb_st(__amdgpu_buffer_rsrc_t r, unsigned off, double2 v, float2*) {
  __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(rb_u2, make_float2((float)v.x, (float)v.y)), r, off, 0, 0);
}

// A node's data for one relaxation update: the aligned 32-bit word that holds
// its code byte (a word, not the byte, so that a value carried into the next
// loop iteration needs no conversion, which would make the step wait for its
// own prefetches), s and f.  Code buffers are padded to a multiple of 4 bytes.
struct NodeIn {
  unsigned cw;
  double2 s, f;
};
__device__ __forceinline__ unsigned rb_cw_off(unsigned boff) { return boff & ~3u; }
__device__ __forceinline__ unsigned rb_cd(unsigned cw, unsigned boff) { return (cw >> (8 * (boff & 3u))) & 0xffu; }

template <typename S, int DEPTH>
__global__ __launch_bounds__(RB_NT) void k_rbgs_ring(StencilGeom g, int zb, const cplx_t<S>* __restrict__ sc,
                                                   const uint8_t* __restrict__ code,
                                                   const cplx_t<S>* __restrict__ uin, const cplx_t<S>* __restrict__ f,
                                                   cplx_t<S>* __restrict__ uout, double omega) {
  using C = cplx_t<S>;
  __shared__ double2 ring[RB_NS][RB_PL];
  const unsigned lb = xcd_remap(blockIdx.x, gridDim.x);
  const unsigned nbx = (g.nx + RB_TX - 1) / RB_TX, nby = (g.ny + RB_TY - 1) / RB_TY;
  const int bx = lb % nbx, by = (lb / nbx) % nby, bz = lb / (nbx * nby);
  const int gx0 = bx * RB_TX - 2, gy0 = by * RB_TY - 2;  // global (x, y) of LDS position (0, 0)
  const int z0 = bz * zb, z1 = min(g.nz, z0 + zb);
  const int t = threadIdx.x;
  const size_t nxy = (size_t)g.nx * g.ny, nn = nxy * g.nz;
  const __amdgpu_buffer_rsrc_t r_u = rb_rsrc(uin, nn * sizeof(C)), r_f = rb_rsrc(f, nn * sizeof(C)),
                               r_s = rb_rsrc(sc, nn * sizeof(C)), r_c = rb_rsrc(code, (nn + 3) & ~(size_t)3),
                               r_o = rb_rsrc(uout, nn * sizeof(C));
  auto slot = [](int k) { return (k + RB_NS) % RB_NS; };  // k >= -RB_NS
  // node index of LDS position e in plane k, or -1 where there is no node
  auto node = [&](int e, int k) -> long {
    const int gx = gx0 + e % RB_LX, gy = gy0 + e / RB_LX;
    return (k >= 0 && k < g.nz && gx >= 0 && gx < g.nx && gy >= 0 && gy < g.ny)
               ? (long)((size_t)gx + (size_t)g.nx * gy + nxy * k)
               : -1L;
  };
  auto boff = [](long p, unsigned esz) { return p >= 0 ? (unsigned)p * esz : RB_OOB; };
  // staged plane k: thread t holds LDS positions t + RB_NT q (zero where there is no node)
  auto load_plane = [&](int k, double2 (&pre)[RB_QP]) {
#pragma unroll
    for (int q = 0; q < RB_QP; ++q) {
      const int e = t + RB_NT * q;
      pre[q] = rb_ld(r_u, boff(e < RB_PL ? node(e, k) : -1L, sizeof(C)), (const C*)nullptr);
    }
  };
  auto store_plane = [&](int k, const double2 (&pre)[RB_QP]) {
    double2* P = ring[slot(k)];
#pragma unroll
    for (int q = 0; q < RB_QP; ++q)
      if (t + RB_NT * q < RB_PL) P[t + RB_NT * q] = pre[q];
  };
  // red node r (< RB_NRED) of plane k: LDS position on the tile or its one-node rim
  auto red_pos = [&](int r, int k) {
    const int ly = 1 + r / RB_RROW, c = r % RB_RROW;
    const int lx = 1 + ((gx0 + 1 + gy0 + ly + k) & 1) + 2 * c;
    return ly * RB_LX + lx;
  };
  // black node of plane k owned by thread t < RB_NB (32 per row, 8 rows); the
  // other threads address a valid position and store nothing
  const bool bact = t < RB_NB;
  const int tb = bact ? t : t - RB_NB;
  auto black_pos = [&](int k) {
    const int ly = 2 + tb / (RB_TX / 2), c = tb % (RB_TX / 2);
    const int lx = 3 - ((gx0 + gy0 + ly + k) & 1) + 2 * c;
    return ly * RB_LX + lx;
  };
  auto load_node = [&](long p, NodeIn& in) {
    in.cw = __builtin_amdgcn_raw_buffer_load_b32(r_c, rb_cw_off(boff(p, 1)), 0, 0);
    in.s = rb_ld(r_s, boff(p, sizeof(C)), (const C*)nullptr);
    in.f = rb_ld(r_f, boff(p, sizeof(C)), (const C*)nullptr);
  };
  // this thread's u-th red node of plane k: LDS position, node index (-1: none)
  auto red_node = [&](int u, int k, int& e) -> long {
    const int r = t + RB_NT * u;
    e = red_pos(r < RB_NRED ? r : RB_NRED - 1, k);
    return r < RB_NRED ? node(e, k) : -1L;
  };
  // node data of a step's red updates (plane kr) and black update (plane kb)
  auto load_next = [&](int kr, int kb, NodeIn (&rn)[RB_RU], NodeIn& bn) {
#pragma unroll
    for (int u = 0; u < RB_RU; ++u) {
      int e;
      load_node(red_node(u, kr, e), rn[u]);
    }
    load_node(bact ? node(black_pos(kb), kb) : -1L, bn);
  };
  // red half-sweep of plane k; the tile's values go to uout when `own`
  auto red = [&](int k, const NodeIn* in, bool own) {
    double2* P = ring[slot(k)];
    const double2* Pm = ring[slot(k - 1)];
    const double2* Pp = ring[slot(k + 1)];
#pragma unroll
    for (int u = 0; u < RB_RU; ++u) {
      int e;
      const long p = red_node(u, k, e);
      const double2 v = rnd_store<S>(relax_upd<S>(g, rb_cd(in[u].cw, boff(p, 1)), P[e], P[e - 1], P[e + 1], P[e - RB_LX], P[e + RB_LX],
                                                  Pm[e], Pp[e], in[u].s, in[u].f, omega, true));
      if (p >= 0) P[e] = v;
      const int lx = e % RB_LX, ly = e / RB_LX;
      const bool tile = lx >= 2 && lx < RB_TX + 2 && ly >= 2 && ly < RB_TY + 2;
      rb_st(r_o, boff(own && tile ? p : -1L, sizeof(C)), v, (C*)nullptr);
    }
  };
  // prologue: planes z0 - 2 .. z0 + 2 staged, plane z0 + 3 in flight, red of z0 - 1 and z0
  // Prefetch depth DEPTH: step z reads the register set loaded DEPTH - 1 steps
  // earlier (plane z + 3, node data of its updates) and loads the set of step
  // z + DEPTH - 1 into the set step z - 1 used.  The loop is unrolled by DEPTH so
  // that every set keeps its registers (a set carried into differently named
  // registers at the loop's back-edge would make each step wait for its own
  // loads).  The kernel runs with DEPTH = 2; depths 3 and 4 measured no faster.
  struct Pre {
    double2 pl[RB_QP];
    NodeIn rn[RB_RU], bn;
  };
  Pre S_[DEPTH];
  NodeIn r0[RB_RU], r1[RB_RU];
  for (int k = z0 - 2; k <= z0 + 2; ++k) {
    load_plane(k, S_[0].pl);
    store_plane(k, S_[0].pl);
  }
#pragma unroll
  for (int u = 0; u < RB_RU; ++u) {
    int e;
    load_node(red_node(u, z0 - 1, e), r0[u]);
    load_node(red_node(u, z0, e), r1[u]);
  }
#pragma unroll
  for (int j = 0; j < DEPTH - 1; ++j) {
    load_plane(z0 + 3 + j, S_[j].pl);
    load_next(z0 + 1 + j, z0 + j, S_[j].rn, S_[j].bn);
  }
  __syncthreads();
  red(z0 - 1, r0, false);
  red(z0, r1, true);
  auto step = [&](int z, const Pre& cur, Pre& nxt) {
    store_plane(z + 3, cur.pl);  // its slot last held plane z - 3
    load_plane(z + DEPTH + 2, nxt.pl);
    load_next(z + DEPTH, z + DEPTH - 1, nxt.rn, nxt.bn);
    red(z + 1, cur.rn, z + 1 < z1);
    __syncthreads();
    // black half-sweep of plane z on the tile (wavefronts of the first 256 threads)
    if (bact) {
      const int e = black_pos(z);
      const double2* P = ring[slot(z)];
      const double2 v = relax_upd<S>(g, rb_cd(cur.bn.cw, boff(node(e, z), 1)), P[e], P[e - 1], P[e + 1],
                                     P[e - RB_LX], P[e + RB_LX], ring[slot(z - 1)][e], ring[slot(z + 1)][e],
                                     cur.bn.s, cur.bn.f, omega, true);
      rb_st(r_o, boff(z < z1 ? node(e, z) : -1L, sizeof(C)), v, (C*)nullptr);
    }
  };
  // the march is rounded up to a multiple of DEPTH steps: the steps past z1
  // store nothing (no branches around them, so the register sets stay put)
  for (int z = z0; z < z1; z += DEPTH) {
#pragma unroll
    for (int i = 0; i < DEPTH; ++i) step(z + i, S_[i], S_[(i + DEPTH - 1) % DEPTH]);
  }
}

template <typename S>
void jacobi2_from_zero(const StencilGeom& g, const void* sc, const uint8_t* code, const void* f, void* z, double omega,
                       hipStream_t st, const double* fscale, void* fout) {
  using C = cplx_t<S>;
  const int nb = stencil_blocks(g);
  const double n = (double)g.nx * g.ny * g.nz, esz = 2.0 * sizeof(S);
  kprof_begin(KP_STENCIL, st);
  if (g.dim == 3 && g.rows == 2)
    hipLaunchKernelGGL((k_jacobi2z<S, 3, 2>), dim3(nb), dim3(64, g.ty), 0, st, g, (const C*)sc, code, (const C*)f,
                       (C*)z, omega, fscale, (C*)fout);
  else if (g.dim == 3)
    hipLaunchKernelGGL((k_jacobi2z<S, 3, 1>), dim3(nb), dim3(64, g.ty), 0, st, g, (const C*)sc, code, (const C*)f,
                       (C*)z, omega, fscale, (C*)fout);
  else
    hipLaunchKernelGGL((k_jacobi2z<S, 2, 1>), dim3(nb), dim3(64, g.ty), 0, st, g, (const C*)sc, code, (const C*)f,
                       (C*)z, omega, fscale, (C*)fout);
  kprof_end(KP_STENCIL, n * ((fout ? 4 : 3) * esz + 1), st);
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
    const double2 q = ddiv(r, d);
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
  g.rb = 0;
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
  // two rows per thread on large 3D grids (64 x 16 tiles: fewer re-read halo
  // rows; 5.8 against 4.9 TB/s for y = A x at 256^3); small grids keep one row
  // per thread for the block count
  g.rows = (dim == 3 && g.ty == 8) ? 2 : 1;
  g.nt = nn >= ((size_t)1 << 23);
  if (zb <= 0) {
    // enough blocks to fill 256 CUs several times over, long z-marches otherwise
    const long nxy = (long)((g.nx + 63) / 64) * ((g.ny + g.ty * g.rows - 1) / (g.ty * g.rows));
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
  kprof_begin(KP_STENCIL, st);
  if (g.dim == 3 && g.rows == 2)
    hipLaunchKernelGGL((k_stencil<S, 3, MODE, 2>), dim3(nb), blk, 0, st, g, (const C*)sc, code, (const C*)x,
                       (const C*)f, (C*)y, omega, color, part);
  else if (g.dim == 3)
    hipLaunchKernelGGL((k_stencil<S, 3, MODE, 1>), dim3(nb), blk, 0, st, g, (const C*)sc, code, (const C*)x,
                       (const C*)f, (C*)y, omega, color, part);
  else
    hipLaunchKernelGGL((k_stencil<S, 2, MODE, 1>), dim3(nb), blk, 0, st, g, (const C*)sc, code, (const C*)x,
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
void stencil_rbgs_fused(const StencilGeom& g0, const void* sc, const uint8_t* code, const void* f, const void* uin,
                        void* uout, double omega, hipStream_t st) {
  using C = cplx_t<S>;
  // 128 x 8 tiles: the recomputed rim rows are a quarter of the tile's rows
  StencilGeom g = g0;
  g.ty = g.ny >= 8 ? 8 : g0.ty;
  const int nb = ((g.nx + 127) / 128) * ((g.ny + g.ty - 1) / g.ty) * ((g.nz + g.zb - 1) / g.zb);
  const double n = (double)g.nx * g.ny * g.nz, esz = 2.0 * sizeof(S);
  kprof_begin(KP_STENCIL, st);
  // the ring kernel addresses each buffer with 32-bit offsets (fields under 2 GiB)
  const bool small = n * esz < 2147483648.0;
  const bool ring = g.dim == 3 && (g.rb == 1 || (g.rb == 0 && small));
  if (ring) {
    // planes per workgroup: about 1024 workgroups, marches of 2 .. 64 planes
    // (at 256^3 the 32-plane marches measured best, 304 against 314-362 us for
    // 48-96 planes; at 384^3 64 planes, 989 against 1035 us for 32)
    const long tiles = (long)((g.nx + RB_TX - 1) / RB_TX) * ((g.ny + RB_TY - 1) / RB_TY);
    int zb = (int)(tiles * g.nz / 1024);
    zb = zb < 2 ? 2 : zb > 64 ? 64 : zb;
    const long nbr = tiles * ((g.nz + zb - 1) / zb);
    hipLaunchKernelGGL((k_rbgs_ring<S, 2>), dim3((unsigned)nbr), dim3(RB_NT), 0, st, g, zb, (const C*)sc, code,
                       (const C*)uin, (const C*)f, (C*)uout, omega);
  } else if (g.dim == 3)
    hipLaunchKernelGGL((k_rbgs_fused<S, 3>), dim3(nb), dim3(64, g.ty), 0, st, g, (const C*)sc, code, (const C*)uin,
                       (const C*)f, (C*)uout, omega);
  else
    hipLaunchKernelGGL((k_rbgs_fused<S, 2>), dim3(nb), dim3(64, g.ty), 0, st, g, (const C*)sc, code, (const C*)uin,
                       (const C*)f, (C*)uout, omega);
  kprof_end(KP_STENCIL, n * (4 * esz + 1), st);
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
  template void stencil_rbgs_fused<S>(const StencilGeom&, const void*, const uint8_t*, const void*, const void*, \
                                      void*, double, hipStream_t);                                          \
  template void jacobi_from_zero<S>(size_t, double, const void*, const uint8_t*, const void*, void*, double,  \
                                    hipStream_t);                                                           \
  template void jacobi2_from_zero<S>(const StencilGeom&, const void*, const uint8_t*, const void*, void*,     \
                                     double, hipStream_t, const double*, void*);                            \
  template void build_s<S>(size_t, const double*, const double*, void*, hipStream_t);
HELM_INST(double)
HELM_INST(float)
#undef HELM_INST

}  // namespace helm
