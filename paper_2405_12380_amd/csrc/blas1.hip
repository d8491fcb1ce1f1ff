// Krylov vector kernels: deterministic two-stage reductions (complex inner
// products <x, y> = sum conj(x_i) y_i, norms, the GMRES multi-dot V^H w) and
// the vector updates of GMRES/BiCGStab, all accumulating in fp64.
//
// Reductions run on a fixed grid whose size depends only on n, every block
// writes its partial to a fixed slot, and the second stage sums the partials
// in index order: results are bitwise reproducible run to run.
#include "common.h"
#include "internal.h"
#include "prof.h"
#include "stencil_dev.h"

namespace helm {

static constexpr int RED_MAXB = 1024;

int red_nblocks(size_t n) {
  size_t nb = (n + 255) / 256;
  if (nb > RED_MAXB) nb = RED_MAXB;
  if (nb < 1) nb = 1;
  return (int)nb;
}

__global__ __launch_bounds__(256) void k_reduce_cols(const double* __restrict__ part, int nparts, int width,
                                                     double* __restrict__ out) {
  __shared__ double sh[16];
  const int w = blockIdx.x;
  double acc = 0.0;
  // four loads per thread in flight at once, added in index order
  for (int b0 = 0; b0 < nparts; b0 += 4 * 256) {
    double v[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int b = b0 + threadIdx.x + 256 * q;
      v[q] = b < nparts ? part[(size_t)b * width + w] : 0.0;
    }
#pragma unroll
    for (int q = 0; q < 4; ++q) acc += v[q];
  }
  acc = block_sum(acc, sh);
  if (threadIdx.x == 0) out[w] = acc;
}

void reduce_cols(const double* part, int nparts, int width, double* out, hipStream_t st) {
  hipLaunchKernelGGL(k_reduce_cols, dim3(width), dim3(256), 0, st, part, nparts, width, out);
}

template <typename S>
__global__ __launch_bounds__(256) void k_dot_part(size_t n, const cplx_t<S>* __restrict__ x,
                                                  const cplx_t<S>* __restrict__ y, double* __restrict__ part) {
  __shared__ double sh[32];
  double2 acc = czero();
  for (size_t e = blockIdx.x * (size_t)blockDim.x + threadIdx.x; e < n; e += (size_t)gridDim.x * blockDim.x)
    acc = cadd(acc, cconjmul(ldc(x, e), ldc(y, e)));
  acc = block_sum2(acc, sh);
  if (threadIdx.x == 0) {
    part[2 * blockIdx.x] = acc.x;
    part[2 * blockIdx.x + 1] = acc.y;
  }
}

template <typename S>
__global__ __launch_bounds__(256) void k_nrm2_part(size_t n, const cplx_t<S>* __restrict__ x,
                                                   double* __restrict__ part) {
  __shared__ double sh[16];
  double acc = 0.0;
  for (size_t e = blockIdx.x * (size_t)blockDim.x + threadIdx.x; e < n; e += (size_t)gridDim.x * blockDim.x) {
    const double2 v = ldc(x, e);
    acc += v.x * v.x + v.y * v.y;
  }
  acc = block_sum(acc, sh);
  if (threadIdx.x == 0) part[blockIdx.x] = acc;
}

template <typename S>
void dot_part(size_t n, const void* x, const void* y, double* part, hipStream_t st) {
  using C = cplx_t<S>;
  hipLaunchKernelGGL((k_dot_part<S>), dim3(red_nblocks(n)), dim3(256), 0, st, n, (const C*)x, (const C*)y, part);
}
template <typename S>
void nrm2_part(size_t n, const void* x, double* part, hipStream_t st) {
  using C = cplx_t<S>;
  hipLaunchKernelGGL((k_nrm2_part<S>), dim3(red_nblocks(n)), dim3(256), 0, st, n, (const C*)x, part);
}

// ---- multi-dot --------------------------------------------------------------
// Workgroup b owns elements [b C, (b+1) C): w's chunk is staged once in LDS,
// then each wavefront takes every fourth basis vector and streams its chunk
// (C/64 independent coalesced loads per lane), reducing once per vector with
// shuffles.  part[b][2 i + {0,1}] = sum over the chunk of conj(V_i) w.
static int md_chunk(size_t n) { return n <= ((size_t)1 << 21) ? 512 : 2048; }
int multidot_nblocks(size_t n) {
  const size_t c = (size_t)md_chunk(n);
  return (int)((n + c - 1) / c);
}

template <typename S, int CH>
__global__ __launch_bounds__(256) void k_multidot(size_t n, const cplx_t<S>* __restrict__ V, size_t ldv, int nv,
                                                  const cplx_t<S>* __restrict__ w, double* __restrict__ part) {
  __shared__ double2 ws[CH];
  const size_t c0 = (size_t)blockIdx.x * CH;
  for (int t = threadIdx.x; t < CH; t += 256) {
    const size_t e = c0 + t;
    ws[t] = e < n ? ldc(w, e) : czero();
  }
  __syncthreads();
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const bool full = c0 + CH <= n;
  for (int i = wave; i < nv; i += 4) {
    const cplx_t<S>* Vi = V + (size_t)i * ldv + c0;
    double2 acc = czero();
    if (full) {
#pragma unroll
      for (int t = 0; t < CH / 64; ++t) acc = cadd(acc, cconjmul(ldc(Vi, lane + 64 * t), ws[lane + 64 * t]));
    } else {
      for (int t = 0; t < CH / 64; ++t) {
        const int el = lane + 64 * t;
        if (c0 + el < n) acc = cadd(acc, cconjmul(ldc(Vi, el), ws[el]));
      }
    }
    acc.x = wave_sum(acc.x);
    acc.y = wave_sum(acc.y);
    if (lane == 0) {
      part[(size_t)blockIdx.x * 2 * nv + 2 * i] = acc.x;
      part[(size_t)blockIdx.x * 2 * nv + 2 * i + 1] = acc.y;
    }
  }
}

template <typename S>
void multidot_part(size_t n, const void* V, size_t ldv, int nv, const void* w, double* part, hipStream_t st) {
  using C = cplx_t<S>;
  const int nb = multidot_nblocks(n);
  kprof_begin(KP_MULTIDOT, st);
  if (md_chunk(n) == 512)
    hipLaunchKernelGGL((k_multidot<S, 512>), dim3(nb), dim3(256), 0, st, n, (const C*)V, ldv, nv, (const C*)w, part);
  else
    hipLaunchKernelGGL((k_multidot<S, 2048>), dim3(nb), dim3(256), 0, st, n, (const C*)V, ldv, nv, (const C*)w, part);
  kprof_end(KP_MULTIDOT, (double)n * 2 * sizeof(S) * (nv + 1), st);
}

// ---- matvec fused with the multi-dot -----------------------------------------
// w = A z for the workgroup's chunk (the per-node arithmetic of the apply
// stencil, neighbours through the node's code byte), stored and staged in LDS,
// then the same partials of V^H w as k_multidot: one launch and one pass over
// w fewer per Arnoldi step.
template <typename S, int CH>
__global__ __launch_bounds__(256) void k_multidot_apply(StencilGeom g, const cplx_t<S>* __restrict__ sc,
                                                        const uint8_t* __restrict__ code, const cplx_t<S>* __restrict__ z,
                                                        const cplx_t<S>* __restrict__ V, size_t ldv, int nv,
                                                        cplx_t<S>* __restrict__ w, double* __restrict__ part) {
  __shared__ double2 ws[CH];
  const size_t n = (size_t)g.nx * g.ny * g.nz;
  const ptrdiff_t sy = g.nx, sz = (ptrdiff_t)g.nx * g.ny;
  const size_t c0 = (size_t)blockIdx.x * CH;
  for (int t = threadIdx.x; t < CH; t += 256) {
    const size_t e = c0 + t;
    double2 ax = czero();
    if (e < n) {
      const unsigned cd = code[e];
      const double2 c = ldc(z, e);
      if (cd & NB_SELF) {
        ax = c;
      } else {
        const double2 a = sel0(cd & NB_XM, ldc(z, e - ((cd & NB_XM) ? 0 : 1)));
        const double2 b = sel0(cd & NB_XP, ldc(z, e + ((cd & NB_XP) ? 0 : 1)));
        const double2 ee = sel0(cd & NB_YM, ldc(z, e - ((cd & NB_YM) ? 0 : sy)));
        const double2 h = sel0(cd & NB_YP, ldc(z, e + ((cd & NB_YP) ? 0 : sy)));
        const double2 sp = ldc(sc, e);
        double2 acc;
        acc.x = ((c.x - a.x) + (c.x - b.x)) * g.ih2[0];
        acc.y = ((c.y - a.y) + (c.y - b.y)) * g.ih2[0];
        acc.x = acc.x + ((c.x - ee.x) + (c.x - h.x)) * g.ih2[1];
        acc.y = acc.y + ((c.y - ee.y) + (c.y - h.y)) * g.ih2[1];
        if (g.dim == 3) {
          const double2 q = sel0(cd & NB_ZM, ldc(z, e - ((cd & NB_ZM) ? 0 : sz)));
          const double2 u = sel0(cd & NB_ZP, ldc(z, e + ((cd & NB_ZP) ? 0 : sz)));
          acc.x = acc.x + ((c.x - q.x) + (c.x - u.x)) * g.ih2[2];
          acc.y = acc.y + ((c.y - q.y) + (c.y - u.y)) * g.ih2[2];
        }
        ax = csub(acc, cmul(sp, c));
      }
      stc(w, e, ax);
      if (sizeof(S) == sizeof(float)) ax = make_double2((double)(float)ax.x, (double)(float)ax.y);
    }
    ws[t] = ax;
  }
  __syncthreads();
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const bool full = c0 + CH <= n;
  for (int i = wave; i < nv; i += 4) {
    const cplx_t<S>* Vi = V + (size_t)i * ldv + c0;
    double2 acc = czero();
    if (full) {
#pragma unroll
      for (int t = 0; t < CH / 64; ++t) acc = cadd(acc, cconjmul(ldc(Vi, lane + 64 * t), ws[lane + 64 * t]));
    } else {
      for (int t = 0; t < CH / 64; ++t) {
        const int el = lane + 64 * t;
        if (c0 + el < n) acc = cadd(acc, cconjmul(ldc(Vi, el), ws[el]));
      }
    }
    acc.x = wave_sum(acc.x);
    acc.y = wave_sum(acc.y);
    if (lane == 0) {
      part[(size_t)blockIdx.x * 2 * nv + 2 * i] = acc.x;
      part[(size_t)blockIdx.x * 2 * nv + 2 * i + 1] = acc.y;
    }
  }
}

template <typename S>
void multidot_apply(const StencilGeom& g, const void* sc, const uint8_t* code, const void* z, const void* V,
                    size_t ldv, int nv, void* w, double* part, hipStream_t st) {
  using C = cplx_t<S>;
  const size_t n = (size_t)g.nx * g.ny * g.nz;
  const int nb = multidot_nblocks(n);
  kprof_begin(KP_MULTIDOT, st);
  if (md_chunk(n) == 512)
    hipLaunchKernelGGL((k_multidot_apply<S, 512>), dim3(nb), dim3(256), 0, st, g, (const C*)sc, code, (const C*)z,
                       (const C*)V, ldv, nv, (C*)w, part);
  else
    hipLaunchKernelGGL((k_multidot_apply<S, 2048>), dim3(nb), dim3(256), 0, st, g, (const C*)sc, code, (const C*)z,
                       (const C*)V, ldv, nv, (C*)w, part);
  // V once; z, s and the code byte once (z's neighbours from cache); w written
  kprof_end(KP_MULTIDOT, (double)n * (2 * sizeof(S) * (nv + 3) + 1), st);
}

// ---- multi-axpy -------------------------------------------------------------
template <typename S, bool NORM>
__global__ __launch_bounds__(256) void k_multi_axpy(size_t n, const cplx_t<S>* __restrict__ V, size_t ldv, int nv,
                                                    const double* __restrict__ coef, double sgn,
                                                    const cplx_t<S>* base, cplx_t<S>* out,
                                                    double* __restrict__ part) {
  __shared__ double sh[16];
  double nrm = 0.0;
  for (size_t e = blockIdx.x * (size_t)blockDim.x + threadIdx.x; e < n; e += (size_t)gridDim.x * blockDim.x) {
    double2 acc = czero();
    int i = 0;
    for (; i + 4 <= nv; i += 4) {
      const double2 v0 = ldc(V + (size_t)i * ldv, e), v1 = ldc(V + (size_t)(i + 1) * ldv, e);
      const double2 v2 = ldc(V + (size_t)(i + 2) * ldv, e), v3 = ldc(V + (size_t)(i + 3) * ldv, e);
      acc = cadd(acc, cmul(v0, make_double2(coef[2 * i], coef[2 * i + 1])));
      acc = cadd(acc, cmul(v1, make_double2(coef[2 * i + 2], coef[2 * i + 3])));
      acc = cadd(acc, cmul(v2, make_double2(coef[2 * i + 4], coef[2 * i + 5])));
      acc = cadd(acc, cmul(v3, make_double2(coef[2 * i + 6], coef[2 * i + 7])));
    }
    for (; i < nv; ++i) acc = cadd(acc, cmul(ldc(V + (size_t)i * ldv, e), make_double2(coef[2 * i], coef[2 * i + 1])));
    double2 r = base ? ldc(base, e) : czero();
    r.x += sgn * acc.x;
    r.y += sgn * acc.y;
    stc(out, e, r);
    if (NORM) nrm += r.x * r.x + r.y * r.y;
  }
  if (NORM) {
    nrm = block_sum(nrm, sh);
    if (threadIdx.x == 0) part[blockIdx.x] = nrm;
  }
}

template <typename S>
void multi_axpy(size_t n, const void* V, size_t ldv, int nv, const double* coef, double sgn, const void* base,
                void* out, double* part, hipStream_t st) {
  using C = cplx_t<S>;
  const int nb = red_nblocks(n);
  kprof_begin(KP_MULTIAXPY, st);
  if (part)
    hipLaunchKernelGGL((k_multi_axpy<S, true>), dim3(nb), dim3(256), 0, st, n, (const C*)V, ldv, nv, coef, sgn,
                       (const C*)base, (C*)out, part);
  else
    hipLaunchKernelGGL((k_multi_axpy<S, false>), dim3(nb), dim3(256), 0, st, n, (const C*)V, ldv, nv, coef, sgn,
                       (const C*)base, (C*)out, part);
  kprof_end(KP_MULTIAXPY, (double)n * 2 * sizeof(S) * (nv + (base ? 1 : 0) + 1), st);
}

// ---- fused CGS pass: w' = w - V h and the partials of V^H w' --------------------
// One pass over V: w' = w - sum_i V_i h_i is formed and stored, and the partials
// of conj(V_i) w' are produced from the same loaded values.  Two kernels:
//
// k_cgs_fused (nv <= 8): one element per thread, every V_i in registers;
//   conj(V_i) w' is reduced over the wavefront by a reduce-scatter butterfly
//   and then over the four wavefronts of the block in a fixed order.
//   Instantiated for NB = 4 and 8 register slots.
// k_cgs_split (nv > 8): WAVES wavefronts share each 64-element chunk and
//   wavefront q holds the vectors i = q, q + WAVES, ... (NW register slots), so
//   registers per lane stay small while the chunk's loads of all vectors are in
//   flight at once.  Per chunk: the wavefronts' partial sums of V h meet in LDS,
//   w' is formed by every wavefront in the same order (only wavefront 0 reads
//   and writes w; the others take w from LDS), then each wavefront adds
//   conj(V_i) w' for its vectors; after CH chunks one butterfly per wavefront.
//   Each vector belongs to one wavefront, so its partial needs no cross-wave sum.
//   1.4-1.5x faster than the one-element-per-thread form for nv >= 26.
constexpr int CG_MAX = 52;
int cgs_fused_max_nv() { return CG_MAX; }

// reduce-scatter over a wavefront of the 2 NW values x[] (NW a multiple of 4):
// afterwards lane 8g (g = 0..7) holds values [g NW/4, (g + 1) NW/4) in x[0..NW/4)
template <int NW>
__device__ __forceinline__ void wave_rs(double (&x)[2 * NW], int lane) {
  const bool b5 = (lane >> 5) & 1, b4 = (lane >> 4) & 1, b3 = (lane >> 3) & 1;
  constexpr int H1 = NW, H2 = NW / 2, H3 = NW / 4;
#pragma unroll
  for (int q = 0; q < H1; ++q) {
    const double keep = b5 ? x[H1 + q] : x[q], send = b5 ? x[q] : x[H1 + q];
    x[q] = keep + __shfl_xor(send, 32, 64);
  }
#pragma unroll
  for (int q = 0; q < H2; ++q) {
    const double keep = b4 ? x[H2 + q] : x[q], send = b4 ? x[q] : x[H2 + q];
    x[q] = keep + __shfl_xor(send, 16, 64);
  }
#pragma unroll
  for (int q = 0; q < H3; ++q) {
    const double keep = b3 ? x[H3 + q] : x[q], send = b3 ? x[q] : x[H3 + q];
    x[q] = keep + __shfl_xor(send, 8, 64);
  }
#pragma unroll
  for (int q = 0; q < H3; ++q) {
    double t = x[q];
    t += __shfl_xor(t, 4, 64);
    t += __shfl_xor(t, 2, 64);
    t += __shfl_xor(t, 1, 64);
    x[q] = t;
  }
}

template <typename S, int NB>
__global__ __launch_bounds__(256) void k_cgs_fused(size_t n, const cplx_t<S>* __restrict__ V, size_t ldv, int nv,
                                                   const double* __restrict__ h, cplx_t<S>* __restrict__ w,
                                                   double* __restrict__ part) {
  static_assert(NB % 4 == 0, "slot count: a multiple of 4");
  __shared__ double sh[4][2 * NB];
  const size_t e = blockIdx.x * (size_t)256 + threadIdx.x;
  const bool in = e < n;
  double2 v[NB];
#pragma unroll
  for (int i = 0; i < NB; ++i) v[i] = (i < nv && in) ? ldc(V + (size_t)i * ldv, e) : czero();
  double2 s = czero();
#pragma unroll
  for (int i = 0; i < NB; ++i)
    if (i < nv) s = cadd(s, cmul(v[i], make_double2(h[2 * i], h[2 * i + 1])));
  double2 wn = czero();
  if (in) {
    wn = csub(ldc(w, e), s);
    stc(w, e, wn);
    wn = ldc(w, e);  // the stored (possibly rounded) value enters the inner products
  }
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  double x[2 * NB];
#pragma unroll
  for (int i = 0; i < NB; ++i) {
    const double2 d = cconjmul(v[i], wn);  // v[i] = 0 beyond nv
    x[2 * i] = d.x;
    x[2 * i + 1] = d.y;
  }
  wave_rs<NB>(x, lane);
  if ((lane & 7) == 0) {
    const int g = lane >> 3;
#pragma unroll
    for (int q = 0; q < NB / 4; ++q) sh[wave][(NB / 4) * g + q] = x[q];
  }
  __syncthreads();
  for (int t = threadIdx.x; t < 2 * nv; t += 256)
    part[(size_t)blockIdx.x * 2 * nv + t] = (sh[0][t] + sh[1][t]) + (sh[2][t] + sh[3][t]);
}

template <typename S>
__device__ __forceinline__ double2 stored(double2 v) {
  if (sizeof(S) == sizeof(float)) return make_double2((double)(float)v.x, (double)(float)v.y);
  return v;
}

template <typename S, int NW, int WAVES, int CH>
__global__ __launch_bounds__(64 * WAVES) void k_cgs_split(size_t n, const cplx_t<S>* __restrict__ V, size_t ldv,
                                                        int nv, const double* __restrict__ h,
                                                        cplx_t<S>* __restrict__ w, double* __restrict__ part) {
  static_assert(NW % 4 == 0, "slot count: a multiple of 4");
  __shared__ double2 ss[2][WAVES][64];
  __shared__ double2 ws[2][64];
  __shared__ double sh[WAVES][2 * NW];
  const int lane = threadIdx.x & 63;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);  // uniform: h goes to scalar registers
  double x[2 * NW];
#pragma unroll
  for (int k = 0; k < 2 * NW; ++k) x[k] = 0.0;
  double2 hk[NW];
#pragma unroll
  for (int k = 0; k < NW; ++k) {
    const int i = wave + WAVES * k;
    hk[k] = i < nv ? make_double2(h[2 * i], h[2 * i + 1]) : czero();
  }
#pragma unroll 1
  for (int c = 0; c < CH; ++c) {
    const size_t e = ((size_t)blockIdx.x * CH + c) * 64 + lane;
    const bool in = e < n;
    double2 v[NW];
#pragma unroll
    for (int k = 0; k < NW; ++k) {
      const int i = wave + WAVES * k;
      v[k] = (i < nv && in) ? ldc(V + (size_t)i * ldv, e) : czero();
    }
    double2 s = czero();
#pragma unroll
    for (int k = 0; k < NW; ++k) s = cadd(s, cmul(v[k], hk[k]));
    ss[c & 1][wave][lane] = s;
    if (wave == 0) ws[c & 1][lane] = in ? ldc(w, e) : czero();
    __syncthreads();  // (the next write of this buffer comes after the next chunk's barrier)
    double2 t = czero();
#pragma unroll
    for (int q = 0; q < WAVES; ++q) t = cadd(t, ss[c & 1][q][lane]);
    double2 wn = czero();
    if (in) {
      wn = stored<S>(csub(ws[c & 1][lane], t));
      if (wave == 0) stc(w, e, wn);
    }
#pragma unroll
    for (int k = 0; k < NW; ++k) {
      const double2 d = cconjmul(v[k], wn);
      x[2 * k] += d.x;
      x[2 * k + 1] += d.y;
    }
  }
  wave_rs<NW>(x, lane);
  if ((lane & 7) == 0) {
    const int g = lane >> 3;
#pragma unroll
    for (int q = 0; q < NW / 4; ++q) sh[wave][(NW / 4) * g + q] = x[q];
  }
  __syncthreads();
  // value 2k + comp of wavefront q belongs to vector i = q + WAVES k
  for (int t = threadIdx.x; t < 2 * nv; t += 64 * WAVES) {
    const int i = t >> 1, q = i % WAVES, k = i / WAVES;
    part[(size_t)blockIdx.x * 2 * nv + t] = sh[q][2 * k + (t & 1)];
  }
}

int cgs_fused_nblocks(size_t n, int nv) {
  const size_t per = nv <= 16 ? 256 : 512;  // elements per workgroup (see cgs_fused)
  return (int)((n + per - 1) / per);
}

template <typename S>
int cgs_fused(size_t n, const void* V, size_t ldv, int nv, const double* h, void* w, double* part, hipStream_t st) {
  using C = cplx_t<S>;
  const int nb = cgs_fused_nblocks(n, nv);
  const C* Vc = (const C*)V;
  C* wc = (C*)w;
  kprof_begin(KP_CGS, st);
  if (nv <= 4)
    hipLaunchKernelGGL((k_cgs_fused<S, 4>), dim3(nb), dim3(256), 0, st, n, Vc, ldv, nv, h, wc, part);
  else if (nv <= 8)
    hipLaunchKernelGGL((k_cgs_fused<S, 8>), dim3(nb), dim3(256), 0, st, n, Vc, ldv, nv, h, wc, part);
  else if (nv <= 16)  // 4 wavefronts x 4 slots, 4 chunks of 64: 256 elements per workgroup
    hipLaunchKernelGGL((k_cgs_split<S, 4, 4, 4>), dim3(nb), dim3(256), 0, st, n, Vc, ldv, nv, h, wc, part);
  else if (nv <= 32)  // 8 wavefronts x 4 slots, 8 chunks: 512 elements per workgroup
    hipLaunchKernelGGL((k_cgs_split<S, 4, 8, 8>), dim3(nb), dim3(512), 0, st, n, Vc, ldv, nv, h, wc, part);
  else                // 8 wavefronts x 8 slots (nv <= 64)
    hipLaunchKernelGGL((k_cgs_split<S, 8, 8, 8>), dim3(nb), dim3(512), 0, st, n, Vc, ldv, nv, h, wc, part);
  // V once, w read and written
  kprof_end(KP_CGS, (double)n * 2 * sizeof(S) * (nv + 2), st);
  return nb;
}

// ---- simple vector kernels ----------------------------------------------------
#define GRID_STRIDE(e) \
  for (size_t e = blockIdx.x * (size_t)blockDim.x + threadIdx.x; e < n; e += (size_t)gridDim.x * blockDim.x)

static int ew_blocks(size_t n) {
  size_t nb = (n + 255) / 256;
  if (nb > 8192) nb = 8192;
  if (nb < 1) nb = 1;
  return (int)nb;
}

template <typename S>
__global__ void k_scale_dev(size_t n, const cplx_t<S>* x, const double* scal, cplx_t<S>* y) {
  const double a = scal[0];
  GRID_STRIDE(e) stc(y, e, cscale(ldc(x, e), a));
}
template <typename S>
__global__ void k_scale_host(size_t n, const cplx_t<S>* x, double a, cplx_t<S>* y) {
  GRID_STRIDE(e) stc(y, e, cscale(ldc(x, e), a));
}
template <typename S>
__global__ void k_add_inplace(size_t n, const cplx_t<S>* __restrict__ x, cplx_t<S>* __restrict__ y) {
  GRID_STRIDE(e) stc(y, e, cadd(ldc(y, e), ldc(x, e)));
}
template <typename S>
__global__ void k_copy(size_t n, const cplx_t<S>* __restrict__ x, cplx_t<S>* __restrict__ y) {
  GRID_STRIDE(e) y[e] = x[e];
}
template <typename S>
__global__ void k_zero(size_t n, cplx_t<S>* __restrict__ x) {
  GRID_STRIDE(e) stc(x, e, czero());
}
template <typename S>
__global__ void k_axpy_dev(size_t n, const cplx_t<S>* __restrict__ x, cplx_t<S>* __restrict__ y,
                           const double* __restrict__ a) {
  const double2 av = make_double2(a[0], a[1]);
  GRID_STRIDE(e) stc(y, e, cadd(ldc(y, e), cmul(av, ldc(x, e))));
}

template <typename S>
void scale_dev(size_t n, const void* x, const double* scal, void* y, hipStream_t st) {
  using C = cplx_t<S>;
  hipLaunchKernelGGL((k_scale_dev<S>), dim3(ew_blocks(n)), dim3(256), 0, st, n, (const C*)x, scal, (C*)y);
}
template <typename S>
void scale_host(size_t n, const void* x, double a, void* y, hipStream_t st) {
  using C = cplx_t<S>;
  hipLaunchKernelGGL((k_scale_host<S>), dim3(ew_blocks(n)), dim3(256), 0, st, n, (const C*)x, a, (C*)y);
}
template <typename S>
void add_inplace(size_t n, const void* x, void* y, hipStream_t st) {
  using C = cplx_t<S>;
  hipLaunchKernelGGL((k_add_inplace<S>), dim3(ew_blocks(n)), dim3(256), 0, st, n, (const C*)x, (C*)y);
}
template <typename S>
void copy_vec(size_t n, const void* x, void* y, hipStream_t st) {
  using C = cplx_t<S>;
  hipLaunchKernelGGL((k_copy<S>), dim3(ew_blocks(n)), dim3(256), 0, st, n, (const C*)x, (C*)y);
}
template <typename S>
void zero_vec(size_t n, void* x, hipStream_t st) {
  using C = cplx_t<S>;
  hipLaunchKernelGGL((k_zero<S>), dim3(ew_blocks(n)), dim3(256), 0, st, n, (C*)x);
}
template <typename S>
void axpy_dev(size_t n, const void* x, void* y, const double* a, hipStream_t st) {
  using C = cplx_t<S>;
  hipLaunchKernelGGL((k_axpy_dev<S>), dim3(ew_blocks(n)), dim3(256), 0, st, n, (const C*)x, (C*)y, a);
}

// ---- BiCGStab ------------------------------------------------------------------
template <typename S>
__global__ void k_bicg_p(size_t n, const cplx_t<S>* __restrict__ r, const cplx_t<S>* __restrict__ v,
                         cplx_t<S>* __restrict__ p, const BiState* __restrict__ bs, int first) {
  if (bs->flag) return;
  const double2 beta = make_double2(bs->beta[0], bs->beta[1]);
  const double2 om = make_double2(bs->omega[0], bs->omega[1]);
  GRID_STRIDE(e) {
    const double2 re = ldc(r, e);
    if (first) {
      stc(p, e, re);
    } else {
      const double2 t = csub(ldc(p, e), cmul(om, ldc(v, e)));
      stc(p, e, cadd(re, cmul(beta, t)));
    }
  }
}

template <typename S>
__global__ __launch_bounds__(256) void k_bicg_s(size_t n, const cplx_t<S>* __restrict__ r,
                                                const cplx_t<S>* __restrict__ v, cplx_t<S>* __restrict__ s,
                                                const BiState* __restrict__ bs, double* __restrict__ part) {
  __shared__ double sh[16];
  const double2 al = make_double2(bs->alpha[0], bs->alpha[1]);
  double nrm = 0.0;
  GRID_STRIDE(e) {
    const double2 q = csub(ldc(r, e), cmul(al, ldc(v, e)));
    stc(s, e, q);
    nrm += q.x * q.x + q.y * q.y;
  }
  nrm = block_sum(nrm, sh);
  if (threadIdx.x == 0) part[blockIdx.x] = nrm;
}

template <typename S>
__global__ __launch_bounds__(256) void k_two_dot(size_t n, const cplx_t<S>* __restrict__ t,
                                                 const cplx_t<S>* __restrict__ s, double* __restrict__ part) {
  __shared__ double sh[32];
  double2 ts = czero();
  double tt = 0.0;
  GRID_STRIDE(e) {
    const double2 te = ldc(t, e);
    ts = cadd(ts, cconjmul(te, ldc(s, e)));
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

template <typename S>
__global__ __launch_bounds__(256) void k_bicg_update(size_t n, const cplx_t<S>* __restrict__ ph,
                                                     const cplx_t<S>* __restrict__ shat,
                                                     const cplx_t<S>* __restrict__ s, const cplx_t<S>* __restrict__ t,
                                                     const cplx_t<S>* __restrict__ rhat, cplx_t<S>* __restrict__ u,
                                                     cplx_t<S>* __restrict__ r, const BiState* __restrict__ bs,
                                                     double* __restrict__ part) {
  __shared__ double sh[32];
  if (bs->flag) return;  // breakdown flagged on the device: leave u and r as they are
  const double2 al = make_double2(bs->alpha[0], bs->alpha[1]);
  const double2 om = make_double2(bs->omega[0], bs->omega[1]);
  double rr = 0.0;
  double2 rho = czero();
  GRID_STRIDE(e) {
    const double2 ue = cadd(ldc(u, e), cadd(cmul(al, ldc(ph, e)), cmul(om, ldc(shat, e))));
    stc(u, e, ue);
    const double2 re = csub(ldc(s, e), cmul(om, ldc(t, e)));
    stc(r, e, re);
    rr += re.x * re.x + re.y * re.y;
    rho = cadd(rho, cconjmul(ldc(rhat, e), re));
  }
  rr = block_sum(rr, sh);
  rho = block_sum2(rho, sh);
  if (threadIdx.x == 0) {
    part[3 * blockIdx.x] = rr;
    part[3 * blockIdx.x + 1] = rho.x;
    part[3 * blockIdx.x + 2] = rho.y;
  }
}

template <typename S>
void bicg_p(size_t n, const void* r, const void* v, void* p, const BiState* bs, int first, hipStream_t st) {
  using C = cplx_t<S>;
  hipLaunchKernelGGL((k_bicg_p<S>), dim3(ew_blocks(n)), dim3(256), 0, st, n, (const C*)r, (const C*)v, (C*)p, bs,
                     first);
}
template <typename S>
void bicg_s(size_t n, const void* r, const void* v, void* s, const BiState* bs, double* part, hipStream_t st) {
  using C = cplx_t<S>;
  hipLaunchKernelGGL((k_bicg_s<S>), dim3(red_nblocks(n)), dim3(256), 0, st, n, (const C*)r, (const C*)v, (C*)s, bs,
                     part);
}
template <typename S>
void two_dot_part(size_t n, const void* t, const void* s, double* part, hipStream_t st) {
  using C = cplx_t<S>;
  hipLaunchKernelGGL((k_two_dot<S>), dim3(red_nblocks(n)), dim3(256), 0, st, n, (const C*)t, (const C*)s, part);
}
template <typename S>
void bicg_update(size_t n, const void* ph, const void* sh, const void* s, const void* t, const void* rhat, void* u,
                 void* r, const BiState* bs, double* part, hipStream_t st) {
  using C = cplx_t<S>;
  hipLaunchKernelGGL((k_bicg_update<S>), dim3(red_nblocks(n)), dim3(256), 0, st, n, (const C*)ph, (const C*)sh,
                     (const C*)s, (const C*)t, (const C*)rhat, (C*)u, (C*)r, bs, part);
}

__device__ static bool finite2(double2 a) { return isfinite(a.x) && isfinite(a.y); }

__device__ void bicg_step(int step, BiState* bs, const double* red) {
  if (step == BI_RHO) {
    const double2 rho = make_double2(red[0], red[1]);
    if (!finite2(rho)) {
      bs->flag = -5;
      return;
    }
    if (rho.x == 0.0 && rho.y == 0.0) {
      bs->flag = -4;
      return;
    }
    const double2 rho0 = make_double2(bs->rho0[0], bs->rho0[1]);
    const double2 al = make_double2(bs->alpha[0], bs->alpha[1]);
    const double2 om = make_double2(bs->omega[0], bs->omega[1]);
    const double2 beta = cmul(cdiv(rho, rho0), cdiv(al, om));
    bs->beta[0] = beta.x;
    bs->beta[1] = beta.y;
    bs->rho[0] = rho.x;
    bs->rho[1] = rho.y;
  } else if (step == BI_ALPHA) {
    const double2 den = make_double2(red[0], red[1]);
    if (!finite2(den)) {
      bs->flag = -5;
      return;
    }
    if (den.x == 0.0 && den.y == 0.0) {
      bs->flag = -4;
      return;
    }
    const double2 al = cdiv(make_double2(bs->rho[0], bs->rho[1]), den);
    bs->alpha[0] = al.x;
    bs->alpha[1] = al.y;
  } else if (step == BI_SS) {
    bs->ss = sqrt(red[0]);
  } else if (step == BI_OMEGA) {
    const double2 ts = make_double2(red[0], red[1]);
    const double tt = red[2];
    double2 om = czero();
    if (tt != 0.0) om = make_double2(ts.x / tt, ts.y / tt);
    if (!finite2(om)) {
      bs->flag = -5;
      return;
    }
    if (om.x == 0.0 && om.y == 0.0) {
      bs->flag = -4;
      return;
    }
    bs->omega[0] = om.x;
    bs->omega[1] = om.y;
  } else if (step == BI_RR) {
    bs->rr = sqrt(red[0]);
    bs->rho0[0] = bs->rho[0];
    bs->rho0[1] = bs->rho[1];
  } else if (step == BI_INIT) {
    for (int q = 0; q < 2; ++q) {
      bs->rho[q] = 0.0;
      bs->beta[q] = 0.0;
      bs->rho0[q] = bs->alpha[q] = bs->omega[q] = q == 0 ? 1.0 : 0.0;
    }
    bs->ss = 0.0;
    bs->fn = red[0];
    bs->rr = red[1];
    bs->flag = 0;
    bs->pad = 0;
  }
}

// ghost: optional copy of the record in pinned host memory, made visible to
// the host by the kernel itself (the event the host waits on carries no
// system-scope release)
__global__ void k_bicg_scalar(int step, BiState* bs, const double* red, BiState* ghost) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  bicg_step(step, bs, red);
  if (ghost) {
    *ghost = *bs;
    __threadfence_system();
  }
}

void bicg_scalar(int step, BiState* bs, const double* red, hipStream_t st, BiState* ghost) {
  hipLaunchKernelGGL(k_bicg_scalar, dim3(1), dim3(64), 0, st, step, bs, red, ghost);
}

#define HELM_INST(S)                                                                                           \
  template void dot_part<S>(size_t, const void*, const void*, double*, hipStream_t);                           \
  template void nrm2_part<S>(size_t, const void*, double*, hipStream_t);                                       \
  template void multidot_part<S>(size_t, const void*, size_t, int, const void*, double*, hipStream_t);         \
  template void multi_axpy<S>(size_t, const void*, size_t, int, const double*, double, const void*, void*,     \
                              double*, hipStream_t);                                                           \
  template int cgs_fused<S>(size_t, const void*, size_t, int, const double*, void*, double*, hipStream_t);     \
  template void multidot_apply<S>(const StencilGeom&, const void*, const uint8_t*, const void*, const void*,   \
                                  size_t, int, void*, double*, hipStream_t);                                   \
  template void scale_dev<S>(size_t, const void*, const double*, void*, hipStream_t);                          \
  template void scale_host<S>(size_t, const void*, double, void*, hipStream_t);                                \
  template void add_inplace<S>(size_t, const void*, void*, hipStream_t);                                       \
  template void copy_vec<S>(size_t, const void*, void*, hipStream_t);                                          \
  template void zero_vec<S>(size_t, void*, hipStream_t);                                                       \
  template void axpy_dev<S>(size_t, const void*, void*, const double*, hipStream_t);                           \
  template void bicg_p<S>(size_t, const void*, const void*, void*, const BiState*, int, hipStream_t);          \
  template void bicg_s<S>(size_t, const void*, const void*, void*, const BiState*, double*, hipStream_t);      \
  template void two_dot_part<S>(size_t, const void*, const void*, double*, hipStream_t);                       \
  template void bicg_update<S>(size_t, const void*, const void*, const void*, const void*, const void*, void*, \
                               void*, const BiState*, double*, hipStream_t);
HELM_INST(double)
HELM_INST(float)
#undef HELM_INST

}  // namespace helm
