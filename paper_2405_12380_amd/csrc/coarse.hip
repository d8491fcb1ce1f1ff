// Trunk-basis coarse space of App. C and its per-application correction.
//
// Setup (once per network, p_used and k^2): P = first p_used trunk columns with
// scatterer rows zeroed; Cholesky of P^T P with column dropping, Q1 = P S1.
// fp64 basis: the solves use Q1 (it spans the space of the orthonormal
// Q = Q1 S2 of a second CholeskyQR pass, and the correction depends only on
// that span).  fp32 basis: the second pass is run and Q rounded to fp32.  In
// either basis X: B = (L - diag(Re s)) X by a batched real stencil; the
// Galerkin matrix X^T B - i X^T diag(Im s) X (= X^T A X); its inverse by
// Gauss-Jordan with partial pivoting.
//
// Correction z += X (X^T A X)^{-1} X^T r1 (HBM-bound skinny products):
//   k_qt_part   per-block partials of Q^T r1: lanes own columns {l, l+64},
//               the grid's wavefronts sweep Q in four-row groups, one
//               coalesced 2 x 512 B row read per row;
//   k_ainv      c = A_c^{-1} y, one workgroup per row of A_c^{-1};
//   k_skinny    y_i = sum_j Q_ij c_j: lanes own columns, four rows per step,
//               reduced with an 11-shuffle butterfly that leaves row rho's
//               (re, im) in lane 16 rho.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <vector>

#include "common.h"
#include "dense.h"
#include "internal.h"
#include "lib.h"
#include "prof.h"
#include "coarse_dev.h"
#include "stencil_dev.h"

namespace helm {

static constexpr int QT_MAXB = 512;

int qt_nblocks(size_t n) {
  size_t nb = (n + 511) / 512;
  if (nb > QT_MAXB) nb = QT_MAXB;
  if (nb < 1) nb = 1;
  return (int)nb;
}

// the fp32-basis restriction reads half the bytes per row and runs twice the
// workgroups to keep as many bytes in flight
static constexpr int QT32_MAXB = 1024;
int qt_nblocks32(size_t n) {
  size_t nb = (n + 255) / 256;
  if (nb > QT32_MAXB) nb = QT32_MAXB;
  if (nb < 1) nb = 1;
  return (int)nb;
}

// part[b][2j + {0,1}] = sum over the rows of block b of Q_ij x_i (complex x,
// real Q, j < r <= 128).  Rows go in groups of four; wavefront g of the W in
// the grid takes groups g, g + W, g + 2W, ..., so at any moment the whole grid
// reads one contiguous stretch of Q (DRAM pages stay open; this sweep is ~8%
// faster than giving each block a contiguous range).  The row-to-block
// assignment depends only on n, so the partials are reproducible.
template <typename T, typename S>
__global__ __launch_bounds__(256) void k_qt_part(size_t n, int r, const T* __restrict__ Q,
                                                 const cplx_t<S>* __restrict__ x, double* __restrict__ part) {
  __shared__ double sh[4][256];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int c0 = lane, c1 = lane + 64;
  const bool u0 = c0 < r, u1 = c1 < r;
  const size_t W = ((size_t)gridDim.x * blockDim.x) >> 6, ng = (n + 3) / 4;
  double a0r = 0, a0i = 0, a1r = 0, a1i = 0;
  for (size_t g = (blockIdx.x * (size_t)blockDim.x + threadIdx.x) >> 6; g < ng; g += W) {
    double q0[4], q1[4];
    double2 xv[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const size_t ii = 4 * g + u;
      const bool in = ii < n;
      xv[u] = in ? ldc(x, ii) : czero();
      q0[u] = in && u0 ? ldq(Q, ii * r + c0) : 0.0;
      q1[u] = in && u1 ? ldq(Q, ii * r + c1) : 0.0;
    }
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      a0r += q0[u] * xv[u].x;
      a0i += q0[u] * xv[u].y;
      a1r += q1[u] * xv[u].x;
      a1i += q1[u] * xv[u].y;
    }
  }
  sh[wave][2 * c0] = a0r;
  sh[wave][2 * c0 + 1] = a0i;
  sh[wave][2 * c1] = a1r;
  sh[wave][2 * c1 + 1] = a1i;
  __syncthreads();
  for (int e = threadIdx.x; e < 2 * r; e += blockDim.x)
    part[(size_t)blockIdx.x * 2 * r + e] = (sh[0][e] + sh[1][e]) + (sh[2][e] + sh[3][e]);
}

// fp32 basis: each half-wavefront takes one row, lane m of it the four
// columns 4m .. 4m + 3 (one 16-byte load; a wavefront reads two 512 B rows per
// instruction); groups of four row pairs in the same grid sweep.  Rows whose
// length r is not a multiple of 4 are read one float at a time.
template <typename S>
__global__ __launch_bounds__(256) void k_qt_part32(size_t n, int r, const float* __restrict__ Q,
                                                   const cplx_t<S>* __restrict__ x, double* __restrict__ part) {
  constexpr int U = 4;
  __shared__ double sh[4][2][256];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int h = lane >> 5, m = lane & 31;
  const bool v4 = (r & 3) == 0;
  const size_t W = ((size_t)gridDim.x * blockDim.x) >> 6, ng = (n + 2 * U - 1) / (2 * U);
  double acc[8] = {0, 0, 0, 0, 0, 0, 0, 0};
  for (size_t g = (blockIdx.x * (size_t)blockDim.x + threadIdx.x) >> 6; g < ng; g += W) {
    float4 q[U];
    double2 xv[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const size_t ii = 2 * U * g + 2 * u + h;
      const bool in = ii < n;
      xv[u] = in ? ldc(x, ii) : czero();
      if (in && v4 && 4 * m < r) {
        q[u] = *reinterpret_cast<const float4*>(Q + ii * r + 4 * m);
      } else {
        const float* row = Q + ii * r;
        const int c = 4 * m;
        q[u] = make_float4(in && c < r ? row[c] : 0.f, in && c + 1 < r ? row[c + 1] : 0.f,
                           in && c + 2 < r ? row[c + 2] : 0.f, in && c + 3 < r ? row[c + 3] : 0.f);
      }
    }
#pragma unroll
    for (int u = 0; u < U; ++u) {
      acc[0] += (double)q[u].x * xv[u].x;
      acc[1] += (double)q[u].x * xv[u].y;
      acc[2] += (double)q[u].y * xv[u].x;
      acc[3] += (double)q[u].y * xv[u].y;
      acc[4] += (double)q[u].z * xv[u].x;
      acc[5] += (double)q[u].z * xv[u].y;
      acc[6] += (double)q[u].w * xv[u].x;
      acc[7] += (double)q[u].w * xv[u].y;
    }
  }
#pragma unroll
  for (int k = 0; k < 8; ++k) sh[wave][h][8 * m + k] = acc[k];  // = 2 column + (re, im)
  __syncthreads();
  for (int e = threadIdx.x; e < 2 * r; e += blockDim.x) {
    double v = 0.0;
#pragma unroll
    for (int w = 0; w < 4; ++w) v += sh[w][0][e] + sh[w][1][e];
    part[(size_t)blockIdx.x * 2 * r + e] = v;
  }
}

// c = Ainv y: block j computes row j (r x r complex, row-major)
__global__ __launch_bounds__(64) void k_ainv(int r, const double* __restrict__ Ainv, const double* __restrict__ y,
                                             double* __restrict__ c) {
  const int j = blockIdx.x, l = threadIdx.x;
  double2 acc = czero();
  for (int k0 = 0; k0 < r; k0 += 128) {  // both halves' loads in flight at once
    double2 a[2], b[2];
#pragma unroll
    for (int q = 0; q < 2; ++q) {
      const int k = k0 + l + 64 * q;
      const size_t o = 2 * ((size_t)j * r + k);
      a[q] = k < r ? make_double2(Ainv[o], Ainv[o + 1]) : czero();
      b[q] = k < r ? make_double2(y[2 * k], y[2 * k + 1]) : czero();
    }
#pragma unroll
    for (int q = 0; q < 2; ++q) acc = cadd(acc, cmul(a[q], b[q]));
  }
  acc.x = wave_sum(acc.x);
  acc.y = wave_sum(acc.y);
  if (l == 0) {
    c[2 * j] = acc.x;
    c[2 * j + 1] = acc.y;
  }
}

template <typename T, typename S, int MODE>
__global__ __launch_bounds__(256) void k_skinny(size_t n, int r, const T* __restrict__ Q, const double* __restrict__ c,
                                                cplx_t<S>* __restrict__ z, const uint8_t* __restrict__ mask,
                                                const double* __restrict__ scal) {
  skinny_rows<T, S, MODE>(n, r, Q, c, z, mask, scal, (blockIdx.x * (size_t)blockDim.x + threadIdx.x) >> 6,
                          ((size_t)gridDim.x * blockDim.x) >> 6);
}

// fp32 basis version of k_skinny: one row per thread, the row read in 16-byte
// pieces (one float at a time when r is not a multiple of 4), c staged in LDS;
// no cross-lane reduction, so the half-size rows do not leave the shuffles
// dominant.  Same two modes as k_skinny.
template <typename S, int MODE>
__global__ __launch_bounds__(256) void k_skinny32(size_t n, int r, const float* __restrict__ Q,
                                                  const double* __restrict__ c, cplx_t<S>* __restrict__ z,
                                                  const uint8_t* __restrict__ mask, const double* __restrict__ scal) {
  __shared__ double2 cs[128];
  const int t = threadIdx.x;
  if (t < 128) cs[t] = t < r ? make_double2(c[2 * t], c[2 * t + 1]) : czero();
  __syncthreads();
  double sc = 1.0;
  if (MODE == SK_SYNTH) sc = scal[0];
  const bool v4 = (r & 3) == 0;
  const int nq = (r + 3) / 4;  // 16-byte pieces per row (at most 32)
  for (size_t i = blockIdx.x * (size_t)blockDim.x + t; i < n; i += (size_t)gridDim.x * blockDim.x) {
    const float* row = Q + i * r;
    double yr = 0.0, yi = 0.0;
#pragma unroll 1
    for (int j0 = 0; j0 < nq; j0 += 8) {
      float4 q[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        const int cq = 4 * (j0 + u);
        if (j0 + u < nq && v4) {
          q[u] = *reinterpret_cast<const float4*>(row + cq);
        } else {
          q[u] = make_float4(cq < r ? row[cq] : 0.f, cq + 1 < r ? row[cq + 1] : 0.f, cq + 2 < r ? row[cq + 2] : 0.f,
                             cq + 3 < r ? row[cq + 3] : 0.f);
        }
      }
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        const int cq = 4 * (j0 + u);  // <= 124: cs[] beyond r holds zeros
        const double2 c0 = cs[cq], c1 = cs[cq + 1], c2 = cs[cq + 2], c3 = cs[cq + 3];
        yr += (double)q[u].x * c0.x;
        yi += (double)q[u].x * c0.y;
        yr += (double)q[u].y * c1.x;
        yi += (double)q[u].y * c1.y;
        yr += (double)q[u].z * c2.x;
        yi += (double)q[u].z * c2.y;
        yr += (double)q[u].w * c3.x;
        yi += (double)q[u].w * c3.y;
      }
    }
    const double2 y = make_double2(yr, yi);
    if (MODE == SK_ADD) stc(z, i, cadd(ldc(z, i), y));
    else stc(z, i, mask[i] ? czero() : cscale(y, sc));
  }
}

// B = (L - diag(Re s)) Q on real columns (n x r, row-major); masked rows -> 0.
// A row of 4 nodes per workgroup step (threadIdx.y), the 64 lanes across the
// node's columns; absent neighbours (ghost or masked) come from the node's
// neighbour code, so no coordinates are formed.
template <typename S>
__global__ __launch_bounds__(256) void k_batched_lap(StencilGeom g, int r, const double* __restrict__ Q,
                                                     const cplx_t<S>* __restrict__ sc, const uint8_t* __restrict__ code,
                                                     double* __restrict__ B) {
  const size_t n = (size_t)g.nx * g.ny * g.nz;
  const size_t ry = (size_t)g.nx * r, rz = (size_t)g.nx * g.ny * r;
  for (size_t p = blockIdx.x * (size_t)blockDim.y + threadIdx.y; p < n; p += (size_t)gridDim.x * blockDim.y) {
    const unsigned cd = code[p];
    const size_t row = p * r;
    const double sre = ldc(sc, p).x;
    for (int j = threadIdx.x; j < r; j += 64) {
      const size_t e = row + j;
      if (cd & NB_SELF) {
        B[e] = 0.0;
        continue;
      }
      const double c = Q[e];
      const double xm = (cd & NB_XM) ? 0.0 : Q[e - r];
      const double xp = (cd & NB_XP) ? 0.0 : Q[e + r];
      const double ym = (cd & NB_YM) ? 0.0 : Q[e - ry];
      const double yp = (cd & NB_YP) ? 0.0 : Q[e + ry];
      double acc = ((c - xm) + (c - xp)) * g.ih2[0];
      acc = acc + ((c - ym) + (c - yp)) * g.ih2[1];
      if (g.dim == 3) {
        const double zm = (cd & NB_ZM) ? 0.0 : Q[e - rz];
        const double zp = (cd & NB_ZP) ? 0.0 : Q[e + rz];
        acc = acc + ((c - zm) + (c - zp)) * g.ih2[2];
      }
      B[e] = acc - sre * c;
    }
  }
}

template <typename S>
__global__ void k_im_s(size_t n, const cplx_t<S>* __restrict__ sc, double* __restrict__ w) {
  for (size_t p = blockIdx.x * (size_t)blockDim.x + threadIdx.x; p < n; p += (size_t)gridDim.x * blockDim.x)
    w[p] = ldc(sc, p).y;
}

// P = T[:, :pu] (T: n x p, dtype precision) in fp64 with masked rows zeroed
template <typename T>
__global__ void k_mask_cols(size_t n, int p, int pu, const T* __restrict__ Tm, const uint8_t* __restrict__ mask,
                            double* __restrict__ P) {
  const size_t total = n * pu;
  for (size_t e = blockIdx.x * (size_t)blockDim.x + threadIdx.x; e < total; e += (size_t)gridDim.x * blockDim.x) {
    const size_t i = e / pu;
    const int j = (int)(e % pu);
    P[e] = mask[i] ? 0.0 : (double)Tm[i * p + j];
  }
}

// rows of scatterer nodes zeroed in place (T: n x p): the op's cached trunk
// matrix is kept masked, which the network synthesis (zero on the scatterer)
// does not see and the coarse space needs
template <typename T>
__global__ __launch_bounds__(256) void k_zero_masked_rows(size_t n, int p, const uint8_t* __restrict__ mask,
                                                          T* __restrict__ Tm) {
  // one row per wavefront step (threadIdx.y), the lanes across its p entries
  for (size_t i = blockIdx.x * (size_t)blockDim.y + threadIdx.y; i < n; i += (size_t)gridDim.x * blockDim.y)
    if (mask[i])
      for (int c = threadIdx.x; c < p; c += 64) Tm[i * p + c] = T(0);
}

// Qs = (T) Q and Q <- (double) Qs, so the coarse matrix is built from the basis
// actually stored.
template <typename T>
__global__ void k_round_q(size_t total, double* __restrict__ Q, T* __restrict__ Qs) {
  for (size_t e = blockIdx.x * (size_t)blockDim.x + threadIdx.x; e < total; e += (size_t)gridDim.x * blockDim.x) {
    const T v = (T)Q[e];
    Qs[e] = v;
    Q[e] = (double)v;
  }
}

__global__ void k_combine_ac(int r2, const double* __restrict__ re, const double* __restrict__ im,
                             double* __restrict__ Ac) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e < r2) {
    Ac[2 * e] = re[e];
    Ac[2 * e + 1] = -im[e];
  }
}

// Ac = S^T M S for real S (r x r, row-major) and complex M (r x r, interleaved,
// row-major): workgroup i forms row i, first u = S[:, i]^T M (a row, in LDS),
// then Ac[i][j] = sum_b u_b S[b][j]; sums in index order.
__global__ __launch_bounds__(128) void k_sandwich(int r, const double* __restrict__ S, const double* __restrict__ M,
                                                  double* __restrict__ Ac) {
  __shared__ double2 u[128];
  const int i = blockIdx.x, t = threadIdx.x;
  if (t < r) {
    double2 acc = czero();
    for (int a = 0; a < r; ++a) {
      const double sa = S[(size_t)a * r + i];
      acc.x += sa * M[2 * ((size_t)a * r + t)];
      acc.y += sa * M[2 * ((size_t)a * r + t) + 1];
    }
    u[t] = acc;
  }
  __syncthreads();
  if (t < r) {
    double2 acc = czero();
    for (int b = 0; b < r; ++b) {
      const double sb = S[(size_t)b * r + t];
      acc.x += u[b].x * sb;
      acc.y += u[b].y * sb;
    }
    Ac[2 * ((size_t)i * r + t)] = acc.x;
    Ac[2 * ((size_t)i * r + t) + 1] = acc.y;
  }
}

static unsigned ew_grid(size_t total) {
  size_t nb = (total + 255) / 256;
  if (nb > 16384) nb = 16384;
  if (nb < 1) nb = 1;
  return (unsigned)nb;
}

// ---- launchers used by other units ------------------------------------------------
// returns the number of partial rows written
template <typename T, typename S>
int qt_partials(size_t n, int r, const T* Q, const void* x, double* part, hipStream_t st) {
  const int nb = sizeof(T) == sizeof(float) ? qt_nblocks32(n) : qt_nblocks(n);
  kprof_begin(KP_QT, st);
  if (sizeof(T) == sizeof(float))
    hipLaunchKernelGGL((k_qt_part32<S>), dim3(nb), dim3(256), 0, st, n, r, (const float*)Q, (const cplx_t<S>*)x, part);
  else
    hipLaunchKernelGGL((k_qt_part<T, S>), dim3(nb), dim3(256), 0, st, n, r, Q, (const cplx_t<S>*)x, part);
  kprof_end(KP_QT, (double)n * (sizeof(T) * r + 2 * sizeof(S)), st);
  return nb;
}

template <typename T, typename S>
void skinny_apply(size_t n, int r, const T* Q, const double* c, void* z, const uint8_t* mask, const double* scal,
                  int synth, hipStream_t st) {
  size_t waves = (n + 3) / 4;
  size_t nb = (waves + 3) / 4;
  if (nb > 4096) nb = 4096;
  if (nb < 1) nb = 1;
  kprof_begin(KP_SKINNY, st);
  if (sizeof(T) == sizeof(float)) {
    const float* Qf = (const float*)Q;
    nb = (n + 255) / 256;  // one row per thread, grid-strided
    if (nb > 1024) nb = 1024;
    if (synth)
      hipLaunchKernelGGL((k_skinny32<S, SK_SYNTH>), dim3((unsigned)nb), dim3(256), 0, st, n, r, Qf, c, (cplx_t<S>*)z,
                         mask, scal);
    else
      hipLaunchKernelGGL((k_skinny32<S, SK_ADD>), dim3((unsigned)nb), dim3(256), 0, st, n, r, Qf, c, (cplx_t<S>*)z,
                         mask, scal);
  } else if (synth) {
    hipLaunchKernelGGL((k_skinny<T, S, SK_SYNTH>), dim3((unsigned)nb), dim3(256), 0, st, n, r, Q, c, (cplx_t<S>*)z,
                       mask, scal);
  } else {
    hipLaunchKernelGGL((k_skinny<T, S, SK_ADD>), dim3((unsigned)nb), dim3(256), 0, st, n, r, Q, c, (cplx_t<S>*)z, mask,
                       scal);
  }
  // Q once; z read and written (ADD) or du written and the mask read (SYNTH)
  kprof_end(KP_SKINNY, (double)n * (sizeof(T) * r + (synth ? 2 * sizeof(S) + 1 : 4 * sizeof(S))), st);
}
template void skinny_apply<double, double>(size_t, int, const double*, const double*, void*, const uint8_t*,
                                           const double*, int, hipStream_t);
template void skinny_apply<float, float>(size_t, int, const float*, const double*, void*, const uint8_t*,
                                         const double*, int, hipStream_t);
template void skinny_apply<float, double>(size_t, int, const float*, const double*, void*, const uint8_t*,
                                          const double*, int, hipStream_t);

// ---- setup -----------------------------------------------------------------------
void coarse_trim(helm_op_s* op) {
  Coarse& c = op->coarse;
  c.T.release();
  c.T_serial = -1;
  c.W1.release();
  c.W2.release();
}

void coarse_release(helm_op_s* op) {
  Coarse& c = op->coarse;
  c.Q.release();
  c.Ainv.release();
  c.Ac.release();
  c.T.release();
  c.W1.release();
  c.W2.release();
  c.small.release();
  c.qpart.release();
  if (c.pending) {
    (void)hipEventSynchronize(c.ev1);
    (void)hipEventDestroy(c.ev0);
    (void)hipEventDestroy(c.ev1);
    c.pending = false;
  }
  c.valid = false;
  c.T_serial = -1;
}

// Checks the inverse's record (8 ints, then the condition estimate) that the
// set-up copied to host memory, and settles the space: valid with its
// condition estimate and set-up time, or invalid with the error.
static helm_status coarse_settle(helm_op_s* op, const void* rec_host) {
  Coarse& c = op->coarse;
  const int* rec = (const int*)rec_host;
  helm_status s = HELM_OK;
  if (!c.pass1 && (rec[3] != 0 || rec[2] != c.rank))
    s = fail(HELM_E_SINGULAR, "coarse: second CholeskyQR pass lost rank (%d of %d)", rec[2], c.rank);
  else if (rec[0] != 0)
    s = fail(HELM_E_SINGULAR, "coarse: A_c is singular (zero pivot)");
  c.cond_est = *(const double*)(rec + 8);
  float ms = 0.f;
  (void)hipEventElapsedTime(&ms, c.ev0, c.ev1);
  c.setup_ms = ms;
  (void)hipEventDestroy(c.ev0);
  (void)hipEventDestroy(c.ev1);
  c.pending = false;
  c.valid = s == HELM_OK;
  return s;
}

helm_status coarse_finish(helm_op_s* op) {
  Coarse& c = op->coarse;
  if (!c.pending) return HELM_OK;
  hipError_t e = hipEventSynchronize(c.ev1);
  if (e != hipSuccess) {
    (void)hipEventDestroy(c.ev0);
    (void)hipEventDestroy(c.ev1);
    c.pending = false;
    c.valid = false;
    return hip_fail(e, "coarse: inverse wait");
  }
  return coarse_settle(op, op->host + COARSE_REC);
}

template <typename TT, typename S>
static helm_status coarse_build(helm_op_s* op, don_s* net, int p_used, bool qf32, bool defer, hipStream_t st) {
  Coarse& c = op->coarse;
  const size_t n = op->nn;
  helm_status s;
  hipEvent_t e0, e1;
  (void)hipEventCreate(&e0);
  (void)hipEventCreate(&e1);
  (void)hipEventRecord(e0, st);
  // trunk matrix at the op's nodes (cached per network)
  const int p = don_p(net);
  if (c.T_serial != don_serial(net)) {
    if ((s = c.T.ensure(n * (size_t)p * sizeof(TT)))) return s;
    if ((s = don_trunk(net, op, c.T.ptr, st))) return s;
    c.T_serial = don_serial(net);
  }
  const int pu = p_used;
  // fp64 trunk (C128): P is the masked trunk matrix itself, read with its row
  // stride p; fp32 trunk (C64): P is widened into W1
  const bool wide_t = sizeof(TT) == sizeof(double);
  c.q_f32 = qf32 || !wide_t;
  c.pass1 = !c.q_f32;  // fp64 basis: the first pass's basis is the one used
  if (!wide_t && (s = c.W1.ensure(n * (size_t)pu * sizeof(double)))) return s;
  if (c.q_f32 && (s = c.W2.ensure(n * (size_t)pu * sizeof(double)))) return s;
  const size_t small_doubles = (size_t)gram_nblocks(n) * pu * pu + 10 * (size_t)pu * pu + 4096;
  if ((s = c.small.ensure(small_doubles * sizeof(double)))) return s;
  double* part = (double*)c.small.ptr;
  double* G = part + (size_t)gram_nblocks(n) * pu * pu;
  double* X = G + (size_t)pu * pu;
  double* S1 = X + (size_t)pu * pu;
  double* G2 = S1 + (size_t)pu * pu;
  double* are = G2 + (size_t)pu * pu;
  double* aim = are + (size_t)pu * pu;
  double* gjw = aim + (size_t)pu * pu;  // 4 pu^2
  int* info = (int*)(gjw + 4 * (size_t)pu * pu);
  double* cond = (double*)(info + 8);
  double* Q1 = (double*)c.W2.ptr;
  // P = masked first pu columns of T
  const double* P;
  size_t ldp;
  if (wide_t) {
    const size_t nbz = std::min<size_t>((n + 3) / 4, 8192);
    hipLaunchKernelGGL((k_zero_masked_rows<TT>), dim3((unsigned)nbz), dim3(64, 4), 0, st, n, p, op->mask,
                       (TT*)c.T.ptr);
    P = (const double*)c.T.ptr;
    ldp = (size_t)p;
  } else {
    hipLaunchKernelGGL((k_mask_cols<TT>), dim3(ew_grid(n * pu)), dim3(256), 0, st, n, p, pu, (const TT*)c.T.ptr,
                       op->mask, (double*)c.W1.ptr);
    P = (const double*)c.W1.ptr;
    ldp = (size_t)pu;
  }
  // pass 1: G = P^T P, Cholesky with dropping -> S1 (pu x r)
  gram(n, pu, P, ldp, P, ldp, nullptr, part, G, st);
  const double tau = op->dt == HELM_C128 ? 1e-7 : 1e-5;
  chol_drop(pu, G, tau * tau, 1, X, S1, info, st);
  hipError_t e = hipMemcpyAsync(op->host, info, 2 * sizeof(int), hipMemcpyDeviceToHost, st);
  if (e != hipSuccess) return hip_fail(e, "coarse: rank readback");
  if ((s = sync_stream(st, "coarse: pass 1"))) return s;
  const int r = ((int*)op->host)[0];
  c.rank = r;
  c.p_used = pu;
  if (r == 0) {
    c.valid = true;
    c.cond_est = 0.0;
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    return HELM_OK;
  }
  if ((s = c.Q.ensure(n * (size_t)r * (c.q_f32 ? sizeof(float) : sizeof(double)))) ||
      (s = c.W1.ensure(n * (size_t)r * sizeof(double))) || (s = c.Ac.ensure(2 * sizeof(double) * r * r)) ||
      (s = c.Ainv.ensure(2 * sizeof(double) * r * r)) ||
      (s = c.qpart.ensure(sizeof(double) * 2 * (size_t)r * std::max(qt_nblocks(n), qt_nblocks32(n)))))
    return s;
  // the Galerkin matrix X^T A X = X^T B - i X^T diag(Im s) X of an n x r basis
  // X into out (complex r x r); B = (L - diag(Re s)) X and then Im s go
  // through the n x r buffer B
  auto galerkin = [&](const double* X, double* B, double* out) {
    size_t nbl = (n + 3) / 4;
    if (nbl > 16384) nbl = 16384;
    hipLaunchKernelGGL((k_batched_lap<S>), dim3((unsigned)nbl), dim3(64, 4), 0, st, op->geom, r, X,
                       (const cplx_t<S>*)op->sc, op->code, B);
    gram(n, r, X, r, B, r, nullptr, part, are, st);
    hipLaunchKernelGGL((k_im_s<S>), dim3(ew_grid(n)), dim3(256), 0, st, n, (const cplx_t<S>*)op->sc, B);
    gram(n, r, X, r, X, r, B, part, aim, st);
    hipLaunchKernelGGL(k_combine_ac, dim3((r * r + 255) / 256), dim3(256), 0, st, r * r, are, aim, out);
  };
  double* Ac = (double*)c.Ac.ptr;
  if (c.pass1) {
    // fp64 basis: the solves use Q1 = P S1 itself.  The correction
    // Q (Q^T A Q)^{-1} Q^T depends only on the span of the basis, and Q1 spans
    // what Q = Q1 S2 spans (Q1^T Q1 = I up to about cond(P)^2 eps <= 1e-2 at
    // the drop threshold, so Q1^T A Q1 is as well conditioned as A_c); the
    // second pass is run only when the orthonormal basis is inspected.
    gemm<double>((int)n, r, pu, P, ldp, S1, r, nullptr, ACT_NONE, (double*)c.Q.ptr, r, st);
    galerkin((const double*)c.Q.ptr, (double*)c.W1.ptr, Ac);
  } else {
    // fp32 stored basis (when requested, or for C64): CholeskyQR2, Q rounded
    // to its stored values, A_c formed from the rounded basis.  Pass 2:
    // G2 = Q1^T Q1, Cholesky without dropping -> S2 (r x r, into S1); its rank
    // record goes to info[2..3], read back with the inverse's record (every
    // kernel below is sized by r alone, so a lost rank only spoils values).
    gemm<double>((int)n, r, pu, P, ldp, S1, r, nullptr, ACT_NONE, Q1, r, st);
    gram(n, r, Q1, r, Q1, r, nullptr, part, G2, st);
    chol_drop(r, G2, 0.0, 0, X, S1, info + 2, st);
    double* Q = (double*)c.W1.ptr;
    gemm<double>((int)n, r, r, Q1, r, S1, r, nullptr, ACT_NONE, Q, r, st);
    // Q <- its stored values (rounded in place), then B in Q1
    hipLaunchKernelGGL((k_round_q<float>), dim3(ew_grid(n * r)), dim3(256), 0, st, n * (size_t)r, Q, (float*)c.Q.ptr);
    galerkin(Q, Q1, Ac);
  }
  gj_inverse(r, Ac, nullptr, (double*)c.Ainv.ptr, info, cond, st);
  // the inverse's record goes to its own pinned slot; with defer set the
  // space is returned pending and the record is checked by coarse_finish
  // (a caller that waits on later work in the stream finds it complete)
  e = hipMemcpyAsync(op->host + COARSE_REC, info, sizeof(int) * 8 + sizeof(double), hipMemcpyDeviceToHost, st);
  if (e != hipSuccess) return hip_fail(e, "coarse: inverse readback");
  (void)hipEventRecord(e1, st);
  c.ev0 = e0;
  c.ev1 = e1;
  c.pending = true;
  c.valid = true;
  if ((s = launch_check("coarse setup"))) return s;
  return defer ? HELM_OK : coarse_finish(op);
}

helm_status coarse_ensure(helm_op_s* op, don_s* net, int p_used, bool q_fp32, bool no_drop, hipStream_t st,
                          bool defer) {
  Coarse& c = op->coarse;
  helm_status s0 = coarse_finish(op);  // a space left pending by an earlier call
  if (s0) return s0;
  const bool want_f32 = q_fp32 || op->dt == HELM_C64;
  if (!(c.valid && c.net_serial == don_serial(net) && c.p_used == p_used && c.ksq_version == op->ksq_version &&
        c.q_f32 == want_f32)) {
    c.valid = false;
    helm_status s = op->dt == HELM_C128 ? coarse_build<double, double>(op, net, p_used, q_fp32, defer, st)
                                        : coarse_build<float, float>(op, net, p_used, true, defer, st);
    if (s) return s;
    c.net_serial = don_serial(net);
    c.ksq_version = op->ksq_version;
  }
  // the space stays cached either way: a later call that allows dropping uses it
  if (no_drop && c.rank < p_used)
    return fail(HELM_E_SINGULAR, "coarse: %d of the %d trunk columns are numerically dependent and no_drop is set",
                p_used - c.rank, p_used);
  return HELM_OK;
}

helm_status coarse_orthonormal(helm_op_s* op, double* Qout, double* Acout, hipStream_t st) {
  Coarse& c = op->coarse;
  if (!c.valid || !c.pass1) return fail(HELM_E_INVAL, "coarse: no first-pass basis to orthonormalize");
  const size_t n = op->nn;
  const int r = c.rank, pu = c.p_used;
  if (r == 0) return HELM_OK;
  // the regions of the set-up's small buffer (laid out as in coarse_build)
  double* part = (double*)c.small.ptr;
  double* G = part + (size_t)gram_nblocks(n) * pu * pu;
  double* X = G + (size_t)pu * pu;
  double* S2 = X + (size_t)pu * pu;
  double* G2 = S2 + (size_t)pu * pu;
  double* gjw = G2 + 3 * (size_t)pu * pu;
  int* info = (int*)(gjw + 4 * (size_t)pu * pu);
  const double* Q1 = (const double*)c.Q.ptr;
  // second CholeskyQR pass: G2 = Q1^T Q1 = S2^-T S2^-1
  gram(n, r, Q1, r, Q1, r, nullptr, part, G2, st);
  chol_drop(r, G2, 0.0, 0, X, S2, info + 2, st);
  if (Qout) gemm<double>((int)n, r, r, Q1, r, S2, r, nullptr, ACT_NONE, Qout, r, st);
  hipError_t e;
  if (Acout) {
    // A_c = Q^T A Q = S2^T (Q1^T A Q1) S2, formed in the work region, copied out
    hipLaunchKernelGGL(k_sandwich, dim3(r), dim3(128), 0, st, r, (const double*)S2, (const double*)c.Ac.ptr, gjw);
    e = hipMemcpyAsync(Acout, gjw, sizeof(double) * 2 * r * r, hipMemcpyDeviceToHost, st);
    if (e != hipSuccess) return hip_fail(e, "coarse: A_c readback");
  }
  e = hipMemcpyAsync(op->host, info + 2, 2 * sizeof(int), hipMemcpyDeviceToHost, st);
  if (e != hipSuccess) return hip_fail(e, "coarse: second pass readback");
  helm_status s = sync_stream(st, "coarse: second pass");
  if (s) return s;
  const int* rec = (const int*)op->host;
  if (rec[1] != 0 || rec[0] != r)
    return fail(HELM_E_SINGULAR, "coarse: second CholeskyQR pass lost rank (%d of %d)", rec[0], r);
  return launch_check("coarse: orthonormal basis");
}

template <typename S>
helm_status coarse_correct(helm_op_s* op, const void* r1, void* z, hipStream_t st) {
  Coarse& c = op->coarse;
  const int r = c.rank;
  if (r == 0) return HELM_OK;
  const size_t n = op->nn;
  double* part = (double*)c.qpart.ptr;
  double* y = op->red + 1024;
  double* cc = op->red + 2048;
  const int nb = c.q_f32 ? qt_partials<float, S>(n, r, (const float*)c.Q.ptr, r1, part, st)
                         : qt_partials<double, S>(n, r, (const double*)c.Q.ptr, r1, part, st);
  reduce_cols(part, nb, 2 * r, y, st);
  hipLaunchKernelGGL(k_ainv, dim3(r), dim3(64), 0, st, r, (const double*)c.Ainv.ptr, y, cc);
  if (c.q_f32) skinny_apply<float, S>(n, r, (const float*)c.Q.ptr, cc, z, op->mask, nullptr, 0, st);
  else skinny_apply<double, S>(n, r, (const double*)c.Q.ptr, cc, z, op->mask, nullptr, 0, st);
  return launch_check("coarse correction");
}

template helm_status coarse_correct<double>(helm_op_s*, const void*, void*, hipStream_t);
template helm_status coarse_correct<float>(helm_op_s*, const void*, void*, hipStream_t);

}  // namespace helm
