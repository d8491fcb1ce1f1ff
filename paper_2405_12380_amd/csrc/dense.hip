// Dense kernels: the DeepONet layers (MFMA GEMM with fused bias + activation,
// split-K GEMV for small batches, the coordinate input layer of the trunk),
// the tall-skinny Gram products of the trunk-basis setup (MFMA), and
// one-workgroup factorizations of small matrices (Cholesky with column
// dropping, triangular inverse, Gauss-Jordan inverse of the complex coarse
// matrix).
//
// MFMA: v_mfma_f64_16x16x4f64.  Lane l supplies A[l % 16][l / 16] and
// B[l / 16][l % 16] of a 16x4 by 4x16 product; its four accumulator registers
// hold rows (l / 16) + 4 i of column l % 16.  Both dtypes evaluate the network
// layers in fp64 (a C64 network's fp32 weights widened exactly).
#include "common.h"
#include "dense.h"
#include "prof.h"

namespace helm {

typedef double d4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ d4 mfma16(double a, double b, d4 c) {
  return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}
__device__ __forceinline__ int acc_row(int lane, int i) { return (lane >> 4) + 4 * i; }

// tanh for the fp64 layers from expm1: t = e^{2|x|} - 1, tanh|x| = t / (t + 2),
// sign restored (no cancellation near 0; within 5e-16 of the library tanh and
// about 3x cheaper per element, which matters in the trunk GEMM epilogue)
__device__ __forceinline__ double tanh_fast(double x) {
  const double t = expm1(2.0 * fabs(x));
  return copysign(t / (t + 2.0), x);
}

template <typename T>
__device__ __forceinline__ T activate(T x, int act) {
  if (act == ACT_TANH) return tanh_fast(x);
  if (act == ACT_RELU) return x > T(0) ? x : T(0);
  if (act == ACT_LEAKY) return x > T(0) ? x : T(0.01) * x;
  return x;
}

// ---- trunk input layer: h = act(x W + b) at grid-node coordinates --------------
// Workgroup b takes rows [b rpb, (b + 1) rpb) of the output, threads its
// columns (W and b of a column loaded once); the node indices of the first
// row come from one division, the next rows by stepping x, then y, then z.
constexpr int CL_TAB = 1024;  // node coordinates tabulated in LDS per axis up to this length
template <typename T, bool TABBED>
__global__ __launch_bounds__(256) void k_coord_layer(int dim, int nx, int ny, int nz, size_t row0, size_t nrows,
                                                     size_t rpb, const T* __restrict__ W, const T* __restrict__ b,
                                                     int N, int act, T* __restrict__ out) {
  // TABBED: coordinate x_i = (i + 1) / (n + 1) of each axis formed once per
  // workgroup (the same quotients every element would form)
  __shared__ T tab[3][TABBED ? CL_TAB : 1];
  constexpr bool tabbed = TABBED;
  if (tabbed) {
    for (int i = threadIdx.x; i < nx; i += blockDim.x) tab[0][i] = T(i + 1) / T(nx + 1);
    for (int i = threadIdx.x; i < ny; i += blockDim.x) tab[1][i] = T(i + 1) / T(ny + 1);
    for (int i = threadIdx.x; i < nz; i += blockDim.x) tab[2][i] = T(i + 1) / T(nz + 1);
    __syncthreads();
  }
  const size_t r0 = (size_t)blockIdx.x * rpb, r1 = min(nrows, r0 + rpb);
  if (r0 >= r1) return;
  const size_t p0 = row0 + r0;
  int ix = (int)(p0 % nx), iy = (int)((p0 / nx) % ny), iz = (int)(p0 / ((size_t)nx * ny));
  for (int c0 = 0; c0 < N; c0 += blockDim.x) {
    const int c = c0 + threadIdx.x;
    const bool on = c < N;
    const T w0 = on ? W[c] : T(0), w1 = on && dim > 1 ? W[(size_t)N + c] : T(0),
            w2 = on && dim > 2 ? W[2 * (size_t)N + c] : T(0), bc = on ? b[c] : T(0);
    int jx = ix, jy = iy, jz = iz;
    for (size_t r = r0; r < r1; ++r) {
      if (on) {
        const T xc[3] = {tabbed ? tab[0][jx] : T(jx + 1) / T(nx + 1), tabbed ? tab[1][jy] : T(jy + 1) / T(ny + 1),
                         tabbed ? tab[2][jz] : T(jz + 1) / T(nz + 1)};
        T acc = xc[0] * w0;
        if (dim > 1) acc += xc[1] * w1;
        if (dim > 2) acc += xc[2] * w2;
        out[r * (size_t)N + c] = activate<T>(acc + bc, act);
      }
      if (++jx == nx) {
        jx = 0;
        if (++jy == ny) {
          jy = 0;
          ++jz;
        }
      }
    }
  }
}

// ---- MFMA GEMM: C = act(A W + b) ---------------------------------------------
// A: M x K (lda), W: K x N (ldw), C: M x N (ldc), all row-major.  128 x 128 tile
// per workgroup of four wavefronts, each 64 x 64 (4 x 4 MFMA tiles, so every
// operand value read from LDS feeds four products); K staged 16 at a time
// through LDS (A stored k-major) with the next chunk's loads in registers while
// the current chunk is multiplied.  Products are accumulated in k order, four
// at a time.
constexpr int GB_M = 128, GB_N = 128, GB_K = 16, GB_PAD = 4;

template <typename T>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(2))) void k_gemm(int M, int N, int K, const T* __restrict__ A, size_t lda,
                                              const T* __restrict__ W, size_t ldw, const T* __restrict__ bias,
                                              int act, T* __restrict__ C, size_t ldc) {
  __shared__ T As[GB_K][GB_M + GB_PAD];
  __shared__ T Ws[GB_K][GB_N + GB_PAD];
  const int nbn = (N + GB_N - 1) / GB_N;
  const unsigned lb = xcd_remap(blockIdx.x, gridDim.x);
  const int bm = (int)(lb / nbn) * GB_M, bn = (int)(lb % nbn) * GB_N;
  const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
  const int wm = (wave >> 1) * 64, wn = (wave & 1) * 64;
  d4 acc[4][4];
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int b = 0; b < 4; ++b) acc[a][b] = d4{0, 0, 0, 0};
  // A chunk: 128 rows x 16 k (16 consecutive threads read 16 consecutive k of a
  // row); W chunk: 16 k x 128 n (consecutive threads read consecutive n)
  T va[8], vw[8];
  auto load = [&](int k0) {
#pragma unroll
    for (int q = 0; q < 8; ++q) {
      const int e = t + 256 * q;
      const int r = e >> 4, kk = e & 15, gr = bm + r, gk = k0 + kk;
      va[q] = (gr < M && gk < K) ? A[(size_t)gr * lda + gk] : T(0);
      const int wk = e >> 7, c = e & 127, gkw = k0 + wk, gn = bn + c;
      vw[q] = (gkw < K && gn < N) ? W[(size_t)gkw * ldw + gn] : T(0);
    }
  };
  load(0);
  for (int k0 = 0; k0 < K; k0 += GB_K) {
#pragma unroll
    for (int q = 0; q < 8; ++q) {
      const int e = t + 256 * q;
      As[e & 15][e >> 4] = va[q];
      Ws[e >> 7][e & 127] = vw[q];
    }
    __syncthreads();
    if (k0 + GB_K < K) load(k0 + GB_K);
#pragma unroll
    for (int kk = 0; kk < GB_K; kk += 4) {
      T av[4], bv[4];
#pragma unroll
      for (int a = 0; a < 4; ++a) av[a] = As[kk + (lane >> 4)][wm + a * 16 + (lane & 15)];
#pragma unroll
      for (int b = 0; b < 4; ++b) bv[b] = Ws[kk + (lane >> 4)][wn + b * 16 + (lane & 15)];
#pragma unroll
      for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int b = 0; b < 4; ++b) acc[a][b] = mfma16(av[a], bv[b], acc[a][b]);
    }
    __syncthreads();
  }
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int b = 0; b < 4; ++b)
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const int gr = bm + wm + a * 16 + acc_row(lane, i);
        const int gc = bn + wn + b * 16 + (lane & 15);
        if (gr < M && gc < N) {
          T v = acc[a][b][i];
          if (bias) v += bias[gc];
          C[(size_t)gr * ldc + gc] = activate<T>(v, act);
        }
      }
}

// ---- small-batch dense layer (GEMV class), split over K ------------------------
// part[ks][b][n] = sum_{k in split ks} x[b][k] W[k][n]; then finalize adds the
// splits in order, the bias and the activation.
constexpr int SK_COLS = 64;
template <typename T>
__global__ __launch_bounds__(256) void k_small_part(int B, int N, int K, int ksplit, const T* __restrict__ x,
                                                    const T* __restrict__ W, double* __restrict__ part) {
  __shared__ double sh[4][4][SK_COLS];
  const int ncb = (N + SK_COLS - 1) / SK_COLS;
  const int cb = blockIdx.x % ncb, ks = blockIdx.x / ncb;
  const int lane = threadIdx.x & 63, grp = threadIdx.x >> 6;
  const int col = cb * SK_COLS + lane;
  const int kchunk = (K + ksplit - 1) / ksplit;
  const int kb = ks * kchunk, ke = min(K, kb + kchunk);
  double acc[4] = {0, 0, 0, 0};
  if (col < N)
    for (int k = kb + grp; k < ke; k += 4) {
      const double w = (double)W[(size_t)k * N + col];
      for (int b = 0; b < B; ++b) acc[b] += (double)x[(size_t)b * K + k] * w;
    }
  for (int b = 0; b < 4; ++b) sh[grp][b][lane] = acc[b];
  __syncthreads();
  if (grp == 0 && col < N)
    for (int b = 0; b < B; ++b)
      part[((size_t)ks * B + b) * N + col] = (sh[0][b][lane] + sh[1][b][lane]) + (sh[2][b][lane] + sh[3][b][lane]);
}

template <typename T>
__global__ void k_small_final(int B, int N, int ksplit, const double* __restrict__ part, const T* __restrict__ bias,
                              int act, T* __restrict__ y) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= B * N) return;
  const int b = e / N, n = e % N;
  double acc = 0.0;
  for (int ks = 0; ks < ksplit; ++ks) acc += part[((size_t)ks * B + b) * N + n];
  if (bias) acc += (double)bias[n];
  y[e] = (T)activate<double>(acc, act);  // fp64 arithmetic, rounded once to the stored type
}

// ---- tall-skinny weighted Gram: C = X^T diag(w) Y (X, Y: n x r, r <= 128) -------
// Each workgroup reduces a contiguous range of rows into a full 128 x 128 tile
// (four wavefronts of 64 x 64, 4 x 4 MFMA tiles each); rows are staged 16 at a
// time through LDS.  part[b] receives the block's r x r partial.  MODE:
// GRAM_XY (X^T Y), GRAM_XWY (X^T diag(w) Y), GRAM_XX (X^T X: Y is X and is
// neither loaded nor staged a second time), GRAM_XWX (X^T diag(w) X: X staged
// once, the weights applied to the second operand as it is read from LDS).
constexpr int GR_ROWS = 16;
enum { GRAM_XY = 0, GRAM_XWY = 1, GRAM_XX = 2, GRAM_XWX = 3 };
template <int MODE>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(2))) void k_gram(size_t n, int r,
                                              const double* __restrict__ X, size_t ldx,
                                              const double* __restrict__ Y, size_t ldy,
                                              const double* __restrict__ w, size_t rows_per_block,
                                              double* __restrict__ part) {
  constexpr bool SYM = MODE == GRAM_XX || MODE == GRAM_XWX, SW = MODE == GRAM_XWX;
  __shared__ double Xs[GR_ROWS][128 + 1];
  __shared__ double Ys[SYM ? 1 : GR_ROWS][128 + 1];
  __shared__ double ws[GR_ROWS];
  const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
  const int wa = (wave >> 1) * 64, wb = (wave & 1) * 64;
  const size_t i0 = (size_t)blockIdx.x * rows_per_block;
  const size_t i1 = min(n, i0 + rows_per_block);
  d4 acc[4][4];
  for (int a = 0; a < 4; ++a)
    for (int b = 0; b < 4; ++b) acc[a][b] = d4{0, 0, 0, 0};
  // 16 rows x 128 columns of X (and Y) per chunk; the next chunk's loads are in
  // flight while the current one is multiplied
  constexpr int NQ = GR_ROWS * 128 / 256;
  double xv[NQ], yv[SYM ? 1 : NQ], wv = 0.0;
  auto load = [&](size_t ib) {
    if (SW && t < GR_ROWS) wv = ib + t < i1 ? w[ib + t] : 0.0;
#pragma unroll
    for (int q = 0; q < NQ; ++q) {
      const int e = t + 256 * q, rr = e >> 7, cc = e & 127;
      const size_t gi = ib + rr;
      const bool in = gi < i1 && cc < r;
      xv[q] = in ? X[gi * ldx + cc] : 0.0;
      if (!SYM) {
        yv[q] = in ? Y[gi * ldy + cc] : 0.0;
        if (MODE == GRAM_XWY && in) yv[q] *= w[gi];
      }
    }
  };
  if (i0 < i1) load(i0);
  for (size_t ib = i0; ib < i1; ib += GR_ROWS) {
#pragma unroll
    for (int q = 0; q < NQ; ++q) {
      const int e = t + 256 * q, rr = e >> 7, cc = e & 127;
      Xs[rr][cc] = xv[q];
      if (!SYM) Ys[rr][cc] = yv[q];
    }
    if (SW && t < GR_ROWS) ws[t] = wv;
    __syncthreads();
    if (ib + GR_ROWS < i1) load(ib + GR_ROWS);
#pragma unroll
    for (int kk = 0; kk < GR_ROWS; kk += 4) {
      double av[4], bv[4];
      for (int a = 0; a < 4; ++a) av[a] = Xs[kk + (lane >> 4)][wa + a * 16 + (lane & 15)];
      for (int b = 0; b < 4; ++b)
        bv[b] = SYM ? Xs[kk + (lane >> 4)][wb + b * 16 + (lane & 15)] : Ys[kk + (lane >> 4)][wb + b * 16 + (lane & 15)];
      if (SW)
        for (int b = 0; b < 4; ++b) bv[b] *= ws[kk + (lane >> 4)];
      for (int a = 0; a < 4; ++a)
        for (int b = 0; b < 4; ++b) acc[a][b] = mfma16(av[a], bv[b], acc[a][b]);
    }
    __syncthreads();
  }
  double* out = part + (size_t)blockIdx.x * r * r;
  for (int a = 0; a < 4; ++a)
    for (int b = 0; b < 4; ++b)
      for (int i = 0; i < 4; ++i) {
        const int ra = wa + a * 16 + acc_row(lane, i);
        const int cb = wb + b * 16 + (lane & 15);
        if (ra < r && cb < r) out[(size_t)ra * r + cb] = acc[a][b][i];
      }
}

// out[w] = sum_b part[b * width + w] in block order (one thread per w).
__global__ void k_reduce_rows(const double* __restrict__ part, int nparts, size_t width, double* __restrict__ out,
                              double scale) {
  const size_t w = blockIdx.x * (size_t)blockDim.x + threadIdx.x;
  if (w >= width) return;
  double acc = 0.0;
  for (int b0 = 0; b0 < nparts; b0 += 8) {  // eight partials' loads in flight, added in order
    double v[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) v[u] = b0 + u < nparts ? part[(size_t)(b0 + u) * width + w] : 0.0;
#pragma unroll
    for (int u = 0; u < 8; ++u) acc += v[u];
  }
  out[w] = scale * acc;
}

// ---- one-workgroup Cholesky with column dropping -------------------------------
// G: p x p (row-major, fp64) = P^T P, p <= 128, factored in registers (16
// entries per thread) and then kept in LDS for the triangular inverse (128 KiB
// at p = 128; gfx950 gives a workgroup up to 160 KiB).  Right-looking Cholesky
// G = R^T R on the upper triangle; a column whose Schur-complement diagonal is
// <= tau2 * max_j G[j][j] is dropped (its remaining norm is at most tau times
// the largest column norm), which matches Householder QR that skips such
// columns.  R1^{-1} (kept rows/columns) is then formed in the free strictly
// lower triangle (transposed) plus a diagonal array, one thread per column.
// Outputs: S (p x r row-major) with S[kept[a]][:] = (R1^{-1})[a][:] and zero
// rows for dropped columns, so that Q = P S has orthonormal columns in exact
// arithmetic; info[0] = r; info[1] = 1 if a column had to be dropped while
// allow_drop = 0.
__global__ __launch_bounds__(1024) void k_chol_drop(int p, const double* __restrict__ Gin, double tau2, int allow_drop,
                                                    double* __restrict__ S, int* __restrict__ info) {
  extern __shared__ double G[];  // p x p
  __shared__ double xdiag[128];
  __shared__ double rowj[2][128];  // row j of the factorization step, double-buffered
  __shared__ int kept[128];
  __shared__ int s_fail;
  __shared__ double s_thr2;
  const int t = threadIdx.x, nt = blockDim.x;
  for (int e0 = 0; e0 < p * p; e0 += 4 * nt) {  // four loads in flight per thread
    double v[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) v[u] = e0 + t + u * nt < p * p ? Gin[e0 + t + u * nt] : 0.0;
#pragma unroll
    for (int u = 0; u < 4; ++u)
      if (e0 + t + u * nt < p * p) G[e0 + t + u * nt] = v[u];
  }
  __syncthreads();
  if (t == 0) {
    s_fail = 0;
    double mx = 0.0;  // largest squared column norm of P
    for (int j = 0; j < p; ++j) mx = fmax(mx, G[j * p + j]);
    s_thr2 = tau2 * mx;
  }
  __syncthreads();
  const double thr2 = s_thr2;
  // The matrix lives in registers during the factorization: thread (ty, tx) of
  // a 32 x 32 grid holds G[ty + 32 u][tx + 32 v], u, v < 4.  Step j: the
  // holders of row j (final after step j - 1) publish it unscaled in LDS
  // (double-buffered, so one barrier per step), every thread takes the drop
  // decision of column j itself from G[j][j] and updates its entries of the
  // trailing upper triangle with R[j][a] R[j][c], R[j][c] = G[j][c] / piv
  // formed as G[j][c] times the pivot's reciprocal; the holders of row j scale
  // it in their registers.
  const int ty = t >> 5, tx = t & 31;
  double g[4][4];
#pragma unroll
  for (int u = 0; u < 4; ++u)
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int a = ty + 32 * u, c = tx + 32 * v;
      g[u][v] = (a < p && c < p) ? G[a * p + c] : 0.0;
    }
  int nk = 0;
  for (int j = 0; j < p; ++j) {
    const int uj = j >> 5, buf = j & 1;
    if (ty == (j & 31))
#pragma unroll
      for (int u = 0; u < 4; ++u)
        if (u == uj)
#pragma unroll
          for (int v = 0; v < 4; ++v) {
            const int c = tx + 32 * v;
            if (c < p) rowj[buf][c] = g[u][v];
          }
    __syncthreads();
    const double dj = rowj[buf][j];
    const bool keep = dj > thr2;
    const double piv = keep ? sqrt(dj) : -1.0;
    if (t == 0) {
      if (keep) kept[nk] = j;
      else if (!allow_drop) s_fail = 1;
    }
    if (keep) {
      ++nk;
      const double pinv = 1.0 / piv;
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const int a = ty + 32 * u;
        if (a > j && a < p) {
          const double ra = rowj[buf][a] * pinv;
#pragma unroll
          for (int v = 0; v < 4; ++v) {
            const int c = tx + 32 * v;
            if (c >= a && c < p) g[u][v] -= ra * (rowj[buf][c] * pinv);
          }
        } else if (a == j) {
#pragma unroll
          for (int v = 0; v < 4; ++v) {
            const int c = tx + 32 * v;
            if (c >= j && c < p) g[u][v] = (c == j) ? piv : g[u][v] * pinv;
          }
        }
      }
    }
  }
#pragma unroll
  for (int u = 0; u < 4; ++u)
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int a = ty + 32 * u, c = tx + 32 * v;
      if (a < p && c < p) G[a * p + c] = g[u][v];
    }
  __syncthreads();
  const int r = nk;
  // X = R1^{-1}, R1[a][b] = G[kept[a]][kept[b]] (a <= b).  X[a][b] (a < b) is kept
  // at G[kept[b]][kept[a]] (strictly lower, unused by R), X[a][a] in xdiag.
  // Rows a = r-1 .. 0 in turn; column b of row a is formed by the 8 threads
  // 8b .. 8b+7, which split the sum over c and combine it with three shuffles.
  // Column b only reads its own earlier entries, written by the same 8 threads
  // of one wavefront, so the steps are ordered within the wavefront alone.
  {
    const int b = t >> 3, sub = t & 7;
    const bool colb = b < r && (t >> 3) < (nt >> 3);
    const bool full = r == p;  // no column dropped: kept[c] = c, direct addressing
    for (int a = r - 1; a >= 0; --a) {
      double acc = 0.0;
      if (colb && b >= a && full) {
#pragma unroll 4
        for (int c = a + 1 + sub; c < b; c += 8) acc += G[a * p + c] * G[b * p + c];
        if (((b - a - 1) & 7) == sub && b > a) acc += G[a * p + b] * xdiag[b];
      } else if (colb && b >= a)
        for (int c = a + 1 + sub; c <= b; c += 8) {
          const double xcb = (c == b) ? xdiag[b] : G[kept[b] * p + kept[c]];
          acc += G[kept[a] * p + kept[c]] * xcb;
        }
      acc += __shfl_xor(acc, 4, 64);
      acc += __shfl_xor(acc, 2, 64);
      acc += __shfl_xor(acc, 1, 64);
      if (colb && b >= a && sub == 0) {
        const double v = ((a == b ? 1.0 : 0.0) - acc) / G[kept[a] * p + kept[a]];
        if (a == b) xdiag[b] = v;
        else G[kept[b] * p + kept[a]] = v;
      }
      __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
      __builtin_amdgcn_wave_barrier();
    }
  }
  __syncthreads();
  for (int e = t; e < p * r; e += nt) S[e] = 0.0;
  __syncthreads();
  for (int e = t; e < r * r; e += nt) {
    const int a = e / r, b = e % r;
    double v = 0.0;
    if (a == b) v = xdiag[a];
    else if (a < b) v = G[kept[b] * p + kept[a]];
    S[(size_t)kept[a] * r + b] = v;
  }
  if (t == 0) {
    info[0] = r;
    info[1] = s_fail;
  }
}

// ---- Gauss-Jordan inverse of a complex r x r matrix (r <= 128), one workgroup ----
// The matrix lives in registers: thread t owns row t / 8 and the 16 columns
// [16 (t % 8), 16 (t % 8) + 16), rotated by one register after every pivot
// (before pivot k, a[q] holds column 16 (t % 8) + ((q + k) & 15)), so that the
// pivot column is always a[0] of the threads that own it and every register
// index is static.  In-place Gauss-Jordan with partial pivoting
// (largest modulus among the rows not yet used as pivot rows, lowest row on
// ties), without moving rows: per pivot the column is published in LDS (and
// zeroed in the registers), every wavefront picks the pivot row p from the
// published moduli, row p is scaled and broadcast, and every other row is
// updated.  Row p of the final table is then row k of the inverse where p was
// column k's pivot row, and its column c is column p_c (the pivot row of
// column c) of the inverse.  info[0] = 1 if a pivot was zero or non-finite;
// cond[0] = ||A||_1 ||A^{-1}||_1.
__global__ __launch_bounds__(1024) void k_gj_inverse(int r, const double* __restrict__ A, double* __restrict__ Ainv,
                                                     int* __restrict__ info, double* __restrict__ cond) {
  // prow holds the pivot row with one pad entry per 16 columns: the eight
  // column blocks a wavefront reads at once then fall in different LDS banks
  __shared__ double2 pcol[2][128], prow[128 + 8];
  __shared__ double pabs[2][128], csum[128];
  __shared__ double npart[8][128];
  __shared__ int perm[128], rowof[128];
  __shared__ int s_bad;
  const int t = threadIdx.x, lane = t & 63;
  const int i = t >> 3, cb = t & 7, c0 = 16 * cb;
  const bool row_in = i < r;
  bool used = false;  // row i has been a pivot row
  double2 a[16];
#pragma unroll
  for (int q = 0; q < 16; ++q) {
    const int c = c0 + q;
    a[q] = (row_in && c < r) ? make_double2(A[2 * ((size_t)i * r + c)], A[2 * ((size_t)i * r + c) + 1]) : czero();
  }
  // column k (a[0] of its owners) into buffer k & 1 (entries, and the moduli
  // of the rows not yet pivot rows), and zeroed in the registers: the update
  // of column k then leaves -f / pivot there
  auto publish = [&](int k) {
    if (cb == (k >> 4)) {
      const double2 v = a[0];
      a[0] = czero();
      if (row_in) {
        pcol[k & 1][i] = v;
        pabs[k & 1][i] = used ? -1.0 : hypot(v.x, v.y);
      }
    }
  };
  publish(0);
  // ||A||_1: column sums, column t % 128 over rows t / 128 + 8 u (coalesced), the
  // eight partials added in order
  {
    const int c = t & 127, r0 = t >> 7;
    double sm = 0.0;
    if (c < r)
      for (int ii = r0; ii < r; ii += 8) sm += hypot(A[2 * ((size_t)ii * r + c)], A[2 * ((size_t)ii * r + c) + 1]);
    npart[r0][c] = sm;
  }
  if (t == 0) s_bad = 0;
  if (t < 128) rowof[t] = t;  // every row maps in range even if a failed pivot search repeats a row
  __syncthreads();
  if (t < 128) {
    double sm = 0.0;
    for (int q = 0; q < 8; ++q) sm += npart[q][t];
    csum[t] = sm;
  }
  // Per pivot: two barriers.  Every wavefront finds the pivot itself from the
  // published moduli (same data, same order, same result), and the update for
  // column k publishes column k + 1 into the other buffer.
  for (int k = 0; k < r; ++k) {
    const int buf = k & 1;
    double best = -2.0;
    int bi = 0;
    for (int ii = lane; ii < r; ii += 64)
      if (pabs[buf][ii] > best) {
        best = pabs[buf][ii];
        bi = ii;
      }
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
      const double ob = __shfl_xor(best, off, 64);
      const int oi = __shfl_xor(bi, off, 64);
      if (ob > best || (ob == best && oi < bi)) {
        best = ob;
        bi = oi;
      }
    }
    const int p = bi;
    if (t == 0) {
      perm[k] = p;
      rowof[p] = k;
      if (!(best > 0.0) || !isfinite(best)) s_bad = 1;
    }
    // pivot row p: entry k <- 1, row *= 1 / pivot; publish it
    if (i == p) {
      used = true;
      const double2 ipiv = cdiv(make_double2(1.0, 0.0), pcol[buf][p]);
      const bool ownk = cb == (k >> 4);
#pragma unroll
      for (int q = 0; q < 16; ++q) {
        const double2 v = (q == 0 && ownk) ? make_double2(1.0, 0.0) : a[q];
        a[q] = cmul(v, ipiv);
        prow[c0 + q + cb] = a[q];  // slot (cb, q) holds the same column for every thread
      }
    }
    __syncthreads();
    // every other row: A[i][:] <- A[i][:] - f A[p][:] (A[i][k] is 0 here), two
    // fused multiply-adds per component
    if (i != p && row_in) {
      const double2 f = pcol[buf][i];
#pragma unroll
      for (int q = 0; q < 16; ++q) {
        const double2 pv = prow[c0 + q + cb];
        a[q].x = fma(-f.x, pv.x, fma(f.y, pv.y, a[q].x));
        a[q].y = fma(-f.x, pv.y, fma(-f.y, pv.x, a[q].y));
      }
    }
    // rotate: a[q] <- a[q + 1], so a[0] holds column 16 cb + ((k + 1) & 15)
    {
      const double2 a0 = a[0];
#pragma unroll
      for (int q = 0; q < 15; ++q) a[q] = a[q + 1];
      a[15] = a0;
    }
    if (k + 1 < r) publish(k + 1);
    __syncthreads();
  }
  // row i of the table is row rowof[i] of the inverse; its column c is column
  // perm[c]; after r rotations a[q] holds column 16 cb + ((q + r) & 15)
  if (row_in) {
    const int to_row = rowof[i];
#pragma unroll
    for (int q = 0; q < 16; ++q) {
      const int c = c0 + ((q + r) & 15);
      if (c < r) {
        const int to = perm[c];
        Ainv[2 * ((size_t)to_row * r + to)] = a[q].x;
        Ainv[2 * ((size_t)to_row * r + to) + 1] = a[q].y;
      }
    }
  }
  __syncthreads();
  {
    const int c = t & 127, r0 = t >> 7;
    double sm = 0.0;
    if (c < r)
      for (int ii = r0; ii < r; ii += 8)
        sm += hypot(Ainv[2 * ((size_t)ii * r + c)], Ainv[2 * ((size_t)ii * r + c) + 1]);
    npart[r0][c] = sm;
  }
  __syncthreads();
  if (t < 128) {
    double sm = 0.0;
    for (int q = 0; q < 8; ++q) sm += npart[q][t];
    pabs[0][t] = sm;
  }
  __syncthreads();
  if (t == 0) {
    double na = 0.0, ni = 0.0;
    for (int c = 0; c < r; ++c) {
      na = fmax(na, csum[c]);
      ni = fmax(ni, pabs[0][c]);
    }
    cond[0] = na * ni;
    info[0] = s_bad;
  }
}

// ---- launchers -------------------------------------------------------------------
template <typename T>
void coord_layer(int dim, const int n[3], size_t row0, size_t nrows, const T* W, const T* b, int N, int act, T* out,
                 hipStream_t st) {
  // about 4096 workgroups of at least 16 rows each
  size_t rpb = (nrows + 4095) / 4096;
  if (rpb < 16) rpb = 16;
  const size_t nb = (nrows + rpb - 1) / rpb;
  if (nb == 0) return;
  const int ny = dim > 1 ? n[1] : 1, nz = dim > 2 ? n[2] : 1;  // absent axes have one node
  if (n[0] <= CL_TAB && ny <= CL_TAB && nz <= CL_TAB)
    hipLaunchKernelGGL((k_coord_layer<T, true>), dim3((unsigned)nb), dim3(256), 0, st, dim, n[0], ny, nz, row0, nrows,
                       rpb, W, b, N, act, out);
  else
    hipLaunchKernelGGL((k_coord_layer<T, false>), dim3((unsigned)nb), dim3(256), 0, st, dim, n[0], ny, nz, row0, nrows,
                       rpb, W, b, N, act, out);
}

template <typename T>
void gemm(int M, int N, int K, const T* A, size_t lda, const T* W, size_t ldw, const T* bias, int act, T* C,
          size_t ldc, hipStream_t st) {
  kprof_begin(KP_MFMA, st);
  const int nb = ((M + GB_M - 1) / GB_M) * ((N + GB_N - 1) / GB_N);
  hipLaunchKernelGGL((k_gemm<T>), dim3(nb), dim3(256), 0, st, M, N, K, A, lda, W, ldw, bias, act, C, ldc);
  kprof_end(KP_MFMA, 2.0 * M * N * K, st);
}

int small_ksplit(int K) {
  int ks = (K + 255) / 256;
  if (ks > 64) ks = 64;
  if (ks < 1) ks = 1;
  return ks;
}

template <typename T>
void dense_small(int B, int N, int K, const T* x, const T* W, const T* bias, int act, T* y, double* part,
                 hipStream_t st) {
  const int ks = small_ksplit(K);
  const int ncb = (N + SK_COLS - 1) / SK_COLS;
  hipLaunchKernelGGL((k_small_part<T>), dim3(ncb * ks), dim3(256), 0, st, B, N, K, ks, x, W, part);
  hipLaunchKernelGGL((k_small_final<T>), dim3((B * N + 255) / 256), dim3(256), 0, st, B, N, ks, part, bias, act, y);
}

int gram_nblocks(size_t n) {
  // two workgroups per CU (the MFMA pipe needs two wavefronts per SIMD)
  size_t nb = (n + 511) / 512;
  if (nb > 512) nb = 512;
  if (nb < 1) nb = 1;
  return (int)nb;
}

void gram(size_t n, int r, const double* X, size_t ldx, const double* Y, size_t ldy, const double* w, double* part,
          double* out, hipStream_t st) {
  const int nb = gram_nblocks(n);
  size_t rpb = (n + nb - 1) / nb;
  rpb = (rpb + GR_ROWS - 1) / GR_ROWS * GR_ROWS;
  kprof_begin(KP_MFMA, st);
  if (w && X == Y && ldx == ldy)
    hipLaunchKernelGGL(k_gram<GRAM_XWX>, dim3(nb), dim3(256), 0, st, n, r, X, ldx, Y, ldy, w, rpb, part);
  else if (w)
    hipLaunchKernelGGL(k_gram<GRAM_XWY>, dim3(nb), dim3(256), 0, st, n, r, X, ldx, Y, ldy, w, rpb, part);
  else if (X == Y && ldx == ldy)
    hipLaunchKernelGGL(k_gram<GRAM_XX>, dim3(nb), dim3(256), 0, st, n, r, X, ldx, Y, ldy, w, rpb, part);
  else
    hipLaunchKernelGGL(k_gram<GRAM_XY>, dim3(nb), dim3(256), 0, st, n, r, X, ldx, Y, ldy, w, rpb, part);
  kprof_end(KP_MFMA, 2.0 * (double)n * r * r, st);
  const size_t width = (size_t)r * r;
  hipLaunchKernelGGL(k_reduce_rows, dim3((unsigned)((width + 255) / 256)), dim3(256), 0, st, part, nb, width, out,
                     1.0);
}

void reduce_rows(const double* part, int nparts, size_t width, double* out, double scale, hipStream_t st) {
  hipLaunchKernelGGL(k_reduce_rows, dim3((unsigned)((width + 255) / 256)), dim3(256), 0, st, part, nparts, width, out,
                     scale);
}

void chol_drop(int p, double* G, double tau2, int allow_drop, double* X, double* S, int* info, hipStream_t st) {
  (void)X;
  const size_t lds = sizeof(double) * (size_t)p * p;
  static bool attr_set = false;
  if (!attr_set) {
    // G staged in LDS: up to 128 KiB at p = 128 (a gfx950 workgroup may use 160 KiB)
    (void)hipFuncSetAttribute((const void*)k_chol_drop, hipFuncAttributeMaxDynamicSharedMemorySize, 128 * 128 * 8);
    attr_set = true;
  }
  hipLaunchKernelGGL(k_chol_drop, dim3(1), dim3(1024), lds, st, p, G, tau2, allow_drop, S, info);
}

void gj_inverse(int r, const double* A, double* work, double* Ainv, int* info, double* cond, hipStream_t st) {
  (void)work;
  hipLaunchKernelGGL(k_gj_inverse, dim3(1), dim3(1024), 0, st, r, A, Ainv, info, cond);
}

template void coord_layer<double>(int, const int*, size_t, size_t, const double*, const double*, int, int, double*,
                                  hipStream_t);
template void gemm<double>(int, int, int, const double*, size_t, const double*, size_t, const double*, int, double*,
                           size_t, hipStream_t);
template void dense_small<double>(int, int, int, const double*, const double*, const double*, int, double*, double*,
                                  hipStream_t);
template void dense_small<float>(int, int, int, const float*, const float*, const float*, int, float*, double*,
                                 hipStream_t);

}  // namespace helm
