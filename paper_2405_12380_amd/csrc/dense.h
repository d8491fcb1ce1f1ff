// Launchers of the dense kernels (DeepONet layers, Gram products, small
// one-workgroup factorizations).  All enqueue on `st` and return at once.
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>

namespace helm {

enum { ACT_NONE = -1, ACT_TANH = 0, ACT_RELU = 1, ACT_LEAKY = 2 };

// h[r][c] = act(sum_d x_{row0+r}[d] W[d][c] + b[c]) with x_p the coordinates of
// grid node p (x-fastest numbering, (i+1)/(n+1) per axis), r < nrows, c < N
// (instantiated for double)
template <typename T>
void coord_layer(int dim, const int n[3], size_t row0, size_t nrows, const T* W, const T* b, int N, int act, T* out,
                 hipStream_t st);
// C = act(A W + bias) (fp64 MFMA; instantiated for double); bias may be NULL;
// act = ACT_NONE for linear
template <typename T>
void gemm(int M, int N, int K, const T* A, size_t lda, const T* W, size_t ldw, const T* bias, int act, T* C,
          size_t ldc, hipStream_t st);
// y[b][n] = act(sum_k x[b][k] W[k][n] + bias[n]) for a batch B <= 4 (split-K,
// fp64 accumulation, bias and activation; y rounded once to T);
// part needs small_ksplit(K) * B * N doubles
int small_ksplit(int K);
template <typename T>
void dense_small(int B, int N, int K, const T* x, const T* W, const T* bias, int act, T* y, double* part,
                 hipStream_t st);
// out (r x r) = X^T diag(w) Y for X, Y of n rows (row strides ldx, ldy), r <= 128;
// part needs gram_nblocks(n) * r * r doubles; w may be NULL
int gram_nblocks(size_t n);
void gram(size_t n, int r, const double* X, size_t ldx, const double* Y, size_t ldy, const double* w, double* part,
          double* out, hipStream_t st);
void reduce_rows(const double* part, int nparts, size_t width, double* out, double scale, hipStream_t st);
// Cholesky with dropping of columns whose remaining squared norm is <= tau2 times
// the largest squared column norm; G (p x p) is overwritten; X: p*p scratch;
// S: p*p output capacity; info: 2 ints (rank, failed)
void chol_drop(int p, double* G, double tau2, int allow_drop, double* X, double* S, int* info, hipStream_t st);
// inverse of the complex r x r matrix A (interleaved); work: 4*r*r doubles;
// info: 1 int (1 = singular); cond: 1 double
void gj_inverse(int r, const double* A, double* work, double* Ainv, int* info, double* cond, hipStream_t st);

}  // namespace helm
