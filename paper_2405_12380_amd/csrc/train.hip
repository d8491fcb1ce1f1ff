// DeepONet training (App. B network): bf16 MFMA forward and backward with
// fp32 accumulation, fp32 master weights, Adam, mean relative L2 loss.
//
// One step on a batch of S samples and P trunk points:
//   branch:  H_{l+1} = tanh(H_l W_l + b_l) ..., B = H_L (S x 2p)
//   trunk:   the same on the padded coordinates, T (P x p)
//   output:  Ut = Bc T^T (2S x P) with Bc = [B[:, :p]; B[:, p:]] (Re rows, then Im rows)
//   loss:    L = mean_s ||U_s - Y_s|| / ||Y_s||; dUt = (Ut - Y) / (S ||U_s - Y_s|| ||Y_s||)
//   back:    dT = dUt^T Bc, dBc = dUt T, then per layer dW = H^T dZ, db = colsum dZ,
//            dZ_below = (dZ W^T) * (1 - H^2)
//   Adam on the flat fp32 parameters; bf16 copies feed the next step's GEMMs.
// Every matrix product runs in one bf16 GEMM kernel (v_mfma_f32_16x16x32_bf16,
// 128 x 128 tile per 256-thread workgroup, 32-deep k steps staged in LDS, either
// operand read as stored or transposed while staging) with fused epilogues
// (bias + tanh, bias, tanh derivative, fp32) or split-k partials reduced in a
// fixed order.  A step is captured once as a HIP graph and replayed; the
// sample indices and the step counter live on the device.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstring>
#include <vector>

#include "common.h"
#include "internal.h"
#include "lib.h"

typedef __bf16 bf8 __attribute__((ext_vector_type(8)));
typedef float f4 __attribute__((ext_vector_type(4)));

struct don_trainer_s;

namespace helm {

namespace {

constexpr int TM = 128, TN = 128, TK = 32, LDSW = 40;  // tile and LDS row stride (bf16 elements, 80 B)

enum { EP_F32 = 0, EP_BF16 = 1, EP_BIAS_BF16 = 2, EP_BIAS_TANH_BF16 = 3, EP_DTANH_BF16 = 4, EP_PART = 5 };

struct GemmArgs {
  const __bf16* A;
  long lda;
  int ta;  // 0: A is M x K (k contiguous); 1: A is stored K x M
  const __bf16* B;
  long ldb;
  int tb;  // 0: B is stored N x K (k contiguous); 1: B is stored K x N
  int M, N, K, kchunk;
  void* C;
  long ldc;
  const float* bias;
  const __bf16* aux;  // EP_DTANH_BF16: the activation h (M x N, leading dimension ldc)
  int ep;
};

__device__ __forceinline__ float bf2f(__bf16 v) { return (float)v; }

// Apply an epilogue to one value of C(row, col).
__device__ __forceinline__ void ep_store(const GemmArgs& g, int row, int col, float v) {
  const long o = (long)row * g.ldc + col;
  switch (g.ep) {
    case EP_F32:
      ((float*)g.C)[o] = v;
      break;
    case EP_BF16:
      ((__bf16*)g.C)[o] = (__bf16)v;
      break;
    case EP_BIAS_BF16:
      ((__bf16*)g.C)[o] = (__bf16)(v + g.bias[col]);
      break;
    case EP_BIAS_TANH_BF16:
      ((__bf16*)g.C)[o] = (__bf16)tanhf(v + g.bias[col]);
      break;
    case EP_DTANH_BF16: {
      const float h = bf2f(g.aux[o]);
      ((__bf16*)g.C)[o] = (__bf16)(v * (1.0f - h * h));
      break;
    }
    default:  // EP_PART: split-k slice blockIdx.z of an M x N fp32 array
      ((float*)g.C)[(long)blockIdx.z * g.M * g.N + (long)row * g.N + col] = v;
  }
}

// Stage a 128-row x 32-k tile of an operand into LDS as [row][k] (k contiguous).
// trans = 0: rows of G are the tile rows (k contiguous, ld elements apart);
// trans = 1: G is stored k-major (row index = k), the tile is transposed on the way.
__device__ __forceinline__ void stage(const __bf16* __restrict__ G, long ld, int trans, int r0, int R, int k0, int K,
                                      __bf16* __restrict__ S) {
  const int t = threadIdx.x;
  bf8 z;
#pragma unroll
  for (int j = 0; j < 8; ++j) z[j] = (__bf16)0.0f;
  if (!trans) {
#pragma unroll
    for (int pass = 0; pass < 2; ++pass) {
      const int row = (t >> 2) + 64 * pass, kq = (t & 3) * 8;
      bf8 v = z;
      if (r0 + row < R && k0 + kq < K) v = *(const bf8*)(G + (long)(r0 + row) * ld + k0 + kq);
      *(bf8*)(S + row * LDSW + kq) = v;
    }
  } else {
#pragma unroll
    for (int pass = 0; pass < 2; ++pass) {
      const int kr = (t >> 4) + 16 * pass, rq = (t & 15) * 8;
      bf8 v = z;
      if (k0 + kr < K) {
        const long base = (long)(k0 + kr) * ld + r0 + rq;
        if (r0 + rq + 8 <= R) {
          v = *(const bf8*)(G + base);
        } else {
#pragma unroll
          for (int j = 0; j < 8; ++j)
            if (r0 + rq + j < R) v[j] = G[base + j];
        }
      }
#pragma unroll
      for (int j = 0; j < 8; ++j) S[(rq + j) * LDSW + kr] = v[j];
    }
  }
}

// C (M x N) = sum_k A(m, k) B(k, n) over this workgroup's k slice, epilogue g.ep.
// Wavefront w owns the 64 x 64 quadrant (w / 2, w % 2) as 4 x 4 MFMA tiles;
// lane l holds A[l % 16][8 (l / 16) .. +7], B[8 (l / 16) .. +7][l % 16] and
// C[4 (l / 16) + i][l % 16] of a 16 x 16 x 32 product.
__global__ __launch_bounds__(256) void k_gemm_bf16(GemmArgs g) {
  __shared__ __attribute__((aligned(16))) __bf16 As[TM * LDSW];
  __shared__ __attribute__((aligned(16))) __bf16 Bs[TN * LDSW];
  const int m0 = blockIdx.x * TM, n0 = blockIdx.y * TN;
  const int kb = blockIdx.z * g.kchunk;
  const int ke = min(g.K, kb + g.kchunk);
  const int w = threadIdx.x >> 6, l = threadIdx.x & 63;
  const int wm = w >> 1, wn = w & 1;
  f4 acc[4][4];
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) acc[i][j] = f4{0.f, 0.f, 0.f, 0.f};
  for (int k0 = kb; k0 < ke; k0 += TK) {
    stage(g.A, g.lda, g.ta, m0, g.M, k0, ke, As);
    stage(g.B, g.ldb, g.tb, n0, g.N, k0, ke, Bs);
    __syncthreads();
    bf8 a[4], b[4];
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      a[i] = *(const bf8*)(As + (wm * 64 + i * 16 + (l & 15)) * LDSW + 8 * (l >> 4));
      b[i] = *(const bf8*)(Bs + (wn * 64 + i * 16 + (l & 15)) * LDSW + 8 * (l >> 4));
    }
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
      for (int j = 0; j < 4; ++j) acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[i], b[j], acc[i][j], 0, 0, 0);
    __syncthreads();
  }
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j)
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int row = m0 + wm * 64 + i * 16 + 4 * (l >> 4) + q;
        const int col = n0 + wn * 64 + j * 16 + (l & 15);
        if (row < g.M && col < g.N) ep_store(g, row, col, acc[i][j][q]);
      }
}

// sum of split-k slices in a fixed order, then the epilogue
__global__ __launch_bounds__(256) void k_splitk_reduce(GemmArgs g, const float* __restrict__ part, int splits) {
  const long MN = (long)g.M * g.N;
  for (long e = blockIdx.x * 256L + threadIdx.x; e < MN; e += (long)gridDim.x * 256) {
    float v = 0.f;
    for (int z = 0; z < splits; ++z) v += part[z * MN + e];
    ep_store(g, (int)(e / g.N), (int)(e % g.N), v);
  }
}

// partial column sums of a bf16 M x N matrix (N <= 256): part[b][col]
__global__ __launch_bounds__(256) void k_colsum(const __bf16* __restrict__ D, int M, int N, int rows,
                                                float* __restrict__ part) {
  const int col = threadIdx.x;
  if (col >= N) return;
  const int r0 = blockIdx.x * rows, r1 = min(M, r0 + rows);
  float a = 0.f;
  for (int r = r0; r < r1; ++r) a += bf2f(D[(long)r * N + col]);
  part[(long)blockIdx.x * N + col] = a;
}

// fixed-order sum of nb partial rows of width N into out (optionally accumulated to a scalar)
__global__ void k_rows_sum(const float* __restrict__ part, int nb, int N, float* __restrict__ out) {
  for (int c = blockIdx.x * blockDim.x + threadIdx.x; c < N; c += gridDim.x * blockDim.x) {
    float a = 0.f;
    for (int b = 0; b < nb; ++b) a += part[(long)b * N + c];
    out[c] = a;
  }
}

// Branch inputs of the batch: rows idx[step S + s] of the dataset (bf16, padded).
__global__ __launch_bounds__(256) void k_gather(const __bf16* __restrict__ F, long ldf, const int* __restrict__ idx,
                                                const int* __restrict__ step, int S, __bf16* __restrict__ out) {
  const int s = blockIdx.y;
  const int src = idx[(long)step[0] * S + s];
  for (long c = blockIdx.x * 256L + threadIdx.x; c < ldf; c += (long)gridDim.x * 256)
    out[(long)s * ldf + c] = F[(long)src * ldf + c];
}

// Bc (2S x p): row s = B[s][0:p], row S + s = B[s][p:2p]
__global__ void k_to_bc(const __bf16* __restrict__ B, int S, int p, __bf16* __restrict__ Bc) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= 2 * S * p) return;
  const int r = e / p, c = e % p;
  Bc[e] = r < S ? B[(long)r * 2 * p + c] : B[(long)(r - S) * 2 * p + p + c];
}

// dB (S x 2p, bf16) from dBc (2S x p, fp32)
__global__ void k_from_dbc(const float* __restrict__ dBc, int S, int p, __bf16* __restrict__ dB) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= 2 * S * p) return;
  const int s = e / (2 * p), c = e % (2 * p);
  dB[e] = (__bf16)(c < p ? dBc[(long)s * p + c] : dBc[(long)(S + s) * p + (c - p)]);
}

// per (sample, chunk): ||U_s - Y_s||^2 and ||Y_s||^2 over the chunk's points (fp64)
__global__ __launch_bounds__(256) void k_loss_part(const float* __restrict__ Ut, const float2* __restrict__ Y,
                                                   const int* __restrict__ idx, const int* __restrict__ step, int S,
                                                   int P, int chunk, double* __restrict__ part) {
  __shared__ double sh[32];
  const int s = blockIdx.y;
  const long src = idx[(long)step[0] * S + s];
  const int p0 = blockIdx.x * chunk, p1 = min(P, p0 + chunk);
  double dn = 0.0, yn = 0.0;
  for (int q = p0 + threadIdx.x; q < p1; q += 256) {
    const float2 y = Y[src * P + q];
    const double dr = (double)Ut[(long)s * P + q] - y.x, di = (double)Ut[(long)(S + s) * P + q] - y.y;
    dn += dr * dr + di * di;
    yn += (double)y.x * y.x + (double)y.y * y.y;
  }
  dn = block_sum(dn, sh);
  yn = block_sum(yn, sh);
  if (threadIdx.x == 0) {
    part[((long)s * gridDim.x + blockIdx.x) * 2] = dn;
    part[((long)s * gridDim.x + blockIdx.x) * 2 + 1] = yn;
  }
}

// per-sample norms -> weights w_s = 1 / (S ||U_s - Y_s|| ||Y_s||); loss[step] = mean relative error
__global__ void k_loss_final(const double* __restrict__ part, int S, int nch, const int* __restrict__ step,
                             float* __restrict__ w, float* __restrict__ loss) {
  __shared__ double rel[256];
  const int s = threadIdx.x;
  if (s < S) {
    double dn = 0.0, yn = 0.0;
    for (int c = 0; c < nch; ++c) {
      dn += part[((long)s * nch + c) * 2];
      yn += part[((long)s * nch + c) * 2 + 1];
    }
    dn = sqrt(dn);
    yn = sqrt(yn);
    rel[s] = dn / yn;
    w[s] = (float)(dn > 0.0 ? 1.0 / (S * dn * yn) : 0.0);
  }
  __syncthreads();
  if (s == 0) {
    double a = 0.0;
    for (int i = 0; i < S; ++i) a += rel[i];
    loss[step[0]] = (float)(a / S);
  }
}

// dUt (2S x P, bf16) = (Ut - Y) w_s
__global__ __launch_bounds__(256) void k_dU(const float* __restrict__ Ut, const float2* __restrict__ Y,
                                            const int* __restrict__ idx, const int* __restrict__ step,
                                            const float* __restrict__ w, int S, int P, __bf16* __restrict__ dUt) {
  const int s = blockIdx.y;
  const long src = idx[(long)step[0] * S + s];
  const float ws = w[s];
  for (long q = blockIdx.x * 256L + threadIdx.x; q < P; q += (long)gridDim.x * 256) {
    const float2 y = Y[src * P + q];
    dUt[(long)s * P + q] = (__bf16)((Ut[(long)s * P + q] - y.x) * ws);
    dUt[(long)(S + s) * P + q] = (__bf16)((Ut[(long)(S + s) * P + q] - y.y) * ws);
  }
}

// Adam on the flat parameters (fp32), step t = tstep[0] + 1; refreshes the bf16 copies
__global__ __launch_bounds__(256) void k_adam(long n, float* __restrict__ w, const float* __restrict__ g,
                                              float* __restrict__ m, float* __restrict__ v, __bf16* __restrict__ wb,
                                              float lr, float b1, float b2, float eps, const int* __restrict__ tstep) {
  const int t = tstep[0] + 1;
  // bias corrections in fp64: 1 - b2^t in fp32 cancels about 10 bits at b2 = 0.999
  const float c1 = (float)(1.0 - pow((double)b1, (double)t)), c2 = (float)(1.0 - pow((double)b2, (double)t));
  for (long e = blockIdx.x * 256L + threadIdx.x; e < n; e += (long)gridDim.x * 256) {
    const float ge = g[e];
    const float me = b1 * m[e] + (1.0f - b1) * ge;
    const float ve = b2 * v[e] + (1.0f - b2) * ge * ge;
    m[e] = me;
    v[e] = ve;
    const float we = w[e] - lr * (me / c1) / (sqrtf(ve / c2) + eps);
    w[e] = we;
    wb[e] = (__bf16)we;
  }
}

// step index within the call; Adam's step count only when the parameters moved
__global__ void k_tick(int* __restrict__ step, int* __restrict__ tstep, int updated) {
  if (threadIdx.x == 0 && blockIdx.x == 0) {
    step[0] += 1;
    if (updated) tstep[0] += 1;
  }
}

__global__ void k_f32_to_bf16(long n, const float* __restrict__ a, __bf16* __restrict__ b) {
  for (long e = blockIdx.x * 256L + threadIdx.x; e < n; e += (long)gridDim.x * 256) b[e] = (__bf16)a[e];
}

// padded bf16 rows (ld columns) from fp32 rows (cols columns)
__global__ void k_pad_rows(long rows, int cols, const float* __restrict__ a, int ld, __bf16* __restrict__ b) {
  const long n = rows * ld;
  for (long e = blockIdx.x * 256L + threadIdx.x; e < n; e += (long)gridDim.x * 256) {
    const long r = e / ld;
    const int c = (int)(e % ld);
    b[e] = (__bf16)(c < cols ? a[r * cols + c] : 0.0f);
  }
}

template <typename R>
__global__ void k_cvt_pad(int K, int N, int Kp, const R* __restrict__ src, float* __restrict__ dst) {
  const long n = (long)Kp * N;
  for (long e = blockIdx.x * 256L + threadIdx.x; e < n; e += (long)gridDim.x * 256) {
    const int r = (int)(e / N);
    dst[e] = r < K ? (float)src[(long)r * N + (e % N)] : 0.0f;
  }
}

template <typename R>
__global__ void k_cvt_back(int K, int N, const float* __restrict__ src, R* __restrict__ dst) {
  const long n = (long)K * N;
  for (long e = blockIdx.x * 256L + threadIdx.x; e < n; e += (long)gridDim.x * 256) dst[e] = (R)src[e];
}

static unsigned grid_for(long n) {
  long b = (n + 255) / 256;
  if (b > 16384) b = 16384;
  if (b < 1) b = 1;
  return (unsigned)b;
}

static int pad32(int k) { return (k + 31) / 32 * 32; }

}  // namespace

}  // namespace helm

using namespace helm;

struct Layer {
  int K, Kp, N;       // true input width, padded, output width
  size_t offW, offb;  // offsets in the flat parameter arrays (elements)
};

struct don_trainer_s {
  int S = 0, P = 0, d = 0, p = 0;
  float lr = 1e-3f, b1 = 0.9f, b2 = 0.999f, eps = 1e-8f;
  std::vector<Layer> bl, tl;  // branch, trunk
  size_t nparam = 0;
  int max_steps = 0;
  Buffer master, grad, mom, var, wbf;  // flat fp32 / bf16 parameters
  Buffer X;                            // P x Kp trunk inputs (bf16)
  Buffer bact, tact;                   // activations: branch S x (sum of widths), trunk P x (sum of widths)
  Buffer dz0, dz1;                     // trunk backward ping-pong (P x 256 bf16)
  Buffer bdz0, bdz1;                   // branch backward ping-pong
  Buffer Bc, Ut, dUt, dBcp, dBc, dW, cs, lpart, wv, ctr, losses, idx;
  Buffer Fdata;                        // n x Kb_pad bf16
  const float2* Y = nullptr;           // n x P complex64 labels (caller's)
  int ndata = 0;
  size_t tact_off[8] = {0}, bact_off[8] = {0};
  size_t dw_slices = 0;
  hipStream_t st = nullptr;
  hipGraphExec_t step_exec = nullptr;
  ~don_trainer_s() {
    if (step_exec) (void)hipGraphExecDestroy(step_exec);
    if (st) (void)hipStreamDestroy(st);
    for (Buffer* b : {&master, &grad, &mom, &var, &wbf, &X, &bact, &tact, &dz0, &dz1, &bdz0, &bdz1, &Bc, &Ut, &dUt,
                      &dBcp, &dBc, &dW, &cs, &lpart, &wv, &ctr, &losses, &idx, &Fdata})
      b->release();
  }
};

namespace {

void gemm(hipStream_t st, const __bf16* A, long lda, int ta, const __bf16* B, long ldb, int tb, int M, int N, int K,
          void* C, long ldc, int ep, const float* bias = nullptr, const __bf16* aux = nullptr, int splits = 1,
          float* part = nullptr) {
  GemmArgs g{A, lda, ta, B, ldb, tb, M, N, K, 0, C, ldc, bias, aux, ep};
  const int kblocks = K / TK;
  if (splits > kblocks) splits = kblocks;
  if (splits < 1) splits = 1;
  const int per = (kblocks + splits - 1) / splits;
  splits = (kblocks + per - 1) / per;
  g.kchunk = per * TK;
  dim3 grid((M + TM - 1) / TM, (N + TN - 1) / TN, splits);
  if (splits == 1) {
    hipLaunchKernelGGL(k_gemm_bf16, grid, dim3(256), 0, st, g);
    return;
  }
  GemmArgs gp = g;
  gp.ep = EP_PART;
  gp.C = part;
  hipLaunchKernelGGL(k_gemm_bf16, grid, dim3(256), 0, st, gp);
  hipLaunchKernelGGL(k_splitk_reduce, dim3(grid_for((long)M * N)), dim3(256), 0, st, g, (const float*)part, splits);
}

// split count so that about `target` workgroups run (k-slices of at least 256)
int splits_for(int M, int N, int K, int target = 512) {
  const int tiles = ((M + TM - 1) / TM) * ((N + TN - 1) / TN);
  int s = target / (tiles > 0 ? tiles : 1);
  const int maxs = K / 256 > 0 ? K / 256 : 1;
  if (s > maxs) s = maxs;
  return s < 1 ? 1 : s;
}

// forward through one MLP; acts holds every layer's output (bf16), input H0 given
void mlp_fwd(don_trainer_s* t, std::vector<Layer>& L, const __bf16* H0, long ld0, int M, __bf16* acts,
             const size_t* off, float* part) {
  const __bf16* wb = (const __bf16*)t->wbf.ptr;
  const float* mw = (const float*)t->master.ptr;
  const __bf16* H = H0;
  long ld = ld0;
  for (size_t li = 0; li < L.size(); ++li) {
    const Layer& y = L[li];
    __bf16* out = acts + off[li];
    const bool last = li + 1 == L.size();
    const int sp = splits_for(M, y.N, y.Kp, 256);
    gemm(t->st, H, ld, 0, wb + y.offW, y.N, 1, M, y.N, y.Kp, out, y.N, last ? EP_BIAS_BF16 : EP_BIAS_TANH_BF16,
         mw + y.offb, nullptr, sp, part);
    H = out;
    ld = y.N;
  }
}

// backward through one MLP given dZ of its last layer (bf16, M x N_last, in dz_a)
void mlp_bwd(don_trainer_s* t, std::vector<Layer>& L, const __bf16* H0, long ld0, int M, const __bf16* acts,
             const size_t* off, __bf16* dz_a, __bf16* dz_b) {
  const __bf16* wb = (const __bf16*)t->wbf.ptr;
  float* g = (float*)t->grad.ptr;
  float* dwp = (float*)t->dW.ptr;
  float* csp = (float*)t->cs.ptr;
  __bf16* dz = dz_a;
  __bf16* other = dz_b;
  for (int li = (int)L.size() - 1; li >= 0; --li) {
    const Layer& y = L[li];
    const __bf16* Hin = li == 0 ? H0 : acts + off[li - 1];
    const long ldin = li == 0 ? ld0 : L[li - 1].N;
    // dW = H^T dZ (reduction over the M rows, split)
    int sp = (int)((size_t)M / 1024);
    if (sp < 1) sp = 1;
    const size_t cap = t->dw_slices;
    const size_t per_slice = (size_t)y.Kp * y.N;
    if ((size_t)sp * per_slice > cap) sp = (int)(cap / per_slice);
    gemm(t->st, Hin, ldin, 1, dz, y.N, 1, y.Kp, y.N, M, g + y.offW, y.N, EP_F32, nullptr, nullptr, sp, dwp);
    // db = column sums of dZ
    const int rows = 1024;
    const int nb = (M + rows - 1) / rows;
    hipLaunchKernelGGL(k_colsum, dim3(nb), dim3(256), 0, t->st, dz, M, y.N, rows, csp);
    hipLaunchKernelGGL(k_rows_sum, dim3(1), dim3(256), 0, t->st, (const float*)csp, nb, y.N, g + y.offb);
    if (li > 0) {
      // dZ_below = (dZ W^T) * (1 - H_below^2)
      const Layer& z = L[li - 1];
      gemm(t->st, dz, y.N, 0, wb + y.offW, y.N, 0, M, z.N, y.N, other, z.N, EP_DTANH_BF16, nullptr,
           acts + off[li - 1]);
      std::swap(dz, other);
    }
  }
}

void train_step(don_trainer_s* t, bool update) {
  const int S = t->S, P = t->P, p = t->p;
  const int* ctr = (const int*)t->ctr.ptr;
  const int* idx = (const int*)t->idx.ptr;
  float* part = (float*)t->dW.ptr;
  const Layer& b0 = t->bl[0];
  __bf16* bact = (__bf16*)t->bact.ptr;
  __bf16* tact = (__bf16*)t->tact.ptr;
  // branch inputs of the batch occupy the front of the branch activation buffer
  __bf16* Fb = bact;
  hipLaunchKernelGGL(k_gather, dim3(grid_for(b0.Kp) < 64 ? grid_for(b0.Kp) : 64, S), dim3(256), 0, t->st,
                     (const __bf16*)t->Fdata.ptr, (long)b0.Kp, idx, ctr, S, Fb);
  mlp_fwd(t, t->bl, Fb, b0.Kp, S, bact, t->bact_off, part);
  mlp_fwd(t, t->tl, (const __bf16*)t->X.ptr, t->tl[0].Kp, P, tact, t->tact_off, part);
  const __bf16* Bout = bact + t->bact_off[t->bl.size() - 1];
  const __bf16* T = tact + t->tact_off[t->tl.size() - 1];
  __bf16* Bc = (__bf16*)t->Bc.ptr;
  hipLaunchKernelGGL(k_to_bc, dim3((2 * S * p + 255) / 256), dim3(256), 0, t->st, Bout, S, p, Bc);
  // Ut = Bc T^T (2S x P)
  float* Ut = (float*)t->Ut.ptr;
  gemm(t->st, Bc, p, 0, T, p, 0, 2 * S, P, p, Ut, P, EP_F32);
  // loss and dUt
  const int chunk = 4096, nch = (P + chunk - 1) / chunk;
  hipLaunchKernelGGL(k_loss_part, dim3(nch, S), dim3(256), 0, t->st, (const float*)Ut, t->Y, idx, ctr, S, P, chunk,
                     (double*)t->lpart.ptr);
  hipLaunchKernelGGL(k_loss_final, dim3(1), dim3(256), 0, t->st, (const double*)t->lpart.ptr, S, nch, ctr,
                     (float*)t->wv.ptr, (float*)t->losses.ptr);
  __bf16* dUt = (__bf16*)t->dUt.ptr;
  hipLaunchKernelGGL(k_dU, dim3(64, S), dim3(256), 0, t->st, (const float*)Ut, t->Y, idx, ctr, (const float*)t->wv.ptr,
                     S, P, dUt);
  // dT = dUt^T Bc (P x p) -> dZ of the trunk's last layer; dBc = dUt T (2S x p)
  __bf16* dz0 = (__bf16*)t->dz0.ptr;
  gemm(t->st, dUt, P, 1, Bc, p, 1, P, p, 2 * S, dz0, p, EP_BF16);
  float* dBc = (float*)t->dBc.ptr;
  gemm(t->st, dUt, P, 0, T, p, 1, 2 * S, p, P, dBc, p, EP_F32, nullptr, nullptr, splits_for(2 * S, p, P, 512),
       (float*)t->dBcp.ptr);
  __bf16* bdz0 = (__bf16*)t->bdz0.ptr;
  hipLaunchKernelGGL(k_from_dbc, dim3((2 * S * p + 255) / 256), dim3(256), 0, t->st, (const float*)dBc, S, p, bdz0);
  mlp_bwd(t, t->tl, (const __bf16*)t->X.ptr, t->tl[0].Kp, P, tact, t->tact_off, dz0, (__bf16*)t->dz1.ptr);
  mlp_bwd(t, t->bl, Fb, b0.Kp, S, bact, t->bact_off, bdz0, (__bf16*)t->bdz1.ptr);
  if (update)
    hipLaunchKernelGGL(k_adam, dim3(grid_for((long)t->nparam)), dim3(256), 0, t->st, (long)t->nparam,
                       (float*)t->master.ptr, (const float*)t->grad.ptr, (float*)t->mom.ptr, (float*)t->var.ptr,
                       (__bf16*)t->wbf.ptr, t->lr, t->b1, t->b2, t->eps, ctr + 1);
  hipLaunchKernelGGL(k_tick, dim3(1), dim3(64), 0, t->st, (int*)t->ctr.ptr, (int*)t->ctr.ptr + 1, update ? 1 : 0);
}

helm_status sync(don_trainer_s* t, const char* what) { return sync_stream(t->st, what); }

}  // namespace

extern "C" {

helm_status don_train_create(don_net net, const don_train_opts* o, const double* X, don_trainer* out) {
  if (!out) return fail(HELM_E_INVAL, "don_train_create: out is NULL");
  *out = nullptr;
  if (!net || !o || !X) return fail(HELM_E_INVAL, "don_train_create: NULL argument");
  if (net->head != DON_SPLIT_OUTPUT || net->act != DON_TANH)
    return fail(HELM_E_INVAL, "don_train_create: training needs the SPLIT_OUTPUT head and tanh");
  if (o->batch < 32 || o->batch > 128 || o->batch % 32)
    return fail(HELM_E_INVAL, "don_train_create: batch %d must be 32, 64, 96 or 128", o->batch);
  if (o->n_points < 32 || o->n_points % 32)
    return fail(HELM_E_INVAL, "don_train_create: n_points must be a positive multiple of 32");
  if (o->max_steps < 1) return fail(HELM_E_INVAL, "don_train_create: max_steps < 1");
  for (size_t i = 1; i < net->bw.size(); ++i)
    if (net->bw[i] > 256 || net->bw[i] % 32)
      return fail(HELM_E_INVAL, "don_train_create: branch widths after the input must be multiples of 32, <= 256");
  for (size_t i = 1; i < net->tw.size(); ++i)
    if (net->tw[i] > 256 || net->tw[i] % 32)
      return fail(HELM_E_INVAL, "don_train_create: trunk widths after the input must be multiples of 32, <= 256");
  don_trainer_s* t = new don_trainer_s();
  t->S = o->batch;
  t->P = o->n_points;
  t->d = net->tw[0];
  t->p = net->p;
  t->lr = (float)o->lr;
  t->b1 = (float)o->beta1;
  t->b2 = (float)o->beta2;
  t->eps = (float)o->eps;
  t->max_steps = o->max_steps;
  size_t off = 0;
  auto add = [&](std::vector<Layer>& L, const std::vector<int>& wd) {
    for (size_t i = 0; i + 1 < wd.size(); ++i) {
      Layer y;
      y.K = wd[i];
      y.Kp = pad32(wd[i]);
      y.N = wd[i + 1];
      y.offW = off;
      off += ((size_t)y.Kp * y.N + 63) / 64 * 64;
      y.offb = off;
      off += ((size_t)y.N + 63) / 64 * 64;
      L.push_back(y);
    }
  };
  add(t->bl, net->bw);
  add(t->tl, net->tw);
  t->nparam = off;
  helm_status s = HELM_OK;
  auto fin = [&](helm_status e) {
    if (e) delete t;
    return e;
  };
  if (hipStreamCreateWithFlags(&t->st, hipStreamNonBlocking) != hipSuccess)
    return fin(fail(HELM_E_HIP, "don_train_create: stream"));
  const size_t S = t->S, P = t->P;
  size_t bsum = 0, tsum = 0;
  t->bact_off[0] = (size_t)S * t->bl[0].Kp;  // the gathered inputs come first
  for (size_t i = 0; i < t->bl.size(); ++i) {
    t->bact_off[i] = t->bact_off[0] + bsum;
    bsum += S * t->bl[i].N;
  }
  for (size_t i = 0; i < t->tl.size(); ++i) {
    t->tact_off[i] = tsum;
    tsum += P * t->tl[i].N;
  }
  int maxw = 0;
  for (auto& y : t->tl) maxw = std::max(maxw, std::max(y.N, y.Kp));
  int maxbw = 0;
  for (auto& y : t->bl) maxbw = std::max(maxbw, std::max(y.N, y.Kp));
  size_t maxkn = 0;
  for (auto& y : t->tl) maxkn = std::max(maxkn, (size_t)y.Kp * y.N);
  for (auto& y : t->bl) maxkn = std::max(maxkn, (size_t)y.Kp * y.N);
  // split-k partial space: the largest of the dW slices, the forward splits and dBc's
  t->dw_slices = std::max<size_t>(maxkn * 128, (size_t)2 * S * t->p * 512);
  t->dw_slices = std::max<size_t>(t->dw_slices, (size_t)S * 256 * 256);
  const size_t nch = (P + 4095) / 4096;
  if ((s = t->master.ensure(4 * t->nparam)) || (s = t->grad.ensure(4 * t->nparam)) ||
      (s = t->mom.ensure(4 * t->nparam)) || (s = t->var.ensure(4 * t->nparam)) || (s = t->wbf.ensure(2 * t->nparam)) ||
      (s = t->X.ensure(2 * P * t->tl[0].Kp)) || (s = t->bact.ensure(2 * (t->bact_off[0] + bsum))) ||
      (s = t->tact.ensure(2 * tsum)) || (s = t->dz0.ensure(2 * P * maxw)) || (s = t->dz1.ensure(2 * P * maxw)) ||
      (s = t->bdz0.ensure(2 * S * maxbw)) || (s = t->bdz1.ensure(2 * S * maxbw)) ||
      (s = t->Bc.ensure(2 * 2 * S * t->p)) || (s = t->Ut.ensure(4 * 2 * S * P)) || (s = t->dUt.ensure(2 * 2 * S * P)) ||
      (s = t->dBcp.ensure(4 * (size_t)2 * S * t->p * 512)) || (s = t->dBc.ensure(4 * 2 * S * t->p)) ||
      (s = t->dW.ensure(4 * t->dw_slices)) || (s = t->cs.ensure(4 * ((P + 1023) / 1024 + 1) * 256)) ||
      (s = t->lpart.ensure(8 * 2 * S * nch)) || (s = t->wv.ensure(4 * S)) || (s = t->ctr.ensure(64)) ||
      (s = t->losses.ensure(4 * (size_t)o->max_steps)) || (s = t->idx.ensure(4 * (size_t)o->max_steps * S)))
    return fin(s);
  // zero the whole flat state (padding rows stay zero), then copy the weights
  hipError_t e = hipMemsetAsync(t->master.ptr, 0, 4 * t->nparam, t->st);
  if (e == hipSuccess) e = hipMemsetAsync(t->mom.ptr, 0, 4 * t->nparam, t->st);
  if (e == hipSuccess) e = hipMemsetAsync(t->var.ptr, 0, 4 * t->nparam, t->st);
  if (e == hipSuccess) e = hipMemsetAsync(t->grad.ptr, 0, 4 * t->nparam, t->st);
  if (e == hipSuccess) e = hipMemsetAsync(t->ctr.ptr, 0, 64, t->st);
  if (e != hipSuccess) return fin(hip_fail(e, "don_train_create: clear"));
  auto load = [&](std::vector<Layer>& L, std::vector<void*>& W, std::vector<void*>& B) {
    float* m = (float*)t->master.ptr;
    for (size_t i = 0; i < L.size(); ++i) {
      const Layer& y = L[i];
      if (net->dt == HELM_C128) {
        hipLaunchKernelGGL(k_cvt_pad<double>, dim3(grid_for((long)y.Kp * y.N)), dim3(256), 0, t->st, y.K, y.N, y.Kp,
                           (const double*)W[i], m + y.offW);
        hipLaunchKernelGGL(k_cvt_pad<double>, dim3(1), dim3(256), 0, t->st, 1, y.N, 1, (const double*)B[i], m + y.offb);
      } else {
        hipLaunchKernelGGL(k_cvt_pad<float>, dim3(grid_for((long)y.Kp * y.N)), dim3(256), 0, t->st, y.K, y.N, y.Kp,
                           (const float*)W[i], m + y.offW);
        hipLaunchKernelGGL(k_cvt_pad<float>, dim3(1), dim3(256), 0, t->st, 1, y.N, 1, (const float*)B[i], m + y.offb);
      }
    }
  };
  load(t->bl, net->bW, net->bB);
  load(t->tl, net->tW, net->tB);
  hipLaunchKernelGGL(k_f32_to_bf16, dim3(grid_for((long)t->nparam)), dim3(256), 0, t->st, (long)t->nparam,
                     (const float*)t->master.ptr, (__bf16*)t->wbf.ptr);
  // trunk inputs: fp64 P x d -> bf16 padded rows
  {
    Buffer tmp;
    if ((s = tmp.ensure(4 * P * t->d))) return fin(s);
    std::vector<double> hx((size_t)P * t->d);
    e = hipMemcpy(hx.data(), X, sizeof(double) * hx.size(), hipMemcpyDeviceToHost);
    if (e != hipSuccess) {
      tmp.release();
      return fin(hip_fail(e, "don_train_create: X"));
    }
    std::vector<float> fx(hx.begin(), hx.end());
    e = hipMemcpy(tmp.ptr, fx.data(), sizeof(float) * fx.size(), hipMemcpyHostToDevice);
    if (e == hipSuccess)
      hipLaunchKernelGGL(k_pad_rows, dim3(grid_for((long)P * t->tl[0].Kp)), dim3(256), 0, t->st, (long)P, t->d,
                         (const float*)tmp.ptr, t->tl[0].Kp, (__bf16*)t->X.ptr);
    s = e == hipSuccess ? sync(t, "don_train_create") : hip_fail(e, "don_train_create: X");
    tmp.release();
    if (s) return fin(s);
  }
  *out = t;
  return launch_check("don_train_create");
}

helm_status don_train_data(don_trainer t, int n, const float* F, const void* Y) {
  if (!t || !F || !Y || n < 1) return fail(HELM_E_INVAL, "don_train_data: bad argument");
  const Layer& b0 = t->bl[0];
  helm_status s = t->Fdata.ensure((size_t)2 * n * b0.Kp);
  if (s) return s;
  hipLaunchKernelGGL(k_pad_rows, dim3(grid_for((long)n * b0.Kp)), dim3(256), 0, t->st, (long)n, b0.K, F, b0.Kp,
                     (__bf16*)t->Fdata.ptr);
  t->Y = (const float2*)Y;
  t->ndata = n;
  return sync(t, "don_train_data");
}

static helm_status run_steps(don_trainer t, int count, const int* idx, bool update, float* loss_out) {
  if (!t || !idx || count < 1) return fail(HELM_E_INVAL, "don_train: bad argument");
  if (!t->Y) return fail(HELM_E_INVAL, "don_train: no data (don_train_data)");
  if (count > t->max_steps) return fail(HELM_E_INVAL, "don_train: %d steps exceed max_steps %d", count, t->max_steps);
  std::vector<int> h((size_t)count * t->S);
  hipError_t e = hipMemcpy(h.data(), idx, sizeof(int) * h.size(), hipMemcpyDeviceToHost);
  if (e != hipSuccess) return hip_fail(e, "don_train: idx");
  for (int v : h)
    if (v < 0 || v >= t->ndata) return fail(HELM_E_INVAL, "don_train: sample index %d outside [0, %d)", v, t->ndata);
  e = hipMemcpyAsync(t->idx.ptr, idx, sizeof(int) * h.size(), hipMemcpyDeviceToDevice, t->st);
  if (e == hipSuccess) e = hipMemsetAsync(t->ctr.ptr, 0, sizeof(int), t->st);  // step index within this call
  if (e != hipSuccess) return hip_fail(e, "don_train: setup");
  helm_status s;
  if (update) {
    if (!t->step_exec) {
      hipGraph_t g;
      if ((s = sync(t, "don_train: capture"))) return s;
      if (hipStreamBeginCapture(t->st, hipStreamCaptureModeThreadLocal) != hipSuccess)
        return fail(HELM_E_HIP, "don_train: begin capture");
      train_step(t, true);
      e = hipStreamEndCapture(t->st, &g);
      if (e != hipSuccess) return hip_fail(e, "don_train: end capture");
      e = hipGraphInstantiate(&t->step_exec, g, nullptr, nullptr, 0);
      (void)hipGraphDestroy(g);
      if (e != hipSuccess) return hip_fail(e, "don_train: instantiate");
    }
    for (int k = 0; k < count; ++k) {
      e = hipGraphLaunch(t->step_exec, t->st);
      if (e != hipSuccess) return hip_fail(e, "don_train: replay");
    }
  } else {
    for (int k = 0; k < count; ++k) train_step(t, false);
  }
  if (loss_out) {
    e = hipMemcpyAsync(loss_out, t->losses.ptr, sizeof(float) * count, hipMemcpyDeviceToHost, t->st);
    if (e != hipSuccess) return hip_fail(e, "don_train: losses");
  }
  if ((s = sync(t, "don_train"))) return s;
  return launch_check("don_train");
}

helm_status don_train_steps(don_trainer t, int count, const int* idx, float* loss_out, void* stream) {
  if (t && stream && sync_stream((hipStream_t)stream, "don_train_steps")) return HELM_E_HIP;
  return run_steps(t, count, idx, true, loss_out);
}

helm_status don_train_grad(don_trainer t, const int* idx, float* loss, float* grads, void* stream) {
  if (!t || !grads) return fail(HELM_E_INVAL, "don_train_grad: NULL argument");
  if (stream && sync_stream((hipStream_t)stream, "don_train_grad")) return HELM_E_HIP;
  helm_status s = run_steps(t, 1, idx, false, loss);
  if (s) return s;
  hipError_t e = hipMemcpy(grads, t->grad.ptr, 4 * t->nparam, hipMemcpyDeviceToDevice);
  return e == hipSuccess ? HELM_OK : hip_fail(e, "don_train_grad: copy");
}

helm_status don_train_apply(don_trainer t, const float* grads, void* stream) {
  if (!t || !grads) return fail(HELM_E_INVAL, "don_train_apply: NULL argument");
  if (stream && sync_stream((hipStream_t)stream, "don_train_apply")) return HELM_E_HIP;
  hipError_t e = hipMemcpyAsync(t->grad.ptr, grads, 4 * t->nparam, hipMemcpyDeviceToDevice, t->st);
  if (e != hipSuccess) return hip_fail(e, "don_train_apply: copy");
  int* ctr = (int*)t->ctr.ptr;
  hipLaunchKernelGGL(k_adam, dim3(grid_for((long)t->nparam)), dim3(256), 0, t->st, (long)t->nparam,
                     (float*)t->master.ptr, (const float*)t->grad.ptr, (float*)t->mom.ptr, (float*)t->var.ptr,
                     (__bf16*)t->wbf.ptr, t->lr, t->b1, t->b2, t->eps, (const int*)(ctr + 1));
  hipLaunchKernelGGL(k_tick, dim3(1), dim3(64), 0, t->st, ctr, ctr + 1, 1);
  return sync(t, "don_train_apply");
}

helm_status don_train_eval(don_trainer t, int count, const int* idx, float* loss_out, void* stream) {
  if (!loss_out) return fail(HELM_E_INVAL, "don_train_eval: NULL loss_out");
  if (t && stream && sync_stream((hipStream_t)stream, "don_train_eval")) return HELM_E_HIP;
  return run_steps(t, count, idx, false, loss_out);
}

size_t don_train_nparam(don_trainer t) { return t ? t->nparam : 0; }

helm_status don_train_layout(don_trainer t, int which, int layer, int* K, int* Kp, int* N, size_t* offW,
                             size_t* offb) {
  if (!t || (which != 0 && which != 1)) return fail(HELM_E_INVAL, "don_train_layout: bad argument");
  const std::vector<Layer>& L = which == 0 ? t->bl : t->tl;
  if (layer < 0 || layer >= (int)L.size()) return fail(HELM_E_INVAL, "don_train_layout: layer %d", layer);
  const Layer& y = L[layer];
  if (K) *K = y.K;
  if (Kp) *Kp = y.Kp;
  if (N) *N = y.N;
  if (offW) *offW = y.offW;
  if (offb) *offb = y.offb;
  return HELM_OK;
}

helm_status don_train_params(don_trainer t, float* out, void* stream) {
  if (!t || !out) return fail(HELM_E_INVAL, "don_train_params: NULL argument");
  if (stream && sync_stream((hipStream_t)stream, "don_train_params")) return HELM_E_HIP;
  hipError_t e = hipMemcpyAsync(out, t->master.ptr, 4 * t->nparam, hipMemcpyDeviceToDevice, t->st);
  if (e != hipSuccess) return hip_fail(e, "don_train_params");
  return sync(t, "don_train_params");
}

helm_status don_train_export(don_trainer t, don_net net, void* stream) {
  if (!t || !net) return fail(HELM_E_INVAL, "don_train_export: NULL argument");
  if (net->bw.size() != t->bl.size() + 1 || net->tw.size() != t->tl.size() + 1)
    return fail(HELM_E_INVAL, "don_train_export: network shape differs from the trainer's");
  if (stream && sync_stream((hipStream_t)stream, "don_train_export")) return HELM_E_HIP;
  const float* m = (const float*)t->master.ptr;
  auto put = [&](std::vector<Layer>& L, std::vector<void*>& W, std::vector<void*>& B) {
    for (size_t i = 0; i < L.size(); ++i) {
      const Layer& y = L[i];
      if (net->dt == HELM_C128) {
        hipLaunchKernelGGL(k_cvt_back<double>, dim3(grid_for((long)y.K * y.N)), dim3(256), 0, t->st, y.K, y.N,
                           m + y.offW, (double*)W[i]);
        hipLaunchKernelGGL(k_cvt_back<double>, dim3(1), dim3(256), 0, t->st, 1, y.N, m + y.offb, (double*)B[i]);
      } else {
        hipLaunchKernelGGL(k_cvt_back<float>, dim3(grid_for((long)y.K * y.N)), dim3(256), 0, t->st, y.K, y.N,
                           m + y.offW, (float*)W[i]);
        hipLaunchKernelGGL(k_cvt_back<float>, dim3(1), dim3(256), 0, t->st, 1, y.N, m + y.offb, (float*)B[i]);
      }
    }
  };
  put(t->bl, net->bW, net->bB);
  put(t->tl, net->tW, net->tB);
  helm_status s = sync(t, "don_train_export");
  if (s) return s;
  don_touch(net);
  return launch_check("don_train_export");
}

void don_train_free(don_trainer t) { delete t; }

}  // extern "C"
