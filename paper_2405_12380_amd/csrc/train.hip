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
// Every matrix product runs in one bf16 GEMM kernel, C = A B^T with both
// operands k-contiguous (v_mfma_f32_16x16x32_bf16, 128 x 128 tile per
// 256-thread workgroup, 64-deep k steps through LDS with the next step's
// operands prefetched into registers), with fused epilogues (bias + tanh, bias,
// tanh derivative, fp32) or split-k partials reduced in a fixed order.  So that
// every product is of that form, the epilogues also write a transposed copy of
// each activation and each gradient (the backward products reduce over the
// points, which must then be contiguous), and Adam refreshes both W and W^T in
// bf16.  The branch MLP (forward and backward) runs on a second stream beside
// the trunk, and the trunk's bias row sums on a third beside its weight
// products.  Steps are captured as HIP graphs (one step, and eight steps per
// launch) and replayed; the sample indices and the step counter live on the
// device.
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

constexpr int TM = 128, TN = 128, BK = 64, LDSW = 72;  // tile, k step, LDS row stride (bf16, 144 B)

enum { EP_F32 = 0, EP_BF16 = 1, EP_BIAS_BF16 = 2, EP_BIAS_TANH_BF16 = 3, EP_DTANH_BF16 = 4, EP_PART = 5 };

// C (M x N) = A (M x K) B (N x K)^T: both operands k-contiguous ("NT").
struct GemmArgs {
  const __bf16* A;
  long lda;
  const __bf16* B;
  long ldb;
  int M, N, K, kchunk;
  void* C;
  long ldc;
  __bf16* CT;  // optional transposed bf16 copy of the result (N x M, leading dimension ldct)
  long ldct;
  const float* bias;
  const __bf16* aux;  // EP_DTANH_BF16: the activation h (M x N, leading dimension ldc)
  int ep;
};

__device__ __forceinline__ float bf2f(__bf16 v) { return (float)v; }

// tanh x = 1 - 2 / (1 + e^{2x}) with the hardware exponential and reciprocal
// (each within an ulp or so of fp32, far below the bf16 rounding that follows;
// saturates to +-1: e^{2x} = inf gives 1, e^{2x} = 0 gives -1)
__device__ __forceinline__ float fast_tanh(float x) {
  return 1.0f - 2.0f * __builtin_amdgcn_rcpf(1.0f + __expf(2.0f * x));
}

// Epilogue of one value of C(row, col); returns the stored bf16 value for the transposed copy.
__device__ __forceinline__ __bf16 ep_store(const GemmArgs& g, int row, int col, float v, int slice = 0) {
  const long o = (long)row * g.ldc + col;
  __bf16 r = (__bf16)0.0f;
  switch (g.ep) {
    case EP_F32:
      ((float*)g.C)[o] = v;
      break;
    case EP_BF16:
      r = (__bf16)v;
      ((__bf16*)g.C)[o] = r;
      break;
    case EP_BIAS_BF16:
      r = (__bf16)(v + g.bias[col]);
      ((__bf16*)g.C)[o] = r;
      break;
    case EP_BIAS_TANH_BF16:
      r = (__bf16)fast_tanh(v + g.bias[col]);
      ((__bf16*)g.C)[o] = r;
      break;
    case EP_DTANH_BF16: {
      const float h = bf2f(g.aux[o]);
      r = (__bf16)(v * (1.0f - h * h));
      ((__bf16*)g.C)[o] = r;
      break;
    }
    default:  // EP_PART: split-k slice `slice` of an M x N fp32 array
      ((float*)g.C)[(long)slice * g.M * g.N + (long)row * g.N + col] = v;
  }
  return r;
}

// 128 x 128 output tile per 256-thread workgroup over this workgroup's k slice.
// Each thread moves four 16-byte chunks of each operand per 64-deep k step
// (8 threads per 128-byte row segment); the next step's chunks are loaded into
// registers while the current step's 32 MFMAs per wavefront run from LDS.
// Wavefront w owns the 64 x 64 quadrant (w / 2, w % 2) as 4 x 4 tiles of
// v_mfma_f32_16x16x32_bf16: lane l holds A[l % 16][8 (l / 16) .. +7],
// B[l % 16][8 (l / 16) .. +7] (B stored n-major) and C[4 (l / 16) + i][l % 16].
constexpr int CTW = TN + 8;  // LDS row stride of the staged output tile (bf16)

// Position of element (r, c) of the staged output tile: the 16-byte pieces of
// row r are permuted by (r / 8) mod 8, so the column gathers of the transposed
// copy (sixteen lanes reading rows 8 apart) fall in distinct LDS banks; row
// pieces stay contiguous and aligned.
__device__ __forceinline__ int csw(int r, int c) { return r * CTW + ((((c >> 3) ^ ((r >> 3) & 7)) << 3) | (c & 7)); }

__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(3))) void k_gemm_nt(GemmArgs g) {
  // operand tiles during the k loop; the output tile (then its transpose) afterwards
  __shared__ __attribute__((aligned(16))) __bf16 smem[(TM + TN) * LDSW];
  __bf16* As = smem;
  __bf16* Bs = smem + TM * LDSW;
  // logical tile (y fastest, then x, then the k slice): consecutive logical
  // blocks run on one XCD, so the column tiles of a row block, and the tiles of
  // a k slice, read their shared operand rows through that XCD's L2
  const unsigned gx = gridDim.x, gy = gridDim.y;
  const unsigned lb = xcd_remap(blockIdx.x + gx * (blockIdx.y + gy * blockIdx.z), gx * gy * gridDim.z);
  const int byl = lb % gy, bxl = (lb / gy) % gx, bzl = lb / (gx * gy);
  const int m0 = bxl * TM, n0 = byl * TN;
  const int kb = bzl * g.kchunk;
  const int ke = min(g.K, kb + g.kchunk);
  const int t = threadIdx.x, w = t >> 6, l = t & 63;
  const int wm = w >> 1, wn = w & 1;
  bf8 zero;
#pragma unroll
  for (int j = 0; j < 8; ++j) zero[j] = (__bf16)0.0f;
  bf8 ra[4], rb[4];
  auto load = [&](int k0) {
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int c = t + 256 * j, row = c >> 3, kq = (c & 7) * 8;
      ra[j] = m0 + row < g.M ? *(const bf8*)(g.A + (long)(m0 + row) * g.lda + k0 + kq) : zero;
      rb[j] = n0 + row < g.N ? *(const bf8*)(g.B + (long)(n0 + row) * g.ldb + k0 + kq) : zero;
    }
  };
  f4 acc[4][4];
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) acc[i][j] = f4{0.f, 0.f, 0.f, 0.f};
  if (kb < ke) load(kb);
  for (int k0 = kb; k0 < ke; k0 += BK) {
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int c = t + 256 * j, row = c >> 3, kq = (c & 7) * 8;
      *(bf8*)(As + row * LDSW + kq) = ra[j];
      *(bf8*)(Bs + row * LDSW + kq) = rb[j];
    }
    __syncthreads();
    if (k0 + BK < ke) load(k0 + BK);
#pragma unroll
    for (int kk = 0; kk < BK; kk += 32) {
      bf8 a[4], b[4];
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        a[i] = *(const bf8*)(As + (wm * 64 + i * 16 + (l & 15)) * LDSW + kk + 8 * (l >> 4));
        b[i] = *(const bf8*)(Bs + (wn * 64 + i * 16 + (l & 15)) * LDSW + kk + 8 * (l >> 4));
      }
#pragma unroll
      for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j)
          acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[i], b[j], acc[i][j], 0, 0, 0);
    }
    __syncthreads();
  }
  if (g.ep == EP_F32 || g.ep == EP_PART) {
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const int row0 = m0 + wm * 64 + i * 16 + 4 * (l >> 4);
        const int col = n0 + wn * 64 + j * 16 + (l & 15);
        if (col >= g.N) continue;
#pragma unroll
        for (int q = 0; q < 4; ++q)
          if (row0 + q < g.M) ep_store(g, row0 + q, col, acc[i][j][q], bzl);
      }
    return;
  }
  // bf16 results: the epilogue math goes straight from the accumulators into a
  // row-major LDS copy of the tile (the accumulators are read once, so they
  // never need a second set of registers); C is written from it as 16-byte row
  // chunks, and C^T from the same copy, each 16-byte column chunk gathered from
  // eight LDS rows
  __bf16* Cs = smem;  // TM x CTW, reuses the operand tiles (the k loop ended with a barrier)
  if (g.ep == EP_DTANH_BF16) {
    // the activation tile h goes into Cs first, read with 16-byte row loads all
    // in flight at once; each value of C then reads its h from LDS and
    // overwrites it (every position belongs to one thread, so no barrier
    // separates the read from the write)
    bf8 hv[8];
#pragma unroll
    for (int k = 0; k < 8; ++k) {
      const int c = t + 256 * k, rl = c >> 4, cq = (c & 15) * 8;
      const int row = m0 + rl, col = n0 + cq;
      hv[k] = (row < g.M && col + 8 <= g.N) ? *(const bf8*)(g.aux + (long)row * g.ldc + col) : zero;
    }
#pragma unroll
    for (int k = 0; k < 8; ++k) {
      const int c = t + 256 * k, rl = c >> 4, cq = (c & 15) * 8;
      *(bf8*)(Cs + csw(rl, cq)) = hv[k];
    }
    __syncthreads();
  }
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    const int col = n0 + wn * 64 + j * 16 + (l & 15);
    const bool cin = col < g.N;
    const float bias = (cin && (g.ep == EP_BIAS_BF16 || g.ep == EP_BIAS_TANH_BF16)) ? g.bias[col] : 0.0f;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        float v = acc[i][j][q] + bias;
        __bf16* cp = Cs + csw(wm * 64 + i * 16 + 4 * (l >> 4) + q, wn * 64 + j * 16 + (l & 15));
        if (g.ep == EP_BIAS_TANH_BF16) v = fast_tanh(v);
        else if (g.ep == EP_DTANH_BF16) {
          const float h = bf2f(*cp);  // zero outside the M x N result, which is never stored
          v *= 1.0f - h * h;
        }
        *cp = (__bf16)v;
      }
    }
  }
  __syncthreads();
#pragma unroll
  for (int k = 0; k < 8; ++k) {
    const int c = t + 256 * k, rl = c >> 4, cq = (c & 15) * 8;
    const int row = m0 + rl, col = n0 + cq;
    if (row < g.M && col + 8 <= g.N)
      *(bf8*)((__bf16*)g.C + (long)row * g.ldc + col) = *(const bf8*)(Cs + csw(rl, cq));
  }
  if (!g.CT) return;
#pragma unroll
  for (int k = 0; k < 8; ++k) {
    const int c = t + 256 * k, cl = c >> 4, rq = (c & 15) * 8;
    const int col = n0 + cl, row = m0 + rq;
    bf8 v;
#pragma unroll
    for (int u = 0; u < 8; ++u) v[u] = Cs[csw(rq + u, cl)];
    if (col < g.N && row + 8 <= g.M) *(bf8*)(g.CT + (long)col * g.ldct + row) = v;
  }
}

// Whole-MLP forward for a 128-row block (the trunk, whose M is the number of
// points): the block's activation stays in LDS from layer to layer, so only
// the first layer's input is read from HBM; each layer writes its output (h,
// row-major) and its transpose (h^T) for the backward pass.  Four wavefronts,
// wavefront w owning output columns 64 w .. 64 w + 63 of all 128 rows (8 x 4
// tiles of v_mfma_f32_16x16x32_bf16); A fragments come from the LDS
// activation, B fragments straight from W^T (a few hundred KB, resident in L2)
// one 32-deep k step ahead, so the k loop has no barrier.  The k order of the
// accumulation and the epilogue are those of k_gemm_nt, so the values equal
// the layer-by-layer products bit for bit.
constexpr int FW_MAXL = 8, FW_ACT = 256 + 8;  // layers; LDS activation row stride (bf16)
// element (r, c) of the LDS activation, 16-byte pieces permuted per row as in csw
__device__ __forceinline__ int asw(int r, int c) { return r * FW_ACT + ((((c >> 3) ^ ((r >> 3) & 7)) << 3) | (c & 7)); }
struct FwdArgs {
  int L, M;
  int Kp[FW_MAXL], N[FW_MAXL];  // Kp[0] = padded input width; Kp[l + 1] = N[l]; all multiples of 64, <= 256
  const __bf16* X;              // M x Kp[0] input rows
  const __bf16* wt[FW_MAXL];    // W^T, N x Kp, k-contiguous
  const float* bias[FW_MAXL];
  __bf16* h[FW_MAXL];   // M x N
  __bf16* hT[FW_MAXL];  // N x M
};

__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(2, 2))) void k_mlp_fwd(FwdArgs a) {
  __shared__ __attribute__((aligned(16))) __bf16 act[TM * FW_ACT];
  const int m0 = blockIdx.x * TM;
  const int t = threadIdx.x, w = t >> 6, l = t & 63;
  bf8 zero;
#pragma unroll
  for (int j = 0; j < 8; ++j) zero[j] = (__bf16)0.0f;
  {
    const int cpr = a.Kp[0] / 8;  // 16-byte pieces per input row
    for (int c = t; c < TM * cpr; c += 256) {
      const int r = c / cpr, kq = (c % cpr) * 8;
      *(bf8*)(act + asw(r, kq)) = m0 + r < a.M ? *(const bf8*)(a.X + (long)(m0 + r) * a.Kp[0] + kq) : zero;
    }
  }
  __syncthreads();
  for (int li = 0; li < a.L; ++li) {
    const int Kp = a.Kp[li], N = a.N[li];
    const bool last = li + 1 == a.L, on = 64 * w < N;
    f4 acc[8][4];
#pragma unroll
    for (int i = 0; i < 8; ++i)
#pragma unroll
      for (int j = 0; j < 4; ++j) acc[i][j] = f4{0.f, 0.f, 0.f, 0.f};
    if (on) {
      // lane l's B fragment rows: W^T rows 64 w + 16 j + (l % 16), k offset 8 (l / 16);
      // two register sets, each loaded one 32-deep step before it is used
      const __bf16* Wl = a.wt[li] + (long)(64 * w + (l & 15)) * Kp + 8 * (l >> 4);
      bf8 b0[4], b1[4];
      auto loadb = [&](bf8* b, int k) {
#pragma unroll
        for (int j = 0; j < 4; ++j) b[j] = *(const bf8*)(Wl + (long)j * 16 * Kp + k);
        __builtin_amdgcn_sched_barrier(0);  // keep the loads here, a whole step ahead of their use
      };
      auto step = [&](const bf8* b, int k) {
        bf8 av[8];
#pragma unroll
        for (int i = 0; i < 8; ++i) av[i] = *(const bf8*)(act + asw(i * 16 + (l & 15), k + 8 * (l >> 4)));
#pragma unroll
        for (int i = 0; i < 8; ++i)
#pragma unroll
          for (int j = 0; j < 4; ++j) acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(av[i], b[j], acc[i][j], 0, 0, 0);
      };
      loadb(b0, 0);
      for (int k = 0; k < Kp; k += 64) {  // Kp is a multiple of 64
        loadb(b1, k + 32);
        step(b0, k);
        loadb(b0, k + 64 < Kp ? k + 64 : k);  // the last step reloads (unconditional, so waits stay exact)
        step(b1, k + 32);
      }
    }
    __syncthreads();  // every wavefront has finished reading this layer's input
    if (on) {
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const int col = 64 * w + j * 16 + (l & 15);
        const float bias = a.bias[li][col];
#pragma unroll
        for (int i = 0; i < 8; ++i)
#pragma unroll
          for (int q = 0; q < 4; ++q) {
            float v = acc[i][j][q] + bias;
            if (!last) v = fast_tanh(v);
            act[asw(i * 16 + 4 * (l >> 4) + q, col)] = (__bf16)v;
          }
      }
    }
    __syncthreads();
    // h as 16-byte row pieces, h^T as 16-byte column pieces gathered from eight rows
    const int cpr = N / 8;
    for (int c = t; c < TM * cpr; c += 256) {
      const int r = c / cpr, cq = (c % cpr) * 8;
      if (m0 + r < a.M)  // read again only in the backward pass: streaming stores
        __builtin_nontemporal_store(*(const bf8*)(act + asw(r, cq)), (bf8*)(a.h[li] + (long)(m0 + r) * N + cq));
    }
    for (int c = t; c < N * (TM / 8); c += 256) {
      const int col = c / (TM / 8), rq = (c % (TM / 8)) * 8;
      bf8 v;
#pragma unroll
      for (int u = 0; u < 8; ++u) v[u] = act[asw(rq + u, col)];
      if (m0 + rq + 8 <= a.M) __builtin_nontemporal_store(v, (bf8*)(a.hT[li] + (long)col * a.M + m0 + rq));
    }
  }
}

// sum of split-k slices in a fixed order, then the epilogue (and the transposed copy)
__global__ __launch_bounds__(256) void k_splitk_reduce(GemmArgs g, const float* __restrict__ part, int splits) {
  const long MN = (long)g.M * g.N;
  for (long e = blockIdx.x * 256L + threadIdx.x; e < MN; e += (long)gridDim.x * 256) {
    float v = 0.f;
    for (int z0 = 0; z0 < splits; z0 += 8) {  // eight slices' loads in flight, added in slice order
      float x[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) x[u] = z0 + u < splits ? part[(z0 + u) * MN + e] : 0.f;
#pragma unroll
      for (int u = 0; u < 8; ++u) v += x[u];
    }
    const int row = (int)(e / g.N), col = (int)(e % g.N);
    const __bf16 r = ep_store(g, row, col, v);
    if (g.CT) g.CT[(long)col * g.ldct + row] = r;
  }
}

// out[r] = sum of row r of a bf16 R x M matrix (fixed order: per-thread strided sums, then a tree)
__global__ __launch_bounds__(256) void k_rowsum(const __bf16* __restrict__ D, long M, float* __restrict__ out) {
  __shared__ double sh[16];
  const __bf16* row = D + (long)blockIdx.x * M;
  double a = 0.0;
  for (long c0 = threadIdx.x * 8L; c0 < M; c0 += 4 * 256 * 8L) {  // four 16-byte loads in flight, same order
    bf8 v[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const long c = c0 + u * 256 * 8L;
      if (c < M) v[u] = *(const bf8*)(row + c);
    }
#pragma unroll
    for (int u = 0; u < 4; ++u)
      if (c0 + u * 256 * 8L < M)
#pragma unroll
        for (int j = 0; j < 8; ++j) a += (double)bf2f(v[u][j]);
  }
  a = block_sum(a, sh);
  if (threadIdx.x == 0) out[blockIdx.x] = (float)a;
}

// Branch inputs of the batch: rows idx[step S + s] of the dataset (bf16, padded), and the transpose
__global__ __launch_bounds__(256) void k_gather(const __bf16* __restrict__ F, long ldf, const int* __restrict__ idx,
                                                const int* __restrict__ step, int S, __bf16* __restrict__ out,
                                                __bf16* __restrict__ outT) {
  const int s = blockIdx.y;
  const int src = idx[(long)step[0] * S + s];
  for (long c = blockIdx.x * 256L + threadIdx.x; c < ldf; c += (long)gridDim.x * 256) {
    const __bf16 v = F[(long)src * ldf + c];
    out[(long)s * ldf + c] = v;
    outT[c * S + s] = v;
  }
}

// Bc (2S x p): row s = B[s][0:p], row S + s = B[s][p:2p]; BcT its transpose (p x 2S)
__global__ void k_to_bc(const __bf16* __restrict__ B, int S, int p, __bf16* __restrict__ Bc, __bf16* __restrict__ BcT) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= 2 * S * p) return;
  const int r = e / p, c = e % p;
  const __bf16 v = r < S ? B[(long)r * 2 * p + c] : B[(long)(r - S) * 2 * p + p + c];
  Bc[e] = v;
  BcT[(long)c * 2 * S + r] = v;
}

// dB (S x 2p) and its transpose (2p x S), bf16, from dBc (2S x p, fp32)
__global__ void k_from_dbc(const float* __restrict__ dBc, int S, int p, __bf16* __restrict__ dB,
                           __bf16* __restrict__ dBT) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= 2 * S * p) return;
  const int s = e / (2 * p), c = e % (2 * p);
  const __bf16 v = (__bf16)(c < p ? dBc[(long)s * p + c] : dBc[(long)(S + s) * p + (c - p)]);
  dB[e] = v;
  dBT[(long)c * S + s] = v;
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

// dUt (2S x P, bf16) = (Ut - Y) w_s, and its transpose dUtT (P x 2S): a workgroup
// takes 64 points, reads the 2S rows coalesced and writes the point-major copy
// through LDS
__global__ __launch_bounds__(256) void k_dU(const float* __restrict__ Ut, const float2* __restrict__ Y,
                                            const int* __restrict__ idx, const int* __restrict__ step,
                                            const float* __restrict__ w, int S, int P, __bf16* __restrict__ dUt,
                                            __bf16* __restrict__ dUtT) {
  __shared__ __attribute__((aligned(16))) __bf16 tile[64 * (256 + 8)];
  const int q0 = blockIdx.x * 64, t = threadIdx.x, pl = t & 63;
  const int R = 2 * S, ld = R + 8;
  for (int s = t >> 6; s < S; s += 4) {
    const long src = idx[(long)step[0] * S + s];
    const float ws = w[s];
    const int q = q0 + pl;
    __bf16 re = (__bf16)0.0f, im = (__bf16)0.0f;
    if (q < P) {
      const float2 y = Y[src * P + q];
      re = (__bf16)((Ut[(long)s * P + q] - y.x) * ws);
      im = (__bf16)((Ut[(long)(S + s) * P + q] - y.y) * ws);
      dUt[(long)s * P + q] = re;
      dUt[(long)(S + s) * P + q] = im;
    }
    tile[pl * ld + s] = re;
    tile[pl * ld + S + s] = im;
  }
  __syncthreads();
  const int chunks = R / 8;
  for (int c = t; c < 64 * chunks; c += 256) {
    const int pt = c / chunks, rq = (c % chunks) * 8;
    if (q0 + pt < P) *(bf8*)(dUtT + (long)(q0 + pt) * R + rq) = *(const bf8*)(tile + pt * ld + rq);
  }
}

// weight matrices inside the flat parameter array (Kp x N row-major at off,
// the N biases at offb); tile0[L] = index of layer L's first 64 x 64 tile
constexpr int WT_MAX = 16;
struct WTab {
  int n;
  long off[WT_MAX], offb[WT_MAX];
  int Kp[WT_MAX], N[WT_MAX];
  int tile0[WT_MAX + 1];
};

// Adam on the flat parameters (fp32), step t = tstep[0] + 1; refreshes the bf16
// copies W and W^T.  Workgroup b < tile0[n] takes one 64 x 64 tile of a weight
// matrix (coalesced reads and writes along N; the bf16 tile goes through LDS
// so W^T is written along Kp, coalesced too); the next n workgroups take one
// layer's biases each.  The padding between layers in the flat arrays is not
// touched (its gradient is zero and its values never read).
__global__ __launch_bounds__(256) void k_adam(float* __restrict__ w, const float* __restrict__ g,
                                              float* __restrict__ m, float* __restrict__ v, __bf16* __restrict__ wb,
                                              __bf16* __restrict__ wt, WTab tab, float lr, float b1, float b2,
                                              float eps, const int* __restrict__ tstep) {
  __shared__ __bf16 tile[64][66];
  const int t = tstep[0] + 1;
  // bias corrections in fp64: 1 - b2^t in fp32 cancels about 10 bits at b2 = 0.999
  const float c1 = (float)(1.0 - pow((double)b1, (double)t)), c2 = (float)(1.0 - pow((double)b2, (double)t));
  auto update = [&](long e) {
    const float ge = g[e];
    const float me = b1 * m[e] + (1.0f - b1) * ge;
    const float ve = b2 * v[e] + (1.0f - b2) * ge * ge;
    m[e] = me;
    v[e] = ve;
    const float we = w[e] - lr * (me / c1) / (sqrtf(ve / c2) + eps);
    w[e] = we;
    const __bf16 wh = (__bf16)we;
    wb[e] = wh;
    return wh;
  };
  const int b = blockIdx.x;
  if (b < tab.tile0[tab.n]) {
    int L = 0;
    while (b >= tab.tile0[L + 1]) ++L;
    const int tl = b - tab.tile0[L], tcn = tab.N[L] / 64;
    const int r0 = (tl / tcn) * 64, c0 = (tl % tcn) * 64;
    for (int e = threadIdx.x; e < 64 * 64; e += 256) {
      const int r = e >> 6, c = e & 63;
      tile[r][c] = update(tab.off[L] + (long)(r0 + r) * tab.N[L] + c0 + c);
    }
    __syncthreads();
    for (int e = threadIdx.x; e < 64 * 64; e += 256) {
      const int c = e >> 6, r = e & 63;
      wt[tab.off[L] + (long)(c0 + c) * tab.Kp[L] + r0 + r] = tile[r][c];
    }
  } else {
    const int L = b - tab.tile0[tab.n];
    for (int e = threadIdx.x; e < tab.N[L]; e += 256) (void)update(tab.offb[L] + e);
  }
}

// W^T (N x Kp) from W (Kp x N), bf16
__global__ void k_transpose(int Kp, int N, const __bf16* __restrict__ W, __bf16* __restrict__ WT) {
  const long n = (long)Kp * N;
  for (long e = blockIdx.x * 256L + threadIdx.x; e < n; e += (long)gridDim.x * 256) {
    const long r = e / N, c = e % N;
    WT[c * Kp + r] = W[e];
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

// padded bf16 rows (ld columns) from fp32 rows (cols columns); optional transpose (ld x rows)
__global__ void k_pad_rows(long rows, int cols, const float* __restrict__ a, int ld, __bf16* __restrict__ b,
                           __bf16* __restrict__ bT) {
  const long n = rows * ld;
  for (long e = blockIdx.x * 256L + threadIdx.x; e < n; e += (long)gridDim.x * 256) {
    const long r = e / ld;
    const int c = (int)(e % ld);
    const __bf16 v = (__bf16)(c < cols ? a[r * cols + c] : 0.0f);
    b[e] = v;
    if (bT) bT[(long)c * rows + r] = v;
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

static int pad64(int k) { return (k + 63) / 64 * 64; }

}  // namespace

}  // namespace helm

using namespace helm;

struct Layer {
  int K, Kp, N;       // true input width, padded, output width
  size_t offW, offb;  // offsets in the flat parameter arrays (elements)
};

// Activations of one MLP: every layer's output row-major (M x N) and transposed (N x M).
struct Acts {
  Buffer h, hT;
  std::vector<size_t> off;  // per layer, elements
};

struct don_trainer_s {
  int S = 0, P = 0, d = 0, p = 0;
  float lr = 1e-3f, b1 = 0.9f, b2 = 0.999f, eps = 1e-8f;
  std::vector<Layer> bl, tl;  // branch, trunk
  size_t nparam = 0;
  int max_steps = 0;
  Buffer master, grad, mom, var, wbf, wtb;  // flat fp32 parameters, Adam moments, bf16 W and W^T copies
  Buffer X, XT;                             // P x Kp trunk inputs (bf16) and transpose
  Buffer Fb, FbT;                           // S x Kp branch inputs of the batch and transpose
  Acts ba, ta;                              // branch and trunk activations
  Buffer dz[2], dzT[2], bdz[2], bdzT[2];    // backward ping-pong (trunk, branch)
  Buffer Bc, BcT, Ut, dUt, dUtT, dBc, part, lpart, wv, ctr, losses, idx;
  Buffer Fdata;                             // n x Kb_pad bf16
  const float2* Y = nullptr;                // n x P complex64 labels (caller's)
  int ndata = 0;
  size_t part_floats = 0;
  hipStream_t st = nullptr;
  // the branch MLP runs on st2, beside the trunk on st (forked and joined by events)
  hipStream_t st2 = nullptr;
  hipEvent_t ev_fork = nullptr, ev_join = nullptr;
  // the trunk's bias gradients (row sums of dZ^T) run on st3 beside its weight products
  hipStream_t st3 = nullptr;
  hipEvent_t ev_rs = nullptr, ev_rsj = nullptr;
  Buffer bpart;  // split-k partials of the branch products (the trunk's use part)
  hipGraphExec_t step_exec = nullptr;   // one step
  hipGraphExec_t multi_exec = nullptr;  // GRAPH_STEPS steps (fewer gaps between graph launches)
  ~don_trainer_s() {
    if (step_exec) (void)hipGraphExecDestroy(step_exec);
    if (multi_exec) (void)hipGraphExecDestroy(multi_exec);
    if (ev_fork) (void)hipEventDestroy(ev_fork);
    if (ev_join) (void)hipEventDestroy(ev_join);
    if (ev_rs) (void)hipEventDestroy(ev_rs);
    if (ev_rsj) (void)hipEventDestroy(ev_rsj);
    if (st2) (void)hipStreamDestroy(st2);
    if (st3) (void)hipStreamDestroy(st3);
    if (st) (void)hipStreamDestroy(st);
    for (Buffer* b : {&master, &grad, &mom, &var, &wbf, &wtb, &X, &XT, &Fb, &FbT, &ba.h, &ba.hT, &ta.h, &ta.hT, &dz[0],
                      &dz[1], &dzT[0], &dzT[1], &bdz[0], &bdz[1], &bdzT[0], &bdzT[1], &Bc, &BcT, &Ut, &dUt, &dUtT,
                      &dBc, &part, &bpart, &lpart, &wv, &ctr, &losses, &idx, &Fdata})
      b->release();
  }
};

namespace {

// C = A B^T (both k-contiguous), split over k when splits > 1 (partials in `part`)
void gemm(hipStream_t st, const __bf16* A, long lda, const __bf16* B, long ldb, int M, int N, int K, void* C,
          long ldc, int ep, const float* bias = nullptr, const __bf16* aux = nullptr, __bf16* CT = nullptr,
          long ldct = 0, int splits = 1, float* part = nullptr) {
  GemmArgs g{A, lda, B, ldb, M, N, K, 0, C, ldc, CT, ldct, bias, aux, ep};
  const int kblocks = K / BK;
  if (splits > kblocks) splits = kblocks;
  if (splits < 1) splits = 1;
  const int per = (kblocks + splits - 1) / splits;
  splits = (kblocks + per - 1) / per;
  g.kchunk = per * BK;
  dim3 grid((M + TM - 1) / TM, (N + TN - 1) / TN, splits);
  if (splits == 1) {
    hipLaunchKernelGGL(k_gemm_nt, grid, dim3(256), 0, st, g);
    return;
  }
  GemmArgs gp = g;
  gp.ep = EP_PART;
  gp.C = part;
  gp.CT = nullptr;
  hipLaunchKernelGGL(k_gemm_nt, grid, dim3(256), 0, st, gp);
  hipLaunchKernelGGL(k_splitk_reduce, dim3(grid_for((long)M * N)), dim3(256), 0, st, g, (const float*)part, splits);
}

// k-splits so that about `target` workgroups run, each slice at least 256 deep
int splits_for(int M, int N, int K, int target) {
  const int tiles = ((M + TM - 1) / TM) * ((N + TN - 1) / TN);
  int s = target / (tiles > 0 ? tiles : 1);
  const int maxs = K / 256 > 0 ? K / 256 : 1;
  if (s > maxs) s = maxs;
  return s < 1 ? 1 : s;
}

// forward through one MLP from H0 (M x Kp0) and its transpose
// forward through layers 0 .. count - 1 of one MLP, one product per layer
void mlp_fwd(don_trainer_s* t, std::vector<Layer>& L, const __bf16* H0, int M, Acts& a, hipStream_t st, float* part,
             size_t count) {
  const __bf16* wt = (const __bf16*)t->wtb.ptr;
  const float* mw = (const float*)t->master.ptr;
  __bf16* h = (__bf16*)a.h.ptr;
  __bf16* hT = (__bf16*)a.hT.ptr;
  const __bf16* in = H0;
  for (size_t li = 0; li < count; ++li) {
    const Layer& y = L[li];
    const bool last = li + 1 == L.size();
    gemm(st, in, y.Kp, wt + y.offW, y.Kp, M, y.N, y.Kp, h + a.off[li], y.N, last ? EP_BIAS_BF16 : EP_BIAS_TANH_BF16,
         mw + y.offb, nullptr, hT + a.off[li], M, splits_for(M, y.N, y.Kp, 256), part);
    in = h + a.off[li];
  }
}

// forward through layers first .. of one MLP in one launch (k_mlp_fwd); the
// input is H0 for first = 0, else the output of layer first - 1
void mlp_fwd_fused(don_trainer_s* t, std::vector<Layer>& L, const __bf16* H0, int M, Acts& a, hipStream_t st,
                   int first = 0) {
  FwdArgs f{};
  f.L = (int)L.size() - first;
  f.M = M;
  f.X = first == 0 ? H0 : (const __bf16*)a.h.ptr + a.off[first - 1];
  for (int q = 0; q < f.L; ++q) {
    const Layer& y = L[first + q];
    f.Kp[q] = y.Kp;
    f.N[q] = y.N;
    f.wt[q] = (const __bf16*)t->wtb.ptr + y.offW;
    f.bias[q] = (const float*)t->master.ptr + y.offb;
    f.h[q] = (__bf16*)a.h.ptr + a.off[first + q];
    f.hT[q] = (__bf16*)a.hT.ptr + a.off[first + q];
  }
  hipLaunchKernelGGL(k_mlp_fwd, dim3((M + TM - 1) / TM), dim3(256), 0, st, f);
}

// backward through one MLP given dZ of its last layer (row-major dz[0], transposed dzT[0])
// side (optional): stream for each layer's weight and bias gradients, forked
// from st once the layer's dZ is there, so they run beside the product that
// forms the next dZ; st waits for a layer's side work before it overwrites the
// dZ buffers that work reads (two layers on), and at the end
void mlp_bwd(don_trainer_s* t, std::vector<Layer>& L, const __bf16* H0T, int M, Acts& a, Buffer* dz, Buffer* dzT,
             hipStream_t st, float* part, hipStream_t side = nullptr) {
  const __bf16* wb = (const __bf16*)t->wbf.ptr;
  float* g = (float*)t->grad.ptr;
  const __bf16* h = (const __bf16*)a.h.ptr;
  const __bf16* hT = (const __bf16*)a.hT.ptr;
  hipStream_t gs = side ? side : st;  // stream of the gradient products
  int cur = 0;
  bool pending = false;  // side work of the previous layer not yet waited for
  for (int li = (int)L.size() - 1; li >= 0; --li) {
    const Layer& y = L[li];
    const __bf16* inT = li == 0 ? H0T : hT + a.off[li - 1];
    __bf16* d = (__bf16*)dz[cur].ptr;
    __bf16* dT = (__bf16*)dzT[cur].ptr;
    if (side) {
      (void)hipEventRecord(t->ev_rs, st);
      (void)hipStreamWaitEvent(side, t->ev_rs, 0);
    }
    // db = row sums of dZ^T
    hipLaunchKernelGGL(k_rowsum, dim3(y.N), dim3(256), 0, gs, (const __bf16*)dT, (long)M, g + y.offb);
    // dW = H^T dZ (Kp x N): A = H^T (Kp x M), B = dZ^T (N x M), reduction over the M rows
    int sp = splits_for(y.Kp, y.N, M, 512);
    while ((size_t)sp * y.Kp * y.N > t->part_floats && sp > 1) --sp;
    gemm(gs, inT, M, dT, M, y.Kp, y.N, M, g + y.offW, y.N, EP_F32, nullptr, nullptr, nullptr, 0, sp, part);
    if (li > 0) {
      // dZ_below = (dZ W^T) * (1 - H_below^2): A = dZ (M x N), B = W (Kp x N, n-major = k-contiguous)
      const Layer& z = L[li - 1];
      __bf16* dn = (__bf16*)dz[1 - cur].ptr;
      __bf16* dnT = (__bf16*)dzT[1 - cur].ptr;
      // dn / dnT held the previous layer's dZ, read by that layer's side work
      if (pending) (void)hipStreamWaitEvent(st, t->ev_rsj, 0);
      if (side) {
        (void)hipEventRecord(t->ev_rsj, side);  // this layer's side work, waited for one layer on
        pending = true;
      }
      gemm(st, d, y.N, wb + y.offW, y.N, M, z.N, y.N, dn, z.N, EP_DTANH_BF16, nullptr, h + a.off[li - 1], dnT, M);
      cur = 1 - cur;
    } else if (side) {
      (void)hipEventRecord(t->ev_rsj, side);
      pending = true;
    }
  }
  if (pending) (void)hipStreamWaitEvent(st, t->ev_rsj, 0);
}

// Adam step on st (parameters, moments, both bf16 copies)
void adam(don_trainer_s* t, const int* tstep) {
  WTab tab{};
  for (auto* L : {&t->bl, &t->tl})
    for (const Layer& y : *L) {
      tab.off[tab.n] = (long)y.offW;
      tab.offb[tab.n] = (long)y.offb;
      tab.Kp[tab.n] = y.Kp;
      tab.N[tab.n] = y.N;
      tab.tile0[tab.n + 1] = tab.tile0[tab.n] + (y.Kp / 64) * (y.N / 64);
      ++tab.n;
    }
  hipLaunchKernelGGL(k_adam, dim3(tab.tile0[tab.n] + tab.n), dim3(256), 0, t->st, (float*)t->master.ptr,
                     (const float*)t->grad.ptr, (float*)t->mom.ptr, (float*)t->var.ptr, (__bf16*)t->wbf.ptr,
                     (__bf16*)t->wtb.ptr, tab, t->lr, t->b1, t->b2, t->eps, tstep);
}

// st2 starts after the work queued so far on st; st continues after st2's work
void fork(don_trainer_s* t) {
  (void)hipEventRecord(t->ev_fork, t->st);
  (void)hipStreamWaitEvent(t->st2, t->ev_fork, 0);
}
void join(don_trainer_s* t) {
  (void)hipEventRecord(t->ev_join, t->st2);
  (void)hipStreamWaitEvent(t->st, t->ev_join, 0);
}

void train_step(don_trainer_s* t, bool update) {
  const int S = t->S, P = t->P, p = t->p;
  const int* ctr = (const int*)t->ctr.ptr;
  const int* idx = (const int*)t->idx.ptr;
  const Layer& b0 = t->bl[0];
  __bf16* Fb = (__bf16*)t->Fb.ptr;
  __bf16* FbT = (__bf16*)t->FbT.ptr;
  // the two MLPs are independent until the output product: branch on st2, trunk on st
  fork(t);
  hipLaunchKernelGGL(k_gather, dim3(grid_for(b0.Kp) < 64 ? grid_for(b0.Kp) : 64, S), dim3(256), 0, t->st2,
                     (const __bf16*)t->Fdata.ptr, (long)b0.Kp, idx, ctr, S, Fb, FbT);
  // branch: the wide input layer as a split-k product, the rest in one launch
  mlp_fwd(t, t->bl, Fb, S, t->ba, t->st2, (float*)t->bpart.ptr, 1);
  if (t->bl.size() > 1) mlp_fwd_fused(t, t->bl, Fb, S, t->ba, t->st2, 1);
  mlp_fwd_fused(t, t->tl, (const __bf16*)t->X.ptr, P, t->ta, t->st);
  join(t);
  const size_t lb = t->bl.size() - 1, lt = t->tl.size() - 1;
  const __bf16* Bout = (const __bf16*)t->ba.h.ptr + t->ba.off[lb];
  const __bf16* T = (const __bf16*)t->ta.h.ptr + t->ta.off[lt];
  const __bf16* TT = (const __bf16*)t->ta.hT.ptr + t->ta.off[lt];
  __bf16* Bc = (__bf16*)t->Bc.ptr;
  __bf16* BcT = (__bf16*)t->BcT.ptr;
  hipLaunchKernelGGL(k_to_bc, dim3((2 * S * p + 255) / 256), dim3(256), 0, t->st, Bout, S, p, Bc, BcT);
  // Ut = Bc T^T (2S x P)
  float* Ut = (float*)t->Ut.ptr;
  gemm(t->st, Bc, p, T, p, 2 * S, P, p, Ut, P, EP_F32);
  // loss and dUt
  const int chunk = 4096, nch = (P + chunk - 1) / chunk;
  hipLaunchKernelGGL(k_loss_part, dim3(nch, S), dim3(256), 0, t->st, (const float*)Ut, t->Y, idx, ctr, S, P, chunk,
                     (double*)t->lpart.ptr);
  hipLaunchKernelGGL(k_loss_final, dim3(1), dim3(256), 0, t->st, (const double*)t->lpart.ptr, S, nch, ctr,
                     (float*)t->wv.ptr, (float*)t->losses.ptr);
  __bf16* dUt = (__bf16*)t->dUt.ptr;
  __bf16* dUtT = (__bf16*)t->dUtT.ptr;
  hipLaunchKernelGGL(k_dU, dim3((P + 63) / 64), dim3(256), 0, t->st, (const float*)Ut, t->Y, idx, ctr,
                     (const float*)t->wv.ptr, S, P, dUt, dUtT);
  // dT = dUt^T Bc (P x p): A = dUt^T (P x 2S), B = Bc^T (p x 2S) -> dZ of the trunk's last layer
  gemm(t->st, dUtT, 2 * S, BcT, 2 * S, P, p, 2 * S, t->dz[0].ptr, p, EP_BF16, nullptr, nullptr,
       (__bf16*)t->dzT[0].ptr, P);
  // dBc = dUt T (2S x p): A = dUt (2S x P), B = T^T (p x P), reduction over the points
  float* dBc = (float*)t->dBc.ptr;
  gemm(t->st, dUt, P, TT, P, 2 * S, p, P, dBc, p, EP_F32, nullptr, nullptr, nullptr, 0, splits_for(2 * S, p, P, 128),
       (float*)t->part.ptr);
  hipLaunchKernelGGL(k_from_dbc, dim3((2 * S * p + 255) / 256), dim3(256), 0, t->st, (const float*)dBc, S, p,
                     (__bf16*)t->bdz[0].ptr, (__bf16*)t->bdzT[0].ptr);
  // trunk backward captured first (the long chain), the branch's beside it
  fork(t);
  mlp_bwd(t, t->tl, (const __bf16*)t->XT.ptr, P, t->ta, t->dz, t->dzT, t->st, (float*)t->part.ptr, t->st3);
  mlp_bwd(t, t->bl, FbT, S, t->ba, t->bdz, t->bdzT, t->st2, (float*)t->bpart.ptr);
  join(t);
  if (update) {
    adam(t, ctr + 1);
  }
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
  if (o->batch != 64 && o->batch != 128) return fail(HELM_E_INVAL, "don_train_create: batch %d must be 64 or 128", o->batch);
  if (o->n_points < 64 || o->n_points % 64)
    return fail(HELM_E_INVAL, "don_train_create: n_points must be a positive multiple of 64");
  if (o->max_steps < 1) return fail(HELM_E_INVAL, "don_train_create: max_steps < 1");
  if (net->p % 64) return fail(HELM_E_INVAL, "don_train_create: p must be a multiple of 64");
  for (size_t i = 1; i < net->bw.size(); ++i)
    if (net->bw[i] > 256 || net->bw[i] % 64)
      return fail(HELM_E_INVAL, "don_train_create: branch widths after the input must be multiples of 64, <= 256");
  for (size_t i = 1; i < net->tw.size(); ++i)
    if (net->tw[i] > 256 || net->tw[i] % 64)
      return fail(HELM_E_INVAL, "don_train_create: trunk widths after the input must be multiples of 64, <= 256");
  // the trunk runs in one fused launch, the branch's layers after its input layer in another
  if (net->bw.size() + net->tw.size() - 2 > (size_t)WT_MAX || net->tw.size() - 1 > (size_t)FW_MAXL ||
      net->bw.size() - 2 > (size_t)FW_MAXL)
    return fail(HELM_E_INVAL, "don_train_create: too many layers (%d in all, %d in the trunk, %d in the branch at most)",
                WT_MAX, FW_MAXL, FW_MAXL + 1);
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
      y.Kp = pad64(wd[i]);
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
  if (hipStreamCreateWithFlags(&t->st, hipStreamNonBlocking) != hipSuccess ||
      hipStreamCreateWithFlags(&t->st2, hipStreamNonBlocking) != hipSuccess ||
      hipStreamCreateWithFlags(&t->st3, hipStreamNonBlocking) != hipSuccess ||
      hipEventCreateWithFlags(&t->ev_rs, hipEventDisableTiming) != hipSuccess ||
      hipEventCreateWithFlags(&t->ev_rsj, hipEventDisableTiming) != hipSuccess ||
      hipEventCreateWithFlags(&t->ev_fork, hipEventDisableTiming) != hipSuccess ||
      hipEventCreateWithFlags(&t->ev_join, hipEventDisableTiming) != hipSuccess)
    return fin(fail(HELM_E_HIP, "don_train_create: streams and events"));
  const size_t S = t->S, P = t->P;
  auto acts = [&](Acts& a, std::vector<Layer>& L, size_t M) -> helm_status {
    size_t sum = 0;
    for (auto& y : L) {
      a.off.push_back(sum);
      sum += M * y.N;
    }
    helm_status e = a.h.ensure(2 * sum);
    return e ? e : a.hT.ensure(2 * sum);
  };
  int maxw = 0;
  for (auto* L : {&t->bl, &t->tl})
    for (auto& y : *L) maxw = std::max(maxw, y.N);
  size_t maxkn = 0;
  for (auto* L : {&t->bl, &t->tl})
    for (auto& y : *L) maxkn = std::max(maxkn, (size_t)y.Kp * y.N);
  // split-k partials: every split product runs at most 512 workgroups of 128 x 128 tiles
  (void)maxkn;
  t->part_floats = std::max<size_t>((size_t)512 * TM * TN, (size_t)2 * S * t->p * 512);
  const size_t nch = (P + 4095) / 4096;
  const size_t Kb = t->bl[0].Kp, Kt = t->tl[0].Kp;
  if ((s = t->master.ensure(4 * t->nparam)) || (s = t->grad.ensure(4 * t->nparam)) ||
      (s = t->mom.ensure(4 * t->nparam)) || (s = t->var.ensure(4 * t->nparam)) || (s = t->wbf.ensure(2 * t->nparam)) ||
      (s = t->wtb.ensure(2 * t->nparam)) || (s = t->X.ensure(2 * P * Kt)) || (s = t->XT.ensure(2 * P * Kt)) ||
      (s = t->Fb.ensure(2 * S * Kb)) || (s = t->FbT.ensure(2 * S * Kb)) || (s = acts(t->ba, t->bl, S)) ||
      (s = acts(t->ta, t->tl, P)))
    return fin(s);
  for (int k = 0; k < 2; ++k)
    if ((s = t->dz[k].ensure(2 * P * maxw)) || (s = t->dzT[k].ensure(2 * P * maxw)) ||
        (s = t->bdz[k].ensure(2 * S * std::max(maxw, 2 * t->p))) || (s = t->bdzT[k].ensure(2 * S * std::max(maxw, 2 * t->p))))
      return fin(s);
  if ((s = t->Bc.ensure(2 * 2 * S * t->p)) || (s = t->BcT.ensure(2 * 2 * S * t->p)) || (s = t->Ut.ensure(4 * 2 * S * P)) ||
      (s = t->dUt.ensure(2 * 2 * S * P)) || (s = t->dUtT.ensure(2 * 2 * S * P)) || (s = t->dBc.ensure(4 * 2 * S * t->p)) ||
      (s = t->part.ensure(4 * t->part_floats)) || (s = t->bpart.ensure(4 * t->part_floats)) || (s = t->lpart.ensure(8 * 2 * S * nch)) || (s = t->wv.ensure(4 * S)) ||
      (s = t->ctr.ensure(64)) || (s = t->losses.ensure(4 * (size_t)o->max_steps)) ||
      (s = t->idx.ensure(4 * (size_t)o->max_steps * S)))
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
  for (auto* L : {&t->bl, &t->tl})
    for (const Layer& y : *L)
      hipLaunchKernelGGL(k_transpose, dim3(grid_for((long)y.Kp * y.N)), dim3(256), 0, t->st, y.Kp, y.N,
                         (const __bf16*)t->wbf.ptr + y.offW, (__bf16*)t->wtb.ptr + y.offW);
  // trunk inputs: fp64 P x d -> bf16 padded rows and their transpose
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
      hipLaunchKernelGGL(k_pad_rows, dim3(grid_for((long)P * Kt)), dim3(256), 0, t->st, (long)P, t->d,
                         (const float*)tmp.ptr, (int)Kt, (__bf16*)t->X.ptr, (__bf16*)t->XT.ptr);
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
  helm_status s = sync(t, "don_train_data");  // no step may still read the old data
  if (s) return s;
  const void* oldF = t->Fdata.ptr;
  if ((s = t->Fdata.ensure((size_t)2 * n * b0.Kp))) return s;
  // the captured step graphs hold the data pointers as kernel arguments:
  // record them again when either moved
  if (t->Fdata.ptr != oldF || (const float2*)Y != t->Y) {
    if (t->step_exec) (void)hipGraphExecDestroy(t->step_exec);
    if (t->multi_exec) (void)hipGraphExecDestroy(t->multi_exec);
    t->step_exec = t->multi_exec = nullptr;
  }
  hipLaunchKernelGGL(k_pad_rows, dim3(grid_for((long)n * b0.Kp)), dim3(256), 0, t->st, (long)n, b0.K, F, b0.Kp,
                     (__bf16*)t->Fdata.ptr, (__bf16*)nullptr);
  t->Y = (const float2*)Y;
  t->ndata = n;
  return sync(t, "don_train_data");
}

static constexpr int GRAPH_STEPS = 8;

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
    // steps are captured once as graphs of one and of GRAPH_STEPS steps; the
    // sample indices and the step counter live on the device
    auto capture = [&](int steps, hipGraphExec_t* out) -> helm_status {
      hipGraph_t g;
      helm_status s2 = sync(t, "don_train: capture");
      if (s2) return s2;
      if (hipStreamBeginCapture(t->st, hipStreamCaptureModeThreadLocal) != hipSuccess)
        return fail(HELM_E_HIP, "don_train: begin capture");
      for (int k = 0; k < steps; ++k) train_step(t, true);
      hipError_t e2 = hipStreamEndCapture(t->st, &g);
      if (e2 != hipSuccess) return hip_fail(e2, "don_train: end capture");
      e2 = hipGraphInstantiate(out, g, nullptr, nullptr, 0);
      (void)hipGraphDestroy(g);
      return e2 == hipSuccess ? HELM_OK : hip_fail(e2, "don_train: instantiate");
    };
    if (!t->step_exec && (s = capture(1, &t->step_exec))) return s;
    if (count >= GRAPH_STEPS && !t->multi_exec && (s = capture(GRAPH_STEPS, &t->multi_exec))) return s;
    int k = 0;
    for (; k + GRAPH_STEPS <= count; k += GRAPH_STEPS) {
      e = hipGraphLaunch(t->multi_exec, t->st);
      if (e != hipSuccess) return hip_fail(e, "don_train: replay");
    }
    for (; k < count; ++k) {
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
  adam(t, ctr + 1);
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
  if (net->dt == HELM_C64)  // the fp64 trunk copies hold the same (fp32) values
    for (size_t i = 0; i < t->tl.size(); ++i) {
      const Layer& y = t->tl[i];
      hipLaunchKernelGGL(k_cvt_back<double>, dim3(grid_for((long)y.K * y.N)), dim3(256), 0, t->st, y.K, y.N,
                         m + y.offW, (double*)net->tW64[i]);
      hipLaunchKernelGGL(k_cvt_back<double>, dim3(1), dim3(256), 0, t->st, 1, y.N, m + y.offb, (double*)net->tB64[i]);
    }
  helm_status s = sync(t, "don_train_export");
  if (s) return s;
  don_touch(net);
  return launch_check("don_train_export");
}

void don_train_free(don_trainer t) { delete t; }

}  // extern "C"
