// Device bodies of the skinny products of the trunk-basis correction (App. C),
// shared by the single-grid kernels and the batched ones:
//   qt_rows      partials of Q^T x over a row range: lanes own columns {l, l+64},
//                wavefronts stride over rows, one coalesced row read per step;
//   skinny_rows  y_i = sum_j Q_ij c_j: lanes own columns, four rows per step,
//                reduced with an 11-shuffle butterfly that leaves row rho's
//                (re, im) in lane 16 rho.
#pragma once

#include "common.h"

namespace helm {

// basis loads are streaming (each Q value is read once per pass and the basis
// is larger than the caches): non-temporal, so they do not push the Krylov
// vectors out of L2 and the memory-side cache
template <typename T> __device__ __forceinline__ double ldq(const T* q, size_t i) {
  return (double)__builtin_nontemporal_load(q + i);
}

// part[b][2j + {0,1}] = sum_{i in block b} Q_ij x_i  (complex x, real Q, j < r <= 128)
// One 256-thread workgroup: rows [i0, i1); out[2j + {0,1}] for j < r.
template <typename T, typename S>
__device__ __forceinline__ void qt_rows(int r, const T* __restrict__ Q, const cplx_t<S>* __restrict__ x, size_t i0,
                                        size_t i1, double* __restrict__ out) {
  __shared__ double sh[4][256];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int c0 = lane, c1 = lane + 64;
  const bool u0 = c0 < r, u1 = c1 < r;
  double a0r = 0, a0i = 0, a1r = 0, a1i = 0;
  size_t i = i0 + wave;
  for (; i + 12 < i1; i += 16) {
    double q0[4], q1[4];
    double2 xv[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const size_t ii = i + 4 * u;
      xv[u] = ldc(x, ii);
      q0[u] = u0 ? ldq(Q, ii * r + c0) : 0.0;
      q1[u] = u1 ? ldq(Q, ii * r + c1) : 0.0;
    }
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      a0r += q0[u] * xv[u].x;
      a0i += q0[u] * xv[u].y;
      a1r += q1[u] * xv[u].x;
      a1i += q1[u] * xv[u].y;
    }
  }
  for (; i < i1; i += 4) {
    const double2 xv = ldc(x, i);
    const double q0 = u0 ? ldq(Q, i * r + c0) : 0.0;
    const double q1 = u1 ? ldq(Q, i * r + c1) : 0.0;
    a0r += q0 * xv.x;
    a0i += q0 * xv.y;
    a1r += q1 * xv.x;
    a1i += q1 * xv.y;
  }
  sh[wave][2 * c0] = a0r;
  sh[wave][2 * c0 + 1] = a0i;
  sh[wave][2 * c1] = a1r;
  sh[wave][2 * c1 + 1] = a1i;
  __syncthreads();
  for (int e = threadIdx.x; e < 2 * r; e += blockDim.x)
    out[e] = (sh[0][e] + sh[1][e]) + (sh[2][e] + sh[3][e]);
}

enum { SK_ADD = 0, SK_SYNTH = 1 };

// y_i = sum_j Q_ij c_j (complex c).  SK_ADD: z_i += y_i.  SK_SYNTH: z_i = scal[0] *
// y_i, or 0 on masked nodes (scal = s of the DeepONet scaling).
// Wavefront wave_g of nwaves covering rows 0..n-1, four rows per step.
template <typename T, typename S, int MODE>
__device__ __forceinline__ void skinny_rows(size_t n, int r, const T* __restrict__ Q, const double* __restrict__ c,
                                            cplx_t<S>* __restrict__ z, const uint8_t* __restrict__ mask,
                                            const double* __restrict__ scal, size_t wave_g, size_t nwaves) {
  const int lane = threadIdx.x & 63;
  const int c0 = lane, c1 = lane + 64;
  const double2 cc0 = c0 < r ? make_double2(c[2 * c0], c[2 * c0 + 1]) : czero();
  const double2 cc1 = c1 < r ? make_double2(c[2 * c1], c[2 * c1 + 1]) : czero();
  double sc = 1.0;
  if (MODE == SK_SYNTH) sc = scal[0];
  const int b5 = (lane >> 5) & 1, b4 = (lane >> 4) & 1, b3 = (lane >> 3) & 1;
  for (size_t i = wave_g * 4; i < n; i += nwaves * 4) {
    double v[8];
#pragma unroll
    for (int rho = 0; rho < 4; ++rho) {
      const size_t ii = i + rho;
      double q0 = 0.0, q1 = 0.0;
      if (ii < n) {
        if (c0 < r) q0 = ldq(Q, ii * r + c0);
        if (c1 < r) q1 = ldq(Q, ii * r + c1);
      }
      v[2 * rho] = q0 * cc0.x + q1 * cc1.x;
      v[2 * rho + 1] = q0 * cc0.y + q1 * cc1.y;
    }
    // butterfly: after step k each lane keeps half of its remaining values
    double w4[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const double send = v[4 * (1 - b5) + q];
      w4[q] = v[4 * b5 + q] + __shfl_xor(send, 32, 64);
    }
    double w2[2];
#pragma unroll
    for (int q = 0; q < 2; ++q) {
      const double send = w4[2 * (1 - b4) + q];
      w2[q] = w4[2 * b4 + q] + __shfl_xor(send, 16, 64);
    }
    double w1;
    {
      const double send = w2[1 - b3];
      w1 = w2[b3] + __shfl_xor(send, 8, 64);
    }
    w1 += __shfl_xor(w1, 4, 64);
    w1 += __shfl_xor(w1, 2, 64);
    w1 += __shfl_xor(w1, 1, 64);
    // lane holds value index 4 b5 + 2 b4 + b3 = 2 rho + comp
    const double other = __shfl_xor(w1, 8, 64);
    if ((lane & 15) == 0) {
      const size_t ii = i + 2 * b5 + b4;
      if (ii < n) {
        const double2 y = make_double2(w1, other);  // b3 == 0: w1 = re, other = im
        if (MODE == SK_ADD) {
          stc(z, ii, cadd(ldc(z, ii), y));
        } else {
          stc(z, ii, mask[ii] ? czero() : cscale(y, sc));
        }
      }
    }
  }
}

}  // namespace helm
