// Shared device helpers for libhelm's gfx950 kernels: complex arithmetic on
// double2 (all arithmetic is fp64, storage is fp32 or fp64), storage-type
// loads/stores, XCD-aware block remapping and wavefront reductions.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>
#include <stddef.h>

#ifndef HELM_WAVE
#define HELM_WAVE 64
#endif

// Complex storage type for a real storage type S.
template <typename S> struct cvec;
template <> struct cvec<double> { using type = double2; };
template <> struct cvec<float> { using type = float2; };
template <typename S> using cplx_t = typename cvec<S>::type;

__device__ __forceinline__ double2 ldc(const double2* p, size_t i) { return p[i]; }
__device__ __forceinline__ double2 ldc(const float2* p, size_t i) {
  float2 v = p[i];
  return make_double2((double)v.x, (double)v.y);
}
__device__ __forceinline__ void stc(double2* p, size_t i, double2 v) { p[i] = v; }
__device__ __forceinline__ void stc(float2* p, size_t i, double2 v) {
  p[i] = make_float2((float)v.x, (float)v.y);
}
__device__ __forceinline__ double ldr(const double* p, size_t i) { return p[i]; }
__device__ __forceinline__ double ldr(const float* p, size_t i) { return (double)p[i]; }

__device__ __forceinline__ double2 cadd(double2 a, double2 b) { return make_double2(a.x + b.x, a.y + b.y); }
__device__ __forceinline__ double2 csub(double2 a, double2 b) { return make_double2(a.x - b.x, a.y - b.y); }
__device__ __forceinline__ double2 cmul(double2 a, double2 b) {
  return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
// conj(a) * b
__device__ __forceinline__ double2 cconjmul(double2 a, double2 b) {
  return make_double2(a.x * b.x + a.y * b.y, a.x * b.y - a.y * b.x);
}
__device__ __forceinline__ double2 cscale(double2 a, double s) { return make_double2(a.x * s, a.y * s); }
__device__ __forceinline__ double2 cdiv(double2 a, double2 b) {
  // Smith's scaled division: avoids overflow of |b|^2 for large |b|
  if (fabs(b.x) >= fabs(b.y)) {
    double r = b.y / b.x, d = b.x + b.y * r;
    return make_double2((a.x + a.y * r) / d, (a.y - a.x * r) / d);
  } else {
    double r = b.x / b.y, d = b.y + b.x * r;
    return make_double2((a.x * r + a.y) / d, (a.y * r - a.x) / d);
  }
}
__device__ __forceinline__ double2 czero() { return make_double2(0.0, 0.0); }
// r / d for a relaxation update, d = D_p the diagonal of A (1 on scatterer
// nodes, sum_a 2/h_a^2 - s_p elsewhere: far from zero and from overflow):
// one reciprocal of |d|^2, then r conj(d) / |d|^2 (a few ulps, as Smith's
// division, with one fp64 division instead of three)
__device__ __forceinline__ double2 ddiv(double2 r, double2 d) {
  const double inv = 1.0 / (d.x * d.x + d.y * d.y);
  return make_double2((r.x * d.x + r.y * d.y) * inv, (r.y * d.x - r.x * d.y) * inv);
}

// Workgroup b of a launch is dispatched to XCD b % 8.  Remap the hardware block
// id so that each XCD receives one contiguous range of logical blocks: stencil
// neighbours and reused rows then stay in that XCD's L2.
__device__ __forceinline__ unsigned xcd_remap(unsigned bid, unsigned nblocks) {
  const unsigned nx = 8;
  unsigned x = bid % nx, local = bid / nx;
  unsigned full = nblocks / nx, rem = nblocks % nx;
  return x * full + (x < rem ? x : rem) + local;
}

// Sum over a wavefront (64 lanes); every lane gets the total.  Fixed order.
__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

// Deterministic block sum of one double per thread (blockDim.x threads, a
// multiple of 64, at most 1024).  `sh` holds 16 doubles.  Result valid in
// thread 0.
__device__ __forceinline__ double block_sum(double v, double* sh) {
  v = wave_sum(v);
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  if (lane == 0) sh[w] = v;
  __syncthreads();
  double t = 0.0;
  if (threadIdx.x == 0) {
    const int nw = blockDim.x >> 6;
    for (int i = 0; i < nw; ++i) t += sh[i];
  }
  __syncthreads();
  return t;
}

__device__ __forceinline__ double2 block_sum2(double2 v, double* sh) {
  v.x = wave_sum(v.x);
  v.y = wave_sum(v.y);
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  if (lane == 0) {
    sh[2 * w] = v.x;
    sh[2 * w + 1] = v.y;
  }
  __syncthreads();
  double2 t = czero();
  if (threadIdx.x == 0) {
    const int nw = blockDim.x >> 6;
    for (int i = 0; i < nw; ++i) {
      t.x += sh[2 * i];
      t.y += sh[2 * i + 1];
    }
  }
  __syncthreads();
  return t;
}
