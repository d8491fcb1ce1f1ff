// Small dense GMRES work on the device: completion of an Arnoldi column
// (CGS2 coefficients, complex Givens rotations, residual estimate) and the
// upper-triangular back-solve.  O(m) / O(m^2) work in fp64, one thread: the
// host never touches H, so a cycle needs no host round trip except the
// convergence flag.  Restart lengths up to 1000 are supported.
#include "common.h"
#include "internal.h"

namespace helm {

__device__ static inline double2 H_at(const double* H, int m, int i, int j) {
  const size_t o = 2 * ((size_t)j * (m + 1) + i);
  return make_double2(H[o], H[o + 1]);
}
__device__ static inline void H_set(double* H, int m, int i, int j, double2 v) {
  const size_t o = 2 * ((size_t)j * (m + 1) + i);
  H[o] = v.x;
  H[o + 1] = v.y;
}
__device__ static inline double cabs2(double2 a) { return hypot(a.x, a.y); }

// Value held by lane `src` (uniform index) of the wavefront.
__device__ static inline double lane_read(double v, int src) {
  const long long b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_readlane((int)(b & 0xffffffffLL), src);
  const int hi = __builtin_amdgcn_readlane((int)(b >> 32), src);
  return __longlong_as_double(((long long)hi << 32) | (unsigned)lo);
}

// One wavefront: the new column (CGS2 coefficients h1 + h2, or h1 alone when h2
// is NULL) and the previous
// rotations are staged in LDS and, for the first 64 rows, in the lanes'
// registers; lane 0 applies the rotations (inherently sequential), and the
// column is written back in parallel.
__global__ __launch_bounds__(64) void k_arnoldi_finish(int j, int m, double* H, double* g, double* cs, double* sn,
                                                       const double* h1, const double* h2, const double* npart,
                                                       int nparts, GmState* gs, GmState* ghost) {
  __shared__ double col[2 * 1002];
  __shared__ double rc[1001], rs[2 * 1001];
  const int l = threadIdx.x;
  // ||w||^2 from the per-block partials of the last CGS update (fixed order)
  // (sixteen loads per lane in flight at once, then added in index order)
  double ns = 0.0;
  for (int b0 = 0; b0 < nparts; b0 += 16 * 64) {
    double v[16];
#pragma unroll
    for (int q = 0; q < 16; ++q) {
      const int b = b0 + l + 64 * q;
      v[q] = b < nparts ? npart[b] : 0.0;
    }
#pragma unroll
    for (int q = 0; q < 16; ++q) ns += v[q];
  }
  ns = wave_sum(ns);
  // h2 == NULL: one Gram-Schmidt pass, the column is h1 alone
  for (int i = l; i <= j; i += 64) {
    col[2 * i] = h2 ? h1[2 * i] + h2[2 * i] : h1[2 * i];
    col[2 * i + 1] = h2 ? h1[2 * i + 1] + h2[2 * i + 1] : h1[2 * i + 1];
  }
  for (int i = l; i < j; i += 64) {
    rc[i] = cs[i];
    rs[2 * i] = sn[2 * i];
    rs[2 * i + 1] = sn[2 * i + 1];
  }
  // lane q also keeps entry q + 1 of the column and rotation q in registers:
  // the first 64 steps of the rotation chain read them with v_readlane
  double2 bq = czero();
  if (l + 1 <= j)
    bq = h2 ? make_double2(h1[2 * (l + 1)] + h2[2 * (l + 1)], h1[2 * (l + 1) + 1] + h2[2 * (l + 1) + 1])
            : make_double2(h1[2 * (l + 1)], h1[2 * (l + 1) + 1]);
  double cq = l < j ? cs[l] : 0.0;
  double2 sq = l < j ? make_double2(sn[2 * l], sn[2 * l + 1]) : czero();
  // lane 0 alone reads these per-lane values (v_readlane) below: pin them in
  // every lane's registers here, so that no part of their computation can be
  // moved into the lane-0 branch
  __asm__ volatile("" : "+v"(bq.x), "+v"(bq.y), "+v"(cq), "+v"(sq.x), "+v"(sq.y));
  __syncthreads();
  if (l == 0) {
    const double hn = sqrt(ns);
    gs->hn = hn;
    gs->inv_hn = hn != 0.0 ? 1.0 / hn : 0.0;
    // previous rotations G_i = [[c, s], [-conj(s), c]] on rows (i, i+1); the
    // running entry t (row i after rotations 0..i-1) stays in registers, so
    // the dependent chain never waits on LDS
    double2 t = make_double2(col[0], col[1]);
    for (int i = 0; i < j; ++i) {
      double2 b, s;
      double c;
      if (i < 64) {
        b = make_double2(lane_read(bq.x, i), lane_read(bq.y, i));
        c = lane_read(cq, i);
        s = make_double2(lane_read(sq.x, i), lane_read(sq.y, i));
      } else {
        b = make_double2(col[2 * i + 2], col[2 * i + 3]);
        c = rc[i];
        s = make_double2(rs[2 * i], rs[2 * i + 1]);
      }
      const double2 sconj = make_double2(s.x, -s.y);
      const double2 na = cadd(cscale(t, c), cmul(s, b));
      t = csub(cscale(b, c), cmul(sconj, t));
      col[2 * i] = na.x;
      col[2 * i + 1] = na.y;
    }
    const double2 a = t;
    const double b = hn;
    double c;
    double2 s;
    if (b == 0.0) {
      c = 1.0;
      s = czero();
    } else if (a.x == 0.0 && a.y == 0.0) {
      c = 0.0;
      s = make_double2(1.0, 0.0);
    } else {
      const double aa = cabs2(a);
      const double nu = sqrt(aa * aa + b * b);
      c = aa / nu;
      s = cscale(make_double2(a.x / aa, a.y / aa), b / nu);
    }
    cs[j] = c;
    sn[2 * j] = s.x;
    sn[2 * j + 1] = s.y;
    const double2 hjj = cadd(cscale(a, c), cscale(s, b));
    col[2 * j] = hjj.x;
    col[2 * j + 1] = hjj.y;
    col[2 * (j + 1)] = 0.0;
    col[2 * (j + 1) + 1] = 0.0;
    const double2 gj = make_double2(g[2 * j], g[2 * j + 1]);
    const double2 gn = cmul(make_double2(-s.x, s.y), gj);  // -conj(s) g_j
    g[2 * (j + 1)] = gn.x;
    g[2 * (j + 1) + 1] = gn.y;
    g[2 * j] = c * gj.x;
    g[2 * j + 1] = c * gj.y;
    gs->gabs = cabs2(gn);
    gs->flag = (isfinite(hn) && isfinite(gs->gabs)) ? 0 : -5;
    gs->step = j;
    // the host reads this copy (pinned host memory) after synchronizing on an
    // event recorded behind the kernel; that event carries no system-scope
    // release (one at every Arnoldi step cost several microseconds), so the
    // kernel makes these writes visible to the host itself
    ghost->gabs = gs->gabs;
    ghost->hn = hn;
    ghost->inv_hn = gs->inv_hn;
    ghost->flag = gs->flag;
    ghost->step = j;
    __threadfence_system();
  }
  __syncthreads();
  for (int i = l; i <= j + 1; i += 64) H_set(H, m, i, j, make_double2(col[2 * i], col[2 * i + 1]));
}

// Back substitution H[:k,:k] y = g, one wavefront: row i's dot product is
// split over lanes and summed with shuffles, lane 0 forms y_i.  y lives in LDS;
// the upper triangle of H is staged in LDS too when it fits (k <= 76, packed
// rows), otherwise it is read from global memory.
constexpr int BS_LDS_MAX = 76;
__device__ static inline int tri(int k, int i, int c) { return i * k - (i * (i - 1)) / 2 + (c - i); }

__global__ __launch_bounds__(64) void k_backsolve(int k, int m, const double* H, const double* g, double* y) {
  extern __shared__ double lds[];
  double* ys = lds;           // 2k
  double* hl = lds + 2 * k;   // packed upper triangle, k(k+1)/2 complex
  const int l = threadIdx.x;
  const bool staged = k <= BS_LDS_MAX;
  if (staged)
    // the k x k square in batches of 8 entries per lane: the loads of a batch are
    // in flight together before any of them is stored (entries below the
    // diagonal are skipped)
    for (int e0 = 0; e0 < k * k; e0 += 8 * 64) {
      double2 v[8];
#pragma unroll
      for (int q = 0; q < 8; ++q) {
        const int e = e0 + l + 64 * q, i = e / k, c = e % k;
        v[q] = (e < k * k && c >= i) ? H_at(H, m, i, c) : czero();
      }
#pragma unroll
      for (int q = 0; q < 8; ++q) {
        const int e = e0 + l + 64 * q, i = e / k, c = e % k;
        if (e < k * k && c >= i) {
          const int o = tri(k, i, c);
          hl[2 * o] = v[q].x;
          hl[2 * o + 1] = v[q].y;
        }
      }
    }
  __syncthreads();
  for (int i = k - 1; i >= 0; --i) {
    double2 acc = czero();
    for (int c = i + 1 + l; c < k; c += 64) {
      const int o = tri(k, i, c);
      const double2 h = staged ? make_double2(hl[2 * o], hl[2 * o + 1]) : H_at(H, m, i, c);
      acc = cadd(acc, cmul(h, make_double2(ys[2 * c], ys[2 * c + 1])));
    }
    acc.x = wave_sum(acc.x);
    acc.y = wave_sum(acc.y);
    if (l == 0) {
      const int o = tri(k, i, i);
      const double2 hii = staged ? make_double2(hl[2 * o], hl[2 * o + 1]) : H_at(H, m, i, i);
      const double2 v = cdiv(csub(make_double2(g[2 * i], g[2 * i + 1]), acc), hii);
      ys[2 * i] = v.x;
      ys[2 * i + 1] = v.y;
    }
    __syncthreads();
  }
  for (int i = l; i < k; i += 64) {
    y[2 * i] = ys[2 * i];
    y[2 * i + 1] = ys[2 * i + 1];
  }
}

// cycle start from the reduced ||r||^2 in nrm[0]: g = beta e_1 and
// nrm[2] = 1 / beta (0 when beta is 0 or not finite; the host then abandons
// the cycle); ||r||^2 and nrm[1] go to the host record rec (pinned host
// memory, made visible by the kernel itself as in k_arnoldi_finish)
__global__ void k_gmres_start(double* nrm, double* g, int m, double* rec) {
  const double b2 = nrm[0];
  const double beta = sqrt(b2);
  for (int i = threadIdx.x; i < 2 * (m + 1); i += blockDim.x) g[i] = i == 0 ? beta : 0.0;
  if (threadIdx.x == 0) {
    nrm[2] = (beta > 0.0 && isfinite(beta)) ? 1.0 / beta : 0.0;
    rec[0] = b2;
    rec[1] = nrm[1];
    __threadfence_system();
  }
}

void arnoldi_finish(int j, int m, double* H, double* g, double* cs, double* sn, const double* h1, const double* h2,
                    const double* npart, int nparts, GmState* gs, GmState* ghost, hipStream_t st) {
  hipLaunchKernelGGL(k_arnoldi_finish, dim3(1), dim3(64), 0, st, j, m, H, g, cs, sn, h1, h2, npart, nparts, gs, ghost);
}
void gmres_backsolve(int k, int m, const double* H, const double* g, double* y, hipStream_t st) {
  const size_t lds = sizeof(double) * 2 * ((size_t)k + (k <= BS_LDS_MAX ? (size_t)k * (k + 1) / 2 : 0));
  hipLaunchKernelGGL(k_backsolve, dim3(1), dim3(64), lds, st, k, m, H, g, y);
}
void gmres_start(double* nrm, double* g, int m, double* rec, hipStream_t st) {
  hipLaunchKernelGGL(k_gmres_start, dim3(1), dim3(256), 0, st, nrm, g, m, rec);
}

}  // namespace helm
