// DeepONet inference (App. B architecture; App. C trunk matrix).
//
// Trunk: the coordinate input layer is evaluated directly from node indices
// (no coordinate array), the hidden and output layers are fp64 MFMA GEMMs with
// fused bias + activation (both dtypes), row-chunked so the activations stay
// within a bounded buffer at any grid size.  The result T (n x p) is what the trunk-basis
// coarse space and the output synthesis consume.
//
// Full correction du = s N(r / s):  ||r|| (two-stage reduction) -> branch input
// (scaled residual, identity or multilinear resampling onto the branch grid, k
// appended) -> branch layers (split-K GEMV, batch 1 or 2) -> coefficients
// c = b_re + i b_im -> du_i = s sum_j T_ij c_j, zero on scatterer nodes.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <cstring>
#include <cmath>
#include <vector>

#include "common.h"
#include "dense.h"
#include "internal.h"
#include "lib.h"

namespace helm {

static std::atomic<int> g_serial{1};

int don_p(const don_s* net) { return net->p; }
int don_serial(const don_s* net) { return net->serial; }
void don_touch(don_s* net) { net->serial = g_serial.fetch_add(1); }

static int map_act(int a) { return a == DON_TANH ? ACT_TANH : a == DON_RELU ? ACT_RELU : ACT_LEAKY; }

helm_status check_net_for_op(const don_s* net, const helm_op_s* op, int p_used) {
  if (!net) return fail(HELM_E_INVAL, "network is NULL");
  if (net->dt != op->dt) return fail(HELM_E_INVAL, "network dtype %d does not match the op's %d", net->dt, op->dt);
  if (net->tw[0] != op->dim)
    return fail(HELM_E_INVAL, "trunk input width %d does not match grid dimension %d", net->tw[0], op->dim);
  if (op->dim == 2 && net->bgrid[2] != 1) return fail(HELM_E_INVAL, "2D op needs branch_grid[2] = 1");
  if (p_used < 1 || p_used > net->p) return fail(HELM_E_INVAL, "p_used = %d outside [1, %d]", p_used, net->p);
  if ((size_t)p_used > op->nn) return fail(HELM_E_INVAL, "p_used = %d exceeds the node count", p_used);
  return HELM_OK;
}

// ---- kernels ----------------------------------------------------------------------
// s = sqrt(ss / n) and 1/s (0 when s = 0), from the reduced ||r||^2
__global__ void k_scale_of(const double* ss, double n, double* out) {
  if (threadIdx.x == 0 && blockIdx.x == 0) {
    const double s = sqrt(ss[0] / n);
    out[0] = s;
    out[1] = s > 0.0 ? 1.0 / s : 0.0;
  }
}

// branch input, identity sampling: x[0][i] = Re r_i / s, x[1][i] = Im r_i / s
// (SPLIT_INPUT) or x[0][i], x[0][n + i] (SPLIT_OUTPUT); optional k at x[0][2n]
template <typename T, typename S>
__global__ void k_branch_in_identity(size_t n, const cplx_t<S>* __restrict__ r, const double* __restrict__ sv,
                                     int split_input, int k_input, double k, T* __restrict__ x) {
  const double inv = sv[1];
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x) {
    const double2 v = ldc(r, i);
    const size_t off = split_input ? n : n;
    x[i] = (T)(v.x * inv);
    x[off + i] = (T)(v.y * inv);
    if (!split_input && k_input && i == 0) x[2 * n] = (T)k;
  }
}

// branch input by multilinear interpolation onto the branch grid (zero ghosts):
// x[0][j] = sample(Re r / s), x[0][m + j] = sample(Im r / s), x[0][2m] = k
template <typename T, typename S>
__global__ void k_branch_in_sample(int dim, int nx, int ny, int nz, int mx, int my, int mz,
                                   const cplx_t<S>* __restrict__ r, const double* __restrict__ sv, int split_input,
                                   int k_input, double k, T* __restrict__ x) {
  const size_t m = (size_t)mx * my * mz;
  const double inv = sv[1];
  const int ns[3] = {nx, ny, nz}, mt[3] = {mx, my, mz};
  for (size_t j = blockIdx.x * (size_t)blockDim.x + threadIdx.x; j < m; j += (size_t)gridDim.x * blockDim.x) {
    const int jj[3] = {(int)(j % mx), (int)((j / mx) % my), (int)(j / ((size_t)mx * my))};
    int i0[3];
    double w[3];
    for (int a = 0; a < 3; ++a) {
      if (a < dim && mt[a] != ns[a]) {
        const double xt = (double)(jj[a] + 1) / (double)(mt[a] + 1);
        const double t = __dmul_rn(xt, (double)(ns[a] + 1)) - 1.0;
        i0[a] = (int)floor(t);
        w[a] = t - i0[a];
      } else {
        i0[a] = jj[a];
        w[a] = 0.0;
      }
    }
    double2 acc = czero();
    const int nc = 1 << dim;
    for (int cidx = 0; cidx < nc; ++cidx) {
      double wt = 1.0;
      int idx[3] = {0, 0, 0};
      bool inside = true;
      for (int a = 0; a < 3; ++a) {
        const int bit = a < dim ? (cidx >> a) & 1 : 0;
        idx[a] = i0[a] + bit;
        wt *= bit ? w[a] : 1.0 - w[a];
        if (a < dim && (idx[a] < 0 || idx[a] >= ns[a])) inside = false;
      }
      if (!inside || wt == 0.0) continue;
      const size_t p = (size_t)idx[0] + (size_t)nx * ((size_t)idx[1] + (size_t)ny * idx[2]);
      const double2 v = ldc(r, p);
      acc.x += wt * v.x;
      acc.y += wt * v.y;
    }
    const size_t off = m;
    x[j] = (T)(acc.x * inv);
    x[off + j] = (T)(acc.y * inv);
    if (!split_input && k_input && j == 0) x[2 * m] = (T)k;
  }
}

// coefficients c_j = b_re_j + i b_im_j (fp64)
template <typename T>
__global__ void k_coef(int p, int split_input, const T* __restrict__ b, double* __restrict__ c) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= p) return;
  c[2 * j] = (double)b[j];
  c[2 * j + 1] = split_input ? (double)b[p + j] : (double)b[p + j];
}

// fp64 trunk rows rounded once to the stored fp32 trunk matrix (C64)
__global__ void k_narrow(size_t cnt, const double* __restrict__ src, float* __restrict__ dst) {
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < cnt; i += (size_t)gridDim.x * blockDim.x)
    dst[i] = (float)src[i];
}

// ---- drivers -------------------------------------------------------------------------
// The trunk matrix is evaluated in fp64 arithmetic for both dtypes (a C64
// network's fp32 weights widened exactly): the basis of App. C is set-up
// algebra, and an fp32 evaluation's few-ulp errors per layer (about 5e-7 of T
// at the 3D trunk) reach the meta-solver's iterate amplified.  A C64 trunk
// matrix is rounded to fp32 once, as it is stored.
template <typename T>
static helm_status trunk_eval(don_s* net, helm_op_s* op, T* out, hipStream_t st) {
  constexpr bool wide = sizeof(T) == sizeof(double);
  const size_t n = op->nn;
  const int L = (int)net->tw.size() - 1;
  int maxw = 1;
  for (int w : net->tw) maxw = w > maxw ? w : maxw;
  const size_t chunk = n < (size_t)262144 ? n : (size_t)262144;
  helm_status s;
  if ((s = net->tact0.ensure(chunk * maxw * sizeof(double))) ||
      (s = net->tact1.ensure(chunk * maxw * sizeof(double))))
    return s;
  const std::vector<void*>& W = wide ? net->tW : net->tW64;
  const std::vector<void*>& B = wide ? net->tB : net->tB64;
  const int act = map_act(net->act);
  const int p = net->p;
  for (size_t r0 = 0; r0 < n; r0 += chunk) {
    const size_t rc = n - r0 < chunk ? n - r0 : chunk;
    double* h[2] = {(double*)net->tact0.ptr, (double*)net->tact1.ptr};
    // the last layer writes the stored matrix directly (C128) or a scratch chunk
    auto last_out = [&](int slot) { return wide ? (double*)(void*)(out + r0 * p) : h[slot]; };
    double* o = L == 1 ? last_out(1) : h[0];
    coord_layer<double>(op->dim, op->n, r0, rc, (const double*)W[0], (const double*)B[0], net->tw[1],
                        L == 1 ? ACT_NONE : act, o, st);
    int cur = 0;
    for (int l = 1; l < L; ++l) {
      const bool last = l == L - 1;
      o = last ? last_out(1 - cur) : h[1 - cur];
      gemm<double>((int)rc, net->tw[l + 1], net->tw[l], h[cur], net->tw[l], (const double*)W[l], net->tw[l + 1],
                   (const double*)B[l], last ? ACT_NONE : act, o, net->tw[l + 1], st);
      cur = 1 - cur;
    }
    if (!wide) {
      const size_t cnt = rc * (size_t)p;
      hipLaunchKernelGGL(k_narrow, dim3((unsigned)std::min<size_t>((cnt + 255) / 256, 16384)), dim3(256), 0, st, cnt,
                         o, (float*)(void*)(out + r0 * p));
    }
  }
  return launch_check("trunk");
}

helm_status don_trunk(don_s* net, helm_op_s* op, void* out, hipStream_t st) {
  return net->dt == HELM_C128 ? trunk_eval<double>(net, op, (double*)out, st)
                              : trunk_eval<float>(net, op, (float*)out, st);
}

static bool same_grid(const don_s* net, const helm_op_s* op) {
  for (int a = 0; a < 3; ++a)
    if (net->bgrid[a] != op->n[a]) return false;
  return true;
}

template <typename T>
static helm_status full_eval(don_s* net, helm_op_s* op, const void* r, double k, void* du, hipStream_t st,
                             bool input_only = false) {
  const size_t n = op->nn;
  Coarse& c = op->coarse;
  helm_status s;
  if (!input_only && c.T_serial != net->serial) {
    if ((s = c.T.ensure(n * (size_t)net->p * sizeof(T)))) return s;
    if ((s = trunk_eval<T>(net, op, (T*)c.T.ptr, st))) return s;
    c.T_serial = net->serial;
  }
  // s = ||r|| / sqrt(n)
  double* part;
  const int nb = red_nblocks(n);
  if ((s = op_part(op, (size_t)nb, &part))) return s;
  nrm2_part<T>(n, r, part, st);
  double* sv = op->red + 3072;  // [ss, s, 1/s]
  reduce_cols(part, nb, 1, sv, st);
  hipLaunchKernelGGL(k_scale_of, dim3(1), dim3(64), 0, st, sv, (double)n, sv + 1);
  const double* sc = sv + 1;
  // branch input
  const int B = net->head == DON_SPLIT_INPUT ? 2 : 1;
  const int K0 = net->bw[0];
  int maxw = 1;
  for (int w : net->bw) maxw = w > maxw ? w : maxw;
  if ((s = net->act0.ensure((size_t)B * maxw * sizeof(T) + 64)) || (s = net->act1.ensure((size_t)B * maxw * sizeof(T) + 64)))
    return s;
  T* x0 = (T*)net->act0.ptr;
  T* x1 = (T*)net->act1.ptr;
  const int split_in = net->head == DON_SPLIT_INPUT;
  if (same_grid(net, op)) {
    int g = (int)((n + 255) / 256);
    if (g > 8192) g = 8192;
    hipLaunchKernelGGL((k_branch_in_identity<T, T>), dim3(g), dim3(256), 0, st, n, (const cplx_t<T>*)r, sc, split_in,
                       net->k_input, k, x0);
  } else {
    const size_t m = (size_t)net->bgrid[0] * net->bgrid[1] * net->bgrid[2];
    int g = (int)((m + 255) / 256);
    if (g > 8192) g = 8192;
    hipLaunchKernelGGL((k_branch_in_sample<T, T>), dim3(g), dim3(256), 0, st, op->dim, op->n[0], op->n[1], op->n[2],
                       net->bgrid[0], net->bgrid[1], net->bgrid[2], (const cplx_t<T>*)r, sc, split_in, net->k_input,
                       k, x0);
  }
  if (input_only) {
    hipError_t e = hipMemcpyAsync(du, x0, (size_t)B * K0 * sizeof(T), hipMemcpyDeviceToDevice, st);
    if (e != hipSuccess) return hip_fail(e, "deeponet branch input");
    return launch_check("deeponet branch input");
  }
  // branch layers
  const int L = (int)net->bw.size() - 1;
  size_t pneed = 0;
  for (int l = 0; l < L; ++l) {
    const size_t q = (size_t)small_ksplit(net->bw[l]) * B * net->bw[l + 1];
    pneed = q > pneed ? q : pneed;
  }
  if ((s = net->part.ensure(pneed * sizeof(double)))) return s;
  T* h[2] = {x0, x1};
  int cur = 0;
  const int act = map_act(net->act);
  for (int l = 0; l < L; ++l) {
    dense_small<T>(B, net->bw[l + 1], net->bw[l], h[cur], (const T*)net->bW[l], (const T*)net->bB[l],
                   l == L - 1 ? ACT_NONE : act, h[1 - cur], (double*)net->part.ptr, st);
    cur = 1 - cur;
  }
  // coefficients and synthesis
  if ((s = net->coef.ensure(2 * (size_t)net->p * sizeof(double)))) return s;
  hipLaunchKernelGGL((k_coef<T>), dim3((net->p + 63) / 64), dim3(64), 0, st, net->p, split_in, h[cur],
                     (double*)net->coef.ptr);
  skinny_apply<T, T>(n, net->p, (const T*)c.T.ptr, (const double*)net->coef.ptr, du, op->mask, sc, 1, st);
  return launch_check("deeponet full");
}

helm_status don_full(don_s* net, helm_op_s* op, const void* r, double k, void* du, hipStream_t st) {
  return net->dt == HELM_C128 ? full_eval<double>(net, op, r, k, du, st) : full_eval<float>(net, op, r, k, du, st);
}

static helm_status don_branch_input(don_s* net, helm_op_s* op, const void* r, double k, void* out, hipStream_t st) {
  return net->dt == HELM_C128 ? full_eval<double>(net, op, r, k, out, st, true)
                              : full_eval<float>(net, op, r, k, out, st, true);
}

}  // namespace helm

using namespace helm;

extern "C" {

helm_status deeponet_load(helm_dtype dt, const don_desc* d, const double* const* Wb, don_net* out) {
  if (!out) return fail(HELM_E_INVAL, "deeponet_load: out is NULL");
  *out = nullptr;
  if (!d || !Wb || !d->branch_w || !d->trunk_w) return fail(HELM_E_INVAL, "deeponet_load: NULL argument");
  if (dt != HELM_C64 && dt != HELM_C128) return fail(HELM_E_INVAL, "deeponet_load: unknown dtype");
  if (d->n_branch < 2 || d->n_trunk < 2) return fail(HELM_E_INVAL, "deeponet_load: each network needs >= 1 layer");
  if (d->act < DON_TANH || d->act > DON_LEAKY) return fail(HELM_E_INVAL, "deeponet_load: unknown activation");
  if (d->head != DON_SPLIT_OUTPUT && d->head != DON_SPLIT_INPUT) return fail(HELM_E_INVAL, "deeponet_load: unknown head");
  if (d->p < 1 || d->p > 128) return fail(HELM_E_INVAL, "deeponet_load: p = %d outside [1, 128]", d->p);
  for (int i = 0; i < d->n_branch; ++i)
    if (d->branch_w[i] < 1) return fail(HELM_E_INVAL, "deeponet_load: branch width %d < 1", i);
  for (int i = 0; i < d->n_trunk; ++i)
    if (d->trunk_w[i] < 1) return fail(HELM_E_INVAL, "deeponet_load: trunk width %d < 1", i);
  if (d->trunk_w[0] != 2 && d->trunk_w[0] != 3) return fail(HELM_E_INVAL, "deeponet_load: trunk input must be 2 or 3");
  if (d->trunk_w[d->n_trunk - 1] != d->p) return fail(HELM_E_INVAL, "deeponet_load: trunk output must equal p");
  size_t m = 1;
  for (int a = 0; a < 3; ++a) {
    if (d->branch_grid[a] < 1) return fail(HELM_E_INVAL, "deeponet_load: branch_grid[%d] < 1", a);
    m *= (size_t)d->branch_grid[a];
  }
  if (d->trunk_w[0] == 2 && d->branch_grid[2] != 1) return fail(HELM_E_INVAL, "deeponet_load: 2D needs branch_grid[2] = 1");
  if (d->head == DON_SPLIT_OUTPUT) {
    if ((size_t)d->branch_w[0] != 2 * m + (d->k_input ? 1 : 0))
      return fail(HELM_E_INVAL, "deeponet_load: branch input width must be 2*prod(branch_grid)%s", d->k_input ? "+1" : "");
    if (d->branch_w[d->n_branch - 1] != 2 * d->p) return fail(HELM_E_INVAL, "deeponet_load: branch output must be 2p");
  } else {
    if ((size_t)d->branch_w[0] != m || d->k_input)
      return fail(HELM_E_INVAL, "deeponet_load: SPLIT_INPUT needs input width prod(branch_grid) and no k input");
    if (d->branch_w[d->n_branch - 1] != d->p) return fail(HELM_E_INVAL, "deeponet_load: branch output must be p");
  }
  const int nl = (d->n_branch - 1) + (d->n_trunk - 1);
  for (int i = 0; i < 2 * nl; ++i)
    if (!Wb[i]) return fail(HELM_E_INVAL, "deeponet_load: weight pointer %d is NULL", i);
  don_s* net = new don_s();
  net->dt = dt;
  net->act = d->act;
  net->head = d->head;
  net->p = d->p;
  net->k_input = d->k_input ? 1 : 0;
  for (int a = 0; a < 3; ++a) net->bgrid[a] = d->branch_grid[a];
  net->bw.assign(d->branch_w, d->branch_w + d->n_branch);
  net->tw.assign(d->trunk_w, d->trunk_w + d->n_trunk);
  net->serial = g_serial.fetch_add(1);
  const size_t rs = dt == HELM_C128 ? sizeof(double) : sizeof(float);
  auto upload = [&](const double* src, size_t cnt, void** dst) -> helm_status {
    helm_status s = dalloc(dst, cnt * rs);
    if (s) return s;
    std::vector<char> tmp(cnt * rs);
    if (dt == HELM_C128) {
      std::memcpy(tmp.data(), src, cnt * rs);
    } else {
      float* f = (float*)tmp.data();
      for (size_t i = 0; i < cnt; ++i) f[i] = (float)src[i];
    }
    hipError_t e = hipMemcpy(*dst, tmp.data(), cnt * rs, hipMemcpyHostToDevice);
    if (e != hipSuccess) return hip_fail(e, "deeponet_load: upload");
    return HELM_OK;
  };
  // fp64 copy of the fp32-rounded values (the trunk of a C64 network)
  auto upload_widened = [&](const double* src, size_t cnt, void** dst) -> helm_status {
    helm_status s = dalloc(dst, cnt * sizeof(double));
    if (s) return s;
    std::vector<double> tmp(cnt);
    for (size_t i = 0; i < cnt; ++i) tmp[i] = (double)(float)src[i];
    hipError_t e = hipMemcpy(*dst, tmp.data(), cnt * sizeof(double), hipMemcpyHostToDevice);
    if (e != hipSuccess) return hip_fail(e, "deeponet_load: upload");
    return HELM_OK;
  };
  int wi = 0;
  helm_status s = HELM_OK;
  for (int l = 0; l + 1 < d->n_branch && !s; ++l) {
    void *W = nullptr, *b = nullptr;
    s = upload(Wb[wi++], (size_t)d->branch_w[l] * d->branch_w[l + 1], &W);
    if (!s) s = upload(Wb[wi++], (size_t)d->branch_w[l + 1], &b);
    net->bW.push_back(W);
    net->bB.push_back(b);
  }
  for (int l = 0; l + 1 < d->n_trunk && !s; ++l) {
    void *W = nullptr, *b = nullptr;
    const double* srcW = Wb[wi++];
    const double* srcb = Wb[wi++];
    const size_t cW = (size_t)d->trunk_w[l] * d->trunk_w[l + 1], cb = (size_t)d->trunk_w[l + 1];
    s = upload(srcW, cW, &W);
    if (!s) s = upload(srcb, cb, &b);
    net->tW.push_back(W);
    net->tB.push_back(b);
    if (!s && dt == HELM_C64) {
      void *W64 = nullptr, *b64 = nullptr;
      s = upload_widened(srcW, cW, &W64);
      if (!s) s = upload_widened(srcb, cb, &b64);
      net->tW64.push_back(W64);
      net->tB64.push_back(b64);
    }
  }
  if (s) {
    deeponet_free(net);
    return s;
  }
  *out = net;
  return HELM_OK;
}

void deeponet_free(don_net net) {
  if (!net) return;
  for (void* p : net->bW) dfree(p);
  for (void* p : net->bB) dfree(p);
  for (void* p : net->tW) dfree(p);
  for (void* p : net->tB) dfree(p);
  for (void* p : net->tW64) dfree(p);
  for (void* p : net->tB64) dfree(p);
  net->act0.release();
  net->act1.release();
  net->tact0.release();
  net->tact1.release();
  net->part.release();
  net->coef.release();
  delete net;
}

helm_status deeponet_infer(don_net net, helm_op op, int mode, const void* r, double k, void* out, void* stream) {
  if (!net || !op || !out) return fail(HELM_E_INVAL, "deeponet_infer: NULL argument");
  if (mode != DON_TRUNK && mode != DON_FULL && mode != DON_BRANCH_INPUT)
    return fail(HELM_E_INVAL, "deeponet_infer: unknown mode %d", mode);
  helm_status s = check_net_for_op(net, op, 1);
  if (s) return s;
  hipStream_t st = (hipStream_t)stream;
  if (mode == DON_TRUNK) return don_trunk(net, op, out, st);
  if (!r) return fail(HELM_E_INVAL, "deeponet_infer: r is NULL");
  if (r == out) return fail(HELM_E_INVAL, "deeponet_infer: r and out alias");
  if (mode == DON_BRANCH_INPUT) return don_branch_input(net, op, r, k, out, st);
  return don_full(net, op, r, k, out, st);
}

}  // extern "C"
