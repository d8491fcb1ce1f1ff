// Internal launcher declarations shared by the host library's translation
// units.  Every launcher enqueues on the given stream and returns at once.
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

namespace helm {

struct StencilGeom {
  int nx, ny, nz, dim, zb;
  int ty;    // threads per workgroup in y: 4 or 8
  int rows;  // rows per thread (1 or 2): a tile is 64 x ty rows nodes
  bool nt;   // non-temporal output stores (grids much larger than the caches)
  int rb;    // 3D red-black kernel: 0 = the LDS ring below 2 GiB per field, 1 = ring, 2 = register pairs
  double ih2[3];  // 1/h_a^2 (0 for absent axes)
  double dsum;    // sum_a 2/h_a^2, the Laplacian's diagonal
};

StencilGeom make_geom(int dim, const int n[3], int zb);
int stencil_nblocks(const StencilGeom& g);

// ---- stencil.hip ----------------------------------------------------------
// The stencil kernels take the per-node neighbour code built by build_codes
// (bit 0 = masked node, bits 1..6 = absent x-, x+, y-, y+, z-, z+ neighbour).
void build_codes(const StencilGeom& g, const uint8_t* mask, uint8_t* code, hipStream_t st);
template <typename S>
void stencil_apply(const StencilGeom& g, const void* sc, const uint8_t* code, const void* x, void* y,
                   hipStream_t st);
// r = f - A u; part[stencil_nblocks(g)] receives per-block partials of ||r||^2
template <typename S>
void stencil_resid(const StencilGeom& g, const void* sc, const uint8_t* code, const void* f, const void* u,
                   void* r, double* part, hipStream_t st);
template <typename S>
void stencil_jacobi(const StencilGeom& g, const void* sc, const uint8_t* code, const void* f, const void* u,
                    void* unew, double omega, hipStream_t st);
// one red-black sweep in a single pass, uin -> uout (must differ)
template <typename S>
void stencil_rbgs_fused(const StencilGeom& g, const void* sc, const uint8_t* code, const void* f, const void* uin,
                        void* uout, double omega, hipStream_t st);
template <typename S>
void jacobi_from_zero(size_t n, double dsum, const void* sc, const uint8_t* mask, const void* f, void* z,
                      double omega, hipStream_t st);
// two Jacobi sweeps on A z = f from z = 0 in one pass (z must not alias f).
// With fscale (device scalar) the right-hand side is fscale[0] * f, and fout
// (optional, must alias neither f nor z) receives it.
template <typename S>
void jacobi2_from_zero(const StencilGeom& g, const void* sc, const uint8_t* code, const void* f, void* z, double omega,
                       hipStream_t st, const double* fscale = nullptr, void* fout = nullptr);
template <typename S>
void build_s(size_t n, const double* ksq, const double* alpha, void* sc, hipStream_t st);

// ---- blas1.hip ------------------------------------------------------------
int red_nblocks(size_t n);  // number of partials produced by the one-vector reductions
// out[w] = sum_b part[b * width + w], b = 0..nparts-1 (fixed order), for w < width
void reduce_cols(const double* part, int nparts, int width, double* out, hipStream_t st);
template <typename S>
void dot_part(size_t n, const void* x, const void* y, double* part, hipStream_t st);  // 2 per block
template <typename S>
void nrm2_part(size_t n, const void* x, double* part, hipStream_t st);  // 1 per block
// multi-dot: part[b][2*i..] = partial of sum conj(V_i) w, i < nv, V_i = V + i*ldv
int multidot_nblocks(size_t n);
template <typename S>
void multidot_part(size_t n, const void* V, size_t ldv, int nv, const void* w, double* part, hipStream_t st);
// w = A z (the apply stencil) and the multidot_part partials of V^H w in one launch
template <typename S>
void multidot_apply(const StencilGeom& g, const void* sc, const uint8_t* code, const void* z, const void* V,
                    size_t ldv, int nv, void* w, double* part, hipStream_t st);
// out = base + sgn * sum_i V_i coef_i   (coef: nv complex doubles on device; base may be NULL)
// if part != NULL, per-block partials of ||out||^2 are written (red_nblocks(n) of them)
template <typename S>
void multi_axpy(size_t n, const void* V, size_t ldv, int nv, const double* coef, double sgn, const void* base,
                void* out, double* part, hipStream_t st);
// Fused CGS pass for nv <= cgs_fused_max_nv(): w <- w - sum_i V_i h_i, and
// part[b][2i..] = per-block partials of conj(V_i) w_new over
// cgs_fused_nblocks(n, nv) blocks (returned; at most (n + 255) / 256)
int cgs_fused_max_nv();
int cgs_fused_nblocks(size_t n, int nv);
template <typename S>
int cgs_fused(size_t n, const void* V, size_t ldv, int nv, const double* h, void* w, double* part, hipStream_t st);
// y = x * scal[0] (real scale on device)
template <typename S>
void scale_dev(size_t n, const void* x, const double* scal, void* y, hipStream_t st);
// y = x * a (host real scalar)
template <typename S>
void scale_host(size_t n, const void* x, double a, void* y, hipStream_t st);
// y += x
template <typename S>
void add_inplace(size_t n, const void* x, void* y, hipStream_t st);
template <typename S>
void copy_vec(size_t n, const void* x, void* y, hipStream_t st);
template <typename S>
void zero_vec(size_t n, void* x, hipStream_t st);
template <typename S>
void conj_vec(size_t n, const void* x, void* y, hipStream_t st);  // y = conj(x); x == y allowed

// BiCGStab fused updates (scalars live on the device in a BiState)
struct BiState {
  double rho[2], rho0[2], alpha[2], omega[2], beta[2];
  double rr, ss, fn;
  int flag;  // 0 ok, -4 breakdown, -5 non-finite
  int pad;
};
template <typename S>
void bicg_p(size_t n, const void* r, const void* v, void* p, const BiState* bs, int first, hipStream_t st);
template <typename S>
void bicg_s(size_t n, const void* r, const void* v, void* s, const BiState* bs, double* part, hipStream_t st);
template <typename S>
void two_dot_part(size_t n, const void* t, const void* s, double* part, hipStream_t st);  // 4 per block: t^H s, t^H t
template <typename S>
void bicg_update(size_t n, const void* ph, const void* sh, const void* s, const void* t, const void* rhat, void* u,
                 void* r, const BiState* bs, double* part, hipStream_t st);  // part: 3 per block: rr, rhat^H r
template <typename S>
void axpy_dev(size_t n, const void* x, void* y, const double* a, hipStream_t st);  // y += a x, a complex on device
// scalar steps (single thread), reading the reduced values in `red`
void bicg_scalar(int step, BiState* bs, const double* red, hipStream_t st, BiState* ghost = nullptr);
// BI_INIT starts a sweep: rho0 = alpha = omega = 1, the rest 0, flag 0, and
// red[0], red[1] (||f||^2 and ||r||^2 of the sweep's start) left in fn and rr
enum { BI_RHO = 0, BI_ALPHA = 1, BI_SS = 2, BI_OMEGA = 3, BI_RR = 4, BI_INIT = 5 };

// ---- GMRES small dense work (gmres.hip) -------------------------------------
struct GmState {
  double gabs;  // |g_{j+1}|
  double hn;    // ||w|| before normalisation
  double inv_hn;
  int flag;
  int step;     // Arnoldi step j this record belongs to
};
// H: (m+1) x m complex column-major (H + 2*(j*(m+1) + i)); g: m+1 complex; cs: m real; sn: m complex
// h1, h2: reduced CGS passes (j+1 complex each); npart: nparts per-block partials of
// ||w||^2 (summed in order inside); ghost: a second copy of the status record in
// host-mapped memory (device address of pinned host memory)
void arnoldi_finish(int j, int m, double* H, double* g, double* cs, double* sn, const double* h1, const double* h2,
                    const double* npart, int nparts, GmState* gs, GmState* ghost, hipStream_t st);
void gmres_backsolve(int k, int m, const double* H, const double* g, double* y, hipStream_t st);
// g = sqrt(nrm[0]) e_1 (m+1 complex), nrm[2] = 1/sqrt(nrm[0]) (0 if that is 0 or
// not finite), rec[0..1] = nrm[0..1] (rec: device address of pinned host memory)
void gmres_start(double* nrm, double* g, int m, double* rec, hipStream_t st);

// ---- skinny products with the basis (coarse.hip) -----------------------------
// y_i = sum_j Q_ij c_j for Q (n x r, r <= 128) and complex c (2r doubles, device);
// synth = 0: z += y;  synth = 1: z = scal[0] * y with masked nodes set to 0
template <typename T, typename S>
void skinny_apply(size_t n, int r, const T* Q, const double* c, void* z, const uint8_t* mask, const double* scal,
                  int synth, hipStream_t st);

}  // namespace helm
