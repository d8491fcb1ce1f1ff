/*
 * helm.h -- C ABI of libhelm, a GPU library for the DeepONet meta-solvers of
 * Helmholtz scattering problems (Lee, Liu, Zou, Kahana, Turkel, Ranade, Pathak,
 * Karniadakis: "Fast meta-solvers for 3D complex-shape scatterers using neural
 * operators trained on a non-scattering problem", arXiv 2405.12380).
 *
 * Problem (§2, eq. 1, finite-difference form on a uniform grid):
 *     -Delta_h u - k^2 (1 + i alpha) u = f   on unmasked nodes,  u = 0 on the scatterer.
 *
 * Conventions for every entry point
 * ---------------------------------
 * Grid     : n[a] interior nodes on axis a (x = 0, y = 1, z = 2); spacing
 *            h_a = 1/(n[a]+1); node i sits at (i+1) h_a; the layer of nodes just
 *            outside the box is a zero ghost layer.  dim = 2 uses n[0], n[1]
 *            (n[2] is ignored and taken as 1).
 * Layout   : fields are contiguous arrays of n = n[0]*n[1]*n[2] nodes in x-fastest
 *            order, p = i + n[0]*(j + n[1]*l).  A complex field is interleaved
 *            (re, im): complex64 = 2 x float, complex128 = 2 x double.  The op's
 *            dtype fixes the dtype of every field passed to it.
 * Pointers : unless stated otherwise, field pointers are HIP device pointers owned
 *            by the caller; they must not alias each other unless stated.
 * Streams  : `stream` is a hipStream_t passed as void* (NULL = default stream).
 *            Work is enqueued on it; calls documented as synchronous wait for it.
 * Errors   : every call returns a helm_status.  0 = success; 1 = the result is
 *            valid but the iteration did not reach its tolerance; negative values
 *            are errors.  Argument errors (HELM_E_INVAL) are detected before any
 *            work is enqueued and leave every output untouched.  The text of the
 *            last error on the calling thread is returned by helm_last_error().
 * Threads  : an op or a network may be used by one thread / stream at a time.
 */
#ifndef HELM_H
#define HELM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  HELM_OK = 0,
  HELM_NOT_CONVERGED = 1,
  HELM_E_INVAL = -1,     /* malformed argument; nothing was enqueued            */
  HELM_E_NOMEM = -2,     /* device allocation failed                            */
  HELM_E_HIP = -3,       /* a HIP runtime call failed                           */
  HELM_E_BREAKDOWN = -4, /* BiCGStab rho, r_hat^H v or omega became exactly 0   */
  HELM_E_NONFINITE = -5, /* a residual norm became Inf or NaN                   */
  HELM_E_SINGULAR = -6   /* the coarse matrix or a Gram factor lost rank        */
} helm_status;

typedef enum { HELM_C64 = 1, HELM_C128 = 2 } helm_dtype;

typedef struct {
  int dim;  /* 2 or 3 */
  int n[3]; /* interior nodes per axis, each >= 3 */
} helm_grid;

typedef struct helm_op_s* helm_op;
typedef struct don_s* don_net;

/* relaxation kinds for helm_relax and the smoother of meta_solve */
enum { HELM_JACOBI = 0, HELM_RBGS = 1 };

/* ------------------------------------------------------------------------ */
/* Operator                                                                 */
/* ------------------------------------------------------------------------ */

/* Build the discrete operator of §2 eq. 1 on grid g:
 *   (A x)_p = sum_a (1/h_a^2) [(x_p - x_{p-e_a}) + (x_p - x_{p+e_a})] - s_p x_p,
 *   s_p = ksq_p (1 + i alpha_p),                                     (mask_p = 0)
 *   (A x)_p = x_p                                                    (mask_p != 0)
 * where ghost and masked neighbours contribute 0 (the Dirichlet scatterer of
 * §2 is eliminated symmetrically, so A is complex symmetric).
 * ksq, alpha: arrays of n doubles (k^2 and the sponge damping alpha >= 0).
 * mask: array of n bytes, nonzero on scatterer nodes.
 * The three inputs are host arrays; device arrays are accepted as well (each
 * copy takes its direction from the pointer).  They are copied and not kept;
 * the call is synchronous on `stream`.
 * Errors: HELM_E_INVAL for a NULL pointer, dim not 2/3, n[a] < 3, a node count
 * beyond 2^31, or an unknown dtype. */
helm_status helm_setup(const helm_grid* g, helm_dtype dt, const double* ksq, const double* alpha,
                       const uint8_t* mask, void* stream, helm_op* out);

/* Replace k^2 (device array of n doubles, same alpha and mask): the update of
 * an optimisation loop, whose k^2 lives on the device.  Invalidates the cached
 * coarse space.  Synchronous on `stream`. */
helm_status helm_set_ksq(helm_op op, const double* ksq, void* stream);

/* Release an op and its device memory.  NULL is ignored. */
void helm_destroy(helm_op op);

/* Number of grid nodes of an op (0 for NULL). */
size_t helm_size(helm_op op);

/* Tile autotuner for the op's stencil kernels: times y = A x (8 launches after
 * 2 warm-ups, HIP events on `stream`) for every workgroup height ty in {4, 8}
 * (only fixed_ty when it is 4 or 8; 0 = free), z-march length zb in
 * {1, 2, 4, 8, 16, 32} (<= n_z; 1 in 2D), plain or non-temporal output
 * stores and one or two rows per thread (3D), and keeps the fastest for all
 * later stencil work on this op.  The
 * per-node arithmetic does not depend on the tiling, so results of apply,
 * relax and the sweeps are unchanged; reduction partials are regrouped.
 * Outputs (each optional): the chosen ty and zb and its time per launch (us).
 * Synchronous; uses op-owned scratch.  Do not call while a solve on the op is
 * in flight. */
helm_status helm_tune(helm_op op, int fixed_ty, void* stream, int* ty_out, int* zb_out, double* us_out);

/* Red-black sweep kernel of an op (3D; results are the same bit for bit):
 *   HELM_RB_AUTO  : the LDS-ring kernel for fields under 2 GiB, else the
 *                   register-pair kernel (the default);
 *   HELM_RB_RING  : each input plane staged once in LDS, a ring of planes per
 *                   column tile (fields under 2 GiB: 32-bit buffer offsets);
 *   HELM_RB_PAIRS : each lane updates a red/black node pair, red values
 *                   exchanged through registers and LDS (any size; 2D always).
 * HELM_E_INVAL for an unknown value, or RING on a 2D op or a field of 2 GiB
 * or more.  Takes effect for later sweeps. */
enum { HELM_RB_AUTO = 0, HELM_RB_RING = 1, HELM_RB_PAIRS = 2 };
helm_status helm_set_rbgs_kernel(helm_op op, int which);

/* y = A x (§2 eq. 1 as above).  x, y: complex fields; must not alias.  Async. */
helm_status helm_apply(helm_op op, const void* x, void* y, void* stream);

/* r = f - A u (the residual of eq. 2).  If rnorm is non-NULL the call waits for
 * the stream and stores ||r||_2 there (host double).  r must not alias f or u. */
helm_status helm_residual(helm_op op, const void* f, const void* u, void* r, double* rnorm,
                          void* stream);

/* `sweeps` relaxation steps of eq. 2 on A u = f, in place on u (§3.1.1):
 *   HELM_JACOBI: u <- u + omega D^{-1}(f - A u), D = diag(A)
 *                (D_p = sum_a 2/h_a^2 - s_p; 1 on masked nodes);
 *   HELM_RBGS  : the same update applied to the nodes with (i+j+l) even, then
 *                to the odd ones using the new even values (red-black
 *                Gauss-Seidel; SOR when omega != 1).
 * Async.  Uses op-owned scratch memory. */
helm_status helm_relax(helm_op op, int kind, double omega, int sweeps, const void* f, void* u,
                       void* stream);

/* helm_relax for callers that cannot allocate device memory (code under HIP
 * graph capture, tight serving loops, harnesses that forbid allocation): the
 * same sweeps, bit for bit, with the ping-pong field that helm_relax allocates
 * on first use taken from a static device array of 64 MiB instead, which each
 * GPU the library runs on holds until the process ends.  Makes no allocating
 * call.  Fields above 64 MiB (4 Mi nodes complex128, 8 Mi complex64) return
 * HELM_E_INVAL.  Every call on one GPU shares that GPU's array: calls that
 * overlap on one GPU (other streams, other threads) race and must be
 * serialized by the caller.  Async. */
helm_status helm_relax_noalloc(helm_op op, int kind, double omega, int sweeps, const void* f, void* u,
                               void* stream);

/* Krylov inner products (synchronous): out[0] + i out[1] = sum conj(x_p) y_p. */
helm_status helm_dot(helm_op op, const void* x, const void* y, double out[2], void* stream);
/* ||x||_2 (synchronous). */
helm_status helm_nrm2(helm_op op, const void* x, double* out, void* stream);

/* ------------------------------------------------------------------------ */
/* DeepONet (App. B architecture, App. C trunk matrix)                      */
/* ------------------------------------------------------------------------ */

enum { DON_TANH = 0, DON_RELU = 1, DON_LEAKY = 2 };
/* Output heads.  SPLIT_OUTPUT: the branch emits 2p values b, and
 *   N(r) = T b[0:p] + i T b[p:2p]   (the head of App. B);
 * SPLIT_INPUT: the branch emits p values and is applied to Re and Im of the
 * input separately, N(r) = T branch(Re r) + i T branch(Im r). */
enum { DON_SPLIT_OUTPUT = 0, DON_SPLIT_INPUT = 1 };
enum { DON_TRUNK = 0, DON_FULL = 1, DON_BRANCH_INPUT = 2 };

typedef struct {
  int n_branch;        /* number of widths in branch_w (layers + 1)                 */
  const int* branch_w; /* widths, input first.  Input = 2*prod(branch_grid) (+1 if
                          k_input) for SPLIT_OUTPUT, prod(branch_grid) for SPLIT_INPUT */
  int n_trunk;         /* number of widths in trunk_w                                  */
  const int* trunk_w;  /* widths; trunk_w[0] = grid dim, last = p                     */
  int act;             /* hidden-layer activation (DON_TANH, ...); last layers linear */
  int head;            /* DON_SPLIT_OUTPUT or DON_SPLIT_INPUT                          */
  int p;               /* number of trunk basis functions, 1..128                      */
  int branch_grid[3];  /* grid the branch samples its input on (z = 1 in 2D)          */
  int k_input;         /* 1: the wave number is appended to the branch input          */
} don_desc;

/* Upload a network.  Wb = host pointers to W0, b0, W1, b1, ... for the branch
 * layers followed by the trunk layers; W_l is row-major (fan_in x fan_out) so that
 * a layer computes h' = act(h W + b).  Weights are stored in the dtype's real
 * precision (float for HELM_C64, double for HELM_C128).  Synchronous. */
helm_status deeponet_load(helm_dtype dt, const don_desc* d, const double* const* Wb, don_net* out);
void deeponet_free(don_net net);

/* DON_TRUNK: out = T, the n x p trunk matrix [T]_ij = T_j(x_i) at the op's node
 *            coordinates x_i (App. C), row-major, real (float or double per dtype).
 * DON_FULL : out = du = s N(r/s) with s = ||r||_2/sqrt(n) (du = 0 if r = 0), set to
 *            0 on masked nodes: the network correction M2 of eq. 3.  r and out
 *            are complex fields; the branch samples r/s on branch_grid (identity
 *            when it equals the op's grid, multilinear with zero ghosts otherwise).
 * DON_BRANCH_INPUT: out = the branch's input vector for r (what DON_FULL feeds
 *            its first branch layer: r/s sampled on branch_grid, Re then Im,
 *            then k when k_input is set; for SPLIT_INPUT the Re and Im rows),
 *            real in the dtype's precision — the training inputs of App. B.
 * k is the wave number fed to the branch when k_input is set.  Async. */
helm_status deeponet_infer(don_net net, helm_op op, int mode, const void* r, double k, void* out,
                           void* stream);

/* ------------------------------------------------------------------------ */
/* DeepONet training (App. B network; bf16 MFMA, fp32 accumulation)         */
/* ------------------------------------------------------------------------ */

typedef struct don_trainer_s* don_trainer;

typedef struct {
  int n_points;    /* P: trunk evaluation points per sample (positive multiple of 64) */
  int batch;       /* S: samples per step (64 or 128)                               */
  int max_steps;   /* capacity: most steps of one don_train_steps / don_train_eval  */
  double lr, beta1, beta2, eps;  /* Adam                                            */
} don_train_opts;

/* Trainer for `net` (SPLIT_OUTPUT head, tanh; p a multiple of 64; widths after
 * each input multiples of 64 and <= 256; at most 8 trunk layers, 9 branch
 * layers and 16 in all; otherwise HELM_E_INVAL).  It keeps fp32 master copies
 * of the net's weights (input widths padded to multiples of 64 with zero rows),
 * their bf16 copies (W and W^T), Adam's moments, and every activation of a step.  X: device array of P x d fp64 trunk
 * inputs (node coordinates), copied.  One step on samples idx[0..S):
 *   T = trunk(X), B = branch(F_idx), U_s = T B_s[:p] + i T B_s[p:],
 *   L = mean_s ||U_s - Y_s|| / ||Y_s||, gradients by backpropagation, Adam
 *   (Kingma & Ba) on the fp32 parameters.
 * Every product runs as a bf16 MFMA GEMM with fp32 accumulation; tanh and its
 * derivative, biases and the loss are fused or run in fp32 (norms in fp64). */
helm_status don_train_create(don_net net, const don_train_opts* o, const double* X, don_trainer* out);

/* The dataset: n samples; F: device fp32 n x K_b branch inputs (K_b = the
 * net's branch input width), converted to padded bf16 (copied); Y: device
 * complex64 n x P labels, sample-major — kept by pointer, so it must stay
 * valid while the trainer uses it.  May be called again to replace the data
 * (any n); the captured step graphs are then recorded anew.  Synchronous. */
helm_status don_train_data(don_trainer t, int n, const float* F, const void* Y);

/* `count` Adam steps; step k uses samples idx[k S .. k S + S) (device int array,
 * values in [0, n)).  A step is captured once as a HIP graph on the trainer's
 * stream and replayed.  loss_out (optional host array of count floats): the
 * loss of each step before its update.  Waits for `stream` first; synchronous. */
helm_status don_train_steps(don_trainer t, int count, const int* idx, float* loss_out, void* stream);

/* Losses of `count` batches (forward and backward, no update); loss_out: host
 * array of count floats.  Synchronous. */
helm_status don_train_eval(don_trainer t, int count, const int* idx, float* loss_out, void* stream);

/* Loss (host float) and gradients (device fp32 array of don_train_nparam
 * entries, the flat parameter layout) of one batch idx[0..S), no update. */
helm_status don_train_grad(don_trainer t, const int* idx, float* loss, float* grads, void* stream);

/* One Adam step with caller-provided gradients (device fp32, flat layout). */
helm_status don_train_apply(don_trainer t, const float* grads, void* stream);

/* Number of flat fp32 parameters (including padding), and the layout of layer
 * `layer` of the branch (which = 0) or trunk (which = 1): true and padded input
 * width, output width, offsets of W (Kp x N, row-major) and b (N). */
size_t don_train_nparam(don_trainer t);
helm_status don_train_layout(don_trainer t, int which, int layer, int* K, int* Kp, int* N, size_t* offW,
                             size_t* offb);

/* Copy the fp32 master parameters (flat layout) to a device array. */
helm_status don_train_params(don_trainer t, float* out, void* stream);

/* Write the trained weights back into `net` (its dtype); cached trunk matrices
 * and coarse spaces built from the old weights are invalidated. */
helm_status don_train_export(don_trainer t, don_net net, void* stream);

void don_train_free(don_trainer t);

/* ------------------------------------------------------------------------ */
/* Meta-solvers (§3.1.1 eq. 3; §3.1.2 with the trunk basis of App. C)       */
/* ------------------------------------------------------------------------ */

enum { META_JACOBI = 0, META_GS = 1, META_GMRES = 2, META_BICGSTAB = 3 };

typedef struct {
  int kind;        /* META_*                                                        */
  int restart;     /* GMRES(m): m >= 1                                              */
  double tol;      /* stop when ||f - A u||_2 <= tol ||f||_2 (tol >= 0; <= tol when
                      f = 0, where the relative residual is undefined)           */
  int max_iters;   /* Arnoldi steps / BiCGStab iterations / relaxation sweeps       */
  int smoother;    /* HELM_JACOBI or HELM_RBGS                                      */
  int n_r;         /* sweeps per cycle (relaxation) or per preconditioner (Krylov)  */
  double omega;    /* relaxation weight                                             */
  int nn_every;    /* relaxation kinds: network correction after every nn_every sweeps */
  int p_used;      /* Krylov kinds with a network: trunk columns used (1..p)        */
  double k;        /* wave number passed to a network with k_input                  */
  double* history; /* optional host array of max_iters+1 relative residuals, or NULL */
  int q_fp32;      /* Krylov kinds with a network: store the basis Q in fp32 (C128;
                      always so for C64).  A_c is then the Galerkin matrix of the
                      stored basis; halves the bytes of the coarse correction.      */
  int mg_levels;   /* Krylov kinds: 0 = the preconditioner above; L > 0 = one
                      geometric multigrid V-cycle with L coarsenings (§4.3,
                      DeepONet-MG-Krylov): every second node per level, coefficient
                      and mask injected, full weighting, multilinear prolongation,
                      exact solve on the coarsest grid (<= 128 nodes); each n_a + 1
                      must be divisible by 2^L.                                     */
  int mg_nu;       /* smoothing steps before and after the coarse correction: Jacobi
                      sweeps (net == NULL), or with a network a sweeps, one trunk-basis
                      correction of that level with min(p_used, nodes) columns, b
                      sweeps (a = mg_nu / 2, b = mg_nu - a - 1: 2-1-2 for 5)         */
  int no_drop;     /* Krylov kinds with a network: 1 = every one of the p_used trunk
                      columns must be kept; if the QR would drop one (App. C
                      selection: remaining norm <= tau x the largest), the call
                      fails with HELM_E_SINGULAR before iterating and u is
                      untouched.  0 = drop and report the rank in rank_used.
                      Applies to every coarse space the call builds.           */
  int fallback_restart; /* META_JACOBI / META_GS: 0 = none; m >= 1 = standalone
                      GMRES(m) as the fallback of a diverging relaxation: when a
                      cycle ends with a relative residual that is not finite or
                      larger than at the end of the previous cycle (or at u0),
                      u returns to the iterate before that cycle and GMRES(m)
                      (M = I) runs from it to tol within max_iters Arnoldi steps;
                      its steps are reported in fallback_iters and its status
                      is the call's.  Costs one field copy per cycle.            */
  int gs_passes;   /* META_GMRES (and the fallback GMRES): classical Gram-Schmidt
                      passes per Arnoldi step.  0 or 2 = CGS2 (the new vector is
                      projected out of the basis twice); 1 = one projection, the
                      default orthogonalization of PETSc's GMRES, whose solvers
                      the paper's experiments used (section 4): one pass over
                      the basis fewer per step.                                  */
} meta_opts;

typedef struct {
  int iters, matvecs, precond_apps, converged, rank_used, history_len;
  double rel_res;     /* true ||f - A u||_2 / ||f||_2 at exit (||f - A u||_2 if f = 0) */
  double setup_ms;    /* coarse-space construction time (0 when cached)               */
  double solve_ms;    /* iteration time                                               */
  double cond_Ac_est; /* 1-norm condition estimate of the coarse matrix               */
  int fallback_iters; /* Arnoldi steps of the GMRES fallback (0: it did not run);
                         iters keeps counting relaxation sweeps                     */
} meta_stats;

/* Solve A u = f.
 *   META_JACOBI / META_GS: eq. 3 with M1 = nn_every smoother sweeps and M2 = the
 *     network correction (DON_FULL) when net != NULL; plain relaxation otherwise.
 *   META_GMRES / META_BICGSTAB: right-preconditioned GMRES(restart) with classical
 *     Gram-Schmidt (gs_passes), or
 *     BiCGStab, on the true relative residual.  With net != NULL the
 *     preconditioner is M(r) = eq. 3 from z = 0: n_r smoother sweeps on A z = r,
 *     then z += Q A_c^{-1} Q^T (r - A z) where Q spans the first p_used masked
 *     trunk columns (QR with positive diag R; columns whose remaining norm is at
 *     most tau times the largest column norm are dropped, tau = 1e-7 (C128),
 *     1e-5 (C64)) and A_c = Q^T A Q (App. C).  With net == NULL, M = I.
 * u holds u0 on entry and the last iterate on exit (also when not converged).
 * A relaxation kind with fallback_restart >= 1 hands a diverging iteration to
 * standalone GMRES (see meta_opts.fallback_restart).
 * The coarse space is cached on the op, keyed by (net, p_used, q_fp32, k^2 version).
 * Synchronous.  Returns HELM_OK, HELM_NOT_CONVERGED, HELM_E_BREAKDOWN,
 * HELM_E_NONFINITE, HELM_E_SINGULAR (a singular A_c, or a dropped column with
 * no_drop) or an argument/HIP error. */
helm_status meta_solve(helm_op op, don_net net, const meta_opts* o, const void* f, void* u,
                       meta_stats* st, void* stream);

/* z = M(r), the Krylov preconditioner that meta_solve would use for opts o
 * (M = the n_r smoother sweeps alone when net is NULL).  Builds or reuses the
 * coarse space.  r, z: complex fields, no aliasing.  Synchronous. */
helm_status meta_precond(helm_op op, don_net net, const meta_opts* o, const void* r, void* z,
                         void* stream);

/* Inspect the cached coarse space for (net, o->p_used): rank, and optionally the
 * coarse matrix A_c (host, rank x rank complex128, row-major, interleaved, capacity
 * `ac_cap` complex entries) and Q (device, n x rank, row-major, real in the dtype's
 * precision, capacity `q_cap` elements).  Q is the orthonormal basis (App. C) and
 * A_c = Q^T A Q.  With an fp64 basis the solves use the first CholeskyQR pass's
 * basis Q1 = P S1, which spans the same space (the correction depends only on
 * the span); the second pass, Q = Q1 S2 and A_c = S2^T (Q1^T A Q1) S2, is run
 * here (HELM_E_SINGULAR if it loses rank).  Synchronous. */
helm_status meta_coarse_info(helm_op op, don_net net, const meta_opts* o, int* rank, double* Ac,
                             size_t ac_cap, void* Q, size_t q_cap, void* stream);

/* Solve `count` independent problems A_i u_i = f_i (§3.1.2: many grids, wave
 * numbers, scatterers and sources at once) with BiCGStab, right-preconditioned
 * as in meta_solve when net != NULL (M(r) = n_r Jacobi sweeps from zero, then
 * the trunk-basis correction of App. C with p_used columns; M = I otherwise).
 * o->kind must be META_BICGSTAB and o->smoother HELM_JACOBI; tol, max_iters,
 * n_r, omega, p_used and q_fp32 apply to every problem; history is ignored.
 * ops: `count` distinct ops of one dtype and dimension.  f[i], u[i]: complex
 * fields of op i (u[i] holds u0 on entry, the last iterate on exit).
 * st: array of `count` stats (solve_ms is the batch's wall time on the device).
 * Every kernel of an iteration covers all problems and a problem's workgroups
 * exit at once once it has stopped, so convergence is decided on the device;
 * chunks of iterations are captured as one HIP graph on a library stream and
 * replayed.  The coarse spaces are built (or reused) per op first, and their
 * setup work buffers are released afterwards.  Device memory for ten complex
 * fields per problem is allocated for the call.  Synchronous; the caller's
 * stream is waited for before and after.
 * Returns HELM_OK if every problem converged, else the most severe status
 * (an error below 0, or HELM_NOT_CONVERGED); per-problem outcomes are in
 * st[i].converged and st[i].rel_res.  HELM_E_INVAL for a bad argument. */
helm_status meta_solve_batch(int count, const helm_op* ops, don_net net, const meta_opts* o,
                             const void* const* f, void* const* u, meta_stats* st, void* stream);

/* ------------------------------------------------------------------------ */
/* Adjoint: k^2 gradient of a receiver misfit (§2 eq. 1 differentiated)     */
/* ------------------------------------------------------------------------ */

/* Solve the conjugate-transpose system A^H lam = g with the meta-solver of
 * opts o (same kinds, options, statuses and stats as meta_solve; rel_res is
 * ||g - A^H lam|| / ||g||).  A is complex symmetric, so the call runs
 * meta_solve on conj(g) and conjugates the iterate: the preconditioner acting
 * on the adjoint system is M built from A^H, and a cached coarse space of the
 * op is reused.  lam holds the initial guess on entry and the last iterate on
 * exit; g and lam are complex fields of the op's dtype and must not alias.
 * Uses one op-owned field of scratch.  Synchronous. */
helm_status meta_solve_adjoint(helm_op op, don_net net, const meta_opts* o, const void* g, void* lam,
                               meta_stats* st, void* stream);

/* Receiver misfit on the grid plane {i_axis = index} (axis 0 = x, 1 = y,
 * 2 = z):  r = P u - d,  loss = 1/2 ||r||_2^2,  g = P^T r with g = 0 on
 * scatterer nodes (u is 0 there; the loss does not depend on them) and off
 * the plane.  d: device array of the plane's values, complex in the op's
 * dtype, ordered with the remaining axes in x-fastest order (axis 0: y
 * fastest then z; axis 1: x then z; axis 2: x then y; a 2D grid's plane is a
 * line).  g: complex field, overwritten.  If loss is non-NULL the call waits
 * for the stream and stores the loss (host double); otherwise async.
 * Errors: HELM_E_INVAL for NULL pointers, an axis outside the grid, an
 * index outside [0, n[axis]), or g aliasing u or d. */
helm_status helm_misfit(helm_op op, int axis, int index, const void* u, const void* d, void* g, double* loss,
                        void* stream);

/* Pointwise k^2 gradient of a loss L(u) with A(k^2) u = f, given the adjoint
 * state A^H lam = dL/du:  grad_p = Re(conj(lam_p) (1 + i alpha_p) u_p), and 0
 * on scatterer nodes (their identity rows carry no k^2).  grad: real device
 * array of n in the dtype's precision (double for C128, float for C64); it
 * must not alias u or lam.  Async. */
helm_status helm_ksq_gradient(helm_op op, const void* u, const void* lam, void* grad, void* stream);

/* ------------------------------------------------------------------------ */
/* Measurement hook                                                          */
/* ------------------------------------------------------------------------ */

/* Kernel classes timed by the hook. */
enum { HELM_KP_STENCIL = 0,   /* apply / residual / Jacobi / red-black sweeps      */
       HELM_KP_MULTIDOT = 1,  /* GMRES multi-dot V^H w                              */
       HELM_KP_MULTIAXPY = 2, /* GMRES multi-axpy w -= V h and V y                  */
       HELM_KP_QT = 3,        /* coarse restriction Q^T r (per-block partials)      */
       HELM_KP_SKINNY = 4,    /* prolongation z += Q c and the DeepONet synthesis   */
       HELM_KP_CGS = 5,       /* fused CGS pass w -= V h with the partials of V^H w */
       HELM_KP_MFMA = 6 };    /* fp64 MFMA products of the set-up (trunk layers, Gram
                                 and Q products); its "bytes" are algorithmic flops */

/* Per-kernel timing for the whole process: `mask` has bit (1 << HELM_KP_*) set
 * for each kernel class to time (0 disables, -1 times every class); earlier
 * records are cleared (waits for the device).  Each launch of an enabled class
 * is bracketed by two HIP events on its stream, and the algorithmic bytes that
 * launch must move (reads + writes of its operands, each once) are recorded.
 * The events themselves lengthen the gap between dependent launches by a few
 * microseconds, so a timing run enables only the classes it needs. */
helm_status helm_kprof_enable(int mask);
/* Totals since the last enable for one kernel class: launches, summed
 * event-measured duration (ms) and summed algorithmic bytes.  Waits for the
 * recorded events. */
helm_status helm_kprof_read(int kind, int* count, double* total_ms, double* total_bytes);

/* dst = src (bytes a multiple of 16, 16-byte aligned, no overlap) with
 * non-temporal 16-byte loads and stores: the device-copy bandwidth that stencil
 * kernels are compared with.  Async. */
helm_status helm_stream_copy(const void* src, void* dst, size_t bytes, void* stream);

/* Text for a status code / the calling thread's last error message. */
const char* helm_strerror(helm_status s);
const char* helm_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* HELM_H */
