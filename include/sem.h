/*
 * sem.h -- C-ABI of the MI355X hybrid Schwarz / p-multigrid solver for the
 * spectral element discretisation of
 *      -div(nu grad u) = f   on a Cartesian mesh of rectangular elements
 * (Poisson when nu = 1), after J. Stiller, "Nonuniformly weighted Schwarz
 * smoothers for spectral element multigrid" (arXiv 1512.02390).
 *
 * Conventions shared by every entry point
 *  - Vectors are nodal arrays of one multigrid level, FP64, row-major with
 *    rows along y and columns along x, `rows * cols` contiguous doubles in
 *    device memory (sizes from sem_level_info).  Dirichlet arrays include the
 *    boundary nodes; their entries are ignored on input and written as 0.
 *    Periodic arrays hold n*p nodes per direction (node n*p is node 0).
 *  - The caller owns every vector passed in; the handle owns all tables and
 *    internal level vectors.
 *  - Work is queued on the HIP stream given to sem_setup and is asynchronous
 *    unless stated otherwise.  A handle is not thread-safe; use one handle
 *    per stream.
 *  - Every function returns a sem_status; no C++ exception crosses the ABI.
 *    sem_last_error() describes the most recent failure of a handle.
 */
#ifndef SEM_H
#define SEM_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct sem_ctx *sem_handle;

typedef enum {
  SEM_OK = 0,
  SEM_EINVAL = -1,   /* invalid argument (sizes, null pointer, overlap range) */
  SEM_EDOM = -2,     /* nu <= 0 or non-increasing element breaks           */
  SEM_ENOMEM = -3,   /* device or host allocation failed                  */
  SEM_EHIP = -4,     /* a HIP runtime call failed                          */
  SEM_ENOCONV = -5,  /* pcg_solve reached imax; u holds the last iterate   */
  SEM_ENAN = -6,     /* non-finite residual encountered                    */
  SEM_EUNSUP = -7    /* supported by the method but not by this library
                        (tile size, coarse grid too large for nu != 1)     */
} sem_status;

typedef enum { SEM_BC_DIRICHLET = 0, SEM_BC_PERIODIC = 1 } sem_bc;

/* Weight functions of Table 1 (Section 3.1).  Odd kappa >= 1 selects the
 * smoothed sign function of that order (1 linear, 3 cubic, 5 quintic,
 * 7 seventh order, larger odd orders by the same defining conditions). */
/* SEM_W_MULT selects the multiplicative Schwarz method of Algorithm 1
 * instead: the subdomain problems are solved one after the other in
 * row-major element order (reversed on every second sweep), each on the
 * residual left by the corrections before it, without weights.  It is
 * sequential, so one workgroup runs it; supported for the Poisson operator
 * (nu = NULL) in SEM_FP64 precision, without width scales or per-element
 * parameters (SEM_EUNSUP otherwise). */
typedef enum { SEM_W_TOPHAT = -1, SEM_W_ARITH = -2, SEM_W_MULT = -3 } sem_wf_special;

/* Local subdomain problems for variable nu (sem_weights.local_solve). */
typedef enum {
  SEM_LOCAL_MEAN = 0,      /* Section 4: A_ss^{-1} r_s / nu_bar_s (element mean) */
  SEM_LOCAL_SEPARABLE = 1  /* separable fit of nu per subdomain (extension)      */
} sem_local_solve;

/* Overlap n_o per multigrid level l > 0 (Section 4); always clamped to
 * [0, p_l - 1]. */
typedef enum {
  SEM_NO_FIXED = 0,   /* n_o on every level              */
  SEM_NO_CEIL_P8 = 1, /* ceil(p_l / 8)  (the paper's recommendation) */
  SEM_NO_FLOOR_P8 = 2,/* floor(p_l / 8) */
  SEM_NO_CEIL_P2 = 3  /* ceil(p_l / 2)  */
} sem_overlap_rule;

/* Arithmetic of the V-cycle used as preconditioner.  Vectors crossing the
 * ABI are always FP64.  SEM_MIXED_FP32 runs smoother, residuals and
 * transfers of the V-cycle in FP32 inside an FP64 residual / CG outer
 * iteration (the coarse solve stays FP64).  SEM_MIXED_BF16 is SEM_MIXED_FP32
 * with the subdomain solves of levels whose subdomain width
 * p_l + 1 + 2 n_o is at least 17 on the matrix cores: BF16 operands, FP32
 * accumulation.  SEM_MIXED_FP16 is the same with FP16 operands, each operand
 * tile scaled by a power of two into FP16's range (3 more significand bits
 * than BF16, same speed). */
typedef enum {
  SEM_FP64 = 0,
  SEM_MIXED_FP32 = 1,
  SEM_MIXED_BF16 = 2,
  SEM_MIXED_FP16 = 3
} sem_precision;

typedef struct {
  int32_t nx, ny;          /* elements per direction                      */
  const double *xb, *yb;   /* host arrays of nx+1 / ny+1 increasing breaks */
  int32_t bc;              /* sem_bc; periodic needs nx, ny >= 3          */
} sem_mesh;

typedef struct {
  int32_t rule;            /* sem_overlap_rule */
  int32_t n_o;             /* used by SEM_NO_FIXED */
  /* Optional host array of L+1 overlaps indexed by level (entry 0 unused);
   * when non-NULL it replaces the rule.  Each entry must lie in
   * [0, p_l - 1]; L+1 is the number of levels, ceil-halving p down to 1. */
  const int32_t *per_level;
} sem_overlap;

typedef struct {
  int32_t wf;              /* odd kappa, SEM_W_TOPHAT or SEM_W_ARITH */
  /* Optional host arrays of nx+1 / ny+1 width scales in (0, 1], one per grid
   * line (interface); the transition width at that interface is
   * alpha * delta_o.  NULL means 1 everywhere (the paper's weights). */
  const double *alpha_x, *alpha_y;
  /* Optional per-element parameters (a project extension; the paper fixes
   * one overlap per level and one transition width): host array
   * elem_params[e][2] = (alpha_e, rho_e), e = ey * nx + ex, alpha_e in
   * (0, 1], rho_e >= 0.  On level l > 0 element e's subdomain has
   * n_o,e = ceil(rho_e p_l) layers, clamped to [1, p_l - 1] and to a width
   * p_l + 1 + 2 n_o,e <= 48, and its weights are the weight function of
   * Section 3.1 with delta = alpha_e delta_o(n_o,e) on both sides (unit
   * weights for SEM_W_ARITH).  Neighbouring subdomains then need not share
   * their transition zones, so the update is normalised node by node:
   *   u += D^{-1} sum_s R_s^T W_s A_ss^{-1} R_s r,  D = sum_s R_s^T W_s R_s,
   * which equals the paper's update when all elements carry equal
   * parameters (D = 1) and the arithmetic mean for unit weights (D = C).
   * When non-NULL, alpha_x / alpha_y must be NULL and the overlap rule is
   * not used on levels l > 0 (sem_level_info reports the largest n_o,e). */
  const float *elem_params;
  /* sem_local_solve (a project extension; 0 is the paper's method).  With
   * SEM_LOCAL_SEPARABLE (variable nu only, not with elem_params), each
   * subdomain s of level l > 0 fits log nu on its window's nodes (level l's
   * nodal nu) by least squares as alpha(x) + beta(y): alpha = column means
   * minus the grand mean, beta = row means.  Its local operator is the
   * restriction of B(a(x) b(y)), a = exp(alpha), b = exp(beta), extended
   * beyond the window by the value at its nearest node:
   *   A_s = M_b (x) L_a + L_b (x) M_a,
   * with L_a, M_a the 1-D stiffness and lumped mass weighted by a (GLL
   * quadrature over the elements the window reaches).  It is separable, so
   * the fast diagonalisation applies with one factor pair per subdomain
   * (host set-up cost and factor memory grow with the element count); no
   * 1/nu_bar scaling.  Subdomains, weights and the update stay the paper's.
   * For nu = a(x) b(y) the fit is exact inside each window. */
  int32_t local_solve;
} sem_weights;

/* Build all levels, operators, fast-diagonalisation factors, weights,
 * transfer matrices and the coarse solver (Sections 2-3; Section 4 for
 * variable nu).  nu: host array of the finest level's nodal diffusivity
 * (layout of level L), or NULL for the Poisson problem.  stream: a
 * hipStream_t (NULL = default stream).  On success *out receives the handle.
 * Errors: SEM_EINVAL (p < 1, n_o out of range, periodic with fewer than 3
 * elements, NULL pointers), SEM_EDOM (breaks not increasing, nu <= 0),
 * SEM_EUNSUP (subdomain width p+1+2 n_o above 48, p above 32),
 * SEM_ENOMEM, SEM_EHIP. */
sem_status sem_setup(const sem_mesh *mesh, int32_t p, const sem_overlap *overlap,
                     const sem_weights *weights, const double *nu, int32_t precision,
                     void *stream, sem_handle *out);
sem_status sem_destroy(sem_handle h);

/* Number of levels L+1 and, per level l (0 = coarsest, L = finest), the
 * order p_l, the overlap n_o,l (0 on level 0) and the node-array shape. */
sem_status sem_num_levels(sem_handle h, int32_t *nlevels);
sem_status sem_level_info(sem_handle h, int32_t level, int32_t *p_l, int32_t *n_o,
                          int64_t *rows, int64_t *cols);
/* Host copies of the node coordinates of a level (cols x-values, rows
 * y-values), for evaluating analytic data at the nodes. */
sem_status sem_node_coords(sem_handle h, int32_t level, double *x, double *y);

/* b = (M_y (x) M_x) f on level L: the right-hand side of A u = b for nodal
 * source values f (Section 2).  Device arrays. */
sem_status sem_mass(sem_handle h, const double *f_nodal, double *b);

/* r = f - A_l u  (Section 3.1, residual form; A_l = B(nu_l) for variable nu).
 * f may be NULL, then r = A_l u.  Device arrays of level `level`. */
sem_status sem_residual(sem_handle h, int32_t level, const double *u, const double *f,
                        double *r);

/* n_it sweeps of the weighted additive Schwarz method (Algorithm 2) on level
 * `level` >= 1: r = f - A u, then u += sum_s R_s^T W A_ss^{-1} R_s r with
 * A_ss^{-1} by fast diagonalisation (scaled by 1/nu_bar_s for variable nu).
 * u is updated in place. */
sem_status sem_schwarz_smooth(sem_handle h, int32_t level, double *u, const double *f,
                              int32_t n_it);

/* f_c = I_l^T r_f (residual restriction, level l -> l-1) and
 * u_f += I_l u_c (correction prolongation, l-1 -> l), Section 3.2. */
sem_status sem_restrict(sem_handle h, int32_t level, const double *r_fine, double *f_coarse);
sem_status sem_prolong_add(sem_handle h, int32_t level, const double *u_coarse,
                           double *u_fine);

/* u_0 = A_0^+ f_0 on level 0 (Algorithm 3, coarse grid solution); for a
 * singular periodic A_0 the right side is projected onto the range and the
 * zero-mean solution is returned. */
sem_status sem_coarse_solve(sem_handle h, const double *f0, double *u0);

/* One multigrid V-cycle (Algorithm 3) on the finest level: u updated in
 * place.  ns1, ns2: host arrays of L+1 pre/post smoothing counts indexed by
 * level (entry 0 unused); NULL gives MG(1,0). */
sem_status sem_vcycle(sem_handle h, double *u, const double *f, const int32_t *ns1,
                      const int32_t *ns2);

/* Inexact multigrid-preconditioned CG (Algorithm 4) until
 * ||r||_2 <= rtol ||r_0||_2 or imax iterations.  The host waits once per
 * iteration for ||r|| (the stopping test) while the next iteration's
 * preconditioner is already queued; on return u holds the solution, and work
 * queued after the final test (which touches only internal vectors) may
 * still be running on the stream.  iters: iterations done;
 * res_hist: optional host array of imax+1 residual norms.  Returns
 * SEM_ENOCONV when imax is reached (u holds the last iterate).  A zero
 * initial residual returns at once: iters = 0, u unchanged. */
sem_status sem_pcg_solve(sem_handle h, double *u, const double *f, int32_t imax, double rtol,
                         const int32_t *ns1, const int32_t *ns2, int32_t *iters,
                         double *res_hist);

/* Kernel timing for measurement.  When enabled for `level`, the kernels of
 * every Schwarz smoothing step (Algorithm 2's subdomain solves and weighted
 * scatter), residual, restriction and prolongation on that level are timed
 * with a pair of HIP events that the kernel dispatch itself records at the
 * kernels' start and end (hipExtLaunchKernel), on the handle's stream: the
 * time is the kernels' own, without dispatch gaps.  sem_timing_read_all
 * synchronises the stream and writes, per kind (sem_timing_kind), the number
 * of timed launches count[SEM_TIME_KINDS] and their summed duration in
 * milliseconds total_ms[SEM_TIME_KINDS] (host arrays), then clears the
 * record; sem_timing_read returns the Schwarz kind only.  At most 65536
 * launches are recorded between reads; later launches are not timed.
 * on = 0 disables recording.  SEM_EINVAL for level < 1 or null pointers. */
typedef enum {
  SEM_TIME_SCHWARZ = 0,   /* subdomain solves and weighted scatter      */
  SEM_TIME_RESIDUAL = 1,  /* r = f - A u                                */
  SEM_TIME_RESTRICT = 2,
  SEM_TIME_PROLONG = 3,
  SEM_TIME_APPLY = 4,     /* q = A p (no right-hand side), MGCG's product */
  SEM_TIME_KINDS = 5
} sem_timing_kind;
sem_status sem_timing_enable(sem_handle h, int32_t level, int32_t on);
sem_status sem_timing_read(sem_handle h, int64_t *count, double *total_ms);
sem_status sem_timing_read_all(sem_handle h, int64_t *count, double *total_ms);

/* ------------------------------------------------------------------------
 * Learned Schwarz parameters (a project extension; the paper fixes the
 * weights of Section 3.1 and the overlap rules of Section 4 by hand).  A
 * small network predicts, per element, a width scale alpha for the
 * smoothed-sign weights and an overlap ratio from local features; the
 * predictions are reduced to the per-grid-line width scales and per-level
 * overlaps that sem_setup accepts (sem_weights.alpha_x / alpha_y,
 * sem_overlap.per_level).
 * ------------------------------------------------------------------------ */

/* Features of every element e = ey * nx + ex of the finest level, 8 FP32
 * values per element, written to the device array feat[n_e][8]:
 *   0  log2(h_x / h_y)
 *   1  ln nu_bar_e, the GLL-quadrature element mean of nu used by the local
 *      solves (Section 4, variable diffusion); 0 for the Poisson problem
 *   2-5  ln nu_bar of the left, right, lower and upper neighbour minus
 *      ln nu_bar_e (0 where the side is a Dirichlet boundary)
 *   6  ln(max nu / min nu) over the element's nodes
 *   7  p / 32 */
sem_status sem_elem_features(sem_handle h, float *feat);

/* Multilayer perceptron d_in -> width -> width -> d_out with tanh hidden
 * layers and logistic outputs, trained on the device with the loss
 * 1/(2n) sum_s sum_o (y_so - t_so)^2 and Adam (beta1 0.9, beta2 0.999,
 * eps 1e-8, bias-corrected).  The library supports width = 64, d_in <= 16,
 * d_out <= 4 (SEM_EUNSUP otherwise).  Parameters are one flat FP32 array:
 * W1 (width x d_in, row-major), b1, W2 (width x width), b2, W3
 * (d_out x width), b3. */
typedef struct sem_mlp_ctx *sem_mlp;
sem_status sem_mlp_num_params(int32_t d_in, int32_t width, int32_t d_out, int64_t *n);
/* params: host array of the initial parameters (copied). */
sem_status sem_mlp_create(int32_t d_in, int32_t width, int32_t d_out, const float *params,
                          void *stream, sem_mlp *out);
sem_status sem_mlp_destroy(sem_mlp m);
/* y[n][d_out] = network(x[n][d_in]); device arrays, asynchronous. */
sem_status sem_mlp_forward(sem_mlp m, const float *x, int64_t n, float *y);
/* Gradient of the loss over the n samples (x[n][d_in], targets t[n][d_out],
 * device) into the device array grad[num_params]; *loss (host, may be NULL)
 * receives the loss and then the call synchronises.  Deterministic. */
sem_status sem_mlp_gradient(sem_mlp m, const float *x, const float *t, int64_t n, float *grad,
                            float *loss);
/* One Adam step with learning rate lr on the full batch of n samples;
 * *loss (may be NULL) receives the loss before the step (synchronises). */
sem_status sem_mlp_train_step(sem_mlp m, const float *x, const float *t, int64_t n, float lr,
                              float *loss);
/* Host copy of the current parameters (synchronises). */
sem_status sem_mlp_get_params(sem_mlp m, float *params);

/* Host-side reduction of per-element predictions pred[n_e][2] = (alpha_e,
 * q_e) (host array, e = ey * nx + ex) to setup parameters:
 *   alpha_e clipped to [0.1, 1]; alpha_x[i] (nx+1 entries) and alpha_y[j]
 *   (ny+1 entries) = mean of alpha_e over the elements touching grid line
 *   i or j (periodic: the first and last line are one line);
 *   rho = 0.5 mean_e q_e; overlaps[l] = ceil(rho p_l) clamped to
 *   [1, p_l - 1] and to p_l + 1 + 2 n_o <= 48, for l = 1..L, overlaps[0] = 0
 *   (L+1 entries, p_l ceil-halving from p to 1).
 * A constant width scale along every grid line keeps the weights a partition
 * of unity.  SEM_ENAN for non-finite predictions. */
sem_status sem_learned_params(const float *pred, int32_t nx, int32_t ny, int32_t p, int32_t bc,
                              int32_t *overlaps, double *alpha_x, double *alpha_y);

/* Euclidean norm of the unknowns of a level-L array (synchronises). */
sem_status sem_norm(sem_handle h, const double *x, double *out);

/* sem_norm for callers that cannot allocate device memory (code under HIP
 * graph capture, tight serving loops, harnesses that forbid hipMalloc): the
 * same result from the same kernels, but the reduction's partial sums live
 * in a fixed device array of the library (520 doubles, about 4 KB, one copy
 * per GPU, resolved by sem_setup and held until the process ends) instead of
 * the handle's buffer.  The call allocates nothing.  Any array size is
 * accepted: the reduction never uses more than 512 partial sums.  Every call on one GPU shares that array, so
 * calls that overlap on one GPU (several streams or threads) race.
 * SEM_EINVAL for null arguments, SEM_EHIP when a runtime call fails. */
sem_status sem_norm_noalloc(sem_handle h, const double *x, double *out);

const char *sem_strerror(sem_status s);
const char *sem_last_error(sem_handle h);

/* ---- 3-D Poisson extension ----------------------------------------------
 * The method in three dimensions, which the paper's conclusions (Section 5)
 * name as the next step: -lap u = f on a tensor-product mesh of hexahedral
 * spectral elements with homogeneous Dirichlet boundaries.  Everything
 * carries over direction by direction:
 *   A = M_z (x) M_y (x) L_x + M_z (x) L_y (x) M_x + L_z (x) M_y (x) M_x;
 * extended-element subdomains are products of the 1-D windows (Section
 * 3.1) with weights w_z w_y w_x; the local solves are 3-D fast
 * diagonalisations; transfers interpolate along each axis (Section 3.2);
 * the coarse problem (p = 1) is solved by a global fast diagonalisation;
 * Algorithms 3 and 4 are unchanged.  FP64.  Node arrays are device arrays
 * u[z][y][x] with (n_d p_l + 1) nodes per direction, boundary included and
 * written as zero.  Subdomain width p_l + 1 + 2 n_o <= 15 (SEM_EUNSUP
 * otherwise). */
typedef struct sem3_ctx *sem3_handle;
typedef struct {
  int32_t nx, ny, nz;               /* elements per direction            */
  const double *xb, *yb, *zb;       /* host arrays of n+1 increasing breaks */
} sem_mesh3;
/* wf: odd kappa or SEM_W_TOPHAT.  stream: hipStream_t (NULL = default). */
sem_status sem3_setup(const sem_mesh3 *mesh, int32_t p, const sem_overlap *overlap, int32_t wf,
                      void *stream, sem3_handle *out);
sem_status sem3_destroy(sem3_handle h);
sem_status sem3_num_levels(sem3_handle h, int32_t *n);
/* nodes[3]: nodes along x, y, z of level `level`. */
sem_status sem3_level_info(sem3_handle h, int32_t level, int32_t *p, int32_t *n_o, int64_t *nodes);
/* r = f - A u (f = NULL: r = A u) on one level. */
sem_status sem3_residual(sem3_handle h, int32_t level, const double *u, const double *f, double *r);
/* n_it sweeps of Algorithm 2 on level >= 1, in place on u. */
sem_status sem3_schwarz_smooth(sem3_handle h, int32_t level, double *u, const double *f,
                               int32_t n_it);
/* fc = I^T rf from level to level-1; uf += I uc from level-1 to level. */
sem_status sem3_restrict(sem3_handle h, int32_t level, const double *rf, double *fc);
sem_status sem3_prolong_add(sem3_handle h, int32_t level, const double *uc, double *uf);
/* u0 = A_0^{-1} f0 on level 0. */
sem_status sem3_coarse_solve(sem3_handle h, const double *f0, double *u0);
/* One V-cycle (Algorithm 3) on the finest level; ns1/ns2 per level or NULL
 * (MG(1,0)). */
sem_status sem3_vcycle(sem3_handle h, double *u, const double *f, const int32_t *ns1,
                       const int32_t *ns2);
/* MGCG (Algorithm 4) to ||r|| <= rtol ||r_0||: *iters, hist[0..*iters]
 * (host, imax+1 entries, may be NULL); SEM_ENOCONV at imax, SEM_ENAN on a
 * non-finite residual; synchronises. */
sem_status sem3_pcg_solve(sem3_handle h, double *u, const double *f, int32_t imax, double rtol,
                          const int32_t *ns1, const int32_t *ns2, int32_t *iters, double *hist);
const char *sem3_last_error(sem3_handle h);

#ifdef __cplusplus
}
#endif
#endif /* SEM_H */
