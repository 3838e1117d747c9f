// Device kernels of the SEM Schwarz / p-multigrid solver (gfx950).
#pragma once
#include <hip/hip_runtime.h>
#include <cstdint>

namespace sem {

constexpr int kMaxTile = 48;     // largest subdomain width m = p + 1 + 2 n_o
constexpr int kMaxOrder = 32;    // largest polynomial order p
constexpr int kTaskSlots = 24;   // elements per FDM work item (>= 64 / m)

// One FDM work item: up to 64/m elements sharing the same x- and y-type of
// subdomain (hence the same fast-diagonalisation factors), processed by one
// 64-wide wavefront with one lane per tile column.
struct FdmTask {
  int32_t ty, tx, count, pad;
  int32_t elem[kTaskSlots];      // (ey << 16) | ex
};

// Geometry of one level's node array.
struct Grid {
  int32_t nx, ny;        // elements
  int32_t p;             // order
  int32_t rows, cols;    // node array (Dirichlet includes boundary nodes)
  int32_t periodic;      // 0 Dirichlet, 1 periodic
};

template <typename T>
struct ResidualArgs {
  Grid g;
  const T *u, *f;        // f may be null: out = A u
  T *out;
  const T *Lhat;         // (p+1)^2 reference stiffness
  const T *D, *DT;       // (p+1)^2 derivative matrix and its transpose (variable nu)
  const T *w;            // p+1 GLL weights
  const T *sx, *sy;      // per element 2/h (x: nx, y: ny)
  const T *mx, *my;      // per element h/2
  // variable diffusivity (null for the Poisson operator), with the GLL weight
  // of the contraction direction folded in: nu(row, col) w_(row mod p) as a
  // node array, and nu(row, col) w_(col mod p) transposed (cols x rows)
  const T *nu;
  const T *nuT;
  // flux scratch of the variable-nu residual (owned by the level):
  // gy: (ny (p+1)) x cols, gx: (nx (p+1)) x rows
  T *gy, *gx;
  // optional fused dot product (with f null only): when dot_x is non-null,
  // block b of the residual kernel writes sum over its owned nodes of
  // dot_x * out to dot_part[b] (residual_blocks() entries, summed by
  // launch_reduce)
  const T *dot_x;
  double *dot_part;
};
// Element rows per block of the residual kernels: for the Poisson operator as
// many as fit about 44 KB of LDS, at most 4 (the kernel's template argument
// and the block count below both come from here); elem_bytes: sizeof of the
// arithmetic type.
constexpr int residual_rows(int p, bool nu, int elem_bytes) {
  if (nu) return 1;   // the variable-nu pair keeps one element row per block
  const int W = (64 / p) * p, LW = W + p + 1;
  const long per_row = (long)(p + 1) * LW * elem_bytes + (p > 16 ? (long)p * W * elem_bytes : 0);
  const long k = 45056 / per_row;
  return k >= 4 ? 4 : (k < 1 ? 1 : (int)k);
}
// Number of blocks (strips of 64/p elements times residual_rows element rows)
// of the residual kernel on a grid.
inline long residual_blocks(const Grid &g, bool nu, int elem_bytes) {
  const int ne = 64 / g.p, kr = residual_rows(g.p, nu, elem_bytes);
  return (long)((g.nx + ne - 1) / ne) * ((g.ny + kr - 1) / kr);
}

// Matrix-core operands of the reduced-precision Schwarz kernel, prepared at
// set-up from the FP64 factors: for every subdomain type the two B-operand
// matrices of its direction (y: S_y and (W_y S_y)^T; x: S_x and S_x^T) in
// the lane layout of v_mfma_f32_16x16x32_{f16,bf16}, as 16-bit values
// scaled by 2^-e (FP16: e per matrix brings its largest magnitude into
// [0.5, 1); BF16: e = 0).  Layout [type][matrix][KC][NB][64 lanes] of 8
// values (16 bytes) each, NB = ceil(m / 16), KC = ceil(NB / 2); the k index
// of value s in lane l of chunk c is 32 c + 4 (l / 16) + s for s < 4 and
// 32 c + 16 + 4 (l / 16) + s - 4 for s >= 4 (the row order in which the
// accumulators of the previous product arrive), the n index 16 J + l % 16.
struct MfmaOps {
  const uint4 *by = nullptr, *bx = nullptr;
  const int32_t *ey = nullptr, *ex = nullptr;   // [type][2] exponents e
};

template <typename T>
struct FdmArgs {
  Grid g;
  int32_t n_o, m;
  const FdmTask *tasks;
  int32_t ntasks;
  const T *r;
  T *u;
  const T *Sx, *SxT, *SyW, *SyT;  // per type m*m; SyW = diag(w_y) S_y
  const T *dinv;                  // per (ty, tx) pair m*m, tile index ty * ntx + tx
  int32_t ntx;                    // number of x types, or 0 when every subdomain has
                                  // its own types (ty = tx) and its own tile
  const T *wx;                    // per x-element m weights
  const T *nuinv;                 // per element 1/nu_bar or null
  // Per-element weights (learned parameters): when non-null, element
  // e = ey nx + ex has its own 1-D weights wel[e][0, m) along y and
  // wel[e][m, 2m) along x (SyW then holds the unweighted S_y, and wx is not
  // used), and every contribution is multiplied by the node's dnorm = 1/D,
  // D the sum of the subdomain weights at the node (Shepard normalisation).
  const T *wel = nullptr;
  const T *dnorm = nullptr;
  MfmaOps mo{};                   // matrix-core operands (reduced-precision path only)
};

// Multiplicative Schwarz sweeps (Algorithm 1) of one level, Poisson, FP64:
// n_it sweeps, alternately forward and reversed over e = ey nx + ex.
struct MultArgs {
  Grid g;
  int32_t n_o, m, n_it;
  const double *f;
  double *u;
  const double *Lhat, *w;          // reference stiffness, GLL weights
  const double *sx, *sy, *mx, *my;  // per element 2/h and h/2
  const double *Sy, *SyT, *Sx, *SxT;  // unweighted factors per type, m*m
  const double *dinv;              // per (ty, tx) pair m*m, tile ty * ntx + tx
  int32_t ntx;
  const int32_t *tx_of, *ty_of;    // subdomain type per element column / row
};
void launch_mult(const MultArgs &a, hipStream_t s);

template <typename T>
void launch_residual(const ResidualArgs<T> &a, hipStream_t s);
// FP32 tables and vectors, BF16 (fp16 = false) or FP16 matrix-core products
// with FP32 accumulation (m <= 48); used for tiles of at least kMfmaMinTile
// nodes.
constexpr int kMfmaMinTile = 17;
void launch_fdm_mfma(const FdmArgs<float> &a, bool fp16, hipStream_t s);
template <typename T>
void launch_fdm(const FdmArgs<T> &a, hipStream_t s);

// Transfers between level l-1 (order pc = ceil(pf/2)) and level l (order pf),
// Section 3.2.  Restriction fc = I^T rf (each fine node counted once), also
// zeroing uc_zero when non-null; prolongation uf += I uc.  E is the
// (pf+1) x (pc+1) interpolation matrix, ET its transpose.
template <typename T>
void launch_restrict(const Grid &gf, const Grid &gc, const T *rf, T *fc, T *uc_zero, const T *ET,
                     hipStream_t s);
template <typename T>
void launch_prolong(const Grid &gf, const Grid &gc, const T *uc, T *uf, const T *E, hipStream_t s);

// C(M x N) = op(A) op(B) on strided views, optional elementwise scale by S
// (same shape as C, leading dimension lds); C has leading dimension ldc.
void launch_gemm(int M, int N, int K, const double *A, long ars, long acs, const double *B,
                 long brs, long bcs, double *C, long ldc, const double *S, long lds,
                 hipStream_t s);
// C (nr x nc) = S .* (L F R) in one launch, for nr, nc <= kSandwichMax: L is
// nr x nr with element (i, k) at L[i lrs + k lcs], F nr x nc with leading
// dimension ldf, R nc x nc with element (k, j) at R[k rrs + j rcs]; S (null:
// no scaling) and C with leading dimensions lds and ldc.  F and C may be
// FP32 arrays (instantiated: double/double, float/double, double/float); the
// arithmetic is FP64.
constexpr int kSandwichMax = 128;
template <typename TF, typename TC>
void launch_sandwich(int nr, int nc, const double *L, long lrs, long lcs, const TF *F, long ldf,
                     const double *R, long rrs, long rcs, const double *S, long lds, TC *C,
                     long ldc, hipStream_t s);
// y = Minv x on the unknown block of a node array (dense inverse, var nu);
// x and y FP64 or FP32, the arithmetic FP64.
template <typename T>
void launch_dense_matvec(int n, const double *Minv, const T *x, long xoff, int xcols, int nux,
                         T *y, hipStream_t s);

// Vector helpers over whole node arrays of n entries.
template <typename T>
void launch_mass(const Grid &g, const T *f, T *b, const T *w, const T *mx, const T *my,
                 hipStream_t s);
template <typename T>
void launch_zero_boundary(const Grid &g, T *x, hipStream_t s);
template <typename T>
void launch_fill(T *x, long n, T v, hipStream_t s);
template <typename Ta, typename Tb>
void launch_convert(const Ta *in, Tb *out, long n, double scale, hipStream_t s);

// Deterministic two-stage reductions.  partial must hold kRedBlocks doubles
// per output; results land in device memory res[0..].
constexpr int kRedBlocks = 512;
// res[0] = sum x*y
void launch_dot(const double *x, const double *y, long n, double *partial, double *res,
                hipStream_t s);
// res[0] = sum x
void launch_sum(const double *x, long n, double *partial, double *res, hipStream_t s);
// res = sum of partial[0 .. nb) (fixed order).
void launch_reduce(const double *partial, int nb, double *res, hipStream_t s);
// x -= res[0] / count on the unknowns of g (mean removal, periodic)
void launch_sub_mean(const Grid &g, double *x, const double *sum, hipStream_t s);
// The MGCG loop's reductions without second-stage launches: the consumers add
// the partial sums themselves (every block, fixed order).
//   partial[b] = z.(r - ro), partial[kRedBlocks + b] = z.r  (b < red_blocks(n))
void launch_dot2_partials(const double *z, const double *r, const double *ro, long n,
                          double *partial, hipStream_t s);
//   z = (double) z32, and the partials as above
void launch_convert_dot2_partials(const float *z32, double *z, const double *r, const double *ro,
                                  long n, double *partial, hipStream_t s);
//   alpha = delta[0] / sum(pq_part[0 .. npq)); u += alpha p;
//   r_out = r_in - alpha q (r_in is left as it was: the caller keeps it as
//   the previous residual); rr_part[b] = partial sums of r_out.r_out
//   (returned: their count).  When non-null it also writes the next
//   V-cycle's inputs: r32 = (float) r_out, z32 = 0 or z64 = 0
int launch_cg_update2(const double *delta, const double *pq_part, int npq, double *u,
                      const double *p, const double *r_in, double *r_out, const double *q,
                      long n, double *rr_part, hipStream_t s, float *r32 = nullptr,
                      float *z32 = nullptr, double *z64 = nullptr);
//   beta = sum(slot 0) / delta[0]; p = z + beta p; delta_new[0] = sum(slot 1)
//   (d2_part as written by launch_dot2_partials for the same n)
void launch_cg_direction2(const double *d2_part, const double *delta, double *delta_new,
                          double *p, const double *z, long n, hipStream_t s);
// y += alpha x
void launch_axpy(double alpha, const double *x, double *y, long n, hipStream_t s);

}  // namespace sem

namespace sem {

// Learned Schwarz parameters (project extension): MLP d_in -> 64 -> 64 -> d_out.
constexpr int kMlpMaxIn = 16;
constexpr int kMlpMaxOut = 4;
constexpr int kMlpFeatures = 8;   // features per element

long mlp_num_params(int d_in, int d_out);
// Forward (part == null) or forward + backward of the mean squared error
// 1/(2n) sum (y - t)^2 over n samples; each of the nblk workgroups writes one
// row of `stride` (>= np + 1) partial sums: the gradient, then the loss.
void launch_mlp(const float *P, int d_in, int d_out, const float *X, const float *T, long n,
                float *Y, float *part, long stride, int nblk, hipStream_t s);
// Sums the partial rows; writes the gradient (if grad) and loss (if loss);
// with adam != 0 updates P, m, v (c1, c2: bias corrections 1/(1-beta^t)).
void launch_mlp_reduce(const float *part, int nblk, long stride, long np, float *grad, float *loss,
                       float *P, float *m, float *v, float lr, float c1, float c2, int adam,
                       hipStream_t s);
void launch_features(const Grid &g, const double *nu, const double *nuinv, const double *hx,
                     const double *hy, float *F, hipStream_t s);

}  // namespace sem
