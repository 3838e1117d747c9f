// The coarse-grid solve and the vector kernels of the multigrid-preconditioned CG (Section 3.3).
#include "common.h"
#include "kernels.h"

#include <stdexcept>

namespace sem {

LaunchTiming &launch_timing() {
  static thread_local LaunchTiming t;
  return t;
}

namespace {

// ---------------------------------------------------------------------------
// Small dense GEMM (coarse fast diagonalisation), 16x16 tiles.
// ---------------------------------------------------------------------------
constexpr int TB = 16;
__global__ void k_gemm(int M, int N, int K, const double *__restrict__ A, long ars, long acs,
                       const double *__restrict__ B, long brs, long bcs, double *__restrict__ C,
                       long ldc, const double *__restrict__ S, long lds_) {
  __shared__ double sa[TB][TB + 1], sb[TB][TB + 1];
  const int tx = threadIdx.x, ty = threadIdx.y;
  const int row = blockIdx.y * TB + ty, col = blockIdx.x * TB + tx;
  double acc = 0.0;
  for (int k0 = 0; k0 < K; k0 += TB) {
    const int ka = k0 + tx, kb = k0 + ty;
    sa[ty][tx] = (row < M && ka < K) ? A[row * ars + ka * acs] : 0.0;
    sb[ty][tx] = (kb < K && col < N) ? B[kb * brs + col * bcs] : 0.0;
    __syncthreads();
#pragma unroll
    for (int k = 0; k < TB; ++k) acc = fma(sa[ty][k], sb[k][tx], acc);
    __syncthreads();
  }
  if (row < M && col < N) {
    if (S) acc *= S[row * lds_ + col];
    C[row * ldc + col] = acc;
  }
}

// ---------------------------------------------------------------------------
// Two-sided product C = S .* (L F R) for the coarse fast diagonalisation, one
// launch instead of two GEMMs.  One block of 8 wavefronts per 16-row strip of
// C: wavefront w forms columns [16 w, 16 w + 16) of G = L(strip, :) F with the
// FP64 matrix-core product v_mfma_f64_16x16x4 (A 16x4: lane i + 16 k holds
// A(i, k); B 4x16: lane j + 16 k holds B(k, j); the 16x16 result: lane
// j + 16 g holds rows g, g + 4, g + 8, g + 12 of column j), keeps the strip of
// G in LDS, then forms the same columns of G R.  The B operands are rows of F
// and R, read 16 consecutive values at a time; L is read through its
// transpose (lrs = 1 reads it coalesced too).  All operand loads of the
// first product are issued before it.
// ---------------------------------------------------------------------------
typedef double dbl4 __attribute__((ext_vector_type(4)));
constexpr int kSwSteps = kSandwichMax / 4;   // k steps of 4

// TF, TC: element types of F and C (FP32 arrays of the mixed-precision cycle
// are read and written directly; the arithmetic is FP64).
template <typename TF, typename TC>
__global__ __launch_bounds__(512) void k_sandwich(int nr, int nc, const double *__restrict__ L,
                                                  long lrs, long lcs, const TF *__restrict__ F,
                                                  long ldf, const double *__restrict__ R, long rrs,
                                                  long rcs, const double *__restrict__ S,
                                                  long lds_, TC *__restrict__ C, long ldc) {
  __shared__ double G[16][kSandwichMax + 1];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int i = lane & 15, kq = lane >> 4;
  const int row = blockIdx.x * 16 + i;   // strip row of this lane's A operand
  const int col = w * 16 + i;            // column of this lane's B operands
  double a1[kSwSteps], b1[kSwSteps];
#pragma unroll
  for (int t = 0; t < kSwSteps; ++t) {
    const int k = 4 * t + kq;
    a1[t] = (row < nr && k < nr) ? L[(long)row * lrs + (long)k * lcs] : 0.0;
    b1[t] = (k < nr && col < nc) ? (double)F[(long)k * ldf + col] : 0.0;
  }
  dbl4 acc = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
  for (int t = 0; t < kSwSteps; ++t)
    acc = __builtin_amdgcn_mfma_f64_16x16x4f64(a1[t], b1[t], acc, 0, 0, 0);
#pragma unroll
  for (int r = 0; r < 4; ++r) G[kq + 4 * r][col] = acc[r];
  // the second product's B operands, loaded while the strip is completed
  double b2[kSwSteps];
#pragma unroll
  for (int t = 0; t < kSwSteps; ++t) {
    const int k = 4 * t + kq;
    b2[t] = (k < nc && col < nc) ? R[(long)k * rrs + (long)col * rcs] : 0.0;
  }
  __syncthreads();
  dbl4 acc2 = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
  for (int t = 0; t < kSwSteps; ++t)
    acc2 = __builtin_amdgcn_mfma_f64_16x16x4f64(G[i][4 * t + kq], b2[t], acc2, 0, 0, 0);
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    const int ci = blockIdx.x * 16 + kq + 4 * r;
    if (ci < nr && col < nc) {
      double v = acc2[r];
      if (S) v *= S[(long)ci * lds_ + col];
      C[(long)ci * ldc + col] = (TC)v;
    }
  }
}

// y[unknown i] = sum_j Minv[i][j] x[unknown j]; unknowns form an nux-wide
// block starting at xoff of a node array with xcols columns.
template <typename T>
__global__ void k_dense_matvec(int n, const double *__restrict__ Minv,
                               const T *__restrict__ x, long xoff, int xcols, int nux,
                               T *__restrict__ y) {
  __shared__ double red[256];
  const int i = blockIdx.x;
  double s = 0.0;
  for (int j = threadIdx.x; j < n; j += blockDim.x) {
    const int jr = j / nux, jc = j - jr * nux;
    s = fma(Minv[(long)i * n + j], (double)x[xoff + (long)jr * xcols + jc], s);
  }
  red[threadIdx.x] = s;
  __syncthreads();
  for (int st = blockDim.x / 2; st > 0; st >>= 1) {
    if (threadIdx.x < st) red[threadIdx.x] += red[threadIdx.x + st];
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    const int ir = i / nux, ic = i - ir * nux;
    y[xoff + (long)ir * xcols + ic] = (T)red[0];
  }
}

// b = M f at unknowns, 0 at Dirichlet boundary nodes.
template <typename T>
__global__ void k_mass(Grid g, const T *__restrict__ f, T *__restrict__ b, const T *__restrict__ w,
                       const T *__restrict__ mx, const T *__restrict__ my) {
  const long idx = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= (long)g.rows * g.cols) return;
  const int row = (int)(idx / g.cols), col = (int)(idx - (long)row * g.cols);
  if (!g.periodic && (row == 0 || col == 0 || row == g.rows - 1 || col == g.cols - 1)) {
    b[idx] = T(0);
    return;
  }
  auto diag = [&](int i, int n_el, const T *h) -> T {
    int e = min(i / g.p, n_el - 1);
    int a = i - e * g.p;
    T v = h[e] * w[a];
    if (a == 0 && (g.periodic || e > 0)) v += h[g.periodic ? wrap(e - 1, n_el) : e - 1] * w[g.p];
    return v;
  };
  b[idx] = diag(row, g.ny, my) * diag(col, g.nx, mx) * f[idx];
}

template <typename T>
__global__ void k_zero_boundary(Grid g, T *__restrict__ x) {
  const long n = 2L * g.cols + 2L * g.rows;
  const long idx = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= n) return;
  long pos;
  if (idx < g.cols)
    pos = idx;
  else if (idx < 2L * g.cols)
    pos = (long)(g.rows - 1) * g.cols + (idx - g.cols);
  else if (idx < 2L * g.cols + g.rows)
    pos = (idx - 2L * g.cols) * g.cols;
  else
    pos = (idx - 2L * g.cols - g.rows) * g.cols + g.cols - 1;
  x[pos] = T(0);
}

template <typename T>
__global__ void k_fill(T *__restrict__ x, long n, T v) {
  const long idx = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx < n) x[idx] = v;
}

template <typename Ta, typename Tb>
__global__ void k_convert(const Ta *__restrict__ in, Tb *__restrict__ out, long n, double scale) {
  const long idx = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx < n) out[idx] = (Tb)((double)in[idx] * scale);
}

// ---------------------------------------------------------------------------
// Deterministic reductions: kRedBlocks partial sums per output, then one
// block adds them in a fixed order.
// ---------------------------------------------------------------------------
constexpr int RT = 256;

__device__ __forceinline__ double block_sum(double v, double *red) {
  red[threadIdx.x] = v;
  __syncthreads();
  for (int st = RT / 2; st > 0; st >>= 1) {
    if (threadIdx.x < st) red[threadIdx.x] += red[threadIdx.x + st];
    __syncthreads();
  }
  return red[0];
}

// Sum of part[0 .. n) in every thread of the block, in a fixed order (the
// order of k_reduce_final): consumers of a reduction add its partial sums
// themselves, each block redundantly, instead of waiting for a separate
// one-block launch.
__device__ __forceinline__ double sum_partials(const double *__restrict__ part, int n,
                                               double *red) {
  double s = 0.0;
  for (int i = threadIdx.x; i < n; i += RT) s += part[i];
  const double t = block_sum(s, red);
  __syncthreads();   // red is reused by the caller
  return t;
}

__global__ void k_dot_partial(const double *__restrict__ x, const double *__restrict__ y, long n,
                              double *__restrict__ partial) {
  __shared__ double red[RT];
  double s = 0.0;
  for (long i = (long)blockIdx.x * RT + threadIdx.x; i < n; i += (long)gridDim.x * RT)
    s = fma(x[i], y[i], s);
  s = block_sum(s, red);
  if (threadIdx.x == 0) partial[blockIdx.x] = s;
}

__global__ void k_dot2_partial(const double *__restrict__ z, const double *__restrict__ r,
                               const double *__restrict__ ro, long n, double *__restrict__ partial) {
  __shared__ double red[RT];
  double s0 = 0.0, s1 = 0.0;
  for (long i = (long)blockIdx.x * RT + threadIdx.x; i < n; i += (long)gridDim.x * RT) {
    s0 = fma(z[i], r[i] - ro[i], s0);
    s1 = fma(z[i], r[i], s1);
  }
  s0 = block_sum(s0, red);
  __syncthreads();
  s1 = block_sum(s1, red);
  if (threadIdx.x == 0) {
    partial[blockIdx.x] = s0;
    partial[kRedBlocks + blockIdx.x] = s1;
  }
}

__global__ void k_sum_partial(const double *__restrict__ x, long n, double *__restrict__ partial) {
  __shared__ double red[RT];
  double s = 0.0;
  for (long i = (long)blockIdx.x * RT + threadIdx.x; i < n; i += (long)gridDim.x * RT) s += x[i];
  s = block_sum(s, red);
  if (threadIdx.x == 0) partial[blockIdx.x] = s;
}

// res[k] = sum of partial[k * kRedBlocks ...]; one block per output
__global__ void k_reduce_final(const double *__restrict__ partial, int nb, double *__restrict__ res) {
  __shared__ double red[RT];
  double s = 0.0;
  for (int i = threadIdx.x; i < nb; i += RT) s += partial[blockIdx.x * kRedBlocks + i];
  s = block_sum(s, red);
  if (threadIdx.x == 0) res[blockIdx.x] = s;
}

__global__ void k_sub_mean(Grid g, double *__restrict__ x, const double *__restrict__ sum) {
  const long n = (long)g.rows * g.cols;
  const long idx = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx < n) x[idx] -= sum[0] / (double)n;
}

// z = (double) z32 and the partial sums of z.(r - ro) and z.r (the inputs of
// the Polak-Ribiere beta) in one pass.
__global__ void k_convert_dot2(const float *__restrict__ z32, double *__restrict__ z,
                               const double *__restrict__ r, const double *__restrict__ ro, long n,
                               double *__restrict__ partial) {
  __shared__ double red[RT];
  double s0 = 0.0, s1 = 0.0;
  for (long i = (long)blockIdx.x * RT + threadIdx.x; i < n; i += (long)gridDim.x * RT) {
    const double zi = (double)z32[i];
    z[i] = zi;
    s0 = fma(zi, r[i] - ro[i], s0);
    s1 = fma(zi, r[i], s1);
  }
  s0 = block_sum(s0, red);
  __syncthreads();
  s1 = block_sum(s1, red);
  if (threadIdx.x == 0) {
    partial[blockIdx.x] = s0;
    partial[kRedBlocks + blockIdx.x] = s1;
  }
}

__global__ void k_axpy(double alpha, const double *__restrict__ x, double *__restrict__ y, long n) {
  const long idx = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx < n) y[idx] = fma(alpha, x[idx], y[idx]);
}

// MGCG update with the reductions folded in: alpha = delta / (p.q), p.q the
// sum of the npq partials of the A p residual kernel; r.r partials (one per
// block) for the host; optionally the next V-cycle's inputs (r in FP32, a
// zero initial guess in FP32 or FP64).
__global__ void k_cg_update2(const double *__restrict__ delta, const double *__restrict__ pq_part,
                             int npq, double *__restrict__ u, const double *__restrict__ p,
                             const double *__restrict__ r_in, double *__restrict__ r_out,
                             const double *__restrict__ q, long n,
                             double *__restrict__ rr_part, float *__restrict__ r32,
                             float *__restrict__ z32, double *__restrict__ z64) {
  __shared__ double red[RT];
  const double alpha = delta[0] / sum_partials(pq_part, npq, red);
  double s = 0.0;
  for (long i = (long)blockIdx.x * RT + threadIdx.x; i < n; i += (long)gridDim.x * RT) {
    u[i] = fma(alpha, p[i], u[i]);
    const double ri = fma(-alpha, q[i], r_in[i]);
    r_out[i] = ri;
    s = fma(ri, ri, s);
    if (r32) r32[i] = (float)ri;
    if (z32) z32[i] = 0.0f;
    if (z64) z64[i] = 0.0;
  }
  s = block_sum(s, red);
  if (threadIdx.x == 0) rr_part[blockIdx.x] = s;
}

// Polak-Ribiere direction with the reductions folded in: num = z.(r - ro) and
// delta_new = z.r are the sums of the nb partials in d2_part (slots 0 and 1,
// kRedBlocks apart); beta = num / delta; p = z + beta p; block 0 stores
// delta_new (a different slot than delta: other blocks still read it).  The
// previous residual needs no copy: the update writes the new one into the
// other of two buffers.
__global__ void k_cg_direction2(const double *__restrict__ d2_part, int nb,
                                const double *__restrict__ delta, double *__restrict__ delta_new,
                                double *__restrict__ p, const double *__restrict__ z, long n) {
  __shared__ double red[RT];
  const double num = sum_partials(d2_part, nb, red);
  const double dn = sum_partials(d2_part + kRedBlocks, nb, red);
  const double beta = num / delta[0];
  for (long i = (long)blockIdx.x * RT + threadIdx.x; i < n; i += (long)gridDim.x * RT)
    p[i] = fma(beta, p[i], z[i]);
  if (blockIdx.x == 0 && threadIdx.x == 0) delta_new[0] = dn;
}

int red_blocks(long n) {
  long b = (n + RT - 1) / RT;
  return (int)(b < kRedBlocks ? (b > 0 ? b : 1) : kRedBlocks);
}

}  // namespace

void launch_gemm(int M, int N, int K, const double *A, long ars, long acs, const double *B,
                 long brs, long bcs, double *C, long ldc, const double *S, long lds,
                 hipStream_t s) {
  dim3 grid(ceil_div(N, TB), ceil_div(M, TB));
  hipLaunchKernelGGL(k_gemm, grid, dim3(TB, TB), 0, s, M, N, K, A, ars, acs, B, brs, bcs, C, ldc,
                     S, lds);
}

template <typename TF, typename TC>
void launch_sandwich(int nr, int nc, const double *L, long lrs, long lcs, const TF *F, long ldf,
                     const double *R, long rrs, long rcs, const double *S, long lds, TC *C,
                     long ldc, hipStream_t s) {
  if (nr <= 0 || nc <= 0) return;
  if (nr > kSandwichMax || nc > kSandwichMax)
    throw std::runtime_error("coarse two-sided product larger than 128");
  hipLaunchKernelGGL((k_sandwich<TF, TC>), dim3(ceil_div(nr, 16)), dim3(512), 0, s, nr, nc, L,
                     lrs, lcs, F, ldf, R, rrs, rcs, S, lds, C, ldc);
}
template void launch_sandwich<double, double>(int, int, const double *, long, long,
                                              const double *, long, const double *, long, long,
                                              const double *, long, double *, long, hipStream_t);
template void launch_sandwich<float, double>(int, int, const double *, long, long, const float *,
                                             long, const double *, long, long, const double *,
                                             long, double *, long, hipStream_t);
template void launch_sandwich<double, float>(int, int, const double *, long, long,
                                             const double *, long, const double *, long, long,
                                             const double *, long, float *, long, hipStream_t);

template <typename T>
void launch_dense_matvec(int n, const double *Minv, const T *x, long xoff, int xcols, int nux,
                         T *y, hipStream_t s) {
  hipLaunchKernelGGL((k_dense_matvec<T>), dim3(n), dim3(256), 0, s, n, Minv, x, xoff, xcols, nux,
                     y);
}
template void launch_dense_matvec<double>(int, const double *, const double *, long, int, int,
                                          double *, hipStream_t);
template void launch_dense_matvec<float>(int, const double *, const float *, long, int, int,
                                         float *, hipStream_t);

template <typename T>
void launch_mass(const Grid &g, const T *f, T *b, const T *w, const T *mx, const T *my,
                 hipStream_t s) {
  const long n = (long)g.rows * g.cols;
  hipLaunchKernelGGL(k_mass<T>, dim3(ceil_div(n, 256)), dim3(256), 0, s, g, f, b, w, mx, my);
}
template void launch_mass<double>(const Grid &, const double *, double *, const double *,
                                  const double *, const double *, hipStream_t);

template <typename T>
void launch_zero_boundary(const Grid &g, T *x, hipStream_t s) {
  if (g.periodic) return;
  const long n = 2L * g.cols + 2L * g.rows;
  hipLaunchKernelGGL(k_zero_boundary<T>, dim3(ceil_div(n, 256)), dim3(256), 0, s, g, x);
}
template void launch_zero_boundary<double>(const Grid &, double *, hipStream_t);
template void launch_zero_boundary<float>(const Grid &, float *, hipStream_t);

template <typename T>
void launch_fill(T *x, long n, T v, hipStream_t s) {
  if (n > 0) hipLaunchKernelGGL(k_fill<T>, dim3(ceil_div(n, 256)), dim3(256), 0, s, x, n, v);
}
template void launch_fill<double>(double *, long, double, hipStream_t);
template void launch_fill<float>(float *, long, float, hipStream_t);

template <typename Ta, typename Tb>
void launch_convert(const Ta *in, Tb *out, long n, double scale, hipStream_t s) {
  if (n > 0)
    hipLaunchKernelGGL((k_convert<Ta, Tb>), dim3(ceil_div(n, 256)), dim3(256), 0, s, in, out, n,
                       scale);
}
template void launch_convert<double, float>(const double *, float *, long, double, hipStream_t);
template void launch_convert<float, double>(const float *, double *, long, double, hipStream_t);

void launch_reduce(const double *partial, int nb, double *res, hipStream_t s) {
  hipLaunchKernelGGL(k_reduce_final, dim3(1), dim3(RT), 0, s, partial, nb, res);
}

int launch_dot_partials(const double *x, const double *y, long n, double *partial,
                        hipStream_t s) {
  const int nb = red_blocks(n);
  hipLaunchKernelGGL(k_dot_partial, dim3(nb), dim3(RT), 0, s, x, y, n, partial);
  return nb;
}

void launch_dot(const double *x, const double *y, long n, double *partial, double *res,
                hipStream_t s) {
  const int nb = red_blocks(n);
  hipLaunchKernelGGL(k_dot_partial, dim3(nb), dim3(RT), 0, s, x, y, n, partial);
  hipLaunchKernelGGL(k_reduce_final, dim3(1), dim3(RT), 0, s, partial, nb, res);
}

void launch_sum(const double *x, long n, double *partial, double *res, hipStream_t s) {
  const int nb = red_blocks(n);
  hipLaunchKernelGGL(k_sum_partial, dim3(nb), dim3(RT), 0, s, x, n, partial);
  hipLaunchKernelGGL(k_reduce_final, dim3(1), dim3(RT), 0, s, partial, nb, res);
}

void launch_sub_mean(const Grid &g, double *x, const double *sum, hipStream_t s) {
  const long n = (long)g.rows * g.cols;
  hipLaunchKernelGGL(k_sub_mean, dim3(ceil_div(n, 256)), dim3(256), 0, s, g, x, sum);
}

void launch_dot2_partials(const double *z, const double *r, const double *ro, long n,
                          double *partial, hipStream_t s) {
  hipLaunchKernelGGL(k_dot2_partial, dim3(red_blocks(n)), dim3(RT), 0, s, z, r, ro, n, partial);
}

void launch_convert_dot2_partials(const float *z32, double *z, const double *r, const double *ro,
                                  long n, double *partial, hipStream_t s) {
  hipLaunchKernelGGL(k_convert_dot2, dim3(red_blocks(n)), dim3(RT), 0, s, z32, z, r, ro, n,
                     partial);
}

int launch_cg_update2(const double *delta, const double *pq_part, int npq, double *u,
                      const double *p, const double *r_in, double *r_out, const double *q,
                      long n, double *rr_part, hipStream_t s, float *r32, float *z32,
                      double *z64) {
  const int nb = red_blocks(n);
  hipLaunchKernelGGL(k_cg_update2, dim3(nb), dim3(RT), 0, s, delta, pq_part, npq, u, p, r_in,
                     r_out, q, n, rr_part, r32, z32, z64);
  return nb;
}

void launch_cg_direction2(const double *d2_part, const double *delta, double *delta_new,
                          double *p, const double *z, long n, hipStream_t s) {
  const int nb = red_blocks(n);
  hipLaunchKernelGGL(k_cg_direction2, dim3(nb), dim3(RT), 0, s, d2_part, nb, delta, delta_new, p,
                     z, n);
}

void launch_axpy(double alpha, const double *x, double *y, long n, hipStream_t s) {
  hipLaunchKernelGGL(k_axpy, dim3(ceil_div(n, 256)), dim3(256), 0, s, alpha, x, y, n);
}


}  // namespace sem
