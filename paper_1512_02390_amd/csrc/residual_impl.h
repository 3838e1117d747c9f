// Kernel templates of the sum-factorised residual; instantiated in
// residual_inst_*.hip.
#pragma once
// Sum-factorised SEM residual r = f - A u (Section 2, tensor-product
// operator), and further down the two-pass residual of the variable-
// coefficient operator B(nu) (Section 4).
//
// Poisson work decomposition: one block per (strip of NE = 64/p consecutive
// elements in x) x (one element row in y), of one or two 64-lane wavefronts
// with the same lane map (the second takes half of every loop's outputs, see
// nu_waves / poisson_waves below).  Every element owns the
// nodes [e p, e p + p) in each direction; the shared left/bottom node also
// receives the contribution of the neighbouring element, recomputed here so
// that no two wavefronts write the same node (no atomics, deterministic).
//
//  1. lane = node column: the column's p+1 values of the element row stay in
//     registers; the p owned rows are staged in LDS with a halo of p columns
//     on the left and one on the right; the element below's contribution to
//     the shared bottom node is contracted right away.
//  2. x-part, lane = (row, element): contracts its row segment with the
//     wave-uniform 1-D operator (scalar-register operands) and writes the p
//     results to LDS (over the staged rows for p <= 16).
//  3. y-part, lane = node column: one output row per iteration, combined at
//     once with the x-part and the assembled diagonal mass,
//       (A u)(row, col) = M_y(row) xpart + M_x(col) ypart,
//     and stored; the y-part never goes through LDS.

#include "common.h"
#include "kernels.h"

namespace sem {
namespace {

// Dot product of a wave-uniform matrix row (scalar-register operands) with a
// register-resident segment, in two interleaved chains.
template <typename T, int N>
__device__ __forceinline__ T udot(cptr<T> row, const T (&x)[N]) {
  T a0 = T(0), a1 = T(0);
#pragma unroll
  for (int i = 0; i + 1 < N; i += 2) {
    a0 = fma(row[i], x[i], a0);
    a1 = fma(row[i + 1], x[i + 1], a1);
  }
  if constexpr (N % 2) a0 = fma(row[N - 1], x[N - 1], a0);
  return a0 + a1;
}

// out[o * ostride] = s * (Op row o) . x  for o < nout, where Op is a
// wave-uniform (P+1)-column table.  The loop is kept rolled: each iteration
// brings one table row into scalar registers.
// Rows per iteration: two when a table row is at most 128 bytes (the next
// row's scalar loads then overlap the current row's FMAs), else one.
template <typename T, int P>
constexpr int rows_per_iter() { return (P + 1) * (int)sizeof(T) <= 128 ? 2 : 1; }

template <typename T, int P>
__device__ __forceinline__ void rows_apply(cptr<T> Op, const T (&x)[P + 1], T s,
                                           T *out, int ostride, int nout) {
#pragma unroll rows_per_iter<T, P>()
  for (int o = 0; o < nout; ++o) out[o * ostride] = s * udot<T, P + 1>(Op + o * (P + 1), x);
}

// Sum over the 64 lanes of a wavefront, result in every lane.
__device__ __forceinline__ double wave_sum64(double v) {
#pragma unroll
  for (int s = 32; s > 0; s >>= 1) v += __shfl_xor(v, s, 64);
  return v;
}

// Per-block partial of the fused dot product: the wavefronts' sums added in
// wavefront order, written by thread 0 to part[block].  Every thread of the
// block calls it (it holds a barrier when the block has several wavefronts).
__device__ __forceinline__ void block_dot_part(double dsum, double *dsw, int wi, int nwaves,
                                               double *part) {
  dsum = wave_sum64(dsum);
  if (nwaves > 1) {
    if ((threadIdx.x & 63) == 0) dsw[wi] = dsum;
    __syncthreads();
    if (threadIdx.x == 0) {
      dsum = dsw[0];
      for (int i = 1; i < nwaves; ++i) dsum += dsw[i];
    }
  }
  if (threadIdx.x == 0) part[(long)blockIdx.y * gridDim.x + blockIdx.x] = dsum;
}

// Load a node-array segment of P+1 consecutive nodes along a row or a column.
template <typename T, int P>
__device__ __forceinline__ void load_col(const T *__restrict__ u, int row0, int col, const Grid &g,
                                         bool on, T (&seg)[P + 1]) {
#pragma unroll
  for (int b = 0; b <= P; ++b) {
    const T v = node_value(u, row0 + b, on ? col : 1, g.rows, g.cols, g.periodic);
    seg[b] = on ? v : T(0);
  }
}

// Nodal coefficient at (row, col): periodic indices wrap, Dirichlet indices
// are clamped into the stored array (only lanes whose result is discarded
// ever ask for a node outside it).
template <typename T>
__device__ __forceinline__ T coef_value(const T *__restrict__ a, int row, int col, int rows,
                                        int cols, int periodic) {
  // both index forms, then a select (no branch: see node_value)
  const int r = periodic ? wrap(row, rows) : min(max(row, 0), rows - 1);
  const int c = periodic ? wrap(col, cols) : min(max(col, 0), cols - 1);
  return a[(long)r * cols + c];
}

// Wavefronts per block of the residual kernels.  With one block per element
// strip and element row, one wavefront per block leaves the SIMDs under-
// occupied at these sizes; from p = 8 (Poisson: p = 4) a second wavefront
// holds the same lane map and takes half of the outputs of every loop, while
// the staging into LDS and the boundary writes stay with wave 0.
template <int P>
constexpr int nu_waves() { return P >= 8 ? 2 : 1; }
template <int P>
constexpr int poisson_waves() { return P >= 4 ? 2 : 1; }

// Wave w's share [lo, hi) of n outputs.
template <int NW>
__device__ __forceinline__ void share(int n, int w, int &lo, int &hi) {
  const int h = (n + NW - 1) / NW;
  lo = min(n, w * h);
  hi = min(n, lo + h);
}

template <typename T, int P, int NW, int KR>
__global__ __launch_bounds__(64 * NW * KR) void k_residual(ResidualArgs<T> A) {
  constexpr int NE = 64 / P;
  constexpr int W = NE * P;
  constexpr int LW = W + P + 1;
  // For P <= 16 the x-part results overwrite the staged rows (one LDS array);
  // larger orders keep them apart so that the left segment can be read after
  // the main contraction without holding it in registers.
  constexpr bool kAlias = P <= 16;
  // rows 0..P of the element row; rows below P with a halo of p columns on the
  // left and one on the right, row P (the top row) on the strip's columns only
  __shared__ T su_all[KR][P + 1][LW];
  __shared__ T sxp_all[KR][kAlias ? 1 : P][kAlias ? 1 : W];  // x-part per owned node
  __shared__ T ytop[KR][W];        // y-part of element row k at its top row (for row k + 1)
  __shared__ double dsw[KR * NW];  // per-wave parts of the fused dot product
  const Grid g = A.g;
  const int per = g.periodic;
  const int lane = threadIdx.x & 63;
  // wave (k, w): element row k of the block, output rows / x-part columns [lo, hi)
  const int wi = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int k = wi / NW, w = wi - (wi / NW) * NW;
  int lo, hi;
  share<NW>(P, w, lo, hi);
  const int e0 = blockIdx.x * NE;
  const int ey = blockIdx.y * KR + k;
  const bool act = ey < g.ny;   // element rows past the last: barriers only
  const int c0 = e0 * P;
  const int r0 = ey * P;
  const int eym = per ? wrap(ey - 1, g.ny) : ey - 1;
  const bool has_below = per || ey > 0;
  T(&su)[P + 1][LW] = su_all[k];
  auto sxp = [&](int a, int c) -> T & {
    if constexpr (kAlias) return su[a][c];
    else return sxp_all[k][a][c];
  };

  // ---- column of the element row (lane = column) ---------------------------
  const int c = lane;
  const int gc = c0 + c;
  // last column needed by this strip: the right end of its last element
  const int last_col = min(c0 + W, g.nx * P);
  const bool col_lane = act && c < W && gc <= last_col;
  const int q = c / P, al = c - (c / P) * P;
  const int ex = e0 + q;
  const bool out_lane = col_lane && ex < g.nx;
  // right-hand side and dot-product operand of this wave's output rows, issued
  // first so that their latency overlaps the staging and the x-part
  // (f and dot_x are never both given: one array of loads serves either)
  constexpr int HR = (P + NW - 1) / NW;
  const T *hsrc = A.f ? A.f : A.dot_x;
  T hv[HR];
#pragma unroll
  for (int t = 0; t < HR; ++t) {
    const long idx = (long)(r0 + lo + t) * g.cols + gc;
    const bool on = out_lane && lo + t < hi;
    hv[t] = (on && hsrc) ? hsrc[idx] : T(0);
  }
  // the column's u segment: wave 0 loads it and stages it for the others
  T yv[P + 1];
  if (w == 0 && act) {
    load_col<T, P>(A.u, r0, gc, g, col_lane, yv);
    if (col_lane) {
#pragma unroll
      for (int a = 0; a <= P; ++a) su[a][P + c] = yv[a];
    }
  }
  // halo columns of the owned rows
  if (act && w == 0 && (lane < P || (lane == P && c0 + W <= last_col))) {
    const int kk = lane < P ? lane : P + W;
    const int col = lane < P ? c0 - P + lane : c0 + W;
    T hl[P];   // all loads first, then the LDS stores
#pragma unroll
    for (int a = 0; a < P; ++a) hl[a] = node_value(A.u, r0 + a, col, g.rows, g.cols, per);
#pragma unroll
    for (int a = 0; a < P; ++a) su[a][kk] = hl[a];
  }
  // the first element row of the block recomputes the contribution of the
  // element below to its shared bottom row; the others take it from the
  // element row below them in the block (ytop, after the x-part)
  T extra_y = T(0);
  if (k == 0 && has_below && lo == 0 && act) {
    T seg[P + 1];
    load_col<T, P>(A.u, r0 - P, gc, g, col_lane, seg);
    extra_y = A.sy[eym] * udot<T, P + 1>(as_const(A.Lhat) + P * (P + 1), seg);
  }
  __syncthreads();
  if (w > 0 && col_lane) {
#pragma unroll
    for (int a = 0; a <= P; ++a) yv[a] = su[a][P + c];
  }
  // the y-part of this element row at its top row, for the element row above
  if (w == NW - 1 && k + 1 < KR && col_lane)
    ytop[k][c] = A.sy[ey] * udot<T, P + 1>(as_const(A.Lhat) + P * (P + 1), yv);

  // ---- x-part (lane = (row a, element q)) -------------------------------------
  {
    const int q = lane / P, a = lane - (lane / P) * P;
    const int ex = e0 + q;
    const bool xlane = act && lane < W && ex < g.nx;
    const bool has_left = per || ex > 0;
    const int exm = per ? wrap(ex - 1, g.nx) : ex - 1;
    // contribution of the left neighbour to the shared left node, formed
    // first so that only the own segment stays in registers
    T extra_x = T(0);
    T seg[P + 1];
    if (xlane && has_left && lo == 0) {
#pragma unroll
      for (int b = 0; b <= P; ++b) seg[b] = su[a][q * P + b];
      extra_x = A.sx[exm] * udot<T, P + 1>(as_const(A.Lhat) + P * (P + 1), seg);
    }
    if (xlane) {
#pragma unroll
      for (int b = 0; b <= P; ++b) seg[b] = su[a][P + q * P + b];
    }
    if constexpr (kAlias) __syncthreads();   // the results overwrite su below
    if (xlane) {
      T *xrow = &sxp(a, q * P);
      rows_apply<T, P>(as_const(A.Lhat) + lo * (P + 1), seg, A.sx[ex], xrow + lo, 1, hi - lo);
      if (lo == 0) xrow[0] += extra_x;
    }
  }
  __syncthreads();

  // ---- y-part combined with the x-part and the assembled mass (lane = column) ----
  //   (A u)(row, col) = M_y(row) xpart + M_x(col) ypart
  if (k > 0 && lo == 0 && col_lane) extra_y = ytop[k - 1][c];
  double dsum = 0.0;   // fused dot product (see ResidualArgs::dot_x)
  if (out_lane) {
    const bool has_left = per || ex > 0;
    const int exm = per ? wrap(ex - 1, g.nx) : ex - 1;
    const T mxc = A.mx[ex] * A.w[al] + ((al == 0 && has_left) ? A.mx[exm] * A.w[P] : T(0));
    const T sy = as_const(A.sy)[ey];
#pragma unroll
    for (int t = 0; t < HR; ++t) {
      const int a = lo + t;
      if (a >= hi) break;
      // the row address passes an optimisation barrier: the unrolled loop
      // then fetches one operator row at a time instead of all of them
      const cptr<T> orow = as_const(opaque(A.Lhat + a * (P + 1)));
      T yp = sy * udot<T, P + 1>(orow, yv);
      if (a == 0) yp += extra_y;
      const int row = r0 + a;
      // (wave-uniform table reads through the constant space: scalar loads
      // that need not wait for the previous row's store)
      const T myr = as_const(A.my)[ey] * as_const(A.w)[a] +
                    ((a == 0 && has_below) ? as_const(A.my)[max(eym, 0)] * as_const(A.w)[P] : T(0));
      const T au = myr * sxp(a, c) + mxc * yp;
      T v = A.f ? hv[t] - au : au;
      if (!per && (row == 0 || gc == 0)) v = T(0);
      A.out[(long)row * g.cols + gc] = v;
      if (A.dot_x) dsum += (double)v * (double)hv[t];
    }
    if (w == 0 && !per && ey == g.ny - 1) A.out[(long)(g.rows - 1) * g.cols + gc] = T(0);
  }
  if (act && w == 0 && !per && lane == 0 && e0 + NE >= g.nx) {
#pragma unroll
    for (int a = 0; a < P; ++a) A.out[(long)(r0 + a) * g.cols + g.cols - 1] = T(0);
    if (ey == g.ny - 1) A.out[(long)(g.rows - 1) * g.cols + g.cols - 1] = T(0);
  }
  if (A.dot_x) block_dot_part(dsum, dsw, wi, KR * NW, A.dot_part);
}

// ---------------------------------------------------------------------------
// Variable-coefficient residual in two passes (Section 4, operator B(nu)):
// B(nu) u = sum over elements of D_y^T G_y + D_x^T G_x with the fluxes
// G_y = w nu (D_y u) and G_x = w nu (D_x u) per element.  Pass 1 forms every
// flux exactly once; pass 2 contracts them with D^T and assembles, each node
// owned by one wavefront as in k_residual.  Flux layouts:
//   gy[(ey (p+1) + b) * cols + col]: element row ey, local row b, node column;
//   gx[(ex (p+1) + c) * rows + row]: element column ex, local column c, node
//   row (transposed, so that one lane per row reads and writes coalesced).
// ---------------------------------------------------------------------------

template <typename T, int P, int NW>
__global__ __launch_bounds__(64 * NW) void k_flux(ResidualArgs<T> A) {
  constexpr int NE = 64 / P;
  constexpr int W = NE * P;
  __shared__ T su[P][W + 1];   // owned rows of the strip and its right end
  const Grid g = A.g;
  const int per = g.periodic;
  const int lane = threadIdx.x & 63;
  const int w = NW > 1 ? __builtin_amdgcn_readfirstlane(threadIdx.x >> 6) : 0;
  int lo, hi;
  share<NW>(P + 1, w, lo, hi);
  const int e0 = blockIdx.x * NE;
  const int ey = blockIdx.y;
  const int c0 = e0 * P;
  const int r0 = ey * P;
  const int last_col = min(c0 + W, g.nx * P);
  // ---- y flux, lane = node column --------------------------------------------
  {
    const int c = lane;
    const int gc = c0 + c;
    // columns of the strip up to its right end are staged; the periodic end
    // column (index cols, node 0) is staged but owns no flux column
    const bool col_lane = c < W && gc <= last_col;
    T seg[P + 1];
    load_col<T, P>(A.u, r0, gc, g, col_lane, seg);
    if (col_lane && w == 0) {
#pragma unroll
      for (int a = 0; a < P; ++a) su[a][c] = seg[a];
    }
    if (col_lane && gc < g.cols) {
      T *out = A.gy + (long)ey * (P + 1) * g.cols + gc;
      // the coefficients of this wave's rows, loaded before the first store
      constexpr int HB = (P + 1 + NW - 1) / NW;
      T nv[HB];
#pragma unroll
      for (int t = 0; t < HB; ++t)
        nv[t] = lo + t < hi ? coef_value(A.nu, r0 + lo + t, gc, g.rows, g.cols, per) : T(0);
#pragma unroll
      for (int t = 0; t < HB; ++t) {
        const int b = lo + t;
        if (b >= hi) break;
        out[(long)b * g.cols] = udot<T, P + 1>(as_const(opaque(A.D + b * (P + 1))), seg) * nv[t];
      }
    }
    // right end of the strip (first column of the next strip)
    if (w == 0 && lane < P && c0 + W <= last_col)
      su[lane][W] = node_value(A.u, r0 + lane, c0 + W, g.rows, g.cols, per);
  }
  __syncthreads();
  // ---- x flux, lane = (row a, element q) -------------------------------------
  {
    const int q = lane / P, a = lane - (lane / P) * P;
    const int ex = e0 + q;
    if (lane < W && ex < g.nx) {
      T seg[P + 1];
#pragma unroll
      for (int d = 0; d <= P; ++d) seg[d] = su[a][q * P + d];
      const int row = r0 + a;
      T *out = A.gx + (long)ex * (P + 1) * g.rows + row;
      constexpr int HB = (P + 1 + NW - 1) / NW;
      T nv[HB];
#pragma unroll
      for (int t = 0; t < HB; ++t)
        nv[t] = lo + t < hi ? coef_value(A.nuT, ex * P + lo + t, row, g.cols, g.rows, per) : T(0);
#pragma unroll
      for (int t = 0; t < HB; ++t) {
        const int c = lo + t;
        if (c >= hi) break;
        out[(long)c * g.rows] = udot<T, P + 1>(as_const(opaque(A.D + c * (P + 1))), seg) * nv[t];
      }
    }
  }
}

template <typename T, int P, int NW>
__global__ __launch_bounds__(64 * NW) void k_residual_nu(ResidualArgs<T> A) {
  constexpr int NE = 64 / P;
  constexpr int W = NE * P;
  __shared__ T sxp[P][W];   // x-part per owned node
  __shared__ double dsum1;  // wave 1's part of the fused dot product
  const Grid g = A.g;
  const int per = g.periodic;
  const int lane = threadIdx.x & 63;
  const int w = NW > 1 ? __builtin_amdgcn_readfirstlane(threadIdx.x >> 6) : 0;
  int lo, hi;
  share<NW>(P, w, lo, hi);
  const int e0 = blockIdx.x * NE;
  const int ey = blockIdx.y;
  const int c0 = e0 * P;
  const int r0 = ey * P;
  const int eym = per ? wrap(ey - 1, g.ny) : ey - 1;
  const bool has_below = per || ey > 0;
  const int c = lane;
  const int gc = c0 + c;
  const int last_col = min(c0 + W, g.nx * P);
  const bool col_lane = c < W && gc <= last_col;
  const int gcs = (col_lane && gc < g.cols) ? gc : c0;   // an existing column
  // y-direction fluxes of this element row's column, and (for the wave that
  // owns output row 0) the element below's contribution to the shared bottom
  // node
  T yv[P + 1];
  {
    const T *gy = A.gy + (long)ey * (P + 1) * g.cols + gcs;
#pragma unroll
    for (int b = 0; b <= P; ++b) yv[b] = gy[(long)b * g.cols];
  }
  T extra_y = T(0);
  if (has_below && lo == 0) {
    T v[P + 1];
    const T *gy = A.gy + (long)eym * (P + 1) * g.cols + gcs;
#pragma unroll
    for (int b = 0; b <= P; ++b) v[b] = gy[(long)b * g.cols];
    extra_y = A.sy[eym] * udot<T, P + 1>(as_const(A.DT) + P * (P + 1), v);
  }
  // ---- x-part, lane = (row a, element q) -------------------------------------
  {
    const int q = lane / P, a = lane - (lane / P) * P;
    const int ex = e0 + q;
    if (lane < W && ex < g.nx) {
      const int row = r0 + a;
      T v[P + 1];
      {
        const T *gx = A.gx + (long)ex * (P + 1) * g.rows + row;
#pragma unroll
        for (int b = 0; b <= P; ++b) v[b] = gx[(long)b * g.rows];
      }
      rows_apply<T, P>(as_const(A.DT) + lo * (P + 1), v, A.sx[ex], &sxp[a][q * P + lo], 1,
                       hi - lo);
      if (lo == 0 && (per || ex > 0)) {
        const int exm = per ? wrap(ex - 1, g.nx) : ex - 1;
        const T *gx = A.gx + (long)exm * (P + 1) * g.rows + row;
#pragma unroll
        for (int b = 0; b <= P; ++b) v[b] = gx[(long)b * g.rows];
        sxp[a][q * P] += A.sx[exm] * udot<T, P + 1>(as_const(A.DT) + P * (P + 1), v);
      }
    }
  }
  __syncthreads();
  // ---- y-part combined with the x-part and the assembled mass (lane = column) ----
  double dsum = 0.0;   // fused dot product (see ResidualArgs::dot_x)
  const int q = c / P, al = c - (c / P) * P;
  const int ex = e0 + q;
  if (col_lane && ex < g.nx) {
    const bool has_left = per || ex > 0;
    const int exm = per ? wrap(ex - 1, g.nx) : ex - 1;
    const T mxc = A.mx[ex] * A.w[al] + ((al == 0 && has_left) ? A.mx[exm] * A.w[P] : T(0));
    const T sy = as_const(A.sy)[ey];
    // right-hand side and dot operand loaded before the first store (see k_residual)
    constexpr int HR = (P + NW - 1) / NW;
    // (f and dot_x are never both given: one array of loads serves either.
    // The loads sit in one block under the uniform test, with rows past the
    // wave's share clamped to a valid one: a branch per load would end the
    // scheduling region at each, and the loads would wait one by one.)
    const T *hsrc = A.f ? A.f : A.dot_x;
    T hv[HR];
    if (hsrc) {
#pragma unroll
      for (int t = 0; t < HR; ++t)
        hv[t] = hsrc[(long)(r0 + max(min(lo + t, hi - 1), 0)) * g.cols + gc];
    } else {
#pragma unroll
      for (int t = 0; t < HR; ++t) hv[t] = T(0);
    }
#pragma unroll
    for (int t = 0; t < HR; ++t) {
      const int a = lo + t;
      if (a >= hi) break;
      const cptr<T> orow = as_const(opaque(A.DT + a * (P + 1)));
      T yp = sy * udot<T, P + 1>(orow, yv);
      if (a == 0) yp += extra_y;
      const int row = r0 + a;
      // (wave-uniform table reads through the constant space: scalar loads
      // that need not wait for the previous row's store)
      const T myr = as_const(A.my)[ey] * as_const(A.w)[a] +
                    ((a == 0 && has_below) ? as_const(A.my)[max(eym, 0)] * as_const(A.w)[P] : T(0));
      const T au = myr * sxp[a][c] + mxc * yp;
      T v = A.f ? hv[t] - au : au;
      if (!per && (row == 0 || gc == 0)) v = T(0);
      A.out[(long)row * g.cols + gc] = v;
      if (A.dot_x) dsum += (double)v * (double)hv[t];
    }
    if (w == 0 && !per && ey == g.ny - 1) A.out[(long)(g.rows - 1) * g.cols + gc] = T(0);
  }
  if (w == 0 && !per && lane == 0 && e0 + NE >= g.nx) {
#pragma unroll
    for (int a = 0; a < P; ++a) A.out[(long)(r0 + a) * g.cols + g.cols - 1] = T(0);
    if (ey == g.ny - 1) A.out[(long)(g.rows - 1) * g.cols + g.cols - 1] = T(0);
  }
  if (A.dot_x) {
    dsum = wave_sum64(dsum);
    if constexpr (NW > 1) {
      // wave 0 + wave 1, in that order
      if (w == 1 && lane == 0) dsum1 = dsum;
      __syncthreads();
      if (w == 0) dsum += dsum1;
    }
    if (w == 0 && lane == 0) A.dot_part[(long)blockIdx.y * gridDim.x + blockIdx.x] = dsum;
  }
}

}  // namespace

template <typename T, int P>
void launch_residual_p(const ResidualArgs<T> &a, hipStream_t s) {
  constexpr int NE = 64 / P;
  if (a.nu) {
    constexpr int NW = nu_waves<P>();
    static_assert(residual_rows(P, true, sizeof(T)) == 1, "one element row per block");
    dim3 grid(ceil_div(a.g.nx, NE), a.g.ny);
    klaunch((k_flux<T, P, NW>), grid, dim3(64 * NW), 0, s, a);
    klaunch((k_residual_nu<T, P, NW>), grid, dim3(64 * NW), 0, s, a);
  } else {
    constexpr int NW = poisson_waves<P>(), KR = residual_rows(P, false, sizeof(T));
    dim3 grid(ceil_div(a.g.nx, NE), ceil_div(a.g.ny, KR));
    klaunch((k_residual<T, P, NW, KR>), grid, dim3(64 * NW * KR), 0, s, a);
  }
}

}  // namespace sem
