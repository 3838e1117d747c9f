// Kernel templates of the sum-factorised residual; instantiated in
// residual_inst_*.hip.
#pragma once
// Sum-factorised SEM residual r = f - A u (Section 2, tensor-product
// operator; Section 4 for the variable-coefficient operator B(nu)).
//
// Work decomposition: one 64-lane wavefront per (strip of NE = 64/p
// consecutive elements in x) x (one element row in y).  Every element owns the
// nodes [e p, e p + p) in each direction; the shared left/bottom node also
// receives the contribution of the neighbouring element, recomputed here so
// that no two wavefronts write the same node (no atomics, deterministic).
//
//  y-part: lane = node column; the column's 2p+1 values of the element row and
//          the one below are held in registers and contracted with the
//          wave-uniform 1-D operator (scalar-register operands).
//  x-part: the p owned rows are staged in LDS with a halo of p columns on the
//          left and one on the right; lane = (row, element) contracts its row
//          segment, writes the result back to LDS, and the column lanes pick
//          it up.
// The two directions are combined with the assembled diagonal mass:
//   (A u)(row, col) = M_y(row) xpart + M_x(col) ypart.

#include "common.h"
#include "kernels.h"

namespace sem {
namespace {

// Dot product of a wave-uniform matrix row (scalar-register operands) with a
// register-resident segment, in two interleaved chains.
template <typename T, int N>
__device__ __forceinline__ T udot(const T *__restrict__ row, const T (&x)[N]) {
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
template <typename T, int P>
__device__ __forceinline__ void rows_apply(const T *__restrict__ Op, const T (&x)[P + 1], T s,
                                           T *out, int ostride, int nout) {
#pragma unroll 1
  for (int o = 0; o < nout; ++o) out[o * ostride] = s * udot<T, P + 1>(Op + o * (P + 1), x);
}

// Variable-coefficient flux of one element segment: v[a] = w_a nu_a (D seg)[a],
// computed through the lane's private LDS slot pv; nu_at(a) gives nu at local
// node a (read on the fly to keep register pressure low).
template <typename T, int P, typename NuAt>
__device__ __forceinline__ void nu_flux(const T *__restrict__ D, const T *__restrict__ w,
                                        const T (&seg)[P + 1], NuAt nu_at, T *pv, T (&v)[P + 1]) {
  rows_apply<T, P>(D, seg, T(1), pv, 1, P + 1);
  const T *__restrict__ wq = opaque(w);
#pragma unroll
  for (int a = 0; a <= P; ++a) v[a] = pv[a] * (wq[a] * nu_at(a));
}

// s * (row P of a uniform table) . x through the rolled loop (one row).
template <typename T, int P>
__device__ __forceinline__ T last_row(const T *__restrict__ Op, const T (&x)[P + 1], T s, T *pv) {
  rows_apply<T, P>(opaque(Op) + P * (P + 1), x, s, pv, 1, 1);
  return pv[0];
}

// Load a node-array segment of P+1 consecutive nodes along a row or a column.
template <typename T, int P>
__device__ __forceinline__ void load_col(const T *__restrict__ u, int row0, int col, const Grid &g,
                                         bool on, T (&seg)[P + 1]) {
#pragma unroll
  for (int b = 0; b <= P; ++b) seg[b] = on ? node_value(u, row0 + b, col, g.rows, g.cols, g.periodic) : T(0);
}

// Nodal coefficient at (row, col): periodic indices wrap, Dirichlet indices
// are clamped into the stored array (only lanes whose result is discarded
// ever ask for a node outside it).
template <typename T>
__device__ __forceinline__ T coef_value(const T *__restrict__ a, int row, int col, int rows,
                                        int cols, int periodic) {
  if (periodic) {
    row = wrap(row, rows);
    col = wrap(col, cols);
  } else {
    row = min(max(row, 0), rows - 1);
    col = min(max(col, 0), cols - 1);
  }
  return a[(long)row * cols + col];
}

template <typename T, int P, bool NU>
__global__ __launch_bounds__(64) void k_residual(ResidualArgs<T> A) {
  constexpr int NE = 64 / P;
  constexpr int W = NE * P;
  constexpr int LW = W + P + 1;
  __shared__ T su[P][LW];                      // owned rows, halo p left, 1 right
  __shared__ T sxp[P][W];                      // x-part per owned node
  __shared__ T syp[P][W];                      // y-part per owned node
  __shared__ T spv[NU ? 64 : 1][NU ? P + 2 : 1];  // private flux slots (variable nu)
  const Grid g = A.g;
  const int per = g.periodic;
  const int lane = threadIdx.x;
  const int e0 = blockIdx.x * NE;
  const int ey = blockIdx.y;
  const int c0 = e0 * P;
  const int r0 = ey * P;
  const int eym = per ? wrap(ey - 1, g.ny) : ey - 1;
  const bool has_below = per || ey > 0;
  T *pv = NU ? &spv[lane][0] : nullptr;

  // ---- y-part (lane = column) ----------------------------------------------
  const int c = lane;
  const int gc = c0 + c;
  // last column needed by this strip: the right end of its last element
  const int last_col = min(c0 + W, g.nx * P);
  const bool col_lane = c < W && gc <= last_col;
  const int gcs = col_lane ? gc : 0;  // a safe column for idle lanes
  T *ycol = &syp[0][col_lane ? c : 0];
  {
    T seg[P + 1];
    load_col<T, P>(A.u, r0, gc, g, col_lane, seg);
    // stage the owned rows for the x-part
    if (col_lane) {
#pragma unroll
      for (int a = 0; a < P; ++a) su[a][P + c] = seg[a];
    }
    if constexpr (NU) {
      T v[P + 1];
      nu_flux<T, P>(A.D, A.w, seg,
                    [&](int b) { return coef_value(A.nu, r0 + b, gcs, g.rows, g.cols, per); }, pv, v);
      if (col_lane) rows_apply<T, P>(A.DT, v, A.sy[ey], ycol, W, P);
    } else {
      if (col_lane) rows_apply<T, P>(A.Lhat, seg, A.sy[ey], ycol, W, P);
    }
  }
  if (has_below) {
    // the element below contributes to the shared bottom row (local node P)
    T seg[P + 1];
    load_col<T, P>(A.u, r0 - P, gc, g, col_lane, seg);
    T extra;
    if constexpr (NU) {
      T v[P + 1];
      nu_flux<T, P>(A.D, A.w, seg,
                    [&](int b) { return coef_value(A.nu, r0 - P + b, gcs, g.rows, g.cols, per); }, pv, v);
      extra = last_row<T, P>(A.DT, v, A.sy[eym], pv);
    } else {
      extra = A.sy[eym] * udot<T, P + 1>(opaque(A.Lhat) + P * (P + 1), seg);
    }
    if (col_lane) ycol[0] += extra;
  }
  // halo columns of the owned rows
  if (lane < P || (lane == P && c0 + W <= last_col)) {
    const int k = lane < P ? lane : P + W;
    const int col = lane < P ? c0 - P + lane : c0 + W;
#pragma unroll
    for (int a = 0; a < P; ++a) su[a][k] = node_value(A.u, r0 + a, col, g.rows, g.cols, per);
  }
  __syncthreads();

  // ---- x-part (lane = (row a, element q)) -------------------------------------
  {
    const int q = lane / P, a = lane - (lane / P) * P;
    const int ex = e0 + q;
    if (lane < W && ex < g.nx) {
      T *xrow = &sxp[a][q * P];
      T seg[P + 1];
#pragma unroll
      for (int b = 0; b <= P; ++b) seg[b] = su[a][P + q * P + b];
      if constexpr (NU) {
        T v[P + 1];
        nu_flux<T, P>(A.D, A.w, seg,
                      [&](int b) { return coef_value(A.nu, r0 + a, c0 + q * P + b, g.rows, g.cols, per); },
                      pv, v);
        rows_apply<T, P>(A.DT, v, A.sx[ex], xrow, 1, P);
      } else {
        rows_apply<T, P>(A.Lhat, seg, A.sx[ex], xrow, 1, P);
      }
      if (per || ex > 0) {
        const int exm = per ? wrap(ex - 1, g.nx) : ex - 1;
#pragma unroll
        for (int b = 0; b <= P; ++b) seg[b] = su[a][q * P + b];
        T extra;
        if constexpr (NU) {
          T v[P + 1];
          nu_flux<T, P>(A.D, A.w, seg,
                        [&](int b) {
                          return coef_value(A.nu, r0 + a, c0 + q * P - P + b, g.rows, g.cols, per);
                        },
                        pv, v);
          extra = last_row<T, P>(A.DT, v, A.sx[exm], pv);
        } else {
          extra = A.sx[exm] * udot<T, P + 1>(opaque(A.Lhat) + P * (P + 1), seg);
        }
        xrow[0] += extra;
      }
    }
  }
  __syncthreads();

  // ---- combine with the assembled mass and store -------------------------------------
  const int q = c / P, al = c - (c / P) * P;
  const int ex = e0 + q;
  if (col_lane && ex < g.nx) {
    const bool has_left = per || ex > 0;
    const int exm = per ? wrap(ex - 1, g.nx) : ex - 1;
    const T mxc = A.mx[ex] * A.w[al] + ((al == 0 && has_left) ? A.mx[exm] * A.w[P] : T(0));
#pragma unroll
    for (int a = 0; a < P; ++a) {
      const int row = r0 + a;
      const T myr = A.my[ey] * A.w[a] + ((a == 0 && has_below) ? A.my[eym] * A.w[P] : T(0));
      const T au = myr * sxp[a][c] + mxc * syp[a][c];
      T v = A.f ? A.f[(long)row * g.cols + gc] - au : au;
      if (!per && (row == 0 || gc == 0)) v = T(0);
      A.out[(long)row * g.cols + gc] = v;
    }
    if (!per && ey == g.ny - 1) A.out[(long)(g.rows - 1) * g.cols + gc] = T(0);
  }
  if (!per && lane == 0 && e0 + NE >= g.nx) {
#pragma unroll
    for (int a = 0; a < P; ++a) A.out[(long)(r0 + a) * g.cols + g.cols - 1] = T(0);
    if (ey == g.ny - 1) A.out[(long)(g.rows - 1) * g.cols + g.cols - 1] = T(0);
  }
}

}  // namespace

template <typename T, int P>
void launch_residual_p(const ResidualArgs<T> &a, hipStream_t s) {
  constexpr int NE = 64 / P;
  dim3 grid(ceil_div(a.g.nx, NE), a.g.ny);
  if (a.nu)
    hipLaunchKernelGGL((k_residual<T, P, true>), grid, dim3(64), 0, s, a);
  else
    hipLaunchKernelGGL((k_residual<T, P, false>), grid, dim3(64), 0, s, a);
}

}  // namespace sem
