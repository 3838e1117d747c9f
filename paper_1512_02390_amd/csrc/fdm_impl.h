#pragma once
// Weighted additive Schwarz correction (Section 3.1, Algorithm 2): for every
// extended element s,
//     u += R_s^T (W_y (x) W_x) (S_y (x) S_x) D_s (S_y^T (x) S_x^T) R_s r
// with D_s = diag(1 / (nu_bar_s (lambda_y,i + lambda_x,j))) -- the fast
// diagonalisation of A_ss^{-1} (Lynch-Rice-Thomas), scaled by 1/nu_bar_s for
// variable diffusion (Section 4).
//
// Mapping onto gfx950: one work item of EPW = 64/m elements that share their
// subdomain type in x and in y, so the factor matrices S, S^T are wave-
// uniform: they enter every FMA as scalar-register operands (wide tiles) or
// as broadcast reads of a copy staged in LDS once per block (m <= 16).  A
// work item runs on one 64-lane wavefront (k_fdm) or, for mid-size tiles, on
// two that split every stage's outputs (k_fdm2, further down).
//   stage 1  lane = tile column j: T1[:, j] = S_y^T r_s[:, j]      (m^2 FMA)
//   LDS transpose (one m x m tile per element)
//   stage 2  lane = tile row i:    T2[i, :] = T1[i, :] S_x         (m^2 FMA)
//            T2 *= D_s
//   stage 3                        T3[i, :] = T2[i, :] S_x^T       (m^2 FMA)
//   LDS transpose back
//   stage 4  lane = tile column j: du[:, j] = W_y S_y T3[:, j]     (m^2 FMA)
// Each stage loops over its outputs; one output is the dot product of one
// uniform matrix row (a few wide scalar loads) with the lane's register-
// resident input vector, so only one matrix row at a time occupies scalar
// registers, and the result goes straight to LDS (or to the atomic add).
// The weighted tile is added into u with hardware FP64 atomics (overlapping
// subdomains touch the same nodes); rounding order therefore varies between
// runs at the 1e-16 level.
//
// Dirichlet boundaries: tile positions that are not unknowns read r = 0 and
// are never written; their S rows/columns are identity padding with
// lambda = 1, which keeps them decoupled.
#include "common.h"
#include "kernels.h"

#include <type_traits>

namespace sem {
namespace {

// Dot product of a wave-uniform matrix row (scalar operands) with a
// register-resident vector, in two interleaved chains.
template <typename T, int M>
__device__ __forceinline__ T urow_dot(cptr<T> row, const T (&x)[M]) {
  T a0 = T(0), a1 = T(0);
#pragma unroll
  for (int i = 0; i + 1 < M; i += 2) {
    a0 = fma(row[i], x[i], a0);
    a1 = fma(row[i + 1], x[i + 1], a1);
  }
  if constexpr (M % 2) a0 = fma(row[M - 1], x[M - 1], a0);
  return a0 + a1;
}

// The same with the row in LDS (uniform address: one broadcast read per
// element of the row, returned in order, so the next rows can be in flight).
template <typename T, int M>
__device__ __forceinline__ T lrow_dot(const T *row, const T (&x)[M]) {
  T a0 = T(0), a1 = T(0);
#pragma unroll
  for (int i = 0; i + 1 < M; i += 2) {
    a0 = fma(row[i], x[i], a0);
    a1 = fma(row[i + 1], x[i + 1], a1);
  }
  if constexpr (M % 2) a0 = fma(row[M - 1], x[M - 1], a0);
  return a0 + a1;
}

// Small tiles take their factor matrices from LDS.  With few wavefronts per
// SIMD, a scalar-register row costs one full cache round trip per row
// (scalar loads complete out of order, so each use waits for all of them);
// staging the four matrices once, with vector loads that are all in flight
// together, costs one round trip per wavefront.  Wide tiles keep the scalar
// path: there the FMAs dominate and broadcast LDS reads would compete with
// them for issue slots.
template <typename T, int M>
constexpr bool fdm_lds_factors() { return M <= 16; }

// Output rows per loop iteration: two for small tiles, so that the scalar
// loads of the next factor row overlap the current row's FMAs; one row (the
// largest set of factor values held in scalar registers) beyond that.
template <typename T, int M>
constexpr int fdm_rows_per_iter() { return M * (int)sizeof(T) <= 128 ? 2 : 1; }

template <typename T, int M>
__global__ __launch_bounds__(64) void k_fdm(FdmArgs<T> A) {
  constexpr int RU = fdm_rows_per_iter<T, M>();
  constexpr int EPW = 64 / M;
  constexpr int LS = M + 1;  // LDS row stride
  // one tile per element slot; lanes beyond the last slot read slot EPW-1
  // and never write
  __shared__ T lds[EPW * M * LS];
  constexpr bool LF = fdm_lds_factors<T, M>();
  __shared__ T fac[LF ? 4 * M * M : 1];   // S_y^T, diag(w_y) S_y, S_x, S_x^T
  const FdmTask *__restrict__ task = A.tasks + blockIdx.x;
  const int ty = task->ty, tx = task->tx, cnt = task->count;
  const int lane = threadIdx.x;
  const int k = lane / M;
  const int j = lane - k * M;
  const bool act = k < cnt;
  const bool has_tile = k < EPW;
  const int packed = task->elem[act ? k : 0];
  const int ey = packed >> 16, ex = packed & 0xffff;
  const Grid g = A.g;
  const int per = g.periodic;
  // wave-uniform factor matrices: every row is read with scalar loads
  // (constant address space: scalar loads also in the loop that scatters)
  const cptr<T> SyT = as_const(A.SyT) + (long)ty * M * M;   // S_y^T
  const cptr<T> SyW = as_const(A.SyW) + (long)ty * M * M;   // diag(w_y) S_y
  const cptr<T> Sx = as_const(A.Sx) + (long)tx * M * M;     // S_x
  const cptr<T> SxT = as_const(A.SxT) + (long)tx * M * M;   // S_x^T
  const int row0 = ey * g.p - A.n_o;
  int gc = ex * g.p - A.n_o + j;
  bool vc;
  if (per) {
    gc = wrap(gc, g.cols);
    vc = true;
  } else {
    vc = gc >= 1 && gc <= g.cols - 2;
  }
  T *tile = lds + (has_tile ? k : EPW - 1) * M * LS;
  if constexpr (LF) {
    const T *src[4] = {A.SyT + (long)ty * M * M, A.SyW + (long)ty * M * M,
                       A.Sx + (long)tx * M * M, A.SxT + (long)tx * M * M};
#pragma unroll
    for (int q = 0; q < 4; ++q)
#pragma unroll
      for (int i = lane; i < M * M; i += 64) fac[q * M * M + i] = src[q][i];
  }

  // ---- gather the residual tile column (branch-free, always in bounds) ----
  T X[M];
#pragma unroll
  for (int i = 0; i < M; ++i) {
    int gr = row0 + i;
    bool ok;
    if (per) {
      gr += (gr < 0) ? g.rows : 0;
      gr -= (gr >= g.rows) ? g.rows : 0;
      ok = act;
    } else {
      ok = act && vc && gr >= 1 && gr <= g.rows - 2;
    }
    const long idx = ok ? (long)gr * g.cols + gc : 0;
    const T v = A.r[idx];
    X[i] = ok ? v : T(0);
  }
  // the row of 1/(lambda_y + lambda_x) used in stage 2 (lane = tile row j),
  // fetched now so that its latency overlaps stage 1
  const T *__restrict__ d = A.dinv + ((long)ty * A.ntx + tx) * M * M + j * M;
  const T s = A.nuinv ? A.nuinv[(long)ey * g.nx + ex] : T(1);
  T dv[M <= 32 ? M : 1];
  if constexpr (M <= 32) {
#pragma unroll
    for (int c = 0; c < M; ++c) dv[c] = d[c];
  }
  // ---- stage 1: T1 = S_y^T R, lane = column j; row a of T1 -> LDS ----------
  if constexpr (LF) {
    __syncthreads();   // factor matrices staged
#pragma unroll
    for (int a = 0; a < M; ++a) {
      const T v = lrow_dot<T, M>(fac + a * M, X);
      if (has_tile) tile[a * LS + j] = v;
    }
  } else {
#pragma unroll RU
    for (int a = 0; a < M; ++a) {
      const T v = urow_dot<T, M>(SyT + a * M, X);
      if (has_tile) tile[a * LS + j] = v;
    }
  }
  __syncthreads();
  // ---- stage 2: T2 = T1 S_x, lane = row j, divided by nu_bar (lambda_y + lambda_x)
#pragma unroll
  for (int b = 0; b < M; ++b) X[b] = tile[j * LS + b];
  if constexpr (M <= 32) {
    // the eigenvalue row sits in registers next to the tile row
#pragma unroll
    for (int c = 0; c < M; ++c) dv[c] *= s;
    if constexpr (LF) {
#pragma unroll
      for (int c = 0; c < M; ++c) {
        const T v = lrow_dot<T, M>(fac + 3 * M * M + c * M, X);
        if (has_tile) tile[j * LS + c] = v;
      }
    } else {
#pragma unroll RU
      for (int c = 0; c < M; ++c) {
        const T v = urow_dot<T, M>(SxT + c * M, X);
        if (has_tile) tile[j * LS + c] = v;
      }
    }
#pragma unroll
    for (int c = 0; c < M; ++c) X[c] = tile[j * LS + c] * dv[c];
  } else {
    // large tiles: scale each output as it is produced
#pragma unroll 1
    for (int c = 0; c < M; ++c) {
      const T v = urow_dot<T, M>(SxT + c * M, X) * (d[c] * s);
      if (has_tile) tile[j * LS + c] = v;
    }
#pragma unroll
    for (int c = 0; c < M; ++c) X[c] = tile[j * LS + c];
  }
  // ---- stage 3: T3 = T2 S_x^T ------------------------------------------------------
  if constexpr (LF) {
#pragma unroll
    for (int b = 0; b < M; ++b) {
      const T v = lrow_dot<T, M>(fac + 2 * M * M + b * M, X);
      if (has_tile) tile[j * LS + b] = v;
    }
  } else {
#pragma unroll RU
    for (int b = 0; b < M; ++b) {
      const T v = urow_dot<T, M>(Sx + b * M, X);
      if (has_tile) tile[j * LS + b] = v;
    }
  }
  __syncthreads();
  // ---- stage 4: du = diag(w_y) S_y T3, lane = column j; weighted scatter-add ------
#pragma unroll
  for (int a = 0; a < M; ++a) X[a] = tile[a * LS + j];
  const T *__restrict__ we = A.wel ? A.wel + ((long)ey * g.nx + ex) * 2 * M : nullptr;
  const T wxj = (act && vc) ? (we ? we[M + j] : A.wx[(long)ex * M + j]) : T(0);
#pragma unroll RU
  for (int i = 0; i < M; ++i) {
    T v;
    if constexpr (LF)
      v = lrow_dot<T, M>(fac + M * M + i * M, X);
    else
      v = urow_dot<T, M>(SyW + i * M, X);
    int gr = row0 + i;
    bool vr;
    if (per) {
      gr = wrap(gr, g.rows);
      vr = true;
    } else {
      vr = gr >= 1 && gr <= g.rows - 2;
    }
    if (act && vc && vr) {
      const long node = (long)gr * g.cols + gc;
      T c = v * wxj;
      if (we) c *= we[i] * A.dnorm[node];
      atomic_add(&A.u[node], c);
    }
  }
}

// Wide tiles: two wavefronts per work item.  Both hold the same lane ->
// (element slot, tile column/row) map; wave w computes the outputs
// [w H, min(M, (w + 1) H)) of every stage (H = ceil(M / 2)): rows of T1,
// columns of T2 and T3, rows of du.  The tile stays in one LDS buffer; a
// barrier separates every stage's reads of a tile row from the other wave's
// writes to it.  Twice the wavefronts at half the serial work each: more
// latency hiding and finer packing onto the SIMDs.  Not for FP64 rows wider
// than 32 (256 bytes): there the split kernel spills scalar registers and
// measured slower than one wavefront; nor below 9 nodes, where the extra
// barriers cost more than the shorter chains save.
template <typename T, int M>
constexpr bool fdm_two_waves() { return M >= 9 && M * (int)sizeof(T) <= 256; }

template <int V>
using ic = std::integral_constant<int, V>;
template <typename T, int M>
constexpr int kRowsPerIter = fdm_rows_per_iter<T, M>();

template <typename T, int M>
__global__ __launch_bounds__(128) void k_fdm2(FdmArgs<T> A) {
  constexpr int EPW = 64 / M;
  constexpr int LS = M + 1;  // LDS row stride
  constexpr int H = (M + 1) / 2;
  __shared__ T lds[EPW * M * LS];
  constexpr bool LF = fdm_lds_factors<T, M>();
  __shared__ T fac[LF ? 4 * M * M : 1];   // S_y^T, diag(w_y) S_y, S_x, S_x^T
  const FdmTask *__restrict__ task = A.tasks + blockIdx.x;
  const int ty = task->ty, tx = task->tx, cnt = task->count;
  const int lane = threadIdx.x & 63;
  // wave index, stated uniform so that the halves below are scalar branches
  const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int k = lane / M;
  const int j = lane - k * M;
  const bool act = k < cnt;
  const bool has_tile = k < EPW;
  const int packed = task->elem[act ? k : 0];
  const int ey = packed >> 16, ex = packed & 0xffff;
  const Grid g = A.g;
  const int per = g.periodic;
  const cptr<T> SyT = as_const(A.SyT) + (long)ty * M * M;   // S_y^T
  const cptr<T> SyW = as_const(A.SyW) + (long)ty * M * M;   // diag(w_y) S_y
  const cptr<T> Sx = as_const(A.Sx) + (long)tx * M * M;     // S_x
  const cptr<T> SxT = as_const(A.SxT) + (long)tx * M * M;   // S_x^T
  const int row0 = ey * g.p - A.n_o;
  int gc = ex * g.p - A.n_o + j;
  bool vc;
  if (per) {
    gc = wrap(gc, g.cols);
    vc = true;
  } else {
    vc = gc >= 1 && gc <= g.cols - 2;
  }
  T *tile = lds + (has_tile ? k : EPW - 1) * M * LS;
  T X[M];
  if constexpr (LF) {
    const T *src[4] = {A.SyT + (long)ty * M * M, A.SyW + (long)ty * M * M,
                       A.Sx + (long)tx * M * M, A.SxT + (long)tx * M * M};
#pragma unroll
    for (int q = 0; q < 4; ++q)
      for (int i = threadIdx.x; i < M * M; i += 128) fac[q * M * M + i] = src[q][i];
  }
  // row q of factor matrix f (0: S_y^T, 1: diag(w_y) S_y, 2: S_x, 3: S_x^T)
  // dotted with the lane's vector, from LDS or scalar registers
  auto rdot = [&](int f, int q) -> T {
    if constexpr (LF) {
      return lrow_dot<T, M>(fac + f * M * M + q * M, X);
    } else {
      const cptr<T> base = f == 0 ? SyT : f == 1 ? SyW : f == 2 ? Sx : SxT;
      return urow_dot<T, M>(base + q * M, X);
    }
  };
  const T *__restrict__ d = A.dinv + ((long)ty * A.ntx + tx) * M * M + j * M;
  const T s = A.nuinv ? A.nuinv[(long)ey * g.nx + ex] : T(1);

  // ---- gather the residual tile column (both waves) --------------------------------
#pragma unroll
  for (int i = 0; i < M; ++i) {
    int gr = row0 + i;
    bool ok;
    if (per) {
      gr += (gr < 0) ? g.rows : 0;
      gr -= (gr >= g.rows) ? g.rows : 0;
      ok = act;
    } else {
      ok = act && vc && gr >= 1 && gr <= g.rows - 2;
    }
    const long idx = ok ? (long)gr * g.cols + gc : 0;
    const T v = A.r[idx];
    X[i] = ok ? v : T(0);
  }
  // each stage on the wave's half of the outputs, with compile-time bounds
  auto half = [&](auto body) {
    if (w == 0)
      body(ic<0>{}, ic<H>{});
    else
      body(ic<H>{}, ic<M>{});
  };
  if constexpr (LF) __syncthreads();   // factor matrices staged
  // ---- stage 1: rows a of T1 = S_y^T R (lane = column j) ---------------------------
  half([&](auto lo, auto hi) {
#pragma unroll kRowsPerIter<T, M>
    for (int a = decltype(lo)::value; a < decltype(hi)::value; ++a) {
      const T v = rdot(0, a);
      if (has_tile) tile[a * LS + j] = v;
    }
  });
  __syncthreads();
#pragma unroll
  for (int b = 0; b < M; ++b) X[b] = tile[j * LS + b];   // row j of T1
  __syncthreads();
  // ---- stage 2: columns c of T2 = T1 S_x, divided by nu_bar (lambda_y + lambda_x)
  // as the row is read back for stage 3 (the eigenvalue row's loads are all
  // in flight together there, instead of one round trip per output) ----------------
  half([&](auto lo, auto hi) {
#pragma unroll kRowsPerIter<T, M>
    for (int c = decltype(lo)::value; c < decltype(hi)::value; ++c) {
      const T v = rdot(3, c);
      if (has_tile) tile[j * LS + c] = v;
    }
  });
  __syncthreads();
#pragma unroll
  for (int c = 0; c < M; ++c) X[c] = tile[j * LS + c] * (d[c] * s);   // row j of T2
  __syncthreads();
  // ---- stage 3: columns b of T3 = T2 S_x^T ----------------------------------------
  half([&](auto lo, auto hi) {
#pragma unroll kRowsPerIter<T, M>
    for (int b = decltype(lo)::value; b < decltype(hi)::value; ++b) {
      const T v = rdot(2, b);
      if (has_tile) tile[j * LS + b] = v;
    }
  });
  __syncthreads();
  // ---- stage 4: rows i of du = diag(w_y) S_y T3 (lane = column j); scatter-add ----
#pragma unroll
  for (int a = 0; a < M; ++a) X[a] = tile[a * LS + j];
  const T *__restrict__ we = A.wel ? A.wel + ((long)ey * g.nx + ex) * 2 * M : nullptr;
  const T wxj = (act && vc) ? (we ? we[M + j] : A.wx[(long)ex * M + j]) : T(0);
  half([&](auto lo, auto hi) {
#pragma unroll kRowsPerIter<T, M>
    for (int i = decltype(lo)::value; i < decltype(hi)::value; ++i) {
      const T v = rdot(1, i);
      int gr = row0 + i;
      bool vr;
      if (per) {
        gr = wrap(gr, g.rows);
        vr = true;
      } else {
        vr = gr >= 1 && gr <= g.rows - 2;
      }
      if (act && vc && vr) {
        const long node = (long)gr * g.cols + gc;
        T c = v * wxj;
        if (we) c *= we[i] * A.dnorm[node];
        atomic_add(&A.u[node], c);
      }
    }
  });
}

}  // namespace

template <typename T, int M>
void launch_fdm_m(const FdmArgs<T> &a, hipStream_t s) {
  if (a.ntasks <= 0) return;
  if constexpr (fdm_two_waves<T, M>())
    klaunch((k_fdm2<T, M>), dim3(a.ntasks), dim3(128), 0, s, a);
  else
    klaunch((k_fdm<T, M>), dim3(a.ntasks), dim3(64), 0, s, a);
}

}  // namespace sem
