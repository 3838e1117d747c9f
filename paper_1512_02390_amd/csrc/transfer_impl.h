// p-multigrid transfers (Section 3.2): the embedded interpolation I_l from
// level l-1 (order PC = ceil(PF/2)) to level l (order PF) and its transpose.
// Per element I_l = E_y (x) E_x with E[a][c] = l^c_c(xi^f_a).
//
// One block per (strip of NE = 64/PF elements in x) x (one element row), of
// one or two 64-lane wavefronts, sum-factorised in two 1-D passes through LDS.  Every output
// node has one owner (the element whose left/bottom half-open range holds it),
// so no atomics are needed and the result is deterministic.
//
// Restriction f_c = I^T r: each fine node counted once.  In 1-D,
//   f_c[e pc + g] = sum_{a=0..pf} E[a][g] r[e pf + a]
//                 + [g == 0] sum_{a=0..pf-1} E[a][pc] r[(e-1) pf + a].
// Prolongation u_f += I u_c: u_f[e pf + a] += sum_c E[a][c] u_c[e pc + c].
#pragma once
#include "common.h"
#include "kernels.h"

namespace sem {
namespace {

// Wavefronts per block: two from PF = 8 on (one block per element strip and
// element row leaves the SIMDs under-occupied with one).  Both hold the same
// lane map; loops over outputs are split, boundary writes stay with wave 0.
template <int PF>
constexpr int transfer_waves() { return PF >= 8 ? 2 : 1; }

// Wave w's share [lo, hi) of n outputs.
template <int NW>
__device__ __forceinline__ void tshare(int n, int w, int &lo, int &hi) {
  const int h = (n + NW - 1) / NW;
  lo = min(n, w * h);
  hi = min(n, lo + h);
}

template <typename T, int N>
__device__ __forceinline__ T tdot(cptr<T> row, const T (&x)[N]) {
  T a0 = T(0), a1 = T(0);
#pragma unroll
  for (int i = 0; i + 1 < N; i += 2) {
    a0 = fma(row[i], x[i], a0);
    a1 = fma(row[i + 1], x[i + 1], a1);
  }
  if constexpr (N % 2) a0 = fma(row[N - 1], x[N - 1], a0);
  return a0 + a1;
}

// Restriction.  ET = E^T, (PC+1) x (PF+1).  Also writes zero into uc_zero (the
// coarse correction) at every coarse node it owns, when uc_zero is non-null.
template <typename T, int PF, int NW>
__global__ __launch_bounds__(64 * NW) void k_restrict(Grid gf, Grid gc, const T *__restrict__ rf,
                                                 T *__restrict__ fc, T *__restrict__ uc_zero,
                                                 const T *__restrict__ ET) {
  constexpr int PC = (PF + 1) / 2;
  constexpr int NE = 64 / PF;
  constexpr int W = NE * PF;
  constexpr int LW = W + PF + 1;   // fine columns c0 - PF .. c0 + W
  __shared__ T st[PC][LW];
  const int per = gf.periodic;
  const int lane = threadIdx.x & 63;
  const int w = NW > 1 ? __builtin_amdgcn_readfirstlane(threadIdx.x >> 6) : 0;
  const int e0 = blockIdx.x * NE;
  const int ey = blockIdx.y;
  const int c0 = e0 * PF;
  const int r0 = ey * PF;
  const bool has_below = per || ey > 0;
  const int last_col = min(c0 + W, gf.nx * PF);  // right end of the strip's last element
  // ---- y pass: fine column -> PC coarse rows of this element row ----------
  for (int k = threadIdx.x; k < LW; k += 64 * NW) {
    const int col = c0 - PF + k;
    if (col > last_col) break;
    const bool colok = per || col >= 0;
    T seg[PF + 1];
#pragma unroll
    for (int a = 0; a <= PF; ++a)
      seg[a] = colok ? node_value_guarded(rf, r0 + a, col, gf.rows, gf.cols, per) : T(0);
    T segb[PF + 1];
#pragma unroll
    for (int a = 0; a <= PF; ++a)
      segb[a] = (colok && has_below && a < PF) ? node_value_guarded(rf, r0 - PF + a, col, gf.rows, gf.cols, per)
                                               : T(0);
#pragma unroll 1
    for (int b = 0; b < PC; ++b) st[b][k] = tdot<T, PF + 1>(as_const(ET) + b * (PF + 1), seg);
    st[0][k] += tdot<T, PF + 1>(as_const(ET) + PC * (PF + 1), segb);
  }
  __syncthreads();
  // ---- x pass: lane = (coarse row b, element q) -----------------------------
  const int q = lane / PC, b = lane - (lane / PC) * PC;
  const int ex = e0 + q;
  if (lane < NE * PC && ex < gf.nx) {
    T seg[PF + 1], segl[PF + 1];
#pragma unroll
    for (int a = 0; a <= PF; ++a) seg[a] = st[b][PF + q * PF + a];
    const bool has_left = per || ex > 0;
#pragma unroll
    for (int a = 0; a <= PF; ++a) segl[a] = (has_left && a < PF) ? st[b][q * PF + a] : T(0);
    const int crow = ey * PC + b;
    T *out = fc + (long)crow * gc.cols + ex * PC;
    T *uz = uc_zero ? uc_zero + (long)crow * gc.cols + ex * PC : nullptr;
    const bool zrow = !per && crow == 0;
    int glo, ghi;
    tshare<NW>(PC, w, glo, ghi);
#pragma unroll 1
    for (int g = glo; g < ghi; ++g) {
      T v = tdot<T, PF + 1>(as_const(ET) + g * (PF + 1), seg);
      if (g == 0) v += tdot<T, PF + 1>(as_const(ET) + PC * (PF + 1), segl);
      const bool zero = zrow || (!per && ex == 0 && g == 0);
      out[g] = zero ? T(0) : v;
      if (uz) uz[g] = T(0);
    }
  }
  // ---- Dirichlet: the last coarse row and column are boundary nodes ----------
  if (!per && w == 0) {
    if (ey == gf.ny - 1) {
      for (int cc = lane; cc < NE * PC + 1; cc += 64) {
        const int ccol = e0 * PC + cc;
        if (ccol < gc.cols && (cc < NE * PC || e0 + NE >= gf.nx)) {
          fc[(long)(gc.rows - 1) * gc.cols + ccol] = T(0);
          if (uc_zero) uc_zero[(long)(gc.rows - 1) * gc.cols + ccol] = T(0);
        }
      }
    }
    if (e0 + NE >= gf.nx && lane < PC) {
      const int crow = ey * PC + lane;
      fc[(long)crow * gc.cols + gc.cols - 1] = T(0);
      if (uc_zero) uc_zero[(long)crow * gc.cols + gc.cols - 1] = T(0);
    }
  }
}

// Prolongation u_f += I u_c.  E is (PF+1) x (PC+1) row-major.
template <typename T, int PF, int NW>
__global__ __launch_bounds__(64 * NW) void k_prolong(Grid gf, Grid gc, const T *__restrict__ uc,
                                                T *__restrict__ uf, const T *__restrict__ E) {
  constexpr int PC = (PF + 1) / 2;
  constexpr int NE = 64 / PF;
  constexpr int W = NE * PF;
  __shared__ T st[PC + 1][W];
  const int per = gf.periodic;
  const int lane = threadIdx.x & 63;
  const int w = NW > 1 ? __builtin_amdgcn_readfirstlane(threadIdx.x >> 6) : 0;
  int alo, ahi;   // this wave's fine outputs a
  tshare<NW>(PF, w, alo, ahi);
  const int e0 = blockIdx.x * NE;
  const int ey = blockIdx.y;
  const int c0 = e0 * PF;
  const int r0 = ey * PF;
  // ---- x pass: lane = (coarse row b in 0..PC, element q) ------------------------
  {
    const int q = lane / (PC + 1), b = lane - (lane / (PC + 1)) * (PC + 1);
    const int ex = e0 + q;
    if (lane < NE * (PC + 1) && ex < gf.nx) {
      T seg[PC + 1];
#pragma unroll
      for (int c = 0; c <= PC; ++c)
        seg[c] = node_value_guarded(uc, ey * PC + b, ex * PC + c, gc.rows, gc.cols, per);
#pragma unroll 1
      for (int a = alo; a < ahi; ++a)
        st[b][q * PF + a] = tdot<T, PC + 1>(as_const(E) + a * (PC + 1), seg);
    }
  }
  __syncthreads();
  // ---- y pass: lane = fine column ------------------------------------------------
  const int c = lane;
  const int ex = e0 + c / PF;
  if (c < W && ex < gf.nx) {
    const int col = c0 + c;
    if (per || col > 0) {
      T seg[PC + 1];
#pragma unroll
      for (int b = 0; b <= PC; ++b) seg[b] = st[b][c];
      T *out = uf + (long)r0 * gf.cols + col;
      // this wave's fine rows of u, loaded together before any store
      constexpr int HA = (PF + NW - 1) / NW;
      T ov[HA];
#pragma unroll
      for (int t = 0; t < HA; ++t) ov[t] = alo + t < ahi ? out[(long)(alo + t) * gf.cols] : T(0);
#pragma unroll
      for (int t = 0; t < HA; ++t) {
        const int a = alo + t;
        if (a >= ahi) break;
        const T v = tdot<T, PC + 1>(as_const(E) + a * (PC + 1), seg);
        if (per || r0 + a > 0) out[(long)a * gf.cols] = ov[t] + v;
      }
    }
  }
}

}  // namespace

template <typename T, int PF>
void launch_restrict_p(const Grid &gf, const Grid &gc, const T *rf, T *fc, T *uc_zero,
                       const T *ET, hipStream_t s) {
  constexpr int NE = 64 / PF;
  constexpr int NW = transfer_waves<PF>();
  dim3 grid(ceil_div(gf.nx, NE), gf.ny);
  klaunch((k_restrict<T, PF, NW>), grid, dim3(64 * NW), 0, s, gf, gc, rf, fc, uc_zero,
                     ET);
}

template <typename T, int PF>
void launch_prolong_p(const Grid &gf, const Grid &gc, const T *uc, T *uf, const T *E,
                      hipStream_t s) {
  constexpr int NE = 64 / PF;
  constexpr int NW = transfer_waves<PF>();
  dim3 grid(ceil_div(gf.nx, NE), gf.ny);
  klaunch((k_prolong<T, PF, NW>), grid, dim3(64 * NW), 0, s, gf, gc, uc, uf, E);
}

}  // namespace sem
