// Weighted additive Schwarz correction (Section 3.1, Algorithm 2) with the
// fast-diagonalisation solve on the matrix cores: BF16 operands, FP32
// accumulation (the reduced-precision smoother of the mixed-precision
// V-cycle; the outer residual and CG stay FP64).  Same result as k_fdm up to
// BF16 rounding of the operands:
//     du = W_y S_y [ D_s .* (S_y^T R S_x) ] S_x^T W_x,  u += du.
//
// One 64-lane wavefront per work item (elements of one subdomain type pair,
// processed one after another).  The m x m tile is padded to n = 16 NB and
// cut into 16 x 16 blocks; every block product is one
// v_mfma_f32_16x16x16_bf16.  With its lane layouts, the accumulator layout of
// a block X equals the B-operand layout of X and the A-operand layout of X^T,
// so the chain is written as four products that each take the previous
// result, transposed, as the A operand:
//     P1^T = R^T S_y,  P2 = P1 S_x (.* D_s),  Q^T = P2^T (W_y S_y)^T,
//     du = Q S_x^T,
// and no intermediate ever leaves the registers.  The four factor matrices of
// the work item's type pair stay in registers as BF16 B operands.
#include "common.h"
#include "kernels.h"

namespace sem {
namespace {

typedef short bf16x4 __attribute__((ext_vector_type(4)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

// FP32 -> BF16, round to nearest even (inputs are finite).
__device__ __forceinline__ short bf16_rne(float x) {
  uint32_t u = __float_as_uint(x);
  u += 0x7FFFu + ((u >> 16) & 1u);
  return (short)(u >> 16);
}

__device__ __forceinline__ bf16x4 pack(const f32x4 &v) {
  bf16x4 r;
  r[0] = bf16_rne(v[0]);
  r[1] = bf16_rne(v[1]);
  r[2] = bf16_rne(v[2]);
  r[3] = bf16_rne(v[3]);
  return r;
}

// Block (I, J) of the product of the NB x NB block matrices X^T and B, where
// X is given in accumulator layout (X^T as A operands) and B in B layout.
template <int NB>
__device__ __forceinline__ void chain(const bf16x4 (&Xa)[NB][NB], const bf16x4 (&B)[NB][NB],
                                      f32x4 (&Y)[NB][NB]) {
#pragma unroll
  for (int I = 0; I < NB; ++I)
#pragma unroll
    for (int J = 0; J < NB; ++J) {
      f32x4 acc = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
      for (int K = 0; K < NB; ++K)
        acc = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(Xa[K][I], B[K][J], acc, 0, 0, 0);
      Y[I][J] = acc;
    }
}

template <int NB>
__device__ __forceinline__ void to_operands(const f32x4 (&Y)[NB][NB], bf16x4 (&Xa)[NB][NB]) {
#pragma unroll
  for (int I = 0; I < NB; ++I)
#pragma unroll
    for (int J = 0; J < NB; ++J) Xa[I][J] = pack(Y[I][J]);
}

template <int NB>
__global__ __launch_bounds__(64) void k_fdm_mfma(FdmArgs<float> A) {
  const FdmTask *__restrict__ task = A.tasks + blockIdx.x;
  const int ty = task->ty, tx = task->tx, cnt = task->count;
  const int m = A.m;
  const int lane = threadIdx.x;
  const int c16 = lane & 15;        // column within a block
  const int r4 = (lane >> 4) * 4;   // first of the lane's 4 rows within a block
  const Grid g = A.g;
  const int per = g.periodic;
  const float *__restrict__ SyT = A.SyT + (long)ty * m * m;   // S_y^T
  const float *__restrict__ SyW = A.SyW + (long)ty * m * m;   // diag(w_y) S_y
  const float *__restrict__ Sx = A.Sx + (long)tx * m * m;     // S_x
  const float *__restrict__ dv = A.dinv + ((long)ty * A.ntx + tx) * m * m;

  // factor matrices in B layout: element (k, n) of block (K, J) at
  // k = 16 K + r4 + j, n = 16 J + c16; zero outside the m x m tile
  bf16x4 BSy[NB][NB], BSx[NB][NB], BSyWT[NB][NB], BSxT[NB][NB];
  f32x4 Dv[NB][NB];   // 1 / (lambda_y + lambda_x) in accumulator layout
#pragma unroll
  for (int K = 0; K < NB; ++K)
#pragma unroll
    for (int J = 0; J < NB; ++J) {
      f32x4 sy, sx, sw, st, d;
      const int n = 16 * J + c16;
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const int k = 16 * K + r4 + j;
        const bool ok = k < m && n < m;
        sy[j] = ok ? SyT[n * m + k] : 0.f;     // S_y[k][n]
        sx[j] = ok ? Sx[k * m + n] : 0.f;      // S_x[k][n]
        sw[j] = ok ? SyW[n * m + k] : 0.f;     // (W_y S_y)^T[k][n]
        st[j] = ok ? Sx[n * m + k] : 0.f;      // S_x^T[k][n]
        d[j] = ok ? dv[k * m + n] : 0.f;       // D[k][n] (row k of the accumulator)
      }
      BSy[K][J] = pack(sy);
      BSx[K][J] = pack(sx);
      BSyWT[K][J] = pack(sw);
      BSxT[K][J] = pack(st);
      Dv[K][J] = d;
    }

  for (int e = 0; e < cnt; ++e) {
    const int packed = task->elem[e];
    const int ey = packed >> 16, ex = packed & 0xffff;
    const int row0 = ey * g.p - A.n_o, col0 = ex * g.p - A.n_o;
    const float s = A.nuinv ? A.nuinv[(long)ey * g.nx + ex] : 1.0f;
    // gather R in accumulator layout: block (K, I) holds rows 16K + r4 + j,
    // columns 16I + c16 of the tile
    bf16x4 Ra[NB][NB];
#pragma unroll
    for (int K = 0; K < NB; ++K)
#pragma unroll
      for (int I = 0; I < NB; ++I) {
        f32x4 v;
        int gc = col0 + 16 * I + c16;
        bool okc;
        if (per) {
          gc = wrap(gc, g.cols);
          okc = 16 * I + c16 < m;
        } else {
          okc = 16 * I + c16 < m && gc >= 1 && gc <= g.cols - 2;
        }
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          const int a = 16 * K + r4 + j;
          int gr = row0 + a;
          bool ok;
          if (per) {
            gr = wrap(gr, g.rows);
            ok = okc && a < m;
          } else {
            ok = okc && a < m && gr >= 1 && gr <= g.rows - 2;
          }
          const long idx = ok ? (long)gr * g.cols + gc : 0;
          const float x = A.r[idx];
          v[j] = ok ? x : 0.f;
        }
        Ra[K][I] = pack(v);
      }
    f32x4 Y[NB][NB];
    bf16x4 Xa[NB][NB];
    chain<NB>(Ra, BSy, Y);          // P1^T = R^T S_y
    to_operands<NB>(Y, Xa);
    chain<NB>(Xa, BSx, Y);          // P2 = P1 S_x
#pragma unroll
    for (int I = 0; I < NB; ++I)
#pragma unroll
      for (int J = 0; J < NB; ++J) Y[I][J] *= Dv[I][J] * s;   // .* D_s / nu_bar
    to_operands<NB>(Y, Xa);
    chain<NB>(Xa, BSyWT, Y);        // Q^T = P2^T (W_y S_y)^T
    to_operands<NB>(Y, Xa);
    chain<NB>(Xa, BSxT, Y);         // du = Q S_x^T
    // weighted scatter-add: block (I, J) holds rows 16I + r4 + j, columns 16J + c16
#pragma unroll
    for (int J = 0; J < NB; ++J) {
      const int n = 16 * J + c16;
      int gc = col0 + n;
      bool okc;
      if (per) {
        gc = wrap(gc, g.cols);
        okc = n < m;
      } else {
        okc = n < m && gc >= 1 && gc <= g.cols - 2;
      }
      const float wxn = okc ? A.wx[(long)ex * m + n] : 0.f;
#pragma unroll
      for (int I = 0; I < NB; ++I)
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          const int a = 16 * I + r4 + j;
          int gr = row0 + a;
          bool ok;
          if (per) {
            gr = wrap(gr, g.rows);
            ok = okc && a < m;
          } else {
            ok = okc && a < m && gr >= 1 && gr <= g.rows - 2;
          }
          if (ok) atomic_add(&A.u[(long)gr * g.cols + gc], Y[I][J][j] * wxn);
        }
    }
  }
}

}  // namespace

void launch_fdm_bf16(const FdmArgs<float> &a, hipStream_t s) {
  if (a.ntasks <= 0) return;
  if (a.m <= 16)
    hipLaunchKernelGGL(k_fdm_mfma<1>, dim3(a.ntasks), dim3(64), 0, s, a);
  else if (a.m <= 32)
    hipLaunchKernelGGL(k_fdm_mfma<2>, dim3(a.ntasks), dim3(64), 0, s, a);
  else
    hipLaunchKernelGGL(k_fdm_mfma<3>, dim3(a.ntasks), dim3(64), 0, s, a);
}

}  // namespace sem
