// Weighted additive Schwarz correction (Section 3.1, Algorithm 2) with the
// fast-diagonalisation solve on the matrix cores: BF16 or FP16 operands, FP32
// accumulation (the reduced-precision smoother of the mixed-precision
// V-cycle; the outer residual and CG stay FP64).  Same result as k_fdm up to
// the rounding of the operands:
//     du = W_y S_y [ D_s .* (S_y^T R S_x) ] S_x^T W_x,  u += du.
//
// One 64-lane wavefront per work item (elements of one subdomain type pair,
// processed one after another).  The m x m tile is padded to n = 16 NB and
// cut into 16 x 16 blocks; every block product is one
// v_mfma_f32_16x16x16_{bf16,f16}.  With their lane layouts, the accumulator
// layout of a block X equals the B-operand layout of X and the A-operand
// layout of X^T, so the chain is written as four products that each take the
// previous result, transposed, as the A operand:
//     P1^T = R^T S_y,  P2 = P1 S_x (.* D_s),  Q^T = P2^T (W_y S_y)^T,
//     du = Q S_x^T,
// and no intermediate ever leaves the registers.  The four factor matrices of
// the work item's type pair stay in registers as B operands.  FP16 operands
// are scaled tile by tile by powers of two (exact), and the correction is
// scaled back before the scatter.
#include "common.h"
#include "kernels.h"

#include <stdexcept>

namespace sem {
namespace {

typedef float f32x4 __attribute__((ext_vector_type(4)));

// Operand formats of the 16x16x16 products.  Both share one lane layout:
// A: lane l holds row l % 16, k = 4 (l / 16) + j;  B: k = 4 (l / 16) + j,
// column l % 16;  accumulator: row 4 (l / 16) + j, column l % 16.
struct OpBF16 {
  typedef short v4 __attribute__((ext_vector_type(4)));
  // BF16 keeps the FP32 exponent range: no scaling needed
  static constexpr bool kScaled = false;
  // FP32 -> BF16, round to nearest even (inputs are finite)
  static __device__ __forceinline__ short cvt(float x) {
    uint32_t u = __float_as_uint(x);
    u += 0x7FFFu + ((u >> 16) & 1u);
    return (short)(u >> 16);
  }
  static __device__ __forceinline__ f32x4 mma(v4 a, v4 b, f32x4 c) {
    return __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, b, c, 0, 0, 0);
  }
};

struct OpF16 {
  typedef _Float16 v4 __attribute__((ext_vector_type(4)));
  // FP16 has a 5-bit exponent (normal range 2^-14 .. 65504): every operand
  // tile is scaled by a power of two that brings its largest magnitude into
  // [0.5, 1) before the conversion, so no entry overflows and underflow only
  // touches entries below 2^-14 of the tile's largest one
  static constexpr bool kScaled = true;
  static __device__ __forceinline__ _Float16 cvt(float x) { return (_Float16)x; }   // RNE
  static __device__ __forceinline__ f32x4 mma(v4 a, v4 b, f32x4 c) {
    return __builtin_amdgcn_mfma_f32_16x16x16f16(a, b, c, 0, 0, 0);
  }
};

template <class Op>
__device__ __forceinline__ typename Op::v4 pack(const f32x4 &v, float sc) {
  typename Op::v4 r;
  r[0] = Op::cvt(v[0] * sc);
  r[1] = Op::cvt(v[1] * sc);
  r[2] = Op::cvt(v[2] * sc);
  r[3] = Op::cvt(v[3] * sc);
  return r;
}

// Largest magnitude over the wavefront's NB x NB accumulator blocks.
template <int NB>
__device__ __forceinline__ float wave_amax(const f32x4 (&Y)[NB][NB]) {
  float v = 0.f;
#pragma unroll
  for (int I = 0; I < NB; ++I)
#pragma unroll
    for (int J = 0; J < NB; ++J)
#pragma unroll
      for (int j = 0; j < 4; ++j) v = fmaxf(v, fabsf(Y[I][J][j]));
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v = fmaxf(v, __shfl_xor(v, off));
  return v;
}

// e with amax = f 2^e, f in [0.5, 1) (0 for a zero tile): scaling by 2^-e
// is exact and puts the largest magnitude into [0.5, 1).
__device__ __forceinline__ int scale_exp(float amax) {
  return amax > 0.f ? __builtin_amdgcn_frexp_expf(amax) : 0;
}

// Block (I, J) of the product of the NB x NB block matrices X^T and B, where
// X is given in accumulator layout (X^T as A operands) and B in B layout.
template <class Op, int NB>
__device__ __forceinline__ void chain(const typename Op::v4 (&Xa)[NB][NB],
                                      const typename Op::v4 (&B)[NB][NB], f32x4 (&Y)[NB][NB]) {
#pragma unroll
  for (int I = 0; I < NB; ++I)
#pragma unroll
    for (int J = 0; J < NB; ++J) {
      f32x4 acc = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
      for (int K = 0; K < NB; ++K) acc = Op::mma(Xa[K][I], B[K][J], acc);
      Y[I][J] = acc;
    }
}

// Accumulators -> operands of the next product; with scaled operands the
// tile is first brought to [0.5, 1) and the exponent added to E.
template <class Op, int NB>
__device__ __forceinline__ void to_operands(const f32x4 (&Y)[NB][NB], typename Op::v4 (&Xa)[NB][NB],
                                            int &E) {
  float sc = 1.f;
  if constexpr (Op::kScaled) {
    const int e = scale_exp(wave_amax<NB>(Y));
    E += e;
    sc = ldexpf(1.f, -e);
  }
#pragma unroll
  for (int I = 0; I < NB; ++I)
#pragma unroll
    for (int J = 0; J < NB; ++J) Xa[I][J] = pack<Op>(Y[I][J], sc);
}

template <class Op, int NB>
__global__ __launch_bounds__(64) void k_fdm_mfma(FdmArgs<float> A) {
  typedef typename Op::v4 v4;
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
  v4 BSy[NB][NB], BSx[NB][NB], BSyWT[NB][NB], BSxT[NB][NB];
  f32x4 Dv[NB][NB];   // 1 / (lambda_y + lambda_x) in accumulator layout
  int Ef = 0;         // exponent of the factor scalings (scaled operands)
  {
    f32x4 fy[NB][NB], fx[NB][NB], fw[NB][NB], ft[NB][NB];
#pragma unroll
    for (int K = 0; K < NB; ++K)
#pragma unroll
      for (int J = 0; J < NB; ++J) {
        const int n = 16 * J + c16;
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          const int k = 16 * K + r4 + j;
          const bool ok = k < m && n < m;
          fy[K][J][j] = ok ? SyT[n * m + k] : 0.f;    // S_y[k][n]
          fx[K][J][j] = ok ? Sx[k * m + n] : 0.f;     // S_x[k][n]
          fw[K][J][j] = ok ? SyW[n * m + k] : 0.f;    // (W_y S_y)^T[k][n]
          ft[K][J][j] = ok ? Sx[n * m + k] : 0.f;     // S_x^T[k][n]
          Dv[K][J][j] = ok ? dv[k * m + n] : 0.f;     // D[k][n] (row k of the accumulator)
        }
      }
    float sy = 1.f, sx = 1.f, sw = 1.f, st = 1.f;
    if constexpr (Op::kScaled) {
      const int ey = scale_exp(wave_amax<NB>(fy)), ex = scale_exp(wave_amax<NB>(fx));
      const int ew = scale_exp(wave_amax<NB>(fw)), et = scale_exp(wave_amax<NB>(ft));
      Ef = ey + ex + ew + et;
      sy = ldexpf(1.f, -ey);
      sx = ldexpf(1.f, -ex);
      sw = ldexpf(1.f, -ew);
      st = ldexpf(1.f, -et);
    }
#pragma unroll
    for (int K = 0; K < NB; ++K)
#pragma unroll
      for (int J = 0; J < NB; ++J) {
        BSy[K][J] = pack<Op>(fy[K][J], sy);
        BSx[K][J] = pack<Op>(fx[K][J], sx);
        BSyWT[K][J] = pack<Op>(fw[K][J], sw);
        BSxT[K][J] = pack<Op>(ft[K][J], st);
      }
  }

  for (int e = 0; e < cnt; ++e) {
    const int packed = task->elem[e];
    const int ey = packed >> 16, ex = packed & 0xffff;
    const int row0 = ey * g.p - A.n_o, col0 = ex * g.p - A.n_o;
    const float s = A.nuinv ? A.nuinv[(long)ey * g.nx + ex] : 1.0f;
    // gather R in accumulator layout: block (K, I) holds rows 16K + r4 + j,
    // columns 16I + c16 of the tile
    f32x4 Y[NB][NB];
#pragma unroll
    for (int K = 0; K < NB; ++K)
#pragma unroll
      for (int I = 0; I < NB; ++I) {
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
          Y[K][I][j] = ok ? x : 0.f;
        }
      }
    int E = Ef;   // du = 2^E times the last accumulator (scaled operands)
    v4 Xa[NB][NB];
    to_operands<Op, NB>(Y, Xa, E);
    chain<Op, NB>(Xa, BSy, Y);      // P1^T = R^T S_y
    to_operands<Op, NB>(Y, Xa, E);
    chain<Op, NB>(Xa, BSx, Y);      // P2 = P1 S_x
#pragma unroll
    for (int I = 0; I < NB; ++I)
#pragma unroll
      for (int J = 0; J < NB; ++J) Y[I][J] *= Dv[I][J] * s;   // .* D_s / nu_bar
    to_operands<Op, NB>(Y, Xa, E);
    chain<Op, NB>(Xa, BSyWT, Y);    // Q^T = P2^T (W_y S_y)^T
    to_operands<Op, NB>(Y, Xa, E);
    chain<Op, NB>(Xa, BSxT, Y);     // du = Q S_x^T
    const float back = Op::kScaled ? ldexpf(1.f, E) : 1.f;
    const float *__restrict__ we = A.wel ? A.wel + ((long)ey * g.nx + ex) * 2 * m : nullptr;
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
      const float wxn = okc ? (we ? we[m + n] : A.wx[(long)ex * m + n]) * back : 0.f;
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
          if (ok) {
            const long node = (long)gr * g.cols + gc;
            float c = Y[I][J][j] * wxn;
            if (we) c *= we[a] * A.dnorm[node];
            atomic_add(&A.u[node], c);
          }
        }
    }
  }
}

}  // namespace

template <class Op>
static void launch_op(const FdmArgs<float> &a, hipStream_t s) {
  if (a.m <= 16)
    klaunch((k_fdm_mfma<Op, 1>), dim3(a.ntasks), dim3(64), 0, s, a);
  else if (a.m <= 32)
    klaunch((k_fdm_mfma<Op, 2>), dim3(a.ntasks), dim3(64), 0, s, a);
  else
    klaunch((k_fdm_mfma<Op, 3>), dim3(a.ntasks), dim3(64), 0, s, a);
}

void launch_fdm_mfma(const FdmArgs<float> &a, bool fp16, hipStream_t s) {
  if (a.ntasks <= 0) return;
  if (a.m > 48) throw std::runtime_error("matrix-core Schwarz kernel: tile wider than 48");
  if (fp16)
    launch_op<OpF16>(a, s);
  else
    launch_op<OpBF16>(a, s);
}

}  // namespace sem
